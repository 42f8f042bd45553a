"""Pins of the oracle's angular-momentum correction of the force. With the
total-order truncation the interaction energy is invariant under rotations of
positions and moments together, so over a closed set with symmetric
availability (an open lattice, every sub-grid a target) the forces that are
the exact gradient of that energy and the cells' spin torques balance:
sum_i (X_i x F_i + tau_i) = 0 and sum_i F_i = 0. The force evaluated from L
alone fails the torque balance; adding the correction restores it to
rounding. Also pinned: the corrected force equals the complex-step gradient of
the energy 1/2 sum_i sum_a (M_a(i)/a!) L_a(i), equals the force assembled
from the oracle's target-side derivatives, and the correction vanishes for
mass-only sources and targets. CPU only."""
import numpy as np

import oracle
import synthetic
from torque import FACT, SUB3, cross, eval_force, spin_torque

def closed_case(seed=7, n=3):
    rng = synthetic._rng(seed)
    M, X = synthetic.store_field(n, rng, 2.0, 3.0, 0.6, sep=6.0)
    return synthetic.lattice_batch(n, periodic=False), M, X


def balances(M, X, F, L):
    tau = spin_torque(M, L)
    P = np.abs(F.sum(1)) / np.abs(F).sum(1)
    J = np.abs((cross(X, F) + tau).sum(1)) / (np.abs(cross(X, F)) + np.abs(tau)).sum(1)
    return P.max(), J.max()


def test_torque_balance_needs_the_correction():
    batch, M, X = closed_case()
    L = oracle.batched_forward(batch, M, X)
    dF = oracle.batched_forward_amc(batch, M, X)
    Fe = eval_force(M, L)
    p0, j0 = balances(M, X, Fe, L)
    p1, j1 = balances(M, X, Fe + dF, L)
    assert p0 < 1e-14 and p1 < 1e-14          # linear momentum either way
    assert j1 < 1e-14                          # corrected: total angular momentum to rounding
    assert j0 > 1e-9                           # uncorrected: fails by far more than rounding
    assert np.abs(dF).max() < 1e-3 * np.abs(Fe).max()  # a small correction


def test_corrected_force_is_the_gradient_of_the_energy():
    """Complex step of E = 1/2 sum_i sum_a (M_a/a!) L_a(i) (the moments held
    fixed) with respect to one cell's centre."""
    batch, M, X = closed_case(seed=8)
    L = oracle.batched_forward(batch, M, X)
    F = eval_force(M, L) + oracle.batched_forward_amc(batch, M, X)
    h = 1e-30
    for c, k in ((13 * SUB3 + 100, 0), (4 * SUB3 + 511, 1), (22 * SUB3 + 7, 2)):
        Xim = np.zeros_like(X)
        Xim[k, c] = h
        _, Lim = oracle.batched_forward_cs(batch, M, X, Xim)
        dE = 0.5 * float(np.sum(M / FACT[:, None] * Lim)) / h
        assert abs(F[k, c] + dE) <= 1e-12 * np.abs(F[:, c]).max(), (c, k, F[k, c], -dE)


def test_matches_the_target_side_derivatives():
    """-sum_{|a| <= 3} (M_a/a!) dL_a/dX_i,k, from the target-side derivatives,
    is the corrected force."""
    batch, M, X = synthetic.batched_config(2, 9, missing_frac=0.5)
    tg = batch["tgt"]
    Mt = M.reshape(20, -1, SUB3)[:, tg].reshape(20, -1)
    D = oracle.batched_forward_tgrad(batch, M, X)
    L = oracle.batched_forward(batch, M, X)
    dF, A = oracle.batched_forward_amc(batch, M, X, want_abs=True)
    Fc = np.zeros((3, Mt.shape[1]))
    for g in range(20):
        for k in range(3):
            Fc[k] -= Mt[g] / FACT[g] * D[g, k]
    Fe = eval_force(Mt, L)
    scale = np.abs(Fe).max(axis=0)
    assert np.all(np.abs(Fc - (Fe + dF)) <= 1e-13 * scale + 1e-300)


def test_vanishes_for_mass_only_cells():
    batch, M, X = synthetic.batched_config(2, 10, missing_frac=0.3)
    M0 = np.zeros_like(M)
    M0[0] = M[0]
    assert np.all(oracle.batched_forward_amc(batch, M0, X) == 0.0)
