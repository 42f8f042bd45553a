"""GPU parity of the forward with the angular-momentum correction of the force
(ot_fmm_multipole_batched_amc) against the oracle, through the C ABI, and the
conservation law that fixes the correction, checked on the GPU's outputs: over
a closed set (open lattice, every sub-grid a target) the force from L (GPU
evaluation pass) plus the correction, with the cells' spin torques from L,
balances sum_i (X_i x F_i + tau_i) = 0 to rounding, while the force from L
alone does not."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import oracle  # noqa: E402
import synthetic  # noqa: E402
from parity import assert_parity  # noqa: E402
from torque import cross, spin_torque  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def ot():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08058_amd as ot
    return ot


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _empty(*shape):
    import torch
    return torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("sched", [1, 3, 0x11, 0x13, 0x21, 0x23, 0x31, 0x33, 0])
def test_small_periodic_with_missing(ot, sched):
    batch, M, X = synthetic.batched_config(2, 141, missing_frac=0.5)
    plan = ot.Plan.from_batch(batch)
    NT = batch["T"] * 512
    Md, Xd = _dev(M), _dev(X)
    L, dF = _empty(20, NT), _empty(3, NT)
    plan.multipole_batched_amc(Md, Xd, L, dF, sched=sched)
    Lh, dFh = _host(L), _host(dF)
    ref, A = oracle.batched_forward(batch, M, X, want_abs=True)
    assert_parity(Lh, ref, TOL, what="amc L", A=A)
    dref, dA = oracle.batched_forward_amc(batch, M, X, want_abs=True)
    print("dF worst", assert_parity(dFh, dref, TOL, what="amc dF", A=dA))
    L2, dF2 = _empty(20, NT), _empty(3, NT)
    plan.multipole_batched_amc(Md, Xd, L2, dF2, sched=sched)
    assert np.array_equal(_host(L2), Lh) and np.array_equal(_host(dF2), dFh)
    if sched:
        # the same F sums as the forward with saved sums of the same schedule
        L3, C3 = _empty(20, NT), _empty(24, NT)
        plan.multipole_batched_save(Md, Xd, L3, C3, sched=sched)
        assert np.array_equal(_host(L3), Lh)


def test_open_subset_of_targets(ot):
    rng = synthetic._rng(142)
    M, X = synthetic.store_field(3, rng, 2.0, 3.0, 0.6, sep=6.0)
    full = synthetic.lattice_batch(3, periodic=False)
    tg = np.array([13, 4, 22], np.int32)
    nbr = full["nbr"][tg].copy()
    nbr[0, [5, 21]] = -1
    batch = {"S": 27, "T": 3, "tgt": tg, "nbr": nbr, "shift": None, "period": None}
    plan = ot.Plan.from_batch(batch)
    L, dF = _empty(20, 3 * 512), _empty(3, 3 * 512)
    plan.multipole_batched_amc(_dev(M), _dev(X), L, dF)
    dref, dA = oracle.batched_forward_amc(batch, M, X, want_abs=True)
    assert_parity(_host(dF), dref, TOL, what="amc dF open subset", A=dA)


def test_angular_momentum_balance_on_the_gpu_outputs(ot):
    import torch
    rng = synthetic._rng(143)
    M, X = synthetic.store_field(3, rng, 2.0, 3.0, 0.6, sep=6.0)
    batch = synthetic.lattice_batch(3, periodic=False)
    plan = ot.Plan.from_batch(batch)
    n = batch["S"] * 512
    Md, Xd = _dev(M), _dev(X)
    L, dF = _empty(20, n), _empty(3, n)
    plan.multipole_batched_amc(Md, Xd, L, dF)
    F = torch.empty((3, n), dtype=torch.float64, device="cuda")
    W = torch.empty((n,), dtype=torch.float64, device="cuda")
    ot.ot_fmm_evaluate(Md, L, F, W)
    Lh, dFh, Fh = _host(L), _host(dF), _host(F)
    tau = spin_torque(M, Lh)

    def balance(Ft):
        J = np.abs((cross(X, Ft) + tau).sum(1)) / (np.abs(cross(X, Ft)) + np.abs(tau)).sum(1)
        P = np.abs(Ft.sum(1)) / np.abs(Ft).sum(1)
        return float(J.max()), float(P.max())

    j1, p1 = balance(Fh + dFh)
    j0, p0 = balance(Fh)
    print("angular momentum balance: corrected %.2e, from L alone %.2e; linear %.2e, %.2e" % (j1, j0, p1, p0))
    assert j1 < 1e-13 and p1 < 1e-13
    assert j0 > 1e-9


def test_config5_sampled(ot):
    """The benchmark's 32^3-sub-grid workload: 8 seeded targets (half with
    missing neighbours) against the oracle."""
    import torch
    batch, M, X = synthetic.config5()
    plan = ot.Plan.from_batch(batch)
    NT = batch["T"] * 512
    L = torch.empty((20, NT), dtype=torch.float64, device="cuda")
    dF = torch.empty((3, NT), dtype=torch.float64, device="cuda")
    plan.multipole_batched_amc(_dev(M), _dev(X), L, dF)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(dF).all())
    rng = np.random.default_rng(145)
    miss = batch["missing_targets"]
    sel = np.array(sorted(set(rng.choice(miss, 4, replace=False).tolist())
                          | set(rng.choice(batch["T"], 4, replace=False).tolist())), np.int32)
    idx = torch.from_numpy(sel).long().cuda()
    got = dF.reshape(3, -1, 512)[:, idx].reshape(3, -1).cpu().numpy()
    del L, dF
    dref, dA = oracle.batched_forward_amc(batch, M, X, tsel=sel, want_abs=True)
    assert_parity(got, dref, TOL, what="config5 dF", A=dA)
