"""Pins of the oracle's target-side derivatives of the forward,
D[a, k](i) = dL_a(i)/dX_i,k with the sources' centres held fixed (the sums
the one-pass adjoint saves in the forward): complex-step derivatives of the
plain forward sum with only the target cell's centre perturbed, equality of
the entries that name the same derivative of G (a + e_k = a' + e_k'), and
Laplace's equation; for the total-order truncation and the full one (every
source moment for every output order). CPU only."""
import numpy as np
import pytest

import oracle
import synthetic

SUB3 = 512


def _periodic_case():
    # 2^3 periodic sub-grids: a target's own sub-grid sits only in slot 13,
    # so the cell is never a source of itself (nor of its own image)
    return synthetic.batched_config(2, 301, missing_frac=0.5)


def _open_case():
    rng = synthetic._rng(302)
    M, X = synthetic.store_field(3, rng, 2.0, 3.0, 0.6, sep=6.0)
    full = synthetic.lattice_batch(3, periodic=False)
    tg = np.array([13, 4], np.int32)
    nbr = full["nbr"][tg].copy()
    nbr[0, [5, 21]] = -1
    return {"S": 27, "T": 2, "tgt": tg, "nbr": nbr, "shift": None, "period": None}, M, X


@pytest.mark.parametrize("full", [False, True])
@pytest.mark.parametrize("case", ["periodic", "open"])
def test_complex_step_of_the_forward(case, full):
    batch, M, X = _periodic_case() if case == "periodic" else _open_case()
    D, A = oracle.batched_forward_tgrad(batch, M, X, want_abs=True, full=full)
    h = 1e-30
    for t, cell in [(0, 0), (0, 300), (1, 511), (batch["T"] - 1, 137)]:
        c = int(batch["tgt"][t]) * SUB3 + cell
        col = t * SUB3 + cell
        for k in range(3):
            Xim = np.zeros_like(X)
            Xim[k, c] = h
            _, Lim = oracle.batched_forward_cs(batch, M, X, Xim, tsel=[t], full=full)
            cs = Lim[:, cell] / h
            err = np.abs(cs - D[:, k, col])
            assert np.all(err <= 1e-13 * A[:, k, col] + 1e-300), (case, t, cell, k, err.max())


@pytest.mark.parametrize("full", [False, True])
def test_entries_naming_the_same_derivative_are_equal(full):
    batch, M, X = _periodic_case()
    D = oracle.batched_forward_tgrad(batch, M, X, full=full)
    exps = [oracle.multi_index(g) for g in range(20)]
    index = {tuple(e): g for g, e in enumerate(exps)}
    npair = 0
    for a, ea in enumerate(exps):
        for k in range(3):
            g = list(ea)
            g[k] += 1
            for a2, ea2 in enumerate(exps):
                for k2 in range(3):
                    g2 = list(ea2)
                    g2[k2] += 1
                    if g2 == g and (a2, k2) != (a, k):
                        assert np.array_equal(D[a, k], D[a2, k2])
                        npair += 1
    assert npair > 0 and index[(0, 0, 0)] == 0


@pytest.mark.parametrize("full", [False, True])
def test_laplace_trace(full):
    """sum_k D[g + e_k, k] = sum_beta s_beta M_beta lap G_{g+beta} = 0."""
    batch, M, X = _periodic_case()
    D, A = oracle.batched_forward_tgrad(batch, M, X, want_abs=True, full=full)
    exps = [tuple(oracle.multi_index(g)) for g in range(20)]
    index = {e: g for g, e in enumerate(exps)}
    for g, e in enumerate(exps):
        if sum(e) > 2:
            continue
        tr = np.zeros(D.shape[2])
        scale = np.zeros(D.shape[2])
        for k in range(3):
            ek = list(e)
            ek[k] += 1
            a = index[tuple(ek)]
            tr += D[a, k]
            scale += A[a, k]
        assert np.all(np.abs(tr) <= 1e-13 * scale + 1e-300), (e, np.abs(tr).max())


def test_full_orders_one_to_three_are_the_full_forward():
    """Under the full truncation every output order keeps every source
    moment, so D[a, k] for |a| <= 2 is the full forward's L_{a+e_k}."""
    batch, M, X = _periodic_case()
    D = oracle.batched_forward_tgrad(batch, M, X, full=True)
    L, A = oracle.batched_forward(batch, M, X, want_abs=True, full=True)
    exps = [tuple(oracle.multi_index(g)) for g in range(20)]
    index = {e: g for g, e in enumerate(exps)}
    for a, e in enumerate(exps):
        if sum(e) > 2:
            continue
        for k in range(3):
            ek = list(e)
            ek[k] += 1
            g = index[tuple(ek)]
            assert np.all(np.abs(D[a, k] - L[g]) <= 1e-13 * A[g] + 1e-300), (e, k)
