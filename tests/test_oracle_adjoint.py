"""Pins of the oracle's batched forward and of its adjoint: the batched sum
against the single-block sum on the gathered halo (periodic shifts and
missing neighbours included), the dot-product test for the moment gradient
(the loss is linear in the moments), complex-step derivatives for the
centre-of-mass gradient, central differences, and translation invariance.
CPU only."""
import numpy as np
import pytest

import oracle
import synthetic

SUB3 = 512


def gather_halo(batch, M, X, t):
    """24^3 halo arrays of target t from the store: missing neighbours get zero
    moments and their (finite) centres, periodic images their shift."""
    Mh = np.zeros((M.shape[0], 24 ** 3))
    Xh = np.zeros((3, 24 ** 3))
    lz, ly, lx = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    loc = (lx + 8 * ly + 64 * lz).ravel()
    for slot in range(27):
        sx, sy, sz = slot % 3, (slot // 3) % 3, slot // 9
        hidx = ((8 * sx + lx) + 24 * (8 * sy + ly) + 576 * (8 * sz + lz)).ravel()
        blk = batch["nbr"][t, slot]
        src = batch["nbr"][t, 13] if blk < 0 else blk
        Xh[:, hidx] = X[:, src * SUB3 + loc]
        if batch.get("shift") is not None:
            sh = batch["shift"][t, slot].astype(np.float64) * batch["period"]
            Xh[:, hidx] += sh[:, None]
        if blk < 0:
            Xh[:, hidx] += 8.0 * (np.array([sx, sy, sz]) - 1)[:, None]  # keep it away
            continue
        Mh[:, hidx] = M[:, blk * SUB3 + loc]
    return Mh, Xh


def small_open_case(targets=(13, 4, 22), missing=((13, 5), (13, 21), (4, 13 + 1))):
    """Store of 3^3 sub-grids on an open lattice; a few of them are targets,
    some neighbour entries are knocked out (asymmetric availability)."""
    rng = synthetic._rng(99)
    M, X = synthetic.store_field(3, rng, 2.0, 3.0, 0.6, sep=6.0)
    full = synthetic.lattice_batch(3, periodic=False)
    tg = np.array(targets, np.int32)
    nbr = full["nbr"][tg].copy()
    for ti, slot in missing:
        row = list(targets).index(ti)
        if slot != 13:
            nbr[row, slot] = -1
    batch = {"S": 27, "T": len(tg), "tgt": tg, "nbr": nbr, "shift": None, "period": None}
    return batch, M, X


def test_batched_matches_block_on_gathered_halo_open():
    batch, M, X = small_open_case()
    L, A = oracle.batched_forward(batch, M, X, want_abs=True)
    for t in range(batch["T"]):
        Mh, Xh = gather_halo(batch, M, X, t)
        Lb = oracle.block_forward(Mh, Xh)
        sl = slice(t * SUB3, (t + 1) * SUB3)
        assert np.all(np.abs(Lb - L[:, sl]) <= 1e-13 * A[:, sl])


def test_batched_matches_block_on_gathered_halo_periodic():
    batch, M, X = synthetic.batched_config(2, 5, missing_frac=0.5)
    sel = np.array([0, 3, 7], np.int32)
    L, A = oracle.batched_forward(batch, M, X, tsel=sel, want_abs=True)
    for q, t in enumerate(sel):
        Mh, Xh = gather_halo(batch, M, X, t)
        Lb = oracle.block_forward(Mh, Xh)
        sl = slice(q * SUB3, (q + 1) * SUB3)
        assert np.all(np.abs(Lb - L[:, sl]) <= 1e-13 * A[:, sl])


def test_missing_neighbour_drops_exactly_its_pairs():
    """Knocking out a neighbour removes exactly the pairs it contributed:
    L(all) - L(all but slot) = L(self + slot) - L(self only)."""
    batch, M, X = synthetic.batched_config(2, 6)
    t, slot = 0, 4

    def run(keep):
        b = dict(batch)
        b["nbr"] = batch["nbr"].copy()
        drop = [s for s in range(27) if s not in keep]
        b["nbr"][t, drop] = -1
        return oracle.batched_forward(b, M, X, tsel=[t])

    full = run(range(27))
    miss = run([s for s in range(27) if s != slot])
    part = run([13, slot]) - run([13])
    scale = np.abs(full).max(axis=1, keepdims=True)
    assert np.all(np.abs(full - miss - part) <= 1e-13 * scale)
    assert np.abs(part).max() > 0


def _loss(batch, M, X, w):
    return float(np.sum(w * oracle.batched_forward(batch, M, X)))


def test_moment_gradient_dot_product():
    batch, M, X = small_open_case()
    w = synthetic.weights(batch["T"], 5)
    gM, gX = oracle.batched_backward(batch, M, X, w)
    rng = np.random.default_rng(8)
    V = rng.standard_normal(M.shape) * np.abs(M).max(axis=1, keepdims=True)
    l0 = _loss(batch, M, X, w)
    l1 = _loss(batch, M + V, X, w)
    lv = _loss(batch, V, X, w)          # the loss is linear in M
    dot = float(np.sum(gM * V))
    assert abs((l1 - l0) - dot) <= 1e-10 * abs(dot)
    assert abs(lv - dot) <= 1e-12 * abs(dot)


def test_position_gradient_complex_step():
    batch, M, X = small_open_case(targets=(13, 4), missing=((13, 5), (4, 14)))
    w = synthetic.weights(batch["T"], 6)
    gM, gX = oracle.batched_backward(batch, M, X, w)
    h = 1e-30
    cells = [13 * SUB3 + 7, 13 * SUB3 + 300, 4 * SUB3 + 511, 0 * SUB3 + 100, 5 * SUB3 + 3,
             14 * SUB3 + 64]
    for n, c in enumerate(cells):
        k = n % 3
        Xim = np.zeros_like(X)
        Xim[k, c] = h
        Lre, Lim = oracle.batched_forward_cs(batch, M, X, Xim)
        d = float(np.sum(w * Lim)) / h
        scale = np.abs(gX).max()
        assert abs(gX[k, c] - d) <= 1e-12 * scale + 1e-11 * abs(d), (c, k, gX[k, c], d)


def test_position_gradient_central_difference():
    batch, M, X = small_open_case(targets=(13,), missing=())
    w = synthetic.weights(batch["T"], 7)
    gM, gX = oracle.batched_backward(batch, M, X, w)
    eps = 1e-6
    for c, k in [(13 * SUB3 + 77, 0), (12 * SUB3 + 5, 2)]:
        Xp = X.copy()
        Xm = X.copy()
        Xp[k, c] += eps
        Xm[k, c] -= eps
        Lp = oracle.batched_forward(batch, M, Xp)
        Lm = oracle.batched_forward(batch, M, Xm)
        d = float(np.sum(w * (Lp - Lm))) / (2 * eps)
        assert abs(gX[k, c] - d) <= 1e-6 * np.abs(gX).max()


def test_position_gradients_sum_to_zero():
    batch, M, X = small_open_case()
    w = synthetic.weights(batch["T"], 9)
    gM, gX = oracle.batched_backward(batch, M, X, w)
    assert np.all(np.abs(gX.sum(axis=1)) <= 1e-12 * np.abs(gX).sum(axis=1))


def test_backward_selection_matches_full():
    batch, M, X = small_open_case()
    w = synthetic.weights(batch["T"], 10)
    gM, gX = oracle.batched_backward(batch, M, X, w)
    sel = np.array([26, 13, 0], np.int32)
    gMs, gXs = oracle.batched_backward(batch, M, X, w, ssel=sel)
    for q, s in enumerate(sel):
        assert np.array_equal(gMs[:, q * SUB3:(q + 1) * SUB3], gM[:, s * SUB3:(s + 1) * SUB3])
        assert np.array_equal(gXs[:, q * SUB3:(q + 1) * SUB3], gX[:, s * SUB3:(s + 1) * SUB3])


def test_unreferenced_store_subgrid_has_zero_gradient():
    batch, M, X = small_open_case(targets=(0,), missing=())
    w = synthetic.weights(batch["T"], 11)
    gM, gX = oracle.batched_backward(batch, M, X, w, ssel=[26])
    assert np.all(gM == 0) and np.all(gX == 0)


@pytest.mark.parametrize("bad", ["self", "range"])
def test_invalid_descriptor_rejected(bad):
    batch, M, X = small_open_case(targets=(13,), missing=())
    nbr = batch["nbr"].copy()
    if bad == "self":
        nbr[0, 13] = 12
    else:
        nbr[0, 3] = 27
    b = dict(batch)
    b["nbr"] = nbr
    with pytest.raises(ValueError):
        oracle.batched_forward(b, M, X)
