"""Pins of the oracle's coarse substitute for missing neighbours: a coarse
cell J (the parent of 2x2x2 missing fine cells) stands in for its children
when all of them would be in the target's stencil. CPU only.

The references are fine-level sums computed with the oracle's single-block
form on purpose-built halos that hold masses only in the children of the
coarse cells included for one target cell -- an independent route through
the stencil test, the halo geometry and the periodic shifts:
  * children that are point masses at one common point per coarse cell give
    exactly the same field as the coarse cell (the pin of the inclusion rule,
    the coarse-cell geometry and the shifts);
  * children spread around that point by a scale a differ from the coarse
    cell by the truncated expansion, an error falling like a^(4-n) in the
    outputs of order n (the pin of the coarse moments' use)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import oracle  # noqa: E402
import synthetic  # noqa: E402

SUB3 = 512
N = 4  # 4^3 store, 2^3 parents


def _children_groups():
    """Store-local cell ids (64, 8) of the 2x2x2 cells under each parent-level
    cell position within a sub-grid (group g = gx + 4 gy + 16 gz)."""
    out = np.zeros((64, 8), np.int64)
    for g in range(64):
        gx, gy, gz = g % 4, (g // 4) % 4, g // 16
        k = 0
        for c in (0, 1):
            for b in (0, 1):
                for a in (0, 1):
                    out[g, k] = (2 * gx + a) + 8 * (2 * gy + b) + 64 * (2 * gz + c)
                    k += 1
    return out


def _store(spread, seed=71):
    """Fine store of N^3 sub-grids: in every group of 8 children, point masses
    (no moments) at a common point, or at that point + spread * offsets."""
    rng = np.random.default_rng(seed)
    S = N ** 3
    M = np.zeros((20, S * SUB3))
    X = np.zeros((3, S * SUB3))
    groups = _children_groups()
    off = rng.uniform(-1, 1, (S, 64, 8, 3))
    for s in range(S):
        sx, sy, sz = s % N, (s // N) % N, s // (N * N)
        for g in range(64):
            gx, gy, gz = g % 4, (g // 4) % 4, g // 16
            centre = np.array([8 * sx + 2 * gx + 1.0, 8 * sy + 2 * gy + 1.0, 8 * sz + 2 * gz + 1.0])
            centre += rng.uniform(-0.2, 0.2, 3)
            cells = s * SUB3 + groups[g]
            X[:, cells] = (centre[None, :] + spread * off[s, g]).T
            M[0, cells] = rng.uniform(0.5, 1.5, 8)
    return M, X


def _case(periodic, seed=72):
    batch = synthetic.lattice_batch(N, periodic=periodic)
    batch = synthetic.apply_missing(batch, 0.6, synthetic._rng(seed))
    coarse, octant = synthetic.coarse_tables(N, batch)
    assert (coarse >= 0).sum() > 10
    return batch, coarse, octant


def _fine_reference(batch, M, X, t, ci, coarse):
    """Sum over the children of the coarse cells included for target cell ci of
    target t, via the single-block oracle on a halo holding only them."""
    full = synthetic.lattice_batch(N, periodic=batch.get("period") is not None)
    li = (ci % 8, (ci // 8) % 8, ci // 64)
    hi = (li[0] + 8, li[1] + 8, li[2] + 8)
    Mh = np.zeros((20, 13824))
    Xh = np.zeros((3, 13824))
    hidx = np.arange(13824)
    Xh[0], Xh[1], Xh[2] = hidx % 24 + 1e6, (hidx // 24) % 24, hidx // 576   # massless, far away
    tg = batch["tgt"][t]
    # the target's own cells (positions only)
    loc = np.arange(SUB3)
    lx, ly, lz = loc % 8, (loc // 8) % 8, loc // 64
    own = (8 + lx) + 24 * (8 + ly) + 576 * (8 + lz)
    Xh[:, own] = X[:, tg * SUB3 + loc]
    included = 0
    for slot in range(27):
        if coarse[t, slot] < 0:
            continue
        b = full["nbr"][t, slot]
        so = (slot % 3, (slot // 3) % 3, slot // 9)
        sh = np.zeros(3)
        if batch.get("shift") is not None:
            sh = batch["shift"][t, slot].astype(np.float64) * batch["period"]
        for J in range(64):
            cj = (J % 4, (J // 4) % 4, J // 16)
            kids = []
            for n in range(8):
                d = (n & 1, (n >> 1) & 1, n >> 2)
                hj = tuple(8 * so[k] + 2 * cj[k] + d[k] for k in range(3))
                kids.append(hj)
            if not all(oracle.in_stencil(hi, hj) for hj in kids):
                continue
            included += 1
            for hj in kids:
                lj = [hj[k] - 8 * so[k] for k in range(3)]
                cell = b * SUB3 + lj[0] + 8 * lj[1] + 64 * lj[2]
                h = hj[0] + 24 * hj[1] + 576 * hj[2]
                Mh[:, h] = M[:, cell]
                Xh[:, h] = X[:, cell] + sh
    L = oracle.block_forward(Mh, Xh)
    return L[:, ci], included


@pytest.mark.parametrize("periodic,full", [(False, False), (True, False), (True, True)])
def test_coincident_children_equal_their_coarse_cell(periodic, full):
    """Point masses at one point: the coarse cell carries the mass alone, so
    both truncations give the fine sum up to rounding."""
    batch, coarse, octant = _case(periodic)
    M, X = _store(0.0)
    Mp, Xp = oracle.m2m(synthetic.octree_children(N), M, X)
    ts = [t for t in range(batch["T"]) if (coarse[t] >= 0).any()][:3]
    got, A = oracle.coarse_fine(batch, X, coarse, octant, Mp, Xp, tsel=ts, want_abs=True, full=full)
    rng = np.random.default_rng(5)
    for q, t in enumerate(ts):
        for ci in rng.choice(SUB3, 4, replace=False):
            ref, included = _fine_reference(batch, M, X, t, ci, coarse)
            assert included > 0
            col = q * SUB3 + ci
            assert np.all(np.abs(got[:, col] - ref) <= 1e-13 * A[:, col]), (t, ci)


@pytest.mark.parametrize("full", [False, True])
def test_spread_children_converge_at_the_truncation_order(full):
    """Children spread by a: the coarse moments of order k grow like a^k. The
    total-order substitute drops moments of order 4 - n from the outputs of
    order n (error ~ a^(4-n)); the full one keeps every moment up to order 3
    in every output (error ~ a^4 in all of them)."""
    batch, coarse, octant = _case(False, seed=73)
    t = next(t for t in range(batch["T"]) if (coarse[t] >= 0).sum() >= 2)
    M, X = _store(0.1)
    ci = next(c for c in range(0, SUB3, 37) if _fine_reference(batch, M, X, t, c, coarse)[1] > 0)
    errs = []
    for a in (0.2, 0.1, 0.05):
        M, X = _store(a)
        Mp, Xp = oracle.m2m(synthetic.octree_children(N), M, X)
        got = oracle.coarse_fine(batch, X, coarse, octant, Mp, Xp, tsel=[t], full=full)[:, ci]
        ref, _ = _fine_reference(batch, M, X, t, ci, coarse)
        errs.append(np.abs(got - ref))
    for order, comps in enumerate(([0], [1, 2, 3], list(range(4, 10)), list(range(10, 20)))):
        e = [float(np.max(x[comps])) for x in errs]
        # (the dipole about the centre of mass is zero: order-3 outputs of the
        # total order lose the quadrupole first)
        rate = 2.0 ** (4 if full else max(4 - order, 2))
        assert e[1] < e[0] / (0.6 * rate) and e[2] < e[1] / (0.6 * rate), (order, e)
        # and not faster: the rate is that of the first omitted order
        assert e[1] > e[0] / (1.6 * rate) and e[2] > e[1] / (1.6 * rate), (order, e)


def test_arguments_are_validated():
    batch, coarse, octant = _case(False)
    M, X = _store(0.0)
    Mp, Xp = oracle.m2m(synthetic.octree_children(N), M, X)
    t, s = np.argwhere(batch["nbr"] >= 0)[0]
    bad = coarse.copy()
    bad[t, s] = 0                      # a present neighbour cannot have a substitute
    with pytest.raises(ValueError):
        oracle.coarse_fine(batch, X, bad, octant, Mp, Xp, tsel=[0])
    bad_o = octant.copy()
    bad_o[coarse >= 0] = 9
    with pytest.raises(ValueError):
        oracle.coarse_fine(batch, X, coarse, bad_o, Mp, Xp, tsel=[0])
    z = oracle.coarse_fine(batch, X, coarse, octant, np.zeros_like(Mp), Xp, tsel=[0, 1])
    assert np.all(z == 0.0)
