"""Pins of the oracle's tree passes around the interaction -- the upward pass
(M2M / P2M), the downward pass (L2L) and the local evaluation of forces and
energy -- against facts fixed by mathematics: moments summed directly over
point masses, exact re-expansion of cubic polynomials, far-field closed
forms, Newton's third law and the symmetry of the pair energy. CPU only."""
import itertools
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import oracle  # noqa: E402
import synthetic  # noqa: E402
from symbolic import EXP3, EXP4, green_mp  # noqa: E402

SUB3 = 512


def fact(e):
    return math.factorial(e[0]) * math.factorial(e[1]) * math.factorial(e[2])


def point_moments(x, m, centre):
    """Raw moments of point masses about `centre` (the definition)."""
    d = x - centre
    return np.array([np.sum(m * d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** c) for a, b, c in EXP3])


def child_cells_of_parent_cell(pc):
    """(octant, child-local cell ids) of the 2x2x2 child cells under parent cell pc."""
    X, Y, Z = pc % 8, (pc // 8) % 8, pc // 64
    o = X // 4 + 2 * (Y // 4) + 4 * (Z // 4)
    cells = []
    for c, b, a in itertools.product((0, 1), repeat=3):
        lx, ly, lz = 2 * (X % 4) + a, 2 * (Y % 4) + b, 2 * (Z % 4) + c
        cells.append(lx + 8 * ly + 64 * lz)
    return o, cells


def random_children(Sp, rng):
    """Child node ids: a permutation of 0..8*Sp-1 (each child node has one parent)."""
    return rng.permutation(8 * Sp).astype(np.int32).reshape(Sp, 8)


def leaf_points(Sc, rng, per_cell=4):
    """Point masses inside every child cell (global cell index = store index)."""
    ncell = Sc * SUB3
    base = rng.uniform(0, 50, (ncell, 3))
    x = base[:, None, :] + rng.uniform(-0.4, 0.4, (ncell, per_cell, 3))
    m = rng.uniform(0.1, 2.0, (ncell, per_cell))
    m[rng.random(ncell) < 0.05] = 0.0          # some empty cells
    return x, m


def cell_data(x, m):
    """P2M by the definition: mass, centre of mass, raw moments about it."""
    n = x.shape[0]
    M = np.zeros((20, n))
    X = np.zeros((3, n))
    for i in range(n):
        tot = m[i].sum()
        c = (m[i][:, None] * x[i]).sum(0) / tot if tot > 0 else x[i].mean(0)
        X[:, i] = c
        M[:, i] = point_moments(x[i], m[i], c)
    return M, X


@pytest.fixture(scope="module")
def two_level():
    rng = np.random.default_rng(12)
    Sp = 2
    ch = random_children(Sp, rng)
    x, m = leaf_points(8 * Sp, rng)
    Mc, Xc = cell_data(x, m)
    return ch, x, m, Mc, Xc


def test_m2m_equals_moments_of_all_points(two_level):
    ch, x, m, Mc, Xc = two_level
    Mp, Xp = oracle.m2m(ch, Mc, Xc)
    rng = np.random.default_rng(1)
    for p in range(ch.shape[0]):
        for pc in rng.choice(SUB3, 40, replace=False):
            o, cells = child_cells_of_parent_cell(pc)
            idx = ch[p, o] * SUB3 + np.array(cells)
            xs = x[idx].reshape(-1, 3)
            ms = m[idx].reshape(-1)
            tot = ms.sum()
            centre = (ms[:, None] * xs).sum(0) / tot if tot > 0 else Xc[:, idx].mean(axis=1)
            ref = point_moments(xs, ms, centre)
            col = p * SUB3 + pc
            assert np.allclose(Xp[:, col], centre, rtol=0, atol=1e-12)
            # scale of order n: sum of the term magnitudes m |x - X|^n (the
            # dipole about the centre of mass is itself rounding noise)
            dist = np.abs(xs - centre).max(axis=1)
            for n in range(4):
                sel = [a for a in range(20) if sum(EXP3[a]) == n]
                scale = max(1e-300, np.abs(ref[sel]).max(), float(np.sum(ms * dist ** n)))
                assert np.all(np.abs(Mp[sel, col] - ref[sel]) <= 1e-12 * scale), (p, pc, n)


def test_m2m_of_point_masses_is_p2m():
    """Children that are point masses (mass only): the parent's moments are
    sum m_c (X_c - X_p)^b exactly (P2M)."""
    rng = np.random.default_rng(3)
    ch = random_children(1, rng)
    Mc = np.zeros((20, 8 * SUB3))
    Mc[0] = rng.uniform(0.5, 1.5, 8 * SUB3)
    Xc = rng.uniform(0, 10, (3, 8 * SUB3))
    Mp, Xp = oracle.m2m(ch, Mc, Xc)
    for pc in range(0, SUB3, 37):
        o, cells = child_cells_of_parent_cell(pc)
        idx = ch[0, o] * SUB3 + np.array(cells)
        ref = point_moments(Xc[:, idx].T, Mc[0, idx], Xp[:, pc])
        assert np.allclose(Mp[:, pc], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
        # dipole about the centre of mass vanishes
        assert np.all(np.abs(Mp[1:4, pc]) <= 1e-13 * Mp[0, pc] * 10)


def test_m2m_conserves_mass_and_handles_empty_cells():
    rng = np.random.default_rng(4)
    ch = random_children(1, rng)
    Mc = np.zeros((20, 8 * SUB3))
    Xc = rng.uniform(0, 10, (3, 8 * SUB3))
    Mc[0, : 4 * SUB3] = rng.uniform(0, 1, 4 * SUB3)
    Mp, Xp = oracle.m2m(ch, Mc, Xc)
    assert np.isclose(Mp[0].sum(), Mc[0].sum(), rtol=1e-14)
    empty = Mp[0] == 0
    assert empty.any()
    for pc in np.nonzero(empty)[0][:20]:
        o, cells = child_cells_of_parent_cell(pc)
        idx = ch[0, o] * SUB3 + np.array(cells)
        assert np.allclose(Xp[:, pc], Xc[:, idx].mean(axis=1), rtol=1e-15)
        assert np.all(Mp[:, pc] == 0.0)


def test_m2m_two_levels_equals_direct():
    """Grandparent moments by two upward passes = moments of all 64 points."""
    rng = np.random.default_rng(5)
    ch_top = random_children(1, rng)            # grandparent -> 8 parents
    ch_mid = random_children(8, rng)            # 8 parents -> 64 leaves
    x, m = leaf_points(64, rng, per_cell=2)
    Mc, Xc = cell_data(x, m)
    Mmid, Xmid = oracle.m2m(ch_mid, Mc, Xc)
    Mtop, Xtop = oracle.m2m(ch_top, Mmid, Xmid)
    for pc in (0, 77, 300, 511):
        o, cells = child_cells_of_parent_cell(pc)
        pts_x, pts_m = [], []
        for cmid in cells:
            p_mid = ch_top[0, o]
            o2, cells2 = child_cells_of_parent_cell(cmid)
            idx = ch_mid[p_mid, o2] * SUB3 + np.array(cells2)
            pts_x.append(x[idx].reshape(-1, 3))
            pts_m.append(m[idx].reshape(-1))
        xs, ms = np.concatenate(pts_x), np.concatenate(pts_m)
        centre = (ms[:, None] * xs).sum(0) / ms.sum()
        ref = point_moments(xs, ms, centre)
        dist = np.abs(xs - centre).max(axis=1)
        for n in range(4):
            sel = [a for a in range(20) if sum(EXP3[a]) == n]
            scale = max(np.abs(ref[sel]).max(), float(np.sum(ms * dist ** n)))
            assert np.all(np.abs(Mtop[sel, pc] - ref[sel]) <= 1e-12 * scale)


def _cubic_derivatives(c, centre, at):
    """All derivatives up to order 3 at `at` of phi(x) = sum_a c_a (x-centre)^a / a!,
    by differentiating the monomials directly."""
    d = at - centre
    out = np.zeros(20)
    for a, ea in enumerate(EXP3):          # derivative order a
        s = 0.0
        for b, eb in enumerate(EXP3):      # monomial (x-centre)^b / b!
            if any(eb[k] < ea[k] for k in range(3)):
                continue
            r = [eb[k] - ea[k] for k in range(3)]
            coef = c[b] / fact(eb)
            for k in range(3):
                coef *= math.factorial(eb[k]) / math.factorial(r[k])
            s += coef * d[0] ** r[0] * d[1] ** r[1] * d[2] ** r[2]
        out[a] = s
    return out


def test_l2l_is_exact_for_cubics():
    rng = np.random.default_rng(6)
    ch = random_children(1, rng)
    Lp = rng.standard_normal((20, SUB3))
    Xp = rng.uniform(0, 4, (3, SUB3))
    Xc = rng.uniform(0, 4, (3, 8 * SUB3))
    L0 = rng.standard_normal((20, 8 * SUB3))
    Lc = oracle.l2l(ch, Lp, Xp, Xc, L0)
    for pc in range(0, SUB3, 29):
        o, cells = child_cells_of_parent_cell(pc)
        for cell in cells:
            j = ch[0, o] * SUB3 + cell
            ref = _cubic_derivatives(Lp[:, pc], Xp[:, pc], Xc[:, j])
            assert np.allclose(Lc[:, j] - L0[:, j], ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_l2l_far_field_error_rate(order):
    """Parent expansion of a far point mass, shifted by d: output order n
    deviates from the exact derivative at the child centre by O(d^(4-n))."""
    sel = [a for a in range(20) if sum(EXP3[a]) == order]
    xs = np.array([17.0, -9.0, 11.0])
    errs = []
    for h in (0.2, 0.1, 0.05):
        ch = np.arange(8, dtype=np.int32)[None, :]
        Xp = np.zeros((3, SUB3))
        Lp = np.tile(np.array(oracle.green(Xp[:, 0] - xs, 3))[:, None], (1, SUB3))
        Xc = np.zeros((3, 8 * SUB3))
        Xc[:, 0] = [h, -0.7 * h, 0.4 * h]
        Lc = oracle.l2l(ch, Lp, Xp, Xc, np.zeros((20, 8 * SUB3)))
        exact = np.array([float(v) for v in green_mp(Xc[:, 0] - xs, 3)])
        errs.append(np.max(np.abs(Lc[sel, 0] - exact[sel])) / np.max(np.abs(exact[sel])))
    want = 2.0 ** (4 - order)
    for e0, e1 in zip(errs, errs[1:]):
        assert 0.7 * want <= e0 / e1 <= 1.4 * want, (order, errs)


def test_evaluate_point_mass_closed_form():
    rng = np.random.default_rng(7)
    N = 100
    M = np.zeros((20, N))
    M[0] = rng.uniform(0.5, 2, N)
    L = rng.standard_normal((20, N))
    F, W = oracle.evaluate(M, L)
    assert np.allclose(F, -M[0] * L[1:4], rtol=1e-15, atol=0)
    assert np.allclose(W, 0.5 * M[0] * L[0], rtol=1e-15, atol=0)


def test_evaluate_pair_newton_and_energy_symmetry():
    """Two cells that see only each other: F_i = -F_j, and each cell's share
    of the pair energy is the same (the truncated pair energy is symmetric)."""
    rng = np.random.default_rng(8)
    g = synthetic._halo_coords()
    X = (g + 0.5).T.astype(np.float64).copy()
    M = np.zeros((20, 24 ** 3))
    hi, hj = (9, 10, 8), (14, 12, 13)
    assert oracle.in_stencil(hi, hj)
    for h in (hi, hj):
        idx = h[0] + 24 * h[1] + 576 * h[2]
        xs = X[:, idx] + 0.3 * rng.uniform(-1, 1, (6, 3))
        ms = rng.uniform(0.5, 1.5, 6)
        c = (ms[:, None] * xs).sum(0) / ms.sum()
        M[:, idx] = point_moments(xs, ms, c)
        X[:, idx] = c
    L = oracle.block_forward(M, X)
    ti = (hi[0] - 8) + 8 * (hi[1] - 8) + 64 * (hi[2] - 8)
    tj = (hj[0] - 8) + 8 * (hj[1] - 8) + 64 * (hj[2] - 8)
    ii = hi[0] + 24 * hi[1] + 576 * hi[2]
    jj = hj[0] + 24 * hj[1] + 576 * hj[2]
    F, W = oracle.evaluate(M[:, [ii, jj]], L[:, [ti, tj]])
    assert np.all(np.abs(F[:, 0] + F[:, 1]) <= 1e-14 * np.abs(F).max())
    assert abs(W[0] - W[1]) <= 1e-14 * abs(W[0])


def test_wrappers_accept_non_contiguous_inputs():
    """Column-gathered (Fortran-ordered) arrays give the same results as their
    C-ordered copies."""
    rng = np.random.default_rng(14)
    ch = random_children(1, rng)
    cols = rng.permutation(8 * SUB3)
    Lc = rng.standard_normal((20, 8 * SUB3))[:, cols]
    Xc = rng.uniform(0, 8, (3, 8 * SUB3))[:, cols]
    Lp = rng.standard_normal((20, SUB3))
    Xp = rng.uniform(0, 8, (3, SUB3))
    assert not Lc.flags["C_CONTIGUOUS"]
    a = oracle.l2l(ch, Lp, Xp, Xc, Lc)
    b = oracle.l2l(ch, Lp, Xp, np.ascontiguousarray(Xc), np.ascontiguousarray(Lc))
    assert np.array_equal(a, b)
    F1, W1 = oracle.evaluate(Lc, Lc)
    F2, W2 = oracle.evaluate(np.ascontiguousarray(Lc), np.ascontiguousarray(Lc))
    assert np.array_equal(F1, F2) and np.array_equal(W1, W2)
