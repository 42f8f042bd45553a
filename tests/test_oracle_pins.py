"""Pins of the CPU oracle's forward sum against facts fixed by mathematics,
independent of the oracle's own code: symbolic derivatives, Laplace's
equation, lattice-point counts, closed forms for one source, direct
summation over point masses, Newton's third law, symmetries and 30-digit
arithmetic. CPU only."""
import itertools
import math
import os
import sys

import mpmath
import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import oracle  # noqa: E402
import synthetic  # noqa: E402
from symbolic import EXP3, EXP4, _derivative_functions, green_mp  # noqa: E402

HALO = 24
H3 = HALO ** 3


def comp_index(e):
    return EXP4.index(tuple(e))


def halo_index(x, y, z):
    return x + HALO * y + HALO * HALO * z


def target_index(x, y, z):
    """central cell (halo coords 8..15) -> output column"""
    return (x - 8) + 8 * (y - 8) + 64 * (z - 8)


# ---------------------------------------------------------------------------
# Green's function derivatives
# ---------------------------------------------------------------------------
def test_component_order_is_graded_lex_x_major():
    names = ["1", "x", "y", "z", "xx", "xy", "xz", "yy", "yz", "zz",
             "xxx", "xxy", "xxz", "xyy", "xyz", "xzz", "yyy", "yyz", "yzz", "zzz"]
    for g, name in enumerate(names):
        e = oracle.multi_index(g)
        want = (name.count("x"), name.count("y"), name.count("z")) if name != "1" else (0, 0, 0)
        assert e == want
    assert [oracle.multi_index(g) for g in range(35)] == EXP4


@pytest.mark.parametrize("r", [(1.3, -2.1, 0.7), (-5.5, 0.25, 3.0), (0.0, 0.0, 4.5),
                               (8.1, 7.9, -8.3)])
def test_green_matches_symbolic_derivatives(r):
    ref = [float(v) for v in green_mp(r, 4)]
    got = oracle.green(r, 4)
    for n in range(5):
        sel = [g for g, e in enumerate(EXP4) if sum(e) == n]
        scale = max(abs(ref[g]) for g in sel)
        for g in sel:
            assert abs(got[g] - ref[g]) <= 4e-15 * scale, (n, EXP4[g], got[g], ref[g])


def test_green_is_harmonic():
    rng = np.random.default_rng(7)
    for _ in range(20):
        r = rng.uniform(-9, 9, 3)
        if np.dot(r, r) < 16:
            continue
        G = oracle.green(r, 4)
        for e in EXP3[:10]:   # |gamma| <= 2, so gamma + 2 e_k has order <= 4
            tr = sum(G[comp_index(np.add(e, 2 * np.eye(3, dtype=int)[k]))] for k in range(3))
            n = sum(e) + 2
            scale = max(abs(G[g]) for g in range(35) if sum(EXP4[g]) == n)
            assert abs(tr) <= 1e-14 * scale


# ---------------------------------------------------------------------------
# Stencil
# ---------------------------------------------------------------------------
def _lattice_points(r2max):
    rng = range(-5, 6)
    return sum(1 for p in itertools.product(rng, rng, rng) if p[0] ** 2 + p[1] ** 2 + p[2] ** 2 <= r2max)


@pytest.mark.parametrize("parity", list(itertools.product((0, 1), repeat=3)))
def test_stencil_size_is_seven_parent_balls(parity):
    """Sources are the 8 children of the N parent cells within distance 4 of
    the target's parent, minus the N near cells (|d| <= 4): 7 N sources,
    with N the number of integer points in a ball of radius 4."""
    hi = np.array([8, 8, 8]) + np.array(parity)
    n = 0
    for hj in itertools.product(range(HALO), repeat=3):
        n += oracle.in_stencil(hi, hj)
    N = _lattice_points(16)
    assert N == 257
    assert n == 7 * N == 1799


def test_stencil_is_symmetric_and_reflection_invariant():
    rng = np.random.default_rng(3)
    for _ in range(3000):
        i = rng.integers(0, 24, 3)
        j = rng.integers(0, 24, 3)
        a = oracle.in_stencil(i, j)
        assert a == oracle.in_stencil(j, i)
        assert a == oracle.in_stencil(23 - i, 23 - j)
        assert a == oracle.in_stencil(i[[1, 2, 0]], j[[1, 2, 0]])
        # even lattice translations leave the criterion unchanged
        s = 2 * rng.integers(-2, 3, 3)
        if np.all((i + s >= 0) & (i + s < 24) & (j + s >= 0) & (j + s < 24)):
            assert a == oracle.in_stencil(i + s, j + s)


# ---------------------------------------------------------------------------
# Closed forms for a single source
# ---------------------------------------------------------------------------
def _empty_block(nm):
    g = synthetic._halo_coords()
    X = (g + 0.5).T.astype(np.float64).copy()
    return np.zeros((nm, H3)), X


def test_single_monopole_source_closed_form():
    M, X = _empty_block(1)
    j = halo_index(3, 11, 14)
    M[0, j] = 1.7
    X[:, j] += [0.07, -0.03, 0.09]
    L = oracle.block_forward(M, X)
    ti = (8, 8, 13)
    hit = 0
    for tx, ty, tz in itertools.product(range(8, 16), repeat=3):
        col = target_index(tx, ty, tz)
        i = halo_index(tx, ty, tz)
        inside = oracle.in_stencil((tx, ty, tz), (3, 11, 14))
        if not inside:
            assert np.all(L[:, col] == 0.0)
            continue
        hit += 1
        if (tx, ty, tz) != ti and hit > 5:
            continue
        ref = [1.7 * float(v) for v in green_mp(X[:, i] - X[:, j], 3)]
        for a in range(20):
            n = sum(EXP3[a])
            scale = max(abs(ref[b]) for b in range(20) if sum(EXP3[b]) == n)
            assert abs(L[a, col] - ref[a]) <= 4e-15 * scale
    assert hit > 0


def test_multipole_with_only_mass_equals_monopole():
    b = synthetic.monopole_block(5)
    M = np.zeros((20, H3))
    M[0] = b["mass"]
    L1 = oracle.block_forward(b["mass"][None], b["com"])
    L20 = oracle.block_forward(M, b["com"])
    assert np.array_equal(L1, L20)


# ---------------------------------------------------------------------------
# Direct summation over point masses: the expansion error shrinks at the
# rate of the first omitted order
# ---------------------------------------------------------------------------
def _moments_about(xc, mc, centre):
    d = xc - centre
    return np.array([(mc * d[:, 0] ** a * d[:, 1] ** b * d[:, 2] ** c).sum() for a, b, c in EXP3])


def _direct(xt, xc, mc):
    out = np.zeros(20)
    for x, m in zip(xc, mc):
        out += m * oracle.green(xt - x, 3)
    return out


def _expansion_error(scale, mmax, rng_seed=11):
    rng = np.random.default_rng(rng_seed)
    M, X = _empty_block(20)
    j = halo_index(2, 12, 12)        # source cell
    t = (9, 12, 12)                  # target cell, d = (7, 0, 0): inside the stencil
    assert oracle.in_stencil(t, (2, 12, 12))
    centre = X[:, j] + np.array([0.05, -0.04, 0.03])   # expansion centre, not the COM
    xc = centre + scale * rng.uniform(-1, 1, (8, 3))
    mc = rng.uniform(0.5, 1.5, 8)
    M[:, j] = _moments_about(xc, mc, centre)
    X[:, j] = centre
    L = oracle.block_forward(M, X, mmax=mmax)[:, target_index(*t)]
    xt = X[:, halo_index(*t)]
    ref = _direct(xt, xc, mc)
    return L, ref


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_expansion_error_scales_with_omitted_order(order):
    """With total-order truncation 3, output order n keeps source moments up
    to order 3-n: halving the source size must divide the error by 2^(4-n)."""
    sel = [a for a in range(20) if sum(EXP3[a]) == order]
    errs = []
    for s in (0.1, 0.05, 0.025):
        L, ref = _expansion_error(s, 3)
        errs.append(np.max(np.abs(L[sel] - ref[sel])) / np.max(np.abs(ref[sel])))
    want = 2.0 ** (4 - order)
    for e0, e1 in zip(errs, errs[1:]):
        assert 0.75 * want <= e0 / e1 <= 1.3 * want, (order, errs)


@pytest.mark.parametrize("mmax", [0, 1, 2])
def test_potential_error_falls_with_moment_order(mmax):
    """L_0 keeping moments up to order p has an error of order (a/r)^(p+1)."""
    errs = []
    for s in (0.1, 0.05, 0.025):
        L, ref = _expansion_error(s, mmax)
        errs.append(abs(L[0] - ref[0]) / abs(ref[0]))
    want = 2.0 ** (mmax + 1)
    for e0, e1 in zip(errs, errs[1:]):
        assert 0.75 * want <= e0 / e1 <= 1.3 * want, (mmax, errs)
    # and each added order reduces the error at fixed size
    Lp, ref = _expansion_error(0.2, mmax)
    Lq, _ = _expansion_error(0.2, mmax + 1)
    assert abs(Lq[0] - ref[0]) < abs(Lp[0] - ref[0])


def test_eight_symmetric_children_equal_monopole():
    """8 equal children at (+-a,+-a,+-a): isotropic quadrupole, no dipole or
    octupole, so the multipole sum equals the monopole sum (Laplace)."""
    rng = np.random.default_rng(2)
    g = synthetic._halo_coords()
    X = (g + 0.5 + rng.uniform(-0.1, 0.1, g.shape)).T.copy()
    m = rng.uniform(0.5, 1.5, H3)
    a = 0.23
    oct_ = np.array(list(itertools.product((-a, a), repeat=3)))
    M = np.zeros((20, H3))
    for k, (p, q, r) in enumerate(EXP3):
        M[k] = (m / 8) * np.sum(oct_[:, 0] ** p * oct_[:, 1] ** q * oct_[:, 2] ** r)
    Lm, A = oracle.block_forward(M, X, want_abs=True)
    L0 = oracle.block_forward(m[None], X)
    assert np.all(np.abs(Lm - L0) <= 1e-13 * A + 1e-300)


# ---------------------------------------------------------------------------
# Exact identities of the truncated sum
# ---------------------------------------------------------------------------
def test_laplace_trace_of_outputs():
    b = synthetic.multipole_block(1002)
    L, A = oracle.block_forward(b["M"], b["com"], want_abs=True)
    for e in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        idx = [comp_index(np.add(e, 2 * np.eye(3, dtype=int)[k])) for k in range(3)]
        tr = L[idx[0]] + L[idx[1]] + L[idx[2]]
        scale = A[idx[0]] + A[idx[1]] + A[idx[2]]
        assert np.all(np.abs(tr) <= 1e-13 * scale)


def _force(M, L):
    """F_k = - sum_{|a|<=2} M_a / a! L_{a+e_k}: force on a cell's point masses
    from the local expansion, to the order the truncation keeps."""
    F = np.zeros((3, L.shape[1]))
    for a, e in enumerate(EXP3[:10]):
        fact = math.factorial(e[0]) * math.factorial(e[1]) * math.factorial(e[2])
        for k in range(3):
            F[k] -= M[a] / fact * L[comp_index(np.add(e, np.eye(3, dtype=int)[k]))]
    return F


def test_newton_third_law_single_pair():
    rng = np.random.default_rng(4)
    M, X = _empty_block(20)
    i = halo_index(8, 9, 10)
    j = halo_index(13, 11, 9)
    assert oracle.in_stencil((8, 9, 10), (13, 11, 9))
    for c in (i, j):
        xc = X[:, c] + 0.2 * rng.uniform(-1, 1, (8, 3))
        mc = rng.uniform(0.5, 1.5, 8)
        com = (mc[:, None] * xc).sum(0) / mc.sum()
        M[:, c] = _moments_about(xc, mc, com)
        X[:, c] = com
    L = oracle.block_forward(M, X)
    ci, cj = target_index(8, 9, 10), target_index(13, 11, 9)
    F = _force(M[:, [i, j]], L[:, [ci, cj]])
    assert np.all(np.abs(F[:, 0] + F[:, 1]) <= 1e-14 * np.abs(F[:, 0]).max())
    assert np.abs(F[:, 0]).max() > 1e-6


def test_newton_third_law_closed_domain():
    """Every cell is a target and availability is symmetric: the total force
    vanishes (to rounding)."""
    batch, M, X = synthetic.batched_config(2, 77, periodic=False)
    L = oracle.batched_forward(batch, M, X)
    F = _force(M, L)
    tot = F.sum(axis=1)
    assert np.all(np.abs(tot) <= 1e-13 * np.abs(F).sum(axis=1))


def test_translation_invariance():
    b = synthetic.multipole_block(1002)
    L, A = oracle.block_forward(b["M"], b["com"], want_abs=True)
    Lt = oracle.block_forward(b["M"], b["com"] + np.array([[0.37], [-0.21], [0.5]]))
    assert np.all(np.abs(Lt - L) <= 1e-12 * A)


def test_reflection_and_permutation_equivariance():
    b = synthetic.multipole_block(1002)
    M, X = b["M"], b["com"]
    L, A = oracle.block_forward(M, X, want_abs=True)
    idx = np.arange(H3)
    x, y, z = idx % 24, (idx // 24) % 24, idx // 576
    # reflection x -> 24 - x about the block centre
    src = halo_index(23 - x, y, z)
    Mr = M[:, src] * np.array([(-1.0) ** e[0] for e in EXP3])[:, None]
    Xr = X[:, src].copy()
    Xr[0] = 24.0 - Xr[0]
    Lr = oracle.block_forward(Mr, Xr)
    t = np.arange(512)
    tx, ty, tz = t % 8, (t // 8) % 8, t // 64
    back = (7 - tx) + 8 * ty + 64 * tz
    want = L[:, back] * np.array([(-1.0) ** e[0] for e in EXP3])[:, None]
    assert np.all(np.abs(Lr - want) <= 1e-13 * A[:, back])
    # cyclic axis permutation P(x, y, z) = (y, z, x): the new cell n holds the
    # old cell o with P(o) = n, i.e. o = (n_z, n_x, n_y); a new exponent
    # (a, b, c) is the old exponent (c, a, b), for moments and outputs alike
    old_of_new = halo_index(z, x, y)
    perm_comp = [EXP3.index((e[2], e[0], e[1])) for e in EXP3]
    Mp = M[perm_comp][:, old_of_new]
    Xp = X[[1, 2, 0]][:, old_of_new]
    Lp = oracle.block_forward(Mp, Xp)
    old_t = tz + 8 * tx + 64 * ty
    want = L[perm_comp][:, old_t]
    assert np.all(np.abs(Lp - want) <= 1e-13 * A[perm_comp][:, old_t])


def test_thirty_digit_sum():
    """One target cell summed over its 1799 sources in 30-digit arithmetic,
    with derivatives from symbolic differentiation."""
    b = synthetic.multipole_block(1002)
    M, X = b["M"], b["com"]
    L, A = oracle.block_forward(M, X, want_abs=True)
    coef = []
    for e in EXP3:
        fac = math.factorial(e[0]) * math.factorial(e[1]) * math.factorial(e[2])
        coef.append(mpmath.mpf((-1) ** sum(e)) / fac)
    terms = [(a, bb, comp_index(np.add(EXP3[a], EXP3[bb])))
             for a in range(20) for bb in range(20) if sum(EXP3[a]) + sum(EXP3[bb]) <= 3]
    fns = _derivative_functions()[:20]
    for t in [(8, 8, 8), (13, 10, 15)]:
        i = halo_index(*t)
        with mpmath.workdps(30):
            acc = [mpmath.mpf(0)] * 20
            for hj in itertools.product(range(HALO), repeat=3):
                if not oracle.in_stencil(t, hj):
                    continue
                j = halo_index(*hj)
                r = [mpmath.mpf(float(X[k, i])) - mpmath.mpf(float(X[k, j])) for k in range(3)]
                G = [f(*r) for f in fns]
                for a, bb, ab in terms:
                    acc[a] += coef[bb] * mpmath.mpf(float(M[bb, j])) * G[ab]
        col = target_index(*t)
        for a in range(20):
            assert abs(L[a, col] - float(acc[a])) <= 2e-14 * A[a, col]
