"""Pins of the oracle's full truncation (every output order |alpha| <= 3 keeps
every source moment |beta| <= 3, so derivatives of G to order 6), against
facts fixed by mathematics and independent of its code: symbolic
derivatives to order 6 (sympy, 30 digits), the order <= 4 closed forms
written with Kronecker deltas, Laplace's equation for the derivatives and
the outputs, mass-only sources (where both truncations coincide), the
batched form against the single-block form on the gathered halo, and direct
summation over point masses, whose error must now fall like a^4 for every
output order (the total-order truncation: like a^(4-n)). CPU only.

Planted mistakes each fail one of these: a wrong sign or double factorial
in the general closed form (symbolic), a dropped Hobson term (symbolic,
harmonic), a truncation still at |alpha| + |beta| <= 3 (direct summation),
a wrong multi-index sum table (symbolic via the single-source closed form);
in the adjoint, a transposed gradient component (complex step, central
differences) and a dropped s_beta in the moment gradient (dot product).

The adjoint (derivatives to order 7) is pinned by the dot-product test (the
loss is linear in the moments), complex-step derivatives of the full forward
(step 1e-30, no cancellation), central differences and translation
invariance (the position gradients sum to zero)."""
import itertools
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import oracle  # noqa: E402
import synthetic  # noqa: E402
from symbolic import EXP3, green_mp  # noqa: E402
from test_oracle_adjoint import gather_halo  # noqa: E402

EXP6 = synthetic.moment_exponents(6)
HALO = 24
H3 = HALO ** 3
SUB3 = 512


def halo_index(x, y, z):
    return x + HALO * y + HALO * HALO * z


def target_index(x, y, z):
    return (x - 8) + 8 * (y - 8) + 64 * (z - 8)


@pytest.mark.parametrize("r", [(1.3, -2.1, 0.7), (-5.5, 0.25, 3.0), (0.0, 0.0, 4.5),
                               (8.1, 7.9, -8.3)])
def test_general_closed_form_matches_symbolic_derivatives_to_order_6(r):
    ref = [float(v) for v in green_mp(r, 6)]
    got = oracle.green_general(r, 6)
    assert len(got) == len(EXP6) == 84
    for n in range(7):
        sel = [g for g, e in enumerate(EXP6) if sum(e) == n]
        scale = max(abs(ref[g]) for g in sel)
        for g in sel:
            assert abs(got[g] - ref[g]) <= 2e-14 * scale, (n, EXP6[g], got[g], ref[g])


@pytest.mark.parametrize("r", [(1.3, -2.1, 0.7), (-6.5, 3.25, 4.0)])
def test_general_closed_form_matches_symbolic_derivatives_at_order_7(r):
    """Order 7 enters the position gradient of the full truncation."""
    exp7 = synthetic.moment_exponents(7)
    ref = [float(v) for v in green_mp(r, 7)]
    got = oracle.green_general(r, 7)
    sel = [g for g, e in enumerate(exp7) if sum(e) == 7]
    scale = max(abs(ref[g]) for g in sel)
    for g in sel:
        assert abs(got[g] - ref[g]) <= 2e-14 * scale, (exp7[g], got[g], ref[g])


def test_general_closed_form_equals_the_order_4_forms():
    rng = np.random.default_rng(3)
    for _ in range(20):
        r = rng.uniform(-9, 9, 3)
        a = oracle.green(r, 4)
        b = oracle.green_general(r, 4)
        for n in range(5):
            sel = [g for g, e in enumerate(EXP6[:35]) if sum(e) == n]
            assert np.max(np.abs(a[sel] - b[sel])) <= 4e-15 * np.max(np.abs(a[sel]))


def test_general_closed_form_is_harmonic_to_order_6():
    idx = {e: g for g, e in enumerate(EXP6)}
    rng = np.random.default_rng(4)
    for _ in range(10):
        G = oracle.green_general(rng.uniform(-6, 6, 3), 6)
        # the closed form is an alternating sum: its rounding scales with the
        # magnitude of its order, as in the comparison with sympy above
        scale = [max(abs(G[g]) for g, f in enumerate(EXP6) if sum(f) == n) for n in range(7)]
        for e in EXP6:
            if sum(e) > 4:
                continue
            terms = [G[idx[(e[0] + 2 * (k == 0), e[1] + 2 * (k == 1), e[2] + 2 * (k == 2))]]
                     for k in range(3)]
            assert abs(sum(terms)) <= 1e-13 * scale[sum(e) + 2], e


def _empty_block(nm):
    g = synthetic._halo_coords()
    X = (g + 0.5).T.astype(np.float64).copy()
    return np.zeros((nm, H3)), X


def test_mass_only_sources_give_the_total_order_result():
    """With M_beta = 0 for |beta| > 0 both truncations keep the same terms
    (equal up to the rounding of the two closed forms of the derivatives)."""
    b = synthetic.monopole_block(7)
    M = np.zeros((20, H3))
    M[0] = b["mass"]
    Lt, A = oracle.block_forward(M, b["com"], want_abs=True)
    Lf = oracle.block_forward(M, b["com"], full=True)
    assert np.all(np.abs(Lt - Lf) <= 1e-14 * A)


def test_single_dipole_source_closed_form():
    """One source carrying only a dipole d: L_alpha = -d . grad G_alpha(r) for
    every output order, including order 3 (which the total-order truncation
    drops)."""
    M, X = _empty_block(20)
    j = halo_index(3, 11, 14)
    d = np.array([0.3, -0.2, 0.5])
    M[1:4, j] = d
    X[:, j] += [0.07, -0.03, 0.09]
    L = oracle.block_forward(M, X, full=True)
    t = (8, 9, 13)
    assert oracle.in_stencil(t, (3, 11, 14))
    i = halo_index(*t)
    G = [float(v) for v in green_mp(X[:, i] - X[:, j], 4)]
    idx4 = {e: g for g, e in enumerate(synthetic.moment_exponents(4))}
    for a, e in enumerate(EXP3):
        # s_beta = -1 for |beta| = 1: L_alpha = -sum_k d_k G_{alpha + e_k}
        ref = -sum(d[k] * G[idx4[(e[0] + (k == 0), e[1] + (k == 1), e[2] + (k == 2))]] for k in range(3))
        n = sum(e)
        scale = max(abs(G[g]) for g, f in enumerate(synthetic.moment_exponents(4)) if sum(f) == n + 1)
        assert abs(L[a, target_index(*t)] - ref) <= 1e-14 * scale * np.abs(d).sum(), e


def test_laplace_trace_of_full_outputs():
    b = synthetic.multipole_block(1002)
    L, A = oracle.block_forward(b["M"], b["com"], want_abs=True, full=True)
    comp = {e: g for g, e in enumerate(EXP3)}
    for e in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]:
        idx = [comp[tuple(np.add(e, 2 * np.eye(3, dtype=int)[k]))] for k in range(3)]
        tr = L[idx[0]] + L[idx[1]] + L[idx[2]]
        scale = A[idx[0]] + A[idx[1]] + A[idx[2]]
        assert np.all(np.abs(tr) <= 1e-13 * scale)


def test_full_batched_matches_block_on_gathered_halo():
    batch, M, X = synthetic.batched_config(2, 5, missing_frac=0.5)
    sel = np.array([0, 5], np.int32)
    L, A = oracle.batched_forward(batch, M, X, tsel=sel, want_abs=True, full=True)
    for q, t in enumerate(sel):
        Mh, Xh = gather_halo(batch, M, X, t)
        Lb = oracle.block_forward(Mh, Xh, full=True)
        sl = slice(q * SUB3, (q + 1) * SUB3)
        assert np.all(np.abs(Lb - L[:, sl]) <= 1e-13 * A[:, sl])


def _moments_about(xc, mc, centre):
    dd = xc - centre
    return np.array([(mc * dd[:, 0] ** a * dd[:, 1] ** b * dd[:, 2] ** c).sum() for a, b, c in EXP3])


def _expansion_error(scale, full, rng_seed=11):
    rng = np.random.default_rng(rng_seed)
    M, X = _empty_block(20)
    j = halo_index(2, 12, 12)
    t = (9, 12, 12)
    assert oracle.in_stencil(t, (2, 12, 12))
    centre = X[:, j] + np.array([0.05, -0.04, 0.03])
    xc = centre + scale * rng.uniform(-1, 1, (8, 3))
    mc = rng.uniform(0.5, 1.5, 8)
    M[:, j] = _moments_about(xc, mc, centre)
    X[:, j] = centre
    L = oracle.block_forward(M, X, full=full)[:, target_index(*t)]
    xt = X[:, halo_index(*t)]
    ref = np.zeros(20)
    for x, m in zip(xc, mc):
        ref += m * oracle.green(xt - x, 3)
    return L, ref


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_full_expansion_error_falls_as_a4_for_every_order(order):
    """Every output keeps moments up to order 3: halving the source size
    divides its error by 2^4 whatever the output order (total order: 2^(4-n))."""
    sel = [a for a in range(20) if sum(EXP3[a]) == order]
    errs = []
    for s in (0.1, 0.05, 0.025):
        L, ref = _expansion_error(s, True)
        errs.append(np.max(np.abs(L[sel] - ref[sel])) / np.max(np.abs(ref[sel])))
    for e0, e1 in zip(errs, errs[1:]):
        assert 0.75 * 16 <= e0 / e1 <= 1.3 * 16, (order, errs)
    # and for n >= 1 it is the more accurate of the two truncations
    if order >= 1:
        Lt, ref = _expansion_error(0.1, False)
        Lf, _ = _expansion_error(0.1, True)
        assert np.max(np.abs(Lf[sel] - ref[sel])) < 0.1 * np.max(np.abs(Lt[sel] - ref[sel]))


def test_orders_out_of_range_are_rejected():
    with pytest.raises(ValueError):
        oracle.green_general((1.0, 2.0, 3.0), 8)
    assert list(itertools.islice(EXP6, 20)) == EXP3


def test_thirty_digit_sum_full():
    """A target cell summed in 30-digit arithmetic over the sources of a few
    halo planes (all other cells carry no moments), with order-6 derivatives
    from symbolic differentiation: the full truncation's assembly and
    rounding, independent of its closed form."""
    import math

    import mpmath
    from symbolic import _derivative_functions

    b = synthetic.multipole_block(1002)
    M, X = b["M"].copy(), b["com"]
    hz = np.arange(H3) // (HALO * HALO)
    M[:, (hz < 4) | (hz > 5)] = 0.0           # sources only in halo planes z = 4, 5
    L, A = oracle.block_forward(M, X, want_abs=True, full=True)
    coef = []
    for e in EXP3:
        fac = math.factorial(e[0]) * math.factorial(e[1]) * math.factorial(e[2])
        coef.append(mpmath.mpf((-1) ** sum(e)) / fac)
    idx6 = {e: g for g, e in enumerate(EXP6)}
    terms = [(a, bb, idx6[tuple(np.add(EXP3[a], EXP3[bb]))]) for a in range(20) for bb in range(20)]
    fns = _derivative_functions(6)
    t = (9, 12, 8)
    i = halo_index(*t)
    n_src = 0
    with mpmath.workdps(30):
        acc = [mpmath.mpf(0)] * 20
        for hx, hy, hz_ in itertools.product(range(HALO), range(HALO), (4, 5)):
            hj = (hx, hy, hz_)
            if not oracle.in_stencil(t, hj):
                continue
            n_src += 1
            j = halo_index(*hj)
            r = [mpmath.mpf(float(X[k, i])) - mpmath.mpf(float(X[k, j])) for k in range(3)]
            G = [f(*r) for f in fns]
            for a, bb, ab in terms:
                acc[a] += coef[bb] * mpmath.mpf(float(M[bb, j])) * G[ab]
    assert n_src > 50
    col = target_index(*t)
    for a in range(20):
        assert abs(L[a, col] - float(acc[a])) <= 2e-14 * A[a, col], (a, L[a, col], float(acc[a]))


# ---------------------------------------------------------------------------
# adjoint of the full truncation (derivatives to order 7)
# ---------------------------------------------------------------------------
from test_oracle_adjoint import small_open_case  # noqa: E402


def _loss_full(batch, M, X, w):
    return float(np.sum(w * oracle.batched_forward(batch, M, X, full=True)))


def _cols(a, sel):
    return a.reshape(a.shape[0], -1, SUB3)[:, sel].reshape(a.shape[0], -1)


def test_full_moment_gradient_dot_product():
    """V nonzero on two store sub-grids only (one a target, one not)."""
    batch, M, X = small_open_case(targets=(13, 4), missing=((13, 5),))
    w = synthetic.weights(batch["T"], 15)
    ssel = np.array([13, 12], np.int32)
    gM, gX = oracle.batched_backward(batch, M, X, w, ssel=ssel, full=True)
    rng = np.random.default_rng(18)
    V = np.zeros_like(M)
    for s_ in ssel:
        V[:, s_ * SUB3:(s_ + 1) * SUB3] = rng.standard_normal((20, SUB3)) * np.abs(M).max(axis=1, keepdims=True)
    l0 = _loss_full(batch, M, X, w)
    l1 = _loss_full(batch, M + V, X, w)
    lv = _loss_full(batch, V, X, w)          # the loss is linear in M
    dot = float(np.sum(gM * _cols(V, ssel)))
    assert abs((l1 - l0) - dot) <= 1e-10 * abs(dot)
    assert abs(lv - dot) <= 1e-12 * abs(dot)
    # and it is not the total-order gradient
    gM_t, _ = oracle.batched_backward(batch, M, X, w, ssel=ssel)
    assert np.max(np.abs(gM - gM_t)) > 1e-6 * np.max(np.abs(gM))


def test_full_position_gradient_complex_step():
    batch, M, X = small_open_case(targets=(13, 4), missing=((13, 5), (4, 14)))
    w = synthetic.weights(batch["T"], 16)
    ssel = np.array([13, 4, 0, 5], np.int32)
    gM, gX = oracle.batched_backward(batch, M, X, w, ssel=ssel, full=True)
    h = 1e-30
    cells = [(13, 7), (13, 300), (4, 511), (0, 100), (5, 3)]
    scale = np.abs(gX).max()
    for n, (sg, cc) in enumerate(cells):
        k = n % 3
        Xim = np.zeros_like(X)
        Xim[k, sg * SUB3 + cc] = h
        Lre, Lim = oracle.batched_forward_cs(batch, M, X, Xim, full=True)
        d = float(np.sum(w * Lim)) / h
        col = list(ssel).index(sg) * SUB3 + cc
        assert abs(gX[k, col] - d) <= 1e-12 * scale + 1e-11 * abs(d), (sg, cc, k, gX[k, col], d)
    # the complex forward's real part is the real forward
    Lf = oracle.batched_forward(batch, M, X, full=True)
    assert np.allclose(Lre, Lf, rtol=1e-14, atol=1e-14 * np.abs(Lf).max())


def test_full_position_gradient_central_difference():
    batch, M, X = small_open_case(targets=(13,), missing=())
    w = synthetic.weights(batch["T"], 17)
    ssel = np.array([13, 12], np.int32)
    gM, gX = oracle.batched_backward(batch, M, X, w, ssel=ssel, full=True)
    eps = 1e-6
    for q, (sg, cc, k) in enumerate([(13, 77, 0), (12, 5, 2)]):
        c = sg * SUB3 + cc
        Xp = X.copy()
        Xm = X.copy()
        Xp[k, c] += eps
        Xm[k, c] -= eps
        d = (_loss_full(batch, M, Xp, w) - _loss_full(batch, M, Xm, w)) / (2 * eps)
        assert abs(gX[k, q * SUB3 + cc] - d) <= 1e-6 * np.abs(gX).max()


def test_full_position_gradients_sum_to_zero():
    batch, M, X = small_open_case(targets=(13,), missing=((13, 5),))
    w = synthetic.weights(batch["T"], 19)
    gM, gX = oracle.batched_backward(batch, M, X, w, full=True)
    assert np.all(np.abs(gX.sum(axis=1)) <= 1e-12 * np.abs(gX).sum(axis=1))
