"""GPU parity of the tree passes around the interaction (upward pass M2M,
downward pass L2L, local evaluation of force and energy) against the CPU
oracle on the same seeded inputs, through the C ABI.

Criterion, element by element: |got - ref| <= TOL * A, where A is the sum of
the magnitudes of the terms of that output (computed here with numpy from the
definition of each pass). Each output is a short sum (at most 160 products),
so both sides round within a few hundred ulp of A; a relative bound on the
output itself would be meaningless for the dipole of the upward pass, which is
zero about the centre of mass up to rounding."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import oracle  # noqa: E402
import synthetic  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12
SUB3 = 512
EXP = synthetic.moment_exponents(3)
IDX = {e: i for i, e in enumerate(EXP)}


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


def _fact(e):
    return math.factorial(e[0]) * math.factorial(e[1]) * math.factorial(e[2])


def _binom(b, g):
    return math.prod(math.comb(b[k], g[k]) for k in range(3))


def _absmono(d, e):
    """|d^e| for d of shape (3, ...)."""
    return np.abs(d[0]) ** e[0] * np.abs(d[1]) ** e[1] * np.abs(d[2]) ** e[2]


def child_cells(children, psel):
    """Store cell ids (len(psel)*512, 8) of the 2x2x2 child cells under each
    cell of the selected parent nodes, written from the octree layout: parent
    cell (X, Y, Z) lies in child node o = (X//4, Y//4, Z//4) and covers its
    cells 2 (X%4) + {0,1}, ... in each axis."""
    pc = np.arange(SUB3)
    X, Y, Z = pc % 8, (pc // 8) % 8, pc // 64
    o = X // 4 + 2 * (Y // 4) + 4 * (Z // 4)
    l0 = 2 * (X % 4) + 8 * 2 * (Y % 4) + 64 * 2 * (Z % 4)
    k = np.arange(8)
    dk = (k % 2) + 8 * ((k // 2) % 2) + 64 * (k // 4)
    blk = children[np.asarray(psel)][:, o]
    return (blk[:, :, None].astype(np.int64) * SUB3 + l0[None, :, None] + dk).reshape(-1, 8)


def m2m_magnitudes(Mc, Xc, cells, Xp):
    """A_b = sum over the 8 children k, sum over g <= b of C(b, g) |M_g(k)| |d_k^e|
    (e = b - g, d_k = X_k - X_p), plus the first-order terms of the same sum in
    the rounding of d_k = X_k - X_p: C(b, g) |M_g(k)| e_i |d_k^(e - e_i)|
    (|X_k,i| + |X_p,i|). The second part is the size of the centre-of-mass
    rounding carried into the moments: a one-ulp difference in X_p (a fused
    multiply-add in the mass-weighted sum on one side, not on the other) moves
    a dipole that cancels to rounding level by |M_0| ulp(|X_p|)."""
    d = Xc[:, cells] - Xp[:, :, None]
    xs = np.abs(Xc[:, cells]) + np.abs(Xp[:, :, None])
    aM = np.abs(Mc[:, cells])
    A = np.zeros((20, cells.shape[0]))
    for b, eb in enumerate(EXP):
        for g, eg in enumerate(EXP):
            e = tuple(eb[i] - eg[i] for i in range(3))
            if min(e) < 0:
                continue
            c = _binom(eb, eg) * aM[g]
            A[b] += (c * _absmono(d, e)).sum(axis=1)
            for i in range(3):
                if e[i] > 0:
                    ei = tuple(e[k] - (k == i) for k in range(3))
                    A[b] += (c * e[i] * _absmono(d, ei) * xs[i]).sum(axis=1)
    return A


def l2l_magnitudes(Lp, Xp, Xc, Lc, cells):
    """A_a = |Lc_a| + sum_{|g| <= 3-|a|} |Lp_{a+g}| |d^g| / g!  for every child cell."""
    n = cells.shape[0]
    pidx = np.repeat(np.arange(n), 8)
    cidx = cells.reshape(-1)
    d = Xc[:, cidx] - Xp[:, pidx]
    A = np.abs(Lc[:, cidx]).copy()
    for a, ea in enumerate(EXP):
        for g, eg in enumerate(EXP):
            s = tuple(ea[i] + eg[i] for i in range(3))
            if sum(s) > 3:
                continue
            A[a] += np.abs(Lp[IDX[s], pidx]) * _absmono(d, eg) / _fact(eg)
    return A, cidx


def evaluate_magnitudes(M, L):
    AF = np.zeros((3, M.shape[1]))
    AW = np.zeros(M.shape[1])
    for a, ea in enumerate(EXP):
        t = np.abs(M[a]) / _fact(ea)
        AW += 0.5 * t * np.abs(L[a])
        if sum(ea) <= 2:
            for k in range(3):
                s = list(ea)
                s[k] += 1
                AF[k] += t * np.abs(L[IDX[tuple(s)]])
    return AF, AW


def check(got, ref, A, what):
    err = np.abs(got - ref)
    bound = TOL * A
    bad = np.argwhere(err > bound)
    ratio = float(np.max(err / np.where(A > 0, A, 1.0)))
    assert bad.size == 0, "%s: %d outputs outside %.0e * A, first %s (got %r ref %r A %r)" % (
        what, len(bad), TOL, bad[0], got[tuple(bad[0])], ref[tuple(bad[0])], A[tuple(bad[0])])
    print("%s: worst |diff| / A = %.2e" % (what, ratio))
    return ratio


def _store(n, seed):
    rng = synthetic._rng(seed)
    M, X = synthetic.store_field(n, rng, 2.0, 3.0, 0.6, sep=4.0 * n / 4)
    return M, X


# ---------------------------------------------------------------------------
# upward pass
# ---------------------------------------------------------------------------
def test_m2m_octree_full(ot):
    n = 4
    M, X = _store(n, 61)
    ch = synthetic.octree_children(n)
    Sp = ch.shape[0]
    ref_M, ref_X = oracle.m2m(ch, M, X)
    tree = ot.Tree(ch, n ** 3)
    Mp, Xp = _empty(20, Sp * SUB3), _empty(3, Sp * SUB3)
    tree.m2m(_dev(M), _dev(X), Mp, Xp)
    got_M, got_X = _host(Mp), _host(Xp)
    cells = child_cells(ch, np.arange(Sp))
    check(got_X, ref_X, np.abs(X[:, cells]).max(axis=2), "m2m centres")
    check(got_M, ref_M, m2m_magnitudes(M, X, cells, ref_X), "m2m moments")
    # the monopole is a plain sum of 8 masses: total mass is conserved
    assert np.isclose(got_M[0].sum(), M[0].sum(), rtol=1e-13)


def test_m2m_permuted_children_unused_nodes_and_empty_cells(ot):
    """Random child permutation over a larger store (some nodes are nobody's
    child); a block of massless cells, with whole parent cells empty (their
    centre is the mean of the child centres and their moments are exact zeros)."""
    n = 4
    M, X = _store(n, 62)
    rng = np.random.default_rng(63)
    ch = rng.permutation(n ** 3)[:40].astype(np.int32).reshape(5, 8)
    M[:, ch[1, 2] * SUB3: ch[1, 2] * SUB3 + 200] = 0.0
    M[:, ch[3, 7] * SUB3:(ch[3, 7] + 1) * SUB3] = 0.0
    ref_M, ref_X = oracle.m2m(ch, M, X)
    tree = ot.Tree(ch, n ** 3)
    Mp, Xp = _empty(20, 5 * SUB3), _empty(3, 5 * SUB3)
    tree.m2m(_dev(M), _dev(X), Mp, Xp)
    got_M, got_X = _host(Mp), _host(Xp)
    cells = child_cells(ch, np.arange(5))
    check(got_X, ref_X, np.abs(X[:, cells]).max(axis=2), "m2m centres")
    check(got_M, ref_M, m2m_magnitudes(M, X, cells, ref_X), "m2m moments")
    empty = ref_M[0] == 0.0
    assert empty.sum() >= 64
    assert np.all(got_M[:, empty] == 0.0)


# ---------------------------------------------------------------------------
# downward pass
# ---------------------------------------------------------------------------
def test_l2l_accumulates_and_leaves_other_nodes(ot):
    n = 4
    M, X = _store(n, 64)
    rng = np.random.default_rng(65)
    perm = rng.permutation(n ** 3).astype(np.int32)
    ch = perm[:48].reshape(6, 8)
    _, Xp = oracle.m2m(ch, M, X)
    Lp = synthetic.local_field(6 * SUB3, rng)
    Lc = synthetic.local_field(n ** 3 * SUB3, rng)
    ref = oracle.l2l(ch, Lp, Xp, X, Lc)
    tree = ot.Tree(ch, n ** 3)
    Lc_d = _dev(Lc)
    tree.l2l(_dev(Lp), _dev(Xp), _dev(X), Lc_d)
    got = _host(Lc_d)
    cells = child_cells(ch, np.arange(6))
    A, cidx = l2l_magnitudes(Lp, Xp, X, Lc, cells)
    check(got[:, cidx], ref[:, cidx], A, "l2l")
    untouched = np.ones(n ** 3 * SUB3, bool)
    untouched[cidx] = False
    assert untouched.sum() == 16 * SUB3
    assert np.array_equal(got[:, untouched], Lc[:, untouched])


def test_l2l_of_a_cubic_potential_is_exact_re_expansion(ot):
    """A parent expansion that is the Taylor series of a cubic about the parent
    centre re-expands without truncation: zero child input plus L2L gives the
    cubic's derivatives at the child centre (evaluated here in closed form)."""
    rng = np.random.default_rng(66)
    ch = np.arange(8, dtype=np.int32).reshape(1, 8)
    Xp = rng.uniform(0, 8, (3, SUB3))
    Xc = rng.uniform(0, 8, (3, 8 * SUB3))
    coef = rng.standard_normal(20)        # phi(y) = sum_g coef_g y^g (y about the origin)

    def derivs(y):
        out = np.zeros((20, y.shape[1]))
        for a, ea in enumerate(EXP):
            for g, eg in enumerate(EXP):
                e = tuple(eg[i] - ea[i] for i in range(3))
                if min(e) < 0:
                    continue
                f = math.prod(math.factorial(eg[i]) // math.factorial(e[i]) for i in range(3))
                out[a] += coef[g] * f * y[0] ** e[0] * y[1] ** e[1] * y[2] ** e[2]
        return out

    Lp = derivs(Xp)
    cells = child_cells(ch, [0])
    expect = derivs(Xc)
    tree = ot.Tree(ch, 8)
    Lc = _dev(np.zeros((20, 8 * SUB3)))
    tree.l2l(_dev(Lp), _dev(Xp), _dev(Xc), Lc)
    got = _host(Lc)
    A, cidx = l2l_magnitudes(Lp, Xp, Xc, np.zeros((20, 8 * SUB3)), cells)
    check(got[:, cidx], expect[:, cidx], 10 * A, "l2l cubic")


# ---------------------------------------------------------------------------
# local evaluation
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ncell", [1, 255, 3 * SUB3 + 77])
def test_evaluate_ragged(ot, ncell):
    rng = np.random.default_rng(67 + ncell)
    M = rng.standard_normal((20, ncell))
    L = synthetic.local_field(ncell, rng)
    rF, rW = oracle.evaluate(M, L)
    F, W = _empty(3, ncell), _empty(ncell)
    ot.ot_fmm_evaluate(_dev(M), _dev(L), F, W)
    AF, AW = evaluate_magnitudes(M, L)
    check(_host(F), rF, AF, "evaluate F")
    check(_host(W), rW, AW, "evaluate W")


# ---------------------------------------------------------------------------
# the 32^3-sub-grid store of the benchmark: parents of all 32768 sub-grids
# ---------------------------------------------------------------------------
def test_tree_passes_full_store_sampled(ot):
    import torch
    n = 32
    batch, M, X = synthetic.config5(n)
    ch = synthetic.octree_children(n)
    Sp = ch.shape[0]
    tree = ot.Tree(ch, n ** 3)
    Md, Xd = _dev(M), _dev(X)
    Mp, Xp = _empty(20, Sp * SUB3), _empty(3, Sp * SUB3)
    tree.m2m(Md, Xd, Mp, Xp)
    psel = np.sort(np.random.default_rng(68).choice(Sp, 24, replace=False)).astype(np.int32)
    cols = (psel[:, None] * SUB3 + np.arange(SUB3)).reshape(-1)
    ref_M, ref_X = oracle.m2m(ch, M, X, psel)
    got_M, got_X = _host(Mp)[:, cols], _host(Xp)[:, cols]
    cells = child_cells(ch, psel)
    check(got_X, ref_X, np.abs(X[:, cells]).max(axis=2), "m2m centres (sampled)")
    check(got_M, ref_M, m2m_magnitudes(M, X, cells, ref_X), "m2m moments (sampled)")
    assert np.isclose(float(Mp[0].sum()), M[0].sum(), rtol=1e-12)

    # downward pass over the full level; oracle on the selected parents only
    # expansion centres of the parent cells: the mean of their child centres
    rng = np.random.default_rng(69)
    Xp_ref = X[:, child_cells(ch, np.arange(Sp))].mean(axis=2)
    Lp = synthetic.local_field(Sp * SUB3, rng)
    Lc = synthetic.local_field(n ** 3 * SUB3, rng)
    Lc_d = _dev(Lc)
    tree.l2l(_dev(Lp), _dev(Xp_ref), Xd, Lc_d)
    sub = ch[psel]
    sub_cells = child_cells(ch, psel)
    ref = oracle.l2l(np.arange(len(psel) * 8, dtype=np.int32).reshape(-1, 8),
                     Lp[:, cols], Xp_ref[:, cols],
                     X[:, (sub.reshape(-1)[:, None] * SUB3 + np.arange(SUB3)).reshape(-1)],
                     Lc[:, (sub.reshape(-1)[:, None] * SUB3 + np.arange(SUB3)).reshape(-1)])
    got = _host(Lc_d)[:, (sub.reshape(-1)[:, None] * SUB3 + np.arange(SUB3)).reshape(-1)]
    # local relabelling: child k of selected parent q is node 8 q + k
    A, cidx = l2l_magnitudes(Lp[:, cols], Xp_ref[:, cols], X, Lc, sub_cells)
    loc = child_cells(np.arange(len(psel) * 8, dtype=np.int32).reshape(-1, 8),
                      np.arange(len(psel))).reshape(-1)
    check(got[:, loc], ref[:, loc], A, "l2l (sampled)")
    del Lc_d

    # evaluation over every cell of the store; oracle on a strided sample
    Ld = _dev(Lc)
    F, W = _empty(3, n ** 3 * SUB3), _empty(n ** 3 * SUB3)
    ot.ot_fmm_evaluate(Md, Ld, F, W)
    s = np.arange(0, n ** 3 * SUB3, 997)
    rF, rW = oracle.evaluate(M[:, s], Lc[:, s])
    AF, AW = evaluate_magnitudes(M[:, s], Lc[:, s])
    torch.cuda.synchronize()
    check(F[:, s].cpu().numpy(), rF, AF, "evaluate F (sampled)")
    check(W[s].cpu().numpy(), rW, AW, "evaluate W (sampled)")


# ---------------------------------------------------------------------------
# interaction + evaluation on the GPU: momentum balance on a closed domain
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [2, 8])
def test_momentum_balance_closed_domain(ot, n):
    """Open lattice with every sub-grid present: the criterion is symmetric
    and so is availability, so with the total-order truncation the forces of
    every interacting pair cancel and the total force vanishes to rounding.
    Forward and evaluation both run on the GPU; n = 2 is also checked against
    the oracle's forces."""
    batch, M, X = synthetic.batched_config(n, 78 + n, periodic=False)
    plan = ot.Plan.from_batch(batch)
    N = batch["T"] * SUB3
    L = _empty(20, N)
    Md = _dev(M)
    plan.multipole_batched(Md, _dev(X), L)
    F, W = _empty(3, N), _empty(N)
    ot.ot_fmm_evaluate(Md, L, F, W)
    f = _host(F)
    tot = f.sum(axis=1)
    scale = np.abs(f).sum(axis=1)
    print("n=%d: |sum F| / sum |F| = %s" % (n, np.abs(tot) / scale))
    assert np.all(np.abs(tot) <= 1e-13 * scale)
    w = _host(W)
    if n == 2:
        rF, rW = oracle.evaluate(M, oracle.batched_forward(batch, M, X))
        assert np.allclose(f, rF, rtol=0, atol=1e-11 * np.abs(rF).max())
        assert np.allclose(w, rW, rtol=0, atol=1e-11 * np.abs(rW).max())
