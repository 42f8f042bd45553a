"""A two-level step assembled from the library's calls only, on the GPU:
upward pass of a fine store to its parent level, the fine interaction plus
coarse substitutes for the fine level's missing neighbours, the interaction
of the parent level, the downward pass of the parent expansions into the
fine coefficients, and the evaluation of force and energy; with either
truncation of the interactions. The oracle runs
the same chain of its own functions on the same seeded inputs; the test
checks that every hand-over between the passes (layouts, centres, store
and parent numbering) agrees.

Criterion: per sub-grid and output group, max |got - ref| <= 1e-12 * max
|ref|, the plain criterion of the single passes, also after the five passes
the rounding differences run through."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import oracle  # noqa: E402
import synthetic  # noqa: E402
from parity import assert_parity  # noqa: E402

pytestmark = pytest.mark.gpu

SUB3 = 512
TOL = 1e-12


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float64)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("periodic,full", [(False, False), (True, False), (True, True)])
def test_two_level_step_matches_the_oracle_chain(periodic, full):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08058_amd as ot

    n = 4
    fine, M, X = synthetic.batched_config(n, 91, missing_frac=0.5, periodic=periodic)
    coarse, octant = synthetic.coarse_tables(n, fine)
    children = synthetic.octree_children(n)
    Sp = children.shape[0]
    parent = synthetic.parent_lattice(n, periodic=periodic)
    assert (coarse >= 0).sum() > 10

    # oracle chain
    Mp_r, Xp_r = oracle.m2m(children, M, X)
    Lf_r = (oracle.batched_forward(fine, M, X, full=full) +
            oracle.coarse_fine(fine, X, coarse, octant, Mp_r, Xp_r, full=full))
    Lp_r = oracle.batched_forward(parent, Mp_r, Xp_r, full=full)
    Lf_r = oracle.l2l(children, Lp_r, Xp_r, X, Lf_r)
    F_r, W_r = oracle.evaluate(M, Lf_r)

    # GPU chain
    f64 = dict(dtype=torch.float64, device="cuda")
    dM, dX = _dev(M), _dev(X)
    tree = ot.Tree(children, fine["S"])
    Mp, Xp = torch.empty((20, Sp * SUB3), **f64), torch.empty((3, Sp * SUB3), **f64)
    tree.m2m(dM, dX, Mp, Xp)
    plan_f = ot.Plan.from_batch(fine)
    plan_f.set_coarse(Sp, coarse, octant)
    Lf = torch.empty((20, fine["T"] * SUB3), **f64)
    if full:
        plan_f.multipole_batched_full(dM, dX, Lf)
    else:
        plan_f.multipole_batched(dM, dX, Lf)
    plan_f.coarse_fine(dX, Mp, Xp, Lf, full=full)
    plan_p = ot.Plan.from_batch(parent)
    Lp = torch.empty((20, parent["T"] * SUB3), **f64)
    if full:
        plan_p.multipole_batched_full(Mp, Xp, Lp)
    else:
        plan_p.multipole_batched(Mp, Xp, Lp)
    tree.l2l(Lp, Xp, dX, Lf)
    F = torch.empty((3, fine["S"] * SUB3), **f64)
    W = torch.empty((fine["S"] * SUB3,), **f64)
    ot.ot_fmm_evaluate(dM, Lf, F, W)

    # the dipole about the centre of mass is zero up to rounding: a relative
    # bound on it is meaningless (the upward pass's own tests bound it by the
    # term magnitudes), so it is left out here
    assert_parity(_host(Mp), Mp_r, 1e-12, groups=[[0], list(range(4, 10)), list(range(10, 20))],
                  what="parent moments")
    print("parent", assert_parity(_host(Lp), Lp_r, TOL, what="parent interaction"))
    print("fine", assert_parity(_host(Lf), Lf_r, TOL, what="fine coefficients"))
    print("force", assert_parity(_host(F), F_r, TOL, what="force"))
    print("energy", assert_parity(_host(W)[None, :], W_r[None, :], TOL, groups=[[0]], what="energy"))
    # the parent level contributes: without it the fine coefficients differ
    assert np.abs(oracle.l2l(children, Lp_r, Xp_r, X, np.zeros_like(Lf_r))).max() > 0


def test_two_level_step_full_size_sampled():
    """The two-level step at the benchmark's size (32^3 fine sub-grids, 20%
    missing 1-9 neighbours, every missing neighbour substituted from the 16^3
    parent level): the whole chain on the GPU, the oracle's chain on the 16
    children of two sampled parents (upward pass of every parent, since the
    coarse substitutes read the parents of the missing neighbours). Fine
    coefficients checked with the A-scaled criterion of the interaction tests
    (A: term magnitudes of the fine and coarse sums), force and energy with
    the plain one."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08058_amd as ot

    n = 32
    fine, M, X = synthetic.config5(n)
    coarse, octant = synthetic.coarse_tables(n, fine)
    children = synthetic.octree_children(n)
    Sp = children.shape[0]
    parent = synthetic.parent_lattice(n, periodic=True)
    assert np.array_equal(fine["tgt"], np.arange(fine["S"]))

    # GPU chain, as the benchmark runs it
    f64 = dict(dtype=torch.float64, device="cuda")
    dM, dX = _dev(M), _dev(X)
    tree = ot.Tree(children, fine["S"])
    Mp, Xp = torch.empty((20, Sp * SUB3), **f64), torch.empty((3, Sp * SUB3), **f64)
    tree.m2m(dM, dX, Mp, Xp)
    plan_f = ot.Plan.from_batch(fine)
    plan_f.set_coarse(Sp, coarse, octant)
    Lf = torch.empty((20, fine["T"] * SUB3), **f64)
    plan_f.multipole_batched(dM, dX, Lf)
    plan_f.coarse_fine(dX, Mp, Xp, Lf)
    plan_p = ot.Plan.from_batch(parent)
    Lp = torch.empty((20, parent["T"] * SUB3), **f64)
    plan_p.multipole_batched(Mp, Xp, Lp)
    tree.l2l(Lp, Xp, dX, Lf)
    F = torch.empty((3, fine["S"] * SUB3), **f64)
    W = torch.empty((fine["S"] * SUB3,), **f64)
    ot.ot_fmm_evaluate(dM, Lf, F, W)
    torch.cuda.synchronize()

    # oracle chain on two sampled parents and their children
    psel = np.sort(np.random.default_rng(97).choice(Sp, 2, replace=False)).astype(np.int32)
    kids = children[psel].reshape(-1).astype(np.int32)          # child k of parent q: 8 q + k
    kcols = (kids[:, None].astype(np.int64) * SUB3 + np.arange(SUB3)).reshape(-1)
    pcols = (psel[:, None].astype(np.int64) * SUB3 + np.arange(SUB3)).reshape(-1)
    Mp_r, Xp_r = oracle.m2m(children, M, X)
    Lf_f, A_f = oracle.batched_forward(fine, M, X, tsel=kids, want_abs=True)
    Lf_c, A_c = oracle.coarse_fine(fine, X, coarse, octant, Mp_r, Xp_r, tsel=kids, want_abs=True)
    Lp_r = oracle.batched_forward(parent, Mp_r, Xp_r, tsel=psel)
    Lf_r = oracle.l2l(np.arange(len(kids), dtype=np.int32).reshape(-1, 8), Lp_r, Xp_r[:, pcols],
                      X[:, kcols], Lf_f + Lf_c)
    F_r, W_r = oracle.evaluate(M[:, kcols], Lf_r)

    got = lambda t: t[..., torch.from_numpy(kcols).cuda()].cpu().numpy()
    print("fine", assert_parity(got(Lf), Lf_r, TOL, what="fine coefficients", A=A_f + A_c))
    print("force", assert_parity(got(F), F_r, TOL, what="force"))
    print("energy", assert_parity(got(W)[None, :], W_r[None, :], TOL, groups=[[0]], what="energy"))
