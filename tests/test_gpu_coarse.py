"""GPU parity of the coarse substitute for missing neighbours (a coarse cell of
the parent level stands in for its 2x2x2 missing fine children when all of
them would be in the target cell's stencil) against the CPU oracle, through
the C ABI. The coarse store is the oracle's upward pass of the same seeded
fine store (an input to both sides), except in the chained test, where the
GPU's own upward pass feeds the GPU path.

Criterion as for the interaction: per sub-grid and order group,
max |got - ref| <= 1e-12 * max(max |ref|, 1e-2 * max A), A the sum of the
magnitudes of the terms."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import oracle  # noqa: E402
import synthetic  # noqa: E402
from parity import assert_parity  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12
SUB3 = 512


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


def _zeros(*shape):
    import torch
    return torch.zeros(shape, dtype=torch.float64, device="cuda")


def included_pairs_per_slot():
    """(target cell, coarse cell) pairs of each slot whose 8 children all pass
    the criterion, counted with numpy from |d|^2 > 16 and parent distance^2
    <= 16 on halo coordinates."""
    c = np.arange(SUB3)
    hi = np.stack([8 + c % 8, 8 + (c // 8) % 8, 8 + c // 64], 1)          # (512, 3)
    J = np.arange(64)
    cj = np.stack([J % 4, (J // 4) % 4, J // 16], 1)                       # (64, 3)
    n = np.arange(8)
    dn = np.stack([n & 1, (n >> 1) & 1, n >> 2], 1)                        # (8, 3)
    out = np.zeros(27, np.int64)
    for s in range(27):
        so = np.array([s % 3, (s // 3) % 3, s // 9])
        hj = 8 * so[None, None, :] + 2 * cj[:, None, :] + dn[None, :, :]   # (64, 8, 3)
        d2 = ((hj[None] - hi[:, None, None]) ** 2).sum(-1)                  # (512, 64, 8)
        p2 = ((hj[None] // 2 - hi[:, None, None] // 2) ** 2).sum(-1)
        out[s] = np.all((d2 > 16) & (p2 <= 16), axis=2).sum()
    return out


def _case(n, seed, frac, periodic):
    batch, M, X = synthetic.batched_config(n, seed, missing_frac=frac, periodic=periodic)
    coarse, octant = synthetic.coarse_tables(n, batch)
    Mp, Xp = oracle.m2m(synthetic.octree_children(n), M, X)
    return batch, M, X, coarse, octant, Mp, Xp


@pytest.mark.parametrize("periodic", [True, False])
def test_coarse_fine_small_all_targets(ot, periodic):
    batch, M, X, coarse, octant, Mp, Xp = _case(4, 81 + periodic, 0.6, periodic)
    assert (coarse >= 0).sum() > 20
    plan = ot.Plan.from_batch(batch)
    Sp = Mp.shape[1] // SUB3
    pairs = plan.set_coarse(Sp, coarse, octant)
    per_slot = included_pairs_per_slot()
    assert pairs == int(sum(per_slot[s] for t, s in zip(*np.nonzero(coarse >= 0))))
    ref, A = oracle.coarse_fine(batch, X, coarse, octant, Mp, Xp, want_abs=True)
    L = _zeros(20, batch["T"] * SUB3)
    dX, dMp, dXp = _dev(X), _dev(Mp), _dev(Xp)
    plan.coarse_fine(dX, dMp, dXp, L)
    got = _host(L)
    assert_parity(got, ref, TOL, what="coarse small", A=A)
    # targets without substitutes are untouched (exact zeros)
    none = np.nonzero(~(coarse >= 0).any(1))[0]
    assert np.all(got.reshape(20, -1, SUB3)[:, none] == 0.0)
    # accumulation: a second call adds the same values again, bit for bit
    plan.coarse_fine(dX, dMp, dXp, L)
    assert np.array_equal(_host(L), 2.0 * got)


def test_coarse_fine_added_to_the_interaction(ot):
    """Fine interaction over the present neighbours, then the coarse
    substitutes, into the same L: equal to the sum of the two oracle parts."""
    batch, M, X, coarse, octant, Mp, Xp = _case(4, 83, 0.5, True)
    plan = ot.Plan.from_batch(batch)
    plan.set_coarse(Mp.shape[1] // SUB3, coarse, octant)
    ref_f, A_f = oracle.batched_forward(batch, M, X, want_abs=True)
    ref_c, A_c = oracle.coarse_fine(batch, X, coarse, octant, Mp, Xp, want_abs=True)
    L = _zeros(20, batch["T"] * SUB3)
    dX = _dev(X)
    plan.multipole_batched(_dev(M), dX, L)
    plan.coarse_fine(dX, _dev(Mp), _dev(Xp), L)
    assert_parity(_host(L), ref_f + ref_c, TOL, what="fine + coarse", A=A_f + A_c)


def test_coarse_fine_fed_by_the_gpu_upward_pass(ot):
    """Chained on the GPU: upward pass (M2M) of the fine store, then the
    coarse substitutes from its output; the oracle chains its own passes."""
    batch, M, X, coarse, octant, Mp, Xp = _case(4, 84, 0.6, False)
    children = synthetic.octree_children(4)
    Sp = children.shape[0]
    tree = ot.Tree(children, batch["S"])
    dM, dX = _dev(M), _dev(X)
    dMp, dXp = _zeros(20, Sp * SUB3), _zeros(3, Sp * SUB3)
    tree.m2m(dM, dX, dMp, dXp)
    plan = ot.Plan.from_batch(batch)
    plan.set_coarse(Sp, coarse, octant)
    L = _zeros(20, batch["T"] * SUB3)
    plan.coarse_fine(dX, dMp, dXp, L)
    ref, A = oracle.coarse_fine(batch, X, coarse, octant, Mp, Xp, want_abs=True)
    # the GPU centres of mass differ from the oracle's by rounding only, a
    # relative change of order 1e-16 in the terms: the same bound holds
    assert_parity(_host(L), ref, TOL, what="m2m -> coarse", A=A)


def test_coarse_fine_config5_sampled(ot):
    """32^3 sub-grids, periodic, 20% of targets missing 1..9 neighbours, all
    missing neighbours substituted from the parent level: one launch over
    every target with substitutes, a seeded sample compared with the oracle."""
    batch, M, X = synthetic.config5()
    coarse, octant = synthetic.coarse_tables(32, batch)
    Mp, Xp = oracle.m2m(synthetic.octree_children(32), M, X)
    plan = ot.Plan.from_batch(batch)
    plan.set_coarse(Mp.shape[1] // SUB3, coarse, octant)
    L = _zeros(20, batch["T"] * SUB3)
    plan.coarse_fine(_dev(X), _dev(Mp), _dev(Xp), L)
    got = _host(L)
    assert np.all(np.isfinite(got))
    with_sub = np.nonzero((coarse >= 0).any(1))[0]
    rng = np.random.default_rng(85)
    sel = np.sort(rng.choice(with_sub, 24, replace=False)).astype(np.int32)
    ref, A = oracle.coarse_fine(batch, X, coarse, octant, Mp, Xp, tsel=sel, want_abs=True)
    cols = got.reshape(20, -1, SUB3)[:, sel].reshape(20, -1)
    assert_parity(cols, ref, TOL, what="config5 coarse", A=A)
    without = np.setdiff1d(np.arange(batch["T"]), with_sub)
    assert np.all(got.reshape(20, -1, SUB3)[:, without[:64]] == 0.0)


def test_set_coarse_rejects_bad_tables(ot):
    batch, M, X, coarse, octant, Mp, Xp = _case(4, 86, 0.5, True)
    plan = ot.Plan.from_batch(batch)
    Sp = Mp.shape[1] // SUB3
    with pytest.raises(ValueError):
        plan.coarse_fine(_dev(X), _dev(Mp), _dev(Xp), _zeros(20, batch["T"] * SUB3))
    t, s = np.argwhere(batch["nbr"] >= 0)[0]
    bad = coarse.copy()
    bad[t, s] = 0
    with pytest.raises(ot.OtFmmError):
        plan.set_coarse(Sp, bad, octant)
    bad = coarse.copy()
    bad[coarse >= 0] = Sp
    with pytest.raises(ot.OtFmmError):
        plan.set_coarse(Sp, bad, octant)
    bad_o = octant.copy()
    bad_o[coarse >= 0] = 8
    with pytest.raises(ot.OtFmmError):
        plan.set_coarse(Sp, coarse, bad_o)
    # the plan keeps working after rejected tables
    plan.set_coarse(Sp, coarse, octant)
    import ctypes
    import torch
    from paper_2303_08058_amd import _lib
    big = torch.zeros(40, batch["T"] * SUB3, dtype=torch.float64, device="cuda")
    L = big[:20]
    dX, dMp = _dev(X), _dev(Mp)
    # comp starting inside L: rejected from the extents, nothing launched
    rc = _lib.ot_fmm_coarse_fine(plan.handle, ctypes.c_void_p(dX.data_ptr()),
                                 ctypes.c_void_p(dMp.data_ptr()),
                                 ctypes.c_void_p(L.data_ptr() + 8 * 512),
                                 ctypes.c_void_p(L.data_ptr()), None)
    assert rc == ot.OT_FMM_EINVAL
    assert np.all(_host(big) == 0.0)


def test_no_substitutes_leaves_L_untouched(ot):
    """Tables without any substitute: zero pairs, nothing launched, L keeps
    its values; replacing them with real tables afterwards works."""
    batch, M, X, coarse, octant, Mp, Xp = _case(4, 87, 0.5, True)
    plan = ot.Plan.from_batch(batch)
    Sp = Mp.shape[1] // SUB3
    none = np.full_like(coarse, -1)
    assert plan.set_coarse(Sp, none, np.zeros_like(octant)) == 0
    import torch
    L = torch.full((20, batch["T"] * SUB3), 3.25, dtype=torch.float64, device="cuda")
    dX, dMp, dXp = _dev(X), _dev(Mp), _dev(Xp)
    plan.coarse_fine(dX, dMp, dXp, L)
    assert np.all(_host(L) == 3.25)
    plan.set_coarse(Sp, coarse, octant)
    L.zero_()
    plan.coarse_fine(dX, dMp, dXp, L)
    ref, A = oracle.coarse_fine(batch, X, coarse, octant, Mp, Xp, want_abs=True)
    assert_parity(_host(L), ref, TOL, what="after replacing tables", A=A)


# ---------------------------------------------------------------------------
# the full truncation (every |b| <= 3 for every output |a| <= 3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("periodic", [True, False])
def test_coarse_fine_full_small_all_targets(ot, periodic):
    batch, M, X, coarse, octant, Mp, Xp = _case(4, 88 + periodic, 0.6, periodic)
    plan = ot.Plan.from_batch(batch)
    plan.set_coarse(Mp.shape[1] // SUB3, coarse, octant)
    ref, A = oracle.coarse_fine(batch, X, coarse, octant, Mp, Xp, want_abs=True, full=True)
    L = _zeros(20, batch["T"] * SUB3)
    dX, dMp, dXp = _dev(X), _dev(Mp), _dev(Xp)
    plan.coarse_fine(dX, dMp, dXp, L, full=True)
    got = _host(L)
    assert_parity(got, ref, TOL, what="coarse full small", A=A)
    # it is not the total order: the order-3 outputs differ by the added terms
    ref_t = oracle.coarse_fine(batch, X, coarse, octant, Mp, Xp)
    assert np.max(np.abs(ref[10:] - ref_t[10:])) > 1e-6 * np.max(np.abs(ref_t[10:]))
    none = np.nonzero(~(coarse >= 0).any(1))[0]
    assert np.all(got.reshape(20, -1, SUB3)[:, none] == 0.0)
    plan.coarse_fine(dX, dMp, dXp, L, full=True)
    assert np.array_equal(_host(L), 2.0 * got)


def test_coarse_fine_full_config5_sampled(ot):
    """32^3 sub-grids, periodic, 20% of targets missing 1..9 neighbours, all
    substituted: the full-truncation launch over every target, sampled."""
    batch, M, X = synthetic.config5()
    coarse, octant = synthetic.coarse_tables(32, batch)
    Mp, Xp = oracle.m2m(synthetic.octree_children(32), M, X)
    plan = ot.Plan.from_batch(batch)
    plan.set_coarse(Mp.shape[1] // SUB3, coarse, octant)
    L = _zeros(20, batch["T"] * SUB3)
    plan.coarse_fine(_dev(X), _dev(Mp), _dev(Xp), L, full=True)
    got = _host(L)
    assert np.all(np.isfinite(got))
    with_sub = np.nonzero((coarse >= 0).any(1))[0]
    rng = np.random.default_rng(89)
    sel = np.sort(rng.choice(with_sub, 12, replace=False)).astype(np.int32)
    ref, A = oracle.coarse_fine(batch, X, coarse, octant, Mp, Xp, tsel=sel, want_abs=True, full=True)
    cols = got.reshape(20, -1, SUB3)[:, sel].reshape(20, -1)
    assert_parity(cols, ref, TOL, what="config5 coarse full", A=A)
