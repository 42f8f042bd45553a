"""GPU parity of the two-pass training step: the forward that also saves the
target-side sums (ot_fmm_multipole_batched_save) and the one-pass adjoint
that uses them (ot_fmm_multipole_backward_saved), through the C ABI, against
the oracle: L against the forward, the saved sums against the oracle's
target-side derivatives dL_a(i)/dX_i,k (the saved component g = a + e_k), the
gradients against the oracle's adjoint (criterion in tests/parity.py,
tolerance 1e-12)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import oracle  # noqa: E402
import synthetic  # noqa: E402
from parity import assert_parity  # noqa: E402
from saved_sums import check_saved  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = 1e-12
# W8 and W8P2, plain / persistent / XCD-aware order / persistent in pieces
SCHEDS = [1, 3, 0x11, 0x13, 0x21, 0x23, 0x31, 0x33]


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


@pytest.mark.parametrize("sched", SCHEDS + [0])
def test_small_periodic_with_missing(ot, sched):
    batch, M, X = synthetic.batched_config(2, 121, missing_frac=0.5)
    w = synthetic.weights(batch["T"], 122)
    plan = ot.Plan.from_batch(batch)
    NS, NT = batch["S"] * 512, batch["T"] * 512
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    L, Cs = _empty(20, NT), _empty(24, NT)
    plan.multipole_batched_save(Md, Xd, L, Cs, sched=sched)
    Lh, Csh = _host(L), _host(Cs)
    ref, A = oracle.batched_forward(batch, M, X, want_abs=True)
    assert_parity(Lh, ref, TOL, what="saved-step L", A=A)
    check_saved(Csh, batch, M, X, "saved sums")
    gM, gX = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward_saved(Md, Xd, wd, Cs, gM, gX, sched=sched)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w)
    gMh, gXh = _host(gM), _host(gX)
    print("gM worst", assert_parity(gMh, gM_ref, TOL, what="saved-step gM"))
    print("gX worst", assert_parity(gXh, gX_ref, TOL, what="saved-step gX"))
    # bitwise reproducible for a fixed schedule
    L2, Cs2, gM2, gX2 = _empty(20, NT), _empty(24, NT), _empty(20, NS), _empty(3, NS)
    plan.multipole_batched_save(Md, Xd, L2, Cs2, sched=sched)
    plan.multipole_backward_saved(Md, Xd, wd, Cs2, gM2, gX2, sched=sched)
    assert np.array_equal(_host(L2), Lh) and np.array_equal(_host(Cs2), Csh)
    assert np.array_equal(_host(gM2), gMh) and np.array_equal(_host(gX2), gXh)


def test_moment_gradient_equals_the_two_pass_adjoint_bitwise(ot):
    """gM comes from the same source-role sums in both adjoints."""
    batch, M, X = synthetic.batched_config(3, 123, missing_frac=0.3)
    w = synthetic.weights(batch["T"], 124)
    plan = ot.Plan.from_batch(batch)
    NS, NT = batch["S"] * 512, batch["T"] * 512
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    L, Cs = _empty(20, NT), _empty(24, NT)
    plan.multipole_batched_save(Md, Xd, L, Cs, sched=3)
    gM, gX = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward_saved(Md, Xd, wd, Cs, gM, gX, sched=3)
    gM2, gX2 = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward(Md, Xd, wd, gM2, gX2, sched=ot.sched_bwd(2, 3))
    assert np.array_equal(_host(gM), _host(gM2))
    gX_ref = oracle.batched_backward(batch, M, X, w)[1]
    assert_parity(_host(gX), gX_ref, TOL, what="gX 3^3")
    assert_parity(_host(gX2), gX_ref, TOL, what="gX 3^3 two-pass")


def test_open_subset_of_targets(ot):
    """Open lattice, a few targets (store sub-grids that are not targets have
    no target role), knocked-out neighbours (asymmetric availability)."""
    rng = synthetic._rng(125)
    M, X = synthetic.store_field(3, rng, 2.0, 3.0, 0.6, sep=6.0)
    full = synthetic.lattice_batch(3, periodic=False)
    tg = np.array([13, 4, 22], np.int32)
    nbr = full["nbr"][tg].copy()
    nbr[0, [5, 21]] = -1
    nbr[1, 14] = -1
    batch = {"S": 27, "T": 3, "tgt": tg, "nbr": nbr, "shift": None, "period": None}
    w = synthetic.weights(3, 126)
    plan = ot.Plan.from_batch(batch)
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    L, Cs = _empty(20, 3 * 512), _empty(24, 3 * 512)
    plan.multipole_batched_save(Md, Xd, L, Cs)
    check_saved(_host(Cs), batch, M, X, "saved sums open")
    gM, gX = _empty(20, 27 * 512), _empty(3, 27 * 512)
    plan.multipole_backward_saved(Md, Xd, wd, Cs, gM, gX)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w)
    assert_parity(_host(gM), gM_ref, TOL, what="open gM")
    assert_parity(_host(gX), gX_ref, TOL, what="open gX")


def test_autograd_both_adjoints(ot):
    import torch
    batch, M, X = synthetic.batched_config(2, 127, missing_frac=0.5)
    plan = ot.Plan.from_batch(batch)
    w = synthetic.weights(batch["T"], 128)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w)
    for save in (True, False):
        Md = _dev(M).requires_grad_(True)
        Xd = _dev(X).requires_grad_(True)
        L = ot.multipole(Md, Xd, plan, save=save)
        (L * _dev(w)).sum().backward()
        assert_parity(_host(Md.grad), gM_ref, TOL, what="autograd gM save=%s" % save)
        assert_parity(_host(Xd.grad), gX_ref, TOL, what="autograd gX save=%s" % save)
    with torch.no_grad():
        L0 = ot.multipole(_dev(M), _dev(X), plan)  # no gradient: plain forward
    assert_parity(_host(L0), oracle.batched_forward(batch, M, X), TOL, what="no-grad L")


@pytest.mark.parametrize("sched", [3, 0x33])
def test_step_graph_replays_match_eager(ot, sched):
    import torch
    batch, M, X = synthetic.batched_config(3, 129, missing_frac=0.3)
    plan = ot.Plan.from_batch(batch)
    Md, Xd = _dev(M), _dev(X)
    wd = _dev(synthetic.weights(batch["T"], 130))
    NS, NT = batch["S"] * 512, batch["T"] * 512
    L0, C0, gM0, gX0 = _empty(20, NT), _empty(24, NT), _empty(20, NS), _empty(3, NS)
    plan.multipole_batched_save(Md, Xd, L0, C0, sched=sched)
    plan.multipole_backward_saved(Md, Xd, wd, C0, gM0, gX0, sched=sched)
    L, C, gM, gX = _empty(20, NT), _empty(24, NT), _empty(20, NS), _empty(3, NS)
    plan.step_graph_create_saved(Md, Xd, L, C, wd, gM, gX, sched, sched)
    for rep in range(3):
        for t in (L, C, gM, gX):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.step_graph_launch()
        torch.cuda.synchronize()
        assert torch.equal(L, L0) and torch.equal(C, C0) and torch.equal(gM, gM0) and torch.equal(gX, gX0), rep
        junk = torch.randn(1 << 20, device="cuda").sum()
        del junk


def test_autotune_saved_leaves_valid_results(ot):
    batch, M, X = synthetic.batched_config(2, 131, missing_frac=0.5)
    w = synthetic.weights(batch["T"], 132)
    plan = ot.Plan.from_batch(batch)
    NS, NT = batch["S"] * 512, batch["T"] * 512
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    L, Cs, gM, gX = _empty(20, NT), _empty(24, NT), _empty(20, NS), _empty(3, NS)
    f, b = plan.autotune_saved(Md, Xd, L, Cs, wd, gM, gX)
    for s in (f, b):
        assert (s & 0xF) in (1, 3) and not (s & ~0x3F)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w)
    assert_parity(_host(L), oracle.batched_forward(batch, M, X), TOL, what="autotune saved L")
    assert_parity(_host(gM), gM_ref, TOL, what="autotune saved gM")
    assert_parity(_host(gX), gX_ref, TOL, what="autotune saved gX")
    L2, Cs2, gM2, gX2 = _empty(20, NT), _empty(24, NT), _empty(20, NS), _empty(3, NS)
    plan.multipole_batched_save(Md, Xd, L2, Cs2)   # AUTO -> tuned
    plan.multipole_backward_saved(Md, Xd, wd, Cs2, gM2, gX2)
    assert np.array_equal(_host(gX2), _host(gX)) and np.array_equal(_host(L2), _host(L))


def test_invalid_schedules_and_overlaps_rejected(ot):
    batch, M, X = synthetic.batched_config(2, 133)
    plan = ot.Plan.from_batch(batch)
    NS, NT = batch["S"] * 512, batch["T"] * 512
    Md, Xd, wd = _dev(M), _dev(X), _dev(synthetic.weights(batch["T"], 134))
    L, Cs, gM, gX = _empty(20, NT), _empty(24, NT), _empty(20, NS), _empty(3, NS)
    for bad in (2, 0x12, 7, 0x10, 0x40 | 1, 1 << 8):
        with pytest.raises(ot.OtFmmError):
            plan.multipole_batched_save(Md, Xd, L, Cs, sched=bad)
        with pytest.raises(ot.OtFmmError):
            plan.multipole_backward_saved(Md, Xd, wd, Cs, gM, gX, sched=bad)
    import torch
    flat = torch.zeros(44 * NT, dtype=torch.float64, device="cuda")
    with pytest.raises(ot.OtFmmError):  # the sums overlapping L
        plan.multipole_batched_save(Md, Xd, flat[:20 * NT].view(20, NT), flat[10 * NT:34 * NT].view(24, NT),
                                    sched=3)
    with pytest.raises(ot.OtFmmError):  # gcom overlapping the sums
        plan.multipole_backward_saved(Md, Xd, wd, flat[:24 * NT].view(24, NT), gM,
                                      flat[:3 * NS].view(3, NS), sched=3)
