"""GPU parity of the batched forward with the full truncation (every output
|alpha| <= 3 keeps every source moment |beta| <= 3; derivatives of G to
order 6) against the CPU oracle's full truncation, through the C ABI.

Criterion as for the total-order forward (tests/parity.py): per sub-grid and
output order, max |got - ref| <= 1e-12 * max(max |ref|, 1e-2 * max A)."""
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


def _empty(*shape):
    import torch
    return torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")


# 1 W8, 2 W16, 3 W8P2; 0x10 persistent; 0x20 XCD-aware work order
@pytest.mark.parametrize("sched", [0, 1, 2, 3, 0x11, 0x21, 0x31, 0x33])
def test_full_small_periodic_with_missing(ot, sched):
    batch, M, X = synthetic.batched_config(2, 23, missing_frac=0.5)
    ref, A = oracle.batched_forward(batch, M, X, want_abs=True, full=True)
    plan = ot.Plan.from_batch(batch)
    L = _empty(20, batch["T"] * SUB3)
    plan.multipole_batched_full(_dev(M), _dev(X), L, sched=sched)
    got = _host(L)
    print("full worst", assert_parity(got, ref, TOL, what="full", A=A))
    L2 = _empty(20, batch["T"] * SUB3)
    plan.multipole_batched_full(_dev(M), _dev(X), L2, sched=sched)
    assert np.array_equal(_host(L2), got)


def test_full_open_domain_differs_from_total_order_by_the_extra_terms(ot):
    """Open 3^3 lattice: the full and total-order launches of the same plan
    differ by the terms |alpha| + |beta| > 3 only -- on the GPU as in the
    oracle."""
    batch, M, X = synthetic.batched_config(3, 24, periodic=False)
    sel = np.array([0, 13, 26], np.int32)
    ref_f, A_f = oracle.batched_forward(batch, M, X, tsel=sel, want_abs=True, full=True)
    ref_t, A_t = oracle.batched_forward(batch, M, X, tsel=sel, want_abs=True)
    plan = ot.Plan.from_batch(batch)
    dM, dX = _dev(M), _dev(X)
    Lf, Lt = _empty(20, batch["T"] * SUB3), _empty(20, batch["T"] * SUB3)
    plan.multipole_batched_full(dM, dX, Lf)
    plan.multipole_batched(dM, dX, Lt)
    cols = lambda a: a.reshape(20, -1, SUB3)[:, sel].reshape(20, -1)
    gf, gt = cols(_host(Lf)), cols(_host(Lt))
    assert_parity(gf, ref_f, TOL, what="full open", A=A_f)
    # order-0 outputs keep every moment in both truncations
    assert_parity(gf[:1], gt[:1], TOL, groups=[[0]], what="order 0 equal", A=A_f[:1])
    # order-3 outputs: the difference is the added moment terms, as in the oracle
    d_gpu, d_ref = gf[10:] - gt[10:], ref_f[10:] - ref_t[10:]
    assert np.max(np.abs(d_ref)) > 1e-6 * np.max(np.abs(ref_t[10:]))
    assert np.max(np.abs(d_gpu - d_ref)) <= 1e-12 * np.max(A_f[10:] + A_t[10:])


def test_full_config3_sampled(ot):
    """16^3 sub-grids, periodic, 15% of targets missing 1-9 neighbours: one
    launch over every target, a seeded sample compared with the oracle."""
    batch, M, X = synthetic.config3()
    plan = ot.Plan.from_batch(batch)
    L = _empty(20, batch["T"] * SUB3)
    plan.multipole_batched_full(_dev(M), _dev(X), L)
    got = _host(L)
    assert np.all(np.isfinite(got))
    rng = np.random.default_rng(31)
    miss = batch["missing_targets"]
    sel = np.sort(np.concatenate([rng.choice(miss, 6, replace=False),
                                  rng.choice(np.setdiff1d(np.arange(batch["T"]), miss), 6,
                                             replace=False)])).astype(np.int32)
    ref, A = oracle.batched_forward(batch, M, X, tsel=sel, want_abs=True, full=True)
    cols = got.reshape(20, -1, SUB3)[:, sel].reshape(20, -1)
    assert_parity(cols, ref, TOL, what="full config3", A=A)


def test_full_rejects_bad_arguments(ot):
    batch, M, X = synthetic.batched_config(2, 25)
    plan = ot.Plan.from_batch(batch)
    dM, dX = _dev(M), _dev(X)
    L = _empty(20, batch["T"] * SUB3)
    with pytest.raises(ot.OtFmmError):
        plan.multipole_batched_full(dM, dX, L, sched=0x07)
    import ctypes
    from paper_2303_08058_amd import _lib
    # L starting inside M: rejected from the extents
    rc = _lib.ot_fmm_multipole_batched_full(plan.handle, ctypes.c_void_p(dM.data_ptr()),
                                            ctypes.c_void_p(dX.data_ptr()),
                                            ctypes.c_void_p(dM.data_ptr() + 8 * 512), 0, None)
    assert rc == ot.OT_FMM_EINVAL


# ---------------------------------------------------------------------------
# adjoint of the full truncation
# ---------------------------------------------------------------------------
# target role | source role << 8: 1 W8, 3 W8P2, 0x10 persistent, 0x20 XCD-local
@pytest.fixture(scope="module")
def small_adjoint_case():
    batch, M, X = synthetic.batched_config(2, 26, missing_frac=0.5)
    w = synthetic.weights(batch["T"], 27)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w, full=True)
    return batch, M, X, w, gM_ref, gX_ref


@pytest.mark.parametrize("sched", [0, 0x0101, 0x0303, 0x2111, 0x1121, 0x3331])
def test_full_adjoint_small_periodic_with_missing(ot, small_adjoint_case, sched):
    batch, M, X, w, gM_ref, gX_ref = small_adjoint_case
    plan = ot.Plan.from_batch(batch)
    NS = batch["S"] * SUB3
    gM, gX = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward_full(_dev(M), _dev(X), _dev(w), gM, gX, sched=sched)
    print("full adjoint gM", assert_parity(_host(gM), gM_ref, TOL, what="full gM"))
    print("full adjoint gX", assert_parity(_host(gX), gX_ref, TOL, what="full gX"))
    gM2, gX2 = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward_full(_dev(M), _dev(X), _dev(w), gM2, gX2, sched=sched)
    assert np.array_equal(_host(gM2), _host(gM)) and np.array_equal(_host(gX2), _host(gX))


def test_full_adjoint_open_lattice_and_autograd(ot):
    """Open 3^3 lattice, every sub-grid a target: the autograd function with
    full=True gives the oracle's gradients of sum(w * L_full)."""
    import torch
    batch, M, X = synthetic.batched_config(3, 28, periodic=False)
    w = synthetic.weights(batch["T"], 29)
    sel = np.array([0, 13, 26], np.int32)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w, ssel=sel, full=True)
    plan = ot.Plan.from_batch(batch)
    cols = lambda a: a.reshape(a.shape[0], -1, SUB3)[:, sel].reshape(a.shape[0], -1)
    ref_L = oracle.batched_forward(batch, M, X, tsel=sel, full=True)
    for save in (True, False):  # one-pass adjoint from saved sums, or two passes
        Mt = _dev(M).requires_grad_(True)
        Xt = _dev(X).requires_grad_(True)
        L = ot.multipole(Mt, Xt, plan, full=True, save=save)
        (L * _dev(w)).sum().backward()
        assert_parity(cols(_host(Mt.grad)), gM_ref, TOL, what="autograd full gM save=%s" % save)
        assert_parity(cols(_host(Xt.grad)), gX_ref, TOL, what="autograd full gX save=%s" % save)
        assert_parity(cols(_host(L.detach())), ref_L, TOL, what="autograd full L save=%s" % save)


def test_full_adjoint_config4_sampled(ot):
    """8^3 sub-grids, open boundary, w ~ N(0, 1): sampled store sub-grids."""
    batch, M, X = synthetic.config4()
    w = synthetic.weights(batch["T"], 2004)
    plan = ot.Plan.from_batch(batch)
    NS = batch["S"] * SUB3
    gM, gX = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward_full(_dev(M), _dev(X), _dev(w), gM, gX)
    sel = np.array([0, 63, 200, 273, 511], np.int32)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w, ssel=sel, full=True)
    cols = lambda a: a.reshape(a.shape[0], -1, SUB3)[:, sel].reshape(a.shape[0], -1)
    print("config4 full gM", assert_parity(cols(_host(gM)), gM_ref, TOL, what="config4 full gM"))
    print("config4 full gX", assert_parity(cols(_host(gX)), gX_ref, TOL, what="config4 full gX"))


def test_full_adjoint_rejects_16_wavefronts(ot):
    batch, M, X = synthetic.batched_config(2, 30)
    plan = ot.Plan.from_batch(batch)
    w = synthetic.weights(batch["T"], 31)
    NS = batch["S"] * SUB3
    with pytest.raises(ot.OtFmmError) as e:
        plan.multipole_backward_full(_dev(M), _dev(X), _dev(w), _empty(20, NS), _empty(3, NS), sched=0x0102)
    assert e.value.code == ot.OT_FMM_EINVAL


@pytest.mark.parametrize("fsched,bsched", [(1, 0x0101), (0x11, 0x1111), (0x33, 0x3331)])
def test_full_caller_captured_graph_replays(ot, fsched, bsched):
    """The full forward and its adjoint captured into a caller's graph
    (torch.cuda.CUDAGraph) replay bit for bit like the eager launches,
    several times with eager work in between (persistent forms record their
    counter resets as kernel nodes)."""
    import torch
    batch, M, X = synthetic.batched_config(3, 97, missing_frac=0.3)
    w = synthetic.weights(batch["T"], 98)
    plan = ot.Plan.from_batch(batch)
    NS, NT = batch["S"] * SUB3, batch["T"] * SUB3
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    refL, refM, refX = _empty(20, NT), _empty(20, NS), _empty(3, NS)
    plan.multipole_batched_full(Md, Xd, refL, sched=fsched)
    plan.multipole_backward_full(Md, Xd, wd, refM, refX, sched=bsched)
    L, gM, gX = _empty(20, NT), _empty(20, NS), _empty(3, NS)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.multipole_batched_full(Md, Xd, L, sched=fsched, stream=s)
        plan.multipole_backward_full(Md, Xd, wd, gM, gX, sched=bsched, stream=s)
    for rep in range(3):
        for t in (L, gM, gX):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(L, refL) and torch.equal(gM, refM) and torch.equal(gX, refX), rep
        junk = torch.randn(1 << 20, device="cuda").sum()
        del junk


def test_full_config5_default_schedule_sampled(ot):
    """32^3 sub-grids (16.8M cells), periodic, 20% missing: the full
    truncation's forward and adjoint in the launch configuration the benchmark
    times (the default schedule), sampled targets and store sub-grids checked
    against the oracle's full truncation."""
    import torch
    batch, M, X = synthetic.config5()
    w = synthetic.weights(batch["T"], 2005)
    plan = ot.Plan.from_batch(batch)
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    NS, NT = batch["S"] * SUB3, batch["T"] * SUB3
    L, gM, gX = _empty(20, NT), _empty(20, NS), _empty(3, NS)
    plan.multipole_batched_full(Md, Xd, L)
    plan.multipole_backward_full(Md, Xd, wd, gM, gX)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(L).all()) and bool(torch.isfinite(gM).all()) and bool(torch.isfinite(gX).all())
    # the two-launch step (forward with saved sums, one-pass adjoint) as timed
    Ls, Cs = _empty(20, NT), _empty(24, NT)
    plan.multipole_batched_save(Md, Xd, Ls, Cs, full=True)
    gMs, gXs = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward_saved(Md, Xd, wd, Cs, gMs, gXs, full=True)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(Ls).all()) and bool(torch.isfinite(Cs).all())
    assert bool(torch.isfinite(gMs).all()) and bool(torch.isfinite(gXs).all())
    rng = np.random.default_rng(2006)
    miss = batch["missing_targets"]
    sel = np.sort(np.concatenate([rng.choice(miss, 2, replace=False),
                                  rng.choice(np.setdiff1d(np.arange(batch["T"]), miss), 2,
                                             replace=False)])).astype(np.int32)
    idx = torch.from_numpy(sel).long().cuda()
    cols = lambda t: t.reshape(t.shape[0], -1, SUB3)[:, idx].reshape(t.shape[0], -1).cpu().numpy()
    ref, A = oracle.batched_forward(batch, M, X, tsel=sel, want_abs=True, full=True)
    print("config5 full L", assert_parity(cols(L), ref, TOL, what="config5 full L", A=A))
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w, ssel=sel[:3], full=True)
    sub = torch.from_numpy(sel[:3]).long().cuda()
    cols3 = lambda t: t.reshape(t.shape[0], -1, SUB3)[:, sub].reshape(t.shape[0], -1).cpu().numpy()
    print("config5 full gM", assert_parity(cols3(gM), gM_ref, TOL, what="config5 full gM"))
    print("config5 full gX", assert_parity(cols3(gX), gX_ref, TOL, what="config5 full gX"))
    print("config5 full saved-step L", assert_parity(cols(Ls), ref, TOL, what="config5 full saved-step L", A=A))
    print("config5 full one-pass gM", assert_parity(cols3(gMs), gM_ref, TOL, what="config5 full one-pass gM"))
    print("config5 full one-pass gX", assert_parity(cols3(gXs), gX_ref, TOL, what="config5 full one-pass gX"))
    csel = sel[:2]
    ci = torch.from_numpy(csel).long().cuda()
    cs_cols = Cs.reshape(24, -1, SUB3)[:, ci].reshape(24, -1).cpu().numpy()
    check_saved(cs_cols, batch, M, X, "config5 full saved sums", tsel=csel, full=True)


# ---------------------------------------------------------------------------
# the two-launch step of the full truncation: forward with the target-side
# sums saved, one-pass adjoint from them
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("sched", [0, 1, 3, 0x11, 0x13, 0x23, 0x33])
def test_full_saved_step_small_periodic_with_missing(ot, small_adjoint_case, sched):
    batch, M, X, w, gM_ref, gX_ref = small_adjoint_case
    plan = ot.Plan.from_batch(batch)
    NS, NT = batch["S"] * SUB3, batch["T"] * SUB3
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    L, Cs = _empty(20, NT), _empty(24, NT)
    plan.multipole_batched_save(Md, Xd, L, Cs, sched=sched, full=True)
    Lh, Csh = _host(L), _host(Cs)
    ref, A = oracle.batched_forward(batch, M, X, want_abs=True, full=True)
    assert_parity(Lh, ref, TOL, what="full saved-step L", A=A)
    print("full saved sums", check_saved(Csh, batch, M, X, "full saved sums", full=True))
    gM, gX = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward_saved(Md, Xd, wd, Cs, gM, gX, sched=sched, full=True)
    gMh, gXh = _host(gM), _host(gX)
    print("full one-pass gM", assert_parity(gMh, gM_ref, TOL, what="full one-pass gM"))
    print("full one-pass gX", assert_parity(gXh, gX_ref, TOL, what="full one-pass gX"))
    L2, Cs2, gM2, gX2 = _empty(20, NT), _empty(24, NT), _empty(20, NS), _empty(3, NS)
    plan.multipole_batched_save(Md, Xd, L2, Cs2, sched=sched, full=True)
    plan.multipole_backward_saved(Md, Xd, wd, Cs2, gM2, gX2, sched=sched, full=True)
    assert np.array_equal(_host(L2), Lh) and np.array_equal(_host(Cs2), Csh)
    assert np.array_equal(_host(gM2), gMh) and np.array_equal(_host(gX2), gXh)


def test_full_saved_step_open_subset_of_targets(ot):
    """Open lattice, three targets with knocked-out neighbours: store
    sub-grids that are not targets have no target role."""
    rng = synthetic._rng(225)
    M, X = synthetic.store_field(3, rng, 2.0, 3.0, 0.6, sep=6.0)
    lat = synthetic.lattice_batch(3, periodic=False)
    tg = np.array([13, 4, 22], np.int32)
    nbr = lat["nbr"][tg].copy()
    nbr[0, [5, 21]] = -1
    nbr[1, 14] = -1
    batch = {"S": 27, "T": 3, "tgt": tg, "nbr": nbr, "shift": None, "period": None}
    w = synthetic.weights(3, 226)
    plan = ot.Plan.from_batch(batch)
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    L, Cs = _empty(20, 3 * SUB3), _empty(24, 3 * SUB3)
    plan.multipole_batched_save(Md, Xd, L, Cs, full=True)
    check_saved(_host(Cs), batch, M, X, "full saved sums open", full=True)
    gM, gX = _empty(20, 27 * SUB3), _empty(3, 27 * SUB3)
    plan.multipole_backward_saved(Md, Xd, wd, Cs, gM, gX, full=True)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w, full=True)
    assert_parity(_host(gM), gM_ref, TOL, what="full open gM")
    assert_parity(_host(gX), gX_ref, TOL, what="full open gX")


def test_full_saved_moment_gradient_equals_the_two_pass_adjoint_bitwise(ot):
    batch, M, X = synthetic.batched_config(3, 227, missing_frac=0.3)
    w = synthetic.weights(batch["T"], 228)
    plan = ot.Plan.from_batch(batch)
    NS, NT = batch["S"] * SUB3, batch["T"] * SUB3
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    L, Cs = _empty(20, NT), _empty(24, NT)
    plan.multipole_batched_save(Md, Xd, L, Cs, sched=3, full=True)
    gM, gX = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward_saved(Md, Xd, wd, Cs, gM, gX, sched=3, full=True)
    gM2, gX2 = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward_full(Md, Xd, wd, gM2, gX2, sched=ot.sched_bwd(1, 3))
    assert np.array_equal(_host(gM), _host(gM2))
    gX_ref = oracle.batched_backward(batch, M, X, w, full=True)[1]
    assert_parity(_host(gX), gX_ref, TOL, what="full gX 3^3")


def test_full_saved_rejects_bad_arguments(ot):
    batch, M, X = synthetic.batched_config(2, 229)
    plan = ot.Plan.from_batch(batch)
    NS, NT = batch["S"] * SUB3, batch["T"] * SUB3
    Md, Xd, wd = _dev(M), _dev(X), _dev(synthetic.weights(batch["T"], 230))
    L, Cs, gM, gX = _empty(20, NT), _empty(24, NT), _empty(20, NS), _empty(3, NS)
    for bad in (2, 0x12, 7, 0x10, 0x40 | 1, 1 << 8):
        with pytest.raises(ot.OtFmmError):
            plan.multipole_batched_save(Md, Xd, L, Cs, sched=bad, full=True)
        with pytest.raises(ot.OtFmmError):
            plan.multipole_backward_saved(Md, Xd, wd, Cs, gM, gX, sched=bad, full=True)
    import torch
    flat = torch.zeros(44 * NT, dtype=torch.float64, device="cuda")
    with pytest.raises(ot.OtFmmError):  # the sums overlapping L
        plan.multipole_batched_save(Md, Xd, flat[:20 * NT].view(20, NT), flat[10 * NT:34 * NT].view(24, NT),
                                    sched=3, full=True)
    with pytest.raises(ot.OtFmmError):  # gcom overlapping the sums
        plan.multipole_backward_saved(Md, Xd, wd, flat[:24 * NT].view(24, NT), gM,
                                      flat[:3 * NS].view(3, NS), sched=3, full=True)
