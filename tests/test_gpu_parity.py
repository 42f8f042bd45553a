"""GPU parity of the HIP kernels against the CPU oracle on the same seeded
inputs (FP64, criterion in tests/parity.py, tolerance 1e-12), through the
C ABI. Small cases are compared element by element in full."""
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


def test_monopole_single_block(ot):
    b = synthetic.monopole_block(1001)
    ref = oracle.block_forward(b["mass"][None], b["com"])
    L = _empty(20, 512)
    ot.ot_fmm_monopole(_dev(b["mass"]), _dev(b["com"]), L)
    print("monopole worst", assert_parity(_host(L), ref, TOL, what="monopole"))


def test_multipole_single_block(ot):
    b = synthetic.multipole_block(1002)
    ref = oracle.block_forward(b["M"], b["com"])
    L = _empty(20, 512)
    ot.ot_fmm_multipole(_dev(b["M"]), _dev(b["com"]), L)
    print("multipole worst", assert_parity(_host(L), ref, TOL, what="multipole"))


# 1 W8, 2 W16, 3 W8P2; 0x10 = persistent launch
# 0x20 = XCD-aware work order
@pytest.mark.parametrize("sched", [1, 2, 3, 0x11, 0x12, 0x13, 0x22, 0x31, 0x32, 0x33])
def test_batched_small_periodic_with_missing(ot, sched):
    batch, M, X = synthetic.batched_config(2, 21, missing_frac=0.5)
    ref = oracle.batched_forward(batch, M, X)
    plan = ot.Plan.from_batch(batch)
    L = _empty(20, batch["T"] * 512)
    plan.multipole_batched(_dev(M), _dev(X), L, sched=sched)
    got = _host(L)
    print("batched worst", assert_parity(got, ref, TOL, what="batched"))
    # bitwise reproducible for a fixed schedule
    L2 = _empty(20, batch["T"] * 512)
    plan.multipole_batched(_dev(M), _dev(X), L2, sched=sched)
    assert np.array_equal(_host(L2), got)


def test_batched_open_subset_targets(ot):
    """Open 3^3 lattice; only some sub-grids are targets, with knocked-out
    neighbours (asymmetric availability)."""
    rng = synthetic._rng(31)
    M, X = synthetic.store_field(3, rng, 2.0, 3.0, 0.6, sep=6.0)
    full = synthetic.lattice_batch(3, periodic=False)
    tg = np.array([13, 4, 22, 0], np.int32)
    nbr = full["nbr"][tg].copy()
    nbr[0, [5, 21, 14]] = -1
    nbr[1, 22] = -1
    batch = {"S": 27, "T": 4, "tgt": tg, "nbr": nbr, "shift": None, "period": None}
    ref = oracle.batched_forward(batch, M, X)
    plan = ot.Plan.from_batch(batch)
    assert plan.pairs() == sum(slot_pair_counts()[s] for t in range(4) for s in range(27)
                               if nbr[t, s] >= 0)
    L = _empty(20, 4 * 512)
    plan.multipole_batched(_dev(M), _dev(X), L)
    assert_parity(_host(L), ref, TOL, what="batched open")


def slot_pair_counts():
    """Pairs between the 8^3 target cells and each neighbour block, counted
    from the criterion with numpy (|d|^2 > 16, parent distance^2 <= 16)."""
    c = np.arange(512)
    loc = np.stack([c % 8, (c // 8) % 8, c // 64], axis=1)
    ti = loc + 8
    out = []
    for slot in range(27):
        off = 8 * np.array([slot % 3, (slot // 3) % 3, slot // 9])
        tj = loc + off
        d = tj[None, :, :] - ti[:, None, :]
        p = tj[None, :, :] // 2 - ti[:, None, :] // 2
        out.append(int(np.count_nonzero(((d * d).sum(-1) > 16) & ((p * p).sum(-1) <= 16))))
    return out


def test_slot_pair_counts_add_up():
    n = slot_pair_counts()
    assert sum(n) == 512 * 1799
    assert n[13] == 173536 and n[14] == 76672 and n[0] == 4536


def _small_adjoint_case():
    rng = synthetic._rng(41)
    M, X = synthetic.store_field(3, rng, 2.0, 3.0, 0.6, sep=6.0)
    full = synthetic.lattice_batch(3, periodic=False)
    tg = np.array([13, 4, 22], np.int32)
    nbr = full["nbr"][tg].copy()
    nbr[0, [5, 21]] = -1
    nbr[1, 14] = -1
    batch = {"S": 27, "T": 3, "tgt": tg, "nbr": nbr, "shift": None, "period": None}
    return batch, M, X


# (target-role schedule, source-role schedule)
@pytest.mark.parametrize("sched", [(1, 1), (2, 1), (3, 3), (2, 3), (0x12, 0x11), (0x11, 0x13), (0x22, 0x21),
                                   (0x32, 0x31), (0x32, 0x33)])
def test_backward_small_open(ot, sched):
    batch, M, X = _small_adjoint_case()
    w = synthetic.weights(batch["T"], 42)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w)
    plan = ot.Plan.from_batch(batch)
    gM = _empty(20, 27 * 512)
    gX = _empty(3, 27 * 512)
    plan.multipole_backward(_dev(M), _dev(X), _dev(w), gM, gX, sched=ot.sched_bwd(*sched))
    print("gM worst", assert_parity(_host(gM), gM_ref, TOL, what="gM"))
    print("gX worst", assert_parity(_host(gX), gX_ref, TOL, what="gX"))


def test_backward_small_periodic_missing(ot):
    batch, M, X = synthetic.batched_config(2, 43, missing_frac=0.5)
    w = synthetic.weights(batch["T"], 44)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w)
    plan = ot.Plan.from_batch(batch)
    gM = _empty(20, batch["S"] * 512)
    gX = _empty(3, batch["S"] * 512)
    plan.multipole_backward(_dev(M), _dev(X), _dev(w), gM, gX)
    assert_parity(_host(gM), gM_ref, TOL, what="gM periodic")
    assert_parity(_host(gX), gX_ref, TOL, what="gX periodic")


# ---------------------------------------------------------------------------
# edge cases
# ---------------------------------------------------------------------------
def test_zero_masses_give_exact_zero(ot):
    b = synthetic.multipole_block(1002)
    L = _empty(20, 512)
    ot.ot_fmm_multipole(_dev(np.zeros((20, 13824))), _dev(b["com"]), L)
    assert np.all(_host(L) == 0.0)


def test_isolated_target_and_single_target(ot):
    """One target whose 26 neighbours are all missing (only its own pairs),
    next to a target with a full neighbourhood, in one launch."""
    batch, M, X = synthetic.batched_config(3, 51, periodic=True)
    tg = np.array([0, 13], np.int32)
    nbr = batch["nbr"][tg].copy()
    nbr[0, [s for s in range(27) if s != 13]] = -1
    b = {"S": 27, "T": 2, "tgt": tg, "nbr": nbr, "shift": batch["shift"][tg],
         "period": batch["period"]}
    ref = oracle.batched_forward(b, M, X)
    plan = ot.Plan.from_batch(b)
    assert plan.pairs() == 173536 + 921088
    L = _empty(20, 2 * 512)
    plan.multipole_batched(_dev(M), _dev(X), L)
    assert_parity(_host(L), ref, TOL, what="isolated")


def test_autograd_function_matches_oracle(ot):
    import torch
    batch, M, X = synthetic.batched_config(2, 61, missing_frac=0.5)
    plan = ot.Plan.from_batch(batch)
    Md = _dev(M).requires_grad_(True)
    Xd = _dev(X).requires_grad_(True)
    w = synthetic.weights(batch["T"], 62)
    L = ot.multipole(Md, Xd, plan)
    (L * _dev(w)).sum().backward()
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w)
    assert_parity(_host(Md.grad), gM_ref, TOL, what="autograd gM")
    assert_parity(_host(Xd.grad), gX_ref, TOL, what="autograd gX")
    assert L.dtype == torch.float64


@pytest.mark.parametrize("persistent", [0, 0x10, 0x30])
def test_step_graph_replays_match_eager(ot, persistent):
    """The captured forward+adjoint graph, replayed several times with eager
    work and synchronisations in between, reproduces the eager results
    bitwise on every replay (persistent launches: the work counters are
    zeroed by a kernel node of the graph on every replay)."""
    import torch
    P = persistent  # 0x10 persistent, 0x30 persistent in the XCD-aware pieces
    fs, bs = 2 | P, ot.sched_bwd(2 | P, (3 if P == 0x30 else 1) | P)
    batch, M, X = synthetic.batched_config(3, 71, missing_frac=0.3)
    plan = ot.Plan.from_batch(batch)
    Md, Xd = _dev(M), _dev(X)
    wd = _dev(synthetic.weights(batch["T"], 72))
    NS, NT = batch["S"] * 512, batch["T"] * 512
    L0, gM0, gX0 = _empty(20, NT), _empty(20, NS), _empty(3, NS)
    plan.multipole_batched(Md, Xd, L0, sched=fs & 0xF)
    plan.multipole_backward(Md, Xd, wd, gM0, gX0, sched=ot.sched_bwd(2, bs >> 8 & 0xF))
    L, gM, gX = _empty(20, NT), _empty(20, NS), _empty(3, NS)
    plan.step_graph_create(Md, Xd, L, wd, gM, gX, fs, bs)
    for rep in range(3):
        L.fill_(float("nan"))
        gX.fill_(float("nan"))
        torch.cuda.synchronize()
        plan.step_graph_launch()
        torch.cuda.synchronize()
        assert torch.equal(L, L0) and torch.equal(gM, gM0) and torch.equal(gX, gX0), rep
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        del junk


def test_autotune_choices_are_valid_and_exact(ot):
    batch, M, X = synthetic.batched_config(3, 81, missing_frac=0.3)
    plan = ot.Plan.from_batch(batch)
    Md, Xd = _dev(M), _dev(X)
    L = _empty(20, batch["T"] * 512)
    f, b = plan.autotune(Md, Xd, L)
    assert (f & 0xF) in (1, 2, 3) and (b & 0xF) in (1, 2, 3) and ((b >> 8) & 0xF) in (1, 3)
    assert not (f & ~0x3F) and not (b & ~0x3F3F)  # a shape and the persistent / local-order flags
    plan.multipole_batched(Md, Xd, L)   # AUTO -> tuned
    ref = oracle.batched_forward(batch, M, X, tsel=[0, 5, 26])
    got = _host(L).reshape(20, 27, 512)[:, [0, 5, 26]].reshape(20, -1)
    assert_parity(got, ref, TOL, what="autotuned")


def test_autotune_with_the_adjoint_leaves_valid_results(ot):
    """Autotuning both passes times the source- and target-role passes apart;
    afterwards gM and gcom hold the adjoint of the chosen schedules, and the
    tuned AUTO backward gives the same results bitwise."""
    batch, M, X = synthetic.batched_config(2, 82, missing_frac=0.5)
    w = synthetic.weights(batch["T"], 83)
    plan = ot.Plan.from_batch(batch)
    NS, NT = batch["S"] * 512, batch["T"] * 512
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    L, gM, gX = _empty(20, NT), _empty(20, NS), _empty(3, NS)
    f, b = plan.autotune(Md, Xd, L, wd, gM, gX)
    assert (b & 0xF) in (1, 2, 3) and ((b >> 8) & 0xF) in (1, 3) and not (b & ~0x3F3F)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w)
    assert_parity(_host(gM), gM_ref, TOL, what="autotune gM")
    assert_parity(_host(gX), gX_ref, TOL, what="autotune gX")
    gM2, gX2 = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward(Md, Xd, wd, gM2, gX2)  # AUTO -> tuned
    assert np.array_equal(_host(gM2), _host(gM)) and np.array_equal(_host(gX2), _host(gX))


def test_invalid_schedule_rejected(ot):
    batch, M, X = synthetic.batched_config(2, 91)
    plan = ot.Plan.from_batch(batch)
    L = _empty(20, batch["T"] * 512)
    for bad in (7, 0x10, 0x14, 0x40 | 2, 0x20):
        with pytest.raises(ot.OtFmmError):
            plan.multipole_batched(_dev(M), _dev(X), L, sched=bad)
    gM, gX = _empty(20, batch["S"] * 512), _empty(3, batch["S"] * 512)
    for bad in (ot.sched_bwd(2, 2), ot.sched_bwd(4, 1), 1 << 16, ot.sched_bwd(2, 0x12), 0x10, 0x14):
        with pytest.raises(ot.OtFmmError):
            plan.multipole_backward(_dev(M), _dev(X), L, gM, gX, sched=bad)


# ---------------------------------------------------------------------------
# full-size workloads, sampled outputs
# ---------------------------------------------------------------------------
def _sample_targets(batch, n_missing, n_random, seed):
    rng = np.random.default_rng(seed)
    miss = batch.get("missing_targets", np.zeros(0, np.int32))
    pick = list(rng.choice(miss, size=min(n_missing, len(miss)), replace=False)) if len(miss) else []
    rest = np.setdiff1d(np.arange(batch["T"]), pick)
    pick += list(rng.choice(rest, size=n_random, replace=False))
    return np.array(sorted(set(int(v) for v in pick)), np.int32)


def _cols(a, sel):
    return a.reshape(a.shape[0], -1, 512)[:, sel].reshape(a.shape[0], -1)


@pytest.fixture(scope="module")
def config3_reference():
    """16^3 sub-grids, periodic, 15% of the targets missing 1-9 neighbours:
    a seeded sample of 256 targets, half of them with missing neighbours,
    and the oracle's outputs and term magnitudes for them (computed once,
    shared by every schedule)."""
    batch, M, X = synthetic.config3()
    sel = _sample_targets(batch, 128, 128, 3)
    assert len(sel) == 256 and len(np.intersect1d(sel, batch["missing_targets"])) >= 128
    ref, A = oracle.batched_forward(batch, M, X, tsel=sel, want_abs=True)
    return batch, M, X, sel, ref, A


@pytest.mark.parametrize("sched", [1, 2, 3, 0x12, 0x22, 0x32])
def test_config3_forward_sampled(ot, config3_reference, sched):
    """Every output of the 16^3-sub-grid launch is produced; 256 seeded
    targets (half with missing neighbours) are compared with the oracle."""
    batch, M, X, sel, ref, A = config3_reference
    plan = ot.Plan.from_batch(batch)
    L = _empty(20, batch["T"] * 512)
    plan.multipole_batched(_dev(M), _dev(X), L, sched=sched)
    got = _host(L)
    assert np.all(np.isfinite(got))
    assert_parity(_cols(got, sel), ref, TOL, what="config3 sched 0x%x" % sched, A=A)


def test_config4_adjoint_full_and_fd():
    """8^3 sub-grids on an open domain, w ~ N(0,1): the gradients of all 512
    store sub-grids against the oracle's gradient, and 256 seeded entries
    against central differences of the GPU forward, outputs differenced
    first. Centres of mass: step 1e-6 (the rounding noise of the differenced
    loss, ~1e-13, limits this check to ~1e-7 relative; measured 3.2e-7 of
    max |grad| on these entries). Moments: L is linear in them, so a unit step
    is exact up to rounding."""
    import torch
    import paper_2303_08058_amd as ot
    batch, M, X = synthetic.config4()
    w = synthetic.weights(batch["T"], 1004 + 100)
    plan = ot.Plan.from_batch(batch)
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    NS = batch["S"] * 512
    gM, gX = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward(Md, Xd, wd, gM, gX)
    gM_h, gX_h = _host(gM), _host(gX)
    assert np.all(np.isfinite(gM_h)) and np.all(np.isfinite(gX_h))
    print("config4: oracle gradient of all %d store sub-grids ..." % batch["S"], flush=True)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w)
    print("config4 gM worst", assert_parity(gM_h, gM_ref, TOL, what="config4 gM"))
    print("config4 gX worst", assert_parity(gX_h, gX_ref, TOL, what="config4 gX"))
    # the one-pass adjoint from the sums its forward saved, on the same reference
    Ls = torch.empty((20, batch["T"] * 512), dtype=torch.float64, device="cuda")
    Cs = torch.empty((24, batch["T"] * 512), dtype=torch.float64, device="cuda")
    plan.multipole_batched_save(Md, Xd, Ls, Cs)
    gM2, gX2 = _empty(20, NS), _empty(3, NS)
    plan.multipole_backward_saved(Md, Xd, wd, Cs, gM2, gX2)
    del Ls, Cs
    print("config4 one-pass gM worst", assert_parity(_host(gM2), gM_ref, TOL, what="config4 one-pass gM"))
    print("config4 one-pass gX worst", assert_parity(_host(gX2), gX_ref, TOL, what="config4 one-pass gX"))

    # central differences of the GPU forward
    rng = np.random.default_rng(4)
    L = torch.empty((20, batch["T"] * 512), dtype=torch.float64, device="cuda")
    Lp, Lm = torch.empty_like(L), torch.empty_like(L)
    ent = rng.integers(0, NS, 256)
    comp = rng.integers(0, 23, 256)
    h = 1e-6
    fd, an = [], []
    for e, c in zip(ent, comp):
        if c < 20:
            step = 1.0
            arr, idx, grad = Md, (int(c), int(e)), gM_h[c, e]
        else:
            step = h
            arr, idx, grad = Xd, (int(c) - 20, int(e)), gX_h[c - 20, e]
        orig = arr[idx].item()
        arr[idx] = orig + step
        plan.multipole_batched(Md, Xd, Lp)
        arr[idx] = orig - step
        plan.multipole_batched(Md, Xd, Lm)
        arr[idx] = orig
        d = float(((Lp - Lm) * wd).sum()) / (2 * step)
        fd.append(d)
        an.append(grad)
    fd, an = np.array(fd), np.array(an)
    is_m = comp < 20
    dev_m = np.max(np.abs(fd[is_m] - an[is_m])) / np.max(np.abs(an[is_m]))
    dev_x = np.max(np.abs(fd[~is_m] - an[~is_m])) / np.max(np.abs(an[~is_m]))
    print("fd max deviation: moments %.2e, centres %.2e (relative to max |grad|)" % (dev_m, dev_x))
    # L is linear in M: differences are exact up to rounding
    assert dev_m <= 1e-9
    assert dev_x <= 1e-6


def test_config5_step_graph_sampled():
    """32^3 sub-grids (16.8M cells), periodic, 20% missing: the benchmark's
    launch configurations (autotuned schedules; the captured two-launch step
    -- forward with saved sums, one-pass adjoint -- and the captured
    three-launch step) with 256 seeded targets and the same 256 store
    sub-grids (half of them with missing neighbours) checked against the
    oracle, and the saved sums of 16 of those targets."""
    import torch
    import paper_2303_08058_amd as ot
    batch, M, X = synthetic.config5()
    w = synthetic.weights(batch["T"], 2005)
    plan = ot.Plan.from_batch(batch)
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    NS, NT = batch["S"] * 512, batch["T"] * 512
    L = torch.empty((20, NT), dtype=torch.float64, device="cuda")
    gM = torch.empty((20, NS), dtype=torch.float64, device="cuda")
    gX = torch.empty((3, NS), dtype=torch.float64, device="cuda")
    fs, bs = plan.autotune(Md, Xd, L, wd, gM, gX)
    print("config5: autotuned 0x%x 0x%x" % (fs, bs), flush=True)
    plan.step_graph_create(Md, Xd, L, wd, gM, gX, fs, bs)
    L.fill_(float("nan"))
    gM.fill_(float("nan"))
    gX.fill_(float("nan"))
    plan.step_graph_launch()
    torch.cuda.synchronize()
    assert bool(torch.isfinite(L).all()) and bool(torch.isfinite(gM).all()) and bool(torch.isfinite(gX).all())
    sel = _sample_targets(batch, 128, 128, 5)
    assert len(sel) == 256
    idx = torch.from_numpy(sel).long().cuda()
    Ls = L.reshape(20, -1, 512)[:, idx].reshape(20, -1).cpu().numpy()
    ssel = batch["tgt"][sel].astype(np.int32)
    sidx = torch.from_numpy(ssel).long().cuda()
    gMs = gM.reshape(20, -1, 512)[:, sidx].reshape(20, -1).cpu().numpy()
    gXs = gX.reshape(3, -1, 512)[:, sidx].reshape(3, -1).cpu().numpy()
    # the two-launch step the benchmark times, on the same buffers
    Cs = torch.empty((24, NT), dtype=torch.float64, device="cuda")
    sf, sb = plan.autotune_saved(Md, Xd, L, Cs, wd, gM, gX)
    print("config5: two-launch step autotuned 0x%x 0x%x" % (sf, sb), flush=True)
    plan.step_graph_create_saved(Md, Xd, L, Cs, wd, gM, gX, sf, sb)
    for t in (L, Cs, gM, gX):
        t.fill_(float("nan"))
    plan.step_graph_launch()
    torch.cuda.synchronize()
    assert bool(torch.isfinite(L).all()) and bool(torch.isfinite(gM).all()) and bool(torch.isfinite(gX).all())
    assert bool(torch.isfinite(Cs).all())
    Ls2 = L.reshape(20, -1, 512)[:, idx].reshape(20, -1).cpu().numpy()
    gMs2 = gM.reshape(20, -1, 512)[:, sidx].reshape(20, -1).cpu().numpy()
    gXs2 = gX.reshape(3, -1, 512)[:, sidx].reshape(3, -1).cpu().numpy()
    csel = sel[::16]
    Css = Cs.reshape(24, -1, 512)[:, torch.from_numpy(csel).long().cuda()].reshape(24, -1).cpu().numpy()
    del L, gM, gX, Cs
    print("config5: oracle forward of 256 targets ...", flush=True)
    ref, A = oracle.batched_forward(batch, M, X, tsel=sel, want_abs=True)
    assert_parity(Ls, ref, TOL, what="config5 L", A=A)
    assert_parity(Ls2, ref, TOL, what="config5 two-launch L", A=A)
    print("config5: oracle gradient of 256 store sub-grids ...", flush=True)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w, ssel=ssel)
    print("config5 gM worst", assert_parity(gMs, gM_ref, TOL, what="config5 gM"))
    print("config5 gX worst", assert_parity(gXs, gX_ref, TOL, what="config5 gX"))
    print("config5 two-launch gM worst", assert_parity(gMs2, gM_ref, TOL, what="config5 two-launch gM"))
    print("config5 two-launch gX worst", assert_parity(gXs2, gX_ref, TOL, what="config5 two-launch gX"))
    print("config5: oracle target-side sums of %d targets ..." % len(csel), flush=True)
    check_saved(Css, batch, M, X, "config5 saved sums", tsel=csel)


# the four (sigma1, sigma2) draws of the 32^3-sub-grid field's recipe
# (sigma in {2, 4}, q ~ U[0.3, 1.0]), on an 8^3-sub-grid periodic store with
# 20% of the targets missing 1-9 neighbours
@pytest.mark.parametrize("seed,sigmas", [(2000, (2.0, 4.0)), (2001, (2.0, 2.0)),
                                         (2002, (4.0, 4.0)), (2003, (4.0, 2.0))])
def test_field_sweep_forward_and_adjoint_sampled(ot, seed, sigmas):
    batch, M, X = synthetic.batched_config(8, seed, missing_frac=0.20, sigma_choices=[2.0, 4.0],
                                           q_range=(0.3, 1.0))
    assert (batch["field"]["sigma1"], batch["field"]["sigma2"]) == sigmas
    w = synthetic.weights(batch["T"], seed + 1)
    plan = ot.Plan.from_batch(batch)
    Md, Xd, wd = _dev(M), _dev(X), _dev(w)
    NS, NT = batch["S"] * 512, batch["T"] * 512
    L = _empty(20, NT)
    gM, gX = _empty(20, NS), _empty(3, NS)
    plan.multipole_batched(Md, Xd, L)
    plan.multipole_backward(Md, Xd, wd, gM, gX)
    sel = _sample_targets(batch, 3, 3, seed)
    ref, A = oracle.batched_forward(batch, M, X, tsel=sel, want_abs=True)
    assert_parity(_cols(_host(L), sel), ref, TOL, what="sweep L", A=A)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w, ssel=sel[:3])
    assert_parity(_cols(_host(gM), sel[:3]), gM_ref, TOL, what="sweep gM")
    assert_parity(_cols(_host(gX), sel[:3]), gX_ref, TOL, what="sweep gX")


def test_overlapping_outputs_rejected(ot):
    """An output whose range overlaps an input is refused with EINVAL and
    nothing is written."""
    import torch
    batch, M, X = synthetic.batched_config(2, 93)
    plan = ot.Plan.from_batch(batch)
    NS, NT = batch["S"] * 512, batch["T"] * 512
    Md, Xd = _dev(M), _dev(X)
    big = torch.zeros(40 * NS, dtype=torch.float64, device="cuda")
    L_in_M = big[: 20 * NT].view(20, NT)
    Mb = big[8 * 512: 8 * 512 + 20 * NS].view(20, NS)   # M shifted by one sub-grid into the same buffer
    Mb.copy_(Md)
    with pytest.raises(ot.OtFmmError) as e:
        plan.multipole_batched(Mb, Xd, L_in_M)
    assert e.value.code == ot.OT_FMM_EINVAL
    w = _dev(synthetic.weights(batch["T"], 94))
    gX = _empty(3, NS)
    with pytest.raises(ot.OtFmmError) as e:
        plan.multipole_backward(Md, Xd, w, w.view(-1)[: 20 * NS].view(20, NS) if NT >= NS else w, gX)
    assert e.value.code == ot.OT_FMM_EINVAL
    # the autotuner and the step-graph capture apply the same rule
    L = _empty(20, NT)
    gM = _empty(20, NS)
    with pytest.raises(ot.OtFmmError) as e:
        plan.autotune(Mb, Xd, L_in_M)
    assert e.value.code == ot.OT_FMM_EINVAL
    with pytest.raises(ot.OtFmmError) as e:
        plan.step_graph_create(Md, Xd, L, w, gM, gM.view(-1)[: 3 * NS].view(3, NS))   # gcom inside gM
    assert e.value.code == ot.OT_FMM_EINVAL
    with pytest.raises(ot.OtFmmError) as e:
        plan.step_graph_create(Md, Xd, L, L, gM, gX)   # gL aliasing L
    assert e.value.code == ot.OT_FMM_EINVAL
    torch.cuda.synchronize()
    assert torch.equal(Mb, Md)  # untouched


@pytest.mark.parametrize("sched", [0x22, 0x12, 0x32])
def test_concurrent_launches_of_one_plan_on_two_streams(ot, sched):
    """Two forward launches of the same plan in flight at once on two streams
    (persistent launches take separate counter slots) give the eager result."""
    import torch
    batch, M, X = synthetic.batched_config(3, 95, missing_frac=0.3)
    plan = ot.Plan.from_batch(batch)
    NT = batch["T"] * 512
    Md, Xd = _dev(M), _dev(X)
    ref = _empty(20, NT)
    plan.multipole_batched(Md, Xd, ref, sched=2)
    torch.cuda.synchronize()
    outs = [_empty(20, NT) for _ in range(4)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    torch.cuda.synchronize()
    for k, L in enumerate(outs):
        plan.multipole_batched(Md, Xd, L, sched=sched, stream=streams[k % 2])
    torch.cuda.synchronize()
    for L in outs:
        assert torch.equal(L, ref)


@pytest.mark.parametrize("sched", [0x22, 0x12, 0x32])
def test_caller_captured_graph_replays(ot, sched):
    """The batched forward captured into a caller's graph (torch.cuda.CUDAGraph)
    replays correctly several times, with eager work in between (the
    persistent form records its counter reset as a kernel node)."""
    import torch
    batch, M, X = synthetic.batched_config(3, 96, missing_frac=0.3)
    plan = ot.Plan.from_batch(batch)
    NT = batch["T"] * 512
    Md, Xd = _dev(M), _dev(X)
    ref = _empty(20, NT)
    plan.multipole_batched(Md, Xd, ref, sched=sched)
    L = _empty(20, NT)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.multipole_batched(Md, Xd, L, sched=sched, stream=s)
    for rep in range(3):
        L.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(L, ref), rep
        junk = torch.randn(1 << 20, device="cuda").sum()
        del junk


@pytest.mark.parametrize("sched", [0x12, 0x32])
def test_captured_graph_beside_eager_persistent_launches(ot, sched):
    """A persistent forward recorded into a caller's graph replays on one
    stream while eager persistent launches of the same plan run on another.
    More eager launches than the plan has per-stream counter sets come first,
    so a rotating assignment of counters would have handed the graph's set to
    one of them. Every replay and every eager launch gives the eager result."""
    import torch
    batch, M, X = synthetic.batched_config(3, 97, missing_frac=0.3)
    plan = ot.Plan.from_batch(batch)
    NT = batch["T"] * 512
    Md, Xd = _dev(M), _dev(X)
    ref = _empty(20, NT)
    plan.multipole_batched(Md, Xd, ref, sched=sched)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    Lg = _empty(20, NT)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s1):
        plan.multipole_batched(Md, Xd, Lg, sched=sched, stream=s1)
    outs = [_empty(20, NT) for _ in range(3)]
    for k in range(70):
        plan.multipole_batched(Md, Xd, outs[k % 3], sched=sched, stream=s2)
    torch.cuda.synchronize()
    for rep in range(3):
        Lg.fill_(float("nan"))
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(s1):
            g.replay()
        for o in outs:
            plan.multipole_batched(Md, Xd, o, sched=sched, stream=s2)
        torch.cuda.synchronize()
        assert torch.equal(Lg, ref), rep
        for o in outs:
            assert torch.equal(o, ref), rep


def test_eight_byte_aligned_arrays(ot):
    """Arrays that start one double past a 16-byte boundary (the alignment of a
    double is what the entry points require): the same bits as aligned ones,
    for the single-block kernel, the batched forward and the two-launch step."""
    import torch
    f64 = dict(dtype=torch.float64, device="cuda")

    def odd(shape, src=None):
        n = int(np.prod(shape))
        t = torch.zeros(n + 1, **f64)[1:].view(*shape)
        assert t.data_ptr() % 16 == 8
        if src is not None:
            t.copy_(torch.from_numpy(np.ascontiguousarray(src)))
        return t

    b = synthetic.multipole_block(1002)
    La, Lo = _empty(20, 512), odd((20, 512))
    ot.ot_fmm_multipole(_dev(b["M"]), _dev(b["com"]), La)
    ot.ot_fmm_multipole(odd((20, 13824), b["M"]), odd((3, 13824), b["com"]), Lo)
    assert np.array_equal(_host(La), _host(Lo))

    batch, M, X = synthetic.batched_config(2, 23, missing_frac=0.3)
    w = synthetic.weights(batch["T"], 24)
    plan = ot.Plan.from_batch(batch)
    NS, NT = batch["S"] * 512, batch["T"] * 512
    Ma, Xa, wa = _dev(M), _dev(X), _dev(w)
    Mo, Xo, wo = odd((20, NS), M), odd((3, NS), X), odd((20, NT), w)
    for sched in (2, 0x33):
        La, Lo = _empty(20, NT), odd((20, NT))
        plan.multipole_batched(Ma, Xa, La, sched=sched)
        plan.multipole_batched(Mo, Xo, Lo, sched=sched)
        assert np.array_equal(_host(La), _host(Lo))
    Ca, Co = _empty(24, NT), odd((24, NT))
    gMa, gXa, gMo, gXo = _empty(20, NS), _empty(3, NS), odd((20, NS)), odd((3, NS))
    plan.multipole_batched_save(Ma, Xa, La, Ca, sched=3)
    plan.multipole_backward_saved(Ma, Xa, wa, Ca, gMa, gXa, sched=3)
    plan.multipole_batched_save(Mo, Xo, Lo, Co, sched=3)
    plan.multipole_backward_saved(Mo, Xo, wo, Co, gMo, gXo, sched=3)
    for a, o in ((La, Lo), (Ca, Co), (gMa, gMo), (gXa, gXo)):
        assert np.array_equal(_host(a), _host(o))
    assert_parity(_host(Lo), oracle.batched_forward(batch, M, X), TOL, what="8-byte aligned L")
