"""Allocation-free batched forward (ot_fmm_multipole_batched_noalloc):
called through the C ABI and compared with the plan-based entry point that
runs the same kernel (ot_fmm_multipole_batched, W16 | PERSISTENT) -- bitwise
-- and with the oracle (1e-12, per sub-grid and order), on two calls in a
row, the second with a smaller input; its host-side size limit; and the
device-side descriptor check, forced from the host with an out-of-range
neighbour id (the kernels drop it, so every access stays in bounds)."""
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


@pytest.fixture(scope="module")
def ot():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08058_amd as ot
    return ot


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _descriptor(ot, batch):
    import torch
    tgt = _dev(np.asarray(batch["tgt"], np.int32))
    nbr = _dev(np.asarray(batch["nbr"], np.int32))
    shift = None if batch.get("shift") is None else _dev(np.asarray(batch["shift"], np.int8))
    return tgt, nbr, shift, batch.get("period")


def _noalloc(ot, batch, M, X):
    import torch
    tgt, nbr, shift, period = _descriptor(ot, batch)
    L = torch.full((20, batch["T"] * 512), float("nan"), dtype=torch.float64, device="cuda")
    ot.ot_fmm_multipole_batched_noalloc(batch["S"], batch["T"], tgt, nbr, shift, period,
                                        _dev(M), _dev(X), L)
    return _host(L)


def _with_plan(ot, batch, M, X):
    import torch
    plan = ot.Plan.from_batch(batch)
    L = torch.full((20, batch["T"] * 512), float("nan"), dtype=torch.float64, device="cuda")
    plan.multipole_batched(_dev(M), _dev(X), L, sched=ot.SCHED_W16 | ot.SCHED_PERSISTENT)
    return _host(L)


def test_two_calls_match_the_plan_entry_point_and_the_oracle(ot):
    print("noalloc: 4^3 periodic store, then 2^3", flush=True)
    big, Mb, Xb = synthetic.batched_config(4, 41, missing_frac=0.5)
    small, Ms, Xs = synthetic.batched_config(2, 42, missing_frac=0.5)
    got_big = _noalloc(ot, big, Mb, Xb)
    assert ot.ot_fmm_noalloc_status()[0] == 0
    got_small = _noalloc(ot, small, Ms, Xs)
    assert ot.ot_fmm_noalloc_status()[0] == 0
    assert np.array_equal(got_big, _with_plan(ot, big, Mb, Xb))
    assert np.array_equal(got_small, _with_plan(ot, small, Ms, Xs))
    w1 = assert_parity(got_big, oracle.batched_forward(big, Mb, Xb), TOL, what="noalloc 4^3")
    w2 = assert_parity(got_small, oracle.batched_forward(small, Ms, Xs), TOL, what="noalloc 2^3")
    print("noalloc worst relative deviation %.2e, %.2e" % (w1, w2), flush=True)


def test_open_subset_of_targets(ot):
    """Open lattice, targets a subset of the store, no shifts (shift and
    period NULL)."""
    rng = synthetic._rng(43)
    M, X = synthetic.store_field(3, rng, 2.0, 3.0, 0.6, sep=6.0)
    full = synthetic.lattice_batch(3, periodic=False)
    tg = np.array([13, 4, 22, 0], np.int32)
    nbr = full["nbr"][tg].copy()
    nbr[0, [5, 21, 14]] = -1
    batch = {"S": 27, "T": 4, "tgt": tg, "nbr": nbr, "shift": None, "period": None}
    got = _noalloc(ot, batch, M, X)
    assert np.array_equal(got, _with_plan(ot, batch, M, X))
    assert_parity(got, oracle.batched_forward(batch, M, X), TOL, what="noalloc open subset")


def test_size_limit_rejected_before_any_work(ot):
    import torch
    T = ot.NOALLOC_MAX_T + 1
    tgt = torch.zeros(T, dtype=torch.int32, device="cuda")
    nbr = torch.full((T, 27), -1, dtype=torch.int32, device="cuda")
    M = torch.zeros((20, 512), dtype=torch.float64, device="cuda")
    X = torch.zeros((3, 512), dtype=torch.float64, device="cuda")
    L = torch.empty((20, T * 512), dtype=torch.float64, device="cuda")
    with pytest.raises(ot.OtFmmError) as ei:
        ot.ot_fmm_multipole_batched_noalloc(1, T, tgt, nbr, None, None, M, X, L)
    assert ei.value.code == ot.OT_FMM_EINVAL
    assert "32768" in str(ei.value)


def test_invalid_entry_is_dropped_reported_and_poisons_L(ot):
    batch, M, X = synthetic.batched_config(2, 44, missing_frac=0.0)
    bad = dict(batch)
    bad["nbr"] = np.array(batch["nbr"], np.int32, copy=True)
    bad["nbr"][3, 7] = batch["S"]  # out of range
    got = _noalloc(ot, bad, M, X)
    n, first = ot.ot_fmm_noalloc_status()
    assert n == 1 and first == 3 * 27 + 7
    assert np.isnan(got).all()
    # the next valid call is unaffected
    good = _noalloc(ot, batch, M, X)
    assert ot.ot_fmm_noalloc_status()[0] == 0
    assert np.array_equal(good, _with_plan(ot, batch, M, X))
