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


@pytest.mark.parametrize("sched", [1, 2])
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


def test_backward_small_open(ot):
    batch, M, X = _small_adjoint_case()
    w = synthetic.weights(batch["T"], 42)
    gM_ref, gX_ref = oracle.batched_backward(batch, M, X, w)
    plan = ot.Plan.from_batch(batch)
    gM = _empty(20, 27 * 512)
    gX = _empty(3, 27 * 512)
    plan.multipole_backward(_dev(M), _dev(X), _dev(w), gM, gX)
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
