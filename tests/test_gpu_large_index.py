"""GPU parity where array indices pass 2^31: a periodic store of 60^3
sub-grids (216,000 sub-grids, 110.6M cells, every one a target), so that every
[20][cells] array (M, L, gL, gM) and the saved sums [24][cells] hold more than
2^31 elements (about 100 GB of device memory in all). The inputs are generated
on the device (synthetic.device_lattice_store); the oracle checks sampled
targets -- the first, the last and two between -- and sampled store
sub-grids on compact copies of their neighbourhoods (the 27 sub-grids of a
target's stencil; the 5^3 sub-grids whose targets reach a source sub-grid),
through the same criterion as the other parity tests (tests/parity.py,
tolerance 1e-12). Launches: the plain forward and the two-launch step, each
in its default schedule."""
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
N = 60


@pytest.fixture(scope="module")
def ot():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08058_amd as ot
    return ot


def _cols(t, ids):
    """Columns of the sub-grids ids of a (ncomp, n*512) device array, on the host."""
    import torch
    idx = torch.as_tensor(np.asarray(ids, np.int64), device=t.device)
    return t.reshape(t.shape[0], -1, SUB3).index_select(1, idx).reshape(t.shape[0], -1).cpu().numpy()


def _compact(batch, targets, store_ids):
    """A batch over the store sub-grids store_ids (in that order) with the
    given targets (store ids of the big batch, which are also its target ids),
    neighbour ids remapped and the shift rows kept."""
    local = {int(s): i for i, s in enumerate(store_ids)}
    tg = np.array([local[int(t)] for t in targets], np.int32)
    nbr = np.array([[local[int(s)] for s in batch["nbr"][t]] for t in targets], np.int32)
    return {"S": len(store_ids), "T": len(targets), "tgt": tg, "nbr": nbr,
            "shift": batch["shift"][np.asarray(targets)].copy(), "period": batch["period"]}


def test_store_past_two_to_the_31_elements(ot):
    import torch
    torch.cuda.empty_cache()
    batch = synthetic.lattice_batch(N)
    S = batch["S"]
    NS = S * SUB3
    assert 20 * NS > 2 ** 31 and 24 * NS > 2 ** 31
    print("large store: %d sub-grids, %d cells; generating on the device" % (S, NS), flush=True)
    M, X = synthetic.device_lattice_store(N, 606)
    g = torch.Generator(device="cuda")
    g.manual_seed(607)
    W = torch.randn((20, NS), generator=g, dtype=torch.float64, device="cuda")
    plan = ot.Plan.from_batch(batch)
    L = torch.empty((20, NS), dtype=torch.float64, device="cuda")
    plan.multipole_batched(M, X, L)
    Ls = torch.empty((20, NS), dtype=torch.float64, device="cuda")
    Cs = torch.empty((ot.NSAVED, NS), dtype=torch.float64, device="cuda")
    plan.multipole_batched_save(M, X, Ls, Cs)
    gM = torch.empty((20, NS), dtype=torch.float64, device="cuda")
    gX = torch.empty((3, NS), dtype=torch.float64, device="cuda")
    plan.multipole_backward_saved(M, X, W, Cs, gM, gX)
    torch.cuda.synchronize()
    print("launches done", flush=True)
    for t in (L, Ls, Cs, gM, gX):
        assert bool(torch.isfinite(t).all())

    # targets: the first, the last (the largest indices) and two between
    for t in (0, S // 3, 2 * S // 3 + 7, S - 1):
        store = [int(s) for s in batch["nbr"][t]]
        cb = _compact(batch, [t], store)
        Mc, Xc = _cols(M, store), _cols(X, store)
        ref, A = oracle.batched_forward(cb, Mc, Xc, want_abs=True)
        print("target %d L" % t, assert_parity(_cols(L, [t]), ref, TOL, what="large L %d" % t, A=A))
        assert_parity(_cols(Ls, [t]), ref, TOL, what="large saved-step L %d" % t, A=A)
        check_saved(_cols(Cs, [t]), cb, Mc, Xc, "large saved sums %d" % t)

    # store sub-grids: their gradients gather over the 27 targets that reach
    # them, whose sources span the 5^3 block around them
    sc = lambda s: np.array([s % N, (s // N) % N, s // (N * N)])
    for j in (S - 1, S // 2 + 11):
        c = sc(j)
        block = []
        for dz in range(-2, 3):
            for dy in range(-2, 3):
                for dx in range(-2, 3):
                    q = np.mod(c + np.array([dx, dy, dz]), N)
                    block.append(int(q[0] + N * q[1] + N * N * q[2]))
        targets = [int(s) for s in batch["nbr"][j]]
        cb = _compact(batch, targets, block)
        Mc, Xc = _cols(M, block), _cols(X, block)
        Wc = _cols(W, targets)
        gM_ref, gX_ref = oracle.batched_backward(cb, Mc, Xc, Wc, ssel=[block.index(j)])
        print("store %d gM" % j, assert_parity(_cols(gM, [j]), gM_ref, TOL, what="large gM %d" % j))
        print("store %d gX" % j, assert_parity(_cols(gX, [j]), gX_ref, TOL, what="large gX %d" % j))
    del M, X, W, L, Ls, Cs, gM, gX
    plan.close()
    torch.cuda.empty_cache()
