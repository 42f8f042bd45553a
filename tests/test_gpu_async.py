"""Per-sub-grid launches through the event-polling executor on the GPU: the
futures become ready only through polling, every continuation runs once, and
the results are bitwise those of the same kernel launched directly (and match
the oracle)."""
import os
import sys
import threading

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))
import oracle  # noqa: E402
import synthetic  # noqa: E402
from parity import assert_parity  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ot():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2303_08058_amd as ot
    return ot


def _blocks(k):
    b = synthetic.multipole_block(1002)
    out = []
    for i in range(k):
        # the same field, rescaled and moved: each block gives a different L
        out.append((b["M"] * (1.0 + 0.25 * i), b["com"] + 0.125 * i))
    return out


@pytest.mark.parametrize("nworkers", [0, 2])
def test_async_multipole_matches_direct_launches(ot, nworkers):
    import torch
    k = 24
    blocks = _blocks(k)
    dev = [(torch.from_numpy(M).cuda(), torch.from_numpy(X).cuda()) for M, X in blocks]
    direct = []
    for M, X in dev:
        L = torch.empty((20, 512), dtype=torch.float64, device="cuda")
        ot.ot_fmm_multipole(M, X, L)
        direct.append(L)
    torch.cuda.synchronize()

    ex = ot.Executor(nstreams=8, nworkers=nworkers)
    outs = [torch.full((20, 512), float("nan"), dtype=torch.float64, device="cuda") for _ in range(k)]
    torch.cuda.synchronize()  # inputs and outputs exist before the pool streams run
    done = []
    lock = threading.Lock()
    futs = []
    for i, ((M, X), L) in enumerate(zip(dev, outs)):
        f = ex.multipole_async(M, X, L)
        f.then(lambda i=i: (lock.acquire(), done.append(i), lock.release()))
        futs.append(f)
    for f in futs:
        f.wait(60.0)
        assert f.is_ready()
    # a last future on every pool stream: all of their work has completed
    for s in range(8):
        ex.get_future(ex.stream(s)).wait(60.0)
    assert ex.outstanding() == 0
    ex.close()
    assert sorted(done) == list(range(k))
    for i in range(k):
        assert torch.equal(outs[i], direct[i]), i
    ref = oracle.block_forward(blocks[0][0], blocks[0][1])
    assert_parity(outs[0].cpu().numpy(), ref, 1e-12, what="async multipole")


def test_future_of_a_torch_stream(ot):
    import torch
    ex = ot.Executor(nstreams=1, nworkers=1)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = torch.ones(1 << 24, dtype=torch.float64, device="cuda")
        b = a * 3.0
    f = ex.get_future(s)
    f.wait(60.0)
    assert ex.outstanding() == 0
    # completed by polling: the stream's work is done, so this read needs no sync
    assert float(b[-1].item()) == 3.0
    f.close()
    ex.close()
