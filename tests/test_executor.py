"""Host-side behaviour of the event-polling futures (ot_fmm_executor_*,
ot_fmm_future_*) with host futures only: no GPU call is made, so these run on
the CPU. The GPU-event path is covered by tests/test_gpu_async.py."""
import threading
import time

import pytest

ot = pytest.importorskip("paper_2303_08058_amd")


def test_continuation_runs_in_poll_without_workers():
    ex = ot.Executor(nstreams=2, nworkers=0)
    f = ex.future()
    ran = []
    f.then(lambda: ran.append(1))
    assert ex.poll() == 0 and ran == []
    f.set_ready()
    assert ran == []            # queued, not run by set_ready itself
    ex.poll()
    assert ran == [1] and f.is_ready()
    f.then(lambda: ran.append(2))   # already ready: queued at once
    f.wait(1.0)
    assert ran == [1, 2]
    f.close()
    ex.close()


def test_many_futures_with_workers_each_continuation_once():
    ex = ot.Executor(nstreams=1, nworkers=3)
    n = 600
    futs = [ex.future() for _ in range(n)]
    hits = [0] * n
    lock = threading.Lock()

    def cont(i):
        def run():
            with lock:
                hits[i] += 1
        return run

    for i, f in enumerate(futs):
        f.then(cont(i))
        f.then(cont(i))

    def setter(lo):
        for f in futs[lo::4]:
            f.set_ready()

    th = [threading.Thread(target=setter, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for f in futs:
        f.wait(5.0)
    deadline = time.time() + 5
    while sum(hits) < 2 * n and time.time() < deadline:
        time.sleep(0.01)
    assert hits == [2] * n
    for f in futs:
        f.close()
    ex.close()


def test_wait_times_out_and_reports():
    ex = ot.Executor(nstreams=1, nworkers=0)
    f = ex.future()
    t0 = time.time()
    with pytest.raises(ot.OtFmmError) as e:
        f.wait(0.05)
    assert e.value.code == ot.OT_FMM_ETIMEDOUT
    assert time.time() - t0 < 2.0
    f.set_ready()
    f.wait(0.05)
    with pytest.raises(ot.OtFmmError) as e:
        f.set_ready()
    assert e.value.code == ot.OT_FMM_EINVAL
    f.close()
    ex.close()


def test_concurrent_pollers_skip_instead_of_waiting():
    ex = ot.Executor(nstreams=1, nworkers=0)
    seen = set()
    lock = threading.Lock()

    def poller():
        for _ in range(2000):
            v = ex.poll()
            with lock:
                seen.add(v)

    th = [threading.Thread(target=poller) for _ in range(6)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert seen <= {-1, 0} and 0 in seen
    ex.close()


def test_destroy_runs_queued_tasks_and_bad_arguments():
    ex = ot.Executor(nstreams=1, nworkers=0)
    ran = []
    for i in range(5):
        ex.post(lambda i=i: ran.append(i))
    assert ex.outstanding() == 0
    ex.close()
    assert ran == [0, 1, 2, 3, 4]
    for ns, nw in ((0, 0), (2000, 0), (1, -1), (1, 1000)):
        with pytest.raises(ot.OtFmmError) as e:
            ot.Executor(ns, nw)
        assert e.value.code == ot.OT_FMM_EINVAL


def test_concurrent_set_ready_succeeds_exactly_once():
    """Threads racing to make one host future ready: one succeeds, the others
    get EINVAL, and its continuation runs once."""
    ex = ot.Executor(nstreams=1, nworkers=2)
    for _ in range(20):
        f = ex.future()
        ran = []
        lock = threading.Lock()

        def cont():
            with lock:
                ran.append(1)
        f.then(cont)
        ok, refused = [], []
        barrier = threading.Barrier(8)

        def racer():
            barrier.wait()
            try:
                f.set_ready()
                ok.append(1)
            except ot.OtFmmError as e:
                assert e.code == ot.OT_FMM_EINVAL
                refused.append(1)
        ts = [threading.Thread(target=racer) for _ in range(8)]
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        f.wait(5.0)
        deadline = time.time() + 5.0
        while not ran and time.time() < deadline:
            time.sleep(0.001)
        assert len(ok) == 1 and len(refused) == 7
        time.sleep(0.01)
        assert ran == [1]
        f.close()
    ex.close()
