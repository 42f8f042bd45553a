"""Host-side parts of bench.py (CPU only): the one-GPU refusal, the exact
pair count it reports, and the CPU-baseline record."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(__file__))
import bench  # noqa: E402
import oracle  # noqa: E402
import synthetic  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_slot_pair_counts_follow_the_criterion():
    """The per-slot counts bench.py uses for the CPU sample: centre, face, edge
    and corner blocks of a full sub-grid's 921,088 pairs, equal to the
    library's own stencil tables (an independent count) and, for one target
    cell per slot, to a brute-force count with the oracle's criterion."""
    lib = os.path.join(ROOT, "paper_2303_08058_amd", "libotfmm.so")
    if not os.path.exists(lib):
        subprocess.check_call([sys.executable, os.path.join(ROOT, "paper_2303_08058_amd", "build.py")])
    import paper_2303_08058_amd as ot
    sp = np.array(bench._slot_pairs(np))
    assert sp.sum() == 921088
    kinds = {0: 173536, 1: 76672, 2: 20936, 3: 4536}  # by number of off-centre axes
    for slot in range(27):
        so = (slot % 3, (slot // 3) % 3, slot // 9)
        assert sp[slot] == kinds[sum(v != 1 for v in so)], slot
    lib_sp, _, _ = ot.ot_fmm_stencil_info()
    assert np.array_equal(sp, lib_sp)
    # cell (3, 5, 2) of the target against every cell of each neighbour block
    hi = (8 + 3, 8 + 5, 8 + 2)
    per_slot = [sum(oracle.in_stencil(hi, (8 * (s % 3) + j % 8, 8 * ((s // 3) % 3) + (j // 8) % 8,
                                             8 * (s // 9) + j // 64)) for j in range(512))
                for s in range(27)]
    assert sum(per_slot) == 1799


def test_cpu_baseline_record():
    batch, M, X = synthetic.batched_config(3, 7, missing_frac=0.3)
    w = synthetic.weights(batch["T"], 8)
    r = bench.cpu_baseline(batch, M, X, w, 0.2, np)
    assert r["kind"] == "oracle" and r["unit"] == "cell-pair interactions/s"
    assert r["value"] > 0 and r["one_core_value"] > 0
    assert r["cores"] == oracle.max_threads() >= 1
    assert "sub-grids" in r["sample"]
