"""The C-ABI library loads, exports every symbol include/ot_fmm.h declares,
and rejects invalid arguments on the host before touching a device. CPU only
(no compute call is made)."""
import ctypes
import os
import re
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ot_fmm.h")
LIB = os.path.join(ROOT, "paper_2303_08058_amd", "libotfmm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ot_fmm_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import subprocess
        import sys
        subprocess.check_call([sys.executable, os.path.join(ROOT, "paper_2303_08058_amd", "build.py")])
    return ctypes.CDLL(LIB)


def test_header_declares_the_four_kernels():
    names = declared_functions()
    for n in ["ot_fmm_monopole", "ot_fmm_multipole", "ot_fmm_multipole_batched",
              "ot_fmm_multipole_backward"]:
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_version_and_strerror(lib):
    lib.ot_fmm_strerror.restype = ctypes.c_char_p
    assert lib.ot_fmm_version() == 100
    assert lib.ot_fmm_strerror(0) == b"ok"
    assert lib.ot_fmm_strerror(-1) == b"invalid argument"


def _plan_create(lib, S, T, tgt, nbr, shift=None, period=None):
    P = ctypes.c_void_p
    lib.ot_fmm_plan_create.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P,
                                       ctypes.POINTER(P)]
    h = P()
    tgt = np.ascontiguousarray(tgt, np.int32)
    nbr = np.ascontiguousarray(nbr, np.int32)
    sh = None if shift is None else np.ascontiguousarray(shift, np.int8)
    pe = None if period is None else np.ascontiguousarray(period, np.float64)
    rc = lib.ot_fmm_plan_create(S, T, tgt.ctypes.data_as(P), nbr.ctypes.data_as(P),
                                None if sh is None else sh.ctypes.data_as(P),
                                None if pe is None else pe.ctypes.data_as(P), ctypes.byref(h))
    return rc, h


def _good():
    nbr = np.full((2, 27), -1, np.int32)
    nbr[0, 13] = 0
    nbr[1, 13] = 1
    nbr[0, 14] = 1
    nbr[1, 12] = 0
    return 2, 2, np.array([0, 1]), nbr


@pytest.mark.parametrize("case", ["S0", "T0", "tgt_range", "tgt_dup", "nbr_range", "self_slot",
                                  "shift_no_period", "conflict", "too_large", "shift_minus128",
                                  "period_nan"])
def test_plan_create_rejects_bad_descriptors(lib, case):
    S, T, tgt, nbr = _good()
    shift, period = None, None
    if case == "S0":
        S = 0
    elif case == "T0":
        T = 0
    elif case == "tgt_range":
        tgt = np.array([0, 2])
    elif case == "tgt_dup":
        tgt = np.array([0, 0])
    elif case == "nbr_range":
        nbr[0, 3] = 5
    elif case == "self_slot":
        nbr[0, 13] = 1
    elif case == "shift_no_period":
        shift = np.zeros((2, 27, 3))
    elif case == "conflict":
        # targets 0 and 1 both claim sub-grid 1 at the same slot
        nbr[0, 14] = 1
        nbr[1, 14] = 1
        nbr[1, 12] = -1
        S, T, tgt = 3, 2, np.array([0, 2])
        nbr[1, 13] = 2
    elif case == "too_large":
        S = 1 << 27                      # 20 x 512 x S doubles exceed 2^40
    elif case == "shift_minus128":
        shift = np.zeros((2, 27, 3))
        shift[0, 14, 0] = -128           # its negation does not fit the reverse table
        period = np.ones(3)
    elif case == "period_nan":
        shift = np.zeros((2, 27, 3))
        period = np.array([1.0, np.nan, 1.0])
    rc, h = _plan_create(lib, S, T, tgt, nbr, shift, period)
    assert rc == -1


def test_kernels_reject_null_and_misaligned_pointers(lib):
    P = ctypes.c_void_p
    for fn in (lib.ot_fmm_monopole, lib.ot_fmm_multipole):
        fn.argtypes = [P, P, P, P]
        buf = (ctypes.c_double * 64)()
        base = ctypes.addressof(buf)
        assert fn(None, base, base, None) == -1
        assert fn(base + 4, base, base, None) == -1
    lib.ot_fmm_multipole_batched.argtypes = [P, P, P, P, ctypes.c_int, P]
    assert lib.ot_fmm_multipole_batched(None, None, None, None, 0, None) == -1
    for fn in (lib.ot_fmm_multipole_batched_save, lib.ot_fmm_multipole_batched_full_save,
               lib.ot_fmm_multipole_batched_amc):
        fn.argtypes = [P, P, P, P, P, ctypes.c_int, P]
        assert fn(None, None, None, None, None, 0, None) == -1
    for fn in (lib.ot_fmm_multipole_backward_saved, lib.ot_fmm_multipole_backward_full_saved):
        fn.argtypes = [P, P, P, P, P, P, P, ctypes.c_int, P]
        assert fn(None, None, None, None, None, None, None, 0, None) == -1
    for fn in (lib.ot_fmm_coarse_fine, lib.ot_fmm_coarse_fine_full):
        fn.argtypes = [P, P, P, P, P, P]
        assert fn(None, None, None, None, None, None) == -1
    lib.ot_fmm_plan_set_coarse.argtypes = [P, ctypes.c_int32, P, P, P]
    assert lib.ot_fmm_plan_set_coarse(None, 1, None, None, None) == -1
    lib.ot_fmm_last_error.restype = ctypes.c_char_p
    assert lib.ot_fmm_last_error() != b""


@pytest.mark.parametrize("case", ["range", "twice", "zero"])
def test_tree_create_rejects_bad_tables(lib, case):
    P = ctypes.c_void_p
    lib.ot_fmm_tree_create.argtypes = [ctypes.c_int32, ctypes.c_int32, P, ctypes.POINTER(P)]
    ch = np.arange(16, dtype=np.int32).reshape(2, 8)
    Sp, Sc = 2, 16
    if case == "range":
        ch[1, 3] = 16
    elif case == "twice":
        ch[1, 3] = 2
    else:
        Sp = 0
    h = P()
    assert lib.ot_fmm_tree_create(Sp, Sc, ch.ctypes.data_as(P), ctypes.byref(h)) == -1


def test_evaluate_rejects_bad_sizes(lib):
    P = ctypes.c_void_p
    lib.ot_fmm_evaluate.argtypes = [ctypes.c_int64, P, P, P, P, P]
    buf = (ctypes.c_double * 64)()
    base = ctypes.addressof(buf)
    assert lib.ot_fmm_evaluate(0, base, base, base, base, None) == -1
    assert lib.ot_fmm_evaluate(4, None, base, base, base, None) == -1


def test_overlapping_outputs_rejected_before_any_device_call(lib):
    """Output ranges that overlap inputs are EINVAL (checked from the extents,
    before the device is touched, so this runs without a GPU)."""
    P = ctypes.c_void_p
    buf = (ctypes.c_double * (30 * 13824))()
    base = ctypes.addressof(buf)
    base += (-base) % 16
    lib.ot_fmm_multipole.argtypes = [P, P, P, P]
    lib.ot_fmm_monopole.argtypes = [P, P, P, P]
    M, com = base, base + 20 * 13824 * 8
    assert lib.ot_fmm_multipole(M, com, M + 8 * 512 * 4, None) == -1          # L inside M
    assert lib.ot_fmm_monopole(M, com, com + 16, None) == -1                   # L inside com
    lib.ot_fmm_evaluate.argtypes = [ctypes.c_int64, P, P, P, P, P]
    n = 1024
    Mv, Lv = base, base + 20 * n * 8
    assert lib.ot_fmm_evaluate(n, Mv, Lv, Lv + 16 * 8, base + 60 * n * 8, None) == -1  # F inside L
    assert lib.ot_fmm_evaluate(n, Mv, Lv, base + 40 * n * 8, base + 41 * n * 8, None) == -1  # W inside F


def test_package_refuses_to_import_without_the_library(tmp_path):
    """No fallback: a copy of the package without libotfmm.so fails to import."""
    import shutil
    import subprocess
    src = os.path.join(ROOT, "paper_2303_08058_amd", "__init__.py")
    pkg = tmp_path / "paper_2303_08058_amd"
    pkg.mkdir()
    shutil.copy(src, pkg / "__init__.py")
    r = subprocess.run([sys.executable, "-c", "import paper_2303_08058_amd"], cwd=str(tmp_path),
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "libotfmm.so is not built" in r.stderr
