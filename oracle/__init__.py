"""Plain FP64 CPU oracle for the FMM cell-to-cell interaction kernels.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The library in
``paper_2303_08058_amd`` never imports, links or calls it, and it shares no
code with that library.

The arithmetic lives in ``ot_oracle.c`` (plain C99 + OpenMP, no fast-math);
this module compiles it with gcc and marshals numpy arrays through ctypes.
Definitions and pins are documented in the C file's header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "ot_oracle.c"), os.path.join(_HERE, "core.inc")]
_LIB = os.path.join(_HERE, "liboracle.so")

NM = 20
SUB3 = 512
HALO3 = 13824

_lib = None


def build(force: bool = True) -> str:
    """Compile ot_oracle.c into liboracle.so next to it (gcc, -O2, no fast-math)."""
    if not force and os.path.exists(_LIB):
        newest = max(os.path.getmtime(p) for p in _SRC)
        if os.path.getmtime(_LIB) >= newest:
            return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-std=gnu99", "-Wall", "-o", tmp, _SRC[0], "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i = ctypes.c_int
    lib.orc_multi_index.argtypes = [i, P]
    lib.orc_green.argtypes = [P, i, P]
    lib.orc_in_stencil.argtypes = [P, P]
    lib.orc_in_stencil.restype = i
    lib.orc_max_threads.restype = i
    lib.orc_green_general.argtypes = [P, i, P]
    lib.orc_green_general.restype = i
    for f in (lib.orc_block_forward, lib.orc_block_forward_full):
        f.argtypes = [P, i, P, i, P, P, i]
        f.restype = i
    for f in (lib.orc_batched_forward, lib.orc_batched_forward_full, lib.orc_batched_forward_tgrad,
              lib.orc_batched_forward_tgrad_full,
              lib.orc_batched_forward_amc):
        f.argtypes = [i, i, P, P, P, P, P, P, P, i, P, P, i]
        f.restype = i
    for f in (lib.orc_batched_forward_cs, lib.orc_batched_forward_cs_full,
              lib.orc_batched_backward, lib.orc_batched_backward_full):
        f.argtypes = [i, i, P, P, P, P, P, P, P, P, i, P, P, i]
        f.restype = i
    for f in (lib.orc_coarse_fine, lib.orc_coarse_fine_full):
        f.argtypes = [i, i, P, P, P, P, P, i, P, P, P, P, P, i, P, P, i]
        f.restype = i
    lib.orc_m2m.argtypes = [i, i, P, P, P, P, i, P, P, i]
    lib.orc_m2m.restype = i
    lib.orc_l2l.argtypes = [i, i, P, P, P, P, P, i]
    lib.orc_l2l.restype = i
    lib.orc_evaluate.argtypes = [ctypes.c_long, P, P, P, P, i]
    lib.orc_evaluate.restype = i
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def max_threads() -> int:
    return _load().orc_max_threads()


def multi_index(g: int):
    out = np.zeros(3, np.int32)
    _load().orc_multi_index(g, _ptr(out))
    return tuple(int(v) for v in out)


def green(r, order: int = 4) -> np.ndarray:
    """All derivatives d^gamma(-1/|r|) for |gamma| <= order, graded-lex order."""
    n = (order + 1) * (order + 2) * (order + 3) // 6
    r = _f64(r)
    out = np.zeros(n, np.float64)
    _load().orc_green(_ptr(r), order, _ptr(out))
    return out


def green_general(r, order: int = 6) -> np.ndarray:
    """d^gamma(-1/|r|) for |gamma| <= order (<= 7) from the general closed form
    (Hobson's formula), graded-lex order."""
    n = (order + 1) * (order + 2) * (order + 3) // 6
    r = _f64(r)
    out = np.zeros(n, np.float64)
    if _load().orc_green_general(_ptr(r), order, _ptr(out)):
        raise ValueError("order must be in 0..7")
    return out


def in_stencil(hi, hj) -> bool:
    a = _i32(hi)
    b = _i32(hj)
    return bool(_load().orc_in_stencil(_ptr(a), _ptr(b)))


def block_forward(M, X, mmax: int = 3, want_abs: bool = False, nthreads: int = 0,
                  full: bool = False):
    """Single 24^3 halo block. M: (nm, 13824) with nm in {1, 20}; X: (3, 13824).
    Returns L (20, 512) [and A (20, 512), the sum of term magnitudes].
    full=True: every output keeps every moment up to mmax (full truncation)."""
    M = _f64(M).reshape(-1, HALO3)
    X = _f64(X).reshape(3, HALO3)
    L = np.zeros((NM, SUB3), np.float64)
    A = np.zeros((NM, SUB3), np.float64) if want_abs else None
    fn = _load().orc_block_forward_full if full else _load().orc_block_forward
    rc = fn(_ptr(M), M.shape[0], _ptr(X), mmax, _ptr(L), _ptr(A), nthreads)
    if rc:
        raise ValueError("orc_block_forward rejected its arguments")
    return (L, A) if want_abs else L


def _batch_args(batch):
    tgt = _i32(batch["tgt"])
    nbr = _i32(batch["nbr"]).reshape(-1, 27)
    shift = batch.get("shift")
    period = batch.get("period")
    shift = None if shift is None else np.ascontiguousarray(shift, dtype=np.int8)
    period = None if period is None else _f64(period)
    return int(batch["S"]), int(batch["T"]), tgt, nbr, shift, period


def batched_forward(batch, M, X, tsel=None, want_abs: bool = False, nthreads: int = 0,
                    full: bool = False):
    """Batched forward over a selection of targets. Returns L (20, nsel*512).
    full=True: the full truncation (every output keeps every moment)."""
    S, T, tgt, nbr, shift, period = _batch_args(batch)
    tsel = np.arange(T, dtype=np.int32) if tsel is None else _i32(tsel)
    M = _f64(M)
    X = _f64(X)
    assert M.shape == (NM, S * SUB3) and X.shape == (3, S * SUB3)
    L = np.zeros((NM, len(tsel) * SUB3), np.float64)
    A = np.zeros_like(L) if want_abs else None
    fn = _load().orc_batched_forward_full if full else _load().orc_batched_forward
    rc = fn(S, T, _ptr(tgt), _ptr(nbr), _ptr(shift), _ptr(period), _ptr(M), _ptr(X), _ptr(tsel),
            len(tsel), _ptr(L), _ptr(A), nthreads)
    if rc:
        raise ValueError("orc_batched_forward rejected its arguments")
    return (L, A) if want_abs else L


def batched_forward_tgrad(batch, M, X, tsel=None, want_abs: bool = False, nthreads: int = 0,
                          full: bool = False):
    """Target-side derivatives of the forward, D[a, k] = dL_a(i)/dX_i,k with the
    sources' centres held fixed, over a selection of targets (full=True: of
    the full truncation's L).
    Returns D (20, 3, nsel*512) (and A, the term magnitudes, if want_abs)."""
    S, T, tgt, nbr, shift, period = _batch_args(batch)
    tsel = np.arange(T, dtype=np.int32) if tsel is None else _i32(tsel)
    M = _f64(M)
    X = _f64(X)
    assert M.shape == (NM, S * SUB3) and X.shape == (3, S * SUB3)
    D = np.zeros((NM, 3, len(tsel) * SUB3), np.float64)
    A = np.zeros_like(D) if want_abs else None
    lib = _load()
    fn = lib.orc_batched_forward_tgrad_full if full else lib.orc_batched_forward_tgrad
    rc = fn(S, T, _ptr(tgt), _ptr(nbr), _ptr(shift), _ptr(period), _ptr(M),
                                           _ptr(X), _ptr(tsel), len(tsel), _ptr(D), _ptr(A), nthreads)
    if rc:
        raise ValueError("orc_batched_forward_tgrad rejected its arguments")
    return (D, A) if want_abs else D


def batched_forward_amc(batch, M, X, tsel=None, want_abs: bool = False, nthreads: int = 0):
    """Angular-momentum correction of the force of each target cell, the
    terms of -dE/dX_i with |a| + |b| = 3 that the force evaluated from L
    lacks. Returns dF (3, nsel*512) (and A, the term magnitudes, if want_abs)."""
    S, T, tgt, nbr, shift, period = _batch_args(batch)
    tsel = np.arange(T, dtype=np.int32) if tsel is None else _i32(tsel)
    M = _f64(M)
    X = _f64(X)
    assert M.shape == (NM, S * SUB3) and X.shape == (3, S * SUB3)
    dF = np.zeros((3, len(tsel) * SUB3), np.float64)
    A = np.zeros_like(dF) if want_abs else None
    rc = _load().orc_batched_forward_amc(S, T, _ptr(tgt), _ptr(nbr), _ptr(shift), _ptr(period), _ptr(M),
                                         _ptr(X), _ptr(tsel), len(tsel), _ptr(dF), _ptr(A), nthreads)
    if rc:
        raise ValueError("orc_batched_forward_amc rejected its arguments")
    return (dF, A) if want_abs else dF


def batched_forward_cs(batch, M, Xre, Xim, tsel=None, nthreads: int = 0, full: bool = False):
    """Complex-position forward (for complex-step derivatives). Returns (Lre, Lim).
    full=True: the full truncation."""
    S, T, tgt, nbr, shift, period = _batch_args(batch)
    tsel = np.arange(T, dtype=np.int32) if tsel is None else _i32(tsel)
    M = _f64(M)
    Xre = _f64(Xre)
    Xim = _f64(Xim)
    Lre = np.zeros((NM, len(tsel) * SUB3), np.float64)
    Lim = np.zeros_like(Lre)
    fn = _load().orc_batched_forward_cs_full if full else _load().orc_batched_forward_cs
    rc = fn(S, T, _ptr(tgt), _ptr(nbr), _ptr(shift), _ptr(period), _ptr(M), _ptr(Xre), _ptr(Xim),
            _ptr(tsel), len(tsel), _ptr(Lre), _ptr(Lim), nthreads)
    if rc:
        raise ValueError("orc_batched_forward_cs rejected its arguments")
    return Lre, Lim


def batched_backward(batch, M, X, gL, ssel=None, nthreads: int = 0, full: bool = False):
    """Gradients of sum(gL * L) w.r.t. moments and centres of mass of the
    selected store sub-grids. Returns gM (20, nsel*512), gX (3, nsel*512).
    full=True: of the full-truncation forward."""
    S, T, tgt, nbr, shift, period = _batch_args(batch)
    ssel = np.arange(S, dtype=np.int32) if ssel is None else _i32(ssel)
    M = _f64(M)
    X = _f64(X)
    gL = _f64(gL)
    assert gL.shape == (NM, T * SUB3)
    gM = np.zeros((NM, len(ssel) * SUB3), np.float64)
    gX = np.zeros((3, len(ssel) * SUB3), np.float64)
    fn = _load().orc_batched_backward_full if full else _load().orc_batched_backward
    rc = fn(S, T, _ptr(tgt), _ptr(nbr), _ptr(shift), _ptr(period), _ptr(M), _ptr(X), _ptr(gL),
            _ptr(ssel), len(ssel), _ptr(gM), _ptr(gX), nthreads)
    if rc:
        raise ValueError("orc_batched_backward rejected its arguments")
    return gM, gX


def coarse_fine(batch, X, coarse, octant, Mp, Xp, tsel=None, want_abs: bool = False,
                nthreads: int = 0, full: bool = False):
    """Coarse contributions (20, nsel*512) for missing neighbours that have a
    coarse substitute: coarse / octant (T, 27), -1 where none; Mp, Xp the
    coarse store. full=True: the full truncation (every |b| <= 3)."""
    S, T, tgt, nbr, shift, period = _batch_args(batch)
    tsel = np.arange(T, dtype=np.int32) if tsel is None else _i32(tsel)
    X = _f64(X)
    Mp = _f64(Mp)
    Xp = _f64(Xp)
    Sp = Mp.shape[1] // SUB3
    coarse = _i32(coarse).reshape(T, 27)
    octant = np.ascontiguousarray(octant, dtype=np.int8).reshape(T, 27)
    L = np.zeros((NM, len(tsel) * SUB3), np.float64)
    A = np.zeros_like(L) if want_abs else None
    fn = _load().orc_coarse_fine_full if full else _load().orc_coarse_fine
    rc = fn(S, T, _ptr(tgt), _ptr(nbr), _ptr(shift), _ptr(period), _ptr(X), Sp,
            _ptr(coarse), _ptr(octant), _ptr(Mp), _ptr(Xp), _ptr(tsel), len(tsel),
            _ptr(L), _ptr(A), nthreads)
    if rc:
        raise ValueError("orc_coarse_fine rejected its arguments")
    return (L, A) if want_abs else L


# ---------------------------------------------------------------------------
# tree passes around the interaction
# ---------------------------------------------------------------------------
def m2m(children, Mc, Xc, psel=None, nthreads: int = 0):
    """Upward pass. children (Sp, 8) child node ids; Mc (20, Sc*512), Xc (3, Sc*512)
    -> Mp (20, nsel*512), Xp (3, nsel*512) for the selected parent nodes."""
    ch = _i32(children).reshape(-1, 8)
    Sp = ch.shape[0]
    Mc = _f64(Mc)
    Xc = _f64(Xc)
    Sc = Mc.shape[1] // SUB3
    psel = np.arange(Sp, dtype=np.int32) if psel is None else _i32(psel)
    Mp = np.zeros((NM, len(psel) * SUB3))
    Xp = np.zeros((3, len(psel) * SUB3))
    rc = _load().orc_m2m(Sp, Sc, _ptr(ch), _ptr(Mc), _ptr(Xc), _ptr(psel), len(psel), _ptr(Mp),
                         _ptr(Xp), nthreads)
    if rc:
        raise ValueError("orc_m2m rejected its arguments")
    return Mp, Xp


def l2l(children, Lp, Xp, Xc, Lc, nthreads: int = 0):
    """Downward pass: returns Lc + shifted parent expansions (Lc is not modified)."""
    ch = _i32(children).reshape(-1, 8)
    Lp = _f64(Lp)
    Xp = _f64(Xp)
    Xc = _f64(Xc)
    out = np.array(Lc, dtype=np.float64, order="C", copy=True)
    Sc = Xc.shape[1] // SUB3
    rc = _load().orc_l2l(ch.shape[0], Sc, _ptr(ch), _ptr(Lp), _ptr(Xp), _ptr(Xc), _ptr(out),
                         nthreads)
    if rc:
        raise ValueError("orc_l2l rejected its arguments")
    return out


def evaluate(M, L, nthreads: int = 0):
    """Per-cell force F (3, N) and energy W (N,) from moments and local expansion."""
    M = _f64(M)
    L = _f64(L)
    N = M.shape[1]
    F = np.zeros((3, N))
    W = np.zeros(N)
    rc = _load().orc_evaluate(N, _ptr(M), _ptr(L), _ptr(F), _ptr(W), nthreads)
    if rc:
        raise ValueError("orc_evaluate rejected its arguments")
    return F, W
