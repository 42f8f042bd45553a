"""MI355X (gfx950) FP64 fast-multipole cell-to-cell interaction kernels.

Thin Python binding of the C ABI in ``include/ot_fmm.h`` (library
``libotfmm.so`` next to this file, built by ``paper_2303_08058_amd/build.py``).
Functions keep the C names and only marshal arguments: device pointers of
float64 torch tensors and the current HIP stream. Every step of the
computation runs in the HIP kernels; there is no CPU fallback, and importing
the package fails if the library has not been built.

Layouts and conventions: see the header (halo blocks [ncomp][13824], stores
[ncomp][S*512], outputs [20][512] or [20][T*512], components in graded
lexicographic order).
"""
from __future__ import annotations

import ctypes
import itertools
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libotfmm.so")

OT_FMM_OK = 0
OT_FMM_EINVAL = -1
OT_FMM_EHIP = -2
OT_FMM_ENOMEM = -3
OT_FMM_EUNSUPPORTED = -4
OT_FMM_ETIMEDOUT = -5

SCHED_AUTO = 0
SCHED_W8 = 1
SCHED_W16 = 2
SCHED_W8P2 = 3
SCHED_PERSISTENT = 0x10  # flag OR-ed into a schedule
SCHED_LOCAL = 0x20       # flag OR-ed into a schedule: XCD-aware work order


def sched_bwd(target_role=SCHED_AUTO, source_role=SCHED_AUTO):
    """Backward schedule: target-role pass in the low byte, source-role pass in the next."""
    return int(target_role) | (int(source_role) << 8)

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libotfmm.so is not built; run `python paper_2303_08058_amd/build.py` "
        "(the HIP library is required, there is no fallback)")

_lib = ctypes.CDLL(LIB_PATH)
_P = ctypes.c_void_p
_I = ctypes.c_int
_I32 = ctypes.c_int32

_lib.ot_fmm_version.restype = _I
_lib.ot_fmm_strerror.argtypes = [_I]
_lib.ot_fmm_strerror.restype = ctypes.c_char_p
_lib.ot_fmm_last_error.restype = ctypes.c_char_p
_lib.ot_fmm_monopole.argtypes = [_P, _P, _P, _P]
_lib.ot_fmm_monopole.restype = _I
_lib.ot_fmm_multipole.argtypes = [_P, _P, _P, _P]
_lib.ot_fmm_multipole.restype = _I
_lib.ot_fmm_plan_create.argtypes = [_I32, _I32, _P, _P, _P, _P, ctypes.POINTER(_P)]
_lib.ot_fmm_plan_create.restype = _I
_lib.ot_fmm_plan_destroy.argtypes = [_P]
_lib.ot_fmm_plan_destroy.restype = _I
_lib.ot_fmm_plan_pairs.argtypes = [_P, ctypes.POINTER(ctypes.c_int64)]
_lib.ot_fmm_plan_pairs.restype = _I
_lib.ot_fmm_multipole_batched_full.argtypes = [_P, _P, _P, _P, _I, _P]
_lib.ot_fmm_multipole_batched_full.restype = _I
_lib.ot_fmm_multipole_backward_full.argtypes = [_P, _P, _P, _P, _P, _P, _I, _P]
_lib.ot_fmm_multipole_backward_full.restype = _I
_lib.ot_fmm_plan_set_coarse.argtypes = [_P, _I32, _P, _P, ctypes.POINTER(ctypes.c_int64)]
_lib.ot_fmm_plan_set_coarse.restype = _I
for _f in (_lib.ot_fmm_coarse_fine, _lib.ot_fmm_coarse_fine_full):
    _f.argtypes = [_P, _P, _P, _P, _P, _P]
    _f.restype = _I
_lib.ot_fmm_multipole_batched.argtypes = [_P, _P, _P, _P, _I, _P]
_lib.ot_fmm_multipole_batched.restype = _I
_lib.ot_fmm_multipole_backward.argtypes = [_P, _P, _P, _P, _P, _P, _I, _P]
_lib.ot_fmm_multipole_backward.restype = _I
_lib.ot_fmm_autotune.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P,
                                 ctypes.POINTER(_I), ctypes.POINTER(_I)]
_lib.ot_fmm_autotune.restype = _I
_lib.ot_fmm_step_graph_create.argtypes = [_P, _P, _P, _P, _P, _P, _P, _I, _I]
_lib.ot_fmm_step_graph_create.restype = _I
_lib.ot_fmm_step_graph_launch.argtypes = [_P, _P]
_lib.ot_fmm_step_graph_launch.restype = _I
_lib.ot_fmm_plan_timing.argtypes = [_P, _I]
_lib.ot_fmm_plan_timing.restype = _I
_lib.ot_fmm_plan_kernel_times.argtypes = [_P, _P, _P]
_lib.ot_fmm_plan_kernel_times.restype = _I
_lib.ot_fmm_multipole_batched_save.argtypes = [_P, _P, _P, _P, _P, _I, _P]
_lib.ot_fmm_multipole_batched_save.restype = _I
_lib.ot_fmm_multipole_batched_full_save.argtypes = [_P, _P, _P, _P, _P, _I, _P]
_lib.ot_fmm_multipole_batched_full_save.restype = _I
_lib.ot_fmm_multipole_backward_full_saved.argtypes = [_P, _P, _P, _P, _P, _P, _P, _I, _P]
_lib.ot_fmm_multipole_backward_full_saved.restype = _I
_lib.ot_fmm_multipole_batched_amc.argtypes = [_P, _P, _P, _P, _P, _I, _P]
_lib.ot_fmm_multipole_batched_amc.restype = _I
_lib.ot_fmm_multipole_backward_saved.argtypes = [_P, _P, _P, _P, _P, _P, _P, _I, _P]
_lib.ot_fmm_multipole_backward_saved.restype = _I
_lib.ot_fmm_autotune_saved.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _P,
                                       ctypes.POINTER(_I), ctypes.POINTER(_I)]
_lib.ot_fmm_autotune_saved.restype = _I
_lib.ot_fmm_step_graph_create_saved.argtypes = [_P, _P, _P, _P, _P, _P, _P, _P, _I, _I]
_lib.ot_fmm_step_graph_create_saved.restype = _I
_lib.ot_fmm_multipole_batched_noalloc.argtypes = [_I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P]
_lib.ot_fmm_multipole_batched_noalloc.restype = _I
_lib.ot_fmm_noalloc_status.argtypes = [ctypes.POINTER(_I32), ctypes.POINTER(_I32)]
_lib.ot_fmm_noalloc_status.restype = _I

_lib.ot_fmm_tree_create.argtypes = [_I32, _I32, _P, ctypes.POINTER(_P)]
_lib.ot_fmm_tree_create.restype = _I
_lib.ot_fmm_tree_destroy.argtypes = [_P]
_lib.ot_fmm_tree_destroy.restype = _I
_lib.ot_fmm_m2m.argtypes = [_P, _P, _P, _P, _P, _P]
_lib.ot_fmm_m2m.restype = _I
_lib.ot_fmm_l2l.argtypes = [_P, _P, _P, _P, _P, _P]
_lib.ot_fmm_l2l.restype = _I
_lib.ot_fmm_evaluate.argtypes = [ctypes.c_int64, _P, _P, _P, _P, _P]
_lib.ot_fmm_evaluate.restype = _I

_lib.ot_fmm_count_pairs.argtypes = [_I32, _I32, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_int64), _P, _P]
_lib.ot_fmm_count_pairs.restype = _I
_lib.ot_fmm_work_orders.argtypes = [_I32, _I32, _P, _P, _P, _P, _I32, _P, _P, _P]
_lib.ot_fmm_work_orders.restype = _I
_lib.ot_fmm_stencil_info.argtypes = [_P, _P, _P]
_lib.ot_fmm_stencil_info.restype = _I
_CB = ctypes.CFUNCTYPE(None, ctypes.c_void_p)
_lib.ot_fmm_executor_create.argtypes = [_I, _I, ctypes.POINTER(_P)]
_lib.ot_fmm_executor_destroy.argtypes = [_P]
_lib.ot_fmm_executor_stream.argtypes = [_P, _I, ctypes.POINTER(_P)]
_lib.ot_fmm_executor_get_future.argtypes = [_P, _P, ctypes.POINTER(_P)]
_lib.ot_fmm_executor_multipole_async.argtypes = [_P, _P, _P, _P, ctypes.POINTER(_P)]
_lib.ot_fmm_executor_post.argtypes = [_P, _CB, _P]
_lib.ot_fmm_executor_poll.argtypes = [_P, ctypes.POINTER(_I)]
_lib.ot_fmm_executor_outstanding.argtypes = [_P, ctypes.POINTER(ctypes.c_int64)]
_lib.ot_fmm_future_create.argtypes = [_P, ctypes.POINTER(_P)]
_lib.ot_fmm_future_set_ready.argtypes = [_P]
_lib.ot_fmm_future_then.argtypes = [_P, _CB, _P]
_lib.ot_fmm_future_is_ready.argtypes = [_P, ctypes.POINTER(_I)]
_lib.ot_fmm_future_wait.argtypes = [_P, ctypes.c_double]
_lib.ot_fmm_future_release.argtypes = [_P]
for _n in ("executor_create", "executor_destroy", "executor_stream", "executor_get_future",
           "executor_multipole_async", "executor_post", "executor_poll", "executor_outstanding",
           "future_create", "future_set_ready", "future_then", "future_is_ready", "future_wait",
           "future_release"):
    getattr(_lib, "ot_fmm_" + _n).restype = _I

KERNELS = ("forward", "adjoint_source", "adjoint_target", "forward_save", "adjoint_saved", "forward_amc")
NSAVED = 24  # saved target-side sums per target cell (ot_fmm_multipole_batched_save)


class OtFmmError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        detail = _lib.ot_fmm_last_error().decode(errors="replace")
        msg = _lib.ot_fmm_strerror(code).decode()
        super().__init__("%s: %s (%d)%s" % (where, msg, code, ": " + detail if detail else ""))


def _check(rc, where):
    if rc != OT_FMM_OK:
        raise OtFmmError(rc, where)


def version() -> int:
    return _lib.ot_fmm_version()


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dptr(t, shape, name):
    """Device pointer of a contiguous float64 GPU tensor of the given shape."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float64 GPU tensor" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return ctypes.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# single sub-grid forms
# ---------------------------------------------------------------------------
def ot_fmm_monopole(mass, com, L, stream=None):
    """mass (13824,), com (3, 13824) -> L (20, 512), all float64 on the GPU."""
    _check(_lib.ot_fmm_monopole(_dptr(mass, (13824,), "mass"), _dptr(com, (3, 13824), "com"),
                                _dptr(L, (20, 512), "L"), _stream(stream)), "ot_fmm_monopole")
    return L


def ot_fmm_multipole(M, com, L, stream=None):
    """M (20, 13824), com (3, 13824) -> L (20, 512), all float64 on the GPU."""
    _check(_lib.ot_fmm_multipole(_dptr(M, (20, 13824), "M"), _dptr(com, (3, 13824), "com"),
                                 _dptr(L, (20, 512), "L"), _stream(stream)), "ot_fmm_multipole")
    return L


# ---------------------------------------------------------------------------
# batched forms
# ---------------------------------------------------------------------------
def _descriptor_arrays(batch):
    """Contiguous, typed and shape-checked (tgt, nbr, shift, period) of a descriptor."""
    T = int(batch["T"])
    tgt = np.ascontiguousarray(batch["tgt"], dtype=np.int32)
    nbr = np.ascontiguousarray(batch["nbr"], dtype=np.int32)
    if tgt.shape != (T,) or nbr.shape != (T, 27):
        raise ValueError("tgt must be (T,) and nbr (T, 27)")
    shift = batch.get("shift")
    period = batch.get("period")
    if shift is not None:
        shift = np.ascontiguousarray(shift, dtype=np.int8)
        if shift.shape != (T, 27, 3):
            raise ValueError("shift must be (T, 27, 3)")
    if period is not None:
        period = np.ascontiguousarray(period, dtype=np.float64)
        if period.shape != (3,):
            raise ValueError("period must be (3,)")
    return tgt, nbr, shift, period


class Plan:
    """Validated batched descriptor with device tables (ot_fmm_plan)."""

    def __init__(self, S, T, tgt, nbr, shift=None, period=None):
        self.S = int(S)
        self.T = int(T)
        tgt, nbr, shift, period = _descriptor_arrays(
            {"S": S, "T": T, "tgt": tgt, "nbr": nbr, "shift": shift, "period": period})
        h = ctypes.c_void_p()
        self._h = None
        _check(_lib.ot_fmm_plan_create(
            self.S, self.T, tgt.ctypes.data_as(_P), nbr.ctypes.data_as(_P),
            None if shift is None else shift.ctypes.data_as(_P),
            None if period is None else period.ctypes.data_as(_P), ctypes.byref(h)),
            "ot_fmm_plan_create")
        self._h = h

    @classmethod
    def from_batch(cls, batch):
        return cls(batch["S"], batch["T"], batch["tgt"], batch["nbr"], batch.get("shift"),
                   batch.get("period"))

    def close(self):
        if self._h is not None:
            _lib.ot_fmm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan is closed")
        return self._h

    def pairs(self) -> int:
        v = ctypes.c_int64()
        _check(_lib.ot_fmm_plan_pairs(self.handle, ctypes.byref(v)), "ot_fmm_plan_pairs")
        return int(v.value)

    def set_coarse(self, Sp, coarse, octant) -> int:
        """Coarse substitutes for missing neighbours: coarse (T, 27) node of a
        coarse store of Sp nodes (-1: none) and octant (T, 27) of that node
        covering the missing block. Returns the included (target cell, coarse
        cell) pairs."""
        coarse = np.ascontiguousarray(coarse, dtype=np.int32)
        octant = np.ascontiguousarray(octant, dtype=np.int8)
        if coarse.shape != (self.T, 27) or octant.shape != (self.T, 27):
            raise ValueError("coarse and octant must be (T, 27)")
        v = ctypes.c_int64()
        _check(_lib.ot_fmm_plan_set_coarse(self.handle, int(Sp), coarse.ctypes.data_as(_P),
                                           octant.ctypes.data_as(_P), ctypes.byref(v)),
               "ot_fmm_plan_set_coarse")
        self.Sp_coarse = int(Sp)
        return int(v.value)

    def coarse_fine(self, com, Mp, comp, L, stream=None, full=False):
        """Adds the coarse substitutes' contributions into L (20, T*512);
        full=True: under the full truncation (ot_fmm_coarse_fine_full)."""
        Sp = getattr(self, "Sp_coarse", 0)
        if Sp <= 0:
            raise ValueError("no coarse substitutes set")
        _, sx, sl = self._shapes()
        fn, name = ((_lib.ot_fmm_coarse_fine_full, "ot_fmm_coarse_fine_full") if full
                    else (_lib.ot_fmm_coarse_fine, "ot_fmm_coarse_fine"))
        _check(fn(self.handle, _dptr(com, sx, "com"), _dptr(Mp, (20, Sp * 512), "Mp"),
                  _dptr(comp, (3, Sp * 512), "comp"), _dptr(L, sl, "L"), _stream(stream)), name)
        return L

    def _shapes(self):
        NS, NT = self.S * 512, self.T * 512
        return (20, NS), (3, NS), (20, NT)

    def multipole_batched(self, M, com, L, sched=SCHED_AUTO, stream=None):
        sm, sx, sl = self._shapes()
        _check(_lib.ot_fmm_multipole_batched(self.handle, _dptr(M, sm, "M"), _dptr(com, sx, "com"),
                                             _dptr(L, sl, "L"), int(sched), _stream(stream)),
               "ot_fmm_multipole_batched")
        return L

    def multipole_batched_full(self, M, com, L, sched=SCHED_AUTO, stream=None):
        """Forward with the full truncation (every output keeps every moment
        up to order 3); L (20, T*512) is overwritten."""
        sm, sx, sl = self._shapes()
        _check(_lib.ot_fmm_multipole_batched_full(self.handle, _dptr(M, sm, "M"), _dptr(com, sx, "com"),
                                                  _dptr(L, sl, "L"), int(sched), _stream(stream)),
               "ot_fmm_multipole_batched_full")
        return L

    def multipole_backward(self, M, com, gL, gM, gcom, sched=SCHED_AUTO, stream=None):
        sm, sx, sl = self._shapes()
        _check(_lib.ot_fmm_multipole_backward(
            self.handle, _dptr(M, sm, "M"), _dptr(com, sx, "com"), _dptr(gL, sl, "gL"),
            _dptr(gM, sm, "gM"), _dptr(gcom, sx, "gcom"), int(sched), _stream(stream)),
            "ot_fmm_multipole_backward")
        return gM, gcom

    def multipole_backward_full(self, M, com, gL, gM, gcom, sched=SCHED_AUTO, stream=None):
        """Adjoint of multipole_batched_full (gM, gcom overwritten)."""
        sm, sx, sl = self._shapes()
        _check(_lib.ot_fmm_multipole_backward_full(
            self.handle, _dptr(M, sm, "M"), _dptr(com, sx, "com"), _dptr(gL, sl, "gL"),
            _dptr(gM, sm, "gM"), _dptr(gcom, sx, "gcom"), int(sched), _stream(stream)),
            "ot_fmm_multipole_backward_full")
        return gM, gcom

    def multipole_batched_save(self, M, com, L, Cs, sched=SCHED_AUTO, stream=None, full=False):
        """Forward that also writes the target-side derivative sums Cs
        (24, T*512) the one-pass adjoint needs (full=True: of the full truncation)."""
        sm, sx, sl = self._shapes()
        fn, name = ((_lib.ot_fmm_multipole_batched_full_save, "ot_fmm_multipole_batched_full_save") if full
                    else (_lib.ot_fmm_multipole_batched_save, "ot_fmm_multipole_batched_save"))
        _check(fn(self.handle, _dptr(M, sm, "M"), _dptr(com, sx, "com"), _dptr(L, sl, "L"),
                  _dptr(Cs, (NSAVED, sl[1]), "Cs"), int(sched), _stream(stream)), name)
        return L, Cs

    def multipole_batched_amc(self, M, com, L, dF, sched=SCHED_AUTO, stream=None):
        """Forward (L) and the angular-momentum correction dF (3, T*512) of
        each target cell's force."""
        sm, sx, sl = self._shapes()
        _check(_lib.ot_fmm_multipole_batched_amc(
            self.handle, _dptr(M, sm, "M"), _dptr(com, sx, "com"), _dptr(L, sl, "L"),
            _dptr(dF, (3, sl[1]), "dF"), int(sched), _stream(stream)), "ot_fmm_multipole_batched_amc")
        return L, dF

    def multipole_backward_saved(self, M, com, gL, Cs, gM, gcom, sched=SCHED_AUTO, stream=None, full=False):
        """One-pass adjoint from the sums of multipole_batched_save (gM, gcom
        overwritten; full=True: of the full truncation)."""
        sm, sx, sl = self._shapes()
        fn, name = ((_lib.ot_fmm_multipole_backward_full_saved, "ot_fmm_multipole_backward_full_saved") if full
                    else (_lib.ot_fmm_multipole_backward_saved, "ot_fmm_multipole_backward_saved"))
        _check(fn(self.handle, _dptr(M, sm, "M"), _dptr(com, sx, "com"), _dptr(gL, sl, "gL"),
                  _dptr(Cs, (NSAVED, sl[1]), "Cs"), _dptr(gM, sm, "gM"), _dptr(gcom, sx, "gcom"), int(sched),
                  _stream(stream)), name)
        return gM, gcom

    def autotune_saved(self, M, com, L, Cs, gL, gM, gcom, stream=None):
        sm, sx, sl = self._shapes()
        f = ctypes.c_int()
        b = ctypes.c_int()
        _check(_lib.ot_fmm_autotune_saved(
            self.handle, _dptr(M, sm, "M"), _dptr(com, sx, "com"), _dptr(L, sl, "L"),
            _dptr(Cs, (NSAVED, sl[1]), "Cs"), _dptr(gL, sl, "gL"), _dptr(gM, sm, "gM"),
            _dptr(gcom, sx, "gcom"), _stream(stream), ctypes.byref(f), ctypes.byref(b)),
            "ot_fmm_autotune_saved")
        return f.value, b.value

    def step_graph_create_saved(self, M, com, L, Cs, gL, gM, gcom, fwd_sched=SCHED_AUTO,
                                bwd_sched=SCHED_AUTO):
        sm, sx, sl = self._shapes()
        _check(_lib.ot_fmm_step_graph_create_saved(
            self.handle, _dptr(M, sm, "M"), _dptr(com, sx, "com"), _dptr(L, sl, "L"),
            _dptr(Cs, (NSAVED, sl[1]), "Cs"), _dptr(gL, sl, "gL"), _dptr(gM, sm, "gM"),
            _dptr(gcom, sx, "gcom"), int(fwd_sched), int(bwd_sched)), "ot_fmm_step_graph_create_saved")

    def autotune(self, M, com, L, gL=None, gM=None, gcom=None, stream=None):
        sm, sx, sl = self._shapes()
        f = ctypes.c_int()
        b = ctypes.c_int()
        _check(_lib.ot_fmm_autotune(
            self.handle, _dptr(M, sm, "M"), _dptr(com, sx, "com"), _dptr(L, sl, "L"),
            _dptr(gL, sl, "gL"), _dptr(gM, sm, "gM"), _dptr(gcom, sx, "gcom"),
            _stream(stream), ctypes.byref(f), ctypes.byref(b)), "ot_fmm_autotune")
        return f.value, b.value

    def step_graph_create(self, M, com, L, gL=None, gM=None, gcom=None, fwd_sched=SCHED_AUTO,
                          bwd_sched=SCHED_AUTO):
        sm, sx, sl = self._shapes()
        _check(_lib.ot_fmm_step_graph_create(
            self.handle, _dptr(M, sm, "M"), _dptr(com, sx, "com"), _dptr(L, sl, "L"),
            _dptr(gL, sl, "gL"), _dptr(gM, sm, "gM"), _dptr(gcom, sx, "gcom"),
            int(fwd_sched), int(bwd_sched)), "ot_fmm_step_graph_create")

    def set_timing(self, enable=True):
        _check(_lib.ot_fmm_plan_timing(self.handle, 1 if enable else 0), "ot_fmm_plan_timing")

    def kernel_times(self):
        """{kernel: (total ms, launches)} since the last call (waits for the events)."""
        ms = np.zeros(len(KERNELS), np.float64)
        n = np.zeros(len(KERNELS), np.int64)
        _check(_lib.ot_fmm_plan_kernel_times(self.handle, ms.ctypes.data_as(_P),
                                             n.ctypes.data_as(_P)), "ot_fmm_plan_kernel_times")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNELS)}

    def step_graph_launch(self, stream=None):
        _check(_lib.ot_fmm_step_graph_launch(self.handle, _stream(stream)),
               "ot_fmm_step_graph_launch")


def ot_fmm_multipole_batched(plan, M, com, L, sched=SCHED_AUTO, stream=None):
    return plan.multipole_batched(M, com, L, sched, stream)


def ot_fmm_multipole_backward(plan, M, com, gL, gM, gcom, sched=SCHED_AUTO, stream=None):
    return plan.multipole_backward(M, com, gL, gM, gcom, sched, stream)


def ot_fmm_multipole_batched_full(plan, M, com, L, sched=SCHED_AUTO, stream=None):
    return plan.multipole_batched_full(M, com, L, sched, stream)


def ot_fmm_multipole_backward_full(plan, M, com, gL, gM, gcom, sched=SCHED_AUTO, stream=None):
    return plan.multipole_backward_full(M, com, gL, gM, gcom, sched, stream)


def ot_fmm_multipole_batched_save(plan, M, com, L, Cs, sched=SCHED_AUTO, stream=None):
    return plan.multipole_batched_save(M, com, L, Cs, sched, stream)


def ot_fmm_multipole_backward_saved(plan, M, com, gL, Cs, gM, gcom, sched=SCHED_AUTO, stream=None):
    return plan.multipole_backward_saved(M, com, gL, Cs, gM, gcom, sched, stream)


def ot_fmm_multipole_batched_full_save(plan, M, com, L, Cs, sched=SCHED_AUTO, stream=None):
    return plan.multipole_batched_save(M, com, L, Cs, sched, stream, full=True)


def ot_fmm_multipole_backward_full_saved(plan, M, com, gL, Cs, gM, gcom, sched=SCHED_AUTO, stream=None):
    return plan.multipole_backward_saved(M, com, gL, Cs, gM, gcom, sched, stream, full=True)


def ot_fmm_multipole_batched_amc(plan, M, com, L, dF, sched=SCHED_AUTO, stream=None):
    return plan.multipole_batched_amc(M, com, L, dF, sched, stream)


def ot_fmm_plan_set_coarse(plan, Sp, coarse, octant):
    return plan.set_coarse(Sp, coarse, octant)


def ot_fmm_coarse_fine(plan, com, Mp, comp, L, stream=None):
    return plan.coarse_fine(com, Mp, comp, L, stream)


def ot_fmm_coarse_fine_full(plan, com, Mp, comp, L, stream=None):
    return plan.coarse_fine(com, Mp, comp, L, stream, full=True)


NOALLOC_MAX_T = 32768


def _iptr(t, shape, dtype, name):
    """Device pointer of a contiguous integer GPU tensor of the given shape and dtype."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s GPU tensor" % (name, dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return ctypes.c_void_p(t.data_ptr())


def ot_fmm_multipole_batched_noalloc(S, T, tgt, nbr, shift, period, M, com, L, stream=None):
    """Allocation-free batched forward (no plan): tgt (T,) and nbr (T, 27)
    int32 GPU tensors, shift (T, 27, 3) int8 GPU tensor or None, period three
    floats or None; M (20, S*512), com (3, S*512) -> L (20, T*512)."""
    S, T = int(S), int(T)
    per = None
    if period is not None:
        per = np.ascontiguousarray(period, dtype=np.float64)
        if per.shape != (3,):
            raise ValueError("period must be (3,)")
    _check(_lib.ot_fmm_multipole_batched_noalloc(
        S, T, _iptr(tgt, (T,), torch.int32, "tgt"), _iptr(nbr, (T, 27), torch.int32, "nbr"),
        _iptr(shift, (T, 27, 3), torch.int8, "shift"),
        None if per is None else per.ctypes.data_as(_P),
        _dptr(M, (20, S * 512), "M"), _dptr(com, (3, S * 512), "com"), _dptr(L, (20, T * 512), "L"),
        _stream(stream)), "ot_fmm_multipole_batched_noalloc")
    return L


def ot_fmm_noalloc_status():
    """(invalid descriptor entries, first invalid entry) of the last
    allocation-free call on the current device (waits for the device)."""
    n = _I32()
    first = _I32()
    _check(_lib.ot_fmm_noalloc_status(ctypes.byref(n), ctypes.byref(first)), "ot_fmm_noalloc_status")
    return int(n.value), int(first.value)


class MultipoleBatched(torch.autograd.Function):
    """L = multipole_batched(M, com) with the hand-written adjoint as backward
    (full=True: the full truncation and its adjoint).

    With a gradient to compute, the forward also keeps the target-side sums
    (24 doubles per target cell) and the backward is the one-pass adjoint
    (save=False: plain forward, two-pass adjoint), for either truncation.

    Usage: L = MultipoleBatched.apply(M, com, plan[, full[, save]])."""

    @staticmethod
    def forward(ctx, M, com, plan, full=False, save=True):
        M = M.contiguous()
        com = com.contiguous()
        L = torch.empty((20, plan.T * 512), dtype=torch.float64, device=M.device)
        use_save = bool(save) and any(ctx.needs_input_grad[:2])
        if use_save:
            Cs = torch.empty((NSAVED, plan.T * 512), dtype=torch.float64, device=M.device)
            plan.multipole_batched_save(M, com, L, Cs, full=full)
            ctx.save_for_backward(M, com, Cs)
        elif full:
            plan.multipole_batched_full(M, com, L)
            ctx.save_for_backward(M, com)
        else:
            plan.multipole_batched(M, com, L)
            ctx.save_for_backward(M, com)
        ctx.plan = plan
        ctx.full = bool(full)
        ctx.use_save = use_save
        return L

    @staticmethod
    def backward(ctx, gL):
        gL = gL.contiguous()
        if ctx.use_save:
            M, com, Cs = ctx.saved_tensors
            gM = torch.empty_like(M)
            gcom = torch.empty_like(com)
            ctx.plan.multipole_backward_saved(M, com, gL, Cs, gM, gcom, full=ctx.full)
        else:
            M, com = ctx.saved_tensors
            gM = torch.empty_like(M)
            gcom = torch.empty_like(com)
            if ctx.full:
                ctx.plan.multipole_backward_full(M, com, gL, gM, gcom)
            else:
                ctx.plan.multipole_backward(M, com, gL, gM, gcom)
        return gM, gcom, None, None, None


def multipole(M, com, plan, full=False, save=True):
    """Differentiable batched multipole interaction (see MultipoleBatched)."""
    return MultipoleBatched.apply(M, com, plan, full, save)


# ---------------------------------------------------------------------------
# tree passes around the interaction
# ---------------------------------------------------------------------------
class Tree:
    """Parent -> 8 children table of one octree level (ot_fmm_tree)."""

    def __init__(self, children, Sc):
        ch = np.ascontiguousarray(children, dtype=np.int32)
        if ch.ndim != 2 or ch.shape[1] != 8:
            raise ValueError("children must be (Sp, 8)")
        self.Sp = int(ch.shape[0])
        self.Sc = int(Sc)
        h = ctypes.c_void_p()
        self._h = None
        _check(_lib.ot_fmm_tree_create(self.Sp, self.Sc, ch.ctypes.data_as(_P), ctypes.byref(h)),
               "ot_fmm_tree_create")
        self._h = h

    def close(self):
        if self._h is not None:
            _lib.ot_fmm_tree_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("tree is closed")
        return self._h

    def m2m(self, Mc, comc, Mp, comp, stream=None):
        nc, npar = self.Sc * 512, self.Sp * 512
        _check(_lib.ot_fmm_m2m(self.handle, _dptr(Mc, (20, nc), "Mc"), _dptr(comc, (3, nc), "comc"),
                               _dptr(Mp, (20, npar), "Mp"), _dptr(comp, (3, npar), "comp"),
                               _stream(stream)), "ot_fmm_m2m")
        return Mp, comp

    def l2l(self, Lp, comp, comc, Lc, stream=None):
        nc, npar = self.Sc * 512, self.Sp * 512
        _check(_lib.ot_fmm_l2l(self.handle, _dptr(Lp, (20, npar), "Lp"), _dptr(comp, (3, npar), "comp"),
                               _dptr(comc, (3, nc), "comc"), _dptr(Lc, (20, nc), "Lc"),
                               _stream(stream)), "ot_fmm_l2l")
        return Lc


def ot_fmm_m2m(tree, Mc, comc, Mp, comp, stream=None):
    return tree.m2m(Mc, comc, Mp, comp, stream)


def ot_fmm_l2l(tree, Lp, comp, comc, Lc, stream=None):
    return tree.l2l(Lp, comp, comc, Lc, stream)


def ot_fmm_evaluate(M, L, F, W, stream=None):
    """M, L (20, n) -> F (3, n), W (n,) per-cell force and energy share."""
    n = int(M.shape[1])
    _check(_lib.ot_fmm_evaluate(n, _dptr(M, (20, n), "M"), _dptr(L, (20, n), "L"),
                                _dptr(F, (3, n), "F"), _dptr(W, (n,), "W"), _stream(stream)),
           "ot_fmm_evaluate")
    return F, W


# ---------------------------------------------------------------------------
# futures completed by event polling
# ---------------------------------------------------------------------------
_callables = {}
_callables_lock = threading.Lock()
_next_key = itertools.count(1)


def _dispatch(user):
    with _callables_lock:
        fn = _callables.pop(user)
    fn()


_DISPATCH = _CB(_dispatch)  # one C entry for every Python callable (kept alive)


def _register(fn):
    key = next(_next_key)
    with _callables_lock:
        _callables[key] = fn
    return ctypes.c_void_p(key)


class Future:
    """A reference to an ot_fmm_future (released on close / garbage collection)."""

    def __init__(self, handle, executor):
        self._h = handle
        self.executor = executor  # keeps the executor alive while the future is

    def then(self, fn):
        _check(_lib.ot_fmm_future_then(self._h, _DISPATCH, _register(fn)), "ot_fmm_future_then")

    def is_ready(self) -> bool:
        r = ctypes.c_int()
        _check(_lib.ot_fmm_future_is_ready(self._h, ctypes.byref(r)), "ot_fmm_future_is_ready")
        return bool(r.value)

    def wait(self, timeout=-1.0):
        _check(_lib.ot_fmm_future_wait(self._h, float(timeout)), "ot_fmm_future_wait")

    def set_ready(self):
        _check(_lib.ot_fmm_future_set_ready(self._h), "ot_fmm_future_set_ready")

    def close(self):
        if self._h is not None:
            _lib.ot_fmm_future_release(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Executor:
    """Stream pool + task queue whose futures are completed by event polling."""

    def __init__(self, nstreams=8, nworkers=0):
        h = ctypes.c_void_p()
        self._h = None
        _check(_lib.ot_fmm_executor_create(int(nstreams), int(nworkers), ctypes.byref(h)),
               "ot_fmm_executor_create")
        self._h = h

    def close(self):
        if self._h is not None:
            _check(_lib.ot_fmm_executor_destroy(self._h), "ot_fmm_executor_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stream(self, i):
        s = ctypes.c_void_p()
        _check(_lib.ot_fmm_executor_stream(self._h, int(i), ctypes.byref(s)), "ot_fmm_executor_stream")
        return s.value

    def get_future(self, stream=None):
        f = ctypes.c_void_p()
        _check(_lib.ot_fmm_executor_get_future(self._h, _stream(stream), ctypes.byref(f)),
               "ot_fmm_executor_get_future")
        return Future(f, self)

    def multipole_async(self, M, com, L):
        f = ctypes.c_void_p()
        _check(_lib.ot_fmm_executor_multipole_async(
            self._h, _dptr(M, (20, 13824), "M"), _dptr(com, (3, 13824), "com"),
            _dptr(L, (20, 512), "L"), ctypes.byref(f)), "ot_fmm_executor_multipole_async")
        return Future(f, self)

    def post(self, fn):
        _check(_lib.ot_fmm_executor_post(self._h, _DISPATCH, _register(fn)), "ot_fmm_executor_post")

    def poll(self) -> int:
        n = ctypes.c_int()
        _check(_lib.ot_fmm_executor_poll(self._h, ctypes.byref(n)), "ot_fmm_executor_poll")
        return n.value

    def outstanding(self) -> int:
        n = ctypes.c_int64()
        _check(_lib.ot_fmm_executor_outstanding(self._h, ctypes.byref(n)), "ot_fmm_executor_outstanding")
        return n.value

    def future(self):
        """A host-side future, made ready by Future.set_ready()."""
        f = ctypes.c_void_p()
        _check(_lib.ot_fmm_future_create(self._h, ctypes.byref(f)), "ot_fmm_future_create")
        return Future(f, self)


# ---------------------------------------------------------------------------
# host-only descriptor and stencil queries (no device needed)
# ---------------------------------------------------------------------------
def ot_fmm_count_pairs(batch):
    """(pairs, work per target, launch order) of a batched descriptor, validated
    as ot_fmm_plan_create validates it."""
    tgt, nbr, shift, period = _descriptor_arrays(batch)
    T = int(batch["T"])
    pairs = ctypes.c_int64()
    work = np.zeros(T, np.int64)
    order = np.zeros(T, np.int32)
    _check(_lib.ot_fmm_count_pairs(int(batch["S"]), T, tgt.ctypes.data_as(_P), nbr.ctypes.data_as(_P),
                                   None if shift is None else shift.ctypes.data_as(_P),
                                   None if period is None else period.ctypes.data_as(_P),
                                   ctypes.byref(pairs), work.ctypes.data_as(_P),
                                   order.ctypes.data_as(_P)), "ot_fmm_count_pairs")
    return pairs.value, work, order


def ot_fmm_stencil_info():
    """(pairs per neighbour slot [27], offsets per target [2], row-table entries [2])."""
    sp = np.zeros(27, np.int64)
    off = np.zeros(2, np.int32)
    rows = np.zeros(2, np.int32)
    _check(_lib.ot_fmm_stencil_info(sp.ctypes.data_as(_P), off.ctypes.data_as(_P), rows.ctypes.data_as(_P)),
           "ot_fmm_stencil_info")
    return sp, off, rows


def ot_fmm_work_orders(batch, nxcd=8):
    """(targets XCD-aware, store sub-grids longest-first, store sub-grids XCD-aware)."""
    tgt, nbr, shift, period = _descriptor_arrays(batch)
    S, T = int(batch["S"]), int(batch["T"])
    fl = np.zeros(T, np.int32)
    rl = np.zeros(S, np.int32)
    rloc = np.zeros(S, np.int32)
    _check(_lib.ot_fmm_work_orders(S, T, tgt.ctypes.data_as(_P), nbr.ctypes.data_as(_P),
                                   None if shift is None else shift.ctypes.data_as(_P),
                                   None if period is None else period.ctypes.data_as(_P), int(nxcd),
                                   fl.ctypes.data_as(_P), rl.ctypes.data_as(_P), rloc.ctypes.data_as(_P)),
           "ot_fmm_work_orders")
    return fl, rl, rloc
