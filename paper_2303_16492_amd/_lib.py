"""ctypes view of the C ABI declared in include/tr.h.

torch is imported before the shared library is opened so that the library's
HIP runtime dependency resolves to the copy torch has already mapped (one
runtime per process).  A missing library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (must precede the library: one HIP runtime)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtrsgd.so")

TR_MAX_ORDER = 8
TR_MAX_RANK = 16

TR_OK = 0
TR_E_ARG, TR_E_SHAPE, TR_E_DTYPE, TR_E_ALIGN, TR_E_WORKSPACE, TR_E_HIP, TR_E_UNSUPPORTED = -1, -2, -3, -4, -5, -6, -7
TR_NOALLOC_SCRATCH_BYTES = 16 << 20
TR_F64, TR_F32, TR_F16, TR_BF16 = 0, 1, 2, 3
TR_PREC_F64, TR_PREC_F32, TR_PREC_BF16, TR_PREC_F16 = 0, 1, 2, 3
TR_LAW_UNIFORM, TR_LAW_LEVERAGE, TR_LAW_EUCLID, TR_LAW_OPTIMAL = 0, 1, 2, 3
TR_STREAM_MODE, TR_STREAM_IDX, TR_STREAM_H, TR_STREAM_ENTRY = 0, 1, 2, 3
TR_DEV_NONFINITE, TR_DEV_NOT_SPD, TR_DEV_ZERO_DIST, TR_DEV_DAMPED = 1, 2, 4, 8


class tr_desc(C.Structure):
    _fields_ = [
        ("N", C.c_int32),
        ("I", C.c_int32 * TR_MAX_ORDER),
        ("R", C.c_int32 * TR_MAX_ORDER),
        ("x_stride", C.c_int64 * TR_MAX_ORDER),
        ("core_dtype", C.c_int32),
        ("x_dtype", C.c_int32),
    ]


class tr_step(C.Structure):
    _fields_ = [
        ("kind", C.c_int32),
        ("alpha", C.c_double),
        ("tau", C.c_double),
        ("eta", C.c_double),
        ("b", C.c_double),
        ("eps", C.c_double),
    ]


class tr_problem(C.Structure):
    _fields_ = [
        ("desc", tr_desc),
        ("cores", C.c_void_p * TR_MAX_ORDER),
        ("accum", C.c_void_p * TR_MAX_ORDER),
        ("X", C.c_void_p),
        ("Xrep", C.c_void_p * TR_MAX_ORDER),
        ("cdf", C.c_void_p * TR_MAX_ORDER),
        ("cdf_J", C.c_void_p),
    ]


class tr_config(C.Structure):
    _fields_ = [
        ("m", C.c_int32),
        ("m_H", C.c_int32),
        ("law", C.c_int32),
        ("scaled", C.c_int32),
        ("prec", C.c_int32),
        ("damping", C.c_double),
        ("rule", tr_step),
        ("seed", C.c_uint64),
        ("damping_schedule", C.c_int32),
        ("damping_tau", C.c_double),
    ]


TR_METHOD_GD, TR_METHOD_SCALED_GD, TR_METHOD_ALS, TR_METHOD_ALS_SAMPLED = 0, 1, 2, 3


class tr_sweep_config(C.Structure):
    _fields_ = [
        ("method", C.c_int32),
        ("m", C.c_int32),
        ("law", C.c_int32),
        ("prec", C.c_int32),
        ("alpha", C.c_double),
        ("damping", C.c_double),
        ("seed", C.c_uint64),
    ]


class tr_completion_config(C.Structure):
    _fields_ = [
        ("B", C.c_int32),
        ("block", C.c_int32),
        ("lam", C.c_double),
        ("rule", tr_step),
        ("seed", C.c_uint64),
    ]


VP = C.c_void_p
PVP = C.POINTER(C.c_void_p)


class tr_batch_item(C.Structure):
    _fields_ = [
        ("desc", tr_desc),
        ("cores", C.c_void_p * 8),
        ("accum", C.c_void_p * 8),
        ("Xrep", C.c_void_p * 8),
        ("t_dev", C.c_void_p),
        ("loss", C.c_void_p),
        ("dev_status", C.c_void_p),
        ("m", C.c_int32),
        ("reserved", C.c_int32),
        ("rule", tr_step),
        ("seed", C.c_uint64),
    ]


class tr_run_opts(C.Structure):
    _fields_ = [
        ("aux", C.c_void_p),
        ("ev_fork", C.c_void_p),
        ("ev_gram", C.c_void_p),
        ("ev_join", C.c_void_p),
        ("ev_begin", PVP),
        ("ev_end", PVP),
        ("ev_inv_begin", PVP),
        ("ev_inv_end", PVP),
    ]

I32, U64, F64, SZ = C.c_int32, C.c_uint64, C.c_double, C.c_size_t
PDESC = C.POINTER(tr_desc)

_SIGS = {
    "tr_abi_version": (I32, []),
    "tr_status_str": (C.c_char_p, [I32]),
    "tr_mode": (I32, [U64, U64, I32]),
    "tr_dist": (I32, [PDESC, I32, I32, VP, VP, VP, VP, SZ, VP]),
    "tr_dist_workspace_size": (SZ, [PDESC, I32, I32]),
    "tr_dist_optimal": (I32, [PDESC, I32, PVP, VP, VP, VP, VP, SZ, VP]),
    "tr_dist_optimal_workspace_size": (SZ, [PDESC, I32]),
    "tr_sample": (I32, [PDESC, U64, U64, I32, I32, PVP, VP, I32, VP, VP, VP]),
    "tr_subchain": (I32, [PDESC, I32, PVP, VP, I32, VP, VP]),
    "tr_grad": (I32, [PDESC, I32, VP, VP, VP, VP, VP, I32, I32, VP, VP, VP, VP, SZ, VP]),
    "tr_grad_workspace_size": (SZ, [PDESC, I32, I32]),
    "tr_gram": (I32, [PDESC, I32, VP, VP, I32, VP, VP, SZ, VP]),
    "tr_gram_workspace_size": (SZ, [PDESC, I32]),
    "tr_update": (I32, [PDESC, I32, VP, VP, VP, F64, C.POINTER(tr_step), U64, VP, VP, VP, SZ, VP]),
    "tr_update_workspace_size": (SZ, [PDESC, I32, I32]),
    "tr_relerr": (I32, [PDESC, PVP, VP, F64, VP, VP, SZ, VP]),
    "tr_relerr_workspace_size": (SZ, [PDESC]),
    "tr_reconstruct": (I32, [PDESC, PVP, VP, VP]),
    "tr_x_replicate": (I32, [PDESC, VP, I32, VP, VP]),
    "tr_run": (I32, [C.POINTER(tr_problem), C.POINTER(tr_config), VP, I32, VP, VP, VP, SZ, VP]),
    "tr_run_events": (I32, [C.POINTER(tr_problem), C.POINTER(tr_config), VP, I32, VP, VP, VP, SZ, PVP, PVP,
                            VP]),
    "tr_run_ex": (I32, [C.POINTER(tr_problem), C.POINTER(tr_config), VP, I32, VP, VP, VP, SZ, VP,
                        C.POINTER(tr_run_opts)]),
    "tr_run_noalloc": (I32, [C.POINTER(tr_problem), C.POINTER(tr_config), VP, I32, VP, VP, VP,
                             C.POINTER(tr_run_opts)]),
    "tr_run_workspace_size": (SZ, [C.POINTER(tr_problem), C.POINTER(tr_config)]),
    "tr_sweep_workspace_size": (SZ, [C.POINTER(tr_problem), C.POINTER(tr_sweep_config)]),
    "tr_completion_workspace_size": (SZ, [PDESC, C.POINTER(tr_completion_config)]),
    "tr_completion_run": (I32, [PDESC, PVP, PVP, VP, VP, C.c_int64, C.POINTER(tr_completion_config), VP, I32, VP,
                                VP, VP, SZ, VP]),
    "tr_sweep_run": (I32, [C.POINTER(tr_problem), C.POINTER(tr_sweep_config), VP, I32, VP, VP, SZ, VP]),
    "tr_batch_table_size": (SZ, [I32]),
    "tr_batch_upload": (I32, [C.POINTER(tr_batch_item), I32, VP, SZ, VP]),
    "tr_batch_run": (I32, [VP, I32, I32, I32, I32, VP]),
    "tr_batch_split_workspace_size": (SZ, [I32, I32]),
    "tr_batch_run_split": (I32, [VP, I32, I32, I32, I32, I32, VP, SZ, VP]),
    "tr_entry_fwd": (I32, [PDESC, PVP, VP, VP, I32, VP, VP, VP, SZ, VP]),
    "tr_entry_bwd": (I32, [PDESC, PVP, VP, VP, I32, F64, VP, PVP, VP, SZ, VP]),
    "tr_entry_workspace_size": (SZ, [PDESC, I32]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2303_16492_amd.build`"
            )
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


class TRError(RuntimeError):
    def __init__(self, fn: str, status: int):
        msg = lib().tr_status_str(status).decode()
        super().__init__(f"{fn} returned {status}: {msg}")
        self.status = status


def check(fn: str, status: int) -> None:
    if status != TR_OK:
        raise TRError(fn, status)


_hip = None


def hip():
    """The HIP runtime this process already uses (torch's), for events."""
    global _hip
    if _hip is None:
        import torch
        h = C.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
        h.hipEventCreateWithFlags.argtypes = [C.POINTER(C.c_void_p), C.c_uint]
        h.hipEventCreateWithFlags.restype = C.c_int
        h.hipEventDestroy.argtypes = [C.c_void_p]
        h.hipEventDestroy.restype = C.c_int
        h.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
        h.hipEventRecord.restype = C.c_int
        h.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        h.hipEventElapsedTime.restype = C.c_int
        _hip = h
    return _hip


HIP_EVENT_DISABLE_TIMING = 0x2


class HipEvent:
    """A raw hipEvent_t owned by Python (destroyed with the object)."""

    def __init__(self, timing: bool = True):
        e = C.c_void_p()
        rc = hip().hipEventCreateWithFlags(C.byref(e), 0 if timing else HIP_EVENT_DISABLE_TIMING)
        if rc != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed: {rc}")
        self.handle = e

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _hip is not None:
            _hip.hipEventDestroy(h)
