"""ctypes loader for libkappa.so (the C ABI declared in include/kappa.h).

Argument marshalling only: every step of the sampler runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkappa.so")

OK, EINVAL, EALIGN, EDEVICE, ENOMEM, EUNSUPPORTED, ERANGE = range(7)
FP64, FP32, FP32_NOTAIL = 0, 1, 2
PARAM_NAMES = ("kstar", "a", "b", "c", "b_over_c", "da", "db", "dc", "lnbeta")
MAX_SEGMENTS = 1 << 24


class KappaError(RuntimeError):
    """A libkappa call returned a non-OK status."""

    def __init__(self, status, func, message):
        self.status = status
        super().__init__(f"{func} failed with status {status}: {message}")


class Segment(ctypes.Structure):
    """kappa_segment: one species in one cell with `count` particles."""
    _fields_ = [
        ("kappa", ctypes.c_double),
        ("theta", ctypes.c_double),
        ("drift", ctypes.c_double * 3),
        ("count", ctypes.c_uint64),
        ("seg_id", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]


class Cell(ctypes.Structure):
    """kappa_cell: the box [lo, lo + size) a segment's positions are drawn in."""
    _fields_ = [
        ("lo", ctypes.c_double * 3),
        ("size", ctypes.c_double * 3),
    ]


_lock = threading.Lock()
_lib = None

# Public entry points: name -> (restype, argtypes)
_vp = ctypes.c_void_p
_u64, _u32, _d, _i = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_int
_st = ctypes.c_int
SIGNATURES = {
    "kappa_params": (_st, [_d, ctypes.POINTER(_d)]),
    "kappa_sample": (_st, [_d, _d, _u64, _u64, _u64, _u32, _i, _vp, _vp, _vp, _vp]),
    "kappa_plan_create": (_st, [ctypes.POINTER(Segment), _u32, _u64, _i, ctypes.POINTER(_vp)]),
    "kappa_plan_total": (_st, [_vp, ctypes.POINTER(_u64)]),
    "kappa_plan_launch": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "kappa_plan_graph_launch": (_st, [_vp, _vp, _vp, _vp, _vp]),
    "kappa_plan_autotune": (_st, [_vp, _vp, _vp, _vp, _i, _vp]),
    "kappa_plan_shape": (_st, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "kappa_plan_set_shape": (_st, [_vp, _i, _i, _i]),
    "kappa_plan_destroy": (_st, [_vp]),
    "kappa_plan_set_cells": (_st, [_vp, ctypes.POINTER(Cell)]),
    "kappa_plan_launch_pic": (_st, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "kappa_plan_graph_launch_pic": (_st, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "kappa_load_particles": (_st, [ctypes.POINTER(Segment), ctypes.POINTER(Cell), _u32, _u64, _i,
                                   _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "kappa_sample_batched": (_st, [ctypes.POINTER(Segment), _u32, _u64, _i, _vp, _vp, _vp, _vp]),
    "kappa_backward_workspace_bytes": (ctypes.c_size_t, [_u64]),
    "kappa_relative_entropy": (_st, [_d, ctypes.POINTER(_u64), _u32, _d, _d, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "kappa_sample_autotune": (_st, [_i, _u64, _vp, _vp, _vp, _i, ctypes.POINTER(_i), ctypes.POINTER(_i), _vp]),
    "kappa_sample_backward": (_st, [_d, _d, _u64, _u64, _u64, _u32, _i, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
    "kappa_sample_backward_noalloc": (_st, [_d, _d, _u64, _u64, _u64, _u32, _i, _vp, _vp, _vp, _vp, _vp]),
    "kappa_philox": (_st, [_u64, _u64, _u64, _u32, _u32, _vp, _vp]),
    "kappa_sample_exact_t": (_st, [_d, _d, _u64, _u64, _i, _vp, _vp, _vp, _vp, _vp]),
    "kappa_sample_exact_pareto": (_st, [_d, _d, _u64, _u64, _i, _vp, _vp, _vp, _vp, _vp]),
    "kappa_speed_histogram": (_st, [_vp, _vp, _vp, _u64, _i, _d, _d, _u32, _vp, _vp]),
    "kappa_divergence_grid": (_st, [_vp, _u32, _vp, _u32, _vp, _vp, _vp, _vp]),
    "kappa_optimum_c": (_st, [_vp, _u32, _vp, _u32, _u32, _vp, _vp, _vp]),
    "kappa_fill_probe": (_st, [_u64, _i, _vp, _vp, _vp, _vp]),
    "kappa_copy_probe": (_st, [_vp, _vp, _u64, _vp]),
    "kappa_issue_probe": (_st, [_i, _vp, _u64, _vp, _u64, ctypes.POINTER(_u32), ctypes.POINTER(_u32),
                                ctypes.POINTER(_d), _vp]),
    "kappa_transcendental_probe": (_st, [_i, _vp, _vp, _u64, _vp]),
    "kappa_clock_probe": (_st, [_d, _d, _u64, _u64, _u64, _u32, _i, _vp, _vp, _vp, _vp, _u64,
                                ctypes.POINTER(_u32), ctypes.POINTER(_d), _vp]),
    "kappa_status_string": (ctypes.c_char_p, [_i]),
    "kappa_last_error": (ctypes.c_char_p, []),
    "kappa_version": (ctypes.c_char_p, []),
}


def load():
    """Load libkappa.so (once).  Raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -m paper_2602_05606_amd.build, or __graft_entry__.build()).  "
                "There is no fallback implementation.")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
        return lib


def check(status, func):
    if status != OK:
        msg = load().kappa_last_error().decode(errors="replace")
        raise KappaError(status, func, msg)
