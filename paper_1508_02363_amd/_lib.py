"""ctypes loader for libdbar.so (the HIP library).  Loading fails loudly: there is no fallback implementation."""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdbar.so")

DBAR_OK = 0
DBAR_EINVAL = -1
DBAR_ENOMEM = -2
DBAR_ENOCONV = -3
DBAR_EDEVICE = -4
DBAR_EAGAIN = -5
DBAR_ENOTFOUND = -6

DBAR_FP64 = 0
DBAR_MIXED = 1
DBAR_FP32 = 2
DBAR_MODE_BATCHED = 0
DBAR_MODE_PLAIN = 1
DBAR_METHOD_PLAIN = 0
DBAR_METHOD_ITERATED = 1
DBAR_SPACE_X = 0
DBAR_SPACE_XI = 1

# every symbol include/dbar.h declares
EXPORTED = [
    "dbar_default_opts", "dbar_solve", "dbar_solve_device", "dbar_apply", "dbar_apply_noalloc", "dbar_transform",
    "dbar_dbar_inverse",
    "dbar_reflection", "dbar_reconstruct", "dbar_autotune", "dbar_set_tile", "dbar_get_tile",
    "dbar_session_create", "dbar_submit", "dbar_poll", "dbar_wait", "dbar_session_get_stats",
    "dbar_request_footprint", "dbar_session_destroy", "dbar_timer_enable", "dbar_timer_num_stages",
    "dbar_timer_stage", "dbar_last_error", "dbar_release", "dbar_version",
]


class TuneResult(ctypes.Structure):
    _fields_ = [("n_variants", ctypes.c_int32 * 2), ("chosen", ctypes.c_int32 * 2),
                ("columns", (ctypes.c_int32 * 4) * 2), ("ms", (ctypes.c_double * 4) * 2),
                ("batch", ctypes.c_int32), ("batch_candidates", ctypes.c_int32 * 4), ("reserved", ctypes.c_int32),
                ("per_entry_ms", ctypes.c_double * 4)]


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("M", ctypes.c_int32), ("L", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("batch", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("reorth", ctypes.c_int32), ("check_every", ctypes.c_int32), ("method", ctypes.c_int32),
                ("space", ctypes.c_int32), ("inner_tol", ctypes.c_double), ("orth_window", ctypes.c_int32),
                ("lanes", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("m1_re", ctypes.c_double),
                ("m1_im", ctypes.c_double), ("cond_estimate", ctypes.c_double), ("err_estimate", ctypes.c_double)]


class SessionOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SessionStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("in_flight", ctypes.c_uint64), ("queued", ctypes.c_uint64), ("bytes_in_use", ctypes.c_size_t),
                ("bytes_reserved", ctypes.c_size_t), ("classes_created", ctypes.c_uint64),
                ("classes_released", ctypes.c_uint64)]


_lib = None
_lock = threading.Lock()


class DbarError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"dbar error {code}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    """Load libdbar.so (built in-tree by __graft_entry__.build() / paper_1508_02363_amd.build_lib)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1508_02363_amd.build_lib`")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        D = ctypes.POINTER(ctypes.c_double)
        G = ctypes.POINTER(Grid)
        lib.dbar_default_opts.argtypes = [ctypes.POINTER(Opts)]
        lib.dbar_default_opts.restype = None
        lib.dbar_solve.argtypes = [G, D, ctypes.c_int64, D, ctypes.c_double, ctypes.POINTER(Opts), D, D,
                                   ctypes.POINTER(Info)]
        lib.dbar_solve_device.argtypes = [G, P, ctypes.c_int64, D, ctypes.c_double, ctypes.POINTER(Opts), P, P,
                                          ctypes.POINTER(Info), P]
        lib.dbar_apply.argtypes = [G, D, D, D, D, ctypes.c_int32]
        lib.dbar_apply_noalloc.argtypes = [G, P, D, P, P, ctypes.c_int32, P]
        lib.dbar_transform.argtypes = [G, ctypes.c_int32, D, D, ctypes.c_int32]
        lib.dbar_dbar_inverse.argtypes = [G, D, D, ctypes.c_int32]
        lib.dbar_autotune.argtypes = [G, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(TuneResult)]
        lib.dbar_set_tile.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        I32P = ctypes.POINTER(ctypes.c_int32)
        lib.dbar_get_tile.argtypes = [ctypes.c_int32, ctypes.c_int32, I32P, I32P, I32P]
        lib.dbar_reflection.argtypes = [G, D, ctypes.c_int64, D, ctypes.c_double, ctypes.POINTER(Opts), D,
                                        ctypes.POINTER(Info)]
        lib.dbar_reconstruct.argtypes = [G, D, ctypes.c_double, ctypes.c_double, ctypes.POINTER(Opts), D,
                                         ctypes.POINTER(Info)]
        if hasattr(lib, "dbar_session_create"):
            lib.dbar_session_create.argtypes = [ctypes.POINTER(SessionOpts), ctypes.POINTER(P)]
            lib.dbar_submit.argtypes = [P, G, D, D, ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]
            lib.dbar_poll.argtypes = [P, ctypes.c_uint64, D, D, ctypes.POINTER(Info), D]
            lib.dbar_wait.argtypes = [P, ctypes.c_uint64, D, D, ctypes.POINTER(Info), D]
            lib.dbar_session_get_stats.argtypes = [P, ctypes.POINTER(SessionStats)]
            lib.dbar_request_footprint.argtypes = [G, ctypes.c_int32, ctypes.c_int32]
            lib.dbar_request_footprint.restype = ctypes.c_size_t
            lib.dbar_session_destroy.argtypes = [P]
            lib.dbar_session_destroy.restype = None
        lib.dbar_timer_enable.argtypes = [ctypes.c_int32]
        lib.dbar_timer_num_stages.argtypes = []
        lib.dbar_timer_stage.argtypes = [ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32, D,
                                         ctypes.POINTER(ctypes.c_int64), D]
        lib.dbar_last_error.argtypes = []
        lib.dbar_last_error.restype = ctypes.c_char_p
        lib.dbar_release.argtypes = []
        lib.dbar_release.restype = None
        lib.dbar_version.argtypes = []
        _lib = lib
        return lib


def check(rc: int, allow=(DBAR_OK,)) -> int:
    if rc not in allow:
        msg = load().dbar_last_error().decode(errors="replace")
        raise DbarError(rc, msg)
    return rc
