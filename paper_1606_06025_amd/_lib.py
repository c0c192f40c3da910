"""ctypes binding of libcsrcolor.so (argument marshalling only).

Every step of a colouring runs in the library's HIP kernels; this module only
passes device pointers, sizes and the current HIP stream.  It raises if the
library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsrcolor.so")

OK = 0
EINVAL = -1
EBADCSR = -2
ENOMEM = -3
EHIP = -4
EOVERFLOW = -5
ENOTSYM = -6
ELIMIT = -7
ETIMEOUT = -8
ETOOBIG = -9

NOALLOC_MAX_N = 1048576
NOALLOC_MAX_NNZ = 33554432

RULE_ID = 0
RULE_DEGREE = 1

ALGO_SGR = 0
ALGO_SGR_TOPO = 1
ALGO_JP = 2

MODE_AUTO = 0
MODE_LOOP = 1
MODE_PERSISTENT = 2
MODE_GRAPH = 3

EXPORTS = ["csrcolor_color", "csrcolor_color_ex", "csrcolor_color_batched", "csrcolor_color_multi",
           "csrcolor_color_noalloc", "csrcolor_strerror", "csrcolor_release_workspace", "csrcolor_version",
           "csrcolor_workspace_bytes", "csrcolor_device_bytes_in_use"]


class Opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("validate", ctypes.c_int32), ("t_wave", ctypes.c_int32),
                ("t_split", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("sync_every", ctypes.c_int32), ("lane_assign", ctypes.c_int32),
                ("lane_detect", ctypes.c_int32), ("firstfit", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("algorithm", ctypes.c_int32), ("seed_lo", ctypes.c_uint32),
                ("seed_hi", ctypes.c_uint32), ("hints", ctypes.c_int32),
                ("live_lists", ctypes.c_int32), ("ordered", ctypes.c_int32),
                ("wake", ctypes.c_int32), ("tile_limits", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("ncolors", ctypes.c_int32), ("rows_sorted", ctypes.c_int32),
                ("max_degree", ctypes.c_int32), ("nnz", ctypes.c_int64), ("cap", ctypes.c_int32),
                ("time_kernels", ctypes.c_int32), ("wsize", ctypes.POINTER(ctypes.c_int64)),
                ("arcs", ctypes.POINTER(ctypes.c_int64)), ("ms_setup", ctypes.c_double),
                ("ms_assign", ctypes.c_double), ("ms_detect", ctypes.c_double),
                ("n_assign", ctypes.c_int32), ("n_detect", ctypes.c_int32),
                ("kernel_bytes", ctypes.POINTER(ctypes.c_int64))]


class CsrColorError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"csrcolor status {status}: {msg}")
        self.status = status


_lib: Optional[ctypes.CDLL] = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load the HIP library (import torch first so one HIP runtime is shared)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "or `python -m paper_1606_06025_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32 = ctypes.c_void_p, ctypes.c_int32
    lib.csrcolor_color.argtypes = [I32, P, P, P, ctypes.POINTER(I32), P]
    lib.csrcolor_color.restype = ctypes.c_int
    # the colour-count argument of csrcolor_color_ex is a DEVICE pointer
    lib.csrcolor_color_ex.argtypes = [I32, P, P, P, P, ctypes.POINTER(Opts), ctypes.POINTER(Stats), P]
    lib.csrcolor_color_ex.restype = ctypes.c_int
    # csrcolor_color_noalloc: n, nnz, rowptr, colidx, colors_out, DEVICE colour count, stream
    lib.csrcolor_color_noalloc.argtypes = [I32, ctypes.c_int64, P, P, P, P, P]
    lib.csrcolor_color_noalloc.restype = ctypes.c_int
    lib.csrcolor_color_batched.argtypes = [I32, I32, P, P, P, P, P, ctypes.POINTER(Opts), P]
    lib.csrcolor_color_batched.restype = ctypes.c_int
    lib.csrcolor_color_multi.argtypes = [I32, P, P, P, P, P, P, ctypes.POINTER(Opts), P]
    lib.csrcolor_color_multi.restype = ctypes.c_int
    lib.csrcolor_strerror.argtypes = [ctypes.c_int]
    lib.csrcolor_strerror.restype = ctypes.c_char_p
    lib.csrcolor_release_workspace.argtypes = []
    lib.csrcolor_release_workspace.restype = None
    lib.csrcolor_workspace_bytes.argtypes = [I32, ctypes.c_int64, ctypes.c_int64]
    lib.csrcolor_workspace_bytes.restype = ctypes.c_int64
    lib.csrcolor_device_bytes_in_use.argtypes = []
    lib.csrcolor_device_bytes_in_use.restype = ctypes.c_int64
    lib.csrcolor_version.argtypes = []
    lib.csrcolor_version.restype = ctypes.c_int
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().csrcolor_strerror(status).decode()


def check(status: int) -> None:
    if status != OK:
        raise CsrColorError(status, strerror(status))
