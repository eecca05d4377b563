"""ctypes declarations of the C ABI in ``include/slu.h`` (marshalling only).

Every entry point of the header is bound under its own name on ``lib``.
Importing this module loads ``libslu.so`` from the package directory and
raises ImportError if it has not been built: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslu.so")

SLU_OK = 0
SLU_ZERO_PIVOT = 1
SLU_NOT_CONVERGED = 2
SLU_ERR_ARG = -1
SLU_ERR_ROWPTR = -2
SLU_ERR_COLIDX = -3
SLU_ERR_UNSORTED = -4
SLU_ERR_PERM = -5
SLU_ERR_STATE = -6
SLU_ERR_WORKSPACE = -7
SLU_ERR_HIP = -8
SLU_ERR_NOMEM = -9
SLU_ERR_NOT_FACTORED = -10
SLU_ERR_LIMIT = -11

SLU_ORDER_NATURAL = 0
SLU_ORDER_GRID_ND = 1
SLU_ORDER_USER = 2
SLU_ORDER_GRAPH_ND = 3
SLU_BLOCK_IRREGULAR = 0
SLU_BLOCK_REGULAR = 1
SLU_SCHEDULE_WAVES = 0
SLU_SCHEDULE_LEVELS = 1
SLU_PRECISION_FP64 = 0
SLU_PRECISION_FP32 = 1
KERNELS = ("scatter", "getrf", "panel", "ssssm")

EXPORTS = [
    "slu_default_options", "slu_analyze", "slu_workspace_size", "slu_bind_workspace",
    "slu_factor", "slu_solve", "slu_solve_transpose", "slu_backward_error", "slu_get_info",
    "slu_get_perm", "slu_get_blockptr", "slu_get_blocking", "slu_get_pattern",
    "slu_get_factors", "slu_error_string", "slu_free", "slu_set_profiling",
    "slu_get_kernel_times", "slu_value_gradient", "slu_set_precision", "slu_solve_refined",
    "slu_analyze_batch", "slu_set_graph", "slu_last_hip_error", "slu_hip_error_string",
    "slu_set_host_threads", "slu_set_getrf_split", "slu_set_getrf_tiled", "slu_solve_noalloc", "slu_set_getrf_tile",
    "slu_set_panel_blocked", "slu_set_solve_tiled", "slu_autotune", "slu_set_lookahead",
]


class slu_options(ctypes.Structure):
    _fields_ = [
        ("sample_points", ctypes.c_int32),
        ("step", ctypes.c_int32),
        ("max_num", ctypes.c_int32),
        ("advance", ctypes.c_int32),
        ("blocking", ctypes.c_int32),
        ("regular_block", ctypes.c_int32),
        ("ordering", ctypes.c_int32),
        ("grid_dims", ctypes.c_int32 * 3),
        ("schedule", ctypes.c_int32),
        ("user_perm", ctypes.c_void_p),
    ]


class slu_tune_entry(ctypes.Structure):
    _fields_ = [
        ("getrf_tiled_rows", ctypes.c_int32),
        ("getrf_tile", ctypes.c_int32),
        ("panel_blocked", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("lookahead", ctypes.c_int32),
        ("ms", ctypes.c_double),
    ]


class slu_info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz_a", ctypes.c_int64),
        ("nnz_s", ctypes.c_int64),
        ("nblocks", ctypes.c_int64),
        ("nonempty_blocks", ctypes.c_int64),
        ("ssssm_tasks", ctypes.c_int64),
        ("flops", ctypes.c_double),
        ("flops_getrf", ctypes.c_double),
        ("flops_panel", ctypes.c_double),
        ("flops_ssssm", ctypes.c_double),
        ("stored_flops", ctypes.c_double),
        ("slab_bytes", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
        ("zero_pivot_col", ctypes.c_int64),
        ("factored", ctypes.c_int32),
        ("max_block", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("waves", ctypes.c_int32),
        ("rounds", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libslu.so is not built (run paper_2512_04389_amd.build.build())")
    # torch ships its own HIP runtime under the same soname.  Loading torch
    # first makes libslu.so bind to that copy; loaded the other way round the
    # process holds two HIP (and HSA) runtimes, and the second one to start
    # finds no device.  Tensors and streams come from torch, so its runtime
    # is the one the library must share.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    p, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    hp = ctypes.c_void_p
    sig = {
        "slu_default_options": (None, [ctypes.POINTER(slu_options)]),
        "slu_analyze": (i32, [i64, p, p, ctypes.POINTER(slu_options), ctypes.POINTER(hp)]),
        "slu_workspace_size": (i32, [hp, ctypes.POINTER(ctypes.c_size_t)]),
        "slu_bind_workspace": (i32, [hp, p, ctypes.c_size_t, p]),
        "slu_factor": (i32, [hp, p, p]),
        "slu_solve": (i32, [hp, p, p, i64, i64, p]),
        "slu_solve_transpose": (i32, [hp, p, p, i64, i64, p]),
        "slu_backward_error": (i32, [hp, p, p, p, i64, i64, i32, p, p]),
        "slu_get_info": (i32, [hp, ctypes.POINTER(slu_info)]),
        "slu_get_perm": (i32, [hp, p]),
        "slu_get_blockptr": (i32, [hp, p]),
        "slu_get_blocking": (i32, [hp, p]),
        "slu_get_pattern": (i32, [hp, p, p]),
        "slu_get_factors": (i32, [hp, p, p, p]),
        "slu_error_string": (ctypes.c_char_p, [i32]),
        "slu_free": (None, [hp]),
        "slu_set_profiling": (i32, [hp, i32]),
        "slu_get_kernel_times": (i32, [hp, p, p]),
        "slu_value_gradient": (i32, [hp, p, p, i64, i64, p, p]),
        "slu_set_precision": (i32, [hp, i32]),
        "slu_set_graph": (i32, [hp, i32]),
        "slu_set_getrf_split": (i32, [hp, ctypes.c_double]),
        "slu_set_getrf_tiled": (i32, [hp, ctypes.c_int]),
        "slu_solve_noalloc": (i32, [hp, p, p, i64, i64, i32, p]),
        "slu_set_getrf_tile": (i32, [hp, ctypes.c_int]),
        "slu_set_panel_blocked": (i32, [hp, ctypes.c_int]),
        "slu_set_lookahead": (i32, [hp, ctypes.c_int, ctypes.c_int]),
        "slu_set_solve_tiled": (i32, [hp, ctypes.c_int, ctypes.c_int]),
        "slu_autotune": (i32, [hp, p, i32, p, i32, ctypes.POINTER(ctypes.c_int), p]),
        "slu_last_hip_error": (i32, []),
        "slu_set_host_threads": (i32, [i32]),
        "slu_hip_error_string": (ctypes.c_char_p, [i32]),
        "slu_analyze_batch": (i32, [i64, p, p, p, p, ctypes.POINTER(slu_options), ctypes.POINTER(hp)]),
        "slu_solve_refined": (i32, [hp, p, p, p, i64, i64, ctypes.c_double, i32, ctypes.POINTER(ctypes.c_int),
                                    p, p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


class SluError(RuntimeError):
    def __init__(self, code, where):
        msg = lib.slu_error_string(code).decode()
        self.hip_error = 0
        if code == SLU_ERR_HIP:
            self.hip_error = lib.slu_last_hip_error()
            msg += " %d: %s" % (self.hip_error, lib.slu_hip_error_string(self.hip_error).decode())
        super().__init__("%s failed: %s (code %d)" % (where, msg, code))
        self.code = code


class ZeroPivot(SluError):
    def __init__(self, col):
        RuntimeError.__init__(self, "zero or non-finite pivot at permuted column %d" % col)
        self.code = SLU_ZERO_PIVOT
        self.col = col


def check(code, where):
    if code != SLU_OK:
        raise SluError(code, where)
