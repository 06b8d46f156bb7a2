"""ctypes declarations of libcpc.so (the C-ABI in include/cpc.h).

The library is loaded from the package directory; there is no fallback: a
missing or unloadable libcpc.so raises immediately.
"""
from __future__ import annotations

import ctypes
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libcpc.so"

CPC_OK, CPC_E_ARG, CPC_E_NOT_SPD, CPC_E_BREAKDOWN, CPC_E_MAXIT, CPC_E_DEVICE, CPC_E_NOMEM = range(7)
STATUS_NAMES = {0: "CPC_OK", 1: "CPC_E_ARG", 2: "CPC_E_NOT_SPD", 3: "CPC_E_BREAKDOWN", 4: "CPC_E_MAXIT",
                5: "CPC_E_DEVICE", 6: "CPC_E_NOMEM"}

PREC = {"combined": 0, "amg": 1, "ilu": 2, "additive": 3, "none": 4, "amg_ilu": 5, "bbar": 6}
OP = {"combined": 0, "amg": 1, "ilu": 2, "additive": 3, "none": 4, "vcycle": 5, "fgs": 6, "bgs": 7,
      "amg_ilu": 8, "bbar": 9}
PRECISION = {"fp64": 0, "fp32": 1}
DENSE = {"auto": 0, "never": 1, "always": 2, "block": 3}

# every entry point declared in include/cpc.h
EXPORTS = ("cpc_default_options", "cpc_setup", "cpc_solve", "cpc_solve_with", "cpc_apply_op", "cpc_spmv",
           "cpc_hierarchy_info", "cpc_get_level", "cpc_get_prolongation", "cpc_get_ilu", "cpc_get_stats",
           "cpc_neg_outer_on_pattern", "cpc_time_kernel", "cpc_destroy", "cpc_last_error", "cpc_tpfa_pattern",
           "cpc_tpfa_values", "cpc_tpfa_logk_grad", "cpc_set_operator_values", "cpc_setup_batch",
           "cpc_solve_batch", "cpc_batch_info", "cpc_smoother_kind", "cpc_smoother_bytes", "cpc_get_ilu_factor", "cpc_solve_noalloc",
           "cpc_spgemm")
KERNEL = {"spmv_pq": 0, "fgs": 1, "bgs": 2, "ilu_l": 3, "ilu_u": 4, "residual": 5, "restrict": 6, "prolong": 7,
          "vcycle": 8, "precond": 9, "iteration": 10, "dense_gemv": 11, "sweep": 12}


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("prec", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_coarse", ctypes.c_int32), ("max_levels", ctypes.c_int32), ("swap_roles", ctypes.c_int32),
                ("check_symmetry", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("rap_on_gpu", ctypes.c_int32), ("sweep_block_rows", ctypes.c_int32),
                ("sweep_threads", ctypes.c_int32), ("dense_smoother", ctypes.c_int32),
                ("tune", ctypes.c_int32), ("verbose", ctypes.c_int32), ("ilu_fill", ctypes.c_int32),
                ("theta", ctypes.c_double), ("sweep_kernel", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("relres", ctypes.c_double),
                ("setup_s", ctypes.c_double), ("solve_s", ctypes.c_double), ("bytes_per_iter", ctypes.c_double),
                ("bytes_initial", ctypes.c_double), ("method_bytes_per_iter", ctypes.c_double),
                ("method_bytes_initial", ctypes.c_double)]


class CpcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load():
    """Load libcpc.so (raises if it is missing: there is no other code path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1205_6113_amd.build`")
    lib = ctypes.CDLL(str(LIB_PATH))
    P = ctypes.c_void_p
    I32 = ctypes.c_int32
    D = ctypes.c_double
    lib.cpc_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.cpc_default_options.restype = None
    lib.cpc_setup.argtypes = [I32, P, P, P, ctypes.POINTER(Options), P, ctypes.POINTER(P)]
    lib.cpc_setup.restype = I32
    lib.cpc_solve.argtypes = [P, P, P, I32, D, I32, ctypes.POINTER(I32), ctypes.POINTER(D)]
    lib.cpc_solve.restype = I32
    lib.cpc_solve_noalloc.argtypes = [P, P, P, I32, D, I32, ctypes.POINTER(I32), ctypes.POINTER(D)]
    lib.cpc_solve_noalloc.restype = I32
    lib.cpc_solve_with.argtypes = [P, I32, P, P, I32, D, I32, ctypes.POINTER(I32), ctypes.POINTER(D)]
    lib.cpc_solve_with.restype = I32
    lib.cpc_apply_op.argtypes = [P, I32, P, P]
    lib.cpc_apply_op.restype = I32
    lib.cpc_spmv.argtypes = [P, I32, P, P]
    lib.cpc_spmv.restype = I32
    lib.cpc_spgemm.argtypes = [I32, I32, I32, P, P, P, P, P, P, P, P, P, ctypes.POINTER(ctypes.c_int64)]
    lib.cpc_spgemm.restype = I32
    lib.cpc_hierarchy_info.argtypes = [P, ctypes.POINTER(I32), P, P, P]
    lib.cpc_hierarchy_info.restype = I32
    lib.cpc_smoother_kind.argtypes = [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]
    lib.cpc_smoother_kind.restype = I32
    lib.cpc_smoother_bytes.argtypes = [P, I32, ctypes.POINTER(ctypes.c_int64)]
    lib.cpc_smoother_bytes.restype = I32
    lib.cpc_get_level.argtypes = [P, I32, P, P, P]
    lib.cpc_get_level.restype = I32
    lib.cpc_get_prolongation.argtypes = [P, I32, ctypes.POINTER(ctypes.c_int64), P, P, P, P]
    lib.cpc_get_prolongation.restype = I32
    lib.cpc_get_ilu.argtypes = [P, P]
    lib.cpc_get_ilu.restype = I32
    lib.cpc_get_ilu_factor.argtypes = [P, ctypes.POINTER(ctypes.c_int64), P, P, P]
    lib.cpc_get_ilu_factor.restype = I32
    lib.cpc_get_stats.argtypes = [P, ctypes.POINTER(Stats)]
    lib.cpc_get_stats.restype = I32
    lib.cpc_neg_outer_on_pattern.argtypes = [P, P, P, P]
    lib.cpc_neg_outer_on_pattern.restype = I32
    lib.cpc_time_kernel.argtypes = [P, I32, I32, I32, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I32),
                                    ctypes.POINTER(D)]
    lib.cpc_time_kernel.restype = I32
    lib.cpc_tpfa_pattern.argtypes = [I32, I32, I32, P, P]
    lib.cpc_tpfa_pattern.restype = I32
    lib.cpc_tpfa_values.argtypes = [I32, I32, I32, D, I32, P, P, P, P]
    lib.cpc_tpfa_values.restype = I32
    lib.cpc_tpfa_logk_grad.argtypes = [I32, I32, I32, D, I32, P, P, P, P, P]
    lib.cpc_tpfa_logk_grad.restype = I32
    lib.cpc_set_operator_values.argtypes = [P, P]
    lib.cpc_set_operator_values.restype = I32
    lib.cpc_setup_batch.argtypes = [I32, P, P, P, P, ctypes.POINTER(Options), P, ctypes.POINTER(P)]
    lib.cpc_setup_batch.restype = I32
    lib.cpc_solve_batch.argtypes = [P, P, P, D, I32, P, P]
    lib.cpc_solve_batch.restype = I32
    lib.cpc_batch_info.argtypes = [P, ctypes.POINTER(I32), P, P]
    lib.cpc_batch_info.restype = I32
    lib.cpc_destroy.argtypes = [P]
    lib.cpc_destroy.restype = None
    lib.cpc_last_error.argtypes = []
    lib.cpc_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def last_error() -> str:
    msg = load().cpc_last_error()
    return msg.decode() if msg else ""


def check(status: int, allow=(CPC_OK,)):
    if status not in allow:
        raise CpcError(status, last_error())
    return status
