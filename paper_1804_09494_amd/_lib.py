"""ctypes declarations of libtucker_hip.so (include/tucker_hip.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation anywhere in the package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtucker_hip.so")

c_i32, c_i64, c_u8, c_f32, c_f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint8, ctypes.c_float, ctypes.c_double
c_void_p, c_int, c_char_p = ctypes.c_void_p, ctypes.c_int, ctypes.c_char_p

TK_OK = 0
STATUS = {0: "TK_OK", 1: "TK_ERR_INVALID_ARG", 2: "TK_ERR_STATE", 3: "TK_ERR_OOM", 4: "TK_ERR_DEVICE",
          5: "TK_ERR_NUMERIC", 6: "TK_ERR_UNSUPPORTED"}
TK_MEM_HOST, TK_MEM_DEVICE = 0, 1
TK_FP32, TK_BF16 = 0, 1
TK_SWEEP_GAUSS_SEIDEL, TK_SWEEP_JACOBI = 0, 1
TK_NOALLOC_SCRATCH_BYTES = 32 << 20
TK_ASSUME_UNIQUE = 1
TK_PART_LITE, TK_PART_COARSE = 0, 1
TK_TTM_AUTO, TK_TTM_VECTOR, TK_TTM_ATOMIC, TK_TTM_FIBER = 0, 1, 2, 3
TK_EIG_AUTO, TK_EIG_GRAM, TK_EIG_MATFREE = 0, 1, 2
TK_MATFREE_MIN_KHAT = 8192


class tk_options(ctypes.Structure):
    _fields_ = [("prec", c_i32), ("sweep", c_i32), ("wg_nnz_target", c_i64), ("lds_rows_cap", c_i32),
                ("refine", c_i32), ("mem_limit_bytes", c_i64),
                ("complete_rank_deficient", c_i32), ("keep_elem_order", c_i32), ("eig_tol", c_f64),
                ("partition", c_i32), ("ttm_kernel", c_i32), ("eig_method", c_i32)]


TK_ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p)
TK_FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, ctypes.c_size_t, c_void_p)


class tk_allocator(ctypes.Structure):
    _fields_ = [("alloc", TK_ALLOC_FN), ("free", TK_FREE_FN), ("user", c_void_p)]


class tk_part_stats(ctypes.Structure):
    _fields_ = [(n, c_i64) for n in ("P", "limit", "m", "L_nonempty", "n_stage1", "E_max", "R_sum", "R_max",
                                     "n_bad")]


# (name, restype, argtypes) of every exported symbol
SIGNATURES = [
    ("tk_create", c_int, [c_int, c_void_p, ctypes.POINTER(tk_allocator), ctypes.POINTER(c_void_p)]),
    ("tk_destroy", None, [c_void_p]),
    ("tk_status_string", c_char_p, [c_int]),
    ("tk_last_error", c_char_p, [c_void_p]),
    ("tk_default_options", c_int, [ctypes.POINTER(tk_options)]),
    ("tk_set_options", c_int, [c_void_p, ctypes.POINTER(tk_options)]),
    ("tk_set_stream", c_int, [c_void_p, c_void_p]),
    ("tk_load_coo", c_int, [c_void_p, c_int, ctypes.POINTER(c_i64), c_i64, ctypes.POINTER(c_void_p), c_void_p,
                            c_int, ctypes.c_uint]),
    ("tk_load_coo_begin", c_int, [c_void_p, c_int, ctypes.POINTER(c_i64), c_i64, ctypes.c_uint]),
    ("tk_load_coo_append", c_int, [c_void_p, c_i64, ctypes.POINTER(c_void_p), c_void_p, c_int]),
    ("tk_load_coo_end", c_int, [c_void_p]),
    ("tk_get_tensor_info", c_int, [c_void_p, ctypes.POINTER(c_i64), ctypes.POINTER(c_f64)]),
    ("tk_get_coo", c_int, [c_void_p, ctypes.POINTER(c_void_p), c_void_p, c_int]),
    ("tk_set_ranks", c_int, [c_void_p, ctypes.POINTER(c_i32)]),
    ("tk_set_slice_order", c_int, [c_void_p, c_int, c_void_p, c_int]),
    ("tk_get_partition_stats", c_int, [c_void_p, c_int, ctypes.POINTER(tk_part_stats)]),
    ("tk_get_partition", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_int]),
    ("tk_set_factor", c_int, [c_void_p, c_int, c_void_p, c_int]),
    ("tk_get_factor", c_int, [c_void_p, c_int, c_void_p, c_int]),
    ("tk_ttm_shape", c_int, [c_void_p, c_int, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64)]),
    ("tk_ttm_chain", c_int, [c_void_p, c_int, c_void_p, c_void_p, c_int]),
    ("tk_ttm_chain_noalloc", c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    ("tk_hooi_iterate", c_int, [c_void_p, c_int, c_void_p]),
    ("tk_init_hosvd", c_int, [c_void_p, c_void_p, c_int, c_void_p]),
    ("tk_core", c_int, [c_void_p, c_void_p, ctypes.POINTER(c_f64), c_int]),
    ("tk_get_timings", c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_int)]),
    ("tk_get_counters", c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_int)]),
    ("tk_load_obs", c_int, [c_void_p, c_int, ctypes.POINTER(c_i64), ctypes.POINTER(c_i32), c_i64,
                            ctypes.POINTER(c_void_p), c_int]),
    ("tk_tucker_eval", c_int, [c_void_p, c_void_p, ctypes.POINTER(c_void_p), c_void_p, c_int]),
    ("tk_tucker_adjoint", c_int, [c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_void_p), c_void_p,
                                  ctypes.POINTER(c_void_p), c_int]),
]

_lib = None


def load():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1804_09494_amd.build.build() "
                              "(there is no fallback implementation)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


class TuckerError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
