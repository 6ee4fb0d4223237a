"""ctypes declarations of the C ABI in include/blrqr.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libblrqr.so")

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p

EXPORTED = [
    "blr_compress", "blr_import", "blr_export", "blr_qr_factor", "blr_apply_qt",
    "blr_lstsq_solve", "blr_query", "blr_destroy", "blr_status_string", "blr_last_error",
    "blr_profile_enable", "blr_profile_read", "blr_matmul", "blr_morton_sort", "blr_rsolve",
    "blr_lstsq_adjoint", "blr_form_q", "blr_qr_factor_batch", "blr_lstsq_solve_batch",
    "blr_apply_qt_noalloc", "blr_mgs_qr",
]
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024   # BLR_NOALLOC_SCRATCH_BYTES
SELFTEST = ["blr_selftest_gemm"]
MATMUL = {"A": 0, "AT": 1, "R": 2}

BLR_OK, BLR_ERR_INVALID, BLR_ERR_STATE, BLR_ERR_OOM, BLR_ERR_DEVICE, BLR_ERR_NONFINITE, BLR_ERR_SINGULAR = range(7)
SRC_KERNEL, SRC_DENSE = 0, 1
KERNEL_LOG2D, KERNEL_INV_R = 0, 1
ADM = {"adjacent": 0, "dist_gt_diam": 1, "weak": 2, "mask": 3}
OVERFLOW = {"dense": 0, "truncate": 1}
VARIANT = {"tiled": 0, "block_column": 1}
PRECISION = {"fp64": 0, "mixed": 1}


class Source(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("x", c_void_p), ("y", c_void_p), ("dim", c_int32),
                ("kernel", c_int32), ("reg", c_double), ("A", c_void_p), ("lda", c_int64),
                ("admissibility", c_int32), ("mask", c_void_p)]


class CompressOpts(ctypes.Structure):
    _fields_ = [("m", c_int64), ("n", c_int64), ("tile", c_int32), ("tol", c_double),
                ("max_rank", c_int32), ("overflow", c_int32), ("seed", ctypes.c_uint64)]


class FactorOpts(ctypes.Structure):
    _fields_ = [("variant", c_int32), ("precision", c_int32), ("ib", c_int32), ("stop_after_k", c_int32),
                ("keep_a", c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("m", c_int64), ("n", c_int64), ("tile", c_int32), ("p", c_int32), ("q", c_int32),
                ("max_rank", c_int32), ("rank_capacity", c_int32), ("state", c_int32),
                ("variant", c_int32), ("precision", c_int32), ("ib", c_int32),
                ("n_dense", c_int64), ("n_lowrank", c_int64), ("n_fill_in", c_int64),
                ("device_bytes", c_int64), ("compress_overflow", c_int64),
                ("factor_overflow", c_int64), ("max_dropped_rel", c_double),
                ("flops_factor", c_double), ("kernel_launches", c_int64),
                ("m_pad", c_int64), ("n_pad", c_int64), ("p_pad", c_int32), ("pad_", c_int32)]


class TilesHost(ctypes.Structure):
    _fields_ = [("fmt", c_void_p), ("rank", c_void_p), ("dense", c_void_p), ("U", c_void_p),
                ("V", c_void_p), ("Y", c_void_p), ("T", c_void_p)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libblrqr.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: run `python -m paper_2208_06194_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.blr_compress.argtypes = [P(Source), P(CompressOpts), c_void_p, P(c_void_p)]
    lib.blr_import.argtypes = [P(CompressOpts), P(TilesHost), c_void_p, P(c_void_p)]
    lib.blr_export.argtypes = [c_void_p, P(TilesHost)]
    lib.blr_qr_factor.argtypes = [c_void_p, P(FactorOpts), c_void_p]
    lib.blr_qr_factor_batch.argtypes = [P(c_void_p), c_int32, P(FactorOpts), c_void_p]
    lib.blr_lstsq_solve_batch.argtypes = [P(c_void_p), c_int32, P(c_void_p), P(c_int64), P(c_void_p),
                                          P(c_int64), c_int32, c_int32, c_void_p]
    lib.blr_apply_qt.argtypes = [c_void_p, c_int32, c_void_p, c_int64, c_int32, c_void_p]
    lib.blr_apply_qt_noalloc.argtypes = [c_void_p, c_int32, c_void_p, c_int64, c_int32, c_void_p]
    lib.blr_lstsq_solve.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_int32, c_int32,
                                    c_void_p, c_void_p]
    lib.blr_matmul.argtypes = [c_void_p, c_int32, c_void_p, c_int64, c_void_p, c_int64, c_int32, c_void_p]
    lib.blr_morton_sort.argtypes = [c_void_p, c_int64, c_int32, c_void_p, c_void_p, c_void_p]
    lib.blr_rsolve.argtypes = [c_void_p, c_int32, c_void_p, c_int64, c_int32, c_void_p]
    lib.blr_form_q.argtypes = [c_void_p, c_void_p, P(c_void_p)]
    lib.blr_mgs_qr.argtypes = [c_void_p, c_void_p, P(c_void_p)]
    lib.blr_lstsq_adjoint.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_int32,
                                      c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.blr_query.argtypes = [c_void_p, P(Info)]
    lib.blr_destroy.argtypes = [c_void_p]
    lib.blr_destroy.restype = None
    lib.blr_status_string.argtypes = [c_int32]
    lib.blr_status_string.restype = ctypes.c_char_p
    lib.blr_last_error.argtypes = []
    lib.blr_last_error.restype = ctypes.c_char_p
    lib.blr_profile_enable.argtypes = [c_void_p, c_int32]
    lib.blr_profile_read.argtypes = [c_void_p, c_int32, P(c_int64), P(c_double), P(c_double)]
    lib.blr_selftest_gemm.argtypes = [c_int32, c_int32, c_int32, c_int32, c_double, c_void_p, c_int64,
                                      c_void_p, c_int64, c_double, c_void_p, c_int64, c_int32, c_void_p]
    lib.blr_selftest_gemm.restype = c_int32
    for name in EXPORTED:
        fn = getattr(lib, name)
        if name not in ("blr_destroy", "blr_status_string", "blr_last_error"):
            fn.restype = c_int32
    _lib = lib
    return lib
