"""The C-ABI library loads and exports every function declared in include/*.h
(no compute calls: runs without a GPU)."""
import ctypes
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names.update(re.findall(r"\b(blr_[a-z0-9_]+)\s*\(", text))
    return names


def test_headers_declare_the_boundary():
    names = declared_functions()
    for fn in ["blr_compress", "blr_qr_factor", "blr_apply_qt", "blr_lstsq_solve", "blr_import",
               "blr_export", "blr_query", "blr_destroy", "blr_status_string", "blr_last_error",
               "blr_qr_factor_batch", "blr_lstsq_solve_batch", "blr_rsolve", "blr_lstsq_adjoint",
               "blr_form_q", "blr_morton_sort", "blr_matmul"]:
        assert fn in names
    # the binding declares exactly the header's entry points
    from paper_2208_06194_amd import _lib
    assert set(_lib.EXPORTED) | set(_lib.SELFTEST) == names


def test_library_exports_every_declared_symbol():
    from paper_2208_06194_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2208_06194_amd import build
        build.build()
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in sorted(declared_functions()):
        assert hasattr(lib, name), name
    # status strings need no device
    lib.blr_status_string.restype = ctypes.c_char_p
    assert lib.blr_status_string(0) == b"ok"
    assert lib.blr_status_string(6) == b"singular R"


def test_invalid_arguments_are_rejected_without_a_device():
    from paper_2208_06194_amd import _lib as L
    lib = L.load()
    h = ctypes.c_void_p()
    # m < n, tile not dividing m, bad tolerance, bad rank cap
    for m, n, tile, tol, cap in [(64, 128, 32, 1e-8, 8), (64, 32, 32, 0.0, 8),
                                 (64, 32, 32, 1e-8, 0), (64, 32, 24, 1e-8, 8), (64, 32, 32, 1e-8, 200)]:
        o = L.CompressOpts(m=m, n=n, tile=tile, tol=tol, max_rank=cap, overflow=0, seed=0)
        src = L.Source(kind=L.SRC_DENSE, A=ctypes.c_void_p(8), lda=m, admissibility=L.ADM["weak"])
        assert lib.blr_compress(ctypes.byref(src), ctypes.byref(o), None, ctypes.byref(h)) == L.BLR_ERR_INVALID
    assert lib.blr_qr_factor(None, None, None) == L.BLR_ERR_INVALID
    assert lib.blr_last_error() != b""


def test_morton_sort_rejects_bad_arguments_without_a_device():
    from paper_2208_06194_amd import _lib as L
    lib = L.load()
    p = ctypes.c_void_p(8)
    assert lib.blr_morton_sort(None, 4, 2, p, None, None) == L.BLR_ERR_INVALID
    assert lib.blr_morton_sort(p, 4, 2, None, None, None) == L.BLR_ERR_INVALID
    assert lib.blr_morton_sort(p, -1, 2, p, None, None) == L.BLR_ERR_INVALID
    assert lib.blr_morton_sort(p, 4, 4, p, None, None) == L.BLR_ERR_INVALID
    assert lib.blr_morton_sort(p, 4, 0, p, None, None) == L.BLR_ERR_INVALID


def test_batched_factor_rejects_bad_arguments_without_a_device():
    from paper_2208_06194_amd import _lib as L
    lib = L.load()
    bc = L.FactorOpts(variant=L.VARIANT["block_column"], precision=L.PRECISION["fp64"], ib=0,
                      stop_after_k=-1, keep_a=0)
    tiled = L.FactorOpts(variant=L.VARIANT["tiled"], precision=L.PRECISION["fp64"], ib=0,
                         stop_after_k=-1, keep_a=0)
    none2 = (ctypes.c_void_p * 2)(None, None)
    assert lib.blr_qr_factor_batch(None, 1, ctypes.byref(bc), None) == L.BLR_ERR_INVALID
    assert lib.blr_qr_factor_batch(none2, 0, ctypes.byref(bc), None) == L.BLR_ERR_INVALID
    assert lib.blr_qr_factor_batch(none2, 2, None, None) == L.BLR_ERR_INVALID
    assert lib.blr_qr_factor_batch(none2, 2, ctypes.byref(tiled), None) == L.BLR_ERR_INVALID
    assert b"block-column" in lib.blr_last_error()
    assert lib.blr_qr_factor_batch(none2, 2, ctypes.byref(bc), None) == L.BLR_ERR_INVALID
    assert b"NULL handle" in lib.blr_last_error()


def test_batched_solve_rejects_bad_arguments_without_a_device():
    from paper_2208_06194_amd import _lib as L
    lib = L.load()
    none1 = (ctypes.c_void_p * 1)(None)
    ld = (ctypes.c_int64 * 1)(8)
    assert lib.blr_lstsq_solve_batch(None, 1, none1, ld, none1, ld, 1, 0, None) == L.BLR_ERR_INVALID
    assert lib.blr_lstsq_solve_batch(none1, 0, none1, ld, none1, ld, 1, 0, None) == L.BLR_ERR_INVALID
    assert lib.blr_lstsq_solve_batch(none1, 1, none1, ld, none1, ld, -1, 0, None) == L.BLR_ERR_INVALID
    assert lib.blr_lstsq_solve_batch(none1, 1, none1, ld, none1, ld, 1, 0, None) == L.BLR_ERR_INVALID
    assert b"NULL" in lib.blr_last_error()
