"""Householder QR of Block Low-Rank matrices on AMD MI355X (gfx950).

The compute path is libblrqr.so (hand-written HIP kernels behind a C ABI,
include/blrqr.h); this package is its Python binding.  The library is loaded
on first use and every entry point raises if it has not been built: there is
no fallback path.
"""
from ._lib import load
from .api import BLRError, BLRMatrix, LstsqFunction, factor_batch, lstsq, lstsq_batch, morton_sort

__all__ = ["BLRMatrix", "BLRError", "LstsqFunction", "factor_batch", "load", "lstsq", "lstsq_batch", "morton_sort"]
