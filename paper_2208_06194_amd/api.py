"""Thin Python binding of libblrqr (include/blrqr.h).

Argument marshalling only: PyTorch supplies device memory and the current
HIP stream; every step of compression, factorization, Q application and the
least-squares solve runs in the library's kernels.  Matrices cross the
boundary in column-major order: an (m, ncols) torch tensor is passed as the
contiguous (ncols, m) tensor of its transpose.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


class BLRError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


def _check(st: int):
    if st != L.BLR_OK:
        lib = L.load()
        raise BLRError(st, f"{lib.blr_status_string(st).decode()}: {lib.blr_last_error().decode()}")


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _colmajor(t: torch.Tensor, copy: bool = False) -> torch.Tensor:
    """(m, k) tensor -> contiguous (k, m) tensor holding its column-major image
    (a new tensor when copy is set; otherwise it may share t's storage, which
    is fine for arguments the library only reads)."""
    if t.dim() == 1:
        t = t[:, None]
    t = t.t()
    return t.clone(memory_format=torch.contiguous_format) if copy else t.contiguous()


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


class LstsqFunction(torch.autograd.Function):
    """X = argmin ||A~ X - B|| as an autograd function.  G is a handle factored
    with keep_a; D, U, V are the tensors the stored tiles of G were built from
    ((p, q, b, b) dense blocks, (p, q, b, rc) low-rank factors): their values
    are not read again, they receive the gradients of the stored tiles.  The
    backward pass is the library's adjoint (blr_lstsq_adjoint)."""

    @staticmethod
    def forward(ctx, B, D, U, V, G):
        X = G.lstsq(B)
        ctx.G = G
        ctx.save_for_backward(B, X)
        return X

    @staticmethod
    def backward(ctx, Xbar):
        B, X = ctx.saved_tensors
        Bbar, dD, dU, dV = ctx.G.lstsq_adjoint(B, X, Xbar.contiguous())
        return Bbar, dD, dU, dV, None


def lstsq(G, B, D, U, V):
    """Differentiable least-squares solve with the factored handle G (see LstsqFunction)."""
    return LstsqFunction.apply(B, D, U, V, G)


def morton_sort(pts: torch.Tensor, stream=None):
    """Morton (Z-order) ordering of (n, dim) device points with coordinates in
    [0, 1): returns (the points in that order, the permutation as int64)."""
    lib = L.load()
    pts = pts.contiguous().to(torch.float64)
    n, dim = pts.shape
    perm = torch.empty(n, dtype=torch.int64, device=pts.device)
    out = torch.empty_like(pts)
    _check(lib.blr_morton_sort(pts.data_ptr(), n, dim, perm.data_ptr(), out.data_ptr(), _stream(stream)))
    return out, perm


def factor_batch(mats, precision: str = "fp64", stop_after_k: int = -1, keep_a: bool = False,
                 stream=None):
    """Block-column QR of several independent BLR matrices as one batch
    (blr_qr_factor_batch): the same result per matrix as mats[i].factor(
    "block_column", precision, ...), with the launches shared."""
    mats = list(mats)
    o = L.FactorOpts(variant=L.VARIANT["block_column"], precision=L.PRECISION[precision], ib=0,
                     stop_after_k=stop_after_k, keep_a=1 if keep_a else 0)
    arr = (ctypes.c_void_p * len(mats))(*[m._h.value for m in mats])
    _check(L.load().blr_qr_factor_batch(arr, len(mats), ctypes.byref(o), _stream(stream)))
    return mats


def lstsq_batch(mats, Bs, max_refine: int = 0, stream=None):
    """X_i = argmin ||A~_i X - B_i|| for factored matrices mats[i] and (m_i,
    nrhs) device tensors Bs[i], as one batch (blr_lstsq_solve_batch); the
    same result per member as mats[i].lstsq(Bs[i], max_refine=max_refine)."""
    mats, Bs = list(mats), list(Bs)
    if len(mats) != len(Bs):
        raise ValueError("one right-hand side block per matrix")
    nrhs = Bs[0].shape[1] if Bs[0].dim() == 2 else 1
    Bc, Xc = [], []
    for G, B in zip(mats, Bs):
        inf = G.info()
        b = _colmajor(B.to(torch.float64))
        if b.shape != (nrhs, inf["m"]):
            raise ValueError("every B must be (m_i, nrhs) with the same nrhs")
        Bc.append(b)
        Xc.append(torch.empty((nrhs, inf["n"]), dtype=torch.float64, device=B.device))
    k = len(mats)
    hs = (ctypes.c_void_p * k)(*[G._h.value for G in mats])
    bp = (ctypes.c_void_p * k)(*[b.data_ptr() for b in Bc])
    xp = (ctypes.c_void_p * k)(*[x.data_ptr() for x in Xc])
    lb = (ctypes.c_int64 * k)(*[G.info()["m"] for G in mats])
    lx = (ctypes.c_int64 * k)(*[G.info()["n"] for G in mats])
    _check(L.load().blr_lstsq_solve_batch(hs, k, bp, lb, xp, lx, nrhs, max_refine, _stream(stream)))
    return [x.t() for x in Xc]


class BLRMatrix:
    """A BLR matrix owned by the library (one handle)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    def __del__(self):
        try:
            if self._h and self._h.value:
                L.load().blr_destroy(self._h)
                self._h = ctypes.c_void_p(0)
        except Exception:
            pass

    # construction ------------------------------------------------------------
    @staticmethod
    def _opts(m, n, tile, tol, max_rank, overflow, seed):
        return L.CompressOpts(m=m, n=n, tile=tile, tol=tol, max_rank=max_rank,
                              overflow=L.OVERFLOW[overflow], seed=seed)

    @classmethod
    def compress_kernel(cls, x: torch.Tensor, y: torch.Tensor, kernel: str, tile: int, tol: float,
                        max_rank: int, admissibility: str = "dist_gt_diam", overflow: str = "dense",
                        reg: float = 1e-3, seed: int = 0, mask: np.ndarray | None = None, stream=None):
        """Compress A_ij = f(|x_i - y_j|) given row/column points on the device."""
        lib = L.load()
        x = x.contiguous().to(torch.float64)
        y = y.contiguous().to(torch.float64)
        m, dim = x.shape
        n = y.shape[0]
        maskc = None if mask is None else np.ascontiguousarray(mask.astype(np.int8))
        src = L.Source(kind=L.SRC_KERNEL, x=x.data_ptr(), y=y.data_ptr(), dim=dim,
                       kernel={"log2d": L.KERNEL_LOG2D, "inv_r": L.KERNEL_INV_R}[kernel], reg=reg,
                       A=None, lda=0, admissibility=L.ADM[admissibility], mask=_ptr(maskc))
        o = cls._opts(m, n, tile, tol, max_rank, overflow, seed)
        h = ctypes.c_void_p()
        _check(lib.blr_compress(ctypes.byref(src), ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def compress_dense(cls, A: torch.Tensor, tile: int, tol: float, max_rank: int,
                       admissibility: str = "weak", mask: np.ndarray | None = None,
                       overflow: str = "dense", seed: int = 0, stream=None):
        """Compress a dense (m, n) device matrix (admissibility 'weak' or 'mask')."""
        lib = L.load()
        m, n = A.shape
        Ac = _colmajor(A.to(torch.float64))
        maskc = None if mask is None else np.ascontiguousarray(mask.astype(np.int8))
        src = L.Source(kind=L.SRC_DENSE, x=None, y=None, dim=0, kernel=0, reg=0.0,
                       A=Ac.data_ptr(), lda=m, admissibility=L.ADM[admissibility], mask=_ptr(maskc))
        o = cls._opts(m, n, tile, tol, max_rank, overflow, seed)
        h = ctypes.c_void_p()
        _check(lib.blr_compress(ctypes.byref(src), ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def import_tiles(cls, m, n, tile, tol, max_rank, fmt, rank, dense, U, V, stream=None):
        """Build from host tiles (layout of blr_tiles_host; U and V are b x rc per tile)."""
        lib = L.load()
        keep = [np.ascontiguousarray(fmt, dtype=np.int8), np.ascontiguousarray(rank, dtype=np.int32),
                np.ascontiguousarray(dense, dtype=np.float64), np.ascontiguousarray(U, dtype=np.float64),
                np.ascontiguousarray(V, dtype=np.float64)]
        t = L.TilesHost(fmt=_ptr(keep[0]), rank=_ptr(keep[1]), dense=_ptr(keep[2]), U=_ptr(keep[3]),
                        V=_ptr(keep[4]), Y=None, T=None)
        o = cls._opts(m, n, tile, tol, max_rank, "dense", 0)
        h = ctypes.c_void_p()
        _check(lib.blr_import(ctypes.byref(o), ctypes.byref(t), _stream(stream), ctypes.byref(h)))
        return cls(h.value)

    # queries -------------------------------------------------------------------
    def info(self) -> dict:
        inf = L.Info()
        _check(L.load().blr_query(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in L.Info._fields_}

    def export(self, with_factor: bool = False) -> dict:
        inf = self.info()
        p, q, b, rc = inf["p"], inf["q"], inf["tile"], inf["rank_capacity"]
        nt = p * q
        out = {
            "fmt": np.zeros(nt, np.int8), "rank": np.zeros(nt, np.int32),
            "dense": np.zeros(nt * b * b), "U": np.zeros(nt * b * rc), "V": np.zeros(nt * b * rc),
        }
        if with_factor:
            out["Y"] = np.zeros(nt * rc * b)
            out["T"] = np.zeros(nt * b * b)
        t = L.TilesHost(fmt=_ptr(out["fmt"]), rank=_ptr(out["rank"]), dense=_ptr(out["dense"]),
                        U=_ptr(out["U"]), V=_ptr(out["V"]), Y=_ptr(out.get("Y")), T=_ptr(out.get("T")))
        _check(L.load().blr_export(self._h, ctypes.byref(t)))
        shaped = {
            "fmt": out["fmt"].reshape(p, q), "rank": out["rank"].reshape(p, q),
            # tile (i,j): column-major b x b -> stored transposed in C order
            "dense": out["dense"].reshape(p, q, b, b).transpose(0, 1, 3, 2),
            "U": out["U"].reshape(p, q, rc, b).transpose(0, 1, 3, 2),
            "V": out["V"].reshape(p, q, rc, b).transpose(0, 1, 3, 2),
        }
        if with_factor:
            shaped["Y"] = out["Y"].reshape(p, q, b, rc).transpose(0, 1, 3, 2)
            shaped["T"] = out["T"].reshape(p, q, b, b).transpose(0, 1, 3, 2)
        shaped["info"] = inf
        return shaped

    # the hot path ----------------------------------------------------------------
    def factor(self, variant: str = "tiled", precision: str = "fp64", stop_after_k: int = -1,
               ib: int = 0, keep_a: bool = False, stream=None):
        o = L.FactorOpts(variant=L.VARIANT[variant], precision=L.PRECISION[precision], ib=ib,
                         stop_after_k=stop_after_k, keep_a=1 if keep_a else 0)
        _check(L.load().blr_qr_factor(self._h, ctypes.byref(o), _stream(stream)))
        return self

    def matmul(self, X: torch.Tensor, op: str = "A", stream=None) -> torch.Tensor:
        """A~ X (op "A", before the factorization), A~^T X ("AT") or R X ("R",
        after it) for a device tensor X with one column per right-hand side."""
        inf = self.info()
        m, n = inf["m"], inf["n"]
        Xc = _colmajor(X.to(torch.float64))
        nrhs, xr = Xc.shape
        yr = m if op == "A" else n
        Yc = torch.empty((nrhs, yr), dtype=torch.float64, device=Xc.device)
        _check(L.load().blr_matmul(self._h, L.MATMUL[op], Xc.data_ptr(), xr, Yc.data_ptr(), yr, nrhs,
                                   _stream(stream)))
        return Yc.t()

    def apply_qt(self, B: torch.Tensor, trans: bool = False, stream=None) -> torch.Tensor:
        """Return Q^T B (trans=False) or Q B (trans=True) for a (m, nrhs) device tensor."""
        Bc = _colmajor(B.to(torch.float64), copy=True)   # overwritten in place by the library
        nrhs, m = Bc.shape
        _check(L.load().blr_apply_qt(self._h, 1 if trans else 0, Bc.data_ptr(), m, nrhs, _stream(stream)))
        return Bc.t()

    def apply_qt_noalloc(self, B: torch.Tensor, trans: bool = False, stream=None) -> torch.Tensor:
        """apply_qt through blr_apply_qt_noalloc (no device allocation inside the
        library; its temporaries live in the per-GPU static scratch)."""
        Bc = _colmajor(B.to(torch.float64), copy=True)   # overwritten in place by the library
        nrhs, m = Bc.shape
        _check(L.load().blr_apply_qt_noalloc(self._h, 1 if trans else 0, Bc.data_ptr(), m, nrhs, _stream(stream)))
        return Bc.t()

    def lstsq(self, B: torch.Tensor, with_resid: bool = False, max_refine: int = 0, stream=None):
        """X = argmin ||A X - B||_F for a (m, nrhs) device tensor; returns (n, nrhs).
        max_refine > 0 refines with FP64 residuals (the factor must keep A~)."""
        inf = self.info()
        m, n = inf["m"], inf["n"]
        Bc = _colmajor(B.to(torch.float64))
        nrhs = Bc.shape[0]
        Xc = torch.empty((nrhs, n), dtype=torch.float64, device=B.device)
        res = torch.empty(nrhs, dtype=torch.float64, device=B.device) if with_resid else None
        _check(L.load().blr_lstsq_solve(self._h, Bc.data_ptr(), m, Xc.data_ptr(), n, nrhs, max_refine,
                                        None if res is None else res.data_ptr(), _stream(stream)))
        X = Xc.t()
        return (X, torch.sqrt(res)) if with_resid else X

    def mgs_qr(self, stream=None) -> "BLRMatrix":
        """Blocked modified Gram-Schmidt QR (the comparison method): this
        handle becomes the explicit Q~; returns R~ as a new n x n handle."""
        h = ctypes.c_void_p()
        _check(L.load().blr_mgs_qr(self._h, _stream(stream), ctypes.byref(h)))
        return BLRMatrix(h.value)

    def form_q(self, stream=None) -> "BLRMatrix":
        """The explicit orthogonal factor Q~ (m x n) as a new BLR matrix with the
        structure, tolerance and rank cap of A~."""
        h = ctypes.c_void_p()
        _check(L.load().blr_form_q(self._h, _stream(stream), ctypes.byref(h)))
        return BLRMatrix(h.value)

    def rsolve(self, X: torch.Tensor, trans: bool = False, stream=None) -> torch.Tensor:
        """R^{-1} X (trans=False) or R^{-T} X (trans=True) for an (n, nrhs) device tensor."""
        Xc = _colmajor(X.to(torch.float64), copy=True)   # overwritten in place by the library
        nrhs, n = Xc.shape
        _check(L.load().blr_rsolve(self._h, 1 if trans else 0, Xc.data_ptr(), n, nrhs, _stream(stream)))
        return Xc.t()

    def lstsq_adjoint(self, B: torch.Tensor, X: torch.Tensor, Xbar: torch.Tensor, stream=None):
        """Gradients of a loss L(X) through X = argmin ||A~ X - B|| (the factor
        must keep A~): returns (dL/dB, dL/dD, dL/dU, dL/dV).  dL/dD is (p, q, b, b)
        with tile (i, j) holding dL/dA~ restricted to that tile (dense tiles
        only; zero elsewhere); dL/dU and dL/dV are (p, q, b, rc) for the factors
        U, V (b x rc) of the low-rank tiles (zero elsewhere)."""
        inf = self.info()
        m, n, p, q, b, rc = inf["m"], inf["n"], inf["p"], inf["q"], inf["tile"], inf["rank_capacity"]
        Bc, Xc, Xbc = _colmajor(B.to(torch.float64)), _colmajor(X.to(torch.float64)), _colmajor(Xbar.to(torch.float64))
        nrhs = Bc.shape[0]
        dev = Bc.device
        Bbar = torch.empty((nrhs, m), dtype=torch.float64, device=dev)
        dD = torch.zeros((p, q, b, b), dtype=torch.float64, device=dev)     # per tile column-major: [i, j, col, row]
        dU = torch.zeros((p, q, rc, b), dtype=torch.float64, device=dev)
        dV = torch.zeros((p, q, rc, b), dtype=torch.float64, device=dev)
        _check(L.load().blr_lstsq_adjoint(self._h, Bc.data_ptr(), m, Xc.data_ptr(), n, Xbc.data_ptr(), n, nrhs,
                                          Bbar.data_ptr(), m, dD.data_ptr(), dU.data_ptr(), dV.data_ptr(),
                                          _stream(stream)))
        return Bbar.t(), dD.transpose(-1, -2), dU.transpose(-1, -2), dV.transpose(-1, -2)

    def profile(self, on: bool = True):
        _check(L.load().blr_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, kernel: str = "fp64"):
        """(launches, total ms, total flops) of the dominant kernel with FP64
        ("fp64") or FP32 ("fp32") operands in the last profiled factor."""
        n, ms, fl = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        _check(L.load().blr_profile_read(self._h, 0 if kernel == "fp64" else 1, ctypes.byref(n),
                                         ctypes.byref(ms), ctypes.byref(fl)))
        return n.value, ms.value, fl.value
