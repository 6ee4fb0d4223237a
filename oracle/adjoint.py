"""Adjoint of the least-squares solve x = argmin ||A x - b||_2 (the use of the
QR factorization that motivates the paper, Section 1).  TEST INFRASTRUCTURE.

Not in the paper: the standard adjoint of a full-column-rank least-squares
solution.  For a scalar loss L(x) with xbar = dL/dx, and with
A^T A = R^T R from the factorization,

    z    = (A^T A)^{-1} xbar = R^{-1} R^{-T} xbar
    r    = b - A x
    bbar = dL/db = A z
    Abar = dL/dA = r z^T - bbar x^T

(x = (A^T A)^{-1} A^T b: differentiating the normal equations gives
A^T A dx = dA^T r - A^T dA x, so <xbar, dx> = <z, dA^T r> - <A z, dA x>).
For a BLR matrix the gradient is restricted to the stored tiles: a dense tile
(i, j) gets Abar_ij; a low-rank tile U V^T gets dL/dU = Abar_ij V and
dL/dV = Abar_ij^T U (the chain rule through A_ij = U V^T).

Everything is dense float64 numpy.  solve="normal" takes z from the normal
matrix A^T A (fine for small, well-conditioned inputs); solve="qr" takes x
and z from a dense Householder QR of A (LAPACK), z = R^{-1} (R^{-T} xbar),
whose error grows with kappa(A)^2 u instead of through the squared matrix
being formed (the reference gradient at larger sizes)."""
from __future__ import annotations

import numpy as np

from .blrmat import BLR, DENSE


def lstsq_adjoint(A: np.ndarray, B: np.ndarray, Xbar: np.ndarray, solve: str = "normal"):
    """Dense adjoint: returns (X, Bbar, Abar) for X = argmin ||A X - B||
    column by column and the loss gradient Xbar = dL/dX."""
    if solve == "qr":
        import scipy.linalg as sl
        Q, R = np.linalg.qr(A)
        X = sl.solve_triangular(R, Q.T @ B)
        Z = sl.solve_triangular(R, sl.solve_triangular(R, Xbar, trans="T"))
    elif solve == "normal":
        X = np.linalg.lstsq(A, B, rcond=None)[0]
        Z = np.linalg.solve(A.T @ A, Xbar)
    else:
        raise ValueError(solve)
    Rs = B - A @ X
    Bbar = A @ Z
    Abar = Rs @ Z.T - Bbar @ X.T
    return X, Bbar, Abar


def tile_gradients(blr: BLR, Abar: np.ndarray):
    """Restrict Abar to the stored tiles of blr: {(i, j): ('D', dD)} for dense
    tiles and {(i, j): ('L', dU, dV)} for low-rank tiles, dU = Abar_ij V and
    dV = Abar_ij^T U."""
    b = blr.b
    out = {}
    for i in range(blr.p):
        for j in range(blr.q):
            G = Abar[i * b:(i + 1) * b, j * b:(j + 1) * b]
            if blr.fmt[i, j] == DENSE:
                out[(i, j)] = ("D", G.copy())
            else:
                out[(i, j)] = ("L", G @ blr.V[(i, j)], G.T @ blr.U[(i, j)])
    return out
