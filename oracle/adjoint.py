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

Everything is dense float64 numpy; the solves use the explicit normal-matrix
solve, which is fine at the small sizes the tests use."""
from __future__ import annotations

import numpy as np

from .blrmat import BLR, DENSE


def lstsq_adjoint(A: np.ndarray, B: np.ndarray, Xbar: np.ndarray):
    """Dense adjoint: returns (X, Bbar, Abar) for X = argmin ||A X - B||
    column by column and the loss gradient Xbar = dL/dX."""
    X = np.linalg.lstsq(A, B, rcond=None)[0]
    Z = np.linalg.solve(A.T @ A, Xbar)
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
