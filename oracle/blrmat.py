"""BLR matrix construction (paper Section 3.1, eq. blr_matrix_def and the
admissibility discussion after it).

A BLR matrix has p x q tiles of size b x b; tile (i,j) is dense (fmt 0) or
U V^T (fmt 1) with U orthonormal.  When b does not divide m or n, the last
tile row or column is narrower (the rectangular blocks the paper notes the
method extends to, Section 3.1).  Readings:
* diagonal tiles (k,k), k < q, are always dense;
* a cluster box is the tight axis-aligned box of the b consecutive points of a
  tile row/column (points are Morton sorted by the caller);
* 'adjacent' rule: dense iff the Euclidean gap between the boxes is 0;
* 'dist_gt_diam' rule: low-rank iff gap > max(diam_row, diam_col), diam being
  the box diagonal;
* 'weak' rule: every off-diagonal tile is low-rank.
"""
from __future__ import annotations

import numpy as np

from . import lowrank

DENSE, LOWRANK = 0, 1


def kernel_matrix(x: np.ndarray, y: np.ndarray, kernel: str, reg: float = 1e-3):
    """A_ij = f(|x_i - y_j|): 'log2d' -> -log(d + reg), 'inv_r' -> 1/(d + reg)."""
    d = np.sqrt(np.sum((x[:, None, :] - y[None, :, :]) ** 2, axis=2))
    if kernel == "log2d":
        return -np.log(d + reg)
    if kernel == "inv_r":
        return 1.0 / (d + reg)
    raise ValueError(kernel)


def cluster_boxes(pts: np.ndarray, b: int):
    """Tight boxes of the clusters of b consecutive points (the last cluster
    holds the remaining points when b does not divide their number)."""
    starts = np.arange(0, pts.shape[0], b)
    return np.minimum.reduceat(pts, starts, axis=0), np.maximum.reduceat(pts, starts, axis=0)


def lowrank_mask(x, y, b, rule: str, p: int, q: int) -> np.ndarray:
    """p x q boolean mask, True where the tile is stored low-rank."""
    if rule == "weak":
        mask = np.ones((p, q), dtype=bool)
    else:
        rlo, rhi = cluster_boxes(x, b)
        clo, chi = cluster_boxes(y, b)
        gapv = np.maximum(0.0, np.maximum(rlo[:, None, :] - chi[None, :, :],
                                          clo[None, :, :] - rhi[:, None, :]))
        gap = np.sqrt(np.sum(gapv ** 2, axis=2))
        if rule == "adjacent":
            mask = gap > 0.0
        elif rule == "dist_gt_diam":
            dr = np.sqrt(np.sum((rhi - rlo) ** 2, axis=1))
            dc = np.sqrt(np.sum((chi - clo) ** 2, axis=1))
            mask = gap > np.maximum(dr[:, None], dc[None, :])
        else:
            raise ValueError(rule)
    for k in range(min(p, q)):
        mask[k, k] = False
    return mask


class BLR:
    """Tile storage: fmt[i,j], D[(i,j)] for dense, U/V[(i,j)] for low-rank."""

    def __init__(self, m: int, n: int, b: int):
        assert m >= n >= 1 and b >= 1
        self.m, self.n, self.b = m, n, b
        self.p, self.q = -(-m // b), -(-n // b)
        self.fmt = np.zeros((self.p, self.q), dtype=np.int8)
        self.D = {}
        self.U = {}
        self.V = {}

    def copy(self) -> "BLR":
        c = BLR(self.m, self.n, self.b)
        c.fmt = self.fmt.copy()
        c.D = {k: v.copy() for k, v in self.D.items()}
        c.U = {k: v.copy() for k, v in self.U.items()}
        c.V = {k: v.copy() for k, v in self.V.items()}
        return c

    def tile(self, i: int, j: int) -> np.ndarray:
        if self.fmt[i, j] == DENSE:
            return self.D[(i, j)]
        return self.U[(i, j)] @ self.V[(i, j)].T

    def rank(self, i: int, j: int) -> int:
        return self.U[(i, j)].shape[1] if self.fmt[i, j] == LOWRANK else -1

    def to_dense(self) -> np.ndarray:
        b = self.b
        A = np.empty((self.m, self.n))
        for i in range(self.p):
            for j in range(self.q):
                A[i * b:(i + 1) * b, j * b:(j + 1) * b] = self.tile(i, j)
        return A


def compress(A: np.ndarray, b: int, eps: float, cap: int, mask: np.ndarray,
             overflow: str = "dense") -> BLR:
    """Compress a dense m x n matrix: tiles where mask is False are stored
    dense, the others by truncated SVD (lowrank.compress_tile)."""
    m, n = A.shape
    blr = BLR(m, n, b)
    for i in range(blr.p):
        for j in range(blr.q):
            blk = A[i * b:(i + 1) * b, j * b:(j + 1) * b]
            if not mask[i, j]:
                blr.fmt[i, j] = DENSE
                blr.D[(i, j)] = blk.copy()
                continue
            res = lowrank.compress_tile(blk, eps, cap, overflow)
            if res[0] == "D":
                blr.fmt[i, j] = DENSE
                blr.D[(i, j)] = res[1]
            else:
                blr.fmt[i, j] = LOWRANK
                blr.U[(i, j)], blr.V[(i, j)] = res[1], res[2]
    return blr
