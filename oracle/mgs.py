"""Blocked modified Gram-Schmidt QR of a BLR matrix: the method the paper
compares its Householder algorithms with (Section 2.1, Alg. 1 "Blocked
Modified Gram-Schmidt"; Section 3.2 for BLR matrices).  TEST
INFRASTRUCTURE: a plain FP64 numpy implementation that follows the steps in
the paper's order, independent of the HIP path.

Step j (block columns j = 0, 1, ...):
  1. Orthogonalize block column j.  Every tile of the column is written in
     left-orthogonal form A_ij = A^U_ij A^V_ij (dense: I times the tile;
     low-rank U V^T: U times V^T), the right factors are stacked,
     B_j = [A^V_0j; A^V_1j; ...; A^V_{p-1}j], and a dense modified
     Gram-Schmidt QR gives B_j = Q^B_j R^B_j.  The block column's orthogonal
     factor is Q_ij = A^U_ij Q^B_ij (a low-rank tile keeps its U, with the
     rows of Q^B as its right factor) and R_jj = R^B_j (eq. blr_mbgs_qj).
  2. For every k > j: R_jk = Q_j^T A_k = sum_i Q_ij^T A_ik and
     A_ik <- A_ik - Q_ij R_jk in BLR arithmetic: the sum is dense if any term
     is dense, else low-rank terms added by rounded additions (Alg. 6) in a
     chain in the order of the sum; the update follows the same rules, so a
     low-rank tile receiving a dense update becomes dense (fill-in).

Readings: unlike the Householder block-column algorithm, the stack of step
j holds every block row (Gram-Schmidt subtracts projections, it annihilates
nothing), and Q~ is formed explicitly in place of A~ (same tile structure,
with fill-in) while R~ is kept apart.  The dense MGS is the column-by-column
textbook form: r_cc = ||a_c||, q_c = a_c / r_cc, then every later column
loses its component along q_c.  Full column rank is assumed (r_cc > 0).
"""
from __future__ import annotations

import numpy as np

from . import blrops, lowrank
from .blrmat import BLR, DENSE, LOWRANK


def mgs(B: np.ndarray):
    """Modified Gram-Schmidt QR of a dense h x w matrix (h >= w):
    returns (Q, R), Q h x w with (nearly) orthonormal columns, R upper
    triangular with a positive diagonal."""
    A = np.array(B, dtype=np.float64, copy=True)
    h, w = A.shape
    Q = np.zeros((h, w))
    R = np.zeros((w, w))
    for c in range(w):
        R[c, c] = np.linalg.norm(A[:, c])
        Q[:, c] = A[:, c] / R[c, c]
        # every later column loses its component along q_c, taken from the
        # column as updated so far (the "modified" form)
        R[c, c + 1:] = Q[:, c] @ A[:, c + 1:]
        A[:, c + 1:] -= np.outer(Q[:, c], R[c, c + 1:])
    return Q, R


class MGSFactor:
    """Q~ (in place of the tiles of A~) and R~ (tiles (j, k), j <= k)."""

    def __init__(self, blr: BLR, eps: float, cap: int):
        self.A = blr
        self.eps, self.cap = eps, cap
        self.b, self.p, self.q = blr.b, blr.p, blr.q
        self.stats = lowrank.Stats()
        self.R = {}
        self.Qv = {}         # (i, j) low-rank tiles of Q~: the rows of Q^B_j (r x w)

    def val(self, i, j):
        A = self.A
        if A.fmt[i, j] == DENSE:
            return ("D", A.D[(i, j)])
        return ("L", A.U[(i, j)], A.V[(i, j)])

    def store(self, i, j, X):
        A = self.A
        if X[0] == "D":
            A.fmt[i, j] = DENSE
            A.D[(i, j)] = X[1]
            A.U.pop((i, j), None)
            A.V.pop((i, j), None)
        else:
            A.fmt[i, j] = LOWRANK
            A.U[(i, j)], A.V[(i, j)] = X[1], X[2]
            A.D.pop((i, j), None)

    def qrep(self, i, j):
        """Q_ij as a reflector-like block: ('D', Q) or ('L', U, Ql) = U Ql."""
        if self.A.fmt[i, j] == DENSE:
            return ("D", self.A.D[(i, j)])
        return ("L", self.A.U[(i, j)], self.Qv[(i, j)])

    def orthogonalize(self, j):
        A = self.A
        parts = [A.D[(i, j)] if A.fmt[i, j] == DENSE else A.V[(i, j)].T for i in range(self.p)]
        Q, R = mgs(np.concatenate(parts, axis=0))
        self.R[(j, j)] = ("D", R)
        off = 0
        for i in range(self.p):
            h = parts[i].shape[0]
            if A.fmt[i, j] == DENSE:
                A.D[(i, j)] = Q[off:off + h].copy()
            else:
                self.Qv[(i, j)] = Q[off:off + h].copy()
                A.V[(i, j)] = self.Qv[(i, j)].T.copy()     # Q_ij = U (Q^B_ij) as a U V^T tile
            off += h

    def project(self, j, k):
        e, c, st = self.eps, self.cap, self.stats
        terms = [blrops.yt_times(self.qrep(i, j), self.val(i, k)) for i in range(self.p)]
        if any(t[0] == "D" for t in terms):
            Rjk = ("D", sum(blrops.dense_of(t) for t in terms))
        else:
            Rjk = terms[0]
            for t in terms[1:]:
                Rjk = blrops.add(Rjk, t, 1.0, e, c, st)
        self.R[(j, k)] = Rjk
        for i in range(self.p):
            upd = blrops.y_times(self.qrep(i, j), Rjk)
            self.store(i, k, blrops.add(self.val(i, k), upd, -1.0, e, c, st))

    def run(self):
        for j in range(self.q):
            self.orthogonalize(j)
            for k in range(j + 1, self.q):
                self.project(j, k)
        return self

    # what is read off the result ------------------------------------------
    def q_dense(self) -> np.ndarray:
        """The explicit m x n orthogonal factor Q~."""
        return self.A.to_dense()

    def r_dense(self) -> np.ndarray:
        b, q = self.b, self.q
        n = self.A.n
        R = np.zeros((q * b, q * b))
        for (j, k), X in self.R.items():
            blk = blrops.dense_of(X)
            R[j * b:j * b + blk.shape[0], k * b:k * b + blk.shape[1]] = blk
        return R[:n, :n]

    def orth(self) -> float:
        """||Q~^T Q~ - I||_F / sqrt(n), Section 5's Orth."""
        Q = self.q_dense()
        n = Q.shape[1]
        return float(np.linalg.norm(Q.T @ Q - np.eye(n)) / np.sqrt(n))

    def res(self, A: np.ndarray) -> float:
        """||Q~ R~ - A||_F / ||A||_F."""
        return float(np.linalg.norm(self.q_dense() @ self.r_dense() - A) / np.linalg.norm(A))


def factor(blr: BLR, eps: float, cap: int, copy: bool = True) -> MGSFactor:
    f = MGSFactor(blr.copy() if copy else blr, eps, cap)
    return f.run()
