"""Block-column-wise Householder BLR-QR (paper Alg. 2 with the operations of
Section 3.3) and left multiplication by Q / Q^T (Alg. 3).

Step k:
  1. stack the left-orthogonal row factors of block column k,
     [A_kk; Av_{k+1,k}; ...; Av_{p,k}] with Av = A (dense) or V^T (low-rank),
     and take its Householder QR: R_kk, Y_k = [Y_kk; Y_{k+1,k}; ...], T_k
     (eq. blr_bch_col_qr); Ytilde_ik = Au_ik Y_ik (I or U_ik);
  2. for every j > k: Z_j = sum_i Ytilde_ik^T A_ij, W_j = T_k^T Z_j,
     A_ij -= Ytilde_ik W_j (eq. blr_bch_apply_bc_reflector).  Reading of the
     accumulation: if any term is dense the sum is dense (OP1) and all terms
     are added exactly; otherwise the low-rank terms are accumulated by
     rounded additions of two terms at a time (OP2, Alg. 6).  Section 3.1
     fixes that every addition of two low-rank terms is recompressed, not the
     order of the sum; the plain reading, and the default here, is the chain
     in the order of the sum, i = k, k+1, ...: Z <- round(Z + term_i).
     zsum="tree" instead adds the same terms in a pairwise tree (the terms are
     the leaves, each level adds neighbouring pairs, the left one first in the
     stack, an odd one out passes to the next level unchanged); both are
     legal orders of the same rounded additions.
"""
from __future__ import annotations

import numpy as np

from . import blrops, dense
from .blrmat import BLR, DENSE, LOWRANK
from .factor import Factor


def chain_sum(terms, add):
    """Sum terms[0] + terms[1] + ... left to right, one rounded addition per
    term: Z = add(...add(add(terms[0], terms[1]), terms[2])...)."""
    terms = list(terms)
    z = terms[0]
    for t in terms[1:]:
        z = add(z, t)
    return z


def pairwise_sum(terms, add):
    """Sum terms[0] + terms[1] + ... two at a time in a pairwise tree: at
    stride s = 1, 2, 4, ... term x (x a multiple of 2s) absorbs term x + s."""
    terms = list(terms)
    n = len(terms)
    s = 1
    while s < n:
        for x in range(0, n - s, 2 * s):
            terms[x] = add(terms[x], terms[x + s])
        s *= 2
    return terms[0]


class BlockColumnFactor(Factor):
    def __init__(self, blr: BLR, eps: float, cap: int, zsum: str = "chain"):
        super().__init__(blr, eps, cap)
        if zsum not in ("chain", "tree"):
            raise ValueError("zsum must be 'chain' or 'tree'")
        self.zsum = chain_sum if zsum == "chain" else pairwise_sum
        self.Tk = {}

    def yrep(self, i, k):
        if i == k:
            return ("D", self.Ykk[k])
        return self.ytilde(i, k)

    def panel(self, k):
        A = self.A
        parts = [A.D[(k, k)]]
        for i in range(k + 1, self.p):
            parts.append(A.D[(i, k)] if A.fmt[i, k] == DENSE else A.V[(i, k)].T)
        F, tau, T = dense.householder_qr(np.concatenate(parts, axis=0))
        Y = dense.unit_lower(F)
        h0 = parts[0].shape[0]
        A.D[(k, k)] = F[:h0].copy()
        self.Ykk[k] = Y[:h0].copy()
        self.Tk[k] = T
        off = h0
        for i in range(k + 1, self.p):
            h = parts[i - k].shape[0]
            Yi = Y[off:off + h].copy()
            off += h
            if A.fmt[i, k] == DENSE:
                A.D[(i, k)] = Yi
                self.Yfmt[(i, k)] = DENSE
            else:
                self.Yl[(i, k)] = Yi
                A.V.pop((i, k))
                self.Yfmt[(i, k)] = LOWRANK

    def apply_column(self, k, j):
        e, c, st = self.eps, self.cap, self.stats
        terms = [blrops.yt_times(self.yrep(i, k), self.val(i, j)) for i in range(k, self.p)]
        if any(t[0] == "D" for t in terms):
            Z = ("D", sum(blrops.dense_of(t) for t in terms))
        else:
            Z = self.zsum(terms, lambda a, t: blrops.add(a, t, 1.0, e, c, st))
        W = blrops.t_times(self.Tk[k], Z, True)
        for i in range(k, self.p):
            upd = blrops.y_times(self.yrep(i, k), W)
            self.store(i, j, blrops.add(self.val(i, j), upd, -1.0, e, c, st))

    def run(self, stop_after_k=None):
        kend = self.q if stop_after_k is None else min(self.q, stop_after_k)
        for k in range(kend):
            self.panel(k)
            for j in range(k + 1, self.q):
                self.apply_column(k, j)
        self.steps_done = kend
        return self

    def _apply(self, B, k, transpose):
        b = self.b
        W = np.zeros((self.Tk[k].shape[0], B.shape[1]))
        for i in range(k, self.p):
            Yr = self.yrep(i, k)
            Bi = B[i * b:(i + 1) * b]
            W += Yr[1].T @ Bi if Yr[0] == "D" else Yr[2].T @ (Yr[1].T @ Bi)
        W = (self.Tk[k].T if transpose else self.Tk[k]) @ W
        for i in range(k, self.p):
            B[i * b:(i + 1) * b] -= blrops.dense_of(blrops.y_times(self.yrep(i, k), ("D", W)))

    def apply_qt(self, B: np.ndarray) -> np.ndarray:
        B = np.array(B, dtype=np.float64, copy=True)
        for k in range(self.steps_done):
            self._apply(B, k, True)
        return B

    def apply_q(self, B: np.ndarray) -> np.ndarray:
        B = np.array(B, dtype=np.float64, copy=True)
        for k in range(self.steps_done - 1, -1, -1):
            self._apply(B, k, False)
        return B


def factor(blr: BLR, eps: float, cap: int, stop_after_k=None,
           copy: bool = True, zsum: str = "chain") -> BlockColumnFactor:
    f = BlockColumnFactor(blr.copy() if copy else blr, eps, cap, zsum)
    return f.run(stop_after_k)
