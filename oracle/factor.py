"""Common state of a factored BLR matrix (both variants) and what is read
off it: the BLR factor R (paper eq. qr_fact with Section 3.3/3.4: R has the
same tile structure as A), the reflector blocks Ytilde_ik, and the BLR
back-substitution used for least squares (the motivation in Section 1)."""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import blrops, dense, lowrank
from .blrmat import BLR, DENSE, LOWRANK


class SingularR(Exception):
    pass


class Factor:
    def __init__(self, blr: BLR, eps: float, cap: int):
        self.A = blr            # modified in place into R (k <= j) and Y (i > k)
        self.eps, self.cap = eps, cap
        self.b, self.p, self.q = blr.b, blr.p, blr.q
        self.stats = lowrank.Stats()
        self.Ykk = {}           # explicit unit-lower Y of diagonal tile k
        self.Yl = {}            # (i,k) -> r x b reflector rows of a low-rank tile
        self.Yfmt = {}          # (i,k) -> DENSE / LOWRANK, format of Ytilde_ik
        self.steps_done = 0

    # tile values -----------------------------------------------------------
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

    def ytilde(self, i, k):
        if self.Yfmt[(i, k)] == DENSE:
            return ("D", self.A.D[(i, k)])
        return ("L", self.A.U[(i, k)], self.Yl[(i, k)])

    # R ---------------------------------------------------------------------
    def r_val(self, k, j):
        if k == j:
            return ("D", np.triu(self.A.D[(k, k)]))
        return self.val(k, j)

    def r_dense(self) -> np.ndarray:
        """The n x n factor R; block row k holds the first (width of block
        column k) rows of the tiles R_kj."""
        b, q, n = self.b, self.q, self.A.n
        R = np.zeros((n, n))
        for k in range(q):
            rk = min(b, n - k * b)
            for j in range(k, q):
                R[k * b:k * b + rk, j * b:(j + 1) * b] = blrops.dense_of(self.r_val(k, j))[:rk]
        return R

    def r_frob(self) -> float:
        return float(np.linalg.norm(self.r_dense()))

    def backsolve(self, C: np.ndarray) -> np.ndarray:
        """X = R^{-1} C by tile back-substitution; C is n x nrhs."""
        b, q = self.b, self.q
        X = np.zeros_like(C)
        for k in range(q - 1, -1, -1):
            y = C[k * b:(k + 1) * b].copy()
            rk = y.shape[0]
            for j in range(k + 1, q):
                Rv = self.r_val(k, j)
                xj = X[j * b:(j + 1) * b]
                y -= (Rv[1] @ xj if Rv[0] == "D" else Rv[1] @ (Rv[2].T @ xj))[:rk]
            X[k * b:(k + 1) * b] = scipy.linalg.solve_triangular(
                np.triu(self.A.D[(k, k)])[:rk], y, lower=False)
        return X

    def check_singular(self):
        """Reading: R is numerically singular when some |R_jj| <= n u ||R||_F."""
        n = self.A.n
        thr = n * np.finfo(np.float64).eps * self.r_frob()
        for k in range(self.q):
            d = np.abs(np.diag(self.A.D[(k, k)]))
            if np.any(d <= thr):
                raise SingularR(k)

    def lstsq(self, B: np.ndarray) -> np.ndarray:
        """argmin ||A x - b|| per column: x = R^{-1} (Q^T b)[:n]."""
        self.check_singular()
        C = self.apply_qt(B)
        return self.backsolve(C[: self.A.n])

    # metrics ---------------------------------------------------------------
    def q_times_r(self) -> np.ndarray:
        m, n = self.A.m, self.A.n
        RR = np.zeros((m, n))
        RR[:n] = self.r_dense()
        return self.apply_q(RR)

    def thin_q(self) -> np.ndarray:
        m, n = self.A.m, self.A.n
        E = np.zeros((m, n))
        E[:n] = np.eye(n)
        return self.apply_q(E)
