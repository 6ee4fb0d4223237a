"""Accuracy metrics of Section 5 (Res and Orth) plus the least-squares
normal-equation residual and a sign-insensitive comparison of R factors.

Readings: Res is reported against both the original matrix A
and the compressed matrix A~; Orth uses the thin factor Q1 = Q[:, :n] of the
rectangular matrix, normalised by sqrt(n)."""
from __future__ import annotations

import numpy as np


def res(f, A: np.ndarray) -> float:
    """||Q R - A||_F / ||A||_F."""
    return float(np.linalg.norm(f.q_times_r() - A) / np.linalg.norm(A))


def orth(f) -> float:
    """||Q1^T Q1 - I||_F / sqrt(n)."""
    Q1 = f.thin_q()
    n = Q1.shape[1]
    return float(np.linalg.norm(Q1.T @ Q1 - np.eye(n)) / np.sqrt(n))


def eta_ne(A: np.ndarray, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Normal-equation residual ||A^T (b - A x)|| / (||A||_F ||b - A x||), per column."""
    r = b - A @ x
    num = np.linalg.norm(A.T @ r, axis=0)
    den = np.linalg.norm(A) * np.linalg.norm(r, axis=0)
    return num / np.where(den == 0, 1.0, den)


def sign_fix(R: np.ndarray, Rref: np.ndarray) -> np.ndarray:
    """D R with D = diag(+-1) chosen so that diag(D R) has the signs of diag(Rref)."""
    d = np.sign(np.diag(R)) * np.sign(np.diag(Rref))
    d[d == 0] = 1.0
    return d[:, None] * R


def r_rel_diff(R: np.ndarray, Rref: np.ndarray) -> float:
    """||D R - Rref||_F / ||Rref||_F (R unique up to row signs for full rank)."""
    return float(np.linalg.norm(sign_fix(R, Rref) - Rref) / np.linalg.norm(Rref))
