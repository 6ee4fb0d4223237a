"""Low-rank arithmetic: epsilon-rank truncation, tile compression and the
rounded low-rank addition (paper Section 3.1, Alg. 6 "Rounded Low-Rank
Addition", and the compression rule stated with eq. blr_matrix_def).

Readings:
* Truncation rank r_eps is the smallest r with
      sqrt(sum_{l >= r} sigma_l^2) <= eps * sqrt(sum_l sigma_l^2),
  i.e. relative to the Frobenius norm of the matrix being (re)compressed
  (ties keep the smaller rank; a zero matrix has rank 0).
* Rank cap: when r_eps exceeds the cap, compression either keeps the tile
  dense (overflow='dense') or truncates to the cap (overflow='truncate').
  Inside the factorization the cap always truncates and the event is counted
  together with the largest dropped relative tail.
"""
from __future__ import annotations

import numpy as np


class Stats:
    """Counters shared by one factorization: truncations at the cap."""

    def __init__(self):
        self.overflow = 0
        self.max_dropped_rel = 0.0
        self.recompressions = 0

    def record_cap(self, s, r, total):
        tail = float(np.sqrt(np.sum(s[r:] ** 2)))
        self.overflow += 1
        if total > 0:
            self.max_dropped_rel = max(self.max_dropped_rel, tail / total)


def trunc_rank(s: np.ndarray, eps: float) -> int:
    """Smallest r with ||s[r:]||_2 <= eps * ||s||_2 (s sorted descending)."""
    s = np.asarray(s, dtype=np.float64)
    if s.size == 0:
        return 0
    total2 = float(np.sum(s * s))
    if total2 == 0.0:
        return 0
    thr2 = (eps * eps) * total2
    # tail2[r] = sum_{l >= r} s_l^2, r = 0..len(s)
    tail2 = np.concatenate([np.cumsum((s * s)[::-1])[::-1], [0.0]])
    for r in range(len(s) + 1):
        if tail2[r] <= thr2:
            return r
    return len(s)


def compress_tile(A: np.ndarray, eps: float, cap: int, overflow: str):
    """Truncated SVD of one admissible tile.  Returns ('L', U, V) with U
    orthonormal (b x r) and V = W_r Sigma_r, or ('D', A) when the eps-rank
    exceeds the cap under overflow='dense'."""
    u, s, wt = np.linalg.svd(A, full_matrices=False)
    r = trunc_rank(s, eps)
    if r > cap:
        if overflow == "dense":
            return ("D", np.array(A, dtype=np.float64, copy=True))
        r = cap
    U = np.ascontiguousarray(u[:, :r])
    V = np.ascontiguousarray(wt[:r, :].T * s[:r])
    return ("L", U, V)


def rounded_add(terms, eps: float, cap: int, stats: Stats):
    """Rounded low-rank addition (Alg. 6) of any number of terms U_t V_t^T:
    stack the bases, QR each stack, SVD the small core R_U R_V^T, keep the
    first r_eps singular triplets: U_C = Q_U u_r, V_C = Q_V v_r sigma_r."""
    b = terms[0][0].shape[0]
    U = np.concatenate([t[0] for t in terms], axis=1)
    V = np.concatenate([t[1] for t in terms], axis=1)
    stats.recompressions += 1
    if U.shape[1] == 0:
        return np.zeros((b, 0)), np.zeros((b, 0))
    Qu, Ru = np.linalg.qr(U)
    Qv, Rv = np.linalg.qr(V)
    u, s, vt = np.linalg.svd(Ru @ Rv.T)
    r = trunc_rank(s, eps)
    if r > cap:
        stats.record_cap(s, cap, float(np.sqrt(np.sum(s * s))))
        r = cap
    Uc = Qu @ u[:, :r]
    Vc = Qv @ (vt[:r, :].T * s[:r])
    return np.ascontiguousarray(Uc), np.ascontiguousarray(Vc)
