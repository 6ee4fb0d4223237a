"""Dense Householder tile operations (paper Section 2.2-2.3, eq. compact WY).

Conventions (readings):
* reflector generation follows LAPACK's larfg: for pivot alpha and tail x,
  beta = -sign(alpha) * ||(alpha, x)||, sign(0) = +1, tau = (beta - alpha)/beta,
  v = x / (alpha - beta) with an implicit leading 1; if ||x|| = 0 then tau = 0,
  v = 0, beta = alpha (H = I).
* T is upper triangular and built by the forward columnwise recurrence
  T[j,j] = tau_j, T[:j, j] = -tau_j * T[:j,:j] @ G[:j, j], where G is the Gram
  matrix of the reflector vectors, so that Q = H_1 H_2 ... H_b = I - Y T Y^T
  (eq. compact WY).  Q^T is applied with T^T.
"""
from __future__ import annotations

import numpy as np


def nrm2(v: np.ndarray) -> float:
    """Euclidean norm with scaling, so that squares cannot overflow."""
    v = np.asarray(v, dtype=np.float64).ravel()
    if v.size == 0:
        return 0.0
    s = float(np.max(np.abs(v)))
    if s == 0.0:
        return 0.0
    w = v / s
    return s * float(np.sqrt(np.dot(w, w)))


def larfg(alpha: float, x: np.ndarray):
    """Householder reflector H = I - tau [1; v][1; v]^T with H [alpha; x] = [beta; 0]."""
    xnorm = nrm2(x)
    if xnorm == 0.0:
        return float(alpha), 0.0, np.zeros_like(x, dtype=np.float64)
    norm = nrm2(np.array([alpha, xnorm]))
    beta = -norm if alpha >= 0.0 else norm
    tau = (beta - alpha) / beta
    v = np.asarray(x, dtype=np.float64) / (alpha - beta)
    return float(beta), float(tau), v


def larft(G: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Upper-triangular T of the compact WY form from the reflector Gram
    matrix G (only its strictly upper part is read) and the taus."""
    nb = len(tau)
    T = np.zeros((nb, nb))
    for j in range(nb):
        T[j, j] = tau[j]
        if j > 0:
            T[:j, j] = -tau[j] * (T[:j, :j] @ G[:j, j])
    return T


def unit_lower(Yp: np.ndarray) -> np.ndarray:
    """Explicit unit-lower-trapezoidal Y from a packed factor (strict lower part)."""
    h, nb = Yp.shape
    Y = np.tril(Yp, -1)
    Y[np.arange(nb), np.arange(nb)] = 1.0
    return Y


def householder_qr(A: np.ndarray):
    """Unblocked Householder QR of an h x nb matrix (h >= nb), column by column.

    Returns (F, tau, T): F holds R in its upper triangle and the reflector
    tails in its strict lower part; T is the nb x nb compact-WY factor.
    Used for the diagonal tile (GEQRT, Section 3.4.1) and for the stacked
    block column (Section 3.3.1)."""
    F = np.array(A, dtype=np.float64, copy=True)
    h, nb = F.shape
    tau = np.zeros(nb)
    for j in range(nb):
        beta, t, v = larfg(F[j, j], F[j + 1:, j])
        F[j, j] = beta
        F[j + 1:, j] = v
        tau[j] = t
        if t != 0.0 and j + 1 < nb:
            # apply H_j to the trailing columns
            w = F[j, j + 1:] + v @ F[j + 1:, j + 1:]
            F[j, j + 1:] -= t * w
            F[j + 1:, j + 1:] -= t * np.outer(v, w)
    Y = unit_lower(F[:, :nb])
    T = larft(Y.T @ Y, tau)
    return F, tau, T


def geqrt(A: np.ndarray):
    """QR of a dense b x b diagonal tile (Section 3.4.1): A = Qkk Rkk with
    Qkk = I - Y T Y^T.  Returns (F, tau, T) as householder_qr."""
    return householder_qr(A)


def apply_qt_left(Y: np.ndarray, T: np.ndarray, C: np.ndarray) -> np.ndarray:
    """C <- (I - Y T Y^T)^T C = C - Y T^T (Y^T C)  (Section 3.4.2)."""
    return C - Y @ (T.T @ (Y.T @ C))


def apply_q_left(Y: np.ndarray, T: np.ndarray, C: np.ndarray) -> np.ndarray:
    """C <- (I - Y T Y^T) C."""
    return C - Y @ (T @ (Y.T @ C))


def tpqrt(R: np.ndarray, B: np.ndarray):
    """QR of the stack [R; B], R upper triangular nb x nb, B mb x nb dense
    (Section 3.4.3).  Reflector j is [e_j; y_j] with y_j in R^mb, so
    Q = I - [I; Y] T [I; Y]^T.  Returns (R', Y, tau, T)."""
    R = np.triu(np.array(R, dtype=np.float64, copy=True))
    Y = np.array(B, dtype=np.float64, copy=True)
    nb = R.shape[1]
    tau = np.zeros(nb)
    for j in range(nb):
        beta, t, v = larfg(R[j, j], Y[:, j])
        R[j, j] = beta
        Y[:, j] = v
        tau[j] = t
        if t != 0.0 and j + 1 < nb:
            w = R[j, j + 1:] + v @ Y[:, j + 1:]
            R[j, j + 1:] -= t * w
            Y[:, j + 1:] -= t * np.outer(v, w)
    # the e_j parts are mutually orthogonal, so the Gram matrix is Y^T Y
    T = larft(Y.T @ Y, tau)
    return R, Y, tau, T


def tpmqrt_t(Y: np.ndarray, T: np.ndarray, C1: np.ndarray, C2: np.ndarray):
    """[C1; C2] <- Q^T [C1; C2] with Q = I - [I; Y] T [I; Y]^T (Section 3.4.4):
    W = T^T (C1 + Y^T C2);  C1 - W;  C2 - Y W."""
    W = T.T @ (C1 + Y.T @ C2)
    return C1 - W, C2 - Y @ W


def tpmqrt_n(Y: np.ndarray, T: np.ndarray, C1: np.ndarray, C2: np.ndarray):
    """[C1; C2] <- Q [C1; C2]: W = T (C1 + Y^T C2)."""
    W = T @ (C1 + Y.T @ C2)
    return C1 - W, C2 - Y @ W
