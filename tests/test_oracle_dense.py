"""Pins of the oracle's dense Householder primitives against LAPACK (numpy),
explicit reflector products and the defining identities."""
import numpy as np
import pytest

from oracle import dense, metrics

U = np.finfo(np.float64).eps


def explicit_reflector(tau, v):
    u = np.concatenate([[1.0], v])
    return np.eye(len(u)) - tau * np.outer(u, u)


@pytest.mark.parametrize("alpha", [3.0, -2.0, 0.0, 1e-300])
def test_larfg_annihilates(alpha):
    rng = np.random.default_rng(1)
    x = rng.standard_normal(7)
    beta, tau, v = dense.larfg(alpha, x)
    H = explicit_reflector(tau, v)
    out = H @ np.concatenate([[alpha], x])
    assert abs(out[0] - beta) <= 1e-14 * abs(beta)
    assert np.max(np.abs(out[1:])) <= 1e-14 * abs(beta)
    assert np.allclose(H @ H.T, np.eye(8), atol=1e-14)
    # LAPACK sign convention: beta has the sign opposite to alpha (sign(0) = +)
    assert beta == -np.sign(alpha if alpha != 0 else 1.0) * abs(beta)
    assert 1.0 <= tau <= 2.0


def test_larfg_zero_tail_is_identity():
    beta, tau, v = dense.larfg(-4.0, np.zeros(5))
    assert tau == 0.0 and beta == -4.0 and not np.any(v)


def test_larfg_no_overflow():
    beta, tau, v = dense.larfg(1e300, np.array([1e300, 1e300]))
    assert np.isfinite(beta) and abs(abs(beta) - np.sqrt(3) * 1e300) < 1e286


@pytest.mark.parametrize("h,nb", [(8, 8), (20, 6), (33, 17)])
def test_householder_qr_matches_lapack_and_product_of_reflectors(h, nb):
    rng = np.random.default_rng(h)
    A = rng.standard_normal((h, nb))
    F, tau, T = dense.householder_qr(A)
    R = np.triu(F[:nb])
    Rl = np.linalg.qr(A, mode="r")
    assert metrics.r_rel_diff(R, Rl) < 1e-14
    # compact WY equals the product of the individual reflectors H_1 ... H_nb
    Y = dense.unit_lower(F)
    Qprod = np.eye(h)
    for j in range(nb):
        Hj = np.eye(h)
        Hj[j:, j:] = explicit_reflector(tau[j], Y[j + 1:, j])
        Qprod = Qprod @ Hj
    Qwy = np.eye(h) - Y @ T @ Y.T
    assert np.allclose(Qwy, Qprod, atol=1e-13)
    assert np.allclose(Qwy[:, :nb] @ R, A, atol=1e-13)
    assert np.allclose(np.tril(T, -1), 0.0)


def test_householder_qr_zero_column():
    A = np.zeros((6, 3))
    A[:, 0] = 1.0
    A[:, 2] = np.arange(6.0)
    F, tau, T = dense.householder_qr(A)
    # column 1 of the reduced matrix is already zero below its pivot
    assert tau[1] == 0.0 and F[1, 1] == 0.0
    Y = dense.unit_lower(F)
    Q = np.eye(6) - Y @ T @ Y.T
    assert np.allclose(Q[:, :3] @ np.triu(F[:3]), A, atol=1e-13)


@pytest.mark.parametrize("mb", [1, 5, 12])
def test_tpqrt_matches_qr_of_stack(mb):
    rng = np.random.default_rng(mb)
    nb = 8
    R0 = np.triu(rng.standard_normal((nb, nb)))
    B = rng.standard_normal((mb, nb))
    Rn, Y, tau, T = dense.tpqrt(R0, B)
    Rl = np.linalg.qr(np.vstack([R0, B]), mode="r")
    assert metrics.r_rel_diff(Rn, Rl) < 1e-14
    # Q = I - [I; Y] T [I; Y]^T is orthogonal and Q^T [R0; B] = [Rn; 0]
    V = np.vstack([np.eye(nb), Y])
    Q = np.eye(nb + mb) - V @ T @ V.T
    assert np.allclose(Q.T @ Q, np.eye(nb + mb), atol=1e-14)
    out = Q.T @ np.vstack([R0, B])
    assert np.allclose(out[:nb], Rn, atol=1e-13)
    assert np.max(np.abs(out[nb:])) < 1e-13
    # and tpmqrt applies exactly that Q^T / Q
    C1, C2 = rng.standard_normal((nb, 3)), rng.standard_normal((mb, 3))
    c1, c2 = dense.tpmqrt_t(Y, T, C1, C2)
    assert np.allclose(np.vstack([c1, c2]), Q.T @ np.vstack([C1, C2]), atol=1e-13)
    c1, c2 = dense.tpmqrt_n(Y, T, C1, C2)
    assert np.allclose(np.vstack([c1, c2]), Q @ np.vstack([C1, C2]), atol=1e-13)


def test_planted_transpose_mistake_is_caught(monkeypatch):
    """A plausible slip (T instead of T^T in the Q^T application) must fail
    the explicit-Q pin above."""
    rng = np.random.default_rng(7)
    nb, mb = 6, 6
    R0 = np.triu(rng.standard_normal((nb, nb)))
    B = rng.standard_normal((mb, nb))
    Rn, Y, tau, T = dense.tpqrt(R0, B)
    V = np.vstack([np.eye(nb), Y])
    Q = np.eye(nb + mb) - V @ T @ V.T
    C1, C2 = rng.standard_normal((nb, 2)), rng.standard_normal((mb, 2))
    bad1, bad2 = dense.tpmqrt_n(Y, T, C1, C2)   # the slip
    assert not np.allclose(np.vstack([bad1, bad2]), Q.T @ np.vstack([C1, C2]), atol=1e-8)
