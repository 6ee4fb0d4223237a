"""Pins of the oracle's blocked MGS BLR-QR (Section 2.1 Alg. 1, Section 3.2),
each against something other than the oracle itself: hand-derived values of
the Lauchli example, LAPACK's R, exact low-rank structure, and the
Householder factorization of the same matrix."""
import numpy as np
import pytest

import synth
from oracle import blockcol, blrmat, metrics, mgs

U = np.finfo(np.float64).eps


def test_lauchli_example_hand_values():
    """A = [[1,1,1],[e,0,0],[0,e,0],[0,0,e]] with e = 1e-8 (1 + e^2 rounds to 1).
    By hand, modified Gram-Schmidt gives q1 = (1, e, 0, 0), q2 = (0, -1, 1, 0)/sqrt2,
    q3 = (0, -1, -1, 2)/sqrt6, so q1.q2 = -e/sqrt2, q1.q3 = -e/sqrt6 and q2.q3 = 0
    (classical Gram-Schmidt would give q2.q3 = 1/2; Householder QR an orthogonal Q)."""
    e = 1e-8
    A = np.array([[1, 1, 1], [e, 0, 0], [0, e, 0], [0, 0, e]], dtype=np.float64)
    Q, R = mgs.mgs(A)
    assert np.allclose(Q[:, 0], [1, e, 0, 0], rtol=0, atol=1e-15)
    assert np.allclose(Q[:, 1], np.array([0, -1, 1, 0]) / np.sqrt(2), atol=1e-12)
    assert np.allclose(Q[:, 2], np.array([0, -1, -1, 2]) / np.sqrt(6), atol=1e-12)
    assert np.isclose(Q[:, 0] @ Q[:, 1], -e / np.sqrt(2), rtol=1e-6)
    assert np.isclose(Q[:, 0] @ Q[:, 2], -e / np.sqrt(6), rtol=1e-6)
    assert abs(Q[:, 1] @ Q[:, 2]) < 1e-15
    # R by hand: r11 = 1, r12 = r13 = 1, r22 = sqrt2 e, r23 = e/sqrt2, r33 = sqrt(3/2) e
    Rh = np.array([[1, 1, 1], [0, np.sqrt(2) * e, e / np.sqrt(2)], [0, 0, np.sqrt(1.5) * e]])
    assert np.allclose(R, Rh, rtol=1e-7, atol=1e-20)


@pytest.mark.parametrize("shape", [(40, 20), (33, 33), (64, 7)])
def test_dense_mgs_against_lapack(shape):
    m, n = shape
    A = np.random.default_rng(m + n).standard_normal((m, n))
    Q, R = mgs.mgs(A)
    kappa = np.linalg.cond(A)
    assert np.array_equal(R, np.triu(R)) and np.all(np.diag(R) > 0)
    assert np.linalg.norm(Q @ R - A) <= 10 * n * U * np.linalg.norm(A)
    # R is unique with a positive diagonal: LAPACK's with its row signs made positive
    Rl = np.linalg.qr(A, mode="r")
    Rl = np.sign(np.diag(Rl))[:, None] * Rl
    assert np.linalg.norm(R - Rl) <= 10 * n * U * kappa * np.linalg.norm(Rl)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 10 * n * U * kappa


def test_dense_mgs_loses_orthogonality_like_kappa():
    """Singular values 1 .. 1e-7: the loss of orthogonality of MGS is bounded
    by a modest multiple of kappa u (Bjorck), far below classical
    Gram-Schmidt's kappa^2 u."""
    rng = np.random.default_rng(4)
    m, n = 60, 30
    Ua, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Va, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Ua * np.logspace(0, -7, n)) @ Va.T
    Q, _ = mgs.mgs(A)
    kappa = 1e7
    loss = np.linalg.norm(Q.T @ Q - np.eye(n))
    assert loss <= 10 * n * U * kappa
    assert loss < 1e-3 * kappa ** 2 * U


def ceil_div(a, b):
    return -(-a // b)


@pytest.mark.parametrize("shape", [(256, 128, 32), (200, 150, 64)])
def test_all_dense_blr_mgs_is_dense_qr(shape):
    """An all-dense BLR matrix (ragged too): Q~ R~ = A and R~ is LAPACK's R
    with a positive diagonal."""
    m, n, b = shape
    A = np.random.default_rng(m * n).standard_normal((m, n))
    blr = blrmat.compress(A, b, 1e-14, b, np.zeros((ceil_div(m, b), ceil_div(n, b)), bool))
    f = mgs.factor(blr, 1e-14, b)
    kappa = np.linalg.cond(A)
    R = f.r_dense()
    assert R.shape == (n, n) and np.array_equal(R, np.triu(R)) and np.all(np.diag(R) > 0)
    Rl = np.linalg.qr(A, mode="r")
    Rl = np.sign(np.diag(Rl))[:, None] * Rl
    assert np.linalg.norm(R - Rl) <= 10 * n * U * kappa * np.linalg.norm(Rl)
    assert f.res(A) <= 10 * n * U
    assert f.orth() <= 10 * n * U * kappa


def test_exactly_low_rank_blr():
    """Random BLR (rank-2 off-diagonal tiles, weak admissibility): the
    factorization keeps Res~ at the truncation tolerance, R~ agrees with the
    Householder block-column R up to row signs, and every low-rank tile of
    Q~ keeps A~'s left factor U."""
    m, n, b, eps = 512, 256, 32, 1e-10
    D, X, Y = synth.random_blr_tiles(2, m, n, b, 2)
    p, q = m // b, n // b
    A = np.empty((m, n))
    for i in range(p):
        for j in range(q):
            A[i * b:(i + 1) * b, j * b:(j + 1) * b] = D[j] if i == j else X[i, j] @ Y[i, j].T
    mask = np.ones((p, q), bool)
    mask[np.arange(q), np.arange(q)] = False
    blr = blrmat.compress(A, b, eps, b, mask)
    At = blr.to_dense()
    f = mgs.factor(blr, eps, b)
    fh = blockcol.factor(blr, eps, b)
    kappa = np.linalg.cond(At)
    assert f.res(At) <= 10 * eps
    assert metrics.r_rel_diff(f.r_dense(), fh.r_dense()) <= 10 * kappa * eps
    for (i, j), Uq in f.A.U.items():
        if j == 0 and blr.fmt[i, j] == 1:
            assert np.array_equal(Uq, blr.U[(i, j)])


def test_householder_keeps_orthogonality_that_mgs_loses():
    """The paper's accuracy comparison (Table res-acc-bem2d, Section 5.2) on
    a synthetic stand-in: a 2D log-kernel matrix with kappa ~ 1e6.  Both
    factorizations reach Res~ at the tolerance; the Householder Q is
    orthogonal to the rounding level while the MGS Q~ loses orthogonality in
    proportion to kappa."""
    m, n, b, eps = 1024, 512, 64, 1e-10
    x, y = synth.kernel_points(0, m, n, 2)
    A = blrmat.kernel_matrix(x, y, "log2d")
    blr = blrmat.compress(A, b, eps, b // 2, blrmat.lowrank_mask(x, y, b, "adjacent", m // b, n // b))
    At = blr.to_dense()
    fm = mgs.factor(blr, eps, b // 2)
    fh = blockcol.factor(blr, eps, b // 2)
    assert fm.res(At) <= 10 * eps and metrics.res(fh, At) <= 10 * eps
    assert metrics.orth(fh) <= 10 * np.sqrt(n) * U
    assert fm.orth() >= 1e4 * metrics.orth(fh)
