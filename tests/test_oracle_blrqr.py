"""Pins of the oracle's BLR-QR (tiled Alg. 4 / Section 3.4 and block-column
Alg. 2 / Section 3.3) against dense LAPACK QR, invariants, the paper's Table
res-acc-random, least-squares optimality and the task/cost model."""
import json
import os

import numpy as np
import pytest

import synth
from oracle import blockcol, blrmat, ledger, metrics, tiled
from oracle.blrmat import DENSE, LOWRANK
from oracle.factor import SingularR

U = np.finfo(np.float64).eps
VARIANTS = [tiled, blockcol]
HERE = os.path.dirname(os.path.abspath(__file__))


def all_dense(A, b):
    m, n = A.shape
    return blrmat.compress(A, b, 1e-12, b, np.zeros((m // b, n // b), bool))


def kernel_blr(seed, m, n, b, eps, cap, rule="adjacent", kern="log2d", dim=2,
               overflow="dense"):
    x, y = synth.kernel_points(seed, m, n, dim)
    A = blrmat.kernel_matrix(x, y, kern)
    mask = blrmat.lowrank_mask(x, y, b, rule, m // b, n // b)
    return A, blrmat.compress(A, b, eps, cap, mask, overflow)


# X1: dense special case ------------------------------------------------------
@pytest.mark.parametrize("mod", VARIANTS)
@pytest.mark.parametrize("shape", [(8, 8, 2), (16, 8, 4), (48, 24, 8), (64, 64, 16), (96, 32, 16)])
def test_all_dense_reduces_to_householder_qr(mod, shape):
    m, n, b = shape
    A = np.random.default_rng(m * n + b).standard_normal((m, n))
    f = mod.factor(all_dense(A, b), 1e-12, b)
    R = f.r_dense()
    Rl = np.linalg.qr(A, mode="r")
    kappa = np.linalg.cond(A)
    assert metrics.r_rel_diff(R, Rl) <= 10 * n * U * kappa
    assert metrics.res(f, A) <= 10 * n * U
    assert metrics.orth(f) <= 10 * np.sqrt(n) * U


@pytest.mark.parametrize("mod", VARIANTS)
def test_exact_compression_reduces_to_dense_qr(mod):
    """eps far below rounding and cap = b: low-rank tiles are exact, so R is
    the dense R up to row signs."""
    m, n, b = 128, 64, 16
    A, blr = kernel_blr(1, m, n, b, 1e-15, b)
    assert np.any(blr.fmt == LOWRANK)
    f = mod.factor(blr, 1e-15, b)
    Rl = np.linalg.qr(A, mode="r")
    kappa = np.linalg.cond(A)
    assert metrics.r_rel_diff(f.r_dense(), Rl) <= 1e-13 * kappa
    assert metrics.res(f, A) <= 1e-13


# X2 / X3: invariants -----------------------------------------------------------
@pytest.mark.parametrize("mod", VARIANTS)
def test_invariants_kernel_matrix(mod):
    m, n, b, eps = 256, 128, 32, 1e-8
    A, blr = kernel_blr(2, m, n, b, eps, 16)
    At = blr.to_dense()
    f = mod.factor(blr, eps, 16)
    assert metrics.res(f, At) <= 10 * eps
    assert metrics.orth(f) <= 1e3 * U
    Bm = np.random.default_rng(0).standard_normal((m, 3))
    assert np.allclose(f.apply_qt(f.apply_q(Bm)), Bm, atol=1e-13)
    assert np.allclose(f.apply_q(f.apply_qt(Bm)), Bm, atol=1e-13)
    # every low-rank R tile has an orthonormal basis (X3)
    for k in range(f.q):
        for j in range(k + 1, f.q):
            if f.A.fmt[k, j] == LOWRANK:
                Uk = f.A.U[(k, j)]
                assert np.linalg.norm(Uk.T @ Uk - np.eye(Uk.shape[1])) <= 1e3 * U
    # Q^T A~ is [R; 0]
    QtA = f.apply_qt(At)
    assert np.linalg.norm(QtA[n:]) <= 10 * eps * np.linalg.norm(At)
    assert np.allclose(np.tril(f.r_dense(), -1), 0.0)


def test_lowrank_tpqrt_eliminates_exactly():
    """Section 3.4.3: with U orthonormal, the T of [R; V^T] makes
    I - [I; U Y] T [I; U Y]^T an orthogonal factor that zeroes U V^T."""
    from oracle import dense
    rng = np.random.default_rng(11)
    b, r = 12, 3
    R0 = np.triu(rng.standard_normal((b, b)))
    Uo = np.linalg.qr(rng.standard_normal((b, r)))[0]
    V = rng.standard_normal((b, r))
    Rn, Y, tau, T = dense.tpqrt(R0, V.T)
    Yt = Uo @ Y
    Vs = np.vstack([np.eye(b), Yt])
    Q = np.eye(2 * b) - Vs @ T @ Vs.T
    assert np.allclose(Q.T @ Q, np.eye(2 * b), atol=1e-13)
    out = Q.T @ np.vstack([R0, Uo @ V.T])
    assert np.allclose(out[:b], Rn, atol=1e-12)
    assert np.max(np.abs(out[b:])) <= 1e-12


# X4: the paper's Table res-acc-random (order of magnitude) -------------------
@pytest.mark.slow
def test_random_blr_matches_table_res_acc_random():
    gold = json.load(open(os.path.join(HERE, "golden", "table_res_acc_random.json")))
    row = gold["rows"][0]
    m, n = row["m"], row["n"]
    b = int(2 * np.sqrt(n))
    A = synth.random_blr_dense(0, m, n, b, 1)
    mask = blrmat.lowrank_mask(None, None, b, "weak", m // b, n // b)
    blr = blrmat.compress(A, b, 1e-10, b, mask)
    assert {blr.rank(i, j) for i in range(m // b) for j in range(n // b)} == {-1, 1}
    ft = tiled.factor(blr, 1e-10, b)
    fb = blockcol.factor(blr, 1e-10, b)
    # at least as accurate as the paper's figures (within one order of magnitude)
    assert metrics.res(ft, A) <= 10 * row["tiled_res"]
    assert metrics.orth(ft) <= 10 * row["tiled_orth"]
    assert metrics.res(fb, A) <= 10 * max(row["blocked_res"], 1e-14)
    assert metrics.orth(fb) <= 10 * max(row["blocked_orth"], 1e-14)
    # the structure is kept under weak admissibility: no fill-in
    assert np.array_equal(ft.A.fmt, blr.fmt) and np.array_equal(fb.A.fmt, blr.fmt)


# X5: least squares --------------------------------------------------------------
@pytest.mark.parametrize("mod", VARIANTS)
def test_lstsq_normal_equations(mod):
    m, n, b, eps = 192, 96, 16, 1e-8
    A, blr = kernel_blr(3, m, n, b, eps, 16, kern="inv_r", dim=3, rule="dist_gt_diam")
    At = blr.to_dense()
    f = mod.factor(blr, eps, 16)
    B = synth.rhs(3, m, 4)
    X = f.lstsq(B)
    # optimality for the matrix actually factored (Q R)
    QR = f.q_times_r()
    assert np.all(metrics.eta_ne(QR, X, B) <= 10 * n * U * 100)
    Xref = np.linalg.lstsq(At, B, rcond=None)[0]
    kappa = np.linalg.cond(At)
    assert np.linalg.norm(X - Xref) / np.linalg.norm(Xref) <= kappa * 10 * eps


@pytest.mark.parametrize("mod", VARIANTS)
def test_singular_r_detected(mod):
    A = np.random.default_rng(4).standard_normal((32, 16))
    A[:, 5] = 0.0
    f = mod.factor(all_dense(A, 8), 1e-12, 8)
    with pytest.raises(SingularR):
        f.lstsq(np.ones((32, 1)))


# X6: schedule independence ------------------------------------------------------
def test_any_topological_order_is_bitwise_identical():
    A, blr = kernel_blr(5, 128, 64, 16, 1e-8, 8)
    f0 = tiled.factor(blr, 1e-8, 8)
    for order, seed in [("random", 1), ("random", 2), ("priority", 0)]:
        f = tiled.factor(blr, 1e-8, 8, order=order, seed=seed)
        assert np.array_equal(f.r_dense(), f0.r_dense())
        for key in f0.Tik:
            assert np.array_equal(f.Tik[key], f0.Tik[key])


def test_dag_edges_follow_the_paper():
    tasks = tiled.task_list(3, 3)
    deps = tiled.build_dag(tasks)
    idx = {t: i for i, t in enumerate(tasks)}
    d = lambda t: {tasks[j] for j in deps[idx[t]]}
    assert d(("larfb", 0, 1)) == {("geqrt", 0)}
    assert ("tpqrt", 1, 0) in d(("tpqrt", 2, 0))
    assert d(("tpmqrt", 2, 0, 1)) >= {("tpqrt", 2, 0), ("tpmqrt", 1, 0, 1)}
    # LARFB(k,j) and TPQRT(i,k) touch different parts of the diagonal tile
    assert ("larfb", 0, 1) not in d(("tpqrt", 1, 0))
    assert d(("geqrt", 1)) == {("tpmqrt", 1, 0, 1)}


# X7: task counts and cost model --------------------------------------------------
def test_task_counts_and_cost_sums():
    for p, q in [(16, 8), (128, 64), (5, 5)]:
        tasks = tiled.task_list(p, q)
        got = {k: sum(1 for t in tasks if t[0] == k) for k in ("geqrt", "larfb", "tpqrt", "tpmqrt")}
        assert got == ledger.tiled_task_counts(p, q)
    assert ledger.tiled_task_counts(128, 64) == {"geqrt": 64, "larfb": 2016, "tpqrt": 6112, "tpmqrt": 214368}
    for (m, n, b, r) in [(2048, 1024, 64, 1), (32768, 16384, 256, 16), (4096, 4096, 128, 7)]:
        assert ledger.t_blocked_sum(m, n, b, r) == pytest.approx(ledger.t_blocked_printed(m, n, b, r), rel=1e-12)
        assert ledger.t_tiled_sum(m, n, b, r) == pytest.approx(ledger.t_tiled_closed(m, n, b, r), rel=1e-12)
    # the printed closed form of T_tiled does not equal its own sum (q = 1:
    # the sum is p b^3 while the printed form gives p b^3 - 5 b^2 r / 6)
    assert ledger.t_tiled_printed(256, 128, 128, 4) != pytest.approx(ledger.t_tiled_sum(256, 128, 128, 4))


def test_tiled_counts_executed():
    A, blr = kernel_blr(6, 128, 64, 16, 1e-8, 8)
    f = tiled.factor(blr, 1e-8, 8)
    assert f.counts == ledger.tiled_task_counts(8, 4)


# X8: the two variants agree -------------------------------------------------------
def test_variants_agree():
    m, n, b, eps = 256, 128, 32, 1e-9
    A, blr = kernel_blr(7, m, n, b, eps, 32, kern="inv_r", dim=3, rule="dist_gt_diam")
    ft = tiled.factor(blr, eps, 32)
    fb = blockcol.factor(blr, eps, 32)
    kappa = np.linalg.cond(A)
    assert metrics.r_rel_diff(ft.r_dense(), fb.r_dense()) <= 10 * kappa * eps


# stop-after-K prefix ----------------------------------------------------------------
@pytest.mark.parametrize("mod", VARIANTS)
def test_prefix_factor(mod):
    A = np.random.default_rng(8).standard_normal((64, 32))
    blr = all_dense(A, 8)
    f = mod.factor(blr, 1e-12, 8, stop_after_k=2)
    QtA = f.apply_qt(A)
    Rl = np.linalg.qr(A, mode="r")
    # the first two block columns are triangularised
    assert np.allclose(np.tril(QtA[:, :16], -1), 0.0, atol=1e-12)
    assert metrics.r_rel_diff(np.triu(QtA[:16, :16]), Rl[:16, :16]) < 1e-13


def test_fill_in_rule_under_strong_admissibility():
    """OP1: a low-rank target that receives a dense update becomes dense."""
    m, n, b, eps = 256, 128, 32, 1e-8
    A, blr = kernel_blr(9, m, n, b, eps, 32, kern="inv_r", dim=3, rule="dist_gt_diam")
    f = tiled.factor(blr, eps, 32)
    before, after = blr.fmt, f.A.fmt
    assert np.all(after <= before)            # formats only go low-rank -> dense


# planted mistakes: each plausible slip in the oracle must fail a pin ---------------
@pytest.mark.parametrize("slip", ["no_transpose", "drop_update", "wrong_sign"])
def test_planted_mistakes_fail_the_dense_pin(monkeypatch, slip):
    from oracle import blrops
    orig_t, orig_add = blrops.t_times, blrops.add
    if slip == "no_transpose":
        monkeypatch.setattr(blrops, "t_times", lambda T, X, trans: orig_t(T, X, False))
    elif slip == "drop_update":
        monkeypatch.setattr(blrops, "add", lambda X, Y, s, *a: orig_add(X, Y, 0.0 if s < 0 else s, *a))
    else:
        monkeypatch.setattr(blrops, "add", lambda X, Y, s, *a: orig_add(X, Y, -s, *a))
    A = np.random.default_rng(9).standard_normal((48, 24))
    f = tiled.factor(all_dense(A, 8), 1e-12, 8)
    assert metrics.r_rel_diff(f.r_dense(), np.linalg.qr(A, mode="r")) > 1e-6


def test_random_blr_tiles_are_the_dense_generator_draws():
    """The tile-factor form of the random-BLR workload (used at benchmark
    size) draws exactly the values of the dense generator."""
    m, n, b, r = 96, 64, 16, 3
    A = synth.random_blr_dense(4, m, n, b, r)
    D, X, Y = synth.random_blr_tiles(4, m, n, b, r)
    for i in range(m // b):
        for j in range(n // b):
            blk = A[i * b:(i + 1) * b, j * b:(j + 1) * b]
            ref = D[i] if i == j else X[i, j] @ Y[i, j].T
            assert np.array_equal(blk, ref)


def test_batch_rows_are_log_uniform_multiples():
    """Row counts of the batched workload: multiples of 2b inside [lo, hi],
    deterministic in the seed, and log-uniform (the logarithms of many draws
    spread evenly over [ln lo, ln hi])."""
    m = synth.batch_rows(0, 64, 4096, 32768, 512)
    assert np.array_equal(m, synth.batch_rows(0, 64, 4096, 32768, 512))
    assert not np.array_equal(m, synth.batch_rows(1, 64, 4096, 32768, 512))
    assert m.min() >= 4096 and m.max() <= 32768 and np.all(m % 512 == 0)
    big = synth.batch_rows(3, 20000, 4096, 32768, 1)
    z = (np.log(big) - np.log(4096)) / (np.log(32768) - np.log(4096))
    hist = np.histogram(z, bins=8, range=(0, 1))[0] / len(z)
    assert np.all(np.abs(hist - 1 / 8) < 0.01)


def test_block_column_sum_orders():
    """The two orders of the block-column accumulation of low-rank terms,
    checked on strings, where the order is visible: the default chain in the
    order of the sum, and the pairwise tree over the terms in index order."""
    from oracle.blockcol import chain_sum, pairwise_sum
    cat = lambda a, b: "(" + a + "+" + b + ")"
    assert chain_sum(["a"], cat) == "a"
    assert chain_sum(list("abcd"), cat) == "(((a+b)+c)+d)"
    assert pairwise_sum(["a"], cat) == "a"
    assert pairwise_sum(["a", "b", "c"], cat) == "((a+b)+c)"
    assert pairwise_sum(list("abcde"), cat) == "(((a+b)+(c+d))+e)"
    assert pairwise_sum(list("abcdefgh"), cat) == "(((a+b)+(c+d))+((e+f)+(g+h)))"


@pytest.mark.parametrize("t", [2, 3, 7, 16])
def test_chain_and_tree_sums_agree_within_rounding_bound(t):
    """Every rounded addition (Alg. 6) moves its sum by at most eps times the
    sum's Frobenius norm (no cap binds here), so each order is within
    (t-1) eps S of the exact sum of t terms, S = sum of the terms' norms, and
    the two orders are within 2 (t-1) eps S of each other.  Both are checked
    against the exact (dense) sum too."""
    from oracle import blrops, lowrank
    from oracle.blockcol import chain_sum, pairwise_sum
    rng = np.random.default_rng(100 + t)
    b, eps = 48, 1e-6
    # terms with a shared decaying spectrum, so that truncation at eps drops
    # a visible tail in every addition
    terms = []
    decay = 10.0 ** -np.arange(12)
    for _ in range(t):
        Uq, _ = np.linalg.qr(rng.standard_normal((b, 12)))
        terms.append(("L", Uq, rng.standard_normal((b, 12)) * decay))
    st = lowrank.Stats()
    add = lambda a, x: blrops.add(a, x, 1.0, eps, b, st)
    zc = blrops.dense_of(chain_sum(terms, add))
    zt = blrops.dense_of(pairwise_sum(terms, add))
    exact = sum(blrops.dense_of(x) for x in terms)
    S = sum(np.linalg.norm(blrops.dense_of(x)) for x in terms)
    assert st.overflow == 0
    assert np.linalg.norm(zc - exact) <= (t - 1) * eps * S * (1 + 1e-6)
    assert np.linalg.norm(zt - exact) <= (t - 1) * eps * S * (1 + 1e-6)
    assert np.linalg.norm(zt - zc) <= 2 * (t - 1) * eps * S * (1 + 1e-6)
    # the truncations are not vacuous: the rounded sums differ from the exact
    assert np.linalg.norm(zc - exact) > 1e-3 * eps * S


def test_block_column_chain_and_tree_factors_agree():
    """Whole factorizations with the two accumulation orders: R agrees up to
    the compression tolerance (C kappa eps) and both residuals are at eps."""
    m, n, b, eps = 512, 256, 32, 1e-8
    A, blr = kernel_blr(21, m, n, b, eps, b, rule="weak", kern="inv_r", dim=3)
    At = blr.to_dense()
    fc = blockcol.factor(blr, eps, b)
    ft = blockcol.factor(blr, eps, b, zsum="tree")
    assert fc.stats.recompressions > 0
    kappa = np.linalg.cond(At)
    Rc, Rt = fc.r_dense(), ft.r_dense()
    assert np.linalg.norm(metrics.sign_fix(Rt, Rc) - Rc) / np.linalg.norm(Rc) <= 10 * kappa * eps
    assert metrics.res(fc, At) <= 10 * eps and metrics.res(ft, At) <= 10 * eps


@pytest.mark.parametrize("solve", ["normal", "qr"])
def test_lstsq_adjoint_matches_finite_differences(solve):
    """The adjoint of x = argmin ||A x - b|| against central differences of
    the exact least-squares map, for b, a dense entry of A and, through a
    low-rank tile A_ij = U V^T, entries of U and V.  L = <Xbar, X>.  Both
    ways of solving (normal matrix, dense QR) give it."""
    from oracle import adjoint, blrmat
    rng = np.random.default_rng(17)
    m, n, b, nrhs = 48, 24, 8, 2
    A0 = rng.standard_normal((m, n))
    blr = blrmat.compress(A0, b, 1e-14, b, np.zeros((m // b, n // b), bool))
    # one low-rank tile with rank 3 factors (U orthonormal), the rest dense
    Uq, _ = np.linalg.qr(rng.standard_normal((b, 3)))
    blr.fmt[4, 1] = 1
    blr.U[(4, 1)], blr.V[(4, 1)] = Uq, rng.standard_normal((b, 3))
    blr.D.pop((4, 1), None)
    A = blr.to_dense()
    B = rng.standard_normal((m, nrhs))
    Xbar = rng.standard_normal((n, nrhs))
    X, Bbar, Abar = adjoint.lstsq_adjoint(A, B, Xbar, solve)
    g = adjoint.tile_gradients(blr, Abar)
    loss = lambda A_, B_: float(np.sum(Xbar * np.linalg.lstsq(A_, B_, rcond=None)[0]))
    h = 1e-6
    E = np.zeros_like(B); E[5, 1] = h
    assert np.isclose((loss(A, B + E) - loss(A, B - E)) / (2 * h), Bbar[5, 1], rtol=1e-6, atol=1e-9)
    E = np.zeros_like(A); E[10, 3] = h      # tile (1, 0), dense
    assert blr.fmt[1, 0] == 0
    assert np.isclose((loss(A + E, B) - loss(A - E, B)) / (2 * h), g[(1, 0)][1][10 - 8, 3], rtol=1e-6, atol=1e-9)
    for which, (r, c) in (("U", (2, 1)), ("V", (6, 2))):
        def dense_with(d):
            U, V = blr.U[(4, 1)].copy(), blr.V[(4, 1)].copy()
            (U if which == "U" else V)[r, c] += d
            A_ = A.copy()
            A_[32:40, 8:16] = U @ V.T
            return A_
        fd = (loss(dense_with(h), B) - loss(dense_with(-h), B)) / (2 * h)
        an = g[(4, 1)][1 if which == "U" else 2][r, c]
        assert np.isclose(fd, an, rtol=1e-6, atol=1e-9), (which, fd, an)


@pytest.mark.parametrize("solve", ["normal", "qr"])
def test_lstsq_adjoint_closed_form_square(solve):
    """Square nonsingular A: x = A^{-1} b, so bbar = A^{-T} xbar and
    Abar = -bbar x^T (the residual is zero)."""
    from oracle import adjoint
    rng = np.random.default_rng(3)
    A = rng.standard_normal((12, 12)) + 12 * np.eye(12)
    B = rng.standard_normal((12, 2))
    Xbar = rng.standard_normal((12, 2))
    X, Bbar, Abar = adjoint.lstsq_adjoint(A, B, Xbar, solve)
    assert np.allclose(Bbar, np.linalg.solve(A.T, Xbar))
    assert np.allclose(Abar, -Bbar @ X.T)


# Ragged edges: b need not divide m or n; the last tile row or column is
# narrower (rectangular blocks, Section 3.1) ---------------------------------
def ceil_div(a, b):
    return -(-a // b)


@pytest.mark.parametrize("mod", VARIANTS)
@pytest.mark.parametrize("shape", [(70, 45, 16), (64, 40, 16), (70, 48, 16), (50, 50, 16),
                                   (37, 20, 8), (33, 33, 32), (20, 7, 16)])
def test_ragged_all_dense_reduces_to_householder_qr(mod, shape):
    m, n, b = shape
    A = np.random.default_rng(m * n + b).standard_normal((m, n))
    blr = blrmat.compress(A, b, 1e-12, b, np.zeros((ceil_div(m, b), ceil_div(n, b)), bool))
    assert np.array_equal(blr.to_dense(), A)
    f = mod.factor(blr, 1e-12, b)
    R = f.r_dense()
    assert R.shape == (n, n) and np.array_equal(R, np.triu(R))
    kappa = np.linalg.cond(A)
    assert metrics.r_rel_diff(R, np.linalg.qr(A, mode="r")) <= 10 * n * U * kappa
    assert metrics.res(f, A) <= 10 * n * U
    assert metrics.orth(f) <= 10 * np.sqrt(n) * U
    Bm = np.random.default_rng(1).standard_normal((m, 3))
    assert np.allclose(f.apply_qt(f.apply_q(Bm)), Bm, atol=1e-13)
    X = f.lstsq(Bm)
    Xl = np.linalg.lstsq(A, Bm, rcond=None)[0]
    assert np.linalg.norm(X - Xl) / np.linalg.norm(Xl) <= 10 * n * U * kappa ** 2
    if m > n:   # a square system has no least-squares residual to test
        assert np.all(metrics.eta_ne(A, X, Bm) <= 10 * n * U)
    else:
        assert np.linalg.norm(A @ X - Bm) <= 10 * n * U * kappa * np.linalg.norm(Bm)


def ragged_kernel_blr(seed, m, n, b, eps, cap, rule="adjacent", kern="log2d", dim=2):
    x, y = synth.kernel_points(seed, m, n, dim)
    A = blrmat.kernel_matrix(x, y, kern)
    mask = blrmat.lowrank_mask(x, y, b, rule, ceil_div(m, b), ceil_div(n, b))
    return A, blrmat.compress(A, b, eps, cap, mask)


def test_ragged_cluster_boxes_cover_every_point():
    pts = synth.points(3, 0, 70, 2)
    lo, hi = blrmat.cluster_boxes(pts, 16)
    assert lo.shape == (5, 2)
    for c in range(5):
        blk = pts[16 * c:16 * (c + 1)]
        assert np.array_equal(lo[c], blk.min(axis=0)) and np.array_equal(hi[c], blk.max(axis=0))


@pytest.mark.parametrize("mod", VARIANTS)
def test_ragged_kernel_matrix_invariants(mod):
    """Low-rank tiles on the narrow edge too: Res~ <= 10 eps, Orth, Q^T A~ =
    [R; 0] and the least-squares normal equations."""
    m, n, b, eps = 300, 170, 32, 1e-8
    A, blr = ragged_kernel_blr(4, m, n, b, eps, 16)
    assert blr.p == 10 and blr.q == 6
    assert np.any(blr.fmt[-1] == LOWRANK) and np.any(blr.fmt[:, -1] == LOWRANK)
    At = blr.to_dense()
    f = mod.factor(blr, eps, 16)
    assert metrics.res(f, At) <= 10 * eps
    assert metrics.orth(f) <= 1e3 * U
    QtA = f.apply_qt(At)
    assert np.linalg.norm(QtA[n:]) <= 10 * eps * np.linalg.norm(At)
    Bm = synth.rhs(4, m, 2)
    X = f.lstsq(Bm)
    assert np.all(metrics.eta_ne(At, X, Bm) <= 10 * eps * np.linalg.cond(At))


def test_ragged_variants_agree_and_dag_order_is_irrelevant():
    m, n, b, eps = 300, 170, 32, 1e-8
    A, blr = ragged_kernel_blr(5, m, n, b, eps, 16)
    ft = tiled.factor(blr, eps, 16)
    fb = blockcol.factor(blr, eps, 16)
    kappa = np.linalg.cond(blr.to_dense())
    assert metrics.r_rel_diff(fb.r_dense(), ft.r_dense()) <= 10 * kappa * eps
    fr = tiled.factor(blr, eps, 16, order="random", seed=3)
    assert np.array_equal(fr.r_dense(), ft.r_dense())


def embed_ragged(A, b):
    """A' = [A 0; 0 E] with tile-multiple sizes: zero rows below A, and for
    each padded column a one in a padded row (E = [I; 0]); one more tile row
    when the padded rows would not hold the identity."""
    m, n = A.shape
    n2 = ceil_div(n, b) * b
    m2 = ceil_div(m, b) * b
    if m2 - m < n2 - n:
        m2 += b
    Ap = np.zeros((m2, n2))
    Ap[:m, :n] = A
    for t in range(n2 - n):
        Ap[m + t, n + t] = 1.0
    return Ap


@pytest.mark.parametrize("mod", VARIANTS)
def test_ragged_embedding_keeps_r_and_least_squares(mod):
    """The tile-multiple embedding A' factors to R' = diag(R, -I) up to row
    signs, and its least-squares solution for [B; 0] is [X; 0] with the
    ragged factorization's X and residual."""
    m, n, b, eps = 300, 170, 32, 1e-8
    A, blr = ragged_kernel_blr(6, m, n, b, eps, 16)
    At = blr.to_dense()
    f = mod.factor(blr, eps, 16)
    Ap = embed_ragged(At, b)
    fp = mod.factor(blrmat.compress(Ap, b, 1e-15, b, np.zeros((Ap.shape[0] // b, Ap.shape[1] // b), bool)),
                    1e-15, b)
    Rp = fp.r_dense()
    kappa = np.linalg.cond(At)
    assert metrics.r_rel_diff(Rp[:n, :n], f.r_dense()) <= 10 * kappa * eps
    assert np.allclose(np.abs(np.diag(Rp)[n:]), 1.0) and np.all(Rp[:n, n:] == 0.0)
    Bm = synth.rhs(6, m, 2)
    Bp = np.zeros((Ap.shape[0], 2))
    Bp[:m] = Bm
    Xp = fp.lstsq(Bp)
    X = f.lstsq(Bm)
    assert np.linalg.norm(Xp[n:]) <= 1e-12 * np.linalg.norm(X)
    assert np.linalg.norm(Xp[:n] - X) <= 10 * kappa * eps * np.linalg.norm(X)
