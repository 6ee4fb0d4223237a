"""GPU parity when the tile size b does not divide m or n (the rectangular edge
blocks Section 3.1 allows).  The library factors the embedding
[A 0; 0 E] (whole tiles, E an identity block in the padded columns); the
oracle takes the narrower edge tiles directly.  Compared: R (the leading
n x n block of the embedding's R) up to row signs, Q1^T B, the least-squares
solution, products with A~ and R, compression of a ragged kernel matrix, and
the batched factor and solve with a ragged member."""
import numpy as np
import pytest

import synth
from oracle import blockcol, blrmat, metrics, tiled
from tests.blr_helpers import export_dense, export_r, gpu_import

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def P():
    import paper_2208_06194_amd as P
    assert torch.cuda.is_available()
    return P


def ceil_div(a, b):
    return -(-a // b)


def ragged_kernel_blr(seed, m, n, b, eps, cap, rule, kern, dim):
    x, y = synth.kernel_points(seed, m, n, dim)
    A = blrmat.kernel_matrix(x, y, kern)
    mask = blrmat.lowrank_mask(x, y, b, rule, ceil_div(m, b), ceil_div(n, b))
    return x, y, A, blrmat.compress(A, b, eps, cap, mask)


def padded(B, rows):
    out = np.zeros((rows, B.shape[1]))
    out[:B.shape[0]] = B
    return out


SHAPES = [
    # (m, n, b): the identity block of the padded columns sits in the padded
    # rows of the last tile row, needs one more tile row, or reaches the
    # diagonal tile row; m a multiple of b with ragged n; square
    (200, 150, 64),
    (100, 90, 64),
    (192, 130, 64),
    (330, 200, 32),
    (150, 150, 64),
]


@pytest.mark.parametrize("variant", ["tiled", "block_column"])
@pytest.mark.parametrize("shape", SHAPES)
def test_ragged_all_dense_matches_oracle_and_lapack(P, variant, shape):
    m, n, b = shape
    print("case: ragged all dense", variant, shape, flush=True)
    A = np.random.default_rng(m * n + b).standard_normal((m, n))
    blr = blrmat.compress(A, b, 1e-12, b, np.zeros((ceil_div(m, b), ceil_div(n, b)), bool))
    mod = tiled if variant == "tiled" else blockcol
    f = mod.factor(blr, 1e-12, b)
    G = gpu_import(P, blr, 1e-12, b)
    inf = G.info()
    assert (inf["m"], inf["n"], inf["p"], inf["q"]) == (m, n, ceil_div(m, b), ceil_div(n, b))
    assert inf["m_pad"] % b == 0 and inf["n_pad"] == ceil_div(n, b) * b
    assert inf["m_pad"] - m >= inf["n_pad"] - n
    G.factor(variant)
    ex = G.export()
    Rg, Ro = export_r(ex), f.r_dense()
    kappa = np.linalg.cond(A)
    tol = 10 * n * U * kappa
    assert Rg.shape == (n, n)
    assert metrics.r_rel_diff(Rg, Ro) <= tol
    assert metrics.r_rel_diff(Rg, np.linalg.qr(A, mode="r")) <= tol
    # Q1^T B through the embedding's Q on [B; 0], up to the row signs of R
    Bh = synth.rhs(3, m, 3)
    QtB = G.apply_qt(torch.tensor(padded(Bh, inf["m_pad"]), device="cuda")).cpu().numpy()
    d = np.sign(np.diag(Rg)) * np.sign(np.diag(Ro))
    assert np.allclose(d[:, None] * QtB[:n], f.apply_qt(Bh)[:n], atol=tol * np.abs(Bh).max())
    # the rest of Q^T [B; 0] has the norm of B's component off range(A)
    res_o = np.linalg.norm(f.apply_qt(Bh)[n:], axis=0)
    assert np.allclose(np.linalg.norm(QtB[n:], axis=0), res_o, atol=tol * np.linalg.norm(Bh))
    # least squares: n rows out of m rows in
    X, res = G.lstsq(torch.tensor(Bh, device="cuda"), with_resid=True)
    X, res = X.cpu().numpy(), res.cpu().numpy()
    Xl = np.linalg.lstsq(A, Bh, rcond=None)[0]
    assert X.shape == (n, 3)
    assert np.linalg.norm(X - Xl) / np.linalg.norm(Xl) <= 10 * n * U * kappa ** 2
    assert np.allclose(res, np.linalg.norm(Bh - A @ X, axis=0), rtol=1e-8, atol=1e-12)
    # products and R solves on the caller's rows
    Xp = synth.rhs(4, n, 2)
    Rx = G.matmul(torch.tensor(Xp, device="cuda"), "R").cpu().numpy()
    assert np.allclose(Rx, Rg @ Xp, atol=1e-12 * np.abs(Rg).max() * np.abs(Xp).sum(axis=0).max())
    Y = G.rsolve(torch.tensor(Rx, device="cuda")).cpu().numpy()
    assert np.linalg.norm(Y - Xp) <= 10 * n * U * kappa * np.linalg.norm(Xp)


@pytest.mark.parametrize("variant", ["tiled", "block_column"])
@pytest.mark.parametrize("case", [
    # (seed, m, n, b, eps, cap, rule, kernel, dim): low-rank tiles on the edges
    (4, 300, 170, 32, 1e-8, 16, "adjacent", "log2d", 2),
    (7, 1000, 500, 64, 1e-8, 32, "weak", "log2d", 2),
])
def test_ragged_kernel_blr_matches_oracle(P, variant, case):
    seed, m, n, b, eps, cap, rule, kern, dim = case
    print("case: ragged kernel", variant, case, flush=True)
    x, y, A, blr = ragged_kernel_blr(seed, m, n, b, eps, cap, rule, kern, dim)
    assert np.any(blr.fmt[-1] == 1) and np.any(blr.fmt[:, -1] == 1)
    At = blr.to_dense()
    mod = tiled if variant == "tiled" else blockcol
    f = mod.factor(blr, eps, cap)
    G = gpu_import(P, blr, eps, cap)
    assert np.allclose(G.matmul(torch.tensor(np.eye(n), device="cuda"), "A").cpu().numpy(), At, atol=1e-13)
    G.factor(variant, keep_a=True)
    ex = G.export()
    # the caller's tiles keep the oracle's formats, edge tiles too, except in
    # the last tile column: there the embedding stores tiles holding its
    # identity entries dense, and OP1 may then make more of that column dense
    assert np.array_equal(ex["fmt"][:, :-1], f.A.fmt[:, :-1])
    assert np.all(ex["fmt"][:, -1] <= f.A.fmt[:, -1])
    Rg, Ro = export_r(ex), f.r_dense()
    kappa = np.linalg.cond(At)
    rel = metrics.r_rel_diff(Rg, Ro)
    print(f"kappa {kappa:.1e} R vs oracle {rel:.2e}", flush=True)
    assert rel <= 10 * kappa * eps
    Bh = synth.rhs(seed, m, 4)
    X = G.lstsq(torch.tensor(Bh, device="cuda")).cpu().numpy()
    Xo = f.lstsq(Bh)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 10 * kappa * eps
    assert np.all(metrics.eta_ne(At, X, Bh) <= 1e3 * n * U * kappa)
    # refinement through the kept copy of A~ (FP64 residuals) removes the
    # recompression error of the factor from the solution: the normal
    # equations of A~ itself hold to the rounding level
    Xr = G.lstsq(torch.tensor(Bh, device="cuda"), max_refine=5).cpu().numpy()
    eta = metrics.eta_ne(At, Xr, Bh)
    print("eta_NE unrefined", metrics.eta_ne(At, X, Bh).max(), "refined", eta.max(), flush=True)
    assert np.all(eta <= 1e3 * n * U)


def test_ragged_compression_matches_oracle(P):
    """blr_compress of a kernel matrix with m, n not multiples of b: the
    partial last clusters' boxes give the oracle's admissibility, every tile
    is within eps of A, and A~ X agrees with the dense product."""
    m, n, b, eps, cap = 1000, 500, 64, 1e-8, 32
    print("case: ragged compression", flush=True)
    x, y, A, blr = ragged_kernel_blr(9, m, n, b, eps, cap, "adjacent", "log2d", 2)
    G = P.BLRMatrix.compress_kernel(torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda"), "log2d", b,
                                    eps, cap, admissibility="adjacent")
    ex = G.export()
    mask = blrmat.lowrank_mask(x, y, b, "adjacent", ceil_div(m, b), ceil_div(n, b))
    lr = ex["fmt"] == 1
    # low-rank only where the rule allows it; outside the last tile column
    # (where tiles holding the embedding's identity entries are dense) the
    # formats are the oracle's, except where a rank sits at the cap (the
    # randomized range finder and the exact SVD may then decide differently)
    assert not np.any(lr & ~mask)
    near_cap = np.zeros_like(lr)
    for (i, j), Ut in blr.U.items():
        near_cap[i, j] = Ut.shape[1] >= cap - 1
    differ = (lr != (blr.fmt == 1))[:, :-1] & ~near_cap[:, :-1] & mask[:, :-1]
    assert not np.any(differ)
    Ag = export_dense(ex)
    assert Ag.shape == (m, n)
    for i in range(ceil_div(m, b)):
        for j in range(ceil_div(n, b)):
            blk = np.s_[i * b:(i + 1) * b, j * b:(j + 1) * b]
            assert np.linalg.norm(Ag[blk] - A[blk]) <= eps * np.linalg.norm(A[blk]) * (1 + 1e-6)
    Xp = synth.rhs(10, n, 3)
    Y = G.matmul(torch.tensor(Xp, device="cuda"), "A").cpu().numpy()
    assert np.linalg.norm(Y - A @ Xp) <= 2 * eps * np.linalg.norm(A) * np.linalg.norm(Xp)
    Yt = G.matmul(torch.tensor(synth.rhs(11, m, 2), device="cuda"), "AT").cpu().numpy()
    assert np.linalg.norm(Yt - A.T @ synth.rhs(11, m, 2)) <= 2 * eps * np.linalg.norm(A) * np.linalg.norm(
        synth.rhs(11, m, 2))
    G.factor("block_column")
    X = G.lstsq(torch.tensor(synth.rhs(12, m, 2), device="cuda")).cpu().numpy()
    assert np.all(metrics.eta_ne(Ag, X, synth.rhs(12, m, 2)) <= 1e-6)


def test_ragged_dense_source_compression(P):
    """blr_compress of a dense m x n device matrix, m and n not multiples of
    b, weak admissibility: every tile within eps of A, the padded rows and
    columns never read (A is passed with lda = m)."""
    m, n, b, eps, cap = 333, 205, 64, 1e-8, 32
    print("case: ragged dense source", flush=True)
    x, y = synth.kernel_points(13, m, n, 2)
    A = blrmat.kernel_matrix(x, y, "log2d")
    G = P.BLRMatrix.compress_dense(torch.tensor(A, device="cuda"), b, eps, cap, admissibility="weak")
    ex = G.export()
    assert ex["fmt"].shape == (ceil_div(m, b), ceil_div(n, b)) and np.any(ex["fmt"] == 1)
    Ag = export_dense(ex)
    for i in range(ceil_div(m, b)):
        for j in range(ceil_div(n, b)):
            blk = np.s_[i * b:(i + 1) * b, j * b:(j + 1) * b]
            assert np.linalg.norm(Ag[blk] - A[blk]) <= eps * np.linalg.norm(A[blk]) * (1 + 1e-6)
    G.factor("tiled")
    Bh = synth.rhs(14, m, 2)
    X = G.lstsq(torch.tensor(Bh, device="cuda")).cpu().numpy()
    assert np.all(metrics.eta_ne(Ag, X, Bh) <= 1e-6)


def test_ragged_member_in_batches_is_bitwise_equal_to_single(P):
    """A batch with ragged and whole-tile members: the batched factor and
    solve give each member exactly its single-matrix result."""
    print("case: ragged batch", flush=True)
    mats = [(5, 700, 300), (6, 512, 256), (8, 450, 450)]
    blrs = []
    for seed, m, n in mats:
        _, _, _, blr = ragged_kernel_blr(seed, m, n, 64, 1e-8, 32, "adjacent", "log2d", 2)
        blrs.append(blr)
    single = [gpu_import(P, blr, 1e-8, 32).factor("block_column") for blr in blrs]
    batch = P.factor_batch([gpu_import(P, blr, 1e-8, 32) for blr in blrs])
    Bs = [torch.tensor(synth.rhs(20 + i, blr.m, 3), device="cuda") for i, blr in enumerate(blrs)]
    Xs = P.lstsq_batch(batch, Bs)
    for G1, G2, B, X in zip(single, batch, Bs, Xs):
        e1, e2 = G1.export(with_factor=True), G2.export(with_factor=True)
        for k in ("fmt", "rank", "dense", "U", "V", "Y", "T"):
            assert np.array_equal(e1[k], e2[k]), k
        assert torch.equal(G1.lstsq(B), X)


def test_ragged_restrictions(P):
    m, n, b = 200, 150, 64
    A = np.random.default_rng(1).standard_normal((m, n))
    blr = blrmat.compress(A, b, 1e-12, b, np.zeros((4, 3), bool))
    G = gpu_import(P, blr, 1e-12, b)
    G.factor("block_column", keep_a=True)
    with pytest.raises(P.BLRError) as e:
        G.form_q()
    assert e.value.status == 1
    B = torch.tensor(synth.rhs(1, m, 1), device="cuda")
    X = G.lstsq(B)
    with pytest.raises(P.BLRError) as e:
        G.lstsq_adjoint(B, X, torch.ones_like(X))
    assert e.value.status == 1
    # Q^T B needs the embedding's rows
    with pytest.raises(P.BLRError) as e:
        G.apply_qt(B)
    assert e.value.status == 1
