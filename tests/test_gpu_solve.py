"""GPU: least squares, mixed precision, prefix factorization, error paths and
edge cases, each against the oracle on the same seeded inputs."""
import numpy as np
import pytest

import synth
from oracle import blockcol, blrmat, metrics, tiled
from oracle.blrmat import LOWRANK
from oracle.factor import SingularR
from tests.blr_helpers import blr_to_host, export_r

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U = np.finfo(np.float64).eps


@pytest.fixture(scope="module")
def P():
    import paper_2208_06194_amd as P
    return P


def gpu_import(P, blr, eps, cap):
    fmt, rank, dense, Uh, Vh = blr_to_host(blr, cap)
    return P.BLRMatrix.import_tiles(blr.m, blr.n, blr.b, eps, cap, fmt, rank, dense, Uh, Vh)


def kernel_blr(seed, m, n, b, eps, cap, kern="inv_r", dim=3, rule="dist_gt_diam"):
    x, y = synth.kernel_points(seed, m, n, dim)
    A = blrmat.kernel_matrix(x, y, kern)
    mask = blrmat.lowrank_mask(x, y, b, rule, m // b, n // b)
    return A, blrmat.compress(A, b, eps, cap, mask)


@pytest.mark.parametrize("rule,kern,dim", [("dist_gt_diam", "inv_r", 3), ("adjacent", "log2d", 2), ("weak", "log2d", 2)])
def test_lstsq_matches_oracle(P, rule, kern, dim):
    print("case: lstsq", rule, flush=True)
    m, n, b, eps, cap = 512, 256, 64, 1e-8, 32
    A, blr = kernel_blr(3, m, n, b, eps, cap, kern, dim, rule)
    At = blr.to_dense()
    f = tiled.factor(blr, eps, cap)
    Bh = synth.rhs(3, m, 5)
    Xo = f.lstsq(Bh)
    G = gpu_import(P, blr, eps, cap)
    G.factor("tiled")
    X, res = G.lstsq(torch.tensor(Bh, device="cuda"), with_resid=True)
    X, res = X.cpu().numpy(), res.cpu().numpy()
    kappa = np.linalg.cond(At)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 10 * kappa * eps
    # residual norms reported by the library are those of the computed solution
    r_true = np.linalg.norm(Bh - f.q_times_r() @ X, axis=0)
    assert np.allclose(res, r_true, rtol=1e-6)
    # normal-equation optimality for the factored matrix
    assert np.all(metrics.eta_ne(f.q_times_r(), X, Bh) <= 1e3 * n * U)


@pytest.mark.parametrize("variant", ["tiled", "block_column"])
def test_lstsq_many_rhs_ragged_blocks(P, variant):
    """20 right-hand sides (two groups of the triangular solve: 16 and 4) and
    b = 96 (a full and a ragged 64-row block per diagonal tile)."""
    print("case: lstsq 20 rhs b 96", variant, flush=True)
    m, n, b, eps, cap = 768, 384, 96, 1e-8, 32
    A, blr = kernel_blr(21, m, n, b, eps, cap)
    At = blr.to_dense()
    mod = tiled if variant == "tiled" else blockcol
    f = mod.factor(blr, eps, cap)
    Bh = synth.rhs(21, m, 20)
    Xo = f.lstsq(Bh)
    G = gpu_import(P, blr, eps, cap)
    G.factor(variant)
    X = G.lstsq(torch.tensor(Bh, device="cuda")).cpu().numpy()
    kappa = np.linalg.cond(At)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 10 * kappa * eps
    assert np.all(metrics.eta_ne(f.q_times_r(), X, Bh) <= 1e3 * n * U)


def test_lstsq_dense_matches_lapack(P):
    print("case: lstsq dense", flush=True)
    m, n, b = 384, 192, 64
    A = np.random.default_rng(5).standard_normal((m, n))
    blr = blrmat.compress(A, b, 1e-12, b, np.zeros((m // b, n // b), bool))
    G = gpu_import(P, blr, 1e-12, b)
    G.factor("tiled")
    Bh = synth.rhs(5, m, 3)
    X = G.lstsq(torch.tensor(Bh, device="cuda")).cpu().numpy()
    Xr = np.linalg.lstsq(A, Bh, rcond=None)[0]
    assert np.linalg.norm(X - Xr) / np.linalg.norm(Xr) <= 100 * n * U * np.linalg.cond(A)


def test_mixed_precision_error_against_fp64_oracle(P):
    print("case: mixed", flush=True)
    m, n, b, eps, cap = 1024, 512, 256, 1e-6, 32
    A, blr = kernel_blr(4, m, n, b, eps, cap)
    At = blr.to_dense()
    f = tiled.factor(blr, eps, cap)
    G = gpu_import(P, blr, eps, cap)
    G.factor("tiled", precision="mixed")
    ex = G.export()
    Rg = export_r(ex)
    rel = metrics.r_rel_diff(Rg, f.r_dense())
    RR = np.zeros((m, n))
    RR[:n] = Rg
    QR = G.apply_qt(torch.tensor(RR, device="cuda"), trans=True).cpu().numpy()
    res = np.linalg.norm(QR - At) / np.linalg.norm(At)
    print(f"mixed: R rel diff vs FP64 oracle {rel:.2e}, Res_At {res:.2e}", flush=True)
    # FP32 products: errors of order sqrt(b) * 2^-24 per update, amplified by the conditioning
    assert res <= 1e-5
    assert rel <= 1e-3


@pytest.mark.parametrize("K", [1, 2, 3])
def test_prefix_factor_matches_oracle(P, K):
    """The first K block rows of R after K steps, up to row signs (R is unique
    up to the signs of its rows; rounding can decide a Householder sign
    differently when a pivot is small next to its column)."""
    print("case: prefix", K, flush=True)
    m, n, b, eps, cap = 512, 256, 64, 1e-8, 16
    A, blr = kernel_blr(6, m, n, b, eps, cap, "log2d", 2, "adjacent")
    f = tiled.factor(blr, eps, cap, stop_after_k=K)
    G = gpu_import(P, blr, eps, cap)
    G.factor("tiled", stop_after_k=K)
    ex = G.export()
    Rg, Ro = np.zeros((K * b, n)), np.zeros((K * b, n))
    for k in range(K):
        for j in range(k, f.q):
            o = f.r_val(k, j)
            Ro[k * b:(k + 1) * b, j * b:(j + 1) * b] = o[1] if o[0] == "D" else o[1] @ o[2].T
            if j == k:
                g = np.triu(ex["dense"][k, k])
            elif ex["fmt"][k, j] == 0:
                g = ex["dense"][k, j]
            else:
                r = ex["rank"][k, j]
                g = ex["U"][k, j][:, :r] @ ex["V"][k, j][:, :r].T
            Rg[k * b:(k + 1) * b, j * b:(j + 1) * b] = g
    sg = np.sign(np.diag(Rg[:, :K * b])) * np.sign(np.diag(Ro[:, :K * b]))
    rel = np.linalg.norm(sg[:, None] * Rg - Ro) / np.linalg.norm(Ro)
    assert rel <= 10 * np.linalg.cond(blr.to_dense()) * eps


def test_zero_tiles_have_rank_zero(P):
    """Weak admissibility on a block-diagonal matrix: every off-diagonal tile is
    the zero matrix, compressed to rank 0; R is the block-diagonal R."""
    print("case: rank0", flush=True)
    m, n, b = 256, 128, 32
    A = np.zeros((m, n))
    rng = np.random.default_rng(2)
    for k in range(n // b):
        A[k * b:(k + 1) * b, k * b:(k + 1) * b] = rng.standard_normal((b, b))
    G = P.BLRMatrix.compress_dense(torch.tensor(A, device="cuda"), b, 1e-8, 16, admissibility="weak")
    ex = G.export()
    assert np.all(ex["rank"][ex["fmt"] == 1] == 0)
    G.factor("tiled")
    Rg = export_r(G.export())
    assert metrics.r_rel_diff(Rg, np.linalg.qr(A, mode="r")) <= 1e-12


def test_truncate_overflow_is_counted(P):
    print("case: truncate", flush=True)
    m, n, b = 256, 128, 32
    A = np.random.default_rng(3).standard_normal((m, n))   # full-rank tiles
    G = P.BLRMatrix.compress_dense(torch.tensor(A, device="cuda"), b, 1e-8, 4, admissibility="weak",
                                   overflow="truncate")
    inf = G.info()
    assert inf["compress_overflow"] == inf["n_lowrank"] > 0
    Gd = P.BLRMatrix.compress_dense(torch.tensor(A, device="cuda"), b, 1e-8, 4, admissibility="weak",
                                    overflow="dense")
    assert Gd.info()["n_lowrank"] == 0


def test_error_paths(P):
    print("case: errors", flush=True)
    from paper_2208_06194_amd import BLRError
    m, n, b = 128, 64, 32
    A = np.random.default_rng(1).standard_normal((m, n))
    At = torch.tensor(A, device="cuda")
    G = P.BLRMatrix.compress_dense(At, b, 1e-8, 8, admissibility="weak")
    with pytest.raises(BLRError) as e:
        G.apply_qt(torch.zeros((m, 1), dtype=torch.float64, device="cuda"))
    assert e.value.status == 2
    G.factor("tiled")
    with pytest.raises(BLRError) as e:
        G.factor("tiled")
    assert e.value.status == 2
    bad = At.clone()
    bad[3, 4] = float("nan")
    with pytest.raises(BLRError) as e:
        P.BLRMatrix.compress_dense(bad, b, 1e-8, 8)
    assert e.value.status == 5
    Z = A.copy()
    Z[:, 7] = 0.0
    Gz = P.BLRMatrix.compress_dense(torch.tensor(Z, device="cuda"), b, 1e-8, 8, admissibility="mask",
                                    mask=np.zeros((m // b, n // b), bool))
    Gz.factor("tiled")
    with pytest.raises(BLRError) as e:
        Gz.lstsq(torch.ones((m, 1), dtype=torch.float64, device="cuda"))
    assert e.value.status == 6


@pytest.mark.parametrize("m,n,b", [(64, 64, 64), (128, 128, 32), (512, 64, 64)])
def test_shapes_single_tile_square_and_single_column(P, m, n, b):
    print("case: shape", m, n, b, flush=True)
    A = np.random.default_rng(m + n).standard_normal((m, n))
    G = P.BLRMatrix.compress_dense(torch.tensor(A, device="cuda"), b, 1e-12, min(b, 64),
                                   admissibility="mask", mask=np.zeros((m // b, n // b), bool))
    G.factor("tiled")
    assert metrics.r_rel_diff(export_r(G.export()), np.linalg.qr(A, mode="r")) <= 100 * n * U * np.linalg.cond(A)


@pytest.mark.parametrize("rule,kern,dim", [("dist_gt_diam", "inv_r", 3), ("weak", "log2d", 2)])
def test_matmul_matches_host_products(P, rule, kern, dim):
    """blr_matmul: A~ X and A~^T X before the factorization, R X after it,
    against host products with the densified tiles."""
    print("case: matmul", rule, flush=True)
    m, n, b, eps, cap = 512, 256, 64, 1e-8, 32
    A, blr = kernel_blr(8, m, n, b, eps, cap, kern, dim, rule)
    At = blr.to_dense()
    G = gpu_import(P, blr, eps, cap)
    X = synth.rhs(8, n, 5)
    Xm = synth.rhs(9, m, 3)
    Y = G.matmul(torch.tensor(X, device="cuda"), "A").cpu().numpy()
    assert np.linalg.norm(Y - At @ X) <= 1e-13 * np.linalg.norm(At) * np.linalg.norm(X)
    Yt = G.matmul(torch.tensor(Xm, device="cuda"), "AT").cpu().numpy()
    assert np.linalg.norm(Yt - At.T @ Xm) <= 1e-13 * np.linalg.norm(At) * np.linalg.norm(Xm)
    with pytest.raises(P.BLRError):
        G.matmul(torch.tensor(X, device="cuda"), "R")      # not factored yet
    G.factor("block_column")
    Rg = export_r(G.export())
    YR = G.matmul(torch.tensor(X, device="cuda"), "R").cpu().numpy()
    assert np.linalg.norm(YR - Rg @ X) <= 1e-13 * np.linalg.norm(Rg) * np.linalg.norm(X)
    with pytest.raises(P.BLRError):
        G.matmul(torch.tensor(X, device="cuda"), "A")      # A~ was overwritten


@pytest.mark.parametrize("variant", ["tiled", "block_column"])
def test_refinement_recovers_fp64_accuracy_from_mixed_factor(P, variant):
    """Least squares on a mixed-precision factor (FP32 MFMA updates): refining
    the augmented system with FP64 residuals through the kept copy of A~
    brings the solution from the FP32 level to the FP64 level of the exact
    least-squares solution of A~ (LAPACK on the densified A~)."""
    print("case: refinement", variant, flush=True)
    m, n, b, eps, cap = 1024, 512, 128, 1e-10, 32
    A, blr = kernel_blr(12, m, n, b, eps, cap)
    At = blr.to_dense()
    Bh = synth.rhs(12, m, 3)
    Xr = np.linalg.lstsq(At, Bh, rcond=None)[0]
    kappa = np.linalg.cond(At)
    G = gpu_import(P, blr, eps, cap)
    G.factor(variant, precision="mixed", keep_a=True)
    Bd = torch.tensor(Bh, device="cuda")
    X0 = G.lstsq(Bd).cpu().numpy()
    e0 = np.linalg.norm(X0 - Xr) / np.linalg.norm(Xr)
    X1, res = G.lstsq(Bd, with_resid=True, max_refine=10)
    X1, res = X1.cpu().numpy(), res.cpu().numpy()
    e1 = np.linalg.norm(X1 - Xr) / np.linalg.norm(Xr)
    print(f"kappa {kappa:.2e}  unrefined {e0:.2e}  refined {e1:.2e}", flush=True)
    assert e1 <= 100 * n * U * kappa
    assert e1 <= e0 * 1e-3
    # the reported residual norms are those of the refined solution
    assert np.allclose(res, np.linalg.norm(Bh - At @ X1, axis=0), rtol=1e-8)
    # products with A~ still work after the in-place factorization
    Xp = synth.rhs(13, n, 2)
    Y = G.matmul(torch.tensor(Xp, device="cuda"), "A").cpu().numpy()
    assert np.linalg.norm(Y - At @ Xp) <= 1e-13 * np.linalg.norm(At) * np.linalg.norm(Xp)


def test_refinement_stops_when_corrections_stop_halving(P):
    """A matrix with kappa = 1e9 (singular values geometric from 1 to 1e-9,
    all tiles dense) factored in the mixed form: kappa u32 >> 1, so the
    corrections from the FP32-updated factor need not contract.  A
    correction larger than half the previous one taken is dropped and the
    column stops with its iterate, so whatever follows the first step adds
    at most dx_1 (1/2 + 1/4 + ...): ||x_10 - x_1|| <= ||x_1 - x_0|| per
    column (without the rule a diverging iteration keeps adding growing
    corrections)."""
    print("case: refinement stagnation", flush=True)
    m, n, b = 512, 256, 64
    rng = np.random.default_rng(31)
    Qa, _ = np.linalg.qr(rng.standard_normal((m, n)))
    Qb, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Qa * np.logspace(0, -9, n)) @ Qb.T
    blr = blrmat.compress(A, b, 1e-12, b, np.zeros((m // b, n // b), bool))
    Bh = synth.rhs(31, m, 4)
    Xr = np.linalg.lstsq(A, Bh, rcond=None)[0]
    G = gpu_import(P, blr, 1e-12, b)
    G.factor("block_column", precision="mixed", keep_a=True)
    Bd = torch.tensor(Bh, device="cuda")
    X0 = G.lstsq(Bd).cpu().numpy()
    X1 = G.lstsq(Bd, max_refine=1).cpu().numpy()
    X10 = G.lstsq(Bd, max_refine=10).cpu().numpy()
    assert np.all(np.isfinite(X10))
    err = [np.linalg.norm(X - Xr, axis=0) / np.linalg.norm(Xr, axis=0) for X in (X0, X1, X10)]
    print("error unrefined", err[0], "after 1 step", err[1], "after up to 10", err[2], flush=True)
    d1 = np.linalg.norm(X1 - X0, axis=0)
    assert np.all(np.linalg.norm(X10 - X1, axis=0) <= d1 * (1 + 1e-9) + 1e-300)


def test_refinement_graph_replays_match_eager_steps(P):
    """The single solve captures one refinement step into a graph and replays
    it, with the step decisions and updates as ordinary launches between the
    replays; the batched solve runs the same steps as ordinary launches.
    Repeated solves on one handle (each capturing its own graph, other calls
    in between) give the batched solve's result bit for bit every time."""
    print("case: refinement graph replays", flush=True)
    m, n, b, eps, cap = 1024, 512, 128, 1e-10, 32
    A, blr = kernel_blr(15, m, n, b, eps, cap)
    G = gpu_import(P, blr, eps, cap)
    G.factor("block_column", precision="mixed", keep_a=True)
    Bd = torch.tensor(synth.rhs(15, m, 3), device="cuda")
    ref = P.lstsq_batch([G], [Bd], max_refine=6)[0]
    for _ in range(3):
        X = G.lstsq(Bd, max_refine=6)
        G.apply_qt(Bd)
        torch.cuda.synchronize()
        assert torch.equal(X, ref)


def test_refinement_requires_the_kept_copy(P):
    m, n, b, eps, cap = 256, 128, 64, 1e-8, 16
    A, blr = kernel_blr(14, m, n, b, eps, cap)
    G = gpu_import(P, blr, eps, cap)
    G.factor("block_column")
    with pytest.raises(P.BLRError) as e:
        G.lstsq(torch.tensor(synth.rhs(14, m, 1), device="cuda"), max_refine=2)
    assert e.value.status == 2      # BLR_ERR_STATE


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_morton_sort_matches_host_order(P, dim):
    """blr_morton_sort against the host Morton order (synth.morton_keys with a
    stable sort): bit-exact permutation, including duplicated points (ties
    keep the original order) and coordinates outside [0, 1) (clamped)."""
    print("case: morton sort", dim, flush=True)
    rng = np.random.default_rng(40 + dim)
    pts = rng.random((100003, dim))
    pts[7] = pts[3]
    pts[11] = pts[3]
    pts[20] = -0.25
    pts[21] = 1.0
    pts[22] = 1.75
    out, perm = P.morton_sort(torch.tensor(pts, device="cuda"))
    ref = np.argsort(synth.morton_keys(pts), kind="stable")
    assert np.array_equal(perm.cpu().numpy(), ref)
    assert np.array_equal(out.cpu().numpy(), pts[ref])
    # the workload generator's points come out unchanged (already in order)
    x, _ = synth.kernel_points(3, 4096, 2048, max(dim, 2))
    _, perm2 = P.morton_sort(torch.tensor(x, device="cuda"))
    assert np.array_equal(perm2.cpu().numpy(), np.arange(4096))
