"""GPU parity at the shapes the benchmark runs, each against the FP64 oracle on
the same seeded, oracle-compressed input:

* the 2D log-kernel workload at its exact size and options (2048 x 1024,
  b = 128, adjacent boxes dense, eps 1e-8, rank cap 16), both variants and
  both overflow policies, with R also against LAPACK's QR of A~;
* a tile size of 1024 in both variants (the tiled TPQRT on tiles taller than
  512 rows with 16-column inner panels, the block-column panel of eight
  128-column reflector blocks);
* the mixed form (FP32 matrix-core products, FP64 reflectors) on block
  columns taller than 1024 rows, where products with K > 1024 add their FP32
  partial sums into FP64 every 1024 of K, at the mixed tolerance 1e-6 and at
  the FP64 tolerance 1e-8, with its error against the FP64 oracle stated.

Bounds (the arithmetic behind each is in the test that uses it):
* FP64, no truncation at the cap: R within 10 kappa eps of the oracle's, up
  to row signs (R is unique up to row signs; a perturbation of relative size
  d moves it by about kappa d), Res~ <= 10 eps.
* Mixed: the backward error of an FP32 product with K-term sums of at most
  1024 is about sqrt(1024) u32 relative to |A||B|; q block steps compound it:
  Res~ <= 10 eps + q sqrt(1024) u32, and R within 10 kappa max(eps, Res~).
"""
import numpy as np
import pytest

from oracle import blockcol, metrics, tiled
from tests.blr_helpers import export_r, gpu_import, kernel_blr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U = np.finfo(np.float64).eps
U32 = float(np.finfo(np.float32).eps) / 2


@pytest.fixture(scope="module")
def P():
    import paper_2208_06194_amd as P
    assert torch.cuda.is_available()
    return P


def gpu_res_orth(G, At, m, n):
    """Res~ = ||Q R - A~||_F / ||A~||_F and Orth = ||Q1^T Q1 - I||_F / sqrt(n),
    with Q applied by the library to [R; 0] and to [I; 0]."""
    Rg = export_r(G.export())
    RR = np.zeros((m, n))
    RR[:n] = Rg
    QR = G.apply_qt(torch.tensor(RR, device="cuda"), trans=True).cpu().numpy()
    res = float(np.linalg.norm(QR - At) / np.linalg.norm(At))
    E = np.zeros((m, n))
    E[:n] = np.eye(n)
    Q1 = G.apply_qt(torch.tensor(E, device="cuda"), trans=True)
    orth = float(torch.linalg.norm(Q1.T @ Q1 - torch.eye(n, dtype=torch.float64, device="cuda"))) / np.sqrt(n)
    return Rg, res, orth


@pytest.mark.parametrize("variant", ["tiled", "block_column"])
@pytest.mark.parametrize("overflow", ["dense", "truncate"])
def test_log2d_workload_exact_config(P, variant, overflow):
    """2048 x 1024 points in the unit square (seed 0, Morton sorted),
    A_ij = -log(|x_i - y_j| + 1e-3), b = 128 (16 x 8 tiles), tiles of adjacent
    boxes dense, the rest truncated SVD at 1e-8 with rank <= 16."""
    m, n, b, eps, cap = 2048, 1024, 128, 1e-8, 16
    print("case: log2d exact config", variant, overflow, flush=True)
    A, blr = kernel_blr(0, m, n, b, eps, cap, "log2d", 2, "adjacent", overflow=overflow)
    At = blr.to_dense()
    comp = float(np.linalg.norm(At - A) / np.linalg.norm(A))
    mod = tiled if variant == "tiled" else blockcol
    f = mod.factor(blr, eps, cap)
    G = gpu_import(P, blr, eps, cap)
    G.factor(variant)
    ex = G.export()
    info = G.info()
    Rg, res, orth = gpu_res_orth(G, At, m, n)
    Ro = f.r_dense()
    res_o = metrics.res(f, At)
    kappa = np.linalg.cond(At)
    rel_o = metrics.r_rel_diff(Rg, Ro)
    rel_l = metrics.r_rel_diff(Rg, np.linalg.qr(At, mode="r"))
    res_a = float(np.linalg.norm(f.q_times_r() - A) / np.linalg.norm(A))
    print(f"{variant} overflow={overflow}: dense {int((blr.fmt == 0).sum())} low-rank {int((blr.fmt == 1).sum())} "
          f"||A~-A||/||A|| {comp:.2e} kappa {kappa:.1e}; Res~ GPU {res:.2e} oracle {res_o:.2e}; Res_A (oracle "
          f"factor) {res_a:.2e}; Orth GPU {orth:.2e}; R vs oracle {rel_o:.2e} vs LAPACK {rel_l:.2e}; truncations "
          f"GPU {info['factor_overflow']} oracle {f.stats.overflow}", flush=True)
    # the same fill-in decisions (OP1: a dense term makes the sum dense)
    assert np.array_equal(ex["fmt"], f.A.fmt)
    # Q is a product of FP64 Householder reflectors with orthonormal U bases
    assert orth <= 1e2 * np.sqrt(n) * U
    if info["factor_overflow"] == 0 and f.stats.overflow == 0:
        assert res <= 10 * eps and res_o <= 10 * eps
        assert rel_o <= 10 * kappa * eps
        assert rel_l <= 10 * kappa * eps
    else:
        # both sides truncate fill-in at the cap: the factorization error is
        # the dropped tail, of the same size on both sides
        assert res <= 2.0 * res_o + 10 * eps
        assert rel_o <= 10 * kappa * max(eps, res_o)
    # Res against the uncompressed A: compression error plus factorization error
    assert res_a <= 10 * max(eps, comp, res_o)


_ORACLE = {}


def oracle_case(variant, seed, m, n, b, eps, cap, kern="inv_r", dim=3, rule="dist_gt_diam"):
    """(A, compressed A~, oracle factor of A~), computed once per module."""
    key = (variant, seed, m, n, b, eps, cap, kern, dim, rule)
    if key not in _ORACLE:
        A, blr = kernel_blr(seed, m, n, b, eps, cap, kern, dim, rule)
        mod = tiled if variant == "tiled" else blockcol
        _ORACLE[key] = (A, blr, mod.factor(blr, eps, cap))
    return _ORACLE[key]


@pytest.mark.parametrize("variant", ["tiled", "block_column"])
def test_tile_size_1024_matches_oracle(P, variant):
    """4096 x 2048 points in the unit cube, 1/(r + 1e-3), b = 1024 (4 x 2
    tiles); at this size every tile is within a box diameter of the others,
    so the matrix is all dense (the dense reduction of both variants)."""
    m, n, b, eps, cap = 4096, 2048, 1024, 1e-8, 50
    print("case: b=1024", variant, flush=True)
    A, blr, f = oracle_case(variant, 12, m, n, b, eps, cap)
    G = gpu_import(P, blr, eps, cap)
    G.factor(variant)
    ex = G.export(with_factor=True)
    At = blr.to_dense()
    kappa = np.linalg.cond(At)
    tol = 10 * n * U * kappa
    Rg, Ro = export_r(ex), f.r_dense()
    rel = metrics.r_rel_diff(Rg, Ro)
    print(f"b=1024 {variant}: tiles dense {int((blr.fmt == 0).sum())}/{blr.p * blr.q}, kappa {kappa:.1e}, "
          f"R vs oracle {rel:.2e} (bound {tol:.1e})", flush=True)
    assert rel <= tol
    assert metrics.r_rel_diff(Rg, np.linalg.qr(At, mode="r")) <= tol
    Bh = np.random.default_rng(3).standard_normal((m, 4))
    QtB = G.apply_qt(torch.tensor(Bh, device="cuda")).cpu().numpy()
    QtB_o = f.apply_qt(Bh)
    # Q1^T B is unique up to the row signs of R (Q1 = A~ R^-1); of the rest
    # only the column norms are (||(Q^T B)[n:]|| = ||(I - Q1 Q1^T) B||)
    d = np.sign(np.diag(Rg)) * np.sign(np.diag(Ro))
    assert np.allclose(d[:, None] * QtB[:n], QtB_o[:n], atol=tol * np.abs(Bh).max())
    assert np.allclose(np.linalg.norm(QtB[n:], axis=0), np.linalg.norm(QtB_o[n:], axis=0), rtol=tol)
    if variant == "block_column":
        # the reflectors of each full-rank stack [A_kk; A_k+1,k; ...] and T_k
        # element by element (both sides take the larfg sign).  The tiled
        # variant's first reflectors come from the QR of the square diagonal
        # tile alone, whose last columns are numerically dependent at this
        # size: their reflectors are fixed by rounding and only R and the
        # products above are compared.
        for k in range(f.q):
            assert np.allclose(np.tril(ex["dense"][k, k], -1), np.tril(f.A.D[(k, k)], -1), atol=10 * tol)
            for i in range(k + 1, f.p):
                assert np.allclose(ex["dense"][i, k], f.A.D[(i, k)], atol=10 * tol)
            assert np.allclose(ex["T"][k, k], f.Tk[k], atol=10 * tol * np.abs(f.Tk[k]).max())


MIXED_CASES = [
    # (variant, seed, m, n, b, cap, kernel, dim, rule)
    # all dense: the first stack holds 4096 rows, so Z_j sums K = 4096 terms
    ("block_column", 13, 4096, 1024, 256, 32, "inv_r", 3, "dist_gt_diam"),
    # weak admissibility on the 2D log kernel: 41 (eps 1e-6) or 28 (1e-8)
    # low-rank tiles whose bases the FP32 products update
    ("block_column", 13, 4096, 1024, 256, 32, "log2d", 2, "weak"),
    # b = 1024: eight-block panels, K up to 4096
    ("block_column", 12, 4096, 2048, 1024, 50, "inv_r", 3, "dist_gt_diam"),
    ("tiled", 13, 4096, 1024, 256, 32, "log2d", 2, "weak"),
]


@pytest.mark.parametrize("eps", [1e-6, 1e-8])
@pytest.mark.parametrize("case", MIXED_CASES)
def test_mixed_against_fp64_oracle(P, case, eps):
    """The mixed form (FP32 matrix-core products, FP64 panels, T and
    recompression) of the same compressed matrix as the FP64 oracle's."""
    variant, seed, m, n, b, cap, kern, dim, rule = case
    print("case: mixed vs FP64 oracle", case, eps, flush=True)
    A, blr, f = oracle_case(variant, seed, m, n, b, eps, cap, kern, dim, rule)
    At = blr.to_dense()
    G = gpu_import(P, blr, eps, cap)
    G.factor(variant, precision="mixed")
    Rg, res, orth = gpu_res_orth(G, At, m, n)
    Ro = f.r_dense()
    res_o = metrics.res(f, At)
    kappa = np.linalg.cond(At)
    rel = metrics.r_rel_diff(Rg, Ro)
    q = n // b
    bound = 10 * eps + q * np.sqrt(1024) * U32
    print(f"mixed {variant} {m}x{n} b={b} eps={eps:g}: low-rank tiles {int((blr.fmt == 1).sum())}; Res~ mixed "
          f"{res:.2e} (FP64 oracle {res_o:.2e}, bound {bound:.1e}); Orth mixed {orth:.2e}; R vs FP64 oracle "
          f"{rel:.2e} (kappa {kappa:.1e})", flush=True)
    assert res <= bound
    assert rel <= 10 * kappa * max(eps, res)
    # the reflectors are FP64; low-rank bases updated by FP32 products are
    # orthonormal to about u32 only, which reaches Q through U Y
    assert orth <= q * np.sqrt(1024) * U32
