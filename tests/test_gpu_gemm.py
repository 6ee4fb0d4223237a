"""The matrix-core GEMM kernel (the dominant kernel of the factorization)
against a plain numpy product, through the selftest hook, on shapes that span
several 64/128 tiles with ragged edges, every transpose and triangular mode."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def run(lib, flags, M, N, K, fp32=0, alpha=0.5, beta=2.0):
    rng = np.random.default_rng(M * N + K + flags)
    ta, tb = flags & 1, flags & 2
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C = rng.standard_normal((M, N))
    S = A
    if flags & 4:
        S = np.tril(A, -1) + np.eye(*A.shape)
    if flags & 8:
        S = A = np.triu(A)
    Aop = S.T if ta else S
    SB = np.tril(B, -1) + np.eye(*B.shape) if flags & 16 else B
    Bop = SB.T if tb else SB
    ref = alpha * Aop @ Bop + beta * C
    dA = torch.tensor(A.T.copy(), device="cuda")
    dB = torch.tensor(B.T.copy(), device="cuda")
    dC = torch.tensor(C.T.copy(), device="cuda")
    st = lib.blr_selftest_gemm(flags, M, N, K, alpha, dA.data_ptr(), A.shape[0], dB.data_ptr(), B.shape[0],
                               beta, dC.data_ptr(), M, fp32, torch.cuda.current_stream().cuda_stream)
    assert st == 0
    out = dC.cpu().numpy().T
    scale = np.abs(alpha) * np.abs(Aop) @ np.abs(Bop) + np.abs(beta * C)
    return np.max(np.abs(out - ref) / scale)


@pytest.fixture(scope="module")
def lib():
    import paper_2208_06194_amd as P
    return P.load()


SHAPES = [(16, 16, 4), (64, 64, 64), (50, 70, 33), (300, 260, 130), (256, 512, 256), (1024, 128, 1024),
          (256, 256, 272), (512, 384, 1056),  # K % 32 == 16: FP64 leaves the 32-deep fast path
          (1000, 16, 3000), (4096, 5, 1024), (130, 1, 77)]  # N <= 16: the skinny kernel (B not transposed)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_gemm_fp64(lib, shape, flags):
    print("case: gemm", shape, flags, flush=True)
    M, N, K = shape
    assert run(lib, flags, M, N, K) <= 4 * K * np.finfo(np.float64).eps


@pytest.mark.parametrize("flags", [1 | 4, 4, 1 | 8, 8, 1 | 4 | 16, 2 | 16])
@pytest.mark.parametrize("shape", [(192, 160, 192), (256, 384, 256), (320, 16, 320)])
def test_gemm_triangular_modes(lib, flags, shape):
    # 256 x 384 runs the fast full-tile kernel for the upper-triangular A modes
    print("case: gemm triangular", flags, shape, flush=True)
    assert run(lib, flags, *shape) <= 1e-13


@pytest.mark.parametrize("shape", [(256, 256, 256), (130, 70, 50), (512, 256, 1024)])
def test_gemm_fp32_compute(lib, shape):
    print("case: gemm fp32", shape, flush=True)
    M, N, K = shape
    # operands rounded to FP32 and FP32 accumulation: a few K * 2^-24
    assert run(lib, 0, M, N, K, fp32=1) <= 4 * K * 2.0 ** -24


def test_gemm_invalid_arguments(lib):
    st = lib.blr_selftest_gemm(0, -1, 4, 4, 1.0, None, 1, None, 1, 0.0, None, 1, 0, None)
    assert st == 1


@pytest.mark.parametrize("flags", [0, 1])
def test_gemm_fp32_long_k_accumulates_in_fp64(lib, flags):
    """FP32 operands with K = 65536 (the stack heights of the block-column
    products): the FP32 partial sums cover at most 1024 of K before they are
    added in FP64, so the normwise error stays at the level of a 1024-long FP32
    sum (about 2^-24 sqrt(256)) instead of growing with sqrt(K)."""
    print("case: gemm fp32 long K", flags, flush=True)
    M, N, K = 256, 256, 65536
    rng = np.random.default_rng(99 + flags)
    A = rng.standard_normal((K, M) if flags & 1 else (M, K))
    B = rng.standard_normal((K, N))
    Aop = A.T if flags & 1 else A
    ref = Aop @ B
    dA = torch.tensor(A.T.copy(), device="cuda")
    dB = torch.tensor(B.T.copy(), device="cuda")
    dC = torch.zeros((N, M), dtype=torch.float64, device="cuda")
    st = lib.blr_selftest_gemm(flags, M, N, K, 1.0, dA.data_ptr(), A.shape[0], dB.data_ptr(), K,
                               0.0, dC.data_ptr(), M, 1, torch.cuda.current_stream().cuda_stream)
    assert st == 0
    out = dC.cpu().numpy().T
    rel = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    print("normwise error / 2^-24:", rel / 2.0 ** -24, flush=True)
    assert rel <= 24 * 2.0 ** -24


@pytest.mark.parametrize("flags", [0, 1, 2])
@pytest.mark.parametrize("K", [1040, 2064, 3072])
def test_gemm_fp32_long_k_alpha_beta_in_place(lib, flags, K):
    """FP32 operands with K over 1024, alpha = 0.5 and beta = 2 with C both
    input and output: the FP64 sums of the 1024-long chunks are added into the
    output tile, the first addition starting from beta C.  K = 1040 and 2064
    end on a partial chunk."""
    print("case: gemm fp32 long K alpha beta", flags, K, flush=True)
    assert run(lib, flags, 256, 384, K, fp32=1) <= 4 * 1024 * 2.0 ** -24
