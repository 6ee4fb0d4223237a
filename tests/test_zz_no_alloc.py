"""GPU: blr_apply_qt_noalloc (Q^T B / Q B with its temporaries in the per-GPU
static scratch) against blr_apply_qt on the same factor: the same kernels and
launch plan, so the results must be bit-identical.  Two calls in a row, the
second with a smaller input; a request beyond the scratch is refused."""
import pytest

import synth
from tests.blr_helpers import gpu_import, kernel_blr

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2208_06194_amd as P
    assert torch.cuda.is_available()
    return P


def factored(P, variant, seed, m, n, b, eps=1e-8, cap=32):
    A, blr = kernel_blr(seed, m, n, b, eps, cap, "log2d", 2, "weak")
    G = gpu_import(P, blr, eps, cap)
    G.factor(variant)
    return G


@pytest.mark.parametrize("variant", ["tiled", "block_column"])
def test_noalloc_apply_matches_apply_qt(P, variant):
    print("case: no-alloc apply", variant, flush=True)
    # first call: 1024 x 512 (b = 128, low-rank tiles by weak admissibility), 9 columns
    G1 = factored(P, variant, 41, 1024, 512, 128)
    B1 = torch.tensor(synth.rhs(41, 1024, 9), device="cuda")
    for trans in (False, True):
        ref = G1.apply_qt(B1, trans=trans)
        out = G1.apply_qt_noalloc(B1, trans=trans)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (variant, trans)
    # second call: a smaller matrix and fewer columns, in the same scratch
    G2 = factored(P, variant, 42, 512, 256, 64)
    B2 = torch.tensor(synth.rhs(42, 512, 3), device="cuda")
    out2 = G2.apply_qt_noalloc(B2)
    torch.cuda.synchronize()
    assert torch.equal(out2, G2.apply_qt(B2))
    # a no-allocation call leaves the device's free memory unchanged (the
    # binding's copy of B comes from torch's cache, warmed by the call above)
    free_before = torch.cuda.mem_get_info()[0]
    out3 = G2.apply_qt_noalloc(B2, trans=True)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free_before
    assert torch.equal(out3, G2.apply_qt(B2, trans=True))
    # and the first matrix again after the smaller one: nothing stale in the scratch
    assert torch.equal(G1.apply_qt_noalloc(B1), G1.apply_qt(B1))


def test_noalloc_apply_refuses_more_than_the_scratch(P):
    """The block-column form needs about 64 b doubles per right-hand side
    (split-K partial sums): 1100 right-hand sides at b = 128 need more than
    the 64 MiB scratch, and the call fails before enqueuing anything."""
    print("case: no-alloc apply over the limit", flush=True)
    from paper_2208_06194_amd import _lib as L
    G = factored(P, "block_column", 43, 1024, 512, 128)
    B = torch.tensor(synth.rhs(43, 1024, 1100), device="cuda")
    with pytest.raises(P.BLRError) as e:
        G.apply_qt_noalloc(B)
    assert e.value.status == L.BLR_ERR_INVALID
    assert "scratch" in str(e.value)
    # the handle still works: the same call within the limit
    Bs = B[:, :5].contiguous()
    assert torch.equal(G.apply_qt_noalloc(Bs), G.apply_qt(Bs))


def test_noalloc_tiled_apply_with_fewer_chains_matches_apply_qt(P):
    """The tiled form plans every step of the application as a chain of its
    own and merges the chains into one launch list; chains k and k + ns share
    a workspace.  At 4096 rows, b = 128 and 1024 right-hand sides a chain's
    workspace is about 6.5 MiB, so the no-allocation call (16 MiB for them)
    runs 2 chains and blr_apply_qt all 8.  Every op keeps the kernel chosen
    for it before the merge, so the results are equal bit for bit, and
    Q (Q^T B) returns B."""
    print("case: no-alloc tiled apply with fewer chains", flush=True)
    G = factored(P, "tiled", 44, 4096, 1024, 128)
    B = torch.tensor(synth.rhs(44, 4096, 1024), device="cuda")
    for trans in (False, True):
        ref = G.apply_qt(B, trans=trans)
        out = G.apply_qt_noalloc(B, trans=trans)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), trans
    back = G.apply_qt(G.apply_qt(B), trans=True)
    assert float((back - B).abs().max()) <= 1e-11 * float(B.abs().max())
