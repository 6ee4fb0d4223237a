"""GPU parity of the batched block-column factorization (blr_qr_factor_batch):
independent BLR matrices of uneven sizes, factored as one batch whose
launches serve the same step of many matrices, end bit for bit as each one
factored alone by blr_qr_factor, and agree with the oracle's block-column
factor (Alg. 2 with Section 3.3) like the single-matrix path.  The members
cover every panel path: stacks of up to 512 rows (32-column register
panels), up to 1024 rows (16-column register panels), taller stacks
(tree panels, batched across members) and, with 256-column tiles, 128-column blocks
applied as block reflectors; low-rank reflector rows and recompressions come
from the kernel matrices' far-field tiles."""
import numpy as np
import pytest

from oracle import blockcol, blrmat, metrics
from tests.blr_helpers import blr_to_host, export_r
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
U = np.finfo(np.float64).eps

# members: (seed, m, n, kernel, dim, admissibility); one (b, eps, cap) per batch
BATCH_B64 = [
    (0, 512, 256, "log2d", 2, "adjacent"),
    (1, 512, 256, "inv_r", 3, "dist_gt_diam"),
    (3, 2048, 512, "inv_r", 3, "dist_gt_diam"),
    (7, 768, 256, "inv_r", 3, "dist_gt_diam"),
    (8, 512, 256, "log2d", 2, "weak"),
    (12, 256, 256, "inv_r", 3, "weak"),
    (9, 1024, 128, "inv_r", 3, "dist_gt_diam"),
]
BATCH_B256 = [
    (4, 4096, 1024, "inv_r", 3, "dist_gt_diam"),
    (10, 2048, 512, "inv_r", 3, "dist_gt_diam"),
    (11, 1024, 512, "log2d", 2, "adjacent"),
]
BATCHES = {"b64": (BATCH_B64, 64, 1e-8, 32), "b256": (BATCH_B256, 256, 1e-8, 32)}


@pytest.fixture(scope="module")
def P():
    import paper_2208_06194_amd as P
    assert torch.cuda.is_available()
    return P


def member_blr(seed, m, n, b, eps, cap, kern, dim, rule):
    x, y = synth.kernel_points(seed, m, n, dim)
    A = blrmat.kernel_matrix(x, y, kern)
    mask = blrmat.lowrank_mask(x, y, b, rule, m // b, n // b)
    return blrmat.compress(A, b, eps, cap, mask)


def gpu_import(P, blr, eps, cap):
    fmt, rank, dense, Uh, Vh = blr_to_host(blr, cap)
    return P.BLRMatrix.import_tiles(blr.m, blr.n, blr.b, eps, cap, fmt, rank, dense, Uh, Vh)


def same_export(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("fmt", "rank", "dense", "U", "V", "Y", "T"))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("batch", sorted(BATCHES))
def test_batch_is_bitwise_equal_to_single_factors(P, batch, precision):
    members, b, eps, cap = BATCHES[batch]
    print("case: batch vs single", batch, precision, flush=True)
    blrs = [member_blr(s, m, n, b, eps, cap, k, d, r) for (s, m, n, k, d, r) in members]
    singles = [gpu_import(P, blr, eps, cap) for blr in blrs]
    for G in singles:
        G.factor("block_column", precision=precision)
    batched = [gpu_import(P, blr, eps, cap) for blr in blrs]
    P.factor_batch(batched, precision=precision)
    torch.cuda.synchronize()
    launches_single = sum(G.info()["kernel_launches"] for G in singles)
    launches_batch = batched[0].info()["kernel_launches"]
    print("launches: single total", launches_single, "batch", launches_batch, flush=True)
    assert launches_batch < launches_single
    for (mem, Gs, Gb) in zip(members, singles, batched):
        es, eb = Gs.export(with_factor=True), Gb.export(with_factor=True)
        assert same_export(es, eb), mem
        a, c = Gs.info(), Gb.info()
        for key in a:
            if key not in ("device_bytes", "kernel_launches"):
                assert a[key] == c[key], (mem, key)
        assert c["state"] == a["state"]


def test_batch_matches_oracle(P):
    members, b, eps, cap = BATCHES["b64"]
    print("case: batch vs oracle", flush=True)
    blrs = [member_blr(s, m, n, b, eps, cap, k, d, r) for (s, m, n, k, d, r) in members]
    Gs = [gpu_import(P, blr, eps, cap) for blr in blrs]
    P.factor_batch(Gs)
    for mem, blr, G in zip(members, blrs, Gs):
        At = blr.to_dense()
        m, n = At.shape
        f = blockcol.factor(blr, eps, cap)
        ex = G.export(with_factor=True)
        assert np.array_equal(ex["fmt"], f.A.fmt), mem
        Rg, Ro = export_r(ex), f.r_dense()
        kappa = np.linalg.cond(At)
        rel = np.linalg.norm(metrics.sign_fix(Rg, Ro) - Ro) / np.linalg.norm(Ro)
        print(mem, "R rel diff", rel, "kappa", kappa, flush=True)
        assert rel <= 10 * kappa * eps
        RR = np.zeros((m, n))
        RR[:n] = Rg
        QR = G.apply_qt(torch.tensor(RR, device="cuda"), trans=True).cpu().numpy()
        res = np.linalg.norm(QR - At) / np.linalg.norm(At)
        assert res <= 10 * eps, (mem, res)
        # the least-squares solve on the batched factor
        Bh = synth.rhs(seed_of(mem), m, 4)
        X = G.lstsq(torch.tensor(Bh, device="cuda")).cpu().numpy()
        Xo = f.lstsq(Bh)
        assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 10 * kappa * eps, mem


def seed_of(mem):
    return 100 + mem[0]


def test_batch_of_one_and_prefix(P):
    """A batch of one equals the single factor; stop_after_k applies to every
    member (members with fewer block columns stop at their last)."""
    members, b, eps, cap = BATCHES["b64"]
    print("case: batch of one, prefix", flush=True)
    blrs = [member_blr(s, m, n, b, eps, cap, k, d, r) for (s, m, n, k, d, r) in members[:3]]
    G1 = gpu_import(P, blrs[2], eps, cap)
    G1.factor("block_column")
    G2 = gpu_import(P, blrs[2], eps, cap)
    P.factor_batch([G2])
    assert same_export(G1.export(with_factor=True), G2.export(with_factor=True))
    singles = [gpu_import(P, blr, eps, cap) for blr in blrs]
    for G in singles:
        G.factor("block_column", stop_after_k=3)
    batched = [gpu_import(P, blr, eps, cap) for blr in blrs]
    P.factor_batch(batched, stop_after_k=3)
    for Gs, Gb in zip(singles, batched):
        assert same_export(Gs.export(with_factor=True), Gb.export(with_factor=True))


def test_batch_rejects_mixed_shapes_and_states(P):
    print("case: batch errors", flush=True)
    a = member_blr(0, 256, 128, 64, 1e-8, 16, "log2d", 2, "adjacent")
    c = member_blr(1, 256, 128, 32, 1e-8, 16, "log2d", 2, "adjacent")
    Ga, Gc = gpu_import(P, a, 1e-8, 16), gpu_import(P, c, 1e-8, 16)
    with pytest.raises(P.BLRError) as e:
        P.factor_batch([Ga, Gc])
    assert e.value.status == 1
    with pytest.raises(P.BLRError) as e:
        P.factor_batch([Ga, Ga])
    assert e.value.status == 1
    Ga.factor("block_column")
    Gd = gpu_import(P, a, 1e-8, 16)
    with pytest.raises(P.BLRError) as e:
        P.factor_batch([Gd, Ga])
    assert e.value.status == 2
    # the failed calls left the compressed member untouched and usable
    P.factor_batch([Gd])
    assert same_export(Ga.export(with_factor=True), Gd.export(with_factor=True))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_solve_is_bitwise_equal_to_single_solves(P, precision):
    """blr_lstsq_solve_batch gives each member exactly blr_lstsq_solve's
    result: FP64 factors without refinement, mixed factors (kept A~) with
    FP64 iterative refinement; one member factored by the tiled variant."""
    members, b, eps, cap = BATCHES["b64"]
    print("case: batched solve", precision, flush=True)
    refine = 5 if precision == "mixed" else 0
    blrs = [member_blr(s, m, n, b, eps, cap, k, d, r) for (s, m, n, k, d, r) in members]
    Gs = [gpu_import(P, blr, eps, cap) for blr in blrs]
    Gs[0].factor("tiled", precision=precision, keep_a=refine > 0)
    P.factor_batch(Gs[1:], precision=precision, keep_a=refine > 0)
    Bs = [torch.tensor(synth.rhs(200 + i, blr.m, 5), device="cuda") for i, blr in enumerate(blrs)]
    singles = [G.lstsq(B, max_refine=refine) for G, B in zip(Gs, Bs)]
    batched = P.lstsq_batch(Gs, Bs, max_refine=refine)
    for mem, blr, xs, xb, B in zip(members, blrs, singles, batched, Bs):
        assert torch.equal(xs, xb), mem
        if precision == "mixed":
            # refinement recovers the FP64 solution of A~
            At = blr.to_dense()
            Xo = np.linalg.lstsq(At, B.cpu().numpy(), rcond=None)[0]
            kappa = np.linalg.cond(At)
            err = np.linalg.norm(xb.cpu().numpy() - Xo) / np.linalg.norm(Xo)
            print(mem, "refined mixed solve vs dense FP64 lstsq", err, "kappa", kappa, flush=True)
            assert err <= 10 * kappa * eps


def test_batched_solve_rejects_bad_batches(P):
    print("case: batched solve errors", flush=True)
    a = member_blr(0, 256, 128, 64, 1e-8, 16, "log2d", 2, "adjacent")
    G = gpu_import(P, a, 1e-8, 16)
    B = torch.tensor(synth.rhs(1, 256, 2), device="cuda")
    with pytest.raises(P.BLRError) as e:
        P.lstsq_batch([G], [B])
    assert e.value.status == 2      # not factored
    G.factor("block_column")
    with pytest.raises(P.BLRError) as e:
        P.lstsq_batch([G], [B], max_refine=2)
    assert e.value.status == 2      # refinement without keep_a
    with pytest.raises(P.BLRError) as e:
        P.lstsq_batch([G, G], [B, B])
    assert e.value.status == 1
    X = P.lstsq_batch([G], [B])[0]
    assert torch.equal(X, G.lstsq(B))
