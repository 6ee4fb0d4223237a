"""GPU: the adjoint of the least-squares solve (blr_lstsq_adjoint) and the R
solves (blr_rsolve) through the C ABI, against the oracle's dense adjoint of
the compressed matrix, and the autograd function built on them."""
import numpy as np
import pytest

import synth
from oracle import adjoint, blrmat
from oracle.blrmat import DENSE
from tests.blr_helpers import blr_to_host, rank_capacity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2208_06194_amd as P
    assert torch.cuda.is_available()
    return P


def setup(P, variant, m=512, n=256, b=64, eps=1e-12, seed=8):
    # 2D log kernel, adjacency rule: 12 of 32 tiles low-rank, ranks 29..51 at 1e-12
    x, y = synth.kernel_points(seed, m, n, 2)
    A = blrmat.kernel_matrix(x, y, "log2d")
    mask = blrmat.lowrank_mask(x, y, b, "adjacent", m // b, n // b)
    cap = b
    blr = blrmat.compress(A, b, eps, cap, mask)
    fmt, rank, dense, Uh, Vh = blr_to_host(blr, cap)
    G = P.BLRMatrix.import_tiles(m, n, b, eps, cap, fmt, rank, dense, Uh, Vh)
    G.factor(variant, keep_a=True)
    return blr, G


@pytest.mark.parametrize("variant", ["tiled", "block_column"])
def test_adjoint_matches_oracle(P, variant):
    print("case: adjoint", variant, flush=True)
    blr, G = setup(P, variant)
    assert (blr.fmt == 1).any() and (blr.fmt == 0).any()
    At = blr.to_dense()
    m, n = At.shape
    rng = np.random.default_rng(5)
    Bh = synth.rhs(6, m, 3)
    Xbh = rng.standard_normal((n, 3))
    B = torch.tensor(Bh, device="cuda")
    X = G.lstsq(B)
    Bbar, dD, dU, dV = G.lstsq_adjoint(B, X, torch.tensor(Xbh, device="cuda"))
    Xo, Bbar_o, Abar_o = adjoint.lstsq_adjoint(At, Bh, Xbh)
    g = adjoint.tile_gradients(blr, Abar_o)
    kappa = np.linalg.cond(At)
    tol = 100 * kappa * 1e-12
    rel = lambda a, o: np.linalg.norm(a - o) / max(np.linalg.norm(o), 1e-300)
    print("kappa", kappa, "X", rel(X.cpu().numpy(), Xo), "Bbar", rel(Bbar.cpu().numpy(), Bbar_o), flush=True)
    assert rel(X.cpu().numpy(), Xo) <= tol
    assert rel(Bbar.cpu().numpy(), Bbar_o) <= tol
    dD, dU, dV = dD.cpu().numpy(), dU.cpu().numpy(), dV.cpu().numpy()
    scale = np.linalg.norm(Abar_o)
    for (i, j), gv in g.items():
        if gv[0] == "D":
            assert np.linalg.norm(dD[i, j] - gv[1]) <= tol * scale, (i, j)
            assert not dU[i, j].any() and not dV[i, j].any()
        else:
            r = blr.rank(i, j)
            assert np.linalg.norm(dU[i, j][:, :r] - gv[1]) <= tol * scale, (i, j)
            assert np.linalg.norm(dV[i, j][:, :r] - gv[2]) <= tol * scale, (i, j)
            assert not dU[i, j][:, r:].any() and not dD[i, j].any()


def test_rsolve_inverts_r(P):
    print("case: rsolve", flush=True)
    blr, G = setup(P, "block_column")
    n = blr.n
    Y = torch.tensor(synth.rhs(9, n, 4), device="cuda")
    RY = G.matmul(Y, "R")
    assert torch.linalg.norm(G.rsolve(RY) - Y) / torch.linalg.norm(Y) <= 1e-9
    # R^T R Y solved back with the two triangular solves
    RtRY = G.rsolve(G.rsolve(RY, trans=False), trans=False)   # R^{-1} R^{-1} R Y = R^{-1} Y
    assert torch.allclose(G.matmul(RtRY, "R"), Y, atol=1e-9 * float(torch.abs(Y).max()))
    Z = G.rsolve(G.matmul(Y, "R"), trans=False)
    W = G.rsolve(Z.clone(), trans=True)     # R^{-T} Y
    # (R^T W = Y) checked through the explicit dense R
    from tests.blr_helpers import export_r
    R = export_r(G.export())
    assert np.allclose(R.T @ W.cpu().numpy(), Y.cpu().numpy(), atol=1e-8 * float(torch.abs(Y).max()))


def test_autograd_function_returns_the_adjoint(P):
    print("case: autograd", flush=True)
    blr, G = setup(P, "block_column")
    m, n, b = blr.m, blr.n, blr.b
    p, q, rc = blr.p, blr.q, rank_capacity(b, b)
    B = torch.tensor(synth.rhs(7, m, 2), device="cuda", requires_grad=True)
    D = torch.zeros((p, q, b, b), dtype=torch.float64, device="cuda", requires_grad=True)
    U = torch.zeros((p, q, b, rc), dtype=torch.float64, device="cuda", requires_grad=True)
    V = torch.zeros((p, q, b, rc), dtype=torch.float64, device="cuda", requires_grad=True)
    Xbar = torch.tensor(np.random.default_rng(2).standard_normal((n, 2)), device="cuda")
    X = P.lstsq(G, B, D, U, V)
    (X * Xbar).sum().backward()
    Bbar, dD, dU, dV = G.lstsq_adjoint(B.detach(), X.detach(), Xbar)
    assert torch.equal(B.grad, Bbar)
    assert torch.equal(D.grad, dD) and torch.equal(U.grad, dU) and torch.equal(V.grad, dV)
