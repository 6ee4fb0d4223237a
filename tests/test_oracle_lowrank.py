"""Pins of truncation, compression and rounded addition (Alg. 6) against the
Eckart-Young theorem (best rank-r approximation = truncated SVD) and the
compression error bound stated with eq. blr_matrix_def."""
import numpy as np
import pytest

from oracle import blrmat, lowrank


def test_trunc_rank_definition():
    s = np.array([4.0, 3.0, 0.0])
    assert lowrank.trunc_rank(s, 0.0) == 2
    assert lowrank.trunc_rank(np.zeros(4), 1e-8) == 0
    assert lowrank.trunc_rank(np.array([]), 1e-8) == 0
    # ||(3,0)|| / ||(4,3,0)|| = 0.6: eps = 0.6 -> rank 1 (ties keep the smaller rank)
    assert lowrank.trunc_rank(s, 0.6) == 1
    assert lowrank.trunc_rank(s, 0.5999) == 2
    assert lowrank.trunc_rank(s, 1.0) == 0


def _lowrank_plus_noise(b, r, noise, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((b, r)) @ rng.standard_normal((r, b)) + noise * rng.standard_normal((b, b))


@pytest.mark.parametrize("eps", [1e-4, 1e-8])
def test_compress_tile_error_bound_and_minimality(eps):
    A = _lowrank_plus_noise(32, 5, 1e-6, 0)
    kind, U, V = lowrank.compress_tile(A, eps, 32, "dense")
    assert kind == "L"
    r = U.shape[1]
    err = np.linalg.norm(U @ V.T - A)
    assert err <= eps * np.linalg.norm(A) * (1 + 1e-12)
    assert np.allclose(U.T @ U, np.eye(r), atol=1e-13)
    # minimal: the best rank r-1 approximation violates the bound
    s = np.linalg.svd(A, compute_uv=False)
    assert np.sqrt(np.sum(s[r - 1:] ** 2)) > eps * np.linalg.norm(A)


def test_compress_tile_overflow_policies():
    A = np.random.default_rng(3).standard_normal((16, 16))   # full rank
    assert lowrank.compress_tile(A, 1e-8, 4, "dense")[0] == "D"
    kind, U, V = lowrank.compress_tile(A, 1e-8, 4, "truncate")
    assert kind == "L" and U.shape[1] == 4
    Z = lowrank.compress_tile(np.zeros((8, 8)), 1e-8, 4, "dense")
    assert Z[0] == "L" and Z[1].shape == (8, 0)


def test_rounded_add_is_truncated_svd_of_the_sum():
    rng = np.random.default_rng(5)
    b = 40
    U1, V1 = np.linalg.qr(rng.standard_normal((b, 6)))[0], rng.standard_normal((b, 6))
    U2, V2 = rng.standard_normal((b, 4)), rng.standard_normal((b, 4))
    # make the sum numerically rank 7 by cancelling a direction
    U2[:, 0] = U1[:, 0]
    V2[:, 0] = -V1[:, 0] * (1 - 1e-9)
    S = U1 @ V1.T + U2 @ V2.T
    st = lowrank.Stats()
    eps = 1e-6
    Uc, Vc = lowrank.rounded_add([(U1, V1), (U2, V2)], eps, 64, st)
    s = np.linalg.svd(S, compute_uv=False)
    r = Uc.shape[1]
    assert r == lowrank.trunc_rank(s, eps)
    err = np.linalg.norm(Uc @ Vc.T - S)
    # Eckart-Young: the error equals the singular-value tail of the dense sum
    assert abs(err - np.sqrt(np.sum(s[r:] ** 2))) <= 1e-12 * np.linalg.norm(S)
    assert np.allclose(Uc.T @ Uc, np.eye(r), atol=1e-13)
    assert st.recompressions == 1 and st.overflow == 0


def test_rounded_add_cap_and_empty():
    rng = np.random.default_rng(6)
    b = 20
    terms = [(rng.standard_normal((b, 5)), rng.standard_normal((b, 5))) for _ in range(2)]
    st = lowrank.Stats()
    Uc, Vc = lowrank.rounded_add(terms, 1e-12, 3, st)
    assert Uc.shape[1] == 3 and st.overflow == 1 and st.max_dropped_rel > 0
    Uc, Vc = lowrank.rounded_add([(np.zeros((b, 0)), np.zeros((b, 0)))], 1e-8, 3, st)
    assert Uc.shape == (b, 0)


def test_kernel_matrix_values():
    x = np.array([[0.0, 0.0], [3.0, 4.0]])
    y = np.array([[0.0, 0.0]])
    A = blrmat.kernel_matrix(x, y, "inv_r", 1e-3)
    assert np.allclose(A[:, 0], [1 / 1e-3, 1 / 5.001])
    A = blrmat.kernel_matrix(x, y, "log2d", 1e-3)
    assert np.allclose(A[:, 0], [-np.log(1e-3), -np.log(5.001)])


def test_admissibility_rules_on_known_boxes():
    # rows: cluster 0 in [0,0.1]^2, cluster 1 in [0.9,1]^2; columns: cluster 0
    # in [0,0.1]^2, cluster 1 in [0.15, 0.25] x [0, 0.1]
    x = np.array([[0, 0], [0.1, 0.1], [0.9, 0.9], [1.0, 1.0]], dtype=float)
    y = np.array([[0, 0], [0.1, 0.1], [0.15, 0.0], [0.25, 0.1]], dtype=float)
    adj = blrmat.lowrank_mask(x, y, 2, "adjacent", 2, 2)
    assert adj.tolist() == [[False, True], [True, False]]   # diagonal forced dense
    far = blrmat.lowrank_mask(x, y, 2, "dist_gt_diam", 2, 2)
    # gap(row0, col1) = 0.05 < diam = 0.141 -> dense; row1 is far from col0
    assert far.tolist() == [[False, False], [True, False]]
    weak = blrmat.lowrank_mask(None, None, 2, "weak", 2, 2)
    assert weak.tolist() == [[False, True], [True, False]]


def test_compression_global_bound():
    import synth
    x, y = synth.kernel_points(4, 256, 128, 2)
    A = blrmat.kernel_matrix(x, y, "log2d")
    mask = blrmat.lowrank_mask(x, y, 32, "adjacent", 8, 4)
    eps = 1e-6
    blr = blrmat.compress(A, 32, eps, 32, mask, "dense")
    assert np.linalg.norm(blr.to_dense() - A) <= eps * np.linalg.norm(A)
    for i in range(8):
        for j in range(4):
            blk = A[i * 32:(i + 1) * 32, j * 32:(j + 1) * 32]
            assert np.linalg.norm(blr.tile(i, j) - blk) <= eps * np.linalg.norm(blk) * (1 + 1e-12)
