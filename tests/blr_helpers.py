"""Helpers shared by the GPU tests: moving tiles between the oracle's BLR
container and the library's host tile layout, and reading R off an export."""
import numpy as np

from oracle.blrmat import BLR, DENSE, LOWRANK


def rank_capacity(cap: int, b: int) -> int:
    return min((cap + 15) // 16 * 16, b)


def blr_to_host(blr: BLR, cap: int):
    """Oracle BLR -> (fmt, rank, dense, U, V) arrays in the blr_tiles_host
    layout (an edge tile of a ragged matrix in the leading rows and columns
    of its b x b slot)."""
    p, q, b = blr.p, blr.q, blr.b
    rc = rank_capacity(cap, b)
    fmt = np.zeros(p * q, np.int8)
    rank = np.zeros(p * q, np.int32)
    dense = np.zeros((p * q, b, b))
    U = np.zeros((p * q, rc, b))
    V = np.zeros((p * q, rc, b))
    for i in range(p):
        for j in range(q):
            t = i * q + j
            if blr.fmt[i, j] == DENSE:
                D = blr.D[(i, j)]
                dense[t, :D.shape[1], :D.shape[0]] = D.T          # column-major
            else:
                r = blr.rank(i, j)
                assert r <= cap
                fmt[t] = 1
                rank[t] = r
                Ut, Vt = blr.U[(i, j)], blr.V[(i, j)]
                U[t, :r, :Ut.shape[0]] = Ut.T
                V[t, :r, :Vt.shape[0]] = Vt.T
    return fmt, rank, dense.ravel(), U.ravel(), V.ravel()


def export_tile(ex, i, j):
    """Dense value of tile (i,j) of an export (R tiles and untouched tiles)."""
    if ex["fmt"][i, j] == 0:
        return ex["dense"][i, j]
    r = ex["rank"][i, j]
    return ex["U"][i, j][:, :r] @ ex["V"][i, j][:, :r].T


def export_r(ex):
    """R (n x n) from an export; for a ragged matrix the leading n x n block
    of the embedding's R."""
    p, q = ex["fmt"].shape
    b = ex["dense"].shape[2]
    R = np.zeros((q * b, q * b))
    for k in range(q):
        for j in range(k, q):
            blk = np.triu(ex["dense"][k, k]) if j == k else export_tile(ex, k, j)
            R[k * b:(k + 1) * b, j * b:(j + 1) * b] = blk
    n = ex["info"]["n"] if "info" in ex else q * b
    return R[:n, :n]


def export_dense(ex):
    """The matrix (m x n) of an export (for a ragged matrix: the caller's rows
    and columns of the edge tiles)."""
    p, q = ex["fmt"].shape
    b = ex["dense"].shape[2]
    A = np.zeros((p * b, q * b))
    for i in range(p):
        for j in range(q):
            A[i * b:(i + 1) * b, j * b:(j + 1) * b] = export_tile(ex, i, j)
    if "info" in ex:
        A = A[:ex["info"]["m"], :ex["info"]["n"]]
    return A


def gpu_import(P, blr: BLR, eps: float, cap: int):
    """The oracle-compressed matrix imported into the library (the oracle's
    tiles are the input of both sides)."""
    fmt, rank, dense, Uh, Vh = blr_to_host(blr, cap)
    return P.BLRMatrix.import_tiles(blr.m, blr.n, blr.b, eps, cap, fmt, rank, dense, Uh, Vh)


def kernel_blr(seed, m, n, b, eps, cap, kern="inv_r", dim=3, rule="dist_gt_diam", overflow="dense"):
    """Seeded kernel matrix (Morton-sorted points) and the oracle's compression of it."""
    import synth
    from oracle import blrmat
    x, y = synth.kernel_points(seed, m, n, dim)
    A = blrmat.kernel_matrix(x, y, kern)
    mask = blrmat.lowrank_mask(x, y, b, rule, m // b, n // b)
    return A, blrmat.compress(A, b, eps, cap, mask, overflow)
