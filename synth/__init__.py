"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds no arithmetic of the factorization method: it only draws
numbers.  Everything is counter based so that any element can be regenerated
independently (and a device-side copy of the generator can reproduce it).

Generator (splitmix64, Steele, Lea & Flood 2014):
    stream key   s = mix(seed * 0x9E3779B97F4A7C15 + stream * 0xD1B54A32D192ED03 + 1)
    word i       w_i = mix(s + (i + 1) * 0x9E3779B97F4A7C15)
    mix(z):  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
             z *= 0x94D049BB133111EB; z ^= z >> 31
    uniform double in [0,1):  (w >> 11) * 2**-53
    standard normal (Box-Muller): u1 = 1 - U(w_{2i}), u2 = U(w_{2i+1}),
             g_i = sqrt(-2 ln u1) * cos(2 pi u2)

Streams: 0 = row points x, 1 = column points y, 2 = right-hand sides,
3 = random-BLR tile entries, 4 = sizes of a batch of matrices.
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_GAMMA2 = np.uint64(0xD1B54A32D192ED03)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

STREAM_X, STREAM_Y, STREAM_RHS, STREAM_TILES, STREAM_BATCH = 0, 1, 2, 3, 4


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def stream_key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        base = (np.uint64(seed) * _GAMMA + np.uint64(stream) * _GAMMA2
                + np.uint64(1))
        return _mix(np.array([base], dtype=np.uint64))[0]


def words(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """Raw 64-bit words w_offset .. w_{offset+count-1} of a stream."""
    key = stream_key(seed, stream)
    idx = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + idx * _GAMMA)


def uniform(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    w = words(seed, stream, count, offset)
    return (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seed: int, stream: int, count: int, offset: int = 0) -> np.ndarray:
    """Standard normals g_offset .. g_{offset+count-1} (Box-Muller, cosine branch)."""
    u = uniform(seed, stream, 2 * count, 2 * offset)
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def morton_keys(pts: np.ndarray) -> np.ndarray:
    """Morton (Z-order) keys: each coordinate quantised to 2**21 levels
    (clamped), bits interleaved most-significant first in coordinate order."""
    npts, d = pts.shape
    q = np.clip(np.floor(pts * (1 << 21)), 0, (1 << 21) - 1).astype(np.uint64)
    key = np.zeros(npts, dtype=np.uint64)
    for level in range(20, -1, -1):
        for c in range(d):
            key = (key << np.uint64(1)) | ((q[:, c] >> np.uint64(level)) & np.uint64(1))
    return key


def morton_sort(pts: np.ndarray) -> np.ndarray:
    order = np.argsort(morton_keys(pts), kind="stable")
    return np.ascontiguousarray(pts[order])


def points(seed: int, stream: int, count: int, dim: int) -> np.ndarray:
    """`count` points uniform in the unit square/cube, Morton sorted.
    Coordinate c of point i is uniform word i*dim + c of the stream."""
    raw = uniform(seed, stream, count * dim).reshape(count, dim)
    return morton_sort(raw)


def kernel_points(seed: int, m: int, n: int, dim: int):
    """Row points x (m) and column points y (n) of a kernel-matrix workload."""
    return points(seed, STREAM_X, m, dim), points(seed, STREAM_Y, n, dim)


def batch_rows(seed: int, count: int, lo: int, hi: int, mult: int) -> np.ndarray:
    """Row counts of a batch of matrices, log-uniform in [lo, hi]: member i
    has exp(ln lo + u_i (ln hi - ln lo)) rounded to the nearest multiple of
    mult and clamped to [lo, hi], with u_i uniform word i of stream 4."""
    u = uniform(seed, STREAM_BATCH, count)
    m = np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))
    m = np.rint(m / mult).astype(np.int64) * mult
    return np.clip(m, lo, hi)


def rhs(seed: int, m: int, nrhs: int) -> np.ndarray:
    """m x nrhs Gaussian right-hand sides, column-major order of draws."""
    return normal(seed, STREAM_RHS, m * nrhs).reshape(nrhs, m).T.copy()


def random_blr_tiles(seed: int, m: int, n: int, b: int, rank: int):
    """The draws of random_blr_dense as tile factors, without forming the
    dense matrix: D[k] (b x b) for the diagonal tiles (k,k), k < n/b, and
    X[i,j], Y[i,j] (b x rank) for every other tile, so that tile (i,j) of
    random_blr_dense is X[i,j] @ Y[i,j].T.  X and Y of diagonal tiles are zero."""
    p, q = m // b, n // b
    per = b * max(b, 2 * rank)
    D = np.empty((q, b, b))
    X = np.zeros((p, q, b, rank))
    Y = np.zeros((p, q, b, rank))
    for i in range(p):
        for j in range(q):
            off = (i * q + j) * per
            if i == j:
                D[i] = normal(seed, STREAM_TILES, b * b, off).reshape(b, b)
            else:
                g = normal(seed, STREAM_TILES, 2 * b * rank, off)
                X[i, j] = g[: b * rank].reshape(b, rank)
                Y[i, j] = g[b * rank:].reshape(b, rank)
    return D, X, Y


def random_blr_dense(seed: int, m: int, n: int, b: int, rank: int) -> np.ndarray:
    """Random BLR test matrix (the random-BLR workload of the paper's first
    experiment): diagonal tiles (k,k), k < n/b, are N(0,1) dense; every other
    tile is X @ Y.T with X, Y b x rank N(0,1).  Tile (i,j) draws its values
    from the tile stream at offset (i*q + j) * b * max(b, 2*rank)."""
    p, q = m // b, n // b
    per = b * max(b, 2 * rank)
    A = np.empty((m, n))
    for i in range(p):
        for j in range(q):
            g = normal(seed, STREAM_TILES, per, (i * q + j) * per)
            if i == j:
                blk = g[: b * b].reshape(b, b)
            else:
                X = g[: b * rank].reshape(b, rank)
                Y = g[b * rank: 2 * b * rank].reshape(b, rank)
                blk = X @ Y.T
            A[i * b:(i + 1) * b, j * b:(j + 1) * b] = blk
    return A
