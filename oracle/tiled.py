"""Tiled Householder BLR-QR (paper Alg. 4 with the operations of Section 3.4)
and left multiplication by Q / Q^T (Alg. 5).

Task set of one k-iteration (Section 3.4, Table blr_bh_operations):
  GEQRT(k)        QR of the diagonal tile (3.4.1)
  LARFB(k,j)      R_kj = Qkk^T A_kj, j > k; a low-rank tile updates U only (3.4.2)
  TPQRT(i,k)      QR of [R_kk; A_ik], i > k; for a low-rank A_ik the QR is of
                  [R_kk; V_ik^T] and Ytilde_ik = U_ik Y_ik with the same T (3.4.3)
  TPMQRT(i,k,j)   [R_kj; A_ij] -= [I; Ytilde_ik] T_ik^T (R_kj + Ytilde_ik^T A_ij)
                  with the OP1-OP4 format rules (3.4.4)

The DAG of Section 4.3 is derived from the tiles each task reads and writes;
`run(order=...)` executes any topological order of it (the result does not
depend on the order, since every tile sees the same sequence of updates).
"""
from __future__ import annotations

import random

import numpy as np

from . import blrops, dense
from .blrmat import BLR, DENSE, LOWRANK
from .factor import Factor

def _yt_dense(Yr, B):
    """Ytilde^T B for a dense block B."""
    return Yr[1].T @ B if Yr[0] == "D" else Yr[2].T @ (Yr[1].T @ B)


PRIORITY = {"geqrt": 0, "tpqrt": 1, "tpmqrt": 2, "larfb": 2}


def task_list(p: int, q: int, stop_after_k: int | None = None):
    """Tasks in the sequential order of Alg. 4 (0-based indices)."""
    kend = q if stop_after_k is None else min(q, stop_after_k)
    tasks = []
    for k in range(kend):
        tasks.append(("geqrt", k))
        for j in range(k + 1, q):
            tasks.append(("larfb", k, j))
        for i in range(k + 1, p):
            tasks.append(("tpqrt", i, k))
            for j in range(k + 1, q):
                tasks.append(("tpmqrt", i, k, j))
    return tasks


def resources(t):
    """(reads, writes) of a task.  The diagonal tile splits into its
    reflector part ('Y', k) and its triangle ('R', k) after GEQRT."""
    kind = t[0]
    if kind == "geqrt":
        k = t[1]
        return [("A", k, k)], [("A", k, k), ("Y", k), ("R", k)]
    if kind == "larfb":
        k, j = t[1], t[2]
        return [("Y", k), ("A", k, j)], [("A", k, j)]
    if kind == "tpqrt":
        i, k = t[1], t[2]
        return [("R", k), ("A", i, k)], [("R", k), ("A", i, k)]
    i, k, j = t[1], t[2], t[3]
    return [("A", i, k), ("A", k, j), ("A", i, j)], [("A", k, j), ("A", i, j)]


def build_dag(tasks):
    """Dependencies of each task (indices of earlier tasks): read-after-write,
    write-after-read and write-after-write on every resource."""
    last_w, readers = {}, {}
    deps = []
    for idx, t in enumerate(tasks):
        rd, wr = resources(t)
        d = set()
        for r in rd:
            if r in last_w:
                d.add(last_w[r])
        for r in wr:
            if r in last_w:
                d.add(last_w[r])
            d.update(readers.get(r, ()))
        for r in rd:
            readers.setdefault(r, set()).add(idx)
        for r in wr:
            last_w[r] = idx
            readers[r] = set()
        d.discard(idx)
        deps.append(sorted(d))
    return deps


def topo_order(tasks, deps, mode: str = "sequential", seed: int = 0):
    """'sequential' (Alg. 4 order), 'random' (uniformly random ready task) or
    'priority' (GEQRT > TPQRT > TPMQRT/LARFB, Section 4.3)."""
    n = len(tasks)
    if mode == "sequential":
        return list(range(n))
    succ = [[] for _ in range(n)]
    indeg = [len(d) for d in deps]
    for i, d in enumerate(deps):
        for j in d:
            succ[j].append(i)
    ready = [i for i in range(n) if indeg[i] == 0]
    rng = random.Random(seed)
    order = []
    while ready:
        if mode == "random":
            pos = rng.randrange(len(ready))
        else:
            pos = min(range(len(ready)),
                      key=lambda a: (PRIORITY[tasks[ready[a]][0]], ready[a]))
        t = ready.pop(pos)
        order.append(t)
        for s in succ[t]:
            indeg[s] -= 1
            if indeg[s] == 0:
                ready.append(s)
    assert len(order) == n
    return order


class TiledFactor(Factor):
    def __init__(self, blr: BLR, eps: float, cap: int):
        super().__init__(blr, eps, cap)
        self.Tkk = {}
        self.Tik = {}
        self.counts = {"geqrt": 0, "larfb": 0, "tpqrt": 0, "tpmqrt": 0}

    # tasks -----------------------------------------------------------------
    def geqrt(self, k):
        F, tau, T = dense.geqrt(self.A.D[(k, k)])
        self.A.D[(k, k)] = F
        self.Ykk[k] = dense.unit_lower(F)
        self.Tkk[k] = T

    def larfb(self, k, j):
        Y, T = self.Ykk[k], self.Tkk[k]
        if self.A.fmt[k, j] == DENSE:
            self.A.D[(k, j)] = dense.apply_qt_left(Y, T, self.A.D[(k, j)])
        else:
            self.A.U[(k, j)] = dense.apply_qt_left(Y, T, self.A.U[(k, j)])

    def tpqrt(self, i, k):
        Dkk = self.A.D[(k, k)]
        if self.A.fmt[i, k] == DENSE:
            bottom = self.A.D[(i, k)]
        else:
            bottom = self.A.V[(i, k)].T
        Rn, Y, tau, T = dense.tpqrt(np.triu(Dkk), bottom)
        self.A.D[(k, k)] = np.tril(Dkk, -1) + Rn
        if self.A.fmt[i, k] == DENSE:
            self.A.D[(i, k)] = Y
            self.Yfmt[(i, k)] = DENSE
        else:
            self.Yl[(i, k)] = Y
            self.A.V.pop((i, k))
            self.Yfmt[(i, k)] = LOWRANK
        self.Tik[(i, k)] = T

    def tpmqrt(self, i, k, j):
        e, c, st = self.eps, self.cap, self.stats
        Yr, T = self.ytilde(i, k), self.Tik[(i, k)]
        R, A = self.val(k, j), self.val(i, j)
        W = blrops.t_times(T, blrops.add(R, blrops.yt_times(Yr, A), 1.0, e, c, st), True)
        self.store(k, j, blrops.add(R, W, -1.0, e, c, st))
        self.store(i, j, blrops.add(A, blrops.y_times(Yr, W), -1.0, e, c, st))

    def run_task(self, t):
        self.counts[t[0]] += 1
        getattr(self, t[0])(*t[1:])

    def run(self, order: str = "sequential", seed: int = 0, stop_after_k=None):
        tasks = task_list(self.p, self.q, stop_after_k)
        deps = build_dag(tasks) if order != "sequential" else None
        for idx in topo_order(tasks, deps, order, seed):
            self.run_task(tasks[idx])
        self.steps_done = self.q if stop_after_k is None else min(self.q, stop_after_k)
        return self

    # Q application (Alg. 5) ------------------------------------------------
    def _blk(self, B, i):
        b = self.b
        return B[i * b:(i + 1) * b]

    def apply_qt(self, B: np.ndarray) -> np.ndarray:
        """B <- Q^T B, replaying the factorization order.  The TPQRT
        reflectors of step k touch the first (width of block column k) rows
        of block row k: all of them except in a narrower last block column."""
        B = np.array(B, dtype=np.float64, copy=True)
        for k in range(self.steps_done):
            Bd = self._blk(B, k)
            Bd[:] = dense.apply_qt_left(self.Ykk[k], self.Tkk[k], Bd)
            Bk = Bd[: self.Tkk[k].shape[0]]
            for i in range(k + 1, self.p):
                Bi = self._blk(B, i)
                Yr = self.ytilde(i, k)
                W = self.Tik[(i, k)].T @ (Bk + _yt_dense(Yr, Bi))
                Bk -= W
                Bi -= blrops.dense_of(blrops.y_times(Yr, ("D", W)))
        return B

    def apply_q(self, B: np.ndarray) -> np.ndarray:
        """B <- Q B: Alg. 5 loop order (k, i descending) with the update read
        as C <- (I - [I; Y] T [I; Y]^T) C (the printed formula lacks 'I -')."""
        B = np.array(B, dtype=np.float64, copy=True)
        for k in range(self.steps_done - 1, -1, -1):
            Bd = self._blk(B, k)
            Bk = Bd[: self.Tkk[k].shape[0]]
            for i in range(self.p - 1, k, -1):
                Bi = self._blk(B, i)
                Yr = self.ytilde(i, k)
                W = self.Tik[(i, k)] @ (Bk + _yt_dense(Yr, Bi))
                Bk -= W
                Bi -= blrops.dense_of(blrops.y_times(Yr, ("D", W)))
            Bd[:] = dense.apply_q_left(self.Ykk[k], self.Tkk[k], Bd)
        return B


def factor(blr: BLR, eps: float, cap: int, order: str = "sequential",
           seed: int = 0, stop_after_k=None, copy: bool = True) -> TiledFactor:
    f = TiledFactor(blr.copy() if copy else blr, eps, cap)
    return f.run(order, seed, stop_after_k)
