"""Format rules of BLR tile arithmetic (paper Section 3.1, OP1-OP4 and
Alg. 6) as used by the reflector applications of Sections 3.3.2 and 3.4.4.

A tile value is ('D', M) or ('L', U, V) meaning U V^T.  A reflector block
Ytilde is ('D', Y) or ('L', Uy, Yl) meaning Uy @ Yl (Yl is r x b).
* OP1: low-rank + dense = dense (so a low-rank target that receives a dense
  update becomes dense: this is the fill-in rule under strong admissibility);
* OP2: low-rank + low-rank = low-rank, rounded (Alg. 6), once per addition;
* OP3/OP4: products with a low-rank factor stay low-rank.
"""
from __future__ import annotations

import numpy as np

from . import lowrank


def dense_of(X):
    return X[1] if X[0] == "D" else X[1] @ X[2].T


def yt_times(Yr, Ar):
    """P = Ytilde^T A."""
    if Yr[0] == "D":
        Y = Yr[1]
        if Ar[0] == "D":
            return ("D", Y.T @ Ar[1])
        return ("L", Y.T @ Ar[1], Ar[2])
    Uy, Yl = Yr[1], Yr[2]
    if Ar[0] == "D":
        return ("L", Yl.T, Ar[1].T @ Uy)
    return ("L", Yl.T @ (Uy.T @ Ar[1]), Ar[2])


def y_times(Yr, W):
    """Ytilde W."""
    if Yr[0] == "D":
        Y = Yr[1]
        if W[0] == "D":
            return ("D", Y @ W[1])
        return ("L", Y @ W[1], W[2])
    Uy, Yl = Yr[1], Yr[2]
    if W[0] == "D":
        return ("L", Uy, W[1].T @ Yl.T)
    return ("L", Uy, W[2] @ (Yl @ W[1]).T)


def t_times(T, X, trans: bool):
    """T^T X (trans) or T X, applied to the left factor of a low-rank X."""
    M = T.T if trans else T
    if X[0] == "D":
        return ("D", M @ X[1])
    return ("L", M @ X[1], X[2])


def add(X, Y, sign: float, eps: float, cap: int, stats):
    """X + sign * Y under OP1/OP2."""
    if X[0] == "D" or Y[0] == "D":
        return ("D", dense_of(X) + sign * dense_of(Y))
    U, V = lowrank.rounded_add([(X[1], X[2]), (sign * Y[1], Y[2])], eps, cap, stats)
    return ("L", U, V)
