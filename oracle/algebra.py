"""O-C: the submatrix recurrence written out with dense index sets (tiny graphs).

TEST INFRASTRUCTURE ONLY (see the package docstring).

This follows the paper's algebraic statement directly, with no sparse data
structure at all:

  * Def 1 (Submatrix multiplication section): V_0 = [n], x_0 = 0 and
    V_k = V_{k-1} \\ supp(x_{k-1}); x_1 = e_s.
  * Theorem 1: x_{k+1} = A[V_{k+1}, V_k] x_k, evaluated here as a dense
    product of the submatrix picked out with ``np.ix_`` and the subvector
    x_k[V_k].  For directed graphs the product uses A^T (rows egress; the
    directed-graph paragraph of the operation-bounds section).
  * The semiring only matters through zero / nonzero (Notation section); three
    are evaluated: Boolean (OR, AND), arithmetic (+, *) and the (min, select)
    pair whose product of a frontier vertex j's value j+1 with A(i, j) is j+1,
    so that x_{k+1}(i) - 1 is the smallest frontier vertex reaching i.
  * Proposition 1 / Appendix A: with selection matrices S_k = diag(1[V_k]) and
    A_k = S_k A S_k, supp(S_{k+1} A_k A^{k-1} x_1) is the step-(k+1) support.

Vertex ids are 0-based; "step k" keeps the paper's 1-based step numbering, so
x_1 = e_s and supp(x_{k+1}) is the set of vertices at distance k.
"""
from __future__ import annotations

from typing import Dict, List

import numpy as np


def dense_adjacency(n: int, ptr, idx) -> np.ndarray:
    """A with A[i, j] = 1 for every CSR entry j in row i (edge i -> j)."""
    a = np.zeros((n, n), dtype=np.int64)
    ptr = np.asarray(ptr, dtype=np.int64)
    for i in range(n):
        for e in range(ptr[i], ptr[i + 1]):
            a[i, int(idx[e])] = 1
    return a


def _semiring_product(sub: np.ndarray, vec: np.ndarray, semiring: str) -> np.ndarray:
    """sub (rows x cols, 0/1) times vec (cols) in the named semiring."""
    if semiring == "boolean":
        return np.array([int(any(sub[r, c] and vec[c] for c in range(sub.shape[1])))
                         for r in range(sub.shape[0])], dtype=np.int64)
    if semiring == "arithmetic":
        return sub @ vec
    if semiring == "minselect":
        out = np.zeros(sub.shape[0], dtype=np.int64)
        for r in range(sub.shape[0]):
            best = 0
            for c in range(sub.shape[1]):
                if sub[r, c] and vec[c]:
                    prod = vec[c]               # select: A is a 0/1 pattern
                    best = prod if best == 0 else min(best, prod)
            out[r] = best
        return out
    raise ValueError(semiring)


def submatrix_steps(a: np.ndarray, s: int, semiring: str = "boolean",
                    symmetric_form: bool = False) -> Dict[str, List]:
    """Run x_{k+1} = M[V_{k+1}, V_k] x_k with M = A^T (M = A when A is symmetric).

    With ``symmetric_form`` the rows are V_k instead of V_{k+1} (the form the
    paper notes is also valid).  Returns the per-step vectors x_1, x_2, ... and
    the sets V_1, V_2, ... as sorted lists.  For the (min, select) semiring the
    input vector at each step holds j+1 at every j in its support.
    """
    n = a.shape[0]
    m = a.T
    V = {0: list(range(n))}
    x = {0: np.zeros(n, dtype=np.int64)}
    # x_1 = e_s; V_1 = V_0 \ supp(x_0) = [n]
    x1 = np.zeros(n, dtype=np.int64)
    x1[s] = 1
    x[1] = x1
    V[1] = [v for v in V[0] if x[0][v] == 0]
    V[2] = [v for v in V[1] if x[1][v] == 0]
    k = 1
    while np.any(x[k] != 0):
        rows = V[k] if symmetric_form else V[k + 1]
        cols = V[k]
        xin = x[k].copy()
        if semiring == "minselect":
            xin = np.where(xin != 0, np.arange(n, dtype=np.int64) + 1, 0)
        sub = m[np.ix_(rows, cols)] if rows and cols else np.zeros((len(rows), len(cols)), np.int64)
        y_sub = _semiring_product(sub, xin[cols], semiring) if rows else np.zeros(0, np.int64)
        nxt = np.zeros(n, dtype=np.int64)
        nxt[rows] = y_sub
        if symmetric_form:
            # rows of the current frontier may appear; S_{k+1} removes them
            nxt[[v for v in range(n) if v not in set(V[k + 1])]] = 0
        x[k + 1] = nxt
        V[k + 2] = [v for v in V[k + 1] if x[k + 1][v] == 0]
        k += 1
    steps = k  # x_k is the first all-zero vector
    return dict(x=[x[i] for i in range(1, steps + 1)],
                V=[V[i] for i in range(1, steps + 2)])


def bfs(a: np.ndarray, s: int):
    """level/parent from the recurrence: Boolean supports give the levels, the
    (min, select) semiring gives the parent."""
    n = a.shape[0]
    level = np.full(n, -1, dtype=np.int64)
    parent = np.full(n, -1, dtype=np.int64)
    sb = submatrix_steps(a, s, "boolean")["x"]
    sm = submatrix_steps(a, s, "minselect")["x"]
    for k, (xb, xm) in enumerate(zip(sb, sm)):       # xb = x_{k+1}: distance k
        for v in np.nonzero(xb)[0]:
            level[v] = k
            parent[v] = s if k == 0 else xm[v] - 1
    return level, parent


def prop1_supports(a: np.ndarray, s: int) -> List[List[int]]:
    """supp(S_{k+1} A_k A^{k-1} x_1) for k = 1, 2, ... (Boolean), using the V_k
    of the recurrence; Appendix A proves these equal supp(x_{k+1})."""
    n = a.shape[0]
    m = (a.T != 0).astype(np.int64)
    steps = submatrix_steps(a, s, "boolean")
    V = steps["V"]                                  # V[0] = V_1, V[1] = V_2, ...
    x1 = np.zeros(n, dtype=np.int64)
    x1[s] = 1
    out = []
    y = x1.copy()                                   # y_1 = x_1
    for k in range(1, len(steps["x"])):
        Sk = np.diag([1 if v in set(V[k - 1]) else 0 for v in range(n)])
        Sk1 = np.diag([1 if v in set(V[k]) else 0 for v in range(n)])
        Ak = Sk @ m @ Sk
        z = (Sk1 @ (Ak @ y) != 0).astype(np.int64)
        out.append(sorted(int(v) for v in np.nonzero(z)[0]))
        y = (m @ y != 0).astype(np.int64)           # y_{k+1} = A y_k (Boolean)
    return out
