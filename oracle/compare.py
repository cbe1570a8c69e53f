"""The search family the Experiments section compares the method against
(SpMV-BFS, SpMSpV-BFS, SpMmSpV-BFS), and the method itself, run step by step
on the CPU with their algebraic operation counts.

TEST INFRASTRUCTURE ONLY: nothing in the product library imports or runs this
module (see the package docstring).  It shares no code with the GPU path.

Counting convention (Experiments section, Table 2): two operations (one
semiring multiply and one add) for every matrix nonzero a step multiplies.  A
search takes one step per level: step k multiplies with the vector of level k,
and the last step finds no new vertex, so steps = eccentricity of s + 1
(the text's "one more than the diameter").

Members (the reading of the Experiments section's descriptions):
  * "spmv"    - dense vector: every nonzero of A is multiplied at every step;
                the vector is the indicator of the frontier F_k, so only
                frontier columns give a non-identity product.
  * "spmspv"  - sparse vector, not masked: x_{k+1} = A^T x_k over the whole
                support of x_k, from x_0 = e_s.  supp(x_k) is then the set W_k
                of vertices that a walk of exactly k edges reaches from s.  The
                visited set is kept aside only to assign levels.
  * "spmmspv" - the vector is the frontier F_k (masked), but every nonzero of
                its columns is multiplied and the visited test comes after the
                product.  2 nnz_c in all (each column is multiplied once).
  * "method"  - the masked submatrix product with Theorem 2's short circuit:
                one multiply per newly reached vertex, 2 (n_c - 1) in all.

Every member computes the same search: a row reached for the first time at
step k gets level k + 1 and, under the (min, select) semiring, the smallest
column of the product's support that reaches it (the smallest frontier
in-neighbour: a vertex of W_k with an edge to an unvisited row lies at
distance exactly k).
"""
from __future__ import annotations

from typing import Tuple

import numpy as np

MEMBERS = ("spmv", "spmspv", "spmmspv", "method")


def _entries(ptr: np.ndarray, idx: np.ndarray, cols: np.ndarray,
             with_cols: bool = True) -> Tuple[np.ndarray, np.ndarray]:
    """(column, row) of every nonzero in the given columns of A^T (out-lists);
    the column array is None unless asked for."""
    cols = cols.astype(np.int64)
    start = ptr[cols]
    deg = ptr[cols + 1] - start
    tot = int(deg.sum())
    if tot == 0:
        return (np.empty(0, np.int64) if with_cols else None), np.empty(0, np.int64)
    first = np.cumsum(deg) - deg
    pos = np.repeat(start - first, deg) + np.arange(tot, dtype=np.int64)
    return (np.repeat(cols, deg) if with_cols else None), idx[pos]


def run(g, s: int, member: str, ops_only: bool = False):
    """One search of `member` from s on a graphgen.CSRGraph.

    Returns (level, parent, ops, steps).  With ops_only the product values
    (hence level / parent) are skipped where the count does not need them:
    level then comes from the supports alone and parent is None.
    """
    if member not in MEMBERS:
        raise ValueError(member)
    n = g.n
    ptr = g.ptr.astype(np.int64)
    idx = g.idx.astype(np.int64)
    deg = np.diff(ptr)
    nnz = int(ptr[-1])
    level = np.full(n, -1, np.int64)
    parent = None if ops_only else np.full(n, -1, np.int64)
    level[s] = 0
    if parent is not None:
        parent[s] = s
    frontier = np.array([s], np.int64)       # F_k
    walk = np.array([s], np.int64)           # W_k (spmspv's vector support)
    ops = 0
    steps = 0
    k = 0
    while True:
        steps += 1
        # this step's multiplications
        if member == "spmv":
            ops += 2 * nnz
        elif member == "spmspv":
            ops += 2 * int(deg[walk].sum())
        elif member == "spmmspv":
            ops += 2 * int(deg[frontier].sum())
        # the product's support and values: columns that carry a nonzero of x_k
        vec = walk if member == "spmspv" else frontier
        cols, rows = _entries(ptr, idx, vec, with_cols=parent is not None)
        reached = np.zeros(n, bool)
        reached[rows] = True
        new = np.nonzero(reached & (level < 0))[0]
        if member == "method":
            ops += 2 * len(new)                  # one multiply per claimed row
        if len(new) == 0:
            break
        level[new] = k + 1
        if parent is not None:
            y = np.full(n, np.iinfo(np.int64).max, np.int64)
            np.minimum.at(y, rows, cols)         # (min, select) product
            parent[new] = y[new]
        frontier = new
        if member == "spmspv":
            walk = np.nonzero(reached)[0]        # supp(x_{k+1}), not masked
        k += 1
    lv = level.astype(np.int32)
    pa = None if parent is None else parent.astype(np.int32)
    return lv, pa, ops, steps
