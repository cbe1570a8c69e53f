"""O-D: brute force on tiny graphs, independent of any search procedure.

TEST INFRASTRUCTURE ONLY (see the package docstring).

level[v] = min{t >= 0 : ((A^T)^t e_s)_v != 0}: the shortest walk length, read off
Boolean matrix powers (a walk of length t from s to v exists iff that entry is
nonzero; the shortest walk is a shortest path).  parent follows the definition
min{u : A(u, v) = 1, level[u] = level[v] - 1}.
"""
from __future__ import annotations

import itertools
from typing import Iterator, Tuple

import numpy as np


def levels_by_powers(a: np.ndarray, s: int) -> np.ndarray:
    n = a.shape[0]
    m = (a.T != 0).astype(np.int64)
    level = np.full(n, -1, dtype=np.int64)
    vec = np.zeros(n, dtype=np.int64)
    vec[s] = 1
    for t in range(n):
        for v in np.nonzero(vec)[0]:
            if level[v] < 0:
                level[v] = t
        vec = (m @ vec != 0).astype(np.int64)
    return level


def parents_by_definition(a: np.ndarray, s: int, level: np.ndarray) -> np.ndarray:
    n = a.shape[0]
    parent = np.full(n, -1, dtype=np.int64)
    parent[s] = s
    for v in range(n):
        if level[v] > 0:
            cands = [u for u in range(n) if a[u, v] and level[u] == level[v] - 1]
            parent[v] = min(cands)
    return parent


def bfs(a: np.ndarray, s: int) -> Tuple[np.ndarray, np.ndarray]:
    lv = levels_by_powers(a, s)
    return lv, parents_by_definition(a, s, lv)


def all_undirected(nv: int) -> Iterator[np.ndarray]:
    """Every simple undirected graph on nv labelled vertices (2^(nv(nv-1)/2))."""
    pairs = list(itertools.combinations(range(nv), 2))
    for mask in range(1 << len(pairs)):
        a = np.zeros((nv, nv), dtype=np.int64)
        for b, (i, j) in enumerate(pairs):
            if mask >> b & 1:
                a[i, j] = a[j, i] = 1
        yield a


def all_directed(nv: int) -> Iterator[np.ndarray]:
    """Every simple directed graph (no self-loops) on nv labelled vertices."""
    arcs = [(i, j) for i in range(nv) for j in range(nv) if i != j]
    for mask in range(1 << len(arcs)):
        a = np.zeros((nv, nv), dtype=np.int64)
        for b, (i, j) in enumerate(arcs):
            if mask >> b & 1:
                a[i, j] = 1
        yield a


def to_csr(a: np.ndarray):
    """Dense 0/1 matrix -> (ptr, idx) int32 CSR of rows, plus CSC (in_ptr, in_idx)."""
    n = a.shape[0]
    ptr = np.zeros(n + 1, dtype=np.int32)
    idx = []
    for i in range(n):
        cols = np.nonzero(a[i])[0]
        idx.extend(cols.tolist())
        ptr[i + 1] = len(idx)
    in_ptr = np.zeros(n + 1, dtype=np.int32)
    in_idx = []
    for j in range(n):
        rows = np.nonzero(a[:, j])[0]
        in_idx.extend(rows.tolist())
        in_ptr[j + 1] = len(in_idx)
    return ptr, np.array(idx, dtype=np.int32), in_ptr, np.array(in_idx, dtype=np.int32)
