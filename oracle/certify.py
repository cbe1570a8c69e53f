"""Certificate I1-I4 for a (level, parent) pair, O(n + nnz), vectorized numpy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

  I1  level[s] = 0, parent[s] = s; level[v] = 0 only for v = s;
      level[v] = -1 exactly when parent[v] = -1.
  I2  every edge u -> v with level[u] >= 0 has level[v] >= 0 and
      level[v] <= level[u] + 1.
  I3  every reached v != s has an edge parent[v] -> v and
      level[parent[v]] = level[v] - 1.
  I4  no edge u -> v with u < parent[v] and level[u] = level[v] - 1.

Why this is complete: I2 along a shortest path gives level <= dist and closes
the reached set under out-edges; I3 gives a parent chain of length level[v]
back to s, so level >= dist and every reached vertex is reachable.  Hence
level = dist exactly, and I4 then fixes parent as the smallest in-neighbour one
level up - the unique answer.
"""
from __future__ import annotations

from typing import List

import numpy as np


def check(n: int, ptr, idx, source: int, level, parent) -> List[str]:
    """Return the list of violated invariants (empty = certified)."""
    ptr = np.asarray(ptr, dtype=np.int64)
    idx = np.asarray(idx, dtype=np.int64)
    level = np.asarray(level, dtype=np.int64)
    parent = np.asarray(parent, dtype=np.int64)
    errs: List[str] = []
    if level.shape != (n,) or parent.shape != (n,):
        return ["shape"]
    # I1
    if level[source] != 0 or parent[source] != source:
        errs.append("I1: source entries")
    zero = np.nonzero(level == 0)[0]
    if len(zero) != 1 or zero[0] != source:
        errs.append("I1: level 0 only at the source")
    if not np.array_equal(level == -1, parent == -1):
        errs.append("I1: unreached <-> parent -1")
    if np.any(level < -1) or np.any(parent < -1) or np.any(parent >= n):
        errs.append("I1: value range")
        return errs
    deg = np.diff(ptr)
    rows = np.repeat(np.arange(n, dtype=np.int64), deg)
    lu = level[rows]
    lv = level[idx]
    # I2
    live = lu >= 0
    if np.any(lv[live] < 0) or np.any(lv[live] > lu[live] + 1):
        errs.append("I2: edge level gap")
    # I3: the parent edge exists (rows sorted, columns sorted within rows => keys sorted)
    reached = np.nonzero((level > 0))[0]
    if len(reached):
        keys = rows * n + idx
        order_ok = bool(np.all(keys[1:] >= keys[:-1])) if len(keys) > 1 else True
        if not order_ok:
            keys = np.sort(keys)
        want = parent[reached] * n + reached
        pos = np.searchsorted(keys, want)
        pos = np.minimum(pos, len(keys) - 1) if len(keys) else pos
        if len(keys) == 0 or np.any(keys[pos] != want):
            errs.append("I3: parent edge missing")
        if np.any(level[parent[reached]] != level[reached] - 1):
            errs.append("I3: parent level")
    # I4
    cand = (lv > 0) & (lu == lv - 1)
    if np.any(rows[cand] < parent[idx[cand]]):
        errs.append("I4: smaller in-neighbour one level up")
    return errs
