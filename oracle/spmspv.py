"""One masked sparse-matrix x sparse-vector product y = A^T[R, C] x over a
chosen semiring, by its definition (the Notation section's semirings; the
submatrix A^T[V_{k+1}, V_k] of Definition 1 is the case R = the rows still
unvisited, C = all columns).

TEST INFRASTRUCTURE ONLY: nothing in the product library imports or runs this
module (see the package docstring).  It shares no code with the GPU path.

A is pattern-only (every stored entry is 1); values are unsigned 64-bit
integers and arithmetic wraps modulo 2^64.  For the entries (i, j) of column
j of A^T (the out-list of j) with j in the vector, C allowing j and R
allowing i, the product adds A(i, j) (x) x(j) into y(i) with (+):

  semiring     (x): 1 (x) v          (+)     identity
  boolean      v != 0                 OR      0
  arithmetic   v                      +       0
  min_plus     v + 1 (saturating)     min     2^64 - 1
  min_select   v                      min     2^64 - 1

y's support is structural: every allowed row that receives at least one
product, whatever its value.  Duplicate vector indices each contribute.  The
result is returned with the support in ascending order.
"""
from __future__ import annotations

from typing import Optional, Tuple

import numpy as np

SEMIRINGS = ("boolean", "arithmetic", "min_plus", "min_select")
MASK64 = (1 << 64) - 1


def _mul(semiring: str, v: int) -> int:
    if semiring == "boolean":
        return 1 if v != 0 else 0
    if semiring == "min_plus":
        return v if v == MASK64 else v + 1
    return v


def _add(semiring: str, a: int, b: int) -> int:
    if semiring == "boolean":
        return a | b
    if semiring == "arithmetic":
        return (a + b) & MASK64
    return a if a < b else b


def _allowed(mask: Optional[np.ndarray], complement: bool, v: int) -> bool:
    if mask is None:
        return True
    bit = bool(mask[v])
    return bit != complement


def masked_spmspv(g, semiring: str, x_idx, x_val, row_mask: Optional[np.ndarray] = None,
                  col_mask: Optional[np.ndarray] = None, row_complement: bool = False,
                  col_complement: bool = False) -> Tuple[np.ndarray, np.ndarray]:
    """y = A^T[R, C] x on a graphgen.CSRGraph.  Masks are boolean arrays of
    length n (None = every index allowed); a complemented mask allows the
    indices it does not hold.  Returns (y_idx int32 ascending, y_val uint64)."""
    if semiring not in SEMIRINGS:
        raise ValueError(semiring)
    ptr, idx = g.ptr, g.idx
    acc = {}
    for j, v in zip(np.asarray(x_idx).tolist(), np.asarray(x_val, dtype=np.uint64).tolist()):
        if not _allowed(col_mask, col_complement, j):
            continue
        p = _mul(semiring, int(v))
        for e in range(int(ptr[j]), int(ptr[j + 1])):
            i = int(idx[e])
            if not _allowed(row_mask, row_complement, i):
                continue
            acc[i] = _add(semiring, acc[i], p) if i in acc else p
    keys = sorted(acc)
    return (np.array(keys, dtype=np.int32),
            np.array([acc[i] for i in keys], dtype=np.uint64))
