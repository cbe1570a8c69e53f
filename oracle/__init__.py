"""CPU oracle for the masked SpMSpV breadth-first search.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs anything from this package: only the tests, the smoke check and the
bench's CPU-baseline leg do.  It shares no code with the GPU path; the two meet
only at the seeded graph generators (``graphgen``), which hold none of the
search's arithmetic.

Contents
  * ``bfs_queue``   (O-A, C): FIFO-queue BFS + a separate pass applying the
                    min-parent definition.
  * ``bfs_alg2``    (O-B, C): the CSR form of the method (Algorithm 2) with an
                    explicit (min, select) semiring and operation counters.
  * ``algebra``     (O-C, numpy): the submatrix recurrence x_{k+1} =
                    A^T[V_{k+1}, V_k] x_k written with dense index sets.
  * ``brute``       (O-D, numpy): levels from Boolean matrix powers.
  * ``certify``     (I1-I4): a complete O(n + nnz) certificate for (level, parent).
  * ``mlp_ref``     float64 reference of the variant-selector network.
  * ``spmspv``      one masked product y = A^T[R, C] x over the Boolean,
                    arithmetic, min-plus or (min, select) semiring, by its
                    definition.
  * ``compare``     the searches the Experiments section compares against
                    (SpMV-BFS, SpMSpV-BFS, SpMmSpV-BFS) and the method, step by
                    step, with their algebraic operation counts (Table 2).

The result every function returns (Theorem 1 gives the levels; the parent tie
rule picks the smallest frontier in-neighbour):
  level[v]  = fewest edges on a path s -> v, -1 if unreached;
  parent[s] = s; parent[v] = min{u in N-(v) : level[u] = level[v]-1}; -1 if unreached.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bfs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build_lib(force: bool = False) -> str:
    """Compile the C oracle with gcc (no GPU toolchain involved)."""
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_POSIX_C_SOURCE=199309L",
                               "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        path = build_lib()
        lib = ctypes.CDLL(path)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_bfs_queue.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p,
                                         ctypes.c_int32, i32p, i32p]
        lib.oracle_bfs_queue.restype = ctypes.c_int
        lib.oracle_bfs_alg2.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_int32,
                                        ctypes.c_int32, i32p, i32p,
                                        ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_bfs_alg2.restype = ctypes.c_int
        lib.oracle_time_queue_bfs.argtypes = [ctypes.c_int32, i32p, i32p, i32p, i32p,
                                              i32p, ctypes.c_int32, i32p, i32p]
        lib.oracle_time_queue_bfs.restype = ctypes.c_double
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _as_i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def bfs_queue(n: int, ptr, idx, source: int, in_ptr=None, in_idx=None
              ) -> Tuple[np.ndarray, np.ndarray]:
    """O-A.  in_ptr/in_idx default to the CSR itself (undirected graphs)."""
    ptr, idx = _as_i32(ptr), _as_i32(idx)
    in_ptr = ptr if in_ptr is None else _as_i32(in_ptr)
    in_idx = idx if in_idx is None else _as_i32(in_idx)
    level = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    rc = _load().oracle_bfs_queue(n, _p32(ptr), _p32(idx), _p32(in_ptr), _p32(in_idx),
                                  int(source), _p32(level), _p32(parent))
    if rc != 0:
        raise ValueError(f"oracle_bfs_queue failed ({rc})")
    return level, parent


def bfs_alg2(n: int, ptr, idx, source: int, mode: int = 0):
    """O-B.  Returns (level, parent, counters) with counters =
    {mults, tests, steps, appended}; see bfs_oracle.c for the three modes."""
    ptr, idx = _as_i32(ptr), _as_i32(idx)
    level = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    cnt = np.zeros(4, dtype=np.int64)
    rc = _load().oracle_bfs_alg2(n, _p32(ptr), _p32(idx), int(source), int(mode),
                                 _p32(level), _p32(parent),
                                 cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError(f"oracle_bfs_alg2 failed ({rc})")
    return level, parent, dict(mults=int(cnt[0]), tests=int(cnt[1]),
                               steps=int(cnt[2]), appended=int(cnt[3]))


def time_queue_bfs(n: int, ptr, idx, sources, in_ptr=None, in_idx=None) -> float:
    """Wall seconds (CLOCK_MONOTONIC, inside C) for O-A from every source in turn."""
    ptr, idx = _as_i32(ptr), _as_i32(idx)
    in_ptr = ptr if in_ptr is None else _as_i32(in_ptr)
    in_idx = idx if in_idx is None else _as_i32(in_idx)
    src = _as_i32(sources)
    level = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int32)
    t = _load().oracle_time_queue_bfs(n, _p32(ptr), _p32(idx), _p32(in_ptr), _p32(in_idx),
                                      _p32(src), len(src), _p32(level), _p32(parent))
    if t < 0:
        raise ValueError("oracle_time_queue_bfs failed")
    return t


def bfs_graph(g, source: int):
    """O-A on a graphgen.CSRGraph."""
    ip, ii = g.csc()
    return bfs_queue(g.n, g.ptr, g.idx, source, ip, ii)


def component_stats(g, level: np.ndarray) -> dict:
    """n_c (reached vertices), nnz_c (out-entries of reached vertices), levels."""
    reached = level >= 0
    deg = np.diff(g.ptr.astype(np.int64))
    nnz_c = int(deg[reached].sum())
    return dict(n_c=int(reached.sum()), nnz_c=nnz_c,
                m_c=nnz_c if g.directed else nnz_c // 2,
                levels=int(level.max()) + 1 if reached.any() else 0)
