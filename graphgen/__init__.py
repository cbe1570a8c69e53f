"""Seeded synthetic graph generators shared by the tests, the bench and the oracle checks.

This module only builds inputs: it holds none of the search's arithmetic.  Every
graph is a pattern-only adjacency matrix A (A(i,j) = 1 for an edge i -> j, rows
are egress as in the paper's directed-graph section) stored as 0-based int32
CSR (out-neighbours, sorted ascending) and, for directed graphs, the CSC
(in-neighbours, sorted ascending).  Undirected graphs are symmetric, so their
CSC is the CSR itself.

The paper measures on SNAP graphs (Table 1) that are not available here; the
generators below make stand-ins of the same kinds: low-diameter power-law
graphs (R-MAT, for com-LiveJournal / com-Orkut), large-diameter planar graphs
(percolated grid, for roadNet-*), and small uniform random graphs (ER).

All randomness comes from numpy's PCG64 `default_rng(seed)`.
"""
from __future__ import annotations

import dataclasses
import hashlib
import os
from typing import Callable, List, Optional, Sequence

import numpy as np

__all__ = [
    "CSRGraph", "from_edges", "erdos_renyi", "rmat", "grid", "block_diagonal",
    "pick_sources", "cached", "path_graph", "cycle_graph", "star_graph",
    "complete_graph", "binary_tree", "full_grid",
]


@dataclasses.dataclass
class CSRGraph:
    """Pattern-only graph in 0-based int32 CSR (+ CSC when directed)."""
    n: int
    ptr: np.ndarray            # int32[n+1]; out-neighbour offsets
    idx: np.ndarray            # int32[ptr[n]]; out-neighbours, ascending per row
    directed: bool = False
    in_ptr: Optional[np.ndarray] = None   # int32[n+1]; in-neighbour offsets (directed only)
    in_idx: Optional[np.ndarray] = None   # int32[nnz]; in-neighbours, ascending per column
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.ptr[-1])

    def out_degree(self) -> np.ndarray:
        return np.diff(self.ptr.astype(np.int64))

    def csc(self):
        """(in_ptr, in_idx): in-neighbour lists; the CSR itself when undirected."""
        if not self.directed:
            return self.ptr, self.idx
        return self.in_ptr, self.in_idx

    def save(self, path: str) -> None:
        arrs = dict(n=np.int64(self.n), ptr=self.ptr, idx=self.idx,
                    directed=np.int8(self.directed))
        if self.directed:
            arrs.update(in_ptr=self.in_ptr, in_idx=self.in_idx)
        tmp = path + ".tmp.npz"
        np.savez(tmp, **arrs)
        os.replace(tmp, path)

    @staticmethod
    def load(path: str, name: str = "") -> "CSRGraph":
        z = np.load(path)  # allow_pickle stays False
        directed = bool(int(z["directed"]))
        return CSRGraph(int(z["n"]), z["ptr"], z["idx"], directed,
                        z["in_ptr"] if directed else None,
                        z["in_idx"] if directed else None, name)


def _csr_from_keys(n: int, keys: np.ndarray):
    """keys = sorted unique int64 (row * n + col) -> (ptr int32, idx int32)."""
    rows = keys // n
    cols = (keys - rows * n).astype(np.int32)
    counts = np.bincount(rows, minlength=n)
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=ptr[1:])
    if ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR offsets")
    return ptr.astype(np.int32), cols


def from_edges(n: int, src: np.ndarray, dst: np.ndarray, directed: bool = False,
               name: str = "") -> CSRGraph:
    """Build a simple graph (no self-loops, no duplicate edges) from an edge list.

    Undirected input is symmetrized.  Neighbour lists come out sorted ascending.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    if not directed:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
    keys = np.unique(src * n + dst)
    del src, dst
    ptr, idx = _csr_from_keys(n, keys)
    if not directed:
        return CSRGraph(n, ptr, idx, False, name=name)
    rows = keys // n
    cols = keys - rows * n
    tkeys = cols * n + rows
    del rows, cols, keys
    tkeys.sort()
    in_ptr, in_idx = _csr_from_keys(n, tkeys)
    return CSRGraph(n, ptr, idx, True, in_ptr, in_idx, name=name)


def erdos_renyi(n: int, avg_degree: float, seed: int) -> CSRGraph:
    """Undirected G(n, M) with M = n*avg_degree/2 uniform ordered pairs, symmetrized."""
    rng = np.random.default_rng(seed)
    m = int(round(n * avg_degree / 2))
    src = rng.integers(0, n, m, dtype=np.int64)
    dst = rng.integers(0, n, m, dtype=np.int64)
    return from_edges(n, src, dst, directed=False, name=f"er_n{n}_d{avg_degree:g}_s{seed}")


def rmat(scale: int, edgefactor: int = 16, seed: int = 1, directed: bool = False,
         a: float = 0.57, b: float = 0.19, c: float = 0.19, permute: bool = True) -> CSRGraph:
    """R-MAT: `scale` independent quadrant draws per edge, no noise, random relabelling."""
    n = 1 << scale
    m = edgefactor * n
    rng = np.random.default_rng(seed)
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    ab, abc = a + b, a + b + c
    for _ in range(scale):
        r = rng.random(m, dtype=np.float32)
        src <<= 1
        dst <<= 1
        src |= (r >= ab)
        dst |= ((r >= a) & (r < ab)) | (r >= abc)
        del r
    if permute:
        perm = rng.permutation(n).astype(np.int64)
        src = perm[src]
        dst = perm[dst]
    kind = "d" if directed else "u"
    return from_edges(n, src, dst, directed=directed, name=f"rmat{kind}_s{scale}_e{edgefactor}_s{seed}")


def grid(width: int, p: float, seed: int, height: Optional[int] = None) -> CSRGraph:
    """Undirected 4-neighbour W x H grid (row-major labels), each lattice edge kept with prob p.

    Horizontal edges are drawn first (row-major), then vertical ones.
    """
    h = width if height is None else height
    w = width
    rng = np.random.default_rng(seed)
    hk = rng.random(h * (w - 1)) < p          # edge (r,c)-(r,c+1)
    vk = rng.random((h - 1) * w) < p          # edge (r,c)-(r+1,c)
    n = w * h
    hk2 = np.zeros((h, w), dtype=bool)
    hk2[:, :-1] = hk.reshape(h, w - 1)        # right neighbour present
    vk2 = np.zeros((h, w), dtype=bool)
    vk2[:-1, :] = vk.reshape(h - 1, w)        # down neighbour present
    right = hk2.ravel()
    down = vk2.ravel()
    left = np.zeros(n, dtype=bool)
    left[1:] = right[:-1]
    up = np.zeros(n, dtype=bool)
    up[w:] = down[:-w]
    deg = up.astype(np.int32) + left + right + down
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=ptr[1:])
    idx = np.empty(int(ptr[-1]), dtype=np.int32)
    v = np.arange(n, dtype=np.int64)
    pos = ptr[:-1].copy()
    for mask, off in ((up, -w), (left, -1), (right, 1), (down, w)):   # ascending order
        sel = np.nonzero(mask)[0]
        idx[pos[sel]] = (v[sel] + off).astype(np.int32)
        pos[sel] += 1
    return CSRGraph(n, ptr.astype(np.int32), idx, False, name=f"grid_{w}x{h}_p{p:g}_s{seed}")


def full_grid(width: int, height: Optional[int] = None) -> CSRGraph:
    """The complete 4-neighbour grid (every lattice edge present)."""
    return grid(width, 2.0, 0, height)   # p > 1 keeps every edge


def block_diagonal(graphs: Sequence[CSRGraph], name: str = "blockdiag"):
    """Pack undirected graphs into one block-diagonal CSR; returns (graph, vertex offsets int64)."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    for g_i, g in enumerate(graphs):
        offs[g_i + 1] = offs[g_i] + g.n
    n = int(offs[-1])
    nnz = sum(g.nnz for g in graphs)
    ptr = np.zeros(n + 1, dtype=np.int64)
    idx = np.empty(nnz, dtype=np.int32)
    e = 0
    for g_i, g in enumerate(graphs):
        o = int(offs[g_i])
        ptr[o + 1:o + g.n + 1] = g.ptr[1:].astype(np.int64) + e
        idx[e:e + g.nnz] = g.idx + o
        e += g.nnz
    if any(g.directed for g in graphs):
        raise ValueError("block_diagonal packs undirected graphs only")
    return CSRGraph(n, ptr.astype(np.int32), idx, False, name=name), offs


def pick_sources(g: CSRGraph, count: int, seed: int) -> np.ndarray:
    """`count` distinct vertices of nonzero out-degree, drawn without replacement."""
    rng = np.random.default_rng(seed)
    cand = np.nonzero(g.out_degree() > 0)[0]
    if count > len(cand):
        raise ValueError("not enough vertices with nonzero degree")
    return np.sort(rng.choice(cand, size=count, replace=False)).astype(np.int32)


# ---- small closed-form families ------------------------------------------------

def path_graph(n: int) -> CSRGraph:
    v = np.arange(n - 1)
    return from_edges(n, v, v + 1, name=f"path{n}")


def cycle_graph(n: int) -> CSRGraph:
    v = np.arange(n)
    return from_edges(n, v, (v + 1) % n, name=f"cycle{n}")


def star_graph(n: int, center: int = 0) -> CSRGraph:
    leaves = np.array([v for v in range(n) if v != center])
    return from_edges(n, np.full(len(leaves), center), leaves, name=f"star{n}")


def complete_graph(n: int) -> CSRGraph:
    u, v = np.triu_indices(n, 1)
    return from_edges(n, u, v, name=f"K{n}")


def binary_tree(n: int) -> CSRGraph:
    v = np.arange(1, n)
    return from_edges(n, (v - 1) // 2, v, name=f"bintree{n}")


# ---- on-disk cache ---------------------------------------------------------------

def cache_dir() -> str:
    d = os.environ.get("BFS_GRAPH_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "bfs_graphs")
    os.makedirs(d, exist_ok=True)
    return d


def cached(key: str, builder: Callable[[], CSRGraph]) -> CSRGraph:
    """Build once and keep as .npz keyed by `key` (which must encode every parameter)."""
    fn = os.path.join(cache_dir(), hashlib.sha1(key.encode()).hexdigest()[:16] + ".npz")
    if os.path.exists(fn):
        try:
            return CSRGraph.load(fn, key)
        except Exception:
            pass
    g = builder()
    g.name = key
    try:
        g.save(fn)
    except OSError:
        pass
    return g


# ---- the named workloads -------------------------------------------------------------

def workload(name: str) -> CSRGraph:
    """The standard synthetic workloads by name (cached)."""
    builders = {
        "er16k": lambda: erdos_renyi(16384, 8, 1),
        "rmat22": lambda: rmat(22, 16, 1, directed=False),
        "grid4096": lambda: grid(4096, 0.9, 3),
        "rmat20d": lambda: rmat(20, 16, 1, directed=True),
    }
    if name in builders:
        return cached(name, builders[name])
    if name.startswith("rmat") and name[4:].isdigit():           # rmatS: undirected, seed 1
        s = int(name[4:])
        return cached(name, lambda: rmat(s, 16, 1, directed=False))
    if name.startswith("rmatd") and name[5:].isdigit():
        s = int(name[5:])
        return cached(name, lambda: rmat(s, 16, 1, directed=True))
    if name.startswith("grid") and name[4:].isdigit():
        w = int(name[4:])
        return cached(name, lambda: grid(w, 0.9, 3))
    raise KeyError(name)


def er_family(count: int = 64, seed_base: int = 1000, lo: int = 10, hi: int = 18,
              dmin: float = 4.0, dmax: float = 32.0) -> List[CSRGraph]:
    """Uneven ER graphs: n_g = round(2^U(lo,hi)), d_g ~ U(dmin,dmax), graph g seeded seed_base+g."""
    out = []
    for g_i in range(count):
        rng = np.random.default_rng(seed_base + g_i)
        n_g = int(round(2.0 ** rng.uniform(lo, hi)))
        d_g = float(rng.uniform(dmin, dmax))
        out.append(erdos_renyi(n_g, d_g, seed_base + g_i))
    return out
