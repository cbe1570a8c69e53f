"""MI355X (gfx950) masked sparse-matrix x sparse-vector breadth-first search.

Python face of libbfs.so (include/bfs.h).  PyTorch supplies device memory and
streams; every step of a search runs in the library's HIP kernels.  There is
no CPU fallback: without the built library every call raises.

    g = Graph.from_csr(n, ptr, idx)                 # numpy / torch int32 CSR
    level, parent = bfs(g, source)                  # torch int32 on cuda
    level, parent = bfs(g, source, variant="pull")  # same bits, other form
"""
from __future__ import annotations

import ctypes
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

from . import _lib
from ._lib import BfsError, LOOPS, VARIANTS, VARIANT_NAMES, LevelRecord, RunOptions

PUSH_IMPL_NAMES = {v: k for k, v in _lib.PUSH_IMPLS.items()}

__all__ = ["Graph", "bfs", "bfs_static", "bfs_batch", "bfs_batch_vm", "batch_vm_workspace_size",
           "batch_workspace_size", "bfs_roots",
           "bfs_compare", "compare_workspace_size", "masked_spmspv",
           "spmspv_workspace_size", "BfsError", "VARIANTS", "LOOPS",
           "Workspace", "make_options"]


def _torch():
    import torch
    return torch


def _i32_host(a) -> np.ndarray:
    t = _torch()
    if isinstance(a, t.Tensor):
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.int32)


def _device_ready():
    """Bring up torch's device context before the library's first HIP call, so
    both share one runtime state (torch owns the memory and streams)."""
    t = _torch()
    if t.cuda.is_available():
        t.cuda.init()


def _stream_handle(stream):
    t = _torch()
    s = stream if stream is not None else t.cuda.current_stream()
    return ctypes.c_void_p(int(s.cuda_stream))


class Graph:
    """A graph resident on the GPU (library-owned copy of CSR and CSC)."""

    def __init__(self, handle: ctypes.c_void_p, n: int, nnz: int, directed: bool):
        self._h = handle
        self.n = n
        self.nnz = nnz
        self.directed = directed

    @classmethod
    def from_csr(cls, n: int, ptr, idx, in_ptr=None, in_idx=None, directed: bool = False,
                 validate_transpose: bool = False, ms_degree_order: Optional[bool] = None) -> "Graph":
        """ms_degree_order: keep (True) or never keep (False) the multi-source
        search's degree-ordered copy; None lets the library decide."""
        L = _lib.lib()
        _device_ready()
        ptr_h, idx_h = _i32_host(ptr), _i32_host(idx)
        flags = 0
        ip = ii = None
        if directed:
            flags |= _lib.BFS_DIRECTED
            if in_ptr is not None:
                ip, ii = _i32_host(in_ptr), _i32_host(in_idx)
        if validate_transpose:
            flags |= _lib.BFS_VALIDATE_TRANSPOSE
        if ms_degree_order is not None:
            flags |= _lib.BFS_MS_DEGREE_ORDER if ms_degree_order else _lib.BFS_MS_NO_DEGREE_ORDER
        vp = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        _lib.check(L.bfs_graph_create(int(n), vp(ptr_h), vp(idx_h), vp(ip), vp(ii), flags,
                                      None, ctypes.byref(h)))
        return cls(h, int(n), int(ptr_h[-1]), bool(directed))

    @classmethod
    def from_graphgen(cls, g, ms_degree_order: Optional[bool] = None) -> "Graph":
        if g.directed:
            return cls.from_csr(g.n, g.ptr, g.idx, g.in_ptr, g.in_idx, directed=True,
                                ms_degree_order=ms_degree_order)
        return cls.from_csr(g.n, g.ptr, g.idx, ms_degree_order=ms_degree_order)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("graph is closed")
        return self._h

    def device_bytes(self) -> int:
        b = ctypes.c_size_t()
        _lib.check(_lib.lib().bfs_graph_info(self.handle, None, None, None, ctypes.byref(b)))
        return int(b.value)

    def workspace_size(self, num_queries: int = 1, claim: bool = False) -> int:
        """Workspace bytes for bfs / bfs_batch on this graph; claim=True also
        covers a batch in the claim-word form (push_impl="claim")."""
        return int(_lib.lib().bfs_workspace_size(self.handle, int(num_queries), 1 if claim else 0))

    def roots_workspace_size(self, nroots: int) -> int:
        return int(_lib.lib().bfs_roots_workspace_size(self.handle, int(nroots)))

    def set_slice_words(self, max_words: int) -> None:
        """Re-cut the sliced push's LDS bitmap slices (at most `max_words` words each)."""
        _lib.check(_lib.lib().bfs_graph_set_slice_words(self.handle, int(max_words)))

    def close(self) -> None:
        if self._h is not None:
            _lib.lib().bfs_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Workspace:
    """A reusable device workspace (256-byte aligned view into a torch buffer)."""

    def __init__(self, nbytes: int, device="cuda"):
        t = _torch()
        self.buf = t.empty(nbytes + 256, dtype=t.uint8, device=device)
        base = self.buf.data_ptr()
        self.off = (-base) % 256
        self.nbytes = nbytes

    @property
    def ptr(self) -> ctypes.c_void_p:
        return ctypes.c_void_p(self.buf.data_ptr() + self.off)

    def fits(self, nbytes: int) -> bool:
        return nbytes <= self.nbytes


def make_options(variant="push", loop="host", levels_per_sync=0, grid_blocks=0,
                 heavy_degree=0, chunk_edges=0, selector=None, trace_capacity=0,
                 time_kernels=False, ms_pull_shift=0,
                 push_impl="auto", ms_ranges=0, count_atomics=0) -> Tuple[RunOptions, Optional[ctypes.Array]]:
    o = RunOptions()
    o.ms_ranges = int(ms_ranges)
    o.count_atomics = int(count_atomics)
    o.push_impl = _lib.PUSH_IMPLS[push_impl] if isinstance(push_impl, str) else int(push_impl)
    o.time_kernels = 1 if time_kernels else 0
    o.variant = VARIANTS[variant] if isinstance(variant, str) else int(variant)
    o.loop_mode = LOOPS[loop] if isinstance(loop, str) else int(loop)
    o.levels_per_sync = int(levels_per_sync)
    o.grid_blocks = int(grid_blocks)
    o.heavy_degree = int(heavy_degree)
    o.chunk_edges = int(chunk_edges)
    o.ms_pull_shift = int(ms_pull_shift)
    o.selector = ctypes.c_void_p(int(selector.data_ptr())) if selector is not None else None
    recs = None
    if trace_capacity:
        recs = (LevelRecord * trace_capacity)()
        o.trace = ctypes.cast(recs, ctypes.POINTER(LevelRecord))
        o.trace_capacity = trace_capacity
    return o, recs


def trace_dicts(o: RunOptions, recs) -> list:
    out = []
    for r in range(o.trace_count):
        x = recs[r]
        out.append(dict(level=x.level, variant=VARIANT_NAMES.get(x.variant, x.variant),
                        frontier=x.frontier, unvisited=x.unvisited,
                        frontier_edges=x.frontier_edges, unvisited_edges=x.unvisited_edges,
                        time_us=x.time_us))
    return out


def bfs(g: Graph, source: int, variant="push", loop="host", level=None, parent=None,
        workspace: Optional[Workspace] = None, stream=None, info: Optional[Dict] = None,
        trace: bool = False, **kw):
    """One search; returns (level, parent) as int32 cuda tensors (stream-ordered)."""
    t = _torch()
    if level is None:
        level = t.empty(g.n, dtype=t.int32, device="cuda")
    if parent is None:
        parent = t.empty(g.n, dtype=t.int32, device="cuda")
    need = g.workspace_size(1)
    if workspace is None or not workspace.fits(need):
        workspace = Workspace(need)
    o, recs = make_options(variant, loop, trace_capacity=(4096 if trace else 0), **kw)
    _lib.check(_lib.lib().bfs_run(g.handle, int(source),
                                  ctypes.c_void_p(level.data_ptr()), ctypes.c_void_p(parent.data_ptr()),
                                  ctypes.byref(o), workspace.ptr, workspace.nbytes,
                                  _stream_handle(stream)))
    if info is not None:
        info["levels"] = o.levels
        info["launches"] = o.launches
        info["kernel_us"] = o.kernel_us
        info["init_us"] = o.init_us
        info["push_used"] = PUSH_IMPL_NAMES.get(int(o.push_used), "list")
        if o.count_atomics:
            info["atomics"] = int(o.atomics)
        if trace:
            info["trace"] = trace_dicts(o, recs)
    return level, parent


def bfs_static(g: Graph, source: int, level=None, parent=None, levels_per_sync: int = 0, stream=None):
    """One plain-push search that allocates nothing on the library side (its
    state lives in the library's own per-GPU array; graphs of at most 2^22
    vertices).  Returns (level, parent); waits for the stream."""
    t = _torch()
    if level is None:
        level = t.empty(g.n, dtype=t.int32, device="cuda")
    if parent is None:
        parent = t.empty(g.n, dtype=t.int32, device="cuda")
    _lib.check(_lib.lib().bfs_run_static(g.handle, int(source), ctypes.c_void_p(level.data_ptr()),
                                         ctypes.c_void_p(parent.data_ptr()), int(levels_per_sync),
                                         _stream_handle(stream)))
    return level, parent


def bfs_roots(g: Graph, roots: Sequence[int], variant="push", loop="host", level=None,
              parent=None, workspace: Optional[Workspace] = None, stream=None,
              info: Optional[Dict] = None, **kw):
    """One search from several roots (e.g. one per block of a block-diagonal pack)."""
    t = _torch()
    roots_h = _i32_host(np.asarray(roots))
    if level is None:
        level = t.empty(g.n, dtype=t.int32, device="cuda")
    if parent is None:
        parent = t.empty(g.n, dtype=t.int32, device="cuda")
    need = g.roots_workspace_size(len(roots_h))
    if workspace is None or not workspace.fits(need):
        workspace = Workspace(need)
    o, _ = make_options(variant, loop, **kw)
    _lib.check(_lib.lib().bfs_run_roots(g.handle, len(roots_h), roots_h.ctypes.data_as(ctypes.c_void_p),
                                        ctypes.c_void_p(level.data_ptr()),
                                        ctypes.c_void_p(parent.data_ptr()), ctypes.byref(o),
                                        workspace.ptr, workspace.nbytes, _stream_handle(stream)))
    if info is not None:
        info["levels"] = o.levels
        info["push_used"] = PUSH_IMPL_NAMES.get(int(o.push_used), "list")
    return level, parent


def batch_workspace_size(graphs) -> int:
    """Workspace bytes bfs_batch needs for queries on these graphs (one per query)."""
    H = (ctypes.c_void_p * len(graphs))(*[gr.handle for gr in graphs])
    return int(_lib.lib().bfs_batch_workspace_size(len(graphs), H))


def _ms_trace(o: RunOptions, recs) -> list:
    """The multi-source trace: level k's direction and, where the host read it,
    the union frontier's size (0 elsewhere)."""
    return [dict(level=recs[r].level, direction=("push", "pull")[recs[r].variant],
                 frontier=recs[r].frontier) for r in range(o.trace_count)]


def bfs_batch(graphs, sources: Sequence[int], variant="push", loop="host", levels=None,
              parents=None, workspace: Optional[Workspace] = None, stream=None,
              info: Optional[dict] = None, trace: bool = False, **kw):
    """Many searches in one call: query q = (graphs[q], sources[q]).  `graphs` may be
    a single Graph (every query on it).  Returns lists of (level, parent) tensors.
    `info`, if given, receives "levels" and, with trace=True (one graph), "trace":
    each level's direction (see bfs_run_batch)."""
    t = _torch()
    nq = len(sources)
    if isinstance(graphs, Graph):
        graphs = [graphs] * nq
    if levels is None:
        levels = [t.empty(gr.n, dtype=t.int32, device="cuda") for gr in graphs]
    if parents is None:
        parents = [t.empty(gr.n, dtype=t.int32, device="cuda") for gr in graphs]
    H = (ctypes.c_void_p * nq)(*[gr.handle for gr in graphs])
    need = batch_workspace_size(graphs)
    if kw.get("push_impl") in ("claim", _lib.PUSH_IMPLS["claim"]) and all(gr is graphs[0] for gr in graphs):
        need = max(need, graphs[0].workspace_size(nq, claim=True))
    if workspace is None or not workspace.fits(need):
        workspace = Workspace(need)
    S = (ctypes.c_int32 * nq)(*[int(s) for s in sources])
    Lp = (ctypes.c_void_p * nq)(*[x.data_ptr() for x in levels])
    Pp = (ctypes.c_void_p * nq)(*[x.data_ptr() for x in parents])
    o, recs = make_options(variant, loop, trace_capacity=(max(gr.n for gr in graphs) + 2) if trace else 0, **kw)
    _lib.check(_lib.lib().bfs_run_batch(nq, H, S, Lp, Pp, ctypes.byref(o), workspace.ptr,
                                        workspace.nbytes, _stream_handle(stream)))
    if info is not None:
        info["levels"] = int(o.levels)
        if not all(gr is graphs[0] for gr in graphs):
            info["push_used"] = PUSH_IMPL_NAMES.get(int(o.push_used), "list")
        if trace:
            info["trace"] = _ms_trace(o, recs)
    return levels, parents


def compare_workspace_size(g: Graph) -> int:
    return int(_lib.lib().bfs_compare_workspace_size(g.handle))


def bfs_compare(g: Graph, source: int, method: str, level=None, parent=None,
                workspace: Optional[Workspace] = None, stream=None):
    """One of the Experiments section's comparison searches ("spmv", "spmspv",
    "spmmspv").  Returns (level, parent, ops, steps); waits for the stream."""
    t = _torch()
    if level is None:
        level = t.empty(g.n, dtype=t.int32, device="cuda")
    if parent is None:
        parent = t.empty(g.n, dtype=t.int32, device="cuda")
    need = compare_workspace_size(g)
    if workspace is None or not workspace.fits(need):
        workspace = Workspace(need)
    ops = ctypes.c_uint64(0)
    steps = ctypes.c_uint32(0)
    _lib.check(_lib.lib().bfs_run_compare(g.handle, int(source), _lib.COMPARE[method],
                                          ctypes.c_void_p(level.data_ptr()),
                                          ctypes.c_void_p(parent.data_ptr()), workspace.ptr,
                                          workspace.nbytes, ctypes.byref(ops), ctypes.byref(steps),
                                          _stream_handle(stream)))
    return level, parent, int(ops.value), int(steps.value)


def spmspv_workspace_size(g: Graph, max_nx: int) -> int:
    return int(_lib.lib().bfs_spmspv_workspace_size(g.handle, int(max_nx)))


def masked_spmspv(g: Graph, semiring: str, x_idx, x_val, row_mask=None, col_mask=None,
                  row_complement: bool = False, col_complement: bool = False,
                  workspace: Optional[Workspace] = None, y_idx=None, y_val=None, stream=None):
    """y = A^T[R, C] x over a semiring ("boolean", "arithmetic", "min_plus",
    "min_select").  x_idx: int32 cuda tensor; x_val: int64 cuda tensor holding
    the uint64 bit patterns; masks: int32 cuda tensors of ceil(n / 32) words or
    None.  The workspace must start zero-filled (a new one is).  Returns
    (y_idx, y_val) views of length ny (ascending indices; y_val as int64 bit
    patterns); waits for the stream."""
    t = _torch()
    nx = int(x_idx.numel())
    need = spmspv_workspace_size(g, nx)
    if workspace is None or not workspace.fits(need):
        workspace = Workspace(need)
        workspace.buf.zero_()
    if y_idx is None:
        y_idx = t.empty(g.n, dtype=t.int32, device="cuda")
    if y_val is None:
        y_val = t.empty(g.n, dtype=t.int64, device="cuda")
    flags = (1 if row_complement else 0) | (2 if col_complement else 0)
    vp = lambda a: None if a is None else ctypes.c_void_p(a.data_ptr())
    ny = ctypes.c_int32(0)
    _lib.check(_lib.lib().bfs_masked_spmspv(g.handle, _lib.SEMIRINGS[semiring], vp(x_idx), vp(x_val), nx,
                                            vp(row_mask), vp(col_mask), flags, vp(y_idx), vp(y_val),
                                            ctypes.byref(ny), workspace.ptr, workspace.nbytes,
                                            _stream_handle(stream)))
    return y_idx[:ny.value], y_val[:ny.value]


def batch_vm_workspace_size(g: Graph, num_sources: int) -> int:
    """Workspace bytes bfs_batch_vm needs for this many sources."""
    return int(_lib.lib().bfs_batch_vm_workspace_size(g.handle, int(num_sources)))


def bfs_batch_vm(g: Graph, sources: Sequence[int], variant="heuristic", level=None, parent=None,
                 workspace: Optional[Workspace] = None, stream=None, info: Optional[dict] = None,
                 trace: bool = False, **kw):
    """Many sources on one graph with vertex-major results: returns (level,
    parent) as int32 cuda tensors of shape [n, ld], ld = 64 * ceil(len / 64);
    column q holds source q's arrays (columns past the sources hold -1).
    `info`, if given, receives "levels" (the largest level over the sources
    plus one) and, with trace=True, "trace" (each level's direction)."""
    t = _torch()
    src = _i32_host(np.asarray(sources))
    ld = 64 * ((len(src) + 63) // 64)
    if level is None:
        level = t.empty((g.n, ld), dtype=t.int32, device="cuda")
    if parent is None:
        parent = t.empty((g.n, ld), dtype=t.int32, device="cuda")
    for name, a in (("level", level), ("parent", parent)):
        if (tuple(a.shape) != (g.n, ld) or a.dtype != t.int32 or not a.is_cuda
                or not a.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous int32 cuda tensor of shape "
                             f"({g.n}, {ld}), got {tuple(a.shape)} {a.dtype} on {a.device}")
    need = batch_vm_workspace_size(g, len(src))
    if workspace is None or not workspace.fits(need):
        workspace = Workspace(need)
    o, recs = make_options(variant, "host", trace_capacity=(g.n + 2) if trace else 0, **kw)
    _lib.check(_lib.lib().bfs_run_batch_vm(g.handle, len(src), src.ctypes.data_as(ctypes.c_void_p),
                                           ctypes.c_void_p(level.data_ptr()),
                                           ctypes.c_void_p(parent.data_ptr()), ctypes.byref(o),
                                           workspace.ptr, workspace.nbytes, _stream_handle(stream)))
    if info is not None:
        info["levels"] = int(o.levels)
        if trace:
            info["trace"] = _ms_trace(o, recs)
    return level, parent
