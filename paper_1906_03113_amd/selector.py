"""The per-level variant selector: training data, training, evaluation.

Push, pull and push-bitmap are three evaluations of the same masked product;
which is fastest depends on the level (a small frontier favours push, a
frontier holding much of the remaining edges favours pull).  The selector is a
12 -> 32 -> 32 -> 3 fp32 network that predicts each form's log device time from
the level's statistics; the level kernel evaluates it on the device and runs
the argmin.  It can never change a result: every form returns the same bits,
and push is the fallback for missing or non-finite weights.

Training data come from the method itself: bfs_profile_levels times every
level under all three forms from the same saved state.  Training runs on the
GPU through the library's own forward / backward / Adam kernels.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np

from . import _lib

N_IN, N_H, N_OUT = 12, 32, 3
VARIANT_ORDER = ("push", "pull", "bitmap")
HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "selector_weights.json")


def _torch():
    import torch
    return torch


def param_count() -> int:
    return int(_lib.lib().bfs_selector_param_count())


def n_trainable() -> int:
    return param_count() - 2 * N_IN


def features(frontier, frontier_edges, unvisited, unvisited_edges, level, n, nnz) -> np.ndarray:
    """The twelve level features (same definitions as the device code), float64 [rows, 12]."""
    f = np.asarray(frontier, np.float64)
    sf = np.asarray(frontier_edges, np.float64)
    u = np.asarray(unvisited, np.float64)
    su = np.asarray(unvisited_edges, np.float64)
    k = np.asarray(level, np.float64)
    n = np.full(f.shape, float(n)) if np.ndim(n) == 0 else np.asarray(n, np.float64)
    nnz = np.full(f.shape, float(nnz)) if np.ndim(nnz) == 0 else np.asarray(nnz, np.float64)
    return np.stack([np.log1p(f), np.log1p(sf), np.log1p(u), np.log1p(su), np.log1p(k), nnz / n,
                     np.log((f + 1) / n), np.log((sf + 1) / (nnz + 1)), np.log((u + 1) / n),
                     np.log((su + 1) / (nnz + 1)), np.log((sf + 1) / (su + 1)),
                     np.log((f + 1) / (u + 1))], axis=-1)


# ---- training data ------------------------------------------------------------------

def profile(G, source: int, reps: int = 2) -> List[Dict]:
    """Per-level times of all three forms for one search (see bfs_profile_levels)."""
    torch = _torch()
    from . import Workspace
    L = _lib.lib()
    level = torch.empty(G.n, dtype=torch.int32, device="cuda")
    parent = torch.empty(G.n, dtype=torch.int32, device="cuda")
    ws = Workspace(G.workspace_size(1))
    snap = Workspace(int(L.bfs_profile_snapshot_size(G.handle)))
    cap = 3 * 200000
    recs = (_lib.LevelRecord * cap)()
    cnt = ctypes.c_uint32(0)
    s = torch.cuda.current_stream()
    _lib.check(L.bfs_profile_levels(G.handle, int(source), ctypes.c_void_p(level.data_ptr()),
                                    ctypes.c_void_p(parent.data_ptr()), ws.ptr, ws.nbytes,
                                    snap.ptr, snap.nbytes, int(reps), recs, cap, ctypes.byref(cnt),
                                    ctypes.c_void_p(int(s.cuda_stream))))
    out: Dict[int, Dict] = {}
    for i in range(cnt.value):
        r = recs[i]
        d = out.setdefault(r.level, dict(level=r.level, frontier=r.frontier, unvisited=r.unvisited,
                                         frontier_edges=r.frontier_edges,
                                         unvisited_edges=r.unvisited_edges,
                                         times=[math.nan] * 3))
        d["times"][r.variant] = r.time_us
    return [out[k] for k in sorted(out)]


def dataset(levels: Sequence[Dict], n: int, nnz: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(raw features [rows,12], log-time targets [rows,3], mask [rows,3]) from profile records."""
    if not levels:
        return np.zeros((0, N_IN)), np.zeros((0, N_OUT)), np.zeros((0, N_OUT))
    X = features([d["frontier"] for d in levels], [d["frontier_edges"] for d in levels],
                 [d["unvisited"] for d in levels], [d["unvisited_edges"] for d in levels],
                 [d["level"] for d in levels], n, nnz)
    T = np.array([d["times"] for d in levels], dtype=np.float64)
    M = np.isfinite(T) & (T > 0)
    T = np.where(M, np.log(np.where(M, T, 1.0)), 0.0)
    return X, T, M.astype(np.float64)


# ---- training on the GPU --------------------------------------------------------------

def init_weights(X: np.ndarray, seed: int = 0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, math.sqrt(2.0 / N_IN), (N_H, N_IN)), np.zeros(N_H),
             rng.normal(0, math.sqrt(2.0 / N_H), (N_H, N_H)), np.zeros(N_H),
             rng.normal(0, math.sqrt(1.0 / N_H), (N_OUT, N_H)), np.zeros(N_OUT)]
    mean = X.mean(0) if len(X) else np.zeros(N_IN)
    std = X.std(0) if len(X) else np.ones(N_IN)
    istd = 1.0 / np.where(std > 1e-6, std, 1.0)
    blob = np.concatenate([p.ravel() for p in parts] + [mean, istd]).astype(np.float32)
    assert blob.size == param_count()
    return blob


class Trainer:
    """Device-resident weights, Adam state and data; one call = one full-batch step."""

    def __init__(self, blob: np.ndarray, X: np.ndarray, T: np.ndarray, M: np.ndarray):
        torch = _torch()
        self.w = torch.tensor(np.asarray(blob, np.float32), device="cuda")
        P = param_count()
        self.grad = torch.zeros(P, dtype=torch.float32, device="cuda")
        self.m = torch.zeros(P, dtype=torch.float32, device="cuda")
        self.v = torch.zeros(P, dtype=torch.float32, device="cuda")
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.X = torch.tensor(np.asarray(X, np.float32), device="cuda").contiguous()
        self.T = torch.tensor(np.asarray(T, np.float32), device="cuda").contiguous()
        self.M = torch.tensor(np.asarray(M, np.float32), device="cuda").contiguous()
        self.inv = 1.0 / max(1.0, float(np.asarray(M).sum()))
        self.t = 0

    def _ptr(self, x):
        return ctypes.c_void_p(x.data_ptr())

    def _stream(self):
        return ctypes.c_void_p(int(_torch().cuda.current_stream().cuda_stream))

    def gradient(self) -> float:
        """Accumulate the gradient of the current weights into self.grad; return the loss."""
        self.loss.zero_()
        _lib.check(_lib.lib().bfs_selector_grad(self._ptr(self.w), self._ptr(self.X), self._ptr(self.T),
                                                self._ptr(self.M), int(self.X.shape[0]),
                                                ctypes.c_float(self.inv), self._ptr(self.grad),
                                                self._ptr(self.loss), self._stream()))
        return float(self.loss.item())

    def step(self, lr: float) -> float:
        loss = self.gradient()
        self.t += 1
        _lib.check(_lib.lib().bfs_selector_adam(self._ptr(self.w), self._ptr(self.grad), self._ptr(self.m),
                                                self._ptr(self.v), self.t, ctypes.c_float(lr),
                                                self._stream()))
        return loss

    def weights(self) -> np.ndarray:
        return self.w.detach().cpu().numpy().copy()


def level_weights(T: np.ndarray, M: np.ndarray, lo: float = 0.25, hi: float = 4.0) -> np.ndarray:
    """Per-row loss weights: sqrt(best time / median best time), clipped to
    [lo, hi], so that the levels that cost the most device time (what the
    regret sums) count more than the many cheap levels of deep searches."""
    t = np.where(M > 0, np.exp(T), np.inf)
    best = t.min(1)
    ok = np.isfinite(best)
    if not ok.any():
        return np.ones(len(T))
    w = np.sqrt(np.where(ok, best, 0.0) / np.median(best[ok]))
    return np.where(ok, np.clip(w, lo, hi), 0.0)


def train(X, T, M, steps: int = 3000, lr: float = 3e-3, seed: int = 0, log=None,
          weighted: bool = True) -> np.ndarray:
    """Full-batch Adam on the masked squared error of the log-times; rows
    weighted by level_weights unless weighted=False."""
    Mw = np.asarray(M, np.float64) * (level_weights(T, M)[:, None] if weighted else 1.0)
    tr = Trainer(init_weights(np.asarray(X), seed), X, T, Mw)
    for i in range(steps):
        loss = tr.step(lr if i < steps * 2 // 3 else lr * 0.2)
        if log and (i % max(1, steps // 10) == 0 or i == steps - 1):
            log(f"[selector] step {i} loss {loss:.5f}")
    return tr.weights()


def predict(blob: np.ndarray, X: np.ndarray) -> np.ndarray:
    torch = _torch()
    w = torch.tensor(np.asarray(blob, np.float32), device="cuda")
    x = torch.tensor(np.asarray(X, np.float32), device="cuda").contiguous()
    y = torch.empty((x.shape[0], N_OUT), dtype=torch.float32, device="cuda")
    _lib.check(_lib.lib().bfs_selector_forward(ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                               ctypes.c_void_p(y.data_ptr()), int(x.shape[0]),
                                               ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))))
    return y.cpu().numpy()


def regret(choice: np.ndarray, T: np.ndarray, M: np.ndarray) -> Dict[str, float]:
    """Sum over levels of (time of the chosen form - best time) / sum of best times;
    also the push-only total relative to the best."""
    t = np.where(M > 0, np.exp(T), np.inf)
    best = t.min(1)
    chosen = t[np.arange(len(t)), choice]
    ok = np.isfinite(best)
    return dict(regret=float((chosen[ok] - best[ok]).sum() / best[ok].sum()),
                push_regret=float((t[ok, 0] - best[ok]).sum() / best[ok].sum()),
                chosen_us=float(chosen[ok].sum()), best_us=float(best[ok].sum()),
                push_us=float(t[ok, 0].sum()))


def choose(blob: np.ndarray, X: np.ndarray) -> np.ndarray:
    y = predict(blob, X)
    return np.argmin(y, axis=1)


def save_weights(path: str, blob: np.ndarray, meta: Dict = None) -> None:
    with open(path, "w") as f:
        json.dump({"format": "bfs-selector-mlp-12-32-32-3", "weights": [float(v) for v in blob],
                   "meta": meta or {}}, f)


def load_weights(path: str = DEFAULT_WEIGHTS):
    """Weights as a cuda float32 tensor, ready for BFS_VARIANT_LEARNED."""
    torch = _torch()
    with open(path) as f:
        d = json.load(f)
    w = np.asarray(d["weights"], np.float32)
    if w.size != param_count():
        raise ValueError(f"{path}: {w.size} weights, expected {param_count()}")
    return torch.tensor(w, device="cuda")


# ---- the multi-source direction ------------------------------------------------------------
#
# bfs_run_batch / bfs_run_batch_vm under BFS_VARIANT_LEARNED ask the same network
# (its first two outputs: push, pull) before every level, over features of the
# union frontier F (vertices in some source's frontier).  Training data come from
# bfs_ms_profile_levels, which times both directions of every level from the
# same saved state.

MS_WEIGHTS = os.path.join(HERE, "selector_ms_weights.json")
MS_DIRECTIONS = ("push", "pull")


def ms_features(frontier, frontier_edges, listed, unsettled, sources, level, n, nnz) -> np.ndarray:
    """The twelve multi-source level features (the device's definitions), float64
    [rows, 12]: f = |F_k|, d = out-degree sum over F_k, c = summed union-frontier
    sizes of levels 0..k, u = (vertex, source) pairs not reached through level k,
    q = number of sources, k, n, nnz."""
    f = np.asarray(frontier, np.float64)
    d = np.asarray(frontier_edges, np.float64)
    c = np.asarray(listed, np.float64)
    u = np.asarray(unsettled, np.float64)
    q = np.asarray(sources, np.float64)
    k = np.asarray(level, np.float64)
    n = np.full(f.shape, float(n)) if np.ndim(n) == 0 else np.asarray(n, np.float64)
    nnz = np.full(f.shape, float(nnz)) if np.ndim(nnz) == 0 else np.asarray(nnz, np.float64)
    return np.stack([np.log1p(f), np.log1p(d), np.log1p(c), np.log1p(q), np.log1p(k), nnz / n,
                     np.log((f + 1) / n), np.log((d + 1) / (nnz + 1)), np.log((u + 1) / (n * q)),
                     np.log((d + 1) / (f + 1)), np.log((f + 1) * q / n),
                     np.log((d + 1) / (nnz - d + 1))], axis=-1)


def ms_profile(G, sources: Sequence[int], reps: int = 2, out=None) -> List[Dict]:
    """Per-level device times of both directions for one multi-source call (see
    bfs_ms_profile_levels).  out: optional (level, parent) int32 cuda tensors of
    shape [n, 64 * ceil(len / 64)] that receive the results."""
    torch = _torch()
    from . import Workspace, batch_vm_workspace_size
    L = _lib.lib()
    src = np.ascontiguousarray(np.asarray(sources, np.int32))
    nq = len(src)
    ld = 64 * ((nq + 63) // 64)
    if out is None:
        out = (torch.empty((G.n, ld), dtype=torch.int32, device="cuda"),
               torch.empty((G.n, ld), dtype=torch.int32, device="cuda"))
    level, parent = out
    ws = Workspace(batch_vm_workspace_size(G, nq))
    snap = Workspace(int(L.bfs_ms_profile_snapshot_size(G.handle, nq)))
    cap = 2 * 100000
    recs = (_lib.LevelRecord * cap)()
    cnt = ctypes.c_uint32(0)
    s = torch.cuda.current_stream()
    _lib.check(L.bfs_ms_profile_levels(G.handle, nq, src.ctypes.data_as(ctypes.c_void_p),
                                       ctypes.c_void_p(level.data_ptr()), ctypes.c_void_p(parent.data_ptr()),
                                       ws.ptr, ws.nbytes, snap.ptr, snap.nbytes, int(reps), recs, cap,
                                       ctypes.byref(cnt), ctypes.c_void_p(int(s.cuda_stream))))
    torch.cuda.synchronize()
    del ws, snap
    res: Dict[int, Dict] = {}
    for i in range(cnt.value):
        r = recs[i]
        d = res.setdefault(r.level, dict(level=r.level, frontier=r.frontier, frontier_edges=r.frontier_edges,
                                         listed=r.unvisited, unsettled=r.unvisited_edges, sources=nq,
                                         times=[math.nan] * N_OUT))
        d["times"][r.variant] = r.time_us
    return [res[k] for k in sorted(res)]


def ms_dataset(levels: Sequence[Dict], n: int, nnz: int) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(features [rows,12], log-time targets [rows,3], mask [rows,3]); the third
    output is never a target (the multi-source search has two directions)."""
    if not levels:
        return np.zeros((0, N_IN)), np.zeros((0, N_OUT)), np.zeros((0, N_OUT))
    X = ms_features([d["frontier"] for d in levels], [d["frontier_edges"] for d in levels],
                    [d["listed"] for d in levels], [d["unsettled"] for d in levels],
                    [d["sources"] for d in levels], [d["level"] for d in levels], n, nnz)
    T = np.array([d["times"] for d in levels], dtype=np.float64)
    T[:, 2] = np.nan
    M = np.isfinite(T) & (T > 0)
    T = np.where(M, np.log(np.where(M, T, 1.0)), 0.0)
    return X, T, M.astype(np.float64)


def ms_choose(blob: np.ndarray, X: np.ndarray) -> np.ndarray:
    """The device's decision: argmin over the push and pull outputs."""
    y = predict(blob, X)[:, :2]
    return np.argmin(y, axis=1)


def ms_heuristic_choice(X: np.ndarray, shift: int = 5) -> np.ndarray:
    """What BFS_VARIANT_HEURISTIC picks from the same rows: pull once the union
    frontier holds more than n >> shift vertices (read back from features 0 and 6)."""
    f = np.expm1(X[:, 0])
    n = (f + 1) / np.exp(X[:, 6])
    return ((np.round(f) * 2.0 ** shift) > np.round(n)).astype(np.int64)


def ms_training_sets(include_large: bool = True):
    """(train, held-out) lists of (name, graph builder, source batches); a batch
    is (count, seed) of seeded picks.  Held out: R-MAT scales and batch sizes
    never trained on."""
    import graphgen
    train = [("er16k", lambda: graphgen.workload("er16k"), [(64, 1), (256, 2)]),
             ("grid512", lambda: graphgen.grid(512, 0.9, 3), [(16, 3), (64, 4)]),
             ("rmatd16", lambda: graphgen.rmat(16, 16, 1, directed=True), [(64, 5), (256, 6)])]
    if include_large:
        train += [("rmat22", lambda: graphgen.workload("rmat22"), [(64, 7), (16, 8)]),
                  ("rmat20d", lambda: graphgen.workload("rmat20d"), [(256, 9), (64, 10)]),
                  ("rmat19", lambda: graphgen.rmat(19, 16, 7), [(128, 11)]),
                  ("grid1024", lambda: graphgen.grid(1024, 0.9, 5), [(16, 12)])]
    held = [(f"rmat{sc}", (lambda sc=sc: graphgen.rmat(sc, 16, 2000 + sc)), [(64, 20 + sc), (192, 40 + sc)])
            for sc in ((16, 18) if not include_large else (16, 17, 18, 21))]
    return train, held


def ms_collect(entries, reps: int = 2, log=None):
    import graphgen
    from . import Graph
    Xs, Ts, Ms = [], [], []
    for name, build, batches in entries:
        g = build() if callable(build) else build
        G = Graph.from_graphgen(g)
        for count, seed in batches:
            src = graphgen.pick_sources(g, count, seed)
            lv = ms_profile(G, src, reps)
            X, T, M = ms_dataset(lv, g.n, g.nnz)
            Xs.append(X); Ts.append(T); Ms.append(M)
            if log:
                log(f"[selector-ms] {name} {count} sources: {len(lv)} levels")
        G.close()
        del g
    return np.concatenate(Xs), np.concatenate(Ts), np.concatenate(Ms)


def ms_main(args, log):
    train_e, held_e = ms_training_sets(include_large=not args.small)
    X, T, M = ms_collect(train_e, log=log)
    Xh, Th, Mh = ms_collect(held_e, log=log)
    log(f"[selector-ms] training rows {len(X)}, held-out rows {len(Xh)}")
    w = train(X, T, M, steps=args.steps, log=log)
    res = {}
    for tag, (x, t, m) in (("train", (X, T, M)), ("held_out", (Xh, Th, Mh))):
        res[tag] = regret(ms_choose(w, x), t, m)
        res[tag]["heuristic_regret"] = regret(ms_heuristic_choice(x), t, m)["regret"]
        log(f"[selector-ms] {tag}: {res[tag]}")
    meta = dict(res, train_rows=int(len(X)), held_rows=int(len(Xh)),
                outputs="push, pull (the third output is unused)")
    save_weights(args.ms_out, w, meta)
    print(json.dumps(res))


# ---- the training recipe ----------------------------------------------------------------

def training_graphs(include_large: bool = True):
    """(name, graph builder, sources) for training, and the held-out groups: R-MAT
    graphs of scales never trained on, and a 4096^2 grid (16.8 M vertices, a
    depth and size beyond every training graph).  Graphs are built one at a
    time when collected."""
    import graphgen
    train = [("er16k", lambda: graphgen.workload("er16k"), [0, 1, 2, 3]),
             ("grid512", lambda: graphgen.grid(512, 0.9, 3), None),
             ("rmatd16", lambda: graphgen.rmat(16, 16, 1, directed=True), None)]
    if include_large:
        train += [("rmat22", lambda: graphgen.workload("rmat22"), None),
                  ("rmat20d", lambda: graphgen.workload("rmat20d"), None),
                  ("rmat19", lambda: graphgen.rmat(19, 16, 7), None),
                  ("rmat21", lambda: graphgen.rmat(21, 16, 8), None),
                  ("grid1024", lambda: graphgen.grid(1024, 0.9, 5), [None, None]),
                  ("grid2048", lambda: graphgen.grid(2048, 0.9, 6), [None])]
    held = {"rmat": [(f"rmat{s}", (lambda s=s: graphgen.rmat(s, 16, 1000 + s)), None)
                     for s in (16, 17, 18, 19, 20, 21)]}
    if include_large:
        held["grid4096"] = [("grid4096", lambda: graphgen.grid(4096, 0.9, 9), [None])]
    return train, held


def _spread(levels: List[Dict], cap: int) -> List[Dict]:
    """At most `cap` of a search's levels, evenly spaced (first and last kept), so
    that a search thousands of levels deep does not outweigh the shallow ones."""
    if cap <= 0 or len(levels) <= cap:
        return levels
    keep = np.unique(np.linspace(0, len(levels) - 1, cap).round().astype(np.int64))
    return [levels[i] for i in keep]


def collect(entries, per_graph: int = 3, reps: int = 2, log=None, cap: int = 0):
    """Profile every search of `entries`; a source list entry of None means a
    seeded pick.  `cap` > 0 keeps at most that many levels of each search."""
    import graphgen
    from . import Graph
    Xs, Ts, Ms = [], [], []
    for name, build, srcs in entries:
        g = build() if callable(build) else build
        G = Graph.from_graphgen(g)
        if srcs is None:
            srcs = graphgen.pick_sources(g, per_graph, 77)
        elif any(x is None for x in srcs):
            srcs = graphgen.pick_sources(g, len(srcs), 78)
        for s in srcs:
            lv = profile(G, int(s), reps)
            X, T, M = dataset(_spread(lv, cap), g.n, g.nnz)
            Xs.append(X); Ts.append(T); Ms.append(M)
            if log:
                log(f"[selector] {name} s={s}: {len(lv)} levels, {len(X)} rows")
        G.close()
        del g
    return np.concatenate(Xs), np.concatenate(Ts), np.concatenate(Ms)


def main(argv=None):
    import argparse
    import sys
    ap = argparse.ArgumentParser(description="collect per-level timings, train the selector, evaluate regret")
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--small", action="store_true", help="skip the large training graphs")
    ap.add_argument("--cap", type=int, default=300, help="levels kept per training search")
    ap.add_argument("--eval", action="store_true",
                    help="only measure the held-out regret of the weights in --out (no training)")
    ap.add_argument("--multi-source", action="store_true",
                    help="train the multi-source direction (push / pull) instead")
    ap.add_argument("--ms-out", default=MS_WEIGHTS)
    args = ap.parse_args(argv)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    torch = _torch()
    torch.cuda.init()                 # the device context first, before any CPU-heavy setup
    if args.multi_source:
        ms_main(args, log)
        return
    train_g, held_g = training_graphs(include_large=not args.small)
    if args.eval:
        with open(args.out) as f:
            w = np.asarray(json.load(f)["weights"], np.float32)
        res = {}
        for k, v in held_g.items():
            Xh, Th, Mh = collect(v, per_graph=2, log=log)
            res[k] = regret(choose(w, Xh), Th, Mh)
            log(f"[selector] held-out {k}: {res[k]}")
        print(json.dumps({"held_out": res}))
        return
    X, T, M = collect(train_g, log=log, cap=args.cap)
    held = {k: collect(v, per_graph=2, log=log) for k, v in held_g.items()}
    log(f"[selector] training rows {len(X)}, held-out rows "
        f"{ {k: len(v[0]) for k, v in held.items()} }")
    w = train(X, T, M, steps=args.steps, log=log)
    res_train = regret(choose(w, X), T, M)
    res_held = {k: regret(choose(w, Xh), Th, Mh) for k, (Xh, Th, Mh) in held.items()}
    log(f"[selector] train {res_train}")
    for k, r in res_held.items():
        log(f"[selector] held-out {k}: {r}")
    meta = {"train": res_train, "held_out": res_held.get("rmat"),
            "train_rows": int(len(X)), "held_rows": {k: int(len(v[0])) for k, v in held.items()},
            "features": "log1p(k) level feature"}
    for k, r in res_held.items():
        if k != "rmat":
            meta[f"held_out_{k}"] = r
    save_weights(args.out, w, meta)
    print(json.dumps({"train": res_train, "held_out": res_held}))


if __name__ == "__main__":
    main()
