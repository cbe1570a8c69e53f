"""Measured search over the launch parameters of a search, cached per graph shape.

The parameters that change speed but never results: the level-loop mode
(host loop, captured graph, persistent kernel), levels per host
synchronisation, workgroups per level launch, the out-degree from which a
column is split into chunks, and the chunk size.  The best set depends on the
graph's shape - a 7,000-level grid wants a small grid of workgroups and no
host round trips, a scale-22 R-MAT wants the whole chip - so it is measured on
the graph itself (a few searches per candidate) and cached under a shape key:

    (device name, directed, round(log2 n), round(log2 average degree), diameter
     class from one probe search: levels <= 64 "low", <= 1024 "mid", else "high")

The cache is a JSON file; `lookup` returns the cached parameters (or the
defaults) for any graph of the same shape.  `tune_batch_width` does the same
for the number of sources per multi-source call (`lookup_batch_width`), and
`tune_pull_shift` for the frontier size from which a multi-source level runs
in the pull form (`lookup_pull_shift`).
"""
from __future__ import annotations

import itertools
import json
import math
import os
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "bfs_autotune.json")

SPACE = {
    "loop": ["host", "graph", "persistent"],
    "levels_per_sync": [8, 64],
    "grid_blocks": [64, 256, 1024, 2048],
    "heavy_degree": [256, 512, 2048],
    "chunk_edges": [512, 1024, 4096],
}


def _torch():
    import torch
    return torch


def shape_key(G, levels: int) -> str:
    torch = _torch()
    name = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"
    avg = max(1.0, G.nnz / max(1, G.n))
    dclass = "low" if levels <= 64 else ("mid" if levels <= 1024 else "high")
    return f"{name}|{'d' if G.directed else 'u'}|n2^{round(math.log2(max(2, G.n)))}|" \
           f"deg2^{round(math.log2(avg))}|{dclass}"


def candidates(levels: int, budget: int, seed: int = 0) -> List[Dict]:
    """All combinations, pruned by what matters for the diameter class, then a
    seeded sample of at most `budget` of them (the defaults always included)."""
    combos = []
    for loop, lps, grid, heavy, chunk in itertools.product(*SPACE.values()):
        if loop == "persistent" and lps != 8:
            continue                          # levels_per_sync is unused there
        if levels > 64 and (heavy, chunk) != (512, 1024):
            continue                          # long thin searches: no long columns to split
        if levels <= 64 and loop == "host" and lps == 64:
            continue
        combos.append(dict(loop=loop, levels_per_sync=lps, grid_blocks=grid,
                           heavy_degree=heavy, chunk_edges=chunk))
    default = dict(loop="graph", levels_per_sync=8 if levels <= 64 else 64, grid_blocks=0,
                   heavy_degree=0, chunk_edges=0)
    rng = np.random.default_rng(seed)
    if len(combos) > budget - 1:
        pick = rng.choice(len(combos), size=budget - 1, replace=False)
        combos = [combos[i] for i in sorted(pick)]
    return [default] + combos


def time_config(G, sources: Sequence[int], kw: Dict, reps: int = 2, variant_kw: Optional[Dict] = None) -> float:
    """Best-of-reps wall time (s) for searching from every source once."""
    torch = _torch()
    import paper_1906_03113_amd as P
    ws = P.Workspace(G.workspace_size(1))
    lv = torch.empty(G.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(G.n, dtype=torch.int32, device="cuda")
    vkw = dict(variant_kw or {"variant": "heuristic"})
    best = math.inf
    for r in range(reps + 1):                 # the first pass warms up (graph capture etc.)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in sources:
            P.bfs(G, int(s), level=lv, parent=pa, workspace=ws, **vkw, **kw)
        torch.cuda.synchronize()
        if r:
            best = min(best, time.perf_counter() - t0)
    return best


def tune(G, sources: Sequence[int], budget: int = 24, cache: str = DEFAULT_CACHE,
         variant_kw: Optional[Dict] = None, log=None) -> Dict:
    """Measure up to `budget` candidates on G; cache and return the fastest."""
    import paper_1906_03113_amd as P
    info = {}
    P.bfs(G, int(sources[0]), info=info, **(variant_kw or {"variant": "heuristic"}))
    levels = int(info["levels"])
    key = shape_key(G, levels)
    results = []
    for kw in candidates(levels, budget):
        t = time_config(G, sources, kw, variant_kw=variant_kw)
        results.append((t, kw))
        if log:
            log(f"[autotune] {key} {kw} -> {t * 1e3:.2f} ms")
    results.sort(key=lambda x: x[0])
    best_t, best = results[0]
    default_t = next(t for t, kw in results if kw["grid_blocks"] == 0)
    entry = {"params": best, "time_s": best_t, "default_time_s": default_t, "levels": levels,
             "candidates": len(results)}
    store(cache, key, entry)
    return dict(key=key, **entry)


def store(cache: str, key: str, entry: Dict) -> None:
    d = {}
    if os.path.exists(cache):
        try:
            with open(cache) as f:
                d = json.load(f)
        except (OSError, ValueError):
            d = {}
    d[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
    tmp = cache + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, cache)


BATCH_WIDTHS = (64, 128, 256)


def time_batches(G, sources: Sequence[int], width: int, reps: int = 2) -> float:
    """Best-of-reps wall time (s) for searching from every source with
    bfs_run_batch calls of `width` sources each (outputs and one workspace
    allocated first; the last call takes the remainder)."""
    torch = _torch()
    import paper_1906_03113_amd as P
    src = [int(s) for s in sources]
    lv = [torch.empty(G.n, dtype=torch.int32, device="cuda") for _ in src]
    pa = [torch.empty(G.n, dtype=torch.int32, device="cuda") for _ in src]
    ws = P.Workspace(G.workspace_size(min(width, len(src))))
    best = math.inf
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(0, len(src), width):
            P.bfs_batch(G, src[b:b + width], levels=lv[b:b + width], parents=pa[b:b + width],
                        workspace=ws, variant="heuristic")
        torch.cuda.synchronize()
        if r:
            best = min(best, time.perf_counter() - t0)
    del lv, pa, ws
    torch.cuda.empty_cache()
    return best


def tune_batch_width(G, sources: Sequence[int], widths: Sequence[int] = BATCH_WIDTHS,
                     cache: str = DEFAULT_CACHE, log=None, timer=None) -> Dict:
    """Sources per multi-source call (64 per mask word, so multiples of 64):
    time the same set of sources in calls of each width, cache the fastest
    under the graph's shape key."""
    import paper_1906_03113_amd as P
    info = {}
    P.bfs(G, int(sources[0]), info=info, variant="heuristic")
    key = shape_key(G, int(info["levels"])) + "|batch"
    timer = timer or time_batches
    times = {}
    for w in widths:
        if w > len(sources) or w % 64:
            continue
        times[w] = timer(G, sources, w)
        if log:
            log(f"[autotune] {key} width {w} -> {times[w] * 1e3:.2f} ms for {len(sources)} sources")
    best = min(times, key=times.get)
    entry = {"width": best, "time_s": times[best], "times_s": {str(w): t for w, t in times.items()},
             "sources": len(sources)}
    store(cache, key, entry)
    return dict(key=key, **entry)


def lookup_batch_width(G, levels: int, cache: str = DEFAULT_CACHE, default: int = 64) -> int:
    """Cached sources per multi-source call for G's shape, else `default`."""
    if not os.path.exists(cache):
        return default
    try:
        with open(cache) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return default
    e = d.get(shape_key(G, levels) + "|batch")
    return int(e["width"]) if e else default


PULL_SHIFTS = (5, 7, 9, 11, 13)


def time_pull_shift(G, sources: Sequence[int], shift: int, reps: int = 2, out=None) -> float:
    """Best-of-reps wall time (s) of one multi-source call over `sources`
    (heuristic direction, the pull threshold n >> shift); `out` = (level,
    parent, workspace) to reuse, else allocated here."""
    torch = _torch()
    import paper_1906_03113_amd as P
    src = [int(s) for s in sources]
    if out is None:
        ld = 64 * ((len(src) + 63) // 64)
        out = (torch.empty((G.n, ld), dtype=torch.int32, device="cuda"),
               torch.empty((G.n, ld), dtype=torch.int32, device="cuda"),
               P.Workspace(P.batch_vm_workspace_size(G, len(src))))
    lv, pa, ws = out
    best = math.inf
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.bfs_batch_vm(G, src, level=lv, parent=pa, workspace=ws, ms_pull_shift=shift)
        torch.cuda.synchronize()
        if r:
            best = min(best, time.perf_counter() - t0)
    return best


def tune_pull_shift(G, sources: Sequence[int], shifts: Sequence[int] = PULL_SHIFTS,
                    cache: Optional[str] = DEFAULT_CACHE, log=None, timer=None) -> Dict:
    """The multi-source direction threshold (pull once the union frontier
    holds more than n >> shift vertices): time one call over the same sources
    at each shift, cache the fastest under the graph's shape key (cache=None:
    measure only)."""
    import paper_1906_03113_amd as P
    info = {}
    P.bfs(G, int(sources[0]), info=info, variant="heuristic")
    key = shape_key(G, int(info["levels"])) + "|ms_pull"
    timer = timer or time_pull_shift
    times = {}
    for sh in shifts:
        if not 1 <= int(sh) <= 31:
            continue
        times[int(sh)] = timer(G, sources, int(sh))
        if log:
            log(f"[autotune] {key} pull shift {sh} -> {times[int(sh)] * 1e3:.3f} ms")
    best = min(times, key=times.get)
    entry = {"shift": best, "time_s": times[best], "times_s": {str(k): t for k, t in times.items()},
             "sources": len(sources)}
    if cache:
        store(cache, key, entry)
    return dict(key=key, **entry)


def lookup_pull_shift(G, levels: int, cache: str = DEFAULT_CACHE, default: int = 0) -> int:
    """Cached multi-source pull shift for G's shape, else `default` (0 = the
    library's n / 32)."""
    if not os.path.exists(cache):
        return default
    try:
        with open(cache) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return default
    e = d.get(shape_key(G, levels) + "|ms_pull")
    return int(e["shift"]) if e else default


def lookup(G, levels: int, cache: str = DEFAULT_CACHE) -> Dict:
    """Cached parameters for G's shape, or {} (the library's defaults)."""
    if not os.path.exists(cache):
        return {}
    try:
        with open(cache) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return {}
    e = d.get(shape_key(G, levels))
    return dict(e["params"]) if e else {}


def main(argv=None):
    import argparse
    import sys
    import graphgen
    ap = argparse.ArgumentParser(description="tune launch parameters for the standard workloads")
    ap.add_argument("--workloads", default="er16k,rmat22,grid4096,rmat20d")
    ap.add_argument("--budget", type=int, default=16)
    ap.add_argument("--sources", type=int, default=2)
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    ap.add_argument("--batch", action="store_true",
                    help="tune the sources per multi-source call instead (256 sources per workload)")
    ap.add_argument("--pull-shift", action="store_true",
                    help="tune the multi-source pull threshold instead (64 sources per workload)")
    a = ap.parse_args(argv)
    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    torch = _torch()
    torch.cuda.init()
    import paper_1906_03113_amd as P
    from . import selector as S
    vkw = {"variant": "learned", "selector": S.load_weights()} if os.path.exists(S.DEFAULT_WEIGHTS) \
        else {"variant": "heuristic"}
    out = {}
    for w in a.workloads.split(","):
        g = graphgen.workload(w)
        G = P.Graph.from_graphgen(g)
        if a.pull_shift:
            r = tune_pull_shift(G, graphgen.pick_sources(g, 64, 123), cache=a.cache, log=log)
            log(f"[autotune] {w}: best pull shift {r['shift']} "
                f"({', '.join(f'{k}: {v * 1e3:.3f} ms' for k, v in r['times_s'].items())})")
            out[w] = r
            G.close()
            continue
        if a.batch:
            src = graphgen.pick_sources(g, 256, 123)
            r = tune_batch_width(G, src, cache=a.cache, log=log)
            log(f"[autotune] {w}: best width {r['width']} "
                f"({', '.join(f'{k}: {v * 1e3:.2f} ms' for k, v in r['times_s'].items())})")
            out[w] = r
            G.close()
            continue
        src = graphgen.pick_sources(g, a.sources, 123)
        r = tune(G, src, a.budget, a.cache, vkw, log)
        log(f"[autotune] {w}: best {r['params']} {r['time_s'] * 1e3:.2f} ms "
            f"(default {r['default_time_s'] * 1e3:.2f} ms)")
        out[w] = r
        G.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
