"""The batching measurements: many sources on one graph in one call, and many
uneven graphs in one launch.

    python -m paper_1906_03113_amd.experiments [--only sources|graphs|compare|spmspv] [--out FILE]

* sources: directed R-MAT scale 20 (edgefactor 16, out-edges), 256 sources of
  nonzero out-degree (seed 41) in one bfs_run_batch call (4 mask words per
  vertex), against the same 256 searches one at a time (plain push, and the
  fixed-rule direction choice with the graph loop).
* graphs: 64 undirected ER graphs, n_g = round(2^U(10,18)), average degree
  U(4,32), graph g seeded 1000+g, packed block-diagonally, the lowest-index
  vertex of nonzero degree of each block as its root: one search from the 64
  roots (persistent kernel, and the graph loop), against 64 separate searches
  on the separate graphs (plain push with the defaults, and with each graph's
  launch parameters from the tuning cache when one is given).

* compare: the Experiments section's comparison searches (SpMV-BFS, SpMSpV-BFS,
  SpMmSpV-BFS) against the method on ER n=16,384, directed R-MAT s20, R-MAT
  s22 and 1024^2 / 4096^2 grids: operation counts and time per search.
* spmspv: the masked SpMSpV primitive on every level of an R-MAT s22 search.

Throughput is GTEPS = sum over the searches of m_c (edges of the reached
component; each undirected edge once, each directed edge once) / wall time,
every graph resident and every output buffer allocated before the timed part.
"""
from __future__ import annotations

import json
import sys
import time
from typing import Dict, List

import numpy as np


def _torch():
    import torch
    return torch


def _edges_reached(g, level: np.ndarray) -> int:
    deg = np.diff(g.ptr.astype(np.int64))
    nz = int(deg[level >= 0].sum())
    return nz if g.directed else nz // 2


def _timed(fn, reps: int = 3) -> float:
    """Best wall time (s) of reps calls after one warm-up call."""
    torch = _torch()
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def many_sources(count: int = 256, seed: int = 41, log=print) -> Dict:
    import graphgen
    import paper_1906_03113_amd as P
    torch = _torch()
    g = graphgen.workload("rmat20d")
    src = [int(s) for s in graphgen.pick_sources(g, count, seed)]
    G = P.Graph.from_graphgen(g)
    n = g.n
    lv = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in src]
    pa = [torch.empty(n, dtype=torch.int32, device="cuda") for _ in src]
    wsb = P.Workspace(G.workspace_size(len(src)))
    P.bfs_batch(G, src, levels=lv, parents=pa, workspace=wsb, variant="heuristic")
    torch.cuda.synchronize()
    m = sum(_edges_reached(g, l.cpu().numpy()) for l in lv)
    t_batch = _timed(lambda: P.bfs_batch(G, src, levels=lv, parents=pa, workspace=wsb, variant="heuristic"))
    log(f"[sources] {len(src)} sources in one call: {t_batch * 1e3:.2f} ms, {m / t_batch / 1e9:.2f} GTEPS")
    del lv, pa, wsb
    torch.cuda.empty_cache()
    ld = 64 * ((len(src) + 63) // 64)
    vl = torch.empty((n, ld), dtype=torch.int32, device="cuda")
    vp = torch.empty((n, ld), dtype=torch.int32, device="cuda")
    wsv = P.Workspace(P.batch_vm_workspace_size(G, len(src)))
    t_vm = _timed(lambda: P.bfs_batch_vm(G, src, level=vl, parent=vp, workspace=wsv, variant="heuristic"))
    log(f"[sources] {len(src)} sources in one call, vertex-major results: {t_vm * 1e3:.2f} ms, "
        f"{m / t_vm / 1e9:.2f} GTEPS")
    del vl, vp, wsv
    torch.cuda.empty_cache()
    l1 = torch.empty(n, dtype=torch.int32, device="cuda")
    p1 = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = P.Workspace(G.workspace_size(1))
    res = {"graph": "R-MAT scale 20, edgefactor 16, directed", "n": n, "nnz": g.nnz,
           "sources": len(src), "edges_m_c": m,
           "one_call": {"ms": t_batch * 1e3, "gteps": m / t_batch / 1e9},
           "one_call_vertex_major": {"ms": t_vm * 1e3, "gteps": m / t_vm / 1e9}}
    for name, kw in (("one_at_a_time_push", dict(variant="push")),
                     ("one_at_a_time_heuristic_graph_loop",
                      dict(variant="heuristic", loop="graph", levels_per_sync=8))):
        def run(kw=kw):
            for s in src:
                P.bfs(G, s, level=l1, parent=p1, workspace=ws, **kw)
        t = _timed(run, reps=2)
        res[name] = {"ms": t * 1e3, "gteps": m / t / 1e9}
        log(f"[sources] {name}: {t * 1e3:.2f} ms, {m / t / 1e9:.2f} GTEPS")
    G.close()
    return res


def many_graphs(count: int = 64, tune_cache: str = "", log=print) -> Dict:
    import graphgen
    import paper_1906_03113_amd as P
    torch = _torch()
    gs = graphgen.er_family(count=count, lo=10, hi=18, dmin=4, dmax=32)
    packed, offs = graphgen.block_diagonal(gs)
    roots, m = [], 0
    for b, g in enumerate(gs):
        nz = np.nonzero(g.out_degree() > 0)[0]
        roots.append(int(offs[b] + (nz[0] if len(nz) else 0)))
    Gp = P.Graph.from_graphgen(packed)
    lv = torch.empty(packed.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(packed.n, dtype=torch.int32, device="cuda")
    wsr = P.Workspace(Gp.roots_workspace_size(len(roots)))
    P.bfs_roots(Gp, roots, level=lv, parent=pa, workspace=wsr, loop="persistent")
    torch.cuda.synchronize()
    m = _edges_reached(packed, lv.cpu().numpy())
    res = {"graphs": count, "n_total": packed.n, "nnz_total": packed.nnz, "edges_m_c": m,
           "n_range": [min(g.n for g in gs), max(g.n for g in gs)]}
    for name, kw in (("one_launch_persistent", dict(loop="persistent")),
                     ("one_search_graph_loop", dict(loop="graph", levels_per_sync=16)),
                     ("one_search_host_loop", dict(loop="host"))):
        t = _timed(lambda kw=kw: P.bfs_roots(Gp, roots, level=lv, parent=pa, workspace=wsr, **kw))
        res[name] = {"ms": t * 1e3, "gteps": m / t / 1e9}
        log(f"[graphs] {name}: {t * 1e3:.2f} ms, {m / t / 1e9:.2f} GTEPS")
    Gp.close()
    del lv, pa, wsr
    torch.cuda.empty_cache()
    # the same 64 searches on the 64 separate graphs
    Gs = [P.Graph.from_graphgen(g) for g in gs]
    outs = [(torch.empty(g.n, dtype=torch.int32, device="cuda"),
             torch.empty(g.n, dtype=torch.int32, device="cuda"),
             P.Workspace(G.workspace_size(1))) for g, G in zip(gs, Gs)]
    local = [int(r - offs[b]) for b, r in enumerate(roots)]
    params: List[Dict] = [{} for _ in gs]
    if tune_cache:
        # each distinct graph shape tuned once (on its first graph), then looked up
        from . import autotune as AT
        tuned_keys = set()
        for b, (g, G) in enumerate(zip(gs, Gs)):
            info = {}
            P.bfs(G, local[b], info=info)
            key = AT.shape_key(G, int(info["levels"]))
            if key not in tuned_keys:
                AT.tune(G, [local[b]], budget=10, cache=tune_cache, variant_kw={"variant": "push"})
                tuned_keys.add(key)
            params[b] = AT.lookup(G, int(info["levels"]), tune_cache)
        res["tuned_shapes"] = len(tuned_keys)
        log(f"[graphs] tuned {len(tuned_keys)} graph shapes")

    def separate(tuned: bool):
        for b, G in enumerate(Gs):
            l, p, w = outs[b]
            P.bfs(G, local[b], level=l, parent=p, workspace=w, **(params[b] if tuned else {}))

    t = _timed(lambda: separate(False))
    res["separate_searches_push"] = {"ms": t * 1e3, "gteps": m / t / 1e9}
    log(f"[graphs] 64 separate searches (push, defaults): {t * 1e3:.2f} ms, {m / t / 1e9:.2f} GTEPS")
    if tune_cache:
        t = _timed(lambda: separate(True))
        res["separate_searches_tuned"] = {"ms": t * 1e3, "gteps": m / t / 1e9}
        log(f"[graphs] 64 separate searches (tuned parameters): {t * 1e3:.2f} ms, {m / t / 1e9:.2f} GTEPS")
    # one multi-graph call (the library runs the queries one after another)
    lvs = [o[0] for o in outs]
    pas = [o[1] for o in outs]
    wsm = P.Workspace(max(G.workspace_size(1) for G in Gs))
    t = _timed(lambda: P.bfs_batch(Gs, local, levels=lvs, parents=pas, workspace=wsm))
    res["multi_graph_call"] = {"ms": t * 1e3, "gteps": m / t / 1e9}
    log(f"[graphs] one bfs_run_batch over the 64 graphs: {t * 1e3:.2f} ms, {m / t / 1e9:.2f} GTEPS")
    for G in Gs:
        G.close()
    return res


def compare(workloads=("er16k", "rmat20d", "rmat22", "grid1024", "grid4096"), log=print) -> Dict:
    """The comparison searches of the Experiments section against the method
    (plain push, and the short-circuit form), one source per graph (the first
    of pick_sources(g, 1, 22)): device operation counts (Table 2's
    convention) and wall time per search, best of 3 after a warm-up.  The
    unmasked SpMSpV-BFS is left out on the 4096^2 grid (its vector covers the
    component within a few hundred of the ~7,000 steps)."""
    import graphgen
    import paper_1906_03113_amd as P
    torch = _torch()
    res = {}
    for w in workloads:
        g = graphgen.grid(1024, 0.9, 3) if w == "grid1024" else graphgen.workload(w)
        G = P.Graph.from_graphgen(g)
        s = int(graphgen.pick_sources(g, 1, 22)[0])
        lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
        pa = torch.empty_like(lv)
        ws = P.Workspace(P.compare_workspace_size(G))
        row = {"n": g.n, "nnz": g.nnz, "source": s}
        for m in ("spmv", "spmspv", "spmmspv"):
            if m == "spmspv" and w == "grid4096":
                continue
            box = {}

            def run(m=m, box=box):
                box["r"] = P.bfs_compare(G, s, m, level=lv, parent=pa, workspace=ws)
            t = _timed(run)
            _, _, ops, steps = box["r"]
            row[m] = {"ms": t * 1e3, "ops": ops, "steps": steps}
            log(f"[compare] {w} {m}: {t * 1e3:.2f} ms, ops {ops}, steps {steps}")
        ws1 = P.Workspace(G.workspace_size(1))
        deep = w.startswith("grid")
        for v in ("push", "short_circuit"):
            kw = dict(variant=v, loop="graph", levels_per_sync=64 if deep else 8)
            t = _timed(lambda kw=kw: P.bfs(G, s, level=lv, parent=pa, workspace=ws1, **kw))
            n_c = int((lv >= 0).sum().item())
            row[v] = {"ms": t * 1e3, "ops": 2 * (n_c - 1)}
            log(f"[compare] {w} method ({v}): {t * 1e3:.2f} ms, ops {2 * (n_c - 1)}")
        res[w] = row
        G.close()
        del ws, ws1, lv, pa
        torch.cuda.empty_cache()
    return res


def spmspv_levels(log=print) -> Dict:
    """The masked SpMSpV primitive on the levels of an R-MAT s22 search: for
    each level k of the search from the first of the 64 bench sources
    (pick_sources(g, 64, 22)[0]), x = F_k with x(j) = j and the row mask = the
    rows visited through level k, complemented; (min, select) and Boolean
    products, wall time of one call (which waits for the stream) after one
    warm-up call.  The levels come from the library's own search."""
    import graphgen
    import paper_1906_03113_amd as P
    torch = _torch()
    g = graphgen.workload("rmat22")
    G = P.Graph.from_graphgen(g)
    s = int(graphgen.pick_sources(g, 64, 22)[0])
    lv, _ = P.bfs(G, s)
    wl = lv.cpu().numpy()
    deg = np.diff(g.ptr.astype(np.int64))
    yi = torch.empty(g.n, dtype=torch.int32, device="cuda")
    yv = torch.empty(g.n, dtype=torch.int64, device="cuda")
    ws = P.Workspace(P.spmspv_workspace_size(G, int((wl >= 0).sum())))
    ws.buf.zero_()
    out = []
    for k in range(int(wl.max()) + 1):
        front = np.nonzero(wl == k)[0].astype(np.int32)
        seen = np.nonzero((wl >= 0) & (wl <= k))[0]
        words = np.zeros((g.n + 31) // 32, np.uint32)
        np.bitwise_or.at(words, seen >> 5, (np.uint32(1) << (seen & 31).astype(np.uint32)))
        xi = torch.from_numpy(front).cuda()
        xv = torch.from_numpy(front.astype(np.int64)).cuda()
        mask = torch.from_numpy(words.view(np.int32)).cuda()
        row = {"level": k, "vector": len(front), "entries": int(deg[front].sum())}
        for sr in ("min_select", "boolean"):
            P.masked_spmspv(G, sr, xi, xv, mask, None, True, workspace=ws, y_idx=yi, y_val=yv)
            t0 = time.perf_counter()
            a, _ = P.masked_spmspv(G, sr, xi, xv, mask, None, True, workspace=ws, y_idx=yi, y_val=yv)
            t = time.perf_counter() - t0
            row[sr] = {"ms": t * 1e3}
            row["support"] = int(a.numel())
            log(f"[spmspv] level {k} |x|={len(front)} entries {row['entries']} {sr}: {t * 1e3:.3f} ms, "
                f"support {a.numel()}")
        out.append(row)
    G.close()
    return {"levels": out}


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="batching measurements (many sources, many graphs)")
    ap.add_argument("--only", choices=["sources", "graphs", "compare", "spmspv"], default=None)
    ap.add_argument("--tune-cache", default="", help="autotune cache for per-graph parameters")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    torch = _torch()
    torch.cuda.init()
    out = {}
    if a.only in (None, "sources"):
        out["many_sources"] = many_sources(log=log)
    if a.only in (None, "graphs"):
        out["many_graphs"] = many_graphs(tune_cache=a.tune_cache, log=log)
    if a.only in (None, "compare"):
        out["compare"] = compare(log=log)
    if a.only in (None, "spmspv"):
        out["spmspv"] = spmspv_levels(log=log)
    txt = json.dumps(out)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
    print(txt)


if __name__ == "__main__":
    main()
