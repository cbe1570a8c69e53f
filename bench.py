"""Throughput of the masked SpMSpV BFS on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat22]

One step = one search from each of the workload's sources (R-MAT scale 22:
64 seeded sources of nonzero degree), the graph resident in HBM.  Prints ONE
JSON line on stdout; progress goes to stderr.

GTEPS = sum over the step's searches of m_c (edges of the reached component,
each undirected edge once) / wall time of the step.  The step is run in
several forms with identical results (config.modes); value = the batched +
learned form: every source in one multi-source call whose direction (push or
pull) at each level is the trained network's choice.
roofline = the plain push's kernels: the algorithmic bytes of a search (the
method's column reads, frontier traffic and outputs, plus the initialisation of
the outputs and bitmaps) / the device time of its init and level launches, the
durations from HIP events around every launch of one extra, separately timed
step.  The batched form's own roofline is in config.modes.batched_learned.
cpu_baseline = the CPU oracle (queue BFS + min-parent pass, one thread pinned
to one core) timed on a bounded sample of the same searches.
config.other_workloads: the Erdos-Renyi, 4096^2 grid and directed R-MAT s20
workloads (plain push and batched + learned, each with the CPU oracle on its
first sources); serving: the request loop over 32 resident graphs at four
Poisson rates (a time-bounded number of queries per rate, stated).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
CSRC = os.path.join(ROOT, "paper_1906_03113_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sl_level_rmat22_push_traffic.md")
KERNEL_SRC = os.path.join(CSRC, "bfs_slice.hip")
MS_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_ms_rmat22_batched_learned_traffic.md")
MS_KERNEL_SRC = os.path.join(CSRC, "bfs_msbfs.hip")


def measured_traffic(path=TRAFFIC_FILE, src=KERNEL_SRC, key="traffic_bytes_per_launch"):
    """HBM bytes per launch (plain push) or per call (the batch) from a committed
    FETCH_SIZE / WRITE_SIZE summary, or None when there is none or the kernel
    source changed since it was measured."""
    import hashlib
    try:
        txt = open(path).read()
        fields = dict(line.split(": ", 1) for line in txt.splitlines()
                      if line.startswith((key + ":", "kernel_source_sha1:")))
        sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
        if fields.get("kernel_source_sha1", "").strip() != sha:
            return None
        return int(float(fields[key]))
    except (OSError, KeyError, ValueError):
        return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


WORKLOADS = {
    # name: (graphgen key, number of sources, source seed, description)
    "rmat22": ("rmat22", 64, 22, "R-MAT scale 22, edgefactor 16, A/B/C/D=.57/.19/.19/.05, "
                                 "permuted labels, undirected, int32 CSR"),
    "er16k": ("er16k", 1, None, "Erdos-Renyi n=16384, avg degree 8, undirected"),
    "grid4096": ("grid4096", 16, 31, "4096x4096 grid, edges kept with p=0.9, undirected"),
    "rmatd20": ("rmat20d", 16, 32, "R-MAT scale 20, edgefactor 16, directed (out-edges)"),
}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def union_frontier_totals(levels, deg):
    """(sum over levels k of |F_k|, sum over k of the out-degree sum of F_k) for
    the union frontiers F_k of a batch (v in F_k when some source reaches v at
    level k), from the searches' level arrays [sources, n]: each vertex counts
    once per distinct level at which some source reaches it."""
    import numpy as np
    L = np.sort(levels.T, axis=1)                      # [n, sources]
    valid = L >= 0
    distinct = valid[:, 0].astype(np.int64)
    distinct += (valid[:, 1:] & (L[:, 1:] != L[:, :-1])).sum(axis=1)
    return int(distinct.sum()), int((distinct * deg).sum())


def batch_bytes(nq, n, sum_f, sum_d):
    """Algorithmic bytes of one multi-source call: per level, the union
    frontier's columns (4 B per entry, 8 B of row pointers per column) and one
    8-byte mask word per entry and 64 sources; and the 2 x 4 bytes of level and
    parent of every (vertex, source) of the outputs."""
    W = (nq + 63) // 64
    return (4 + 8 * W) * sum_d + 8 * sum_f + 8 * nq * n


def time_calls(fn, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def cpu_oracle_gteps(g, sources, m_c, seconds, max_sources=None):
    """The oracle's queue BFS on one pinned core over the first sources (as
    many as fit `seconds`, at most max_sources): (GTEPS, sample text, core)."""
    import oracle
    ip, ii = g.csc()
    allowed = sorted(os.sched_getaffinity(0))
    core = allowed[-1]
    os.sched_setaffinity(0, {core})
    try:
        t_first = oracle.time_queue_bfs(g.n, g.ptr, g.idx, sources[:1], ip, ii)
        cap = len(sources) if max_sources is None else min(len(sources), max_sources)
        count = max(1, min(cap, int(seconds / max(t_first, 1e-6))))
        t_cpu = (oracle.time_queue_bfs(g.n, g.ptr, g.idx, sources[:count], ip, ii)
                 if count > 1 else t_first)
    finally:
        os.sched_setaffinity(0, allowed)
    return float(sum(m_c[:count])) / t_cpu / 1e9, count, t_cpu, core, len(allowed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22", choices=sorted(WORKLOADS))
    ap.add_argument("--sources", type=int, default=0,
                    help="use only the first N of the workload's sources (0 = all; profiling runs)")
    ap.add_argument("--variant", default="push")
    ap.add_argument("--push-impl", default="auto", choices=["auto", "list", "sliced", "claim"])
    ap.add_argument("--loop", default="host")
    ap.add_argument("--levels-per-sync", type=int, default=0)
    ap.add_argument("--grid-blocks", type=int, default=0)
    ap.add_argument("--heavy-degree", type=int, default=0)
    ap.add_argument("--chunk-edges", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-time-kernels", action="store_true")
    ap.add_argument("--plain-only", action="store_true")
    ap.add_argument("--batch-only", action="store_true",
                    help="after the edge counts, only one batched + learned call (counter runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-other-workloads", action="store_true")
    ap.add_argument("--ms-pull-shift", type=int, default=-1,
                    help="heuristic batch's pull threshold n >> shift (-1 = measure 5, 7, ..., 13 first)")
    ap.add_argument("--serve-set", default="full", choices=["small", "full"])
    ap.add_argument("--serve-queries", type=int, default=2000,
                    help="queries per rate and path (fewer when --serve-seconds runs out first)")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="arrival window per rate and path: the queries that arrive in it are served")
    ap.add_argument("--selector", default=None,
                    help="single-source selector weights (JSON); default: the package's")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the search is single-GPU and sharding is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_1906_03113_amd as P
    from paper_1906_03113_amd import selector as SEL

    torch.cuda.init()                 # the device context first, before the graph is built
    key, nsrc, sseed, desc = WORKLOADS[args.workload]
    t0 = time.time()
    log(f"[bench] building graph {key} ...")
    g = graphgen.workload(key)
    log(f"[bench] graph n={g.n} nnz={g.nnz} directed={g.directed} ({time.time() - t0:.1f}s)")
    sources = np.array([0], np.int32) if sseed is None else graphgen.pick_sources(g, nsrc, sseed)
    if args.sources > 0:
        sources = sources[:args.sources]
    torch.cuda.set_device(0)
    G = P.Graph.from_graphgen(g)
    log(f"[bench] resident on GPU: {G.device_bytes() / 1e6:.1f} MB")
    ws = P.Workspace(G.workspace_size(1))
    level = torch.empty(g.n, dtype=torch.int32, device="cuda")
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    kw = dict(variant=args.variant, loop=args.loop, levels_per_sync=args.levels_per_sync,
              grid_blocks=args.grid_blocks, heavy_degree=args.heavy_degree,
              chunk_edges=args.chunk_edges, push_impl=args.push_impl)
    timek = (args.loop == "host") and not args.no_time_kernels

    # edge counts of each search (from the search's own output), and the level
    # arrays of all sources for the batch's union-frontier totals
    deg = np.diff(g.ptr.astype(np.int64))
    m_c, n_c, nnz_c = [], [], []
    all_levels = np.empty((len(sources), g.n), np.int32)
    for i, s in enumerate(sources):
        P.bfs(G, int(s), level=level, parent=parent, workspace=ws, **kw)
        lv = level.cpu().numpy()
        all_levels[i] = lv
        reached = lv >= 0
        nz = int(deg[reached].sum())
        nnz_c.append(nz)
        n_c.append(int(reached.sum()))
        m_c.append(nz if g.directed else nz // 2)
    total_m = float(sum(m_c))
    log(f"[bench] {len(sources)} sources: mean n_c={np.mean(n_c):.0f} mean m_c={np.mean(m_c):.0f}")
    src = [int(s) for s in sources]
    nq = len(src)

    if args.calibrate_copy:
        a = torch.empty(64 << 20, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 268435456 bytes read, 268435456 bytes written")
        del a, b

    msw = SEL.load_weights(SEL.MS_WEIGHTS)
    ms_meta = json.load(open(SEL.MS_WEIGHTS)).get("meta", {})

    def batched_learned(levels=None, parents=None, workspace=None, info=None, trace=False):
        return P.bfs_batch(G, src, variant="learned", selector=msw, levels=levels, parents=parents,
                           workspace=workspace, info=info, trace=trace)

    if args.batch_only:
        bl = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(nq)]
        bp = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(nq)]
        wsb = P.Workspace(G.workspace_size(nq))
        batched_learned(bl, bp, wsb)
        torch.cuda.synchronize()
        log("[bench] one batched + learned call done")
        return

    def step(info_acc=None):
        for s in sources:
            info = {} if info_acc is not None else None
            P.bfs(G, int(s), level=level, parent=parent, workspace=ws, info=info,
                  time_kernels=info_acc is not None, **kw)
            if info_acc is not None:
                info_acc.append(info)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    dt = time_calls(step, args.steps)
    gteps = total_m / dt / 1e9
    log(f"[bench] plain push, {args.steps} steps: {dt * 1e3:.3f} ms/step, {gteps:.2f} GTEPS")

    # the same step once more with every launch bracketed by HIP events (on
    # the stream the kernels run on): the level kernel's launch durations and
    # the init launch's, for the roofline
    roofline = None
    if timek:
        infos = []
        step(infos)
        torch.cuda.synchronize()
        launches = sum(i["launches"] for i in infos)
        level_us = sum(i["kernel_us"] for i in infos)
        init_us = sum(i["init_us"] for i in infos)
        nsearch = len(infos)
        # algorithmic bytes of one search (the method's own traffic): 4 B per
        # entry of every reached column, 8 B for its two row pointers, 8 B to
        # write and read it as a frontier entry, 8 B for its level and parent,
        # and the initialisation of both outputs (8 n) and of two bitmaps (n / 4)
        b_search = [4 * nz + 24 * nc + 8 * g.n + g.n // 4 for nz, nc in zip(nnz_c, n_c)]
        bytes_total = float(sum(b_search))
        kern_us = level_us + init_us
        ach = bytes_total / (kern_us * 1e-6) / 1e9
        used = {i.get("push_used", "list") for i in infos}
        form = used.pop() if len(used) == 1 else "list"
        sliced = form == "sliced"
        kname = ("k_sl_level" if sliced else "k_cw_narrow / k_cw_wide" if form == "claim" else "k_level")
        traffic = measured_traffic() if (args.workload == "rmat22" and sliced) else None
        per_search = [i["kernel_us"] + i["init_us"] for i in infos]
        roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": kname,
                    "push_form": form,
                    "init_kernel": "k_sl_init" if sliced else "k_cw_fill" if form == "claim" else "k_init",
                    "algorithmic_bytes_per_search": round(bytes_total / nsearch),
                    "kernel_us_per_search": round(kern_us / nsearch, 2),
                    "level_kernel_us_per_search": round(level_us / nsearch, 2),
                    "init_us_per_search": round(init_us / nsearch, 2),
                    "median_kernel_us_per_search": round(float(np.median(per_search)), 2),
                    "launches_per_search": round(launches / nsearch, 2),
                    "mean_launch_us": round(level_us / max(launches, 1), 3),
                    # the same bytes over the whole untimed step (host round trips included)
                    "end_to_end_GBps": round(bytes_total / dt / 1e9, 1),
                    "end_to_end_frac": round(bytes_total / dt / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"[bench] {kname}: {launches} launches, {kern_us / nsearch:.1f} us per search "
            f"(init {init_us / nsearch:.1f}), {ach:.1f} GB/s algorithmic ({ach / HBM_PEAK_GBS * 100:.1f}% of 8 TB/s)")

    # per-level view of the first search (stderr only)
    info = {}
    P.bfs(G, int(sources[0]), level=level, parent=parent, workspace=ws, info=info, trace=True,
          time_kernels=timek, **kw)
    for r in info.get("trace", []):
        log(f"[bench]   level {r['level']:5d} {r['variant']:>7s} |F|={r['frontier']:9d} "
            f"sumdeg(F)={r['frontier_edges']:11d} |U|={r['unvisited']:9d} {r['time_us']:9.1f} us")

    cpu = None
    if not args.no_cpu_baseline:
        cg, count, t_cpu, core, ncpu = cpu_oracle_gteps(g, sources, m_c, args.cpu_seconds)
        cpu = {"value": round(cg, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"first {count} of the {len(sources)} sources of the step "
                         f"({t_cpu:.2f} s, single thread, queue BFS + min-parent pass)",
               "pinned_core": core, "host_cpus": ncpu, "host_cpu_model": _cpu_model()}
        log(f"[bench] cpu oracle: {count} searches in {t_cpu:.2f}s = {cg:.4f} GTEPS")

    modes = {"plain_push": {"gteps": round(gteps, 3), "ms_per_step": round(dt * 1e3, 4),
                            "variant": args.variant, "loop": args.loop}}
    headline = "plain_push"
    if not args.plain_only:
        # Theorem 2's short-circuit push (one claim per reached vertex, parents
        # set by a row pass after the last level); level-kernel time from events
        sc_kw = dict(kw, variant="short_circuit")
        P.bfs(G, int(sources[0]), level=level, parent=parent, workspace=ws, **sc_kw)
        dtc = time_calls(lambda: [P.bfs(G, s_, level=level, parent=parent, workspace=ws, **sc_kw)
                                  for s_ in src], args.steps)
        modes["push_short_circuit"] = {"gteps": round(total_m / dtc / 1e9, 3),
                                       "ms_per_step": round(dtc * 1e3, 4), "loop": args.loop}
        log(f"[bench] push, short-circuit: {dtc * 1e3:.3f} ms/step, {total_m / dtc / 1e9:.2f} GTEPS")
        # one search per source, the single-source network picking the form per level
        wpath = args.selector or SEL.DEFAULT_WEIGHTS
        sel_kw = dict(variant="learned", loop="graph", levels_per_sync=8, selector=SEL.load_weights(wpath))
        for s_ in src[:2]:
            P.bfs(G, s_, level=level, parent=parent, workspace=ws, **sel_kw)
        dts = time_calls(lambda: [P.bfs(G, s_, level=level, parent=parent, workspace=ws, **sel_kw)
                                  for s_ in src], args.steps)
        modes["selector_learned"] = {"gteps": round(total_m / dts / 1e9, 3),
                                     "ms_per_step": round(dts * 1e3, 4), "loop": "graph"}
        log(f"[bench] single-source learned selector (graph loop): {dts * 1e3:.3f} ms/step, "
            f"{total_m / dts / 1e9:.2f} GTEPS")
        if nq > 1:
            del ws, level, parent
            torch.cuda.empty_cache()
            bl = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(nq)]
            bp = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(nq)]
            wsb = P.Workspace(G.workspace_size(nq))
            # batched + learned: one multi-source call, the network's direction per level
            binfo = {}
            batched_learned(bl, bp, wsb, info=binfo, trace=True)
            torch.cuda.synchronize()
            dirs = "".join("L" if r["direction"] == "pull" else "P" for r in binfo["trace"])
            dtb = time_calls(lambda: batched_learned(bl, bp, wsb), args.steps)
            sum_f, sum_d = union_frontier_totals(all_levels, deg)
            b_ms = batch_bytes(nq, g.n, sum_f, sum_d)
            ach_b = b_ms / dtb / 1e9
            modes["batched_learned"] = {
                "gteps": round(total_m / dtb / 1e9, 3), "ms_per_step": round(dtb * 1e3, 4),
                "searches_per_call": nq, "directions": dirs,
                "directions_legend": "one letter per level: P push, L pull",
                "held_out_regret": ms_meta.get("held_out", {}).get("regret"),
                "held_out_heuristic_regret": ms_meta.get("held_out", {}).get("heuristic_regret"),
                "roofline": {"bound": "hbm", "achieved": round(ach_b, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(ach_b / HBM_PEAK_GBS, 4),
                             "algorithmic_bytes_per_call": int(b_ms),
                             "union_frontier_vertices": sum_f, "union_frontier_entries": sum_d,
                             "time": "wall time of the call (host round trips included)",
                             "traffic": measured_traffic(MS_TRAFFIC_FILE, MS_KERNEL_SRC,
                                                         "traffic_bytes_per_call")
                             if args.workload == "rmat22" else None}}
            headline = "batched_learned"
            log(f"[bench] batched + learned ({dirs}): {dtb * 1e3:.3f} ms/step, "
                f"{total_m / dtb / 1e9:.2f} GTEPS, {ach_b:.0f} GB/s algorithmic")
            # the same call with the fixed edge-ratio rule, its threshold tuned on these sources
            shift, tuning = args.ms_pull_shift, None
            if shift < 0:
                from paper_1906_03113_amd import autotune as AT
                ld = 64 * ((nq + 63) // 64)
                vl = torch.empty((g.n, ld), dtype=torch.int32, device="cuda")
                vp = torch.empty((g.n, ld), dtype=torch.int32, device="cuda")
                wsv = P.Workspace(P.batch_vm_workspace_size(G, nq))
                tr = AT.tune_pull_shift(
                    G, src, cache=None,
                    timer=lambda G_, s_, sh: AT.time_pull_shift(G_, s_, sh, reps=2, out=(vl, vp, wsv)))
                shift = tr["shift"]
                tuning = {k: round(v * 1e3, 3) for k, v in tr["times_s"].items()}
                del vl, vp, wsv
            hk = dict(variant="heuristic", ms_pull_shift=shift)
            hinfo = {}
            P.bfs_batch(G, src, levels=bl, parents=bp, workspace=wsb, info=hinfo, trace=True, **hk)
            hdirs = "".join("L" if r["direction"] == "pull" else "P" for r in hinfo["trace"])
            dth = time_calls(lambda: P.bfs_batch(G, src, levels=bl, parents=bp, workspace=wsb, **hk),
                             args.steps)
            modes["batched_heuristic"] = {"gteps": round(total_m / dth / 1e9, 3),
                                          "ms_per_step": round(dth * 1e3, 4), "searches_per_call": nq,
                                          "ms_pull_shift": shift or 5, "directions": hdirs,
                                          "pull_shift_tuning_ms_per_call": tuning}
            log(f"[bench] batched, edge-ratio rule (shift {shift}, {hdirs}): {dth * 1e3:.3f} ms/step, "
                f"{total_m / dth / 1e9:.2f} GTEPS")
            del bl, bp, wsb
            torch.cuda.empty_cache()
            # the learned batch with the results in one vertex-major pair of
            # arrays (the search's own layout: no transpose pass); reported
            # beside, not the headline (a different output layout)
            ld = 64 * ((nq + 63) // 64)
            vl = torch.empty((g.n, ld), dtype=torch.int32, device="cuda")
            vp = torch.empty((g.n, ld), dtype=torch.int32, device="cuda")
            wsv = P.Workspace(P.batch_vm_workspace_size(G, nq))
            vk = dict(variant="learned", selector=msw, level=vl, parent=vp, workspace=wsv)
            P.bfs_batch_vm(G, src, **vk)
            dtv = time_calls(lambda: P.bfs_batch_vm(G, src, **vk), args.steps)
            modes["batched_learned_vertex_major"] = {
                "gteps": round(total_m / dtv / 1e9, 3), "ms_per_step": round(dtv * 1e3, 4),
                "searches_per_call": nq, "layout": "vertex-major [n][64 * ceil(sources / 64)]"}
            log(f"[bench] batched + learned, vertex-major results: {dtv * 1e3:.3f} ms/step, "
                f"{total_m / dtv / 1e9:.2f} GTEPS")
            del vl, vp, wsv
    if cpu is not None:
        cpu["gpu_over_cpu"] = round(modes[headline]["gteps"] / cpu["value"], 1)
    G.close()
    del G, all_levels
    torch.cuda.empty_cache()

    others = None
    if not args.plain_only and not args.no_other_workloads and args.workload == "rmat22":
        others = {}
        for wname in ("er16k", "grid4096", "rmatd20"):
            others[wname] = other_workload(wname, args, msw)

    serving = None
    if not args.no_serve and not args.plain_only:
        from paper_1906_03113_amd import serve as SV
        res = SV.experiment(args.serve_set, queries=args.serve_queries, seconds=args.serve_seconds,
                            rates=(0.25, 0.5, 0.8, 0.95), log=log)
        serving = {"graphs": len(res["graphs"]), "graph_names": res["graphs"],
                   "saturation_qps_plain": round(res["saturation_qps_plain"], 1),
                   "queries_per_rate": f"the queries arriving in {args.serve_seconds:g} s at each rate, "
                                       f"at most {args.serve_queries} (time-bounded subset)"}
        for frac, r in res["rates"].items():
            for path, v in r.items():
                if v["failed"]:
                    raise RuntimeError(f"serving at {frac} x saturation: {v['failed']} {path} queries failed")
            serving[f"{frac}x_sat"] = {
                k: {"queries": v["queries"], "p50_ms": round(v["p50_ms"], 3), "p99_ms": round(v["p99_ms"], 3),
                    "achieved_qps": round(v["achieved_qps"], 1)} for k, v in r.items()}

    out = {
        "metric": "GTEPS on R-MAT s22 (64 sources per step): batched + learned form (value) vs the "
                  "plain masked push, every form in config.modes",
        "value": modes[headline]["gteps"],
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": modes[headline]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": desc, "n": g.n, "nnz": g.nnz,
                   "sources": int(len(sources)), "searches_per_step": int(len(sources)),
                   "edges_per_step_m_c": int(total_m), "headline_mode": headline,
                   "best_mode": max(modes, key=lambda m: modes[m]["gteps"]),
                   "modes": modes, "other_workloads": others},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


def other_workload(wname, args, msw):
    """One of the other workloads: plain push (one search per source) and,
    with several sources, the batched + learned call; the CPU oracle on the
    first sources (at most 8); for deep graphs the time per level."""
    import numpy as np
    import torch
    import graphgen
    import paper_1906_03113_amd as P
    key, nsrc, sseed, desc = WORKLOADS[wname]
    t0 = time.time()
    g = graphgen.workload(key)
    sources = np.array([0], np.int32) if sseed is None else graphgen.pick_sources(g, nsrc, sseed)
    src = [int(s) for s in sources]
    G = P.Graph.from_graphgen(g)
    ws = P.Workspace(G.workspace_size(1))
    level = torch.empty(g.n, dtype=torch.int32, device="cuda")
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    deg = np.diff(g.ptr.astype(np.int64))
    m_c, levels = [], []
    for s in src:
        info = {}
        P.bfs(G, s, level=level, parent=parent, workspace=ws, info=info)
        lv = level.cpu().numpy()
        nz = int(deg[lv >= 0].sum())
        m_c.append(nz if g.directed else nz // 2)
        levels.append(int(info["levels"]))
        form = info.get("push_used", "list")
    tm = float(sum(m_c))
    steps = max(1, min(args.steps, 3))
    dt = time_calls(lambda: [P.bfs(G, s, level=level, parent=parent, workspace=ws) for s in src], steps)
    res = {"graph": desc, "n": g.n, "nnz": g.nnz, "sources": len(src), "mean_levels": float(np.mean(levels)),
           "plain_push": {"gteps": round(tm / dt / 1e9, 3), "ms_per_step": round(dt * 1e3, 3),
                          "us_per_level": round(dt * 1e6 / sum(levels), 2), "form": form}}
    if len(src) > 1:
        del ws, level, parent
        torch.cuda.empty_cache()
        bl = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in src]
        bp = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in src]
        wsb = P.Workspace(G.workspace_size(len(src)))
        bk = dict(variant="learned", selector=msw, levels=bl, parents=bp, workspace=wsb)
        P.bfs_batch(G, src, **bk)
        dtb = time_calls(lambda: P.bfs_batch(G, src, **bk), steps)
        res["batched_learned"] = {"gteps": round(tm / dtb / 1e9, 3), "ms_per_step": round(dtb * 1e3, 3),
                                  "us_per_level": round(dtb * 1e6 / max(levels), 2)}
        # the same sources in one call with the push on every level: the
        # library's own choice of form for the batch (claim-word searches in
        # lockstep on thin graphs)
        del wsb
        torch.cuda.empty_cache()
        pk = dict(variant="push", levels=bl, parents=bp)
        P.bfs_batch(G, src, **pk)
        dtp = time_calls(lambda: P.bfs_batch(G, src, **pk), steps)
        res["batched_push"] = {"gteps": round(tm / dtp / 1e9, 3), "ms_per_step": round(dtp * 1e3, 3),
                               "us_per_level": round(dtp * 1e6 / max(levels), 2)}
        del bl, bp
    if not args.no_cpu_baseline:
        cg, count, t_cpu, _, _ = cpu_oracle_gteps(g, sources, m_c, seconds=30.0, max_sources=8)
        res["cpu_baseline"] = {"value": round(cg, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
                               "sample": f"first {count} of the {len(src)} sources ({t_cpu:.2f} s, one thread)"}
    G.close()
    torch.cuda.empty_cache()
    log(f"[bench] {wname}: {json.dumps(res)} ({time.time() - t0:.1f}s)")
    return res


if __name__ == "__main__":
    main()
