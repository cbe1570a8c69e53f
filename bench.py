"""Throughput of the masked SpMSpV BFS on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload rmat22]

One step = one search from each of the workload's sources (R-MAT scale 22:
64 seeded sources of nonzero degree), the graph resident in HBM.  Prints ONE
JSON line on stdout; progress goes to stderr.

value = GTEPS = sum over the step's searches of m_c (edges of the reached
component, each undirected edge once) / wall time of the step.
roofline = the plain push's kernels: the algorithmic bytes of a search (the
method's column reads, frontier traffic and outputs, plus the initialisation of
the outputs and bitmaps) / the device time of its init and level launches, the
durations from HIP events around every launch of one extra, separately timed
step.
cpu_baseline = the CPU oracle (queue BFS + min-parent pass, one thread pinned
to one core) timed on a bounded sample of the same searches.
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sl_level_rmat22_push_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1906_03113_amd", "csrc", "bfs_slice.hip")


def measured_traffic():
    """HBM bytes per level launch of the plain push (k_sl_level) from the
    committed FETCH_SIZE / WRITE_SIZE summary, or None when there is none or
    the kernel source changed since it was measured."""
    import hashlib
    try:
        txt = open(TRAFFIC_FILE).read()
        fields = dict(line.split(": ", 1) for line in txt.splitlines()
                      if line.startswith(("traffic_bytes_per_launch:", "kernel_source_sha1:")))
        sha = hashlib.sha1(open(KERNEL_SRC, "rb").read()).hexdigest()
        if fields.get("kernel_source_sha1", "").strip() != sha:
            return None
        return int(float(fields["traffic_bytes_per_launch"]))
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22", choices=sorted(WORKLOADS))
    ap.add_argument("--variant", default="push")
    ap.add_argument("--loop", default="host")
    ap.add_argument("--levels-per-sync", type=int, default=0)
    ap.add_argument("--grid-blocks", type=int, default=0)
    ap.add_argument("--heavy-degree", type=int, default=0)
    ap.add_argument("--chunk-edges", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-time-kernels", action="store_true")
    ap.add_argument("--plain-only", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--ms-pull-shift", type=int, default=-1,
                    help="multi-source pull threshold n >> shift (-1 = measure 5, 7, ..., 13 first, 0 = n/32)")
    ap.add_argument("--serve-queries", type=int, default=300)
    ap.add_argument("--selector", default=None,
                    help="selector weights (JSON); default: the trained weights in the package")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the search is single-GPU and sharding is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen
    import paper_1906_03113_amd as P

    torch.cuda.init()                 # the device context first, before the graph is built
    key, nsrc, sseed, desc = WORKLOADS[args.workload]
    t0 = time.time()
    log(f"[bench] building graph {key} ...")
    g = graphgen.workload(key)
    log(f"[bench] graph n={g.n} nnz={g.nnz} directed={g.directed} ({time.time() - t0:.1f}s)")
    sources = np.array([0], np.int32) if sseed is None else graphgen.pick_sources(g, nsrc, sseed)
    torch.cuda.set_device(0)
    G = P.Graph.from_graphgen(g)
    log(f"[bench] resident on GPU: {G.device_bytes() / 1e6:.1f} MB")
    ws = P.Workspace(G.workspace_size(1))
    level = torch.empty(g.n, dtype=torch.int32, device="cuda")
    parent = torch.empty(g.n, dtype=torch.int32, device="cuda")
    kw = dict(variant=args.variant, loop=args.loop, levels_per_sync=args.levels_per_sync,
              grid_blocks=args.grid_blocks, heavy_degree=args.heavy_degree,
              chunk_edges=args.chunk_edges)
    timek = (args.loop == "host") and not args.no_time_kernels

    # edge counts of each search (from the search's own output)
    deg = np.diff(g.ptr.astype(np.int64))
    m_c, n_c, nnz_c = [], [], []
    for s in sources:
        P.bfs(G, int(s), level=level, parent=parent, workspace=ws, **kw)
        lv = level.cpu().numpy()
        reached = lv >= 0
        nz = int(deg[reached].sum())
        nnz_c.append(nz)
        n_c.append(int(reached.sum()))
        m_c.append(nz if g.directed else nz // 2)
    total_m = float(sum(m_c))
    log(f"[bench] {len(sources)} sources: mean n_c={np.mean(n_c):.0f} mean m_c={np.mean(m_c):.0f}")

    def step(info_acc=None):
        for s in sources:
            info = {} if info_acc is not None else None
            P.bfs(G, int(s), level=level, parent=parent, workspace=ws, info=info,
                  time_kernels=info_acc is not None, **kw)
            if info_acc is not None:
                info_acc.append(info)

    if args.calibrate_copy:
        a = torch.empty(64 << 20, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 268435456 bytes read, 268435456 bytes written")
        del a, b
    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"[bench] warmup {w + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    dt = (t_end - t_start) / args.steps
    gteps = total_m / dt / 1e9
    log(f"[bench] {args.steps} steps: {dt * 1e3:.3f} ms/step, {gteps:.2f} GTEPS")

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
        sliced = args.variant == "push" and g.n <= 4 * 32768 * 32 and args.loop in ("host", "graph")
        kname = "k_sl_level" if sliced else "k_level"
        traffic = measured_traffic() if (args.workload == "rmat22" and sliced) else None
        per_search = [i["kernel_us"] + i["init_us"] for i in infos]
        roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": kname, "init_kernel": "k_sl_init" if sliced else "k_init",
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
        import oracle
        ip, ii = g.csc()
        # single thread, pinned to one core of those this process may use
        allowed = sorted(os.sched_getaffinity(0))
        core = allowed[-1]
        os.sched_setaffinity(0, {core})
        try:
            t_first = oracle.time_queue_bfs(g.n, g.ptr, g.idx, sources[:1], ip, ii)
            count = max(1, min(len(sources), int(args.cpu_seconds / max(t_first, 1e-6))))
            t_cpu = (oracle.time_queue_bfs(g.n, g.ptr, g.idx, sources[:count], ip, ii)
                     if count > 1 else t_first)
        finally:
            os.sched_setaffinity(0, allowed)
        cpu_gteps = float(sum(m_c[:count])) / t_cpu / 1e9
        cpu = {"value": round(cpu_gteps, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"first {count} of the {len(sources)} sources of the step "
                         f"({t_cpu:.2f} s, single thread, queue BFS + min-parent pass)",
               "pinned_core": core, "host_cpus": len(allowed), "host_cpu_model": _cpu_model(),
               "gpu_over_cpu": round(gteps / cpu_gteps, 1)}
        log(f"[bench] cpu oracle: {count} searches in {t_cpu:.2f}s = {cpu_gteps:.4f} GTEPS")

    # the other configurations of the same step (same sources, same outputs)
    vm_mode = None
    modes = {"plain_push": {"gteps": round(gteps, 3), "ms_per_step": round(dt * 1e3, 4),
                            "variant": args.variant, "loop": args.loop}}
    if not args.plain_only:
        # Theorem 2's short-circuit push (one claim per reached vertex, parents
        # set by a row pass after the last level); level-kernel time from events
        sc_kw = dict(kw, variant="short_circuit")
        P.bfs(G, int(sources[0]), level=level, parent=parent, workspace=ws, **sc_kw)
        sc_infos = []
        torch.cuda.synchronize()
        t0c = time.perf_counter()
        for k in range(args.steps):
            for s in sources:
                info = {}
                P.bfs(G, int(s), level=level, parent=parent, workspace=ws, info=info,
                      time_kernels=timek, **sc_kw)
                sc_infos.append(info)
        torch.cuda.synchronize()
        dtc = (time.perf_counter() - t0c) / args.steps
        modes["push_short_circuit"] = {"gteps": round(total_m / dtc / 1e9, 3),
                                       "ms_per_step": round(dtc * 1e3, 4), "loop": args.loop}
        if timek:
            kus = sum(i["kernel_us"] for i in sc_infos) / (len(sources) * args.steps)
            modes["push_short_circuit"]["level_kernel_us_per_search"] = round(kus, 2)
            b_avg = float(sum(4 * nz + 24 * nc for nz, nc in zip(nnz_c, n_c))) / len(sources)
            modes["push_short_circuit"]["level_kernel_frac_of_hbm"] = round(b_avg / (kus * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
        log(f"[bench] push, short-circuit: {dtc * 1e3:.3f} ms/step, {total_m / dtc / 1e9:.2f} GTEPS")
        from paper_1906_03113_amd import selector as SEL
        wpath = args.selector or SEL.DEFAULT_WEIGHTS
        sel_variant = "learned" if os.path.exists(wpath) else "heuristic"
        sel_kw = dict(variant=sel_variant, loop="graph", levels_per_sync=8)
        if sel_variant == "learned":
            sel_kw["selector"] = SEL.load_weights(wpath)
        for s in sources[:2]:
            P.bfs(G, int(s), level=level, parent=parent, workspace=ws, **sel_kw)
        torch.cuda.synchronize()
        t0s = time.perf_counter()
        for k in range(args.steps):
            for s in sources:
                P.bfs(G, int(s), level=level, parent=parent, workspace=ws, **sel_kw)
        torch.cuda.synchronize()
        dts = (time.perf_counter() - t0s) / args.steps
        modes["selector_" + sel_variant] = {"gteps": round(total_m / dts / 1e9, 3),
                                            "ms_per_step": round(dts * 1e3, 4), "loop": "graph"}
        log(f"[bench] selector ({sel_variant}, graph loop): {dts * 1e3:.3f} ms/step, "
            f"{total_m / dts / 1e9:.2f} GTEPS")
        # all sources in one multi-source call (64 per mask word)
        nq = len(sources)
        if nq > 1:
            src = [int(s) for s in sources]
            ld = 64 * ((nq + 63) // 64)
            vl = torch.empty((g.n, ld), dtype=torch.int32, device="cuda")
            vp = torch.empty((g.n, ld), dtype=torch.int32, device="cuda")
            wsv = P.Workspace(P.batch_vm_workspace_size(G, nq))
            # the multi-source direction threshold (pull once the union
            # frontier holds more than n >> shift vertices): the autotuner's
            # measured search over these sources, before the timed region
            shift, tuning = args.ms_pull_shift, None
            if shift < 0:
                from paper_1906_03113_amd import autotune as AT
                tr = AT.tune_pull_shift(
                    G, src, cache=None,
                    timer=lambda G_, s_, sh: AT.time_pull_shift(G_, s_, sh, reps=2, out=(vl, vp, wsv)))
                shift = tr["shift"]
                tuning = {k: round(v * 1e3, 3) for k, v in tr["times_s"].items()}
                log(f"[bench] multi-source pull shift {shift} "
                    f"(ms per call: {', '.join(f'{k}: {v}' for k, v in tuning.items())})")
            bl = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(nq)]
            bp = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in range(nq)]
            wsb = P.Workspace(G.workspace_size(nq))
            P.bfs_batch(G, src, levels=bl, parents=bp, workspace=wsb, variant="heuristic",
                        ms_pull_shift=shift)
            torch.cuda.synchronize()
            t0b = time.perf_counter()
            for k in range(args.steps):
                P.bfs_batch(G, src, levels=bl, parents=bp, workspace=wsb, variant="heuristic",
                            ms_pull_shift=shift)
            torch.cuda.synchronize()
            dtb = (time.perf_counter() - t0b) / args.steps
            # the per-search algorithmic bytes of the plain form, summed over the
            # batch's searches, over the batch's wall time: what separate
            # searches would have to move, so above-peak values are possible
            # (one read of a column serves every source whose frontier holds it)
            b_step = float(sum(4 * nz + 24 * nc for nz, nc in zip(nnz_c, n_c)))
            modes["batch_multisource"] = {"gteps": round(total_m / dtb / 1e9, 3),
                                          "ms_per_step": round(dtb * 1e3, 4),
                                          "searches_per_call": nq,
                                          "ms_pull_shift": shift or 5,
                                          "pull_shift_tuning_ms_per_call": tuning,
                                          "plain_bytes_per_step": round(b_step),
                                          "plain_bytes_rate_GBps": round(b_step / dtb / 1e9, 1)}
            log(f"[bench] multi-source batch: {dtb * 1e3:.3f} ms/step, {total_m / dtb / 1e9:.2f} GTEPS")
            del bl, bp, wsb
            torch.cuda.empty_cache()
            # the same searches with the results in one vertex-major pair of
            # arrays (the search's own layout: no transpose pass); reported
            # beside, not a candidate for `value` (a different output layout)
            P.bfs_batch_vm(G, src, level=vl, parent=vp, workspace=wsv, ms_pull_shift=shift)
            torch.cuda.synchronize()
            t0v = time.perf_counter()
            for k in range(args.steps):
                P.bfs_batch_vm(G, src, level=vl, parent=vp, workspace=wsv, ms_pull_shift=shift)
            torch.cuda.synchronize()
            dtv = (time.perf_counter() - t0v) / args.steps
            vm_mode = {"gteps": round(total_m / dtv / 1e9, 3), "ms_per_step": round(dtv * 1e3, 4),
                       "searches_per_call": nq, "ms_pull_shift": shift or 5,
                       "layout": "vertex-major [n][64 * ceil(sources / 64)]"}
            log(f"[bench] multi-source batch, vertex-major results: {dtv * 1e3:.3f} ms/step, "
                f"{total_m / dtv / 1e9:.2f} GTEPS")
            del vl, vp, wsv
    best = max(modes, key=lambda m: modes[m]["gteps"])
    if vm_mode is not None:
        modes["batch_multisource_vertex_major"] = vm_mode

    serving = None
    if not args.no_serve and not args.plain_only:
        # free this workload's buffers before the resident set comes in
        del ws, level, parent
        torch.cuda.empty_cache()
        from paper_1906_03113_amd import serve as SV
        res = SV.experiment("small", queries=args.serve_queries, rates=(0.5, 0.95), log=log)
        serving = {"graphs": res["graphs"], "saturation_qps_plain": round(res["saturation_qps_plain"], 1),
                   "queries_per_rate": args.serve_queries}
        for frac, r in res["rates"].items():
            serving[f"{frac}x_sat"] = {
                k: {"p50_ms": round(v["p50_ms"], 3), "p99_ms": round(v["p99_ms"], 3),
                    "achieved_qps": round(v["achieved_qps"], 1)} for k, v in r.items()}

    out = {
        "metric": "GTEPS on R-MAT s22 (64 sources per step): plain masked push vs the batched / "
                  "variant-selecting forms; value = the best form, every form in config.modes",
        "value": modes[best]["gteps"],
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": modes[best]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": desc, "n": g.n, "nnz": g.nnz,
                   "sources": int(len(sources)), "searches_per_step": int(len(sources)),
                   "edges_per_step_m_c": int(total_m), "best_mode": best, "modes": modes},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
