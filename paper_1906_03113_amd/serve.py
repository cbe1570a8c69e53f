"""Continuous-batching BFS query server over graphs resident in HBM.

Queries (graph, source) arrive at any time.  A scheduler keeps them in arrival
order and hands work to a fixed set of workers, each with its own HIP stream,
so the searches of different workers overlap on the device:

  * admission by footprint: a batch starts only if the device bytes of all
    batches in flight plus its own (workspace + outputs, from
    bfs_workspace_size) fit the budget; otherwise it waits - nothing is
    rejected unless a single query can never fit;
  * continuous batching: whenever a worker frees up it takes the oldest waiting
    query and every other waiting query on the same graph (up to max_batch), so
    queries that arrived while others ran join the next batch;
  * a batch of several queries on one graph runs as one multi-source search
    (64 sources per mask word, push or pull per level from the learned
    direction network) when the graph is shallow enough for that to pay,
    otherwise as claim-word searches in lockstep (one launch per level for
    the whole batch); a single query runs alone with its graph's fastest form.

Every query's result is the search's own (level, parent): the same bits alone
or in any mix (tested).  Latency = completion time - arrival time.

The Scheduler holds no device state, so the CPU tests drive it with a
simulated clock and a fake executor.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Query:
    qid: int
    graph: str
    source: int
    arrival: float
    start: float = -1.0
    done: float = -1.0
    error: Optional[str] = None
    result: object = None


@dataclasses.dataclass
class Batch:
    graph: str
    queries: List[Query]
    bytes: int
    worker: int = -1


class Scheduler:
    """Admission and batching decisions; no threads, no device."""

    def __init__(self, footprint: Callable[[str, int], int], budget_bytes: int, max_batch: int = 64):
        self.footprint = footprint
        self.budget = int(budget_bytes)
        self.max_batch = int(max_batch)
        self.waiting: "collections.OrderedDict[int, Query]" = collections.OrderedDict()
        self.in_flight_bytes = 0
        self.peak_bytes = 0
        self.rejected: List[Query] = []

    def submit(self, q: Query) -> None:
        if self.footprint(q.graph, 1) > self.budget:
            q.error = "query can never fit the memory budget"
            self.rejected.append(q)
            return
        self.waiting[q.qid] = q

    def next_batch(self, now: float) -> Optional[Batch]:
        """The oldest waiting query plus the waiting queries on its graph, as many
        as fit the budget (at least the oldest, or nothing if even that does not)."""
        if not self.waiting:
            return None
        head = next(iter(self.waiting.values()))
        same = [q for q in self.waiting.values() if q.graph == head.graph][: self.max_batch]
        take = len(same)
        while take >= 1 and self.in_flight_bytes + self.footprint(head.graph, take) > self.budget:
            take -= 1
        if take == 0:
            return None
        chosen = same[:take]
        for q in chosen:
            del self.waiting[q.qid]
            q.start = now
        b = Batch(head.graph, chosen, self.footprint(head.graph, take))
        self.in_flight_bytes += b.bytes
        self.peak_bytes = max(self.peak_bytes, self.in_flight_bytes)
        return b

    def complete(self, b: Batch, now: float, error: Optional[str] = None) -> None:
        self.in_flight_bytes -= b.bytes
        for q in b.queries:
            q.done = now
            q.error = error


def poisson_arrivals(rate_qps: float, count: int, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_qps, count))


def latency_stats(queries: Sequence[Query]) -> Dict[str, float]:
    """Latency percentiles over the completed queries (NaN when none completed;
    failed queries are counted, never timed)."""
    ok = [q for q in queries if q.error is None and q.done >= 0]
    if not ok:
        nan = float("nan")
        return dict(completed=0, failed=len(queries), p50_ms=nan, p99_ms=nan, mean_ms=nan)
    lat = np.array([q.done - q.arrival for q in ok])
    return dict(completed=len(ok), failed=len(queries) - len(ok),
                p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                mean_ms=float(lat.mean() * 1e3))


def simulate(sched: Scheduler, queries: Sequence[Query], workers: int,
             duration: Callable[[Batch], float], run: Optional[Callable[[Batch], None]] = None) -> None:
    """Discrete-event run of the scheduler with a simulated clock (no device):
    `duration(batch)` gives each batch's service time, `run(batch)` (optional)
    computes results and may raise to fail the batch."""
    import heapq
    events = []                                   # (time, order, kind, payload)
    order = 0
    for q in queries:
        heapq.heappush(events, (q.arrival, order, "arrive", q))
        order += 1
    free = list(range(workers))
    while events:
        now, _, kind, payload = heapq.heappop(events)
        if kind == "arrive":
            sched.submit(payload)
        else:
            b, w = payload
            err = None
            if run is not None:
                try:
                    run(b)
                except Exception as e:            # a failed batch fails its queries only
                    err = f"{type(e).__name__}: {e}"
            sched.complete(b, now, err)
            free.append(w)
        while free:
            b = sched.next_batch(now)
            if b is None:
                break
            w = free.pop()
            b.worker = w
            heapq.heappush(events, (now + duration(b), order, "done", (b, w)))
            order += 1


# ---- the device side ----------------------------------------------------------------------

class GpuExecutor:
    """Runs batches on resident graphs through the library (one stream per worker)."""

    def __init__(self, graphs: Dict[str, object], mode: str = "batched", selector=None,
                 multi_source_max_n: int = 1 << 23, keep_results: bool = False,
                 params: Optional[Dict[str, Dict]] = None, shallow: Optional[Dict[str, bool]] = None,
                 ms_selector=None):
        import torch
        import paper_1906_03113_amd as P
        self.P = P
        self.torch = torch
        self.graphs = graphs
        self.mode = mode                       # "plain": push only, one query at a time
        self.selector = selector               # single-source per-level variant network
        self.ms_selector = ms_selector         # multi-source per-level direction network
        self.ms_max_n = multi_source_max_n
        self.keep = keep_results
        self.params = params or {}             # per-graph launch parameters (autotuned)
        # graphs whose searches take few levels: their batches run as one
        # multi-source search (which reads the frontier size back every level)
        self.shallow = shallow if shallow is not None else {k: True for k in graphs}
        self.local = threading.local()

    def multi_source(self, gname: str, nq: int) -> bool:
        G = self.graphs[gname]
        return (self.mode != "plain" and nq > 1 and G.n <= self.ms_max_n
                and self.shallow.get(gname, False))

    def claim_batch(self, gname: str, nq: int) -> bool:
        """A batch on a deep graph (more than 64 levels): its searches as
        claim-word searches in lockstep, one launch per level for all."""
        return self.mode != "plain" and nq > 1 and not self.shallow.get(gname, False)

    def footprint(self, gname: str, nq: int) -> int:
        G = self.graphs[gname]
        if self.claim_batch(gname, nq):
            ws = G.workspace_size(nq, claim=True)
        else:
            ws = G.workspace_size(nq if self.multi_source(gname, nq) else 1)
        return int(ws) + 8 * G.n * nq

    def _stream(self):
        if not hasattr(self.local, "stream"):
            self.local.stream = self.torch.cuda.Stream()
        return self.local.stream

    def run(self, b: Batch) -> None:
        torch, P = self.torch, self.P
        G = self.graphs[b.graph]
        s = self._stream()
        srcs = [q.source for q in b.queries]
        with torch.cuda.stream(s):
            if self.mode == "plain":
                outs = [P.bfs(G, src, variant="push", stream=s) for src in srcs]
            elif self.multi_source(b.graph, len(srcs)):
                kw = dict(variant="learned", selector=self.ms_selector) if self.ms_selector is not None \
                    else dict(variant="heuristic")
                lv, pa = P.bfs_batch(G, srcs, stream=s, **kw)
                outs = list(zip(lv, pa))
            elif self.claim_batch(b.graph, len(srcs)):
                lv, pa = P.bfs_batch(G, srcs, stream=s, variant="push", push_impl="claim")
                outs = list(zip(lv, pa))
            else:
                kw = dict(variant="learned", selector=self.selector) if self.selector is not None \
                    else dict(variant="heuristic")
                kw.update(self.params.get(b.graph, {}))
                outs = [P.bfs(G, src, stream=s, **kw) for src in srcs]
            s.synchronize()
        for q, o in zip(b.queries, outs):
            q.result = o if self.keep else None


class Server:
    """Worker threads around a Scheduler; submit() from any thread."""

    def __init__(self, executor: GpuExecutor, budget_bytes: int, workers: int = 4, max_batch: int = 64):
        self.ex = executor
        self.sched = Scheduler(executor.footprint, budget_bytes, max_batch)
        self.cv = threading.Condition()
        self.stop = False
        self.t0 = time.perf_counter()
        self.threads = [threading.Thread(target=self._work, args=(w,), daemon=True) for w in range(workers)]
        for t in self.threads:
            t.start()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, q: Query) -> None:
        with self.cv:
            self.sched.submit(q)
            self.cv.notify()

    def _work(self, w: int) -> None:
        while True:
            with self.cv:
                b = None
                while not self.stop:
                    b = self.sched.next_batch(self.now())
                    if b is not None:
                        break
                    self.cv.wait(0.002)
                if b is None:
                    return
            b.worker = w
            err = None
            try:
                self.ex.run(b)
            except Exception as e:
                err = f"{type(e).__name__}: {e}"
            with self.cv:
                self.sched.complete(b, self.now(), err)
                self.cv.notify_all()

    def drain(self, queries: Sequence[Query], timeout: float = 600.0) -> None:
        end = time.perf_counter() + timeout
        with self.cv:
            while any(q.done < 0 and q.error is None for q in queries):
                if time.perf_counter() > end:
                    raise TimeoutError("queries did not finish")
                self.cv.wait(0.01)

    def close(self) -> None:
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()


def run_load(executor: GpuExecutor, graph_names: Sequence[str], sources: Dict[str, np.ndarray],
             rate_qps: float, count: int, seed: int, budget_bytes: int, workers: int,
             max_batch: int = 64, progress=None) -> Dict[str, float]:
    """Poisson arrivals at rate_qps, graph uniform, source uniform among the graph's
    candidate sources; returns latency percentiles and throughput.  `progress`
    (optional) is called with a line every 500 submitted queries."""
    rng = np.random.default_rng(seed)
    arr = poisson_arrivals(rate_qps, count, seed)
    qs = []
    for i, t in enumerate(arr):
        gname = graph_names[int(rng.integers(len(graph_names)))]
        src = int(sources[gname][int(rng.integers(len(sources[gname])))])
        qs.append(Query(i, gname, src, float(t)))
    srv = Server(executor, budget_bytes, workers, max_batch)
    try:
        t_start = srv.now()
        for q in qs:
            delay = q.arrival - (srv.now() - t_start)
            if delay > 0:
                time.sleep(delay)
            q.arrival = srv.now()
            srv.submit(q)
            if progress and (q.qid + 1) % 500 == 0:
                progress(f"[serve]   {q.qid + 1}/{count} queries submitted at {rate_qps:.1f} q/s")
        srv.drain(qs)
        wall = srv.now() - t_start
    finally:
        srv.close()
    st = latency_stats(qs)
    st.update(rate_qps=rate_qps, queries=count, wall_s=wall, achieved_qps=st["completed"] / wall,
              peak_inflight_mb=srv.sched.peak_bytes / 1e6)
    fams = sorted({family(q.graph) for q in qs})
    st["by_family"] = {f: latency_stats([q for q in qs if family(q.graph) == f]) for f in fams}
    return st


def family(name: str) -> str:
    """Graph family of a resident graph's name ("rmat20_1" -> "rmat20")."""
    return name.split("_")[0]


# ---- the serving experiment ---------------------------------------------------------------

def resident_set(which: str = "small"):
    """(name -> graph builder).  "full": R-MAT undirected s16-s21 x 3 seeds, s22 x 2,
    grids 512^2-4096^2 x 3 seeds (32 graphs); "small": one of each up to s20 / 1024^2."""
    import graphgen
    out = {}
    if which == "full":
        for sc in range(16, 22):
            for sd in range(3):
                out[f"rmat{sc}_{sd}"] = (lambda sc=sc, sd=sd: graphgen.rmat(sc, 16, 500 + 10 * sc + sd))
        for sd in range(2):
            out[f"rmat22_{sd}"] = (lambda sd=sd: graphgen.rmat(22, 16, 600 + sd))
        for w in (512, 1024, 2048, 4096):
            for sd in range(3):
                out[f"grid{w}_{sd}"] = (lambda w=w, sd=sd: graphgen.grid(w, 0.9, 700 + sd))
    else:
        for sc in (16, 18, 20):
            out[f"rmat{sc}"] = (lambda sc=sc: graphgen.rmat(sc, 16, 500 + sc))
        for w in (512, 1024):
            out[f"grid{w}"] = (lambda w=w: graphgen.grid(w, 0.9, 700 + w))
    return out


def launch_params(Gs: Dict[str, object], srcs: Dict[str, np.ndarray], selector):
    """Per-graph launch parameters for the serving path, from probe searches on
    each graph: the autotuner's cached choice for the graph's shape if there is
    one, else by diameter class (deep graphs read the frontier size back every
    64 levels instead of every 4); then the faster, on the probe source, of the
    learned per-level form, plain push and the claim-word push (on graphs
    thousands of levels deep the per-level decision costs more than it saves,
    and the claim-word form's lighter levels win).  Also whether the graph is
    shallow (at most 64 levels), which lets its batches run as one
    multi-source search."""
    import torch
    import paper_1906_03113_amd as P
    from . import autotune as AT
    out, shallow = {}, {}
    for name, G in Gs.items():
        s = int(srcs[name][0])
        info = {}
        P.bfs(G, s, variant="learned", selector=selector, info=info)
        levels = int(info["levels"])
        kw = AT.lookup(G, levels)
        kw.pop("loop", None)                   # serving keeps the host loop (no per-query capture)
        if levels > 64:
            kw.setdefault("levels_per_sync", 64)
        best, best_t = None, float("inf")
        for form in (dict(variant="learned", selector=selector), dict(variant="push"),
                     dict(variant="push", push_impl="claim")):
            run = dict(kw, **form)
            P.bfs(G, s, **run)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            P.bfs(G, s, **run)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            if t < best_t:
                best, best_t = form, t
        kw.update(best)
        out[name] = kw
        shallow[name] = levels <= 64
    return out, shallow


def experiment(which="small", queries=400, rates=(0.25, 0.5, 0.8, 0.95), workers=4, seed=5,
               log=None, budget_bytes=64 << 30, seconds=None):
    """Plain (push only, one query at a time) vs batched + learned at fixed
    fractions of the plain path's saturation rate; returns a dict of results.
    Each rate and path serves `queries` Poisson arrivals, or with `seconds`
    set, those arriving within that many seconds (at most `queries`, at least 40)."""
    from concurrent.futures import ThreadPoolExecutor
    import torch
    import paper_1906_03113_amd as P
    from . import selector as S
    torch.cuda.init()
    Gs, srcs = {}, {}
    builders = resident_set(which)
    # the graphs are generated on host threads (the generator's array work
    # releases the interpreter lock) and uploaded one at a time
    with ThreadPoolExecutor(8) as ex:
        futs = {name: ex.submit(build) for name, build in builders.items()}
        for name in builders:
            g = futs.pop(name).result()
            Gs[name] = P.Graph.from_graphgen(g)
            srcs[name] = np.nonzero(g.out_degree() > 0)[0]
            if log:
                log(f"[serve] resident {name}: n={g.n} nnz={g.nnz}")
            del g
    names = sorted(Gs)
    sel = S.load_weights()
    ms_sel = S.load_weights(S.MS_WEIGHTS)
    params, shallow = launch_params(Gs, srcs, sel)
    plain = GpuExecutor(Gs, mode="plain")
    fast = GpuExecutor(Gs, mode="batched", selector=sel, params=params, shallow=shallow, ms_selector=ms_sel)
    # saturation of the plain path: back-to-back queries, one worker
    rng = np.random.default_rng(seed)
    warm = [Query(i, names[int(rng.integers(len(names)))], 0, 0.0) for i in range(len(names))]
    for q in warm:
        q.source = int(srcs[q.graph][0])
        plain.run(Batch(q.graph, [q], 0))
        fast.run(Batch(q.graph, [q], 0))
    sat_q = [Query(i, names[int(rng.integers(len(names)))], 0, 0.0) for i in range(max(40, queries // 4))]
    for q in sat_q:
        q.source = int(srcs[q.graph][int(rng.integers(len(srcs[q.graph])))])
    t0 = time.perf_counter()
    for q in sat_q:
        plain.run(Batch(q.graph, [q], 0))
    sat_qps = len(sat_q) / (time.perf_counter() - t0)
    if log:
        log(f"[serve] plain saturation: {sat_qps:.1f} queries/s")
    res = {"saturation_qps_plain": sat_qps, "graphs": names, "rates": {}}
    for frac in rates:
        rate = frac * sat_qps
        count = queries if seconds is None else max(40, min(queries, int(rate * seconds)))
        r_plain = run_load(plain, names, srcs, rate, count, seed, budget_bytes, workers=1, max_batch=1,
                           progress=log)
        r_fast = run_load(fast, names, srcs, rate, count, seed, budget_bytes, workers=workers,
                          progress=log)
        res["rates"][str(frac)] = {"plain": r_plain, "batched_learned": r_fast}
        if log:
            log(f"[serve] {frac:.2f} x sat ({rate:.1f} q/s): plain p50 {r_plain['p50_ms']:.2f} ms "
                f"p99 {r_plain['p99_ms']:.2f} ms | batched+learned p50 {r_fast['p50_ms']:.2f} ms "
                f"p99 {r_fast['p99_ms']:.2f} ms")
            for f in r_plain["by_family"]:
                a, b = r_plain["by_family"][f], r_fast["by_family"][f]
                log(f"[serve]    {f:9s} n={a['completed']:4d} plain p50 {a['p50_ms']:8.2f} p99 {a['p99_ms']:8.2f}"
                    f" | batched+learned p50 {b['p50_ms']:8.2f} p99 {b['p99_ms']:8.2f}")
    for G in Gs.values():
        G.close()
    return res


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="Poisson query load: plain vs batched + learned")
    ap.add_argument("--set", default="small", choices=["small", "full"])
    ap.add_argument("--queries", type=int, default=2000)
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--seconds", type=float, default=None,
                    help="serve the arrivals of this many seconds per rate (at most --queries)")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    res = experiment(a.set, a.queries, workers=a.workers, log=log, seconds=a.seconds)
    txt = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt)
    print(txt)


if __name__ == "__main__":
    main()
