"""The serving scheduler on the CPU: a simulated clock and a fake executor (the
oracle) - admission by footprint, continuous batching, failures, latency."""
import numpy as np
import pytest

import graphgen
import oracle
from paper_1906_03113_amd.serve import Batch, Query, Scheduler, latency_stats, poisson_arrivals, simulate


def _fp(per_query=100):
    return lambda g, nq: 50 + per_query * nq


def test_admission_never_exceeds_budget():
    sched = Scheduler(_fp(), budget_bytes=400, max_batch=64)
    qs = [Query(i, f"g{i % 5}", 0, arrival=0.01 * i) for i in range(60)]
    simulate(sched, qs, workers=8, duration=lambda b: 0.05 + 0.01 * len(b.queries))
    assert sched.peak_bytes <= 400
    assert all(q.done > 0 and q.error is None for q in qs)
    assert sched.in_flight_bytes == 0


def test_continuous_batching_joins_later_arrivals():
    sched = Scheduler(_fp(), budget_bytes=10 ** 9)
    qs = [Query(0, "a", 1, 0.0), Query(1, "a", 2, 0.1), Query(2, "b", 3, 0.15),
          Query(3, "a", 4, 0.2), Query(4, "a", 5, 0.3)]
    batches = []
    simulate(sched, qs, workers=1, duration=lambda b: 1.0, run=lambda b: batches.append(
        (b.graph, [q.qid for q in b.queries])))
    # q0 alone; then the oldest waiting (q1, graph a) with every waiting a-query; then b
    assert batches == [("a", [0]), ("a", [1, 3, 4]), ("b", [2])]
    assert qs[4].done == pytest.approx(2.0) and qs[2].done == pytest.approx(3.0)
    st = latency_stats(qs)
    assert st["completed"] == 5 and st["p50_ms"] > 0


def test_batch_shrinks_to_fit_budget_and_oversized_query_is_rejected():
    sched = Scheduler(lambda g, nq: (10 ** 6 if g == "huge" else 100 * nq), budget_bytes=250)
    qs = [Query(i, "a", i, 0.0) for i in range(5)] + [Query(9, "huge", 0, 0.0)]
    seen = []
    simulate(sched, qs, workers=4, duration=lambda b: 1.0, run=lambda b: seen.append(len(b.queries)))
    assert max(seen) <= 2 and sum(seen) == 5
    assert qs[-1].error and "never fit" in qs[-1].error
    assert all(q.error is None for q in qs[:5])


def test_failing_batches_fail_only_their_queries():
    sched = Scheduler(_fp(), budget_bytes=10 ** 9)
    qs = [Query(i, "bad" if i % 3 == 0 else "ok", i, 0.01 * i) for i in range(30)]

    def run(b):
        if b.graph == "bad":
            raise RuntimeError("device error")

    simulate(sched, qs, workers=2, duration=lambda b: 0.02, run=run)
    for q in qs:
        assert (q.error is not None) == (q.graph == "bad")
        assert q.done >= 0
    assert latency_stats(qs)["failed"] == 10


def test_latency_stats_without_completions_are_nan():
    """No completed query: the percentiles are undefined (NaN), never 0 ms."""
    qs = [Query(i, "g", i, 0.0) for i in range(4)]
    for q in qs:
        q.error = "device error"
        q.done = 1.0
    st = latency_stats(qs)
    assert st["completed"] == 0 and st["failed"] == 4
    assert all(np.isnan(st[k]) for k in ("p50_ms", "p99_ms", "mean_ms"))
    assert np.isnan(latency_stats([])["p99_ms"])


def test_poisson_arrivals():
    a = poisson_arrivals(200.0, 20000, seed=5)
    assert np.all(np.diff(a) > 0)
    assert abs(np.mean(np.diff(a)) - 1 / 200.0) < 2e-4
    assert np.array_equal(a, poisson_arrivals(200.0, 20000, seed=5))


def test_results_same_alone_and_in_the_mix():
    """With the oracle as executor, a query's result does not depend on what it
    was batched with (the scheduler only groups; each query keeps its own)."""
    gs = {"er": graphgen.erdos_renyi(500, 4, 1), "path": graphgen.path_graph(80)}
    rng = np.random.default_rng(2)
    qs = [Query(i, ["er", "path"][i % 2], int(rng.integers(0, 80)), 0.001 * i) for i in range(40)]

    def run(b):
        g = gs[b.graph]
        for q in b.queries:
            q.result = oracle.bfs_graph(g, q.source)

    sched = Scheduler(_fp(), budget_bytes=10 ** 9, max_batch=8)
    simulate(sched, qs, workers=3, duration=lambda b: 0.01, run=run)
    for q in qs:
        alone = oracle.bfs_graph(gs[q.graph], q.source)
        assert np.array_equal(q.result[0], alone[0]) and np.array_equal(q.result[1], alone[1])
