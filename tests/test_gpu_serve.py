"""The server on the GPU: queries on several resident graphs arriving together,
served by concurrent workers with batching; every query's result equals the
same search run alone (and the oracle)."""
import numpy as np
import pytest

import graphgen
import oracle
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_results_alone_equal_results_in_the_mix(mode):
    P = need_gpu()
    import torch
    from paper_1906_03113_amd import selector as S
    from paper_1906_03113_amd.serve import GpuExecutor, Query, Server
    gens = {"rmat13": graphgen.rmat(13, 16, 31), "rmatd12": graphgen.rmat(12, 16, 32, directed=True),
            "grid64": graphgen.grid(64, 0.9, 33), "er3000": graphgen.erdos_renyi(3000, 5, 34)}
    Gs = {k: P.Graph.from_graphgen(g) for k, g in gens.items()}
    sel = S.load_weights() if mode == "batched" else None
    ex = GpuExecutor(Gs, mode=mode, selector=sel, keep_results=True)
    rng = np.random.default_rng(7)
    names = sorted(gens)
    qs = []
    for i in range(96):
        gname = names[int(rng.integers(len(names)))]
        src = int(rng.integers(gens[gname].n))
        qs.append(Query(i, gname, src, 0.0))
    say(f"[serve] {mode}: 96 queries, 3 workers")
    srv = Server(ex, budget_bytes=8 << 30, workers=3, max_batch=8)
    try:
        for q in qs:
            srv.submit(q)
        srv.drain(qs, timeout=300)
    finally:
        srv.close()
    assert all(q.error is None for q in qs), [q.error for q in qs if q.error][:3]
    torch.cuda.synchronize()
    for q in qs:
        lv, pa = q.result
        lv, pa = lv.cpu().numpy(), pa.cpu().numpy()
        al, ap = P.bfs(Gs[q.graph], q.source)
        torch.cuda.synchronize()
        assert np.array_equal(lv, al.cpu().numpy()) and np.array_equal(pa, ap.cpu().numpy()), q.qid
        if q.qid % 8 == 0:
            wl, wp = oracle.bfs_graph(gens[q.graph], q.source)
            assert np.array_equal(lv, wl) and np.array_equal(pa, wp)
