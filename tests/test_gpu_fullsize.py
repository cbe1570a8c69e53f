"""Parity at the full workload sizes: R-MAT scale 22 (undirected), the 4096^2
percolated grid (thousands of levels) and R-MAT scale 20 (directed), each in
the launch configurations bench.py times; the batching workloads (256
sources in one call, the 64-graph ER pack); the comparison searches and the
masked SpMSpV primitive.  Whole arrays are compared with the oracle (it
finishes in about a second per search at these sizes)."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import certify
from tests.gpu_common import check_all, compare_all, need_gpu, oracle_all, run_gpu, say

pytestmark = pytest.mark.gpu


def _check(g, s, got, tag, cert=False):
    lv, pa = got
    wl, wp = oracle.bfs_graph(g, int(s))
    assert np.array_equal(lv, wl), f"{tag}: level differs at {np.count_nonzero(lv != wl)} vertices"
    assert np.array_equal(pa, wp), f"{tag}: parent differs at {np.count_nonzero(pa != wp)} vertices"
    if cert:
        assert certify.check(g.n, g.ptr, g.idx, int(s), lv, pa) == [], tag


def test_rmat22():
    P = need_gpu()
    from paper_1906_03113_amd import selector as S
    g = graphgen.workload("rmat22")
    G = P.Graph.from_graphgen(g)
    w = S.load_weights()
    src = graphgen.pick_sources(g, 64, 22)
    for i, s in enumerate(src[:2]):
        for kw in (dict(variant="push"), dict(variant="learned", selector=w, loop="graph", levels_per_sync=8),
                   dict(variant="pull"), dict(variant="bitmap"), dict(variant="short_circuit")):
            say(f"[full] rmat22 s={s} {kw.get('variant')}")
            _check(g, s, run_gpu(P, G, s, **kw), f"rmat22/{s}/{kw.get('variant')}", cert=(i == 0 and kw["variant"] == "push"))


def test_rmat22_plain_push_every_source():
    """The plain push as bench.py times it (the sliced form, host loop), from
    every one of the 64 sources, and the list form from the first 8: whole
    arrays against the oracle."""
    P = need_gpu()
    import torch
    g = graphgen.workload("rmat22")
    G = P.Graph.from_graphgen(g)
    src = [int(s) for s in graphgen.pick_sources(g, 64, 22)]
    say("[full] rmat22 oracle from the 64 sources (host threads)")
    want = oracle_all(g, src)
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
    ws = P.Workspace(G.workspace_size(1))

    def run(q, impl):
        P.bfs(G, src[q], level=lv, parent=pa, workspace=ws, variant="push", push_impl=impl)
        torch.cuda.synchronize()
        return lv.cpu().numpy(), pa.cpu().numpy()

    say("[full] rmat22 sliced push x64")
    compare_all(want, src, lambda q: run(q, "sliced"), "rmat22 sliced push")
    say("[full] rmat22 list push x8")
    compare_all(want[:8], src[:8], lambda q: run(q, "list"), "rmat22 list push")


def test_rmat22_batch_of_64():
    """All 64 sources in one call, every query against the oracle: per-source
    and vertex-major results, every direction threshold bench.py chooses
    between (pull from n >> 5, 9, 11, 13 on) and push on every level."""
    P = need_gpu()
    import torch
    g = graphgen.workload("rmat22")
    G = P.Graph.from_graphgen(g)
    src = [int(s) for s in graphgen.pick_sources(g, 64, 22)]
    lv = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in src]
    pa = [torch.empty(g.n, dtype=torch.int32, device="cuda") for _ in src]
    vl = torch.empty((g.n, 64), dtype=torch.int32, device="cuda")
    vp = torch.empty((g.n, 64), dtype=torch.int32, device="cuda")
    say("[full] rmat22 oracle from the 64 sources (host threads)")
    want = oracle_all(g, src)
    from paper_1906_03113_amd import selector as S
    msw = S.load_weights(S.MS_WEIGHTS)
    for kw in (dict(variant="learned", selector=msw),            # the bench's headline call
               dict(variant="heuristic", ms_pull_shift=5), dict(variant="heuristic", ms_pull_shift=9),
               dict(variant="heuristic", ms_pull_shift=11), dict(variant="heuristic", ms_pull_shift=13),
               dict(variant="push")):
        say(f"[full] rmat22 multi-source x64 {kw.get('variant')} {kw.get('ms_pull_shift', '')}")
        P.bfs_batch(G, src, levels=lv, parents=pa, **kw)
        P.bfs_batch_vm(G, src, level=vl, parent=vp, **kw)
        torch.cuda.synchronize()
        compare_all(want, src, lambda q: (lv[q].cpu().numpy(), pa[q].cpu().numpy()), f"rmat22 batch {kw}")
        compare_all(want, src, lambda q: (vl[:, q].cpu().numpy(), vp[:, q].cpu().numpy()), f"rmat22 vm {kw}")


def test_grid4096():
    P = need_gpu()
    from paper_1906_03113_amd import selector as S
    g = graphgen.workload("grid4096")
    G = P.Graph.from_graphgen(g)
    s = int(graphgen.pick_sources(g, 16, 31)[0])
    w = S.load_weights()
    for kw in (dict(variant="push"), dict(variant="learned", selector=w, loop="graph", levels_per_sync=64),
               dict(variant="push", loop="persistent")):
        say(f"[full] grid4096 s={s} {kw}")
        _check(g, s, run_gpu(P, G, s, **{k: v for k, v in kw.items()}), f"grid4096/{kw}")


def test_grid4096_claim_every_source():
    """The 4096^2 grid as bench.py times it: the automatic push form (the
    claim-word push here) from all 16 sources, and the 16 sources in one
    batched + learned call; every query against the oracle."""
    P = need_gpu()
    import torch
    from paper_1906_03113_amd import selector as S
    g = graphgen.workload("grid4096")
    G = P.Graph.from_graphgen(g)
    src = [int(s) for s in graphgen.pick_sources(g, 16, 31)]
    say("[full] grid4096 oracle from the 16 sources (host threads)")
    want = oracle_all(g, src)
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
    ws = P.Workspace(G.workspace_size(1))

    def run(q):
        P.bfs(G, src[q], level=lv, parent=pa, workspace=ws)
        torch.cuda.synchronize()
        return lv.cpu().numpy(), pa.cpu().numpy()
    say("[full] grid4096 automatic push x16")
    compare_all(want, src, run, "grid4096 auto push")
    del ws
    say("[full] grid4096 batched + learned x16")
    bl, bp = P.bfs_batch(G, src, variant="learned", selector=S.load_weights(S.MS_WEIGHTS))
    torch.cuda.synchronize()
    compare_all(want, src, lambda q: (bl[q].cpu().numpy(), bp[q].cpu().numpy()), "grid4096 batch")


def test_rmat20_directed():
    P = need_gpu()
    from paper_1906_03113_amd import selector as S
    g = graphgen.workload("rmat20d")
    G = P.Graph.from_graphgen(g)
    w = S.load_weights()
    for i, s in enumerate(graphgen.pick_sources(g, 16, 32)[:2]):
        for kw in (dict(variant="push"), dict(variant="learned", selector=w, loop="graph", levels_per_sync=8),
                   dict(variant="pull"), dict(variant="short_circuit")):
            say(f"[full] rmat20d s={s} {kw.get('variant')}")
            _check(g, s, run_gpu(P, G, s, **kw), f"rmat20d/{s}", cert=(i == 0))


def test_compare_full_size():
    """The comparison searches at full size: R-MAT s22 (SpMV-BFS, SpMmSpV-BFS)
    and directed R-MAT s20 (all three); level / parent against the oracle, the
    operation counts against the oracle's step-by-step counts."""
    P = need_gpu()
    import torch
    from oracle import compare as C
    for name, methods in (("rmat22", ("spmv", "spmmspv")), ("rmat20d", ("spmv", "spmspv", "spmmspv"))):
        g = graphgen.workload(name)
        G = P.Graph.from_graphgen(g)
        s = int(graphgen.pick_sources(g, 1, 22)[0])
        for m in methods:
            say(f"[full] compare {name} s={s} {m}")
            lv, pa, ops, steps = P.bfs_compare(G, s, m)
            torch.cuda.synchronize()
            _check(g, s, (lv.cpu().numpy(), pa.cpu().numpy()), f"{name}/compare/{m}")
            _, _, wops, wsteps = C.run(g, s, m, ops_only=True)
            assert (ops, steps) == (wops, wsteps), (name, m)
        G.close()


def test_masked_spmspv_full_size():
    """Theorem 1 at full size through the masked SpMSpV primitive: on R-MAT
    s22, for every level k of the oracle's search, the (min, select) product of
    x = F_k (x(j) = j) under the complemented mask of the rows visited through
    level k has the support {v : level[v] = k + 1} and the values parent[v]."""
    P = need_gpu()
    import torch
    g = graphgen.workload("rmat22")
    G = P.Graph.from_graphgen(g)
    s = int(graphgen.pick_sources(g, 64, 22)[0])
    wl, wp = oracle.bfs_graph(g, s)
    ws = P.Workspace(P.spmspv_workspace_size(G, int((wl >= 0).sum())))
    ws.buf.zero_()
    for k in range(int(wl.max()) + 1):
        front = np.nonzero(wl == k)[0].astype(np.int32)
        seen = (wl >= 0) & (wl <= k)
        words = np.zeros((g.n + 31) // 32, np.uint32)
        idx = np.nonzero(seen)[0]
        np.bitwise_or.at(words, idx >> 5, (np.uint32(1) << (idx & 31).astype(np.uint32)))
        say(f"[full] spmspv rmat22 level {k} |x|={len(front)}")
        yi, yv = P.masked_spmspv(G, "min_select", torch.from_numpy(front).cuda(),
                                 torch.from_numpy(front.astype(np.int64)).cuda(),
                                 torch.from_numpy(words.view(np.int32)).cuda(), None, True, workspace=ws)
        torch.cuda.synchronize()
        want = np.nonzero(wl == k + 1)[0]
        assert np.array_equal(yi.cpu().numpy(), want), k
        assert np.array_equal(yv.cpu().numpy(), wp[want].astype(np.int64)), k
    G.close()


def test_rmat20d_batch_of_256():
    """256 sources in one call on directed R-MAT s20 (4 mask words per vertex),
    the launch the batching measurement times; every query against the oracle."""
    P = need_gpu()
    import torch
    g = graphgen.workload("rmat20d")
    G = P.Graph.from_graphgen(g)
    src = [int(s) for s in graphgen.pick_sources(g, 256, 41)]
    say("[full] rmat20d multi-source x256")
    lv, pa = P.bfs_batch(G, src, variant="heuristic")
    torch.cuda.synchronize()
    check_all(g, src, lambda q: (lv[q].cpu().numpy(), pa[q].cpu().numpy()), "rmat20d batch")


def test_er_pack_of_64_graphs():
    """The 64 uneven ER graphs packed block-diagonally, one root per block, as
    one persistent launch and as the graph loop: every block against the
    oracle's search of its own graph."""
    P = need_gpu()
    import torch
    gs = graphgen.er_family(count=64, lo=10, hi=18, dmin=4, dmax=32)
    packed, offs = graphgen.block_diagonal(gs)
    G = P.Graph.from_graphgen(packed)
    roots = []
    for b, g in enumerate(gs):
        nz = np.nonzero(g.out_degree() > 0)[0]
        roots.append(int(offs[b] + (nz[0] if len(nz) else 0)))
    want = [oracle.bfs_graph(g, roots[b] - int(offs[b])) for b, g in enumerate(gs)]
    say("[full] ER x64 as one call over different graphs")
    Gs = [P.Graph.from_graphgen(g) for g in gs]
    ml, mp = P.bfs_batch(Gs, [roots[b] - int(offs[b]) for b in range(len(gs))])
    torch.cuda.synchronize()
    for b in range(len(gs)):
        wl, wp = want[b]
        assert np.array_equal(ml[b].cpu().numpy(), wl), ("mixed", b)
        assert np.array_equal(mp[b].cpu().numpy(), wp), ("mixed", b)
    for loop in ("persistent", "graph"):
        say(f"[full] ER pack x64 loop={loop}")
        lv, pa = P.bfs_roots(G, roots, loop=loop)
        torch.cuda.synchronize()
        lv, pa = lv.cpu().numpy(), pa.cpu().numpy()
        for b in range(len(gs)):
            o0, o1 = int(offs[b]), int(offs[b + 1])
            wl, wp = want[b]
            assert np.array_equal(lv[o0:o1], wl), (loop, b)
            assert np.array_equal(pa[o0:o1], np.where(wp >= 0, wp + o0, -1)), (loop, b)
