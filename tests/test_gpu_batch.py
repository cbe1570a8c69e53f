"""GPU parity of the batched entry points: many sources on one graph (64 per
mask word), many graphs per call, and block-diagonal packs searched from one
root per block.  Every result equals the single-source oracle bit for bit."""
import numpy as np
import pytest

import graphgen
import oracle
from tests.gpu_common import assert_same, check_all, compare_all, need_gpu, oracle_all, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    return need_gpu()


@pytest.mark.parametrize("variant", ["push", "pull", "heuristic"])
@pytest.mark.parametrize("name,nq", [("er", 1), ("er", 2), ("rmat", 64), ("rmat", 65),
                                     ("rmatd", 130), ("grid", 63)])
def test_multi_source_equals_single(P, name, nq, variant):
    import torch
    g = {"er": lambda: graphgen.erdos_renyi(5000, 6, 11),
         "rmat": lambda: graphgen.rmat(13, 16, 12),
         "rmatd": lambda: graphgen.rmat(12, 16, 13, directed=True),
         "grid": lambda: graphgen.grid(60, 0.85, 14)}[name]()
    G = P.Graph.from_graphgen(g)
    rng = np.random.default_rng(nq)
    cand = np.nonzero(g.out_degree() > 0)[0]
    src = rng.choice(cand, size=nq, replace=True)          # duplicates allowed
    if nq > 2:
        src[1] = src[0]
        src[-1] = int(np.nonzero(g.out_degree() == 0)[0][0]) if np.any(g.out_degree() == 0) else src[-1]
    say(f"[batch] {name} nq={nq} {variant}")
    lv, pa = P.bfs_batch(G, [int(s) for s in src], variant=variant)
    torch.cuda.synchronize()
    for q, s in enumerate(src):
        assert_same(g, int(s), (lv[q].cpu().numpy(), pa[q].cpu().numpy()), f"{name}/q{q}/s{s}")


def test_batch_over_different_graphs(P):
    import torch
    gs = [graphgen.erdos_renyi(800 + 37 * i, 4 + i, 20 + i) for i in range(4)]
    Gs = [P.Graph.from_graphgen(g) for g in gs]
    srcs = [int(graphgen.pick_sources(g, 1, 3)[0]) for g in gs]
    say("[batch] 4 different graphs")
    lv, pa = P.bfs_batch(Gs, srcs)
    torch.cuda.synchronize()
    for g, s, l, p in zip(gs, srcs, lv, pa):
        assert_same(g, s, (l.cpu().numpy(), p.cpu().numpy()), "multi-graph")


def test_block_diagonal_uneven_graphs(P):
    """Uneven ER graphs packed block-diagonally, one root per block, one search."""
    import torch
    gs = graphgen.er_family(count=12, lo=6, hi=12)
    packed, offs = graphgen.block_diagonal(gs)
    G = P.Graph.from_graphgen(packed)
    roots = []
    for b, g in enumerate(gs):
        nz = np.nonzero(g.out_degree() > 0)[0]
        roots.append(int(offs[b] + (nz[0] if len(nz) else 0)))
    for loop, variant in (("host", "push"), ("persistent", "push"), ("host", "short_circuit"),
                          ("graph", "short_circuit")):
        say(f"[batch] block-diagonal x{len(gs)} loop={loop} variant={variant}")
        lv, pa = P.bfs_roots(G, roots, loop=loop, variant=variant)
        torch.cuda.synchronize()
        lv, pa = lv.cpu().numpy(), pa.cpu().numpy()
        for b, g in enumerate(gs):
            o0, o1 = int(offs[b]), int(offs[b + 1])
            wl, wp = oracle.bfs_graph(g, roots[b] - o0)
            assert np.array_equal(lv[o0:o1], wl)
            assert np.array_equal(pa[o0:o1], np.where(wp >= 0, wp + o0, -1))


@pytest.mark.parametrize("variant", ["push", "pull", "heuristic"])
@pytest.mark.parametrize("name,nq", [("er", 1), ("rmat", 64), ("rmatd", 130), ("grid", 63)])
def test_vertex_major_batch(P, name, nq, variant):
    """The multi-source batch with [n][ld] results: column q equals source
    q's single-source oracle; columns past the sources hold -1."""
    import torch
    g = {"er": lambda: graphgen.erdos_renyi(5000, 6, 31),
         "rmat": lambda: graphgen.rmat(13, 16, 32),
         "rmatd": lambda: graphgen.rmat(12, 16, 33, directed=True),
         "grid": lambda: graphgen.grid(60, 0.85, 34)}[name]()
    G = P.Graph.from_graphgen(g)
    rng = np.random.default_rng(100 + nq)
    cand = np.nonzero(g.out_degree() > 0)[0]
    src = rng.choice(cand, size=nq, replace=True)
    if nq > 2:
        src[1] = src[0]
    ld = 64 * ((nq + 63) // 64)
    say(f"[batch-vm] {name} nq={nq} {variant}")
    lv, pa = P.bfs_batch_vm(G, [int(s) for s in src], variant=variant)
    torch.cuda.synchronize()
    assert tuple(lv.shape) == (g.n, ld) and tuple(pa.shape) == (g.n, ld)
    lv, pa = lv.cpu().numpy(), pa.cpu().numpy()
    for q, s in enumerate(src):
        assert_same(g, int(s), (lv[:, q].copy(), pa[:, q].copy()), f"{name}/q{q}/s{s}")
    assert np.all(lv[:, nq:] == -1) and np.all(pa[:, nq:] == -1)


def test_vertex_major_reuses_outputs(P):
    """Two calls into the same arrays and workspace, the second with fewer
    sources in the same 64-column word: nothing of the first call survives."""
    import torch
    g = graphgen.rmat(12, 16, 41)
    G = P.Graph.from_graphgen(g)
    cand = np.nonzero(g.out_degree() > 0)[0]
    a = [int(s) for s in cand[:40]]
    b = [int(s) for s in cand[100:117]]
    lv = torch.empty((g.n, 64), dtype=torch.int32, device="cuda")
    pa = torch.empty((g.n, 64), dtype=torch.int32, device="cuda")
    ws = P.Workspace(P.batch_vm_workspace_size(G, 40))
    say("[batch-vm] reuse 40 then 17 sources")
    P.bfs_batch_vm(G, a, level=lv, parent=pa, workspace=ws)
    P.bfs_batch_vm(G, b, level=lv, parent=pa, workspace=ws)
    torch.cuda.synchronize()
    l, p = lv.cpu().numpy(), pa.cpu().numpy()
    for q, s in enumerate(b):
        assert_same(g, s, (l[:, q].copy(), p[:, q].copy()), f"reuse/q{q}")
    assert np.all(l[:, len(b):] == -1) and np.all(p[:, len(b):] == -1)


@pytest.mark.parametrize("name", ["rmat", "grid"])
def test_ms_pull_shift_never_changes_results(P, name):
    """The multi-source direction threshold (all push at 31 ... pull from a
    frontier of n/2 at 1) changes no result, in either output layout; a shift
    above 31 is rejected before any work."""
    import torch
    g = {"rmat": lambda: graphgen.rmat(13, 16, 51), "grid": lambda: graphgen.grid(60, 0.85, 52)}[name]()
    G = P.Graph.from_graphgen(g)
    cand = np.nonzero(g.out_degree() > 0)[0]
    src = [int(s) for s in np.random.default_rng(53).choice(cand, size=70, replace=False)]
    want = oracle_all(g, src)
    for sh in (1, 9, 31):
        say(f"[batch] {name} pull shift {sh}")
        lv, pa = P.bfs_batch(G, src, variant="heuristic", ms_pull_shift=sh)
        vl, vp = P.bfs_batch_vm(G, src, variant="heuristic", ms_pull_shift=sh)
        torch.cuda.synchronize()
        compare_all(want, src, lambda q: (lv[q].cpu().numpy(), pa[q].cpu().numpy()), f"{name}/sh{sh}")
        compare_all(want, src, lambda q: (vl[:, q].cpu().numpy(), vp[:, q].cpu().numpy()), f"{name}/sh{sh}/vm")
    with pytest.raises(P.BfsError):
        P.bfs_batch_vm(G, src, variant="heuristic", ms_pull_shift=32)


@pytest.mark.parametrize("name", ["er", "rmat", "grid_deep", "path"])
def test_vertex_major_level_count(P, name):
    """The level count a multi-source call reports is the largest level over
    its sources plus one, also on deep graphs, where push levels are launched
    several at a time and the last group runs past the end of the search."""
    import torch
    g = {"er": lambda: graphgen.erdos_renyi(3000, 5, 61),
         "rmat": lambda: graphgen.rmat(12, 16, 62),
         "grid_deep": lambda: graphgen.grid(40, 0.75, 63),
         "path": lambda: graphgen.path_graph(203)}[name]()
    G = P.Graph.from_graphgen(g)
    cand = np.nonzero(g.out_degree() > 0)[0]
    src = [int(s) for s in np.random.default_rng(64).choice(cand, size=min(40, len(cand)), replace=False)]
    if name == "path":
        src = [0, 101, 202]                  # eccentricities 202, 101, 202
    for variant in ("push", "heuristic"):
        info = {}
        say(f"[batch-vm] level count {name} {variant}")
        lv, pa = P.bfs_batch_vm(G, src, variant=variant, info=info)
        torch.cuda.synchronize()
        l = lv.cpu().numpy()
        want = max(int(oracle.bfs_graph(g, s)[0].max()) for s in src) + 1
        assert info["levels"] == want, (name, variant, info["levels"], want)
        assert int(l[:, :len(src)].max()) + 1 == want
        for q in (0, len(src) - 1):
            assert_same(g, src[q], (l[:, q].copy(), pa[:, q].cpu().numpy().copy()), f"{name}/q{q}")


@pytest.mark.parametrize("grid_blocks", [1, 3])
@pytest.mark.parametrize("name", ["rmat", "rmatd"])
def test_long_rows_split_across_launches(P, name, grid_blocks):
    """A grid small enough that the long rows' later chunks outnumber its
    waves: each long row's first chunk settles what it finds and a second
    launch scans the later chunks for the rest; both output layouts, pull on
    every level, against the oracle."""
    import torch
    g = {"rmat": lambda: graphgen.rmat(14, 16, 71),
         "rmatd": lambda: graphgen.rmat(13, 16, 72, directed=True)}[name]()
    G = P.Graph.from_graphgen(g)
    cand = np.nonzero(g.out_degree() > 0)[0]
    src = [int(s) for s in np.random.default_rng(73).choice(cand, size=70, replace=False)]
    say(f"[batch] {name} long-row split, {grid_blocks} workgroups")
    lv, pa = P.bfs_batch(G, src, variant="pull", grid_blocks=grid_blocks)
    vl, vp = P.bfs_batch_vm(G, src, variant="pull", grid_blocks=grid_blocks)
    torch.cuda.synchronize()
    check_all(g, src, lambda q: (lv[q].cpu().numpy(), pa[q].cpu().numpy()), f"{name}/split")
    check_all(g, src, lambda q: (vl[:, q].cpu().numpy(), vp[:, q].cpu().numpy()), f"{name}/split/vm")


def test_self_loops_multi_source(P):
    """Self-loops at every vertex (the sources included), duplicate entries:
    every multi-source query, both layouts and every direction policy, equals
    the oracle's search of the clean graph."""
    import torch
    clean = graphgen.rmat(12, 8, 81)
    rows = []
    for v in range(clean.n):
        r = list(clean.idx[clean.ptr[v]:clean.ptr[v + 1]])
        rows.append(sorted(r + r[: len(r) // 4] + [v]))
    ptr = np.zeros(clean.n + 1, np.int32)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([x for r in rows for x in r], np.int32)
    G = P.Graph.from_csr(clean.n, ptr, idx)
    cand = np.nonzero(clean.out_degree() > 0)[0]
    src = [int(s) for s in np.random.default_rng(82).choice(cand, size=70, replace=False)]
    want = oracle_all(clean, src)
    for variant in ("push", "pull", "heuristic"):
        say(f"[batch] self-loops at every vertex, {variant}")
        lv, pa = P.bfs_batch(G, src, variant=variant)
        vl, vp = P.bfs_batch_vm(G, src, variant=variant)
        torch.cuda.synchronize()
        compare_all(want, src, lambda q: (lv[q].cpu().numpy(), pa[q].cpu().numpy()), f"loops/{variant}")
        compare_all(want, src, lambda q: (vl[:, q].cpu().numpy(), vp[:, q].cpu().numpy()), f"loops/{variant}/vm")


@pytest.mark.parametrize("name", ["rmat", "rmatd", "grid", "er"])
def test_range_ordered_pull(P, name):
    """Dense pull levels visiting the in-neighbours range by range (2, 3, 7 or
    64 ranges, forced on these small graphs) give every query the oracle's
    result, in both output layouts; with two mask words the option is ignored."""
    import torch
    g = {"rmat": lambda: graphgen.rmat(13, 16, 71),
         "rmatd": lambda: graphgen.rmat(12, 16, 72, directed=True),
         "grid": lambda: graphgen.grid(70, 0.85, 73),
         "er": lambda: graphgen.erdos_renyi(5003, 7, 74)}[name]()
    G = P.Graph.from_graphgen(g)
    cand = np.nonzero(g.out_degree() > 0)[0]
    rng = np.random.default_rng(75)
    for nq in (64, 37, 65):
        src = [int(s) for s in rng.choice(cand, size=nq, replace=True)]
        want = oracle_all(g, src)
        for ranges in (2, 3, 7, 64):
            for variant in ("pull", "heuristic"):
                say(f"[batch] {name} nq={nq} ranges={ranges} {variant}")
                lv, pa = P.bfs_batch(G, src, variant=variant, ms_ranges=ranges, ms_pull_shift=9)
                vl, vp = P.bfs_batch_vm(G, src, variant=variant, ms_ranges=ranges, ms_pull_shift=9)
                torch.cuda.synchronize()
                compare_all(want, src, lambda q: (lv[q].cpu().numpy(), pa[q].cpu().numpy()),
                            f"{name}/{nq}/{ranges}/{variant}")
                compare_all(want, src, lambda q: (vl[:, q].cpu().numpy(), vp[:, q].cpu().numpy()),
                            f"{name}/{nq}/{ranges}/{variant}/vm")
    with pytest.raises(P.BfsError):
        P.bfs_batch(G, src[:3], variant="pull", ms_ranges=65)


@pytest.mark.parametrize("name", ["rmat", "rmat_dup", "grid", "er_isolated", "rmatd"])
def test_degree_ordered_copy(P, name):
    """The multi-source search over the graph's degree-ordered copy (labels by
    descending degree, lists in the caller's order, results and parents in the
    caller's ids): every query of a 70-source batch, both layouts, every
    direction policy, and small grids whose long rows' later chunks get a
    launch of their own (the chunks skip sources settled by earlier chunks by
    comparing caller ids), against the oracle."""
    import torch
    from paper_1906_03113_amd import selector as S
    if name == "rmat":
        g = graphgen.rmat(14, 16, 91)
        ptr, idx = g.ptr, g.idx
    elif name == "rmat_dup":                       # duplicates and self-loops, clean graph for the oracle
        g = graphgen.rmat(12, 16, 92)
        rows = []
        for v in range(g.n):
            r = list(g.idx[g.ptr[v]:g.ptr[v + 1]])
            rows.append(sorted(r + r[: len(r) // 3] + [v]))
        ptr = np.zeros(g.n + 1, np.int32)
        ptr[1:] = np.cumsum([len(r) for r in rows])
        idx = np.array([x for r in rows for x in r], np.int32)
    elif name == "grid":
        g = graphgen.grid(70, 0.9, 93)
        ptr, idx = g.ptr, g.idx
    elif name == "er_isolated":
        g = graphgen.erdos_renyi(20000, 3.0, 94)   # isolated vertices among them
        ptr, idx = g.ptr, g.idx
    else:                                          # directed: an out-list and an in-list copy
        g = graphgen.rmat(13, 16, 96, directed=True)
        ptr, idx = g.ptr, g.idx
    if g.directed:
        G = P.Graph.from_csr(g.n, ptr, idx, g.in_ptr, g.in_idx, directed=True, ms_degree_order=True)
    else:
        G = P.Graph.from_csr(g.n, ptr, idx, ms_degree_order=True)
    cand = np.nonzero(g.out_degree() > 0)[0]
    src = [int(s) for s in np.random.default_rng(95).choice(cand, size=70, replace=False)]
    src[5] = src[4]                                 # a repeated source
    want = oracle_all(g, src)
    msw = S.load_weights(S.MS_WEIGHTS)
    runs = [dict(variant="push"), dict(variant="pull"), dict(variant="heuristic"),
            dict(variant="learned", selector=msw), dict(variant="pull", grid_blocks=1),
            dict(variant="pull", grid_blocks=3)]
    for kw in runs:
        say(f"[batch] degree-ordered copy {name} {kw.get('variant')} {kw.get('grid_blocks', '')}")
        lv, pa = P.bfs_batch(G, src, **kw)
        vl, vp = P.bfs_batch_vm(G, src, **kw)
        torch.cuda.synchronize()
        compare_all(want, src, lambda q: (lv[q].cpu().numpy(), pa[q].cpu().numpy()), f"{name}/{kw}")
        compare_all(want, src, lambda q: (vl[:, q].cpu().numpy(), vp[:, q].cpu().numpy()), f"{name}/{kw}/vm")
    # the same graph without the copy gives the same arrays
    if g.directed:
        H = P.Graph.from_csr(g.n, ptr, idx, g.in_ptr, g.in_idx, directed=True, ms_degree_order=False)
    else:
        H = P.Graph.from_csr(g.n, ptr, idx, ms_degree_order=False)
    a_l, a_p = P.bfs_batch(H, src, variant="heuristic")
    b_l, b_p = P.bfs_batch(G, src, variant="heuristic")
    torch.cuda.synchronize()
    for q in range(len(src)):
        assert torch.equal(a_l[q], b_l[q]) and torch.equal(a_p[q], b_p[q]), q
