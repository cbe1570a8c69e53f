"""GPU parity of the claim-word push (push_impl "claim") and of batches of
queries on different graphs (which run through it): every query's level[]
and parent[] equal the oracle's bit for bit.  The cases cross the narrow /
wide boundary both ways (frontiers beyond the LDS, too many long columns,
too many entries), the narrow kernel's level budget per launch, hubs split
into chunks, and mixes of graphs of different sizes with repeats."""
import numpy as np
import pytest

import graphgen
from tests.gpu_common import assert_same, compare_all, need_gpu, oracle_all, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    return need_gpu()


def _broom(path_len, leaves, tail, seed):
    """A path of path_len vertices, then a star of `leaves` leaves on its last
    vertex, leaf i continuing into a path of (7 i) mod `tail` vertices: thin,
    then levels far wider than the LDS frontier, then thin again."""
    src, dst = [], []
    for i in range(path_len - 1):
        src.append(i); dst.append(i + 1)
    hub = path_len - 1
    nxt = path_len
    for leaf in range(leaves):
        prev = hub
        for _ in range((7 * leaf) % tail + 1):
            src.append(prev); dst.append(nxt)
            prev = nxt
            nxt += 1
    rng = np.random.default_rng(seed)
    perm = rng.permutation(nxt).astype(np.int32)          # labels scattered
    s = perm[np.array(src)]
    d = perm[np.array(dst)]
    return graphgen.from_edges(nxt, s, d), int(perm[0])


def _wide_level(count, deg, seed):
    """Source -> `count` vertices, each with `deg` further out-neighbours of its own:
    level 1 holds more than 2048 columns of more than four entries."""
    src, dst = [], []
    nxt = 1 + count
    for i in range(count):
        src.append(0); dst.append(1 + i)
        for _ in range(deg):
            src.append(1 + i); dst.append(nxt)
            nxt += 1
    return graphgen.from_edges(nxt, np.array(src), np.array(dst)), 0


def _cases():
    return {
        "er16k": (graphgen.erdos_renyi(16384, 8, 1), None),
        "rmat14": (graphgen.rmat(14, 16, 2), None),
        "rmatd13": (graphgen.rmat(13, 16, 3, directed=True), None),
        "grid200": (graphgen.grid(200, 0.9, 4), None),
        "er_ragged": (graphgen.erdos_renyi(1037, 3, 5), None),
        "path5000": (graphgen.path_graph(5000), 0),             # 5000 levels: two narrow launches
        "star100k": (graphgen.star_graph(100001, 7), 7),       # one column of 10^5 entries
        "star_leaf": (graphgen.star_graph(20001, 3), 11),
        "broom": _broom(300, 12000, 60, 6),
        "wide_long": _wide_level(3000, 6, 7),
        "tree": (graphgen.binary_tree(50000), 0),
    }


@pytest.fixture(scope="module")
def cases():
    return _cases()


@pytest.mark.parametrize("name", ["er16k", "rmat14", "rmatd13", "grid200", "er_ragged", "path5000",
                                  "star100k", "star_leaf", "broom", "wide_long", "tree"])
def test_claim_single_source(P, cases, name):
    g, s0 = cases[name]
    G = P.Graph.from_graphgen(g)
    srcs = [s0] if s0 is not None else [int(s) for s in graphgen.pick_sources(g, 3, 41)]
    for s in srcs:
        say(f"[claim] {name} s={s}")
        info = {}
        got = run_gpu(P, G, s, push_impl="claim", info=info)
        assert_same(g, s, got, f"claim/{name}/{s}")


def test_claim_edge_cases(P):
    import torch
    # one vertex; an isolated source; self-loops and duplicates (same bits as clean)
    g1 = graphgen.CSRGraph(1, np.array([0, 0], np.int32), np.zeros(0, np.int32))
    say("[claim] n1")
    assert_same(g1, 0, run_gpu(P, P.Graph.from_graphgen(g1), 0, push_impl="claim"), "n1")
    g = graphgen.erdos_renyi(3000, 1.0, 9)
    iso = int(np.nonzero(g.out_degree() == 0)[0][0])
    say("[claim] isolated")
    assert_same(g, iso, run_gpu(P, P.Graph.from_graphgen(g), iso, push_impl="claim"), "isolated")
    clean = graphgen.erdos_renyi(2000, 6, 10)
    rng = np.random.default_rng(3)
    rows = []
    for v in range(clean.n):
        r = list(clean.idx[clean.ptr[v]:clean.ptr[v + 1]])
        r += r[: len(r) // 3] + ([v] if v % 7 == 0 else [])
        rng.shuffle(r)
        rows.append(r)
    ptr = np.zeros(clean.n + 1, np.int32)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([x for r in rows for x in r], np.int32)
    G = P.Graph.from_csr(clean.n, ptr, idx)
    for s in (5, 0, 7):                                  # 0 and 7 carry a self-loop
        say(f"[claim] messy s={s}")
        assert_same(clean, s, run_gpu(P, G, s, push_impl="claim"), f"messy/{s}")
    # only the push and the host loop
    with pytest.raises(P.BfsError):
        P.bfs(G, 5, push_impl="claim", variant="pull")
    with pytest.raises(P.BfsError):
        P.bfs(G, 5, push_impl="claim", loop="graph")
    torch.cuda.synchronize()


def test_mixed_graph_batch(P):
    """Queries on many different graphs (ER of log-uniform sizes, a grid, an
    R-MAT, a directed R-MAT, repeats of one graph with different sources) in
    one call: each result equals the oracle's."""
    import torch
    fam = graphgen.er_family(count=24, lo=8, hi=13)
    extra = [graphgen.grid(120, 0.9, 3), graphgen.rmat(12, 16, 4), graphgen.rmat(11, 16, 5, directed=True)]
    gs = fam + extra
    Gs = [P.Graph.from_graphgen(g) for g in gs]
    graphs, srcs, hosts = [], [], []
    for i, (g, G) in enumerate(zip(gs, Gs)):
        reps = 3 if i in (0, len(gs) - 2) else 1           # the same graph several times
        for s in graphgen.pick_sources(g, reps, 50 + i):
            graphs.append(G); srcs.append(int(s)); hosts.append(g)
    say(f"[claim] mixed batch of {len(srcs)} queries on {len(gs)} graphs")
    info = {}
    lv, pa = P.bfs_batch(graphs, srcs, info=info)
    torch.cuda.synchronize()
    for q, (g, s) in enumerate(zip(hosts, srcs)):
        assert_same(g, s, (lv[q].cpu().numpy(), pa[q].cpu().numpy()), f"mixed/q{q}")
    # the same workspace again with another mix, smaller
    ws = P.Workspace(P.batch_workspace_size(graphs))
    P.bfs_batch(graphs, srcs, workspace=ws)
    sub = list(range(0, len(srcs), 3))
    lv2, pa2 = P.bfs_batch([graphs[i] for i in sub], [srcs[i] for i in sub], workspace=ws)
    torch.cuda.synchronize()
    for j, q in enumerate(sub):
        assert_same(hosts[q], srcs[q], (lv2[j].cpu().numpy(), pa2[j].cpu().numpy()), f"mixed2/q{q}")


def test_er_pack_64_graphs(P):
    """64 Erdos-Renyi graphs, n log-uniform in [2^10, 2^16], average degree
    4-32, one source each, one call; every query against the oracle."""
    import torch
    fam = graphgen.er_family(count=64, lo=10, hi=16)
    Gs = [P.Graph.from_graphgen(g) for g in fam]
    srcs = [int(graphgen.pick_sources(g, 1, 60 + i)[0]) for i, g in enumerate(fam)]
    say("[claim] 64-graph ER pack")
    lv, pa = P.bfs_batch(Gs, srcs)
    torch.cuda.synchronize()
    for q, (g, s) in enumerate(zip(fam, srcs)):
        assert_same(g, s, (lv[q].cpu().numpy(), pa[q].cpu().numpy()), f"er64/q{q}")


def test_mixed_batch_rejects_other_variants(P):
    fam = graphgen.er_family(count=2, lo=8, hi=9)
    Gs = [P.Graph.from_graphgen(g) for g in fam]
    with pytest.raises(P.BfsError):
        P.bfs_batch(Gs, [0, 0], variant="pull")


@pytest.mark.parametrize("name", ["grid", "path", "rmat", "broom"])
def test_claim_batch_on_one_graph(P, cases, name):
    """Many sources on one graph as claim-word searches in lockstep (the form
    the library takes by itself for thin graphs beyond 2^22 vertices, asked
    for here): every query equals the oracle's, duplicates included."""
    import torch
    g, s0 = {"grid": (graphgen.grid(150, 0.9, 81), None), "path": (graphgen.path_graph(3000), None),
             "rmat": (graphgen.rmat(12, 16, 82), None), "broom": cases["broom"]}[name]
    G = P.Graph.from_graphgen(g)
    cand = np.nonzero(g.out_degree() > 0)[0]
    src = [int(s) for s in np.random.default_rng(83).choice(cand, size=20, replace=True)]
    src[1] = src[0]
    if s0 is not None:
        src[2] = s0
    want = oracle_all(g, src)
    say(f"[claim] batch of {len(src)} on {name}")
    lv, pa = P.bfs_batch(G, src, push_impl="claim")
    torch.cuda.synchronize()
    compare_all(want, src, lambda q: (lv[q].cpu().numpy(), pa[q].cpu().numpy()), f"claim batch {name}")


def test_auto_form_from_degrees(P):
    """The automatic push picks its form from the out-degrees: claim-word when
    every out-degree is at most 8 (a grid, a path), sliced on a graph with hubs
    of at least 2^17 vertices (R-MAT), the list form on flat degrees (ER) and
    on small graphs; the searches equal the oracle's and report the form."""
    cases = [("grid", graphgen.grid(200, 0.9, 91), "claim"),
             ("path", graphgen.path_graph(3000), "claim"),
             ("rmat17", graphgen.rmat(17, 16, 92), "sliced"),
             ("er17", graphgen.erdos_renyi(1 << 17, 16, 93), "list"),
             ("rmat12", graphgen.rmat(12, 16, 94), "list")]
    for name, g, want in cases:
        G = P.Graph.from_graphgen(g)
        s = int(graphgen.pick_sources(g, 1, 95)[0])
        say(f"[auto] {name} s={s}")
        info = {}
        got = run_gpu(P, G, s, info=info)
        assert info["push_used"] == want, (name, info["push_used"])
        assert_same(g, s, got, f"auto/{name}")
    # several roots over a block-diagonal pack of ER graphs: the list form
    fam = graphgen.er_family(count=8, lo=12, hi=15)
    pack, offs = graphgen.block_diagonal(fam)
    G = P.Graph.from_graphgen(pack)
    roots = [int(o) for o in offs[:-1]]
    info = {}
    say("[auto] ER pack roots")
    P.bfs_roots(G, roots, info=info)
    assert info["push_used"] == "list"


def test_mixed_batch_both_forms(P):
    """Queries on different graphs in either form of the library: the list form
    over the graphs packed into one block-diagonal graph (the automatic choice
    when no graph is thin) and the claim-word form (the automatic choice with a
    grid in the mix); each forced on the other's mix too.  Every query against
    the oracle, repeats of one graph included."""
    import torch
    fam = graphgen.er_family(count=12, lo=9, hi=13)
    flat = fam + [graphgen.rmat(12, 16, 71), graphgen.rmat(11, 16, 72, directed=True)]
    mixes = {"flat": flat, "with_grid": flat[:6] + [graphgen.grid(100, 0.9, 73)]}
    for name, gs in mixes.items():
        Gs = [P.Graph.from_graphgen(g) for g in gs]
        graphs, srcs, hosts = [], [], []
        for i, (g, G) in enumerate(zip(gs, Gs)):
            for s in graphgen.pick_sources(g, 2 if i == 0 else 1, 80 + i):
                graphs.append(G); srcs.append(int(s)); hosts.append(g)
        auto = "claim" if name == "with_grid" else "list"
        for impl in ("auto", "list", "claim"):
            say(f"[mixed] {name} push_impl={impl}")
            info = {}
            lv, pa = P.bfs_batch(graphs, srcs, push_impl=impl, info=info)
            torch.cuda.synchronize()
            assert info["push_used"] == (auto if impl == "auto" else impl), (name, impl, info)
            for q, (g, s) in enumerate(zip(hosts, srcs)):
                assert_same(g, s, (lv[q].cpu().numpy(), pa[q].cpu().numpy()), f"{name}/{impl}/q{q}")
        with pytest.raises(P.BfsError):
            P.bfs_batch(graphs, srcs, push_impl="sliced")
