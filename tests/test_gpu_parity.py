"""GPU parity: the HIP path against the oracle, bit-exact on level[] and parent[].

Every case prints its name before it touches the GPU.  Sizes: small enough for
the oracle to finish in well under a second each, large enough to span many
256-vertex tiles, ragged tails, split (chunked) columns and thousands of levels.
"""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import brute
from tests.conftest import read_fixture
from tests.gpu_common import assert_same, need_gpu, run_gpu, say

pytestmark = pytest.mark.gpu

VARIANTS = ["push", "pull", "bitmap", "heuristic", "short_circuit"]


def _graphs():
    return {
        "er16k": graphgen.erdos_renyi(16384, 8, 1),
        "rmat14": graphgen.rmat(14, 16, 2),
        "rmatd13": graphgen.rmat(13, 16, 3, directed=True),
        "grid128": graphgen.grid(128, 0.9, 4),
        "er_ragged": graphgen.erdos_renyi(1000 + 37, 3, 5),
    }


@pytest.fixture(scope="module")
def graphs():
    return _graphs()


@pytest.fixture(scope="module")
def P():
    return need_gpu()


def test_fig1_and_colcomb(P):
    for fx in ("fig1_path.txt", "colcomb_5x5.txt"):
        recs = read_fixture(fx)
        n = int([r for r in recs if r[0] == "n"][0][1])
        a = np.zeros((n, n), dtype=np.int64)
        for r in recs:
            if r[0] == "row":
                a[int(r[1]) - 1] = [int(v) for v in r[2:]]
        ptr, idx, _, _ = brute.to_csr(a)
        g = graphgen.CSRGraph(n, ptr, idx)
        G = P.Graph.from_graphgen(g)
        for s in range(n):
            for v in VARIANTS:
                say(f"[parity] {fx} s={s} variant={v}")
                assert_same(g, s, run_gpu(P, G, s, variant=v), f"{fx}/{s}/{v}")


@pytest.mark.parametrize("variant", VARIANTS)
def test_variants_on_small_graphs(P, graphs, variant):
    for name, g in graphs.items():
        G = P.Graph.from_graphgen(g)
        for s in graphgen.pick_sources(g, 3, 17):
            say(f"[parity] {name} s={s} variant={variant}")
            assert_same(g, s, run_gpu(P, G, s, variant=variant), f"{name}/{s}/{variant}")


@pytest.mark.parametrize("loop", ["host", "graph", "persistent"])
def test_loop_modes(P, graphs, loop):
    for name in ("er16k", "grid128", "rmatd13"):
        g = graphs[name]
        G = P.Graph.from_graphgen(g)
        for s in graphgen.pick_sources(g, 2, 23):
            for v in ("push", "heuristic", "short_circuit"):
                say(f"[parity] {name} s={s} loop={loop} variant={v}")
                assert_same(g, s, run_gpu(P, G, s, variant=v, loop=loop, levels_per_sync=3),
                            f"{name}/{s}/{loop}/{v}")


def test_split_columns_and_grid_shapes(P, graphs):
    """Tiny split threshold, tiny chunks, odd grid sizes: same bits."""
    g = graphs["rmat14"]
    G = P.Graph.from_graphgen(g)
    s = int(graphgen.pick_sources(g, 1, 5)[0])
    for heavy, chunk, grid in ((32, 64, 1), (32, 64, 7), (64, 1024, 333), (100000, 1024, 2048)):
        for v in ("push", "bitmap", "short_circuit"):
            say(f"[parity] rmat14 s={s} heavy={heavy} chunk={chunk} grid={grid} {v}")
            assert_same(g, s, run_gpu(P, G, s, variant=v, heavy_degree=heavy, chunk_edges=chunk,
                                      grid_blocks=grid), f"split/{heavy}/{chunk}/{grid}")


def test_edge_cases(P):
    # one vertex; an isolated source; a path with thousands of levels; unsorted
    # input with duplicates and self-loops; a directed graph whose CSC is built here
    cases = []
    cases.append(("n1", graphgen.CSRGraph(1, np.array([0, 0], np.int32), np.zeros(0, np.int32)), 0))
    g = graphgen.erdos_renyi(3000, 1.0, 9)
    iso = int(np.nonzero(g.out_degree() == 0)[0][0])
    cases.append(("isolated", g, iso))
    cases.append(("path3000", graphgen.path_graph(3000), 1500))
    cases.append(("star", graphgen.star_graph(2000, 1999), 3))
    for name, g, s in cases:
        G = P.Graph.from_graphgen(g)
        for v in VARIANTS:
            for loop in ("host", "persistent"):
                say(f"[parity] {name} s={s} variant={v} loop={loop}")
                assert_same(g, s, run_gpu(P, G, s, variant=v, loop=loop), f"{name}/{v}/{loop}")
    # messy input: duplicates, self-loops, unsorted rows -> same result as the clean graph
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
    for v in VARIANTS:
        for s in (5, 0, 7, 1995):              # 0, 7 and 1995 carry a self-loop
            say(f"[parity] messy s={s} variant={v}")
            assert_same(clean, s, run_gpu(P, G, s, variant=v), f"messy/{s}/{v}")
    # directed, CSC built by the library vs given
    gd = graphgen.rmat(12, 8, 4, directed=True)
    G1 = P.Graph.from_csr(gd.n, gd.ptr, gd.idx, directed=True)
    G2 = P.Graph.from_csr(gd.n, gd.ptr, gd.idx, gd.in_ptr, gd.in_idx, directed=True,
                          validate_transpose=True)
    for s in graphgen.pick_sources(gd, 2, 1):
        for v in ("push", "pull"):
            say(f"[parity] directed built-CSC s={s} {v}")
            assert_same(gd, s, run_gpu(P, G1, s, variant=v), "dir1")
            assert_same(gd, s, run_gpu(P, G2, s, variant=v), "dir2")


def test_multiroot_block_diagonal(P):
    """Every undirected graph on 5 vertices packed block-diagonally: one search per
    root position equals the brute-force result of each block."""
    mats = list(brute.all_undirected(5))
    gs = []
    for a in mats:
        ptr, idx, _, _ = brute.to_csr(a)
        gs.append(graphgen.CSRGraph(5, ptr, idx))
    packed, offs = graphgen.block_diagonal(gs)
    G = P.Graph.from_graphgen(packed)
    import torch
    for r in range(5):
        for v in ("push", "pull", "bitmap"):
            say(f"[parity] blockdiag5 root={r} variant={v}")
            roots = offs[:-1] + r
            lv, pa = P.bfs_roots(G, roots, variant=v)
            torch.cuda.synchronize()
            lv, pa = lv.cpu().numpy(), pa.cpu().numpy()
            for b, a in enumerate(mats):
                o = int(offs[b])
                bl, bp = brute.bfs(a, r)
                assert np.array_equal(lv[o:o + 5], bl), (b, r, v)
                bp = np.where(bp >= 0, bp + o, -1)
                assert np.array_equal(pa[o:o + 5], bp), (b, r, v)


def test_repeat_runs_identical(P, graphs):
    """Same inputs, different launch shapes and variants, repeated: identical bits."""
    g = graphs["rmat14"]
    G = P.Graph.from_graphgen(g)
    s = int(graphgen.pick_sources(g, 1, 99)[0])
    ref = run_gpu(P, G, s)
    for rep in range(3):
        for v, grid in (("push", 64), ("pull", 5), ("bitmap", 4096), ("heuristic", 17)):
            got = run_gpu(P, G, s, variant=v, grid_blocks=grid)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
