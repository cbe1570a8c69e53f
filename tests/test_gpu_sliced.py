"""GPU parity of the sliced push (the push form with the row mask in LDS):
every search bit-exact against the oracle, for every cut of the bitmap into
1 to 4 slices, both level loops, directed graphs, multi-root packs, self-loops
(one at the source), and the per-level frontier counts of the trace."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import brute
from tests.gpu_common import assert_same, need_gpu, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    return need_gpu()


def _cuts(n):
    """Slice sizes (words) giving 1, 2, 3 and 4 slices for n vertices."""
    words = (n + 31) // 32
    out = [32768]
    for S in (2, 3, 4):
        w = ((words + S - 1) // S + 3) & ~3
        if w >= 4 and (words + w - 1) // w == S:
            out.append(w)
    return out


GRAPHS = [
    ("er16k", lambda: graphgen.erdos_renyi(16384, 8, 1)),
    ("er_ragged", lambda: graphgen.erdos_renyi(1000 + 37, 3, 5)),
    ("rmat14", lambda: graphgen.rmat(14, 16, 2)),
    ("rmatd13", lambda: graphgen.rmat(13, 16, 3, directed=True)),
    ("grid128", lambda: graphgen.grid(128, 0.9, 4)),
]


@pytest.mark.parametrize("name,make", GRAPHS, ids=[g[0] for g in GRAPHS])
def test_every_cut(P, name, make):
    g = make()
    G = P.Graph.from_graphgen(g)
    srcs = graphgen.pick_sources(g, 3, 41)
    for words in _cuts(g.n):
        G.set_slice_words(words)
        for s in srcs:
            for loop, lps in (("host", 0), ("graph", 3)):
                say(f"[sliced] {name} words={words} s={s} loop={loop}")
                assert_same(g, s, run_gpu(P, G, s, variant="push", push_impl="sliced", loop=loop,
                                          levels_per_sync=lps), f"{name}/{words}/{s}/{loop}")


def test_long_parts_chunked(P):
    """Columns whose slice parts reach the chunk threshold (a star and a
    dense hub graph), every cut."""
    hub = graphgen.star_graph(9000, 4321)
    rng = np.random.default_rng(8)
    src = rng.integers(0, 6000, 60000)
    dst = rng.integers(0, 40, 60000)           # 40 hubs of ~1500 entries each
    g2 = graphgen.from_edges(6000, src.astype(np.int32), dst.astype(np.int32))
    for name, g in (("star9000", hub), ("hubs", g2)):
        G = P.Graph.from_graphgen(g)
        for words in _cuts(g.n):
            G.set_slice_words(words)
            for s in graphgen.pick_sources(g, 3, 9):
                say(f"[sliced] {name} words={words} s={s}")
                assert_same(g, s, run_gpu(P, G, s, push_impl="sliced"), f"{name}/{words}/{s}")


def test_self_loops_and_source_loop(P):
    """Self-loops everywhere, one at the source, duplicates and unsorted rows:
    the same bits as the clean graph (the source is visited from the start)."""
    clean = graphgen.erdos_renyi(3000, 6, 12)
    rng = np.random.default_rng(4)
    rows = []
    for v in range(clean.n):
        r = list(clean.idx[clean.ptr[v]:clean.ptr[v + 1]])
        r += r[: len(r) // 2] + ([v, v] if v % 5 == 0 else [])
        rng.shuffle(r)
        rows.append(r)
    ptr = np.zeros(clean.n + 1, np.int32)
    ptr[1:] = np.cumsum([len(r) for r in rows])
    idx = np.array([x for r in rows for x in r], np.int32)
    G = P.Graph.from_csr(clean.n, ptr, idx)
    for words in _cuts(clean.n):
        G.set_slice_words(words)
        for s in (0, 5, 10, 2995):                # every one of these has a self-loop
            for impl in ("sliced", "list"):
                say(f"[sliced] self-loops words={words} s={s} {impl}")
                assert_same(clean, s, run_gpu(P, G, s, push_impl=impl), f"loops/{words}/{s}/{impl}")


def test_directed_built_and_given_csc(P):
    gd = graphgen.rmat(12, 8, 4, directed=True)
    G1 = P.Graph.from_csr(gd.n, gd.ptr, gd.idx, directed=True)
    G2 = P.Graph.from_csr(gd.n, gd.ptr, gd.idx, gd.in_ptr, gd.in_idx, directed=True,
                          validate_transpose=True)
    for words in _cuts(gd.n):
        G1.set_slice_words(words)
        G2.set_slice_words(words)
        for s in graphgen.pick_sources(gd, 3, 2):
            say(f"[sliced] directed words={words} s={s}")
            assert_same(gd, s, run_gpu(P, G1, s, push_impl="sliced"), "dir-built")
            assert_same(gd, s, run_gpu(P, G2, s, push_impl="sliced"), "dir-given")


def test_multiroot_pack(P):
    """Every undirected graph on 5 vertices, packed block-diagonally, one root
    per block: each block equals its brute-force search."""
    import torch
    mats = list(brute.all_undirected(5))
    gs = []
    for a in mats:
        ptr, idx, _, _ = brute.to_csr(a)
        gs.append(graphgen.CSRGraph(5, ptr, idx))
    packed, offs = graphgen.block_diagonal(gs)
    G = P.Graph.from_graphgen(packed)
    for words in _cuts(packed.n):
        G.set_slice_words(words)
        for r in range(5):
            say(f"[sliced] blockdiag5 words={words} root={r}")
            lv, pa = P.bfs_roots(G, offs[:-1] + r, push_impl="sliced")
            torch.cuda.synchronize()
            lv, pa = lv.cpu().numpy(), pa.cpu().numpy()
            for b, a in enumerate(mats):
                o = int(offs[b])
                bl, bp = brute.bfs(a, r)
                assert np.array_equal(lv[o:o + 5], bl), (words, b, r)
                assert np.array_equal(pa[o:o + 5], np.where(bp >= 0, bp + o, -1)), (words, b, r)


def test_trace_counts(P):
    """The per-level records: |F_k| and its degree sum, as the oracle's levels give them."""
    g = graphgen.rmat(14, 16, 6)
    G = P.Graph.from_graphgen(g)
    s = int(graphgen.pick_sources(g, 1, 3)[0])
    info = {}
    say(f"[sliced] trace rmat14 s={s}")
    P.bfs(G, s, push_impl="sliced", info=info, trace=True, time_kernels=True)
    wl, _ = oracle.bfs_graph(g, s)
    deg = np.diff(g.ptr.astype(np.int64))
    tr = info["trace"]
    assert len(tr) == int(wl.max()) + 1
    for r in tr:
        k = r["level"]
        assert r["frontier"] == int(np.count_nonzero(wl == k)), k
        assert r["frontier_edges"] == int(deg[wl == k].sum()), k
        assert r["unvisited"] == int(np.count_nonzero((wl < 0) | (wl > k))), k
    assert info["launches"] >= len(tr) and info["kernel_us"] > 0


def test_errors(P):
    g = graphgen.erdos_renyi(4096, 4, 3)
    G = P.Graph.from_graphgen(g)
    with pytest.raises(P.BfsError):
        run_gpu(P, G, 0, push_impl="sliced", loop="persistent")
    with pytest.raises(P.BfsError):
        run_gpu(P, G, 0, push_impl="sliced", variant="pull")
    with pytest.raises(P.BfsError):
        G.set_slice_words(6)                   # not a multiple of 4
    with pytest.raises(P.BfsError):
        G.set_slice_words(4)                   # 128 words -> 32 slices
    with pytest.raises(P.BfsError):
        run_gpu(P, G, 0, push_impl=7)
    # after the rejected cuts the graph still searches with its last good cut
    assert_same(g, 0, run_gpu(P, G, 0, push_impl="sliced"), "after errors")
