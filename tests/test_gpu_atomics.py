"""The push's parent atomics against Lemma 1: with the pre-read off, the
list-form push issues exactly one atomicMin per pair (j, i) with
level[i] = level[j] + 1 (every product that reaches an unvisited row takes
part in the min-select, none more); with the pre-read on, at least one per
reached row (the claim) and never more than that count.  The results equal
the oracle's either way."""
import numpy as np
import pytest

import graphgen
import oracle
from tests.gpu_common import assert_same, need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    return need_gpu()


def lemma1_pairs(g, level):
    """#{(j, i): j -> i, level[j] >= 0, level[i] = level[j] + 1} from the
    oracle's levels and the CSR of A (rows egress)."""
    deg = np.diff(g.ptr.astype(np.int64))
    src = np.repeat(np.arange(g.n), deg)
    lj = level[src]
    li = level[g.idx.astype(np.int64)]
    return int(np.count_nonzero((lj >= 0) & (li == lj + 1)))


def _graphs():
    return {"er": graphgen.erdos_renyi(20000, 6, 11),
            "rmat13": graphgen.rmat(13, 16, 12),
            "rmatd12": graphgen.rmat(12, 16, 13, directed=True),
            "grid80": graphgen.grid(80, 0.9, 14),
            "star": graphgen.star_graph(30001, 5)}


@pytest.mark.parametrize("name", ["er", "rmat13", "rmatd12", "grid80", "star"])
def test_atomic_count_is_lemma1(P, name):
    import torch
    g = _graphs()[name]
    G = P.Graph.from_graphgen(g)
    for s in [int(x) for x in graphgen.pick_sources(g, 2, 15)]:
        want_l, _ = oracle.bfs_graph(g, s)
        pairs = lemma1_pairs(g, want_l)
        reached = int(np.count_nonzero(want_l >= 0))
        for loop in ("host", "graph"):
            say(f"[atomics] {name} s={s} loop={loop}")
            exact, pre = {}, {}
            lv, pa = P.bfs(G, s, variant="push", push_impl="list", loop=loop, count_atomics=2, info=exact)
            torch.cuda.synchronize()
            assert_same(g, s, (lv.cpu().numpy(), pa.cpu().numpy()), f"{name}/{s}/exact")
            assert exact["atomics"] == pairs, (name, s, loop, exact["atomics"], pairs)
            lv, pa = P.bfs(G, s, variant="push", push_impl="list", loop=loop, count_atomics=1, info=pre)
            torch.cuda.synchronize()
            assert_same(g, s, (lv.cpu().numpy(), pa.cpu().numpy()), f"{name}/{s}/pre")
            assert reached - 1 <= pre["atomics"] <= pairs, (name, s, loop, pre["atomics"], reached, pairs)


def test_atomic_count_errors(P):
    g = graphgen.rmat(17, 16, 16)                  # the sliced form is the automatic choice here
    G = P.Graph.from_graphgen(g)
    with pytest.raises(P.BfsError):
        P.bfs(G, 0, count_atomics=1)
    with pytest.raises(P.BfsError):
        P.bfs(G, 0, push_impl="claim", count_atomics=1)
    with pytest.raises(P.BfsError):
        P.bfs(G, 0, push_impl="list", count_atomics=3)
    with pytest.raises(P.BfsError):
        P.bfs_roots(G, [0, 1], push_impl="list", count_atomics=1)
    info = {}
    P.bfs(G, 0, push_impl="list", count_atomics=2, info=info)   # still usable after the errors
    want_l, _ = oracle.bfs_graph(g, 0)
    assert info["atomics"] == lemma1_pairs(g, want_l)
