"""GPU parity of the comparison searches (SpMV-BFS, SpMSpV-BFS, SpMmSpV-BFS of
the Experiments section): level and parent bit-identical to the oracle's
search, and the device operation counts and step counts equal to the
oracle's step-by-step counts (oracle.compare)."""
import numpy as np
import pytest

import graphgen
from oracle import compare as C
from tests.gpu_common import assert_same, need_gpu, say

pytestmark = pytest.mark.gpu

METHODS = ["spmv", "spmspv", "spmmspv"]


@pytest.fixture(scope="module")
def P():
    return need_gpu()


def _graphs():
    return {
        "er": lambda: graphgen.erdos_renyi(5000, 6, 11),
        "rmat": lambda: graphgen.rmat(13, 16, 12),              # long rows and columns (chunks)
        "rmatd": lambda: graphgen.rmat(12, 16, 13, directed=True),
        "grid": lambda: graphgen.grid(60, 0.85, 14),            # ~150 steps, ragged frontiers
        "star": lambda: graphgen.star_graph(3000, center=17),   # one column / row of 2999 entries
        "path": lambda: graphgen.path_graph(130),
    }


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("name", list(_graphs()))
def test_compare_matches_oracle(P, name, method):
    import torch
    g = _graphs()[name]()
    G = P.Graph.from_graphgen(g)
    srcs = [int(s) for s in graphgen.pick_sources(g, 2, 5)]
    if name == "star":
        srcs = [17, 0]                                       # the hub, then a leaf
    for s in srcs:
        say(f"[compare] {name} {method} s={s}")
        lv, pa, ops, steps = P.bfs_compare(G, s, method)
        torch.cuda.synchronize()
        assert_same(g, s, (lv.cpu().numpy(), pa.cpu().numpy()), f"{name}/{method}/{s}")
        _, _, wops, wsteps = C.run(g, s, method, ops_only=True)
        assert (ops, steps) == (wops, wsteps), (name, method, s)
    G.close()


@pytest.mark.parametrize("method", METHODS)
def test_compare_isolated_source_and_reuse(P, method):
    """A source of out-degree 0 takes one step; the same workspace and outputs
    then serve a second, larger search."""
    import torch
    g = graphgen.rmat(12, 16, 21)
    iso = int(np.nonzero(g.out_degree() == 0)[0][0])
    G = P.Graph.from_graphgen(g)
    ws = P.Workspace(P.compare_workspace_size(G))
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty_like(lv)
    for s in (iso, int(graphgen.pick_sources(g, 1, 3)[0])):
        say(f"[compare] reuse {method} s={s}")
        _, _, ops, steps = P.bfs_compare(G, s, method, level=lv, parent=pa, workspace=ws)
        torch.cuda.synchronize()
        assert_same(g, s, (lv.cpu().numpy(), pa.cpu().numpy()), f"reuse/{method}/{s}")
        _, _, wops, wsteps = C.run(g, s, method, ops_only=True)
        assert (ops, steps) == (wops, wsteps)
    G.close()


def test_compare_rejects_bad_calls(P):
    g = graphgen.erdos_renyi(100, 4, 1)
    G = P.Graph.from_graphgen(g)
    with pytest.raises(P.BfsError):
        P.bfs_compare(G, 100, "spmv")                       # source out of range
    with pytest.raises(P.BfsError):
        P.bfs_compare(G, -1, "spmspv")
    small = P.Workspace(P.compare_workspace_size(G) - 256)
    with pytest.raises(P.BfsError):
        P._lib.check(P._lib.lib().bfs_run_compare(G.handle, 0, 0, None, None, small.ptr,
                                                  small.nbytes, None, None, None))
    G.close()
