"""GPU parity of the masked SpMSpV primitive (bfs_masked_spmspv): every
semiring, row / column masks and their complements, duplicate vector
indices, split long columns; support and values bit-identical to the oracle
(oracle.spmspv).  Also the search of Theorem 1 driven by the primitive."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import spmspv as S
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu
M64 = np.uint64((1 << 64) - 1)


@pytest.fixture(scope="module")
def P():
    return need_gpu()


def _words(mask):
    n = len(mask)
    w = np.zeros((n + 31) // 32, np.uint32)
    idx = np.nonzero(mask)[0]
    np.bitwise_or.at(w, idx >> 5, (np.uint32(1) << (idx & 31).astype(np.uint32)))
    return w


def _dev(P, a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a).view(dtype)).cuda()


def _graphs():
    return {
        "er": lambda: graphgen.erdos_renyi(3000, 6, 31),
        "rmat": lambda: graphgen.rmat(13, 16, 32),              # columns of >= 512 entries
        "rmatd": lambda: graphgen.rmat(12, 16, 33, directed=True),
        "star": lambda: graphgen.star_graph(2500, center=9),
    }


@pytest.mark.parametrize("name", list(_graphs()))
def test_spmspv_matches_oracle(P, name):
    import torch
    g = _graphs()[name]()
    G = P.Graph.from_graphgen(g)
    rng = np.random.default_rng(len(name))
    nx = min(g.n, 1500)
    ws = P.Workspace(P.spmspv_workspace_size(G, 2 * nx))
    ws.buf.zero_()
    for trial in range(3):
        xi = rng.integers(0, g.n, nx).astype(np.int32)
        xi[: nx // 10] = xi[0]                                 # duplicates
        if name == "star":
            xi[1] = 9                                          # the hub (2499 entries)
        xv = rng.integers(0, 1 << 63, nx, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, nx, dtype=np.uint64)
        xv[rng.random(nx) < 0.1] = 0
        xv[rng.random(nx) < 0.05] = M64
        rm = rng.random(g.n) < 0.6
        cm = rng.random(g.n) < 0.8
        for semiring in S.SEMIRINGS:
            for rmask, cmask, rc, cc in ((None, None, False, False), (rm, None, True, False),
                                         (rm, cm, False, True), (None, cm, False, False)):
                say(f"[spmspv] {name} trial {trial} {semiring} masks {rmask is not None}{rc} {cmask is not None}{cc}")
                yi, yv = P.masked_spmspv(G, semiring, _dev(P, xi, np.int32), _dev(P, xv, np.int64),
                                         None if rmask is None else _dev(P, _words(rmask), np.int32),
                                         None if cmask is None else _dev(P, _words(cmask), np.int32),
                                         rc, cc, workspace=ws)
                torch.cuda.synchronize()
                gi = yi.cpu().numpy()
                gv = yv.cpu().numpy().view(np.uint64)
                wi, wv = S.masked_spmspv(g, semiring, xi, xv, rmask, cmask, rc, cc)
                assert np.array_equal(gi, wi), (name, semiring, len(gi), len(wi))
                assert np.array_equal(gv, wv), (name, semiring)
    G.close()


def test_spmspv_edge_cases(P):
    import torch
    g = graphgen.rmat(10, 8, 41)
    G = P.Graph.from_graphgen(g)
    ws = P.Workspace(P.spmspv_workspace_size(G, 64))
    ws.buf.zero_()
    empty = torch.empty(0, dtype=torch.int32, device="cuda")
    yi, yv = P.masked_spmspv(G, "arithmetic", empty, torch.empty(0, dtype=torch.int64, device="cuda"),
                             workspace=ws)
    assert yi.numel() == 0 and yv.numel() == 0
    bad = _dev(P, np.array([3, g.n], np.int32), np.int32)     # an index past the end
    with pytest.raises(P.BfsError) as e:
        P.masked_spmspv(G, "boolean", bad, _dev(P, np.array([1, 1], np.uint64), np.int64), workspace=ws)
    assert e.value.status == P._lib.BFS_ERANGE
    # the workspace is still clean: a good call after the failed one is exact
    xi = np.array([0, 1, 2, 3], np.int32)
    xv = np.array([5, 6, 7, 8], np.uint64)
    yi, yv = P.masked_spmspv(G, "arithmetic", _dev(P, xi, np.int32), _dev(P, xv, np.int64), workspace=ws)
    torch.cuda.synchronize()
    wi, wv = S.masked_spmspv(g, "arithmetic", xi, xv)
    assert np.array_equal(yi.cpu().numpy(), wi) and np.array_equal(yv.cpu().numpy().view(np.uint64), wv)
    # every column masked out
    yi, _ = P.masked_spmspv(G, "min_select", _dev(P, xi, np.int32), _dev(P, xv, np.int64),
                            col_mask=_dev(P, _words(np.ones(g.n, bool)), np.int32), col_complement=True,
                            workspace=ws)
    assert yi.numel() == 0
    G.close()


@pytest.mark.parametrize("name", ["rmat", "rmatd"])
def test_theorem1_search_from_the_primitive(P, name):
    """x_{k+1} = A^T[V_{k+1}, :] x_k with (min, select) over x_k(j) = j and the
    row mask = the visited rows, complemented: the queue search's level and
    parent, bit for bit."""
    import torch
    g = {"rmat": lambda: graphgen.rmat(14, 16, 51), "rmatd": lambda: graphgen.rmat(13, 16, 52, directed=True)}[name]()
    G = P.Graph.from_graphgen(g)
    s = int(graphgen.pick_sources(g, 1, 3)[0])
    ws = P.Workspace(P.spmspv_workspace_size(G, g.n))
    ws.buf.zero_()
    level = np.full(g.n, -1, np.int64)
    parent = np.full(g.n, -1, np.int64)
    level[s], parent[s] = 0, s
    visited = np.zeros(g.n, bool)
    visited[s] = True
    front = np.array([s], np.int32)
    k = 0
    while len(front):
        say(f"[spmspv-bfs] {name} level {k} frontier {len(front)}")
        yi, yv = P.masked_spmspv(G, "min_select", _dev(P, front, np.int32),
                                 _dev(P, front.astype(np.uint64), np.int64),
                                 _dev(P, _words(visited), np.int32), None, True, workspace=ws)
        torch.cuda.synchronize()
        new = yi.cpu().numpy()
        parent[new] = yv.cpu().numpy().view(np.uint64).astype(np.int64)
        level[new] = k + 1
        visited[new] = True
        front = new
        k += 1
    wl, wp = oracle.bfs_graph(g, s)
    assert np.array_equal(level, wl) and np.array_equal(parent, wp)
    G.close()
