"""Pins for the oracle of the comparison searches (SpMV-BFS, SpMSpV-BFS,
SpMmSpV-BFS and the method, Experiments section): hand counts on Figure 1's
graph, closed forms, and Boolean matrix powers on every tiny graph."""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import brute
from oracle import compare as C
from tests.conftest import read_fixture


def _graph(a, directed):
    ptr, idx, ip, ii = brute.to_csr(a)
    if directed:
        return graphgen.CSRGraph(a.shape[0], ptr, idx, True, ip, ii)
    return graphgen.CSRGraph(a.shape[0], ptr, idx, False)


def _fig1():
    recs = read_fixture("fig1_path.txt")
    n = int([r for r in recs if r[0] == "n"][0][1])
    a = np.zeros((n, n), dtype=np.int64)
    for r in recs:
        if r[0] == "row":
            a[int(r[1]) - 1] = [int(v) for v in r[2:]]
    s = int([r for r in recs if r[0] == "source"][0][1]) - 1
    return a, s


def test_figure1_hand_counts():
    a, s = _fig1()
    g = _graph(a, False)
    want = {r[0]: (int(r[1]), int(r[2])) for r in read_fixture("fig1_ops.txt")}
    wl, wp = brute.bfs(a, s)
    for m in C.MEMBERS:
        lv, pa, ops, steps = C.run(g, s, m)
        assert (ops, steps) == want[m], m
        assert np.array_equal(lv, wl) and np.array_equal(pa, wp), m


def _by_powers(a, s):
    """Counts from Boolean powers of A^T alone: W_k = supp((A^T)^k e_s)."""
    n = a.shape[0]
    lv = brute.levels_by_powers(a, s)
    steps = int(lv.max()) + 1
    deg = a.sum(axis=1)
    m = (a.T != 0).astype(np.int64)
    w = np.zeros(n, np.int64)
    w[s] = 1
    walk = 0
    for _ in range(steps):
        walk += int(deg[w != 0].sum())
        w = (m @ w != 0).astype(np.int64)
    return {"spmv": 2 * int(a.sum()) * steps, "spmspv": 2 * walk,
            "spmmspv": 2 * int(deg[lv >= 0].sum()), "method": 2 * (int((lv >= 0).sum()) - 1)}, steps


@pytest.mark.parametrize("nv,directed", [(5, False), (4, True)])
def test_every_tiny_graph_matches_matrix_powers(nv, directed):
    graphs = brute.all_directed(nv) if directed else brute.all_undirected(nv)
    for a in graphs:
        g = _graph(a, directed)
        for s in range(nv):
            want, wsteps = _by_powers(a, s)
            wl, wp = brute.bfs(a, s)
            for m in C.MEMBERS:
                lv, pa, ops, steps = C.run(g, s, m)
                assert ops == want[m] and steps == wsteps, (m, a.tolist(), s)
                assert np.array_equal(lv, wl) and np.array_equal(pa, wp), (m, s)


@pytest.mark.parametrize("name", ["er", "rmat", "rmatd", "grid"])
def test_closed_forms_and_order(name):
    g = {"er": lambda: graphgen.erdos_renyi(4000, 6, 5),
         "rmat": lambda: graphgen.rmat(12, 16, 6),
         "rmatd": lambda: graphgen.rmat(11, 16, 7, directed=True),
         "grid": lambda: graphgen.grid(40, 0.85, 8)}[name]()
    s = int(graphgen.pick_sources(g, 1, 9)[0])
    wl, wp = oracle.bfs_graph(g, s)
    st = oracle.component_stats(g, wl)
    got = {}
    for m in C.MEMBERS:
        lv, pa, ops, steps = C.run(g, s, m)
        assert np.array_equal(lv, wl) and np.array_equal(pa, wp), m
        assert steps == st["levels"], m
        got[m] = ops
        lo, po, ops2, steps2 = C.run(g, s, m, ops_only=True)
        assert (ops2, steps2) == (ops, steps) and po is None and np.array_equal(lo, wl)
    # Table 2's columns: 2(n_c - 1), 2 nnz_c (Claim 1), 2 nnz (D + 1)
    assert got["method"] == 2 * (st["n_c"] - 1)
    assert got["spmmspv"] == 2 * st["nnz_c"]
    assert got["spmv"] == 2 * g.nnz * st["levels"]
    assert got["method"] <= got["spmmspv"] <= got["spmspv"] <= got["spmv"]
