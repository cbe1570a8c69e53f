"""Pins for the masked SpMSpV oracle (oracle.spmspv): the paper's 5x5
column-combination example, dense matrix forms of the same products, walk
counts on a cycle in closed form, and the search of Theorem 1 rebuilt from
repeated masked products."""
import math

import numpy as np
import pytest

import graphgen
import oracle
from oracle import brute
from oracle import spmspv as S
from tests.conftest import read_fixture

M64 = (1 << 64) - 1


def _graph(a, directed):
    ptr, idx, ip, ii = brute.to_csr(a)
    return graphgen.CSRGraph(a.shape[0], ptr, idx, directed, ip if directed else None,
                             ii if directed else None)


def test_colcomb_5x5_boolean_product():
    recs = read_fixture("colcomb_5x5.txt")
    n = int([r for r in recs if r[0] == "n"][0][1])
    a = np.zeros((n, n), dtype=np.int64)
    for r in recs:
        if r[0] == "row":
            a[int(r[1]) - 1] = [int(v) for v in r[2:]]
    x = np.array([int(v) for v in [r for r in recs if r[0] == "x"][0][1:]])
    want = np.array([int(v) for v in [r for r in recs if r[0] == "product"][0][1:]])
    # the printed product is A x; A^T x over A^T = A (the example's matrix is symmetric)
    assert np.array_equal(a, a.T)
    g = _graph(a, False)
    xi = np.nonzero(x)[0]
    yi, yv = S.masked_spmspv(g, "boolean", xi, np.ones(len(xi), np.uint64))
    assert np.array_equal(yi, np.nonzero(want)[0]) and np.all(yv == 1)


def _dense(a, semiring, xi, xv, R, C):
    """The same product from the dense matrix: y(i) over the rows R allows,
    columns j that C allows, A(j, i) = 1 (A^T's column j is j's out-list)."""
    n = a.shape[0]
    at = a.T.astype(bool)
    allowed_c = np.zeros(n, bool)
    vals = {}
    for j, v in zip(xi.tolist(), xv.tolist()):
        if C[j]:
            allowed_c[j] = True
            vals.setdefault(j, []).append(int(v))
    sub = at & R[:, None] & allowed_c[None, :]
    support = np.nonzero(sub.any(axis=1))[0]
    out = []
    for i in support:
        cols = np.nonzero(sub[i])[0]
        prods = [(1 if v else 0) if semiring == "boolean" else
                 (v if v == M64 else v + 1) if semiring == "min_plus" else v
                 for j in cols for v in vals[j]]
        if semiring == "boolean":
            out.append(int(any(prods)))
        elif semiring == "arithmetic":
            out.append(sum(prods) % (1 << 64))
        else:
            out.append(min(prods))
    return support, np.array(out, dtype=np.uint64)


@pytest.mark.parametrize("semiring", S.SEMIRINGS)
@pytest.mark.parametrize("directed", [False, True])
def test_matches_dense_forms(semiring, directed):
    rng = np.random.default_rng(3 + directed)
    for trial in range(30):
        n = int(rng.integers(2, 24))
        a = (rng.random((n, n)) < rng.uniform(0.05, 0.5)).astype(np.int64)
        np.fill_diagonal(a, 0)
        if not directed:
            a = np.maximum(a, a.T)
        g = _graph(a, directed)
        nx = int(rng.integers(0, 2 * n))
        xi = rng.integers(0, n, nx)                         # duplicates allowed
        big = rng.random(nx) < 0.3
        xv = np.where(big, rng.integers(2 ** 62, 2 ** 63, nx).astype(np.uint64) * 2 + 1,
                      rng.integers(0, 5, nx).astype(np.uint64)).astype(np.uint64)
        if nx:
            xv[0] = np.uint64(M64)                           # saturation / wrap edge
        rm = rng.random(n) < 0.6
        cm = rng.random(n) < 0.7
        for rc, cc in ((False, False), (True, False), (False, True), (True, True)):
            R = rm != rc
            C = cm != cc
            yi, yv = S.masked_spmspv(g, semiring, xi, xv, rm, cm, rc, cc)
            wi, wv = _dense(a, semiring, xi, xv, R, C)
            assert np.array_equal(yi, wi) and np.array_equal(yv, wv), (trial, rc, cc)
        yi, yv = S.masked_spmspv(g, semiring, xi, xv)         # no masks
        wi, wv = _dense(a, semiring, xi, xv, np.ones(n, bool), np.ones(n, bool))
        assert np.array_equal(yi, wi) and np.array_equal(yv, wv)


def test_walk_counts_on_a_cycle():
    """Arithmetic semiring: k products from e_s count the walks of length k,
    on the cycle C_n sum over t with k - 2t = d (mod n) of binom(k, t)."""
    n, s = 7, 2
    g = graphgen.cycle_graph(n)
    xi, xv = np.array([s]), np.array([1], np.uint64)
    for k in range(1, 12):
        xi, xv = S.masked_spmspv(g, "arithmetic", xi, xv)
        got = dict(zip(xi.tolist(), xv.tolist()))
        for i in range(n):
            d = (i - s) % n
            want = sum(math.comb(k, t) for t in range(k + 1) if (k - 2 * t - d) % n == 0)
            assert got.get(i, 0) == want, (k, i)


@pytest.mark.parametrize("name", ["er", "rmatd", "grid"])
def test_theorem1_search_from_masked_products(name):
    """x_{k+1} = A^T[V_{k+1}, :] x_k with the row mask = the unvisited rows
    (a complemented visited mask): min_select over x_k(j) = j gives each
    newly reached row its smallest frontier in-neighbour, min_plus over
    x_k(j) = k gives level k + 1 - the queue search's level and parent."""
    g = {"er": lambda: graphgen.erdos_renyi(300, 4, 2),
         "rmatd": lambda: graphgen.rmat(8, 8, 3, directed=True),
         "grid": lambda: graphgen.grid(15, 0.8, 4)}[name]()
    s = int(graphgen.pick_sources(g, 1, 1)[0])
    level = np.full(g.n, -1, np.int64)
    parent = np.full(g.n, -1, np.int64)
    level[s], parent[s] = 0, s
    visited = np.zeros(g.n, bool)
    visited[s] = True
    front = np.array([s])
    k = 0
    while len(front):
        pi, pv = S.masked_spmspv(g, "min_select", front, front.astype(np.uint64), visited, None, True)
        li, lv = S.masked_spmspv(g, "min_plus", front, np.full(len(front), k, np.uint64), visited,
                                 None, True)
        assert np.array_equal(pi, li) and np.all(lv == k + 1)
        parent[pi] = pv.astype(np.int64)
        level[pi] = k + 1
        visited[pi] = True
        front = pi
        k += 1
    wl, wp = oracle.bfs_graph(g, s)
    assert np.array_equal(level, wl) and np.array_equal(parent, wp)
