"""Pins for the CPU oracle: paper fixtures, brute force, closed forms, counts, invariants.

None of these compares the oracle with itself: each checks it against a value
the paper prints, a closed form, an exhaustive brute force that uses no search
procedure, or an invariant that a plausible mistake would break.
"""
import numpy as np
import pytest

import graphgen
import oracle
from oracle import algebra, brute, certify
from tests.conftest import read_fixture


def _dense_from_fixture(recs):
    n = int([r for r in recs if r[0] == "n"][0][1])
    a = np.zeros((n, n), dtype=np.int64)
    for r in recs:
        if r[0] == "row":
            a[int(r[1]) - 1] = [int(v) for v in r[2:]]
    return n, a


def _all_oracles(a, s):
    """Run O-A, O-B (modes 0 and 1), O-C and O-D on a dense 0/1 matrix."""
    n = a.shape[0]
    ptr, idx, ip, ii = brute.to_csr(a)
    out = {"queue": oracle.bfs_queue(n, ptr, idx, s, ip, ii)}
    l0, p0, _ = oracle.bfs_alg2(n, ptr, idx, s, mode=0)
    l1, p1, _ = oracle.bfs_alg2(n, ptr, idx, s, mode=1)
    out["alg2"] = (l0, p0)
    out["alg2_all"] = (l1, p1)
    out["algebra"] = algebra.bfs(a, s)
    out["brute"] = brute.bfs(a, s)
    return out


# ---- Figure 1 -----------------------------------------------------------------------

def test_fig1_levels_parents_and_masks():
    recs = read_fixture("fig1_path.txt")
    n, a = _dense_from_fixture(recs)
    s = int([r for r in recs if r[0] == "source"][0][1]) - 1
    steps = [r for r in recs if r[0] == "step"]
    # the recurrence's per-step supports and masks are the ones the figure draws
    run = algebra.submatrix_steps(a, s, "boolean")
    xs, Vs = run["x"], run["V"]
    for r in steps:
        k = int(r[1])
        i_in, i_out, i_rows, i_cols = r.index("in"), r.index("out"), r.index("rows"), r.index("cols")
        sup_in = {int(v) - 1 for v in r[i_in + 1:i_out]}
        sup_out = {int(v) - 1 for v in r[i_out + 1:i_rows]}
        rows_masked = {int(v) - 1 for v in r[i_rows + 1:i_cols]}
        cols_masked = {int(v) - 1 for v in r[i_cols + 1:]}
        assert set(np.nonzero(xs[k - 1])[0]) == sup_in
        assert set(np.nonzero(xs[k])[0]) == sup_out
        assert set(range(n)) - set(Vs[k]) == rows_masked          # V_{k+1}
        assert set(range(n)) - set(Vs[k - 1]) == cols_masked      # V_k
    assert not np.any(xs[len(steps) + 1]) and len(xs) == len(steps) + 2   # x_6 = 0: done
    # every oracle gives the levels/parents the figure implies
    want_level = np.zeros(n, dtype=np.int64)
    want_parent = np.zeros(n, dtype=np.int64)
    want_level[s], want_parent[s] = 0, s
    for r in steps:
        k = int(r[1])
        src = int(r[r.index("in") + 1]) - 1
        dst = int(r[r.index("out") + 1]) - 1
        want_level[dst], want_parent[dst] = k, src
    for name, (lv, pa) in _all_oracles(a, s).items():
        assert np.array_equal(lv, want_level), name
        assert np.array_equal(pa, want_parent), name


def test_colcomb_example():
    recs = read_fixture("colcomb_5x5.txt")
    n, a = _dense_from_fixture(recs)
    get = {r[0]: np.array([int(v) for v in r[1:]]) for r in recs if r[0] != "row"}
    x = get["x"]
    # the selected columns are the paper's
    assert np.array_equal(a[:, 1], get["col2"]) and np.array_equal(a[:, 2], get["col3"])
    # the unmasked product (one step, all rows and columns) in the Boolean semiring
    prod = algebra._semiring_product(a, x, "boolean")
    assert np.array_equal(prod, get["product"])
    # same support in the arithmetic semiring (only zero / nonzero matters)
    assert np.array_equal(algebra._semiring_product(a, x, "arithmetic") != 0, get["product"] != 0)
    # and the BFS from each vertex of this graph agrees across all oracles
    for s in range(n):
        res = _all_oracles(a, s)
        ref = res["brute"]
        for name, (lv, pa) in res.items():
            assert np.array_equal(lv, ref[0]) and np.array_equal(pa, ref[1]), (name, s)


# ---- exhaustive brute force ----------------------------------------------------------

@pytest.mark.parametrize("nv", [1, 2, 3, 4, 5])
def test_all_undirected_graphs(nv):
    for a in brute.all_undirected(nv):
        ptr, idx, _, _ = brute.to_csr(a)
        for s in range(nv):
            lv_b, pa_b = brute.bfs(a, s)
            lv, pa = oracle.bfs_queue(nv, ptr, idx, s)
            assert np.array_equal(lv, lv_b) and np.array_equal(pa, pa_b)
            for mode in (0, 1):
                l2, p2, c = oracle.bfs_alg2(nv, ptr, idx, s, mode)
                assert np.array_equal(l2, lv_b) and np.array_equal(p2, pa_b)
            assert certify.check(nv, ptr, idx, s, lv, pa) == []


@pytest.mark.parametrize("nv", [2, 3, 4])
def test_all_directed_graphs(nv):
    for a in brute.all_directed(nv):
        ptr, idx, ip, ii = brute.to_csr(a)
        for s in range(nv):
            lv_b, pa_b = brute.bfs(a, s)
            lv, pa = oracle.bfs_queue(nv, ptr, idx, s, ip, ii)
            assert np.array_equal(lv, lv_b) and np.array_equal(pa, pa_b)
            l2, p2, _ = oracle.bfs_alg2(nv, ptr, idx, s, 0)
            assert np.array_equal(l2, lv_b) and np.array_equal(p2, pa_b)
            assert certify.check(nv, ptr, idx, s, lv, pa) == []


def test_algebra_matches_brute_on_sample():
    """O-C (the literal recurrence) on every 4-vertex graph and a sample of 6-vertex ones."""
    rng = np.random.default_rng(7)
    cases = list(brute.all_undirected(4))
    for _ in range(60):
        a = np.triu((rng.random((6, 6)) < 0.4).astype(np.int64), 1)
        cases.append(a + a.T)
    for _ in range(40):
        a = (rng.random((5, 5)) < 0.35).astype(np.int64)
        np.fill_diagonal(a, 0)
        cases.append(a)                                   # directed
    for a in cases:
        for s in range(a.shape[0]):
            lv_b, pa_b = brute.bfs(a, s)
            lv, pa = algebra.bfs(a, s)
            assert np.array_equal(lv, lv_b) and np.array_equal(pa, pa_b)


def test_semiring_supports_agree_and_prop1():
    """Boolean / arithmetic / (min,select) give the same supports (Notation section);
    Proposition 1's transform gives the same supports; the symmetric form too."""
    rng = np.random.default_rng(11)
    for trial in range(30):
        nv = int(rng.integers(3, 8))
        a = np.triu((rng.random((nv, nv)) < 0.45).astype(np.int64), 1)
        if trial % 3 == 2:
            a = (rng.random((nv, nv)) < 0.3).astype(np.int64)
            np.fill_diagonal(a, 0)
        else:
            a = a + a.T
        s = int(rng.integers(0, nv))
        runs = {sr: algebra.submatrix_steps(a, s, sr)["x"] for sr in ("boolean", "arithmetic", "minselect")}
        sym = algebra.submatrix_steps(a, s, "boolean", symmetric_form=True)["x"]
        sb = [set(np.nonzero(x)[0]) for x in runs["boolean"]]
        for sr in ("arithmetic", "minselect"):
            assert [set(np.nonzero(x)[0]) for x in runs[sr]] == sb
        assert [set(np.nonzero(x)[0]) for x in sym] == sb
        p1 = algebra.prop1_supports(a, s)
        assert [set(v) for v in p1] == sb[1:len(p1) + 1]


# ---- closed forms ------------------------------------------------------------------

def test_path_cycle_star_complete_tree():
    g = graphgen.path_graph(50)
    lv, pa = oracle.bfs_graph(g, 0)
    assert np.array_equal(lv, np.arange(50))
    assert np.array_equal(pa, np.r_[0, np.arange(49)])
    lv, pa = oracle.bfs_graph(g, 20)
    assert np.array_equal(lv, np.abs(np.arange(50) - 20))
    for n in (7, 8, 6):
        g = graphgen.cycle_graph(n)
        lv, pa = oracle.bfs_graph(g, 0)
        i = np.arange(n)
        assert np.array_equal(lv, np.minimum(i, n - i))
        if n % 2 == 0:
            assert pa[n // 2] == n // 2 - 1               # tie goes to the smaller index
    g = graphgen.cycle_graph(6)
    assert oracle.bfs_graph(g, 0)[1].tolist() == [0, 0, 1, 2, 5, 0]
    # 4-cycle 0-1-3-2-0 from 0: vertex 3 has parents 1 and 2 one level up
    g4 = graphgen.from_edges(4, np.array([0, 1, 3, 2]), np.array([1, 3, 2, 0]))
    assert oracle.bfs_graph(g4, 0)[1][3] == 1
    for n in (9, 33):
        g = graphgen.star_graph(n, center=4)
        lv, pa = oracle.bfs_graph(g, 4)
        assert np.all(lv[np.arange(n) != 4] == 1) and np.all(pa == 4)
        g = graphgen.complete_graph(n)
        lv, pa = oracle.bfs_graph(g, 3)
        assert np.all(lv[np.arange(n) != 3] == 1) and np.all(pa == 3)
    g = graphgen.binary_tree(127)
    lv, pa = oracle.bfs_graph(g, 0)
    v = np.arange(1, 127)
    assert np.array_equal(pa[1:], (v - 1) // 2)
    assert np.array_equal(lv, np.floor(np.log2(np.arange(127) + 1)).astype(int))


def full_grid_closed_form(w, h, s):
    """Levels and min-parents of a BFS on the complete W x H grid (row-major)."""
    r = np.arange(w * h) // w
    c = np.arange(w * h) % w
    rs, cs = s // w, s % w
    level = np.abs(r - rs) + np.abs(c - cs)
    v = np.arange(w * h)
    parent = np.where(r > rs, v - w,                           # up neighbour (smallest id)
             np.where(c > cs, v - 1,                            # left, same row band
             np.where(c < cs, v + 1,                            # right
             np.where(r < rs, v + w, v))))                      # down; source itself
    # a vertex below-left/right of the source in the same column band: min of candidates
    # candidates one level up: up (if r > rs), left (if c > cs), right (if c < cs), down (if r < rs)
    return level, parent


@pytest.mark.parametrize("w,h", [(33, 17), (64, 64)])
def test_full_grid_closed_form(w, h):
    g = graphgen.full_grid(w, h)
    rng = np.random.default_rng(5)
    for s in [0, w * h - 1, (h // 2) * w + w // 2] + list(rng.integers(0, w * h, 3)):
        lv, pa = oracle.bfs_graph(g, int(s))
        want_l, want_p = full_grid_closed_form(w, h, int(s))
        assert np.array_equal(lv, want_l)
        assert np.array_equal(pa, want_p)


# ---- operation counts (Thm 2, Thm 3, Lemma 1, the 2m remark) ------------------------------

@pytest.mark.parametrize("kind", ["er", "rmat", "grid", "rmatd"])
def test_operation_counts(kind):
    g = {"er": lambda: graphgen.erdos_renyi(3000, 6, 2),
         "rmat": lambda: graphgen.rmat(12, 8, 3),
         "grid": lambda: graphgen.grid(40, 0.8, 4),
         "rmatd": lambda: graphgen.rmat(11, 8, 5, directed=True)}[kind]()
    s = int(graphgen.pick_sources(g, 1, 9)[0])
    lv, pa = oracle.bfs_graph(g, s)
    st = oracle.component_stats(g, lv)
    l0, p0, c0 = oracle.bfs_alg2(g.n, g.ptr, g.idx, s, 0)
    l1, p1, c1 = oracle.bfs_alg2(g.n, g.ptr, g.idx, s, 1)
    assert np.array_equal(l0, lv) and np.array_equal(p0, pa)
    assert np.array_equal(l1, lv) and np.array_equal(p1, pa)
    # Thm 2: one nonzero per row -> exactly n_c - 1 multiplications
    assert c0["mults"] == st["n_c"] - 1
    # Thm 3 proof: every entry of every reached column is tested once
    assert c0["tests"] == st["nnz_c"] == c1["tests"]
    assert c0["steps"] == st["levels"]
    # Lemma 1 form: every pair (j, i) with level[i] = level[j] + 1 is multiplied
    rows = np.repeat(np.arange(g.n), np.diff(g.ptr.astype(np.int64)))
    tree_pairs = int(np.sum((lv[rows] >= 0) & (lv[g.idx] == lv[rows] + 1)))
    assert c1["mults"] == tree_pairs <= st["m_c"]
    if not g.directed:
        # the text's "all nonzeros contribute" modification multiplies m_c nonzeros
        l2, _, c2 = oracle.bfs_alg2(g.n, g.ptr, g.idx, s, 2)
        assert c2["mults"] == st["m_c"]
        assert np.array_equal(l2, lv)


def test_table2_identities():
    """Table 2's Alg 2 column is 2(n-1) on the connected com-* graphs and its SpMV
    column is 4m(D+1) (two operations per semiring step): the convention our
    counters follow (mults = n_c - 1 per search)."""
    for r in read_fixture("table1_table2.txt"):
        name, n, m, d, alg2, spmm, spmsp, spmv = r[0], *map(int, r[1:])
        assert spmv == 4 * m * (d + 1), name
        if name.startswith("com-"):
            assert alg2 == 2 * (n - 1), name
            assert spmm == 4 * m, name
        else:
            assert alg2 < 2 * (n - 1)          # road graphs: a partial component


# ---- the certificate catches planted mistakes ----------------------------------------------

def test_certificate_rejects_corruptions():
    g = graphgen.erdos_renyi(2000, 5, 3)
    s = 7
    lv, pa = oracle.bfs_graph(g, s)
    assert certify.check(g.n, g.ptr, g.idx, s, lv, pa) == []
    reached = np.nonzero(lv > 1)[0]
    v = int(reached[0])

    def bad(l, p):
        return certify.check(g.n, g.ptr, g.idx, s, l, p)

    l2 = lv.copy(); l2[v] += 1
    assert bad(l2, pa)                                       # wrong level
    p2 = pa.copy(); p2[v] = -1
    assert bad(lv, p2)                                       # I1 mismatch
    # a valid-looking parent that is not the minimum
    rows = np.repeat(np.arange(g.n), np.diff(g.ptr.astype(np.int64)))
    for u_, w_ in zip(rows, g.idx):
        cands = [u for u in g.idx[g.ptr[w_]:g.ptr[w_ + 1]] if lv[u] == lv[w_] - 1]
        if lv[w_] > 0 and len(cands) >= 2:
            p3 = pa.copy(); p3[w_] = max(cands)
            assert any(e.startswith("I4") for e in bad(lv, p3))
            break
    else:
        pytest.fail("no vertex with two candidate parents")
    p4 = pa.copy(); p4[v] = int(np.nonzero(lv == lv[v] - 1)[0][-1])
    if p4[v] != pa[v]:
        assert bad(lv, p4)                                   # non-edge or non-min parent
    l5 = lv.copy(); l5[lv == lv.max()] = -1
    p5 = pa.copy(); p5[lv == lv.max()] = -1
    assert bad(l5, p5)                                       # dropped the last level (I2)


def test_planted_oracle_mistake_is_caught(monkeypatch):
    """A max-instead-of-min parent rule (a plausible slip) fails the brute-force pin."""
    a = np.zeros((4, 4), dtype=np.int64)
    for u, v in [(0, 1), (1, 3), (3, 2), (2, 0)]:
        a[u, v] = a[v, u] = 1

    def wrong_parents(a_, s, level):
        n = a_.shape[0]
        parent = np.full(n, -1, dtype=np.int64)
        parent[s] = s
        for v in range(n):
            if level[v] > 0:
                parent[v] = max(u for u in range(n) if a_[u, v] and level[u] == level[v] - 1)
        return parent

    lv = brute.levels_by_powers(a, 0)
    assert not np.array_equal(wrong_parents(a, 0, lv), oracle.bfs_queue(4, *brute.to_csr(a)[:2], 0)[1])
