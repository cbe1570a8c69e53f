"""Autotuner host logic on the CPU: candidate pruning, shape keys, the cache."""
import json
import types

from paper_1906_03113_amd import autotune as A


def _G(n, nnz, directed=False):
    return types.SimpleNamespace(n=n, nnz=nnz, directed=directed)


def test_candidates_include_defaults_and_respect_budget():
    for levels in (8, 7000):
        c = A.candidates(levels, budget=10, seed=1)
        assert len(c) == 10 and c[0]["grid_blocks"] == 0
        assert all(k in c[1] for k in A.SPACE)
        if levels > 64:
            assert all((x["heavy_degree"], x["chunk_edges"]) in ((512, 1024), (0, 0)) for x in c)
    assert A.candidates(8, 10, seed=1) == A.candidates(8, 10, seed=1)


def test_shape_key_buckets():
    a = A.shape_key(_G(1 << 22, 1 << 27), levels=8)
    b = A.shape_key(_G((1 << 22) + 1000, (1 << 27) + 5000), levels=9)
    c = A.shape_key(_G(1 << 22, 1 << 27), levels=5000)
    d = A.shape_key(_G(1 << 22, 1 << 27, directed=True), levels=8)
    assert a == b and a != c and a != d


def test_store_and_lookup(tmp_path):
    cache = str(tmp_path / "tune.json")
    g = _G(1 << 16, 1 << 20)
    assert A.lookup(g, 10, cache) == {}
    key = A.shape_key(g, 10)
    A.store(cache, key, {"params": {"loop": "graph", "grid_blocks": 256}, "time_s": 1.0})
    assert A.lookup(g, 12, cache) == {"loop": "graph", "grid_blocks": 256}
    assert A.lookup(_G(1 << 10, 1 << 12), 10, cache) == {}
    (tmp_path / "bad.json").write_text("{not json")
    assert A.lookup(g, 10, str(tmp_path / "bad.json")) == {}
    assert json.load(open(cache))[key]["time_s"] == 1.0


def test_selector_level_weights_and_spread():
    """Training-row weights grow with the level's best time (sqrt, clipped) and
    ignore levels with no measurement; a deep search keeps evenly spaced
    levels, first and last included."""
    import numpy as np
    from paper_1906_03113_amd import selector as S
    T = np.log(np.array([[1.0, 2.0, 3.0], [4.0, 4.0, 4.0], [100.0, 50.0, 80.0], [1e-3, 1.0, 1.0],
                         [1.0, 1.0, 1.0]]))
    M = np.ones_like(T)
    M[4] = 0.0                                            # no measurement at all
    w = S.level_weights(T, M)
    best = np.array([1.0, 4.0, 50.0, 1e-3])
    med = np.median(best)
    want = np.clip(np.sqrt(best / med), 0.25, 4.0)
    assert np.allclose(w[:4], want) and w[4] == 0.0
    lv = [{"level": i} for i in range(1000)]
    kept = S._spread(lv, 300)
    assert len(kept) == 300 and kept[0]["level"] == 0 and kept[-1]["level"] == 999
    assert all(a["level"] < b["level"] for a, b in zip(kept, kept[1:]))
    assert S._spread(lv[:10], 300) == lv[:10]


def test_batch_width_choice_and_cache(tmp_path, monkeypatch):
    """The width with the smallest measured time is cached under the shape key
    and returned by lookup_batch_width; widths above the source count or not
    a multiple of 64 are not tried."""
    import paper_1906_03113_amd as P

    class FakeGraph:
        n, nnz, directed = 1 << 20, 16 << 20, False

    monkeypatch.setattr(P, "bfs", lambda G, s, info=None, **kw: info.update(levels=7))
    tried = []

    def timer(G, sources, w):
        tried.append(w)
        return {64: 3.0, 128: 2.0, 256: 2.5}[w]

    cache = str(tmp_path / "t.json")
    r = A.tune_batch_width(FakeGraph(), list(range(200)), widths=(64, 100, 128, 256), cache=cache,
                           timer=timer)
    assert tried == [64, 128] and r["width"] == 128
    assert A.lookup_batch_width(FakeGraph(), 7, cache) == 128
    assert A.lookup_batch_width(FakeGraph(), 7, str(tmp_path / "none.json")) == 64


def test_pull_shift_choice_and_cache(tmp_path, monkeypatch):
    """The fastest pull shift is cached under the shape key and returned by
    lookup_pull_shift; shifts outside [1, 31] are not tried; cache=None
    measures without writing."""
    import paper_1906_03113_amd as P

    class FakeGraph:
        n, nnz, directed = 1 << 22, 128 << 20, False

    monkeypatch.setattr(P, "bfs", lambda G, s, info=None, **kw: info.update(levels=7))
    tried = []

    def timer(G, sources, sh):
        tried.append(sh)
        return {5: 7.0, 7: 6.9, 9: 6.8}[sh]

    cache = str(tmp_path / "t.json")
    r = A.tune_pull_shift(FakeGraph(), list(range(64)), shifts=(0, 5, 7, 9, 32), cache=cache, timer=timer)
    assert tried == [5, 7, 9] and r["shift"] == 9
    assert A.lookup_pull_shift(FakeGraph(), 7, cache) == 9
    assert A.lookup_pull_shift(FakeGraph(), 7, str(tmp_path / "none.json")) == 0
    r = A.tune_pull_shift(FakeGraph(), list(range(64)), shifts=(5,), cache=None, timer=timer)
    assert r["shift"] == 5 and A.lookup_pull_shift(FakeGraph(), 7, cache) == 9
