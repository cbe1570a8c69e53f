"""The variant selector on the GPU: its forward / gradient kernels against the
float64 reference, training, per-level profiling, and that no set of weights
can change a search result."""
import os

import numpy as np
import pytest

import graphgen
from oracle import mlp_ref
from tests.gpu_common import assert_same, need_gpu, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    return need_gpu()


def _problem(seed, rows=3000):
    rng = np.random.default_rng(seed)
    blob = rng.normal(0, 0.3, mlp_ref.N_TOTAL)
    blob[mlp_ref.N_TRAIN:mlp_ref.N_TRAIN + 12] = rng.normal(0, 1, 12)
    blob[mlp_ref.N_TRAIN + 12:] = rng.uniform(0.5, 1.5, 12)
    X = rng.normal(0, 2, (rows, 12))
    T = rng.normal(0, 1, (rows, 3))
    M = (rng.random((rows, 3)) < 0.85).astype(np.float64)
    return blob.astype(np.float32), X.astype(np.float32), T.astype(np.float32), M.astype(np.float32)


def test_forward_matches_reference(P):
    from paper_1906_03113_amd import selector as S
    blob, X, _, _ = _problem(1)
    say("[selector] forward")
    y = S.predict(blob, X)
    want, _ = mlp_ref.forward(blob.astype(np.float64), X.astype(np.float64))
    scale = np.abs(want).max()
    assert np.abs(y - want).max() <= 1e-4 * scale + 1e-5


def test_gradient_matches_reference(P):
    from paper_1906_03113_amd import selector as S
    blob, X, T, M = _problem(2)
    inv = 1.0 / M.sum()
    tr = S.Trainer(blob, X, T, M)
    say("[selector] gradient")
    loss = tr.gradient()
    g = tr.grad.cpu().numpy()[:mlp_ref.N_TRAIN].astype(np.float64)
    want = mlp_ref.grad(blob.astype(np.float64), X.astype(np.float64), T.astype(np.float64),
                        M.astype(np.float64), inv)
    assert np.isclose(loss, mlp_ref.loss(blob.astype(np.float64), X.astype(np.float64),
                                         T.astype(np.float64), M.astype(np.float64), inv), rtol=1e-4)
    err = np.abs(g - want).max() / np.abs(want).max()
    cos = float(g @ want / (np.linalg.norm(g) * np.linalg.norm(want)))
    assert err <= 1e-3 and cos >= 0.9999, (err, cos)
    assert np.all(tr.grad.cpu().numpy()[mlp_ref.N_TRAIN:] == 0)       # normalisation not trained


def test_training_reduces_loss(P):
    from paper_1906_03113_amd import selector as S
    rng = np.random.default_rng(3)
    X = rng.normal(0, 1, (2000, 12))
    T = np.stack([X[:, 0] - X[:, 1], np.sin(X[:, 2]), 0.5 * X[:, 3] ** 2], axis=1)
    M = np.ones_like(T)
    blob0 = S.init_weights(X, seed=1)
    inv = 1.0 / M.sum()
    l0 = mlp_ref.loss(blob0.astype(np.float64), X, T, M, inv)
    say("[selector] training")
    w = S.train(X, T, M, steps=600, lr=5e-3)
    l1 = mlp_ref.loss(w.astype(np.float64), X, T, M, inv)
    assert l1 < 0.1 * l0, (l0, l1)


@pytest.mark.parametrize("kind", ["random", "nan", "trained"])
def test_weights_never_change_results(P, kind):
    import torch
    from paper_1906_03113_amd import selector as S
    if kind == "trained":
        if not os.path.exists(S.DEFAULT_WEIGHTS):
            pytest.skip("no trained weights in the tree")
        w = S.load_weights()
    else:
        blob, _, _, _ = _problem(4 if kind == "random" else 5)
        if kind == "nan":
            blob[:50] = np.nan                         # hidden units: ReLU maps NaN to 0
            blob[mlp_ref.N_TRAIN - 3] = np.nan         # an output bias: a NaN prediction
        w = torch.tensor(blob, device="cuda")
    for name, g in (("rmat14", graphgen.rmat(14, 16, 2)), ("rmatd13", graphgen.rmat(13, 16, 3, directed=True)),
                    ("grid96", graphgen.grid(96, 0.9, 5))):
        G = P.Graph.from_graphgen(g)
        for s in graphgen.pick_sources(g, 2, 8):
            say(f"[selector] {kind} weights {name} s={s}")
            info = {}
            lv, pa = P.bfs(G, int(s), variant="learned", selector=w, trace=True, info=info)
            torch.cuda.synchronize()
            assert_same(g, int(s), (lv.cpu().numpy(), pa.cpu().numpy()), f"{kind}/{name}")
            if kind == "nan":
                assert all(r["variant"] == "push" for r in info["trace"])


def test_profile_levels(P):
    from paper_1906_03113_amd import selector as S
    import torch
    g = graphgen.rmat(13, 16, 6)
    G = P.Graph.from_graphgen(g)
    s = int(graphgen.pick_sources(g, 1, 2)[0])
    say("[selector] profile_levels")
    lv = S.profile(G, s, reps=1)
    import oracle
    want_l, _ = oracle.bfs_graph(g, s)
    assert len(lv) == int(want_l.max()) + 1
    for d in lv:
        assert all(np.isfinite(t) and t > 0 for t in d["times"])
        assert d["frontier"] == int((want_l == d["level"]).sum())
    X, T, M = S.dataset(lv, g.n, g.nnz)
    assert X.shape == (len(lv), 12) and M.all()
    want_X = mlp_ref.features([d["frontier"] for d in lv], [d["frontier_edges"] for d in lv],
                              [d["unvisited"] for d in lv], [d["unvisited_edges"] for d in lv],
                              [d["level"] for d in lv], g.n, g.nnz)
    assert np.allclose(X, want_X)


def test_trained_selector_gains_over_push(P):
    """On held-out R-MAT graphs the trained network's per-level choices cost
    less device time than push on every level (exhaustive per-level timing)."""
    from paper_1906_03113_amd import selector as S
    if not os.path.exists(S.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights in the tree")
    import json
    w = np.asarray(json.load(open(S.DEFAULT_WEIGHTS))["weights"], np.float32)
    Xs, Ts, Ms = [], [], []
    for scale in (15, 16):
        g = graphgen.rmat(scale, 16, 4242 + scale)
        G = P.Graph.from_graphgen(g)
        for s in graphgen.pick_sources(g, 2, 9):
            say(f"[selector] gain rmat{scale} s={s}")
            X, T, M = S.dataset(S.profile(G, int(s), reps=2), g.n, g.nnz)
            Xs.append(X); Ts.append(T); Ms.append(M)
    X, T, M = np.concatenate(Xs), np.concatenate(Ts), np.concatenate(Ms)
    r = S.regret(S.choose(w, X), T, M)
    say(f"[selector] held-out: {r}")
    assert r["chosen_us"] < r["push_us"], r
