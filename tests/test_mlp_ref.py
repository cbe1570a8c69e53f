"""Pins for the float64 selector-network reference: the analytic gradient
against central finite differences, the loss against a direct evaluation, and
the features against their definitions at points with known values."""
import numpy as np

from oracle import mlp_ref


def _random_problem(seed, rows=40):
    rng = np.random.default_rng(seed)
    blob = rng.normal(0, 0.4, mlp_ref.N_TOTAL)
    blob[mlp_ref.N_TRAIN:mlp_ref.N_TRAIN + 12] = rng.normal(0, 1, 12)           # mean
    blob[mlp_ref.N_TRAIN + 12:] = rng.uniform(0.5, 2.0, 12)                     # inv std
    x = rng.normal(0, 1.5, (rows, 12))
    t = rng.normal(0, 1, (rows, 3))
    m = (rng.random((rows, 3)) < 0.8).astype(np.float64)
    return blob, x, t, m, 1.0 / max(1.0, m.sum())


def test_gradient_matches_finite_differences():
    blob, x, t, m, inv = _random_problem(1)
    g = mlp_ref.grad(blob, x, t, m, inv)
    assert g.shape == (mlp_ref.N_TRAIN,)
    h = 1e-6
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(mlp_ref.N_TRAIN, 200, replace=False),
                          np.arange(mlp_ref.N_TRAIN - 3, mlp_ref.N_TRAIN)])       # incl. b3
    for i in idx:
        bp, bm = blob.copy(), blob.copy()
        bp[i] += h
        bm[i] -= h
        fd = (mlp_ref.loss(bp, x, t, m, inv) - mlp_ref.loss(bm, x, t, m, inv)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_loss_and_masking():
    blob, x, t, m, inv = _random_problem(3, rows=5)
    y, _ = mlp_ref.forward(blob, x)
    direct = sum(m[r, u] * (y[r, u] - t[r, u]) ** 2 for r in range(5) for u in range(3)) * inv
    assert np.isclose(mlp_ref.loss(blob, x, t, m, inv), direct)
    # a fully masked row contributes nothing to the loss or the gradient
    m2 = m.copy()
    m2[0] = 0
    t2 = t.copy()
    t2[0] += 100.0
    assert np.isclose(mlp_ref.loss(blob, x, t2, m2, inv), mlp_ref.loss(blob, x, t, m2, inv))
    assert np.allclose(mlp_ref.grad(blob, x, t2, m2, inv), mlp_ref.grad(blob, x, t, m2, inv))


def test_identity_network():
    """A hand-built network: y_u = relu(x_u) for u < 3 with x = features (mean 0,
    inv std 1) and positive inputs - checks the layer order and layouts."""
    blob = np.zeros(mlp_ref.N_TOTAL)
    p = {}
    off = 0
    for name, shape in mlp_ref.SIZES:
        p[name] = (off, shape)
        off += int(np.prod(shape))
    W1 = np.zeros((32, 12)); W1[0, 0] = W1[1, 1] = W1[2, 2] = 1
    W2 = np.zeros((32, 32)); W2[0, 0] = W2[1, 1] = W2[2, 2] = 1
    W3 = np.zeros((3, 32)); W3[0, 0] = W3[1, 1] = W3[2, 2] = 1
    for name, val in (("W1", W1), ("W2", W2), ("W3", W3)):
        o, shape = p[name]
        blob[o:o + val.size] = val.ravel()
    blob[mlp_ref.N_TRAIN + 12:] = 1.0
    x = np.array([[0.5, 2.0, -1.0] + [0.0] * 9])
    y, _ = mlp_ref.forward(blob, x)
    assert np.allclose(y, [[0.5, 2.0, 0.0]])


def test_features_definition():
    f = mlp_ref.features(frontier=[9], frontier_edges=[99], unvisited=[49], unvisited_edges=[999],
                         level=[3], n=100, nnz=1000)[0]
    want = [np.log(10), np.log(100), np.log(50), np.log(1000), np.log(4), 10.0,
            np.log(0.1), np.log(100 / 1001), np.log(0.5), np.log(1000 / 1001),
            np.log(100 / 1000), np.log(10 / 50)]
    assert np.allclose(f, want)
