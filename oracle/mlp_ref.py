"""Float64 reference of the variant-selector network (forward, loss, gradient).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written from the
network's definition, independently of the HIP kernels:

  blob = W1[32][12] b1[32] W2[32][32] b2[32] W3[3][32] b3[3] mean[12] inv_std[12]
  x    = (features - mean) * inv_std
  h1   = relu(W1 x + b1),  h2 = relu(W2 h1 + b2),  y = W3 h2 + b3
  loss = inv_norm * sum(mask * (y - t)^2)

`grad` is the analytic gradient with respect to the weights and biases (the
normalisation constants are not trained).  The test suite pins it with
central finite differences.

Level features (the selector's input), from the level's frontier F, the
unvisited remainder U, the level k and the graph's n and nnz:
  log(1+|F|), log(1+sumdeg F), log(1+|U|), log(1+sumdeg U), log(1+k), nnz/n,
  log((|F|+1)/n), log((sumdeg F+1)/(nnz+1)), log((|U|+1)/n),
  log((sumdeg U+1)/(nnz+1)), log((sumdeg F+1)/(sumdeg U+1)), log((|F|+1)/(|U|+1))
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT = 12, 32, 3
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_TRAIN = sum(int(np.prod(s)) for _, s in SIZES)       # 1571
N_TOTAL = N_TRAIN + 2 * N_IN                           # + mean, inv_std


def unpack(blob):
    blob = np.asarray(blob, dtype=np.float64)
    out, off = {}, 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = blob[off:off + size].reshape(shape)
        off += size
    out["mean"] = blob[off:off + N_IN]
    out["istd"] = blob[off + N_IN:off + 2 * N_IN]
    return out


def features(frontier, frontier_edges, unvisited, unvisited_edges, level, n, nnz):
    f = np.asarray(frontier, np.float64)
    sf = np.asarray(frontier_edges, np.float64)
    u = np.asarray(unvisited, np.float64)
    su = np.asarray(unvisited_edges, np.float64)
    k = np.asarray(level, np.float64)
    n = np.broadcast_to(np.asarray(n, np.float64), f.shape)
    nnz = np.broadcast_to(np.asarray(nnz, np.float64), f.shape)
    cols = [np.log1p(f), np.log1p(sf), np.log1p(u), np.log1p(su), np.log1p(k), nnz / n,
            np.log((f + 1) / n), np.log((sf + 1) / (nnz + 1)), np.log((u + 1) / n),
            np.log((su + 1) / (nnz + 1)), np.log((sf + 1) / (su + 1)), np.log((f + 1) / (u + 1))]
    return np.stack(cols, axis=-1)


def forward(blob, feats):
    p = unpack(blob)
    x = (np.asarray(feats, np.float64) - p["mean"]) * p["istd"]
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (x, z1, h1, z2, h2)


def loss(blob, feats, targets, mask, inv_norm):
    y, _ = forward(blob, feats)
    return float(inv_norm * np.sum(np.asarray(mask) * (y - np.asarray(targets)) ** 2))


def grad(blob, feats, targets, mask, inv_norm):
    """d loss / d (W1, b1, W2, b2, W3, b3), flattened in blob order (N_TRAIN values)."""
    p = unpack(blob)
    y, (x, z1, h1, z2, h2) = forward(blob, feats)
    dy = 2.0 * inv_norm * np.asarray(mask) * (y - np.asarray(targets))
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dh2 = dy @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
