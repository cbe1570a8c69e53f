"""Helpers for the GPU parity tests: run the HIP path and the oracle on the same input."""
import sys

import numpy as np
import pytest

import graphgen
import oracle
from oracle import certify


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1906_03113_amd as P
    P._lib.lib()          # raises if the HIP library is not built: no fallback
    return P


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(P, G, s, **kw):
    import torch
    lv, pa = P.bfs(G, int(s), **kw)
    torch.cuda.synchronize()
    return lv.cpu().numpy(), pa.cpu().numpy()


def assert_same(g, s, got, tag=""):
    """Bit-exact comparison with the oracle (O-A) plus the certificate."""
    lv, pa = got
    want_l, want_p = oracle.bfs_graph(g, int(s))
    if not np.array_equal(lv, want_l):
        bad = np.nonzero(lv != want_l)[0]
        raise AssertionError(f"{tag} level mismatch at {len(bad)} vertices, first {bad[:5]}: "
                             f"got {lv[bad[:5]]} want {want_l[bad[:5]]}")
    if not np.array_equal(pa, want_p):
        bad = np.nonzero(pa != want_p)[0]
        raise AssertionError(f"{tag} parent mismatch at {len(bad)} vertices, first {bad[:5]}: "
                             f"got {pa[bad[:5]]} want {want_p[bad[:5]]}")
    assert certify.check(g.n, g.ptr, g.idx, int(s), lv, pa) == [], tag
