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


def check_all(g, sources, fetch, tag, workers=16):
    """Every query against the oracle: fetch(q) -> (level, parent) host arrays
    of query q.  The oracle runs for 16 sources at a time in host threads (its
    C search releases the interpreter lock), beside the comparisons."""
    from concurrent.futures import ThreadPoolExecutor
    ip, ii = g.csc()
    with ThreadPoolExecutor(workers) as ex:
        for base in range(0, len(sources), workers):
            qs = list(range(base, min(base + workers, len(sources))))
            futs = {q: ex.submit(oracle.bfs_queue, g.n, g.ptr, g.idx, int(sources[q]), ip, ii) for q in qs}
            for q in qs:
                lv, pa = fetch(q)
                wl, wp = futs[q].result()
                if not np.array_equal(lv, wl):
                    bad = np.nonzero(lv != wl)[0]
                    raise AssertionError(f"{tag} q{q} s={sources[q]}: level differs at {len(bad)} vertices, "
                                         f"first {bad[:5]}")
                if not np.array_equal(pa, wp):
                    bad = np.nonzero(pa != wp)[0]
                    raise AssertionError(f"{tag} q{q} s={sources[q]}: parent differs at {len(bad)} vertices, "
                                         f"first {bad[:5]}")


def oracle_all(g, sources, workers=16):
    """The oracle's search from every source, in host threads."""
    from concurrent.futures import ThreadPoolExecutor
    ip, ii = g.csc()
    with ThreadPoolExecutor(workers) as ex:
        return list(ex.map(lambda s: oracle.bfs_queue(g.n, g.ptr, g.idx, int(s), ip, ii), sources))


def compare_all(want, sources, fetch, tag):
    """Every query q against the oracle's result want[q] (see oracle_all)."""
    for q, (wl, wp) in enumerate(want):
        lv, pa = fetch(q)
        if not (np.array_equal(lv, wl) and np.array_equal(pa, wp)):
            bl = np.nonzero(lv != wl)[0]
            bp = np.nonzero(pa != wp)[0]
            raise AssertionError(f"{tag} q{q} s={sources[q]}: level differs at {len(bl)}, parent at "
                                 f"{len(bp)} vertices (first {bl[:3]} / {bp[:3]})")
