"""The allocation-free entry point (bfs_run_static) through the C ABI: its
results equal bfs_run's (and the oracle's) bit for bit, on two calls in a row
on one GPU, the second on a smaller graph; graphs above its limit are refused."""
import ctypes

import numpy as np
import pytest

import graphgen
import oracle
from tests.gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


def _static(P, G, s):
    """Call bfs_run_static directly through the C ABI."""
    import torch
    L = P._lib.lib()
    lv = torch.full((G.n,), 7, dtype=torch.int32, device="cuda")    # garbage the call must overwrite
    pa = torch.full((G.n,), 7, dtype=torch.int32, device="cuda")
    st = L.bfs_run_static(G.handle, int(s), ctypes.c_void_p(lv.data_ptr()),
                          ctypes.c_void_p(pa.data_ptr()), 0,
                          ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream)))
    assert st == 0, L.bfs_last_error_detail().decode()
    torch.cuda.synchronize()
    return lv.cpu().numpy(), pa.cpu().numpy()


def _run(P, G, s):
    import torch
    lv, pa = P.bfs(G, int(s), variant="push")
    torch.cuda.synchronize()
    return lv.cpu().numpy(), pa.cpu().numpy()


def test_static_equals_bfs_run_twice_smaller_second():
    P = need_gpu()
    big = graphgen.rmat(16, 16, 8)                   # 65,536 vertices, two slices' worth of words
    small = graphgen.erdos_renyi(3000, 5, 2)
    Gb = P.Graph.from_graphgen(big)
    Gs = P.Graph.from_graphgen(small)
    Gb.set_slice_words(1024)                         # a 2-slice cut on the big graph
    for name, g, G in (("rmat16", big, Gb), ("er3000", small, Gs)):
        for s in graphgen.pick_sources(g, 2, 11):
            say(f"[static] {name} s={s}")
            got = _static(P, G, s)
            ref = _run(P, G, s)
            assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), name
            want_l, want_p = oracle.bfs_graph(g, int(s))
            assert np.array_equal(got[0], want_l) and np.array_equal(got[1], want_p), name


def test_static_refuses_too_large():
    P = need_gpu()
    import torch
    n = 4 * 32768 * 32 + 1                           # one vertex past the limit
    g = graphgen.path_graph(n)
    G = P.Graph.from_graphgen(g)
    L = P._lib.lib()
    lv = torch.empty(n, dtype=torch.int32, device="cuda")
    say("[static] path n=2^22+1 refused")
    st = L.bfs_run_static(G.handle, 0, ctypes.c_void_p(lv.data_ptr()), ctypes.c_void_p(lv.data_ptr()),
                          0, None)
    assert st == P._lib.BFS_EINVAL
    assert b"at most" in L.bfs_last_error_detail()
