"""CPU checks of the C ABI: the library loads, exports every function that
include/bfs.h declares, and rejects malformed input before touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfs.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\**\s*(bfs_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    from paper_1906_03113_amd import _lib
    return _lib.lib()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for must in ("bfs_graph_create", "bfs_graph_destroy", "bfs_graph_info", "bfs_workspace_size",
                 "bfs_run", "bfs_run_batch", "bfs_status_string", "bfs_last_error_detail"):
        assert must in names


def test_every_declared_symbol_is_exported(L):
    for name in _declared_functions():
        assert hasattr(L, name), name


def test_status_strings(L):
    for s in range(6):
        assert L.bfs_status_string(s)
    assert L.bfs_status_string(99) == b"unknown status"


def _create(L, n, ptr, idx, in_ptr=None, in_idx=None, flags=0):
    vp = lambda a: None if a is None else np.ascontiguousarray(a, np.int32).ctypes.data_as(ctypes.c_void_p)
    keep = [np.ascontiguousarray(a, np.int32) for a in (ptr, idx) if a is not None]
    h = ctypes.c_void_p()
    rc = L.bfs_graph_create(n, vp(ptr), vp(idx), vp(in_ptr), vp(in_idx), flags, None, ctypes.byref(h))
    del keep
    return rc, h


def test_validation_errors_without_gpu(L):
    from paper_1906_03113_amd import _lib as B
    ok_ptr = np.array([0, 1, 2], np.int32)
    ok_idx = np.array([1, 0], np.int32)
    cases = [
        (0, ok_ptr, ok_idx, None, None, 0, B.BFS_EINVAL, "n = 0"),
        (-3, ok_ptr, ok_idx, None, None, 0, B.BFS_EINVAL, "n < 0"),
        (2, None, ok_idx, None, None, 0, B.BFS_EINVAL, "NULL ptr"),
        (2, np.array([1, 1, 2], np.int32), ok_idx, None, None, 0, B.BFS_ECSR, "ptr[0]"),
        (2, np.array([0, 2, 1], np.int32), ok_idx, None, None, 0, B.BFS_ECSR, "decreasing"),
        (2, ok_ptr, np.array([1, 2], np.int32), None, None, 0, B.BFS_ECSR, "idx >= n"),
        (2, ok_ptr, np.array([-1, 0], np.int32), None, None, 0, B.BFS_ECSR, "idx < 0"),
        (2, ok_ptr, ok_idx, ok_ptr, None, B.BFS_DIRECTED, B.BFS_EINVAL, "half a CSC"),
        (2, ok_ptr, ok_idx, ok_ptr, ok_idx, 0, B.BFS_EINVAL, "CSC without DIRECTED"),
        (2, ok_ptr, ok_idx, None, None, 1 << 9, B.BFS_EINVAL, "unknown flag"),
        (2, ok_ptr, ok_idx, None, None, B.BFS_MS_DEGREE_ORDER | B.BFS_MS_NO_DEGREE_ORDER, B.BFS_EINVAL,
         "degree order on and off"),
        (2, ok_ptr, ok_idx, np.array([0, 1, 3], np.int32), np.array([1, 0, 0], np.int32),
         B.BFS_DIRECTED, B.BFS_ECSR, "CSC size differs"),
        (2, ok_ptr, ok_idx, np.array([0, 0, 2], np.int32), np.array([0, 1], np.int32),
         B.BFS_DIRECTED | B.BFS_VALIDATE_TRANSPOSE, B.BFS_ECSR, "CSC not transpose"),
    ]
    for n, p, i, ip, ii, fl, want, what in cases:
        rc, h = _create(L, n, p, i, ip, ii, fl)
        assert rc == want, (what, rc, L.bfs_last_error_detail())
        assert h.value is None
        assert L.bfs_last_error_detail()


def test_null_handles(L):
    assert L.bfs_workspace_size(None, 1, 0) == 0
    assert L.bfs_graph_destroy(None) == 0
    assert L.bfs_graph_info(None, None, None, None, None) == 1
    assert L.bfs_run(None, 0, None, None, None, None, 0, None) == 1
    assert L.bfs_run_batch(0, None, None, None, None, None, None, 0, None) == 1
    assert L.bfs_run_roots(None, 1, None, None, None, None, None, 0, None) == 1
    assert L.bfs_roots_workspace_size(None, 3) == 0


def test_no_cpu_fallback_in_product_package():
    """The package never imports the oracle and has no CPU search of its own."""
    pkg = os.path.join(ROOT, "paper_1906_03113_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f


def test_compare_entry_points_reject_bad_arguments(L):
    from paper_1906_03113_amd import _lib as B
    assert L.bfs_compare_workspace_size(None) == 0
    ops = ctypes.c_uint64(7)
    steps = ctypes.c_uint32(7)
    rc = L.bfs_run_compare(None, 0, 0, None, None, None, 0, ctypes.byref(ops), ctypes.byref(steps), None)
    assert rc == B.BFS_EINVAL and L.bfs_last_error_detail()
    assert ops.value == 7 and steps.value == 7          # outputs untouched on error


def test_vertex_major_batch_rejects_bad_arguments(L):
    from paper_1906_03113_amd import _lib as B
    assert L.bfs_batch_vm_workspace_size(None, 64) == 0
    src = (ctypes.c_int32 * 2)(0, 1)
    rc = L.bfs_run_batch_vm(None, 2, src, None, None, None, None, 0, None)
    assert rc == B.BFS_EINVAL and "graph" in L.bfs_last_error_detail().decode()


def test_header_is_plain_c(tmp_path):
    """include/bfs.h is a C99 header (no C++ in the signatures), and a C
    program links the library and gets its validation errors without a GPU."""
    import shutil
    import subprocess
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "abi.c"
    src.write_text(
        '#include <stdio.h>\n#include "bfs.h"\n'
        "int main(void) {\n"
        "    bfs_graph *g = NULL;\n"
        "    int32_t ptr[3] = {0, 1, 2}, idx[2] = {1, 0};\n"
        "    bfs_status s = bfs_graph_create(0, ptr, idx, NULL, NULL, 0, NULL, &g);\n"
        "    if (s != BFS_EINVAL || g != NULL) return 1;\n"
        "    if (bfs_workspace_size(NULL, 1, 0) != 0) return 2;\n"
        '    printf("%s|%s\\n", bfs_status_string(s), bfs_last_error_detail());\n'
        "    return 0;\n}\n")
    exe = tmp_path / "abi"
    lib_dir = os.path.join(ROOT, "paper_1906_03113_amd")
    subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I",
                    os.path.join(ROOT, "include"), str(src), "-L", lib_dir, "-lbfs",
                    "-Wl,-rpath," + lib_dir, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, (r.returncode, r.stderr)
    assert "|" in r.stdout and r.stdout.split("|")[1].strip()


def test_vertex_major_binding_checks_output_shapes():
    """bfs_batch_vm refuses output tensors of the wrong shape, type or device
    before anything reaches the library (no GPU needed)."""
    import torch
    import paper_1906_03113_amd as P

    class FakeGraph:
        n = 10
        handle = None

    good = dict(dtype=torch.int32)
    for lv, pa in ((torch.empty((10, 64), **good), torch.empty((10, 64), **good)),      # host tensors
                   (torch.empty((10, 63), **good), torch.empty((10, 64), **good)),      # wrong shape
                   (torch.empty((10, 64), dtype=torch.int64), torch.empty((10, 64), **good))):
        with pytest.raises(ValueError):
            P.bfs_batch_vm(FakeGraph(), [0, 1], level=lv, parent=pa)


def test_degree_order_flags_pass_validation_without_gpu(L):
    """BFS_MS_DEGREE_ORDER / BFS_MS_NO_DEGREE_ORDER alone (and the first with a
    directed graph) pass argument validation: without a GPU the call then
    fails at its first HIP call, not with BFS_EINVAL."""
    from paper_1906_03113_amd import _lib as B
    ptr = np.array([0, 1, 2], np.int32)
    idx = np.array([1, 0], np.int32)
    for fl, ip, ii in ((B.BFS_MS_DEGREE_ORDER, None, None), (B.BFS_MS_NO_DEGREE_ORDER, None, None),
                       (B.BFS_DIRECTED | B.BFS_MS_DEGREE_ORDER, ptr, idx)):
        rc, h = _create(L, 2, ptr, idx, ip, ii, fl)
        if rc == B.BFS_OK:                         # a GPU is present after all
            L.bfs_graph_destroy(h)
            continue
        assert rc != B.BFS_EINVAL, (fl, L.bfs_last_error_detail())


def test_binding_maps_degree_order_flag(monkeypatch):
    """Graph.from_csr(ms_degree_order=...) passes the matching create flag."""
    import paper_1906_03113_amd as P
    from paper_1906_03113_amd import _lib as B
    seen = []

    class FakeLib:
        def bfs_graph_create(self, n, ptr, idx, ip, ii, flags, stream, out):
            seen.append(flags)
            return B.BFS_OK

    monkeypatch.setattr(B, "lib", lambda: FakeLib())
    monkeypatch.setattr(P, "_device_ready", lambda: None)
    ptr = np.array([0, 1, 2], np.int32)
    idx = np.array([1, 0], np.int32)
    for arg, want in ((None, 0), (True, B.BFS_MS_DEGREE_ORDER), (False, B.BFS_MS_NO_DEGREE_ORDER)):
        g = P.Graph.from_csr(2, ptr, idx, ms_degree_order=arg)
        g._h = None                                    # nothing to free
        assert seen[-1] == want, (arg, seen)
