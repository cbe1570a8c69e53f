"""ctypes binding of libbfs.so (include/bfs.h).  Argument marshalling only:
every step of the search runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbfs.so")

BFS_OK, BFS_EINVAL, BFS_ERANGE, BFS_ECSR, BFS_ENOMEM, BFS_EHIP = range(6)
BFS_DIRECTED, BFS_INPUT_ON_DEVICE, BFS_VALIDATE_TRANSPOSE = 1, 2, 4
BFS_MS_DEGREE_ORDER, BFS_MS_NO_DEGREE_ORDER = 8, 16
VARIANTS = {"push": 0, "pull": 1, "bitmap": 2, "learned": 3, "heuristic": 4, "short_circuit": 5}
VARIANT_NAMES = {v: k for k, v in VARIANTS.items()}
LOOPS = {"host": 0, "graph": 1, "persistent": 2}
PUSH_IMPLS = {"auto": 0, "list": 1, "sliced": 2, "claim": 3}
COMPARE = {"spmv": 0, "spmspv": 1, "spmmspv": 2}
SEMIRINGS = {"boolean": 0, "arithmetic": 1, "min_plus": 2, "min_select": 3}


class LevelRecord(ctypes.Structure):
    _fields_ = [("level", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("frontier", ctypes.c_uint32), ("unvisited", ctypes.c_uint32),
                ("frontier_edges", ctypes.c_uint64), ("unvisited_edges", ctypes.c_uint64),
                ("time_us", ctypes.c_float), ("reserved", ctypes.c_float)]


class RunOptions(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_uint32), ("loop_mode", ctypes.c_uint32),
                ("levels_per_sync", ctypes.c_uint32), ("grid_blocks", ctypes.c_uint32),
                ("heavy_degree", ctypes.c_uint32), ("chunk_edges", ctypes.c_uint32),
                ("ms_pull_shift", ctypes.c_uint32), ("selector", ctypes.c_void_p),
                ("trace", ctypes.POINTER(LevelRecord)), ("trace_capacity", ctypes.c_uint32),
                ("time_kernels", ctypes.c_uint32), ("trace_count", ctypes.c_uint32),
                ("levels", ctypes.c_uint32), ("launches", ctypes.c_uint32),
                ("kernel_us", ctypes.c_float), ("push_impl", ctypes.c_uint32),
                ("init_us", ctypes.c_float), ("ms_ranges", ctypes.c_uint32),
                ("push_used", ctypes.c_uint32), ("count_atomics", ctypes.c_uint32),
                ("reserved0", ctypes.c_uint32), ("atomics", ctypes.c_uint64)]


class BfsError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"bfs status {status}: {detail}")
        self.status = status
        self.detail = detail


_lib = None


def lib():
    """Load libbfs.so; raise if it is not built (there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1906_03113_amd.build` "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    L.bfs_graph_create.argtypes = [i32, vp, vp, vp, vp, u32, vp, ctypes.POINTER(vp)]
    L.bfs_graph_destroy.argtypes = [vp]
    L.bfs_graph_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_int64),
                                 ctypes.POINTER(i32), ctypes.POINTER(sz)]
    L.bfs_workspace_size.argtypes = [vp, i32, u32]
    L.bfs_workspace_size.restype = sz
    L.bfs_run.argtypes = [vp, i32, vp, vp, ctypes.POINTER(RunOptions), vp, sz, vp]
    L.bfs_run_batch.argtypes = [i32, vp, vp, vp, vp, ctypes.POINTER(RunOptions), vp, sz, vp]
    L.bfs_run_roots.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(RunOptions), vp, sz, vp]
    L.bfs_roots_workspace_size.argtypes = [vp, i32]
    L.bfs_roots_workspace_size.restype = sz
    L.bfs_batch_workspace_size.argtypes = [i32, vp]
    L.bfs_batch_workspace_size.restype = sz
    L.bfs_status_string.argtypes = [i32]
    L.bfs_status_string.restype = ctypes.c_char_p
    L.bfs_last_error_detail.argtypes = []
    L.bfs_last_error_detail.restype = ctypes.c_char_p
    for name in ("bfs_graph_create", "bfs_graph_destroy", "bfs_graph_info", "bfs_run",
                 "bfs_run_batch", "bfs_run_roots"):
        getattr(L, name).restype = i32
    _optional(L)
    _lib = L
    return L


def _optional(L):
    """Entry points of the variant selector (same library)."""
    vp, i32, u32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_size_t
    L.bfs_selector_param_count.argtypes = []
    L.bfs_selector_param_count.restype = i32
    L.bfs_selector_forward.argtypes = [vp, vp, vp, i32, vp]
    L.bfs_selector_forward.restype = i32
    L.bfs_selector_grad.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, vp, vp, vp]
    L.bfs_selector_grad.restype = i32
    L.bfs_selector_adam.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, vp]
    L.bfs_selector_adam.restype = i32
    L.bfs_profile_snapshot_size.argtypes = [vp]
    L.bfs_profile_snapshot_size.restype = sz
    L.bfs_profile_levels.argtypes = [vp, i32, vp, vp, vp, sz, vp, sz, i32,
                                     ctypes.POINTER(LevelRecord), u32, ctypes.POINTER(u32), vp]
    L.bfs_profile_levels.restype = i32
    L.bfs_ms_profile_snapshot_size.argtypes = [vp, i32]
    L.bfs_ms_profile_snapshot_size.restype = sz
    L.bfs_ms_profile_levels.argtypes = [vp, i32, vp, vp, vp, vp, sz, vp, sz, i32,
                                        ctypes.POINTER(LevelRecord), u32, ctypes.POINTER(u32), vp]
    L.bfs_ms_profile_levels.restype = i32
    L.bfs_batch_vm_workspace_size.argtypes = [vp, i32]
    L.bfs_batch_vm_workspace_size.restype = sz
    L.bfs_run_batch_vm.argtypes = [vp, i32, vp, vp, vp, ctypes.POINTER(RunOptions), vp, sz, vp]
    L.bfs_run_batch_vm.restype = i32
    L.bfs_compare_workspace_size.argtypes = [vp]
    L.bfs_compare_workspace_size.restype = sz
    L.bfs_run_compare.argtypes = [vp, i32, u32, vp, vp, vp, sz, ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(u32), vp]
    L.bfs_run_compare.restype = i32
    L.bfs_spmspv_workspace_size.argtypes = [vp, i32]
    L.bfs_spmspv_workspace_size.restype = sz
    L.bfs_masked_spmspv.argtypes = [vp, u32, vp, vp, i32, vp, vp, u32, vp, vp,
                                    ctypes.POINTER(i32), vp, sz, vp]
    L.bfs_masked_spmspv.restype = i32
    L.bfs_graph_set_slice_words.argtypes = [vp, u32]
    L.bfs_graph_set_slice_words.restype = i32
    L.bfs_run_static.argtypes = [vp, i32, vp, vp, u32, vp]
    L.bfs_run_static.restype = i32


def check(status: int) -> None:
    if status != BFS_OK:
        detail = lib().bfs_last_error_detail().decode(errors="replace")
        raise BfsError(status, detail)
