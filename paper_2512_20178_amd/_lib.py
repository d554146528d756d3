"""ctypes loader for libshiro.so (the gfx950 HIP library behind include/shiro.h).

There is no fallback: if the library is missing or fails to load, every call
raises.  torch is imported first so that the HIP runtime torch ships is the
one the library binds to (both carry the soname libamdhip64.so.7).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch  # noqa: F401  (loads torch's HIP runtime before the library)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libshiro.so")

SHIRO_OK = 0
ERRORS = {
    -1: "INVALID_ARG",
    -2: "BAD_CSR",
    -3: "OOM",
    -4: "HIP",
    -5: "UNSUPPORTED",
    -6: "NOT_READY",
    -7: "CAPTURING",
    -8: "WORKSPACE",
}

F32 = 0
BF16 = 1

MODE_BATCHED = 0
MODE_PER_BLOCK = 1

DB_OVERWRITE = 1
AGG_ACCUMULATE = 1
OP_SPMM = 1
OP_BACKWARD = 2
OP_PER_BLOCK = 4
OP_ROW_BASED = 8

KERNEL_SPMM = 0
KERNEL_SPMM_T = 1
KERNEL_SDDMM = 2
KERNEL_PARTIAL_C = 3
KERNEL_AGGREGATE_C = 4

CHECK_CSR = 1

# Every function include/shiro.h declares.
EXPORTS = [
    "shiro_version",
    "shiro_last_error",
    "shiro_partition",
    "shiro_partition_subset",
    "shiro_plan_info",
    "shiro_block_nnz",
    "shiro_select_rows",
    "shiro_refresh_selection",
    "shiro_plan_selection",
    "shiro_copy_selection",
    "shiro_pack_B",
    "shiro_spmm",
    "shiro_spmm_backward",
    "shiro_select_c_rows",
    "shiro_copy_c_row_selection",
    "shiro_partial_c",
    "shiro_aggregate_c",
    "shiro_mvc_bipartite",
    "shiro_joint_plan",
    "shiro_prepare",
    "shiro_autotune",
    "shiro_get_tuning",
    "shiro_set_tuning",
    "shiro_graph_begin",
    "shiro_graph_end",
    "shiro_graph_launch",
    "shiro_set_allocator",
    "shiro_plan_destroy",
    "shiro_spmm_noalloc",
    "shiro_build_hash",
]

# shiro_alloc_fn / shiro_free_fn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class ShiroError(RuntimeError):
    def __init__(self, code: int, msg: str):
        self.code = code
        self.name = ERRORS.get(code, str(code))
        super().__init__(f"shiro error {self.name} ({code}): {msg}")


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int64),
        ("n_cols", ctypes.c_int64),
        ("P", ctypes.c_int32),
        ("p", ctypes.c_int32),
        ("M", ctypes.c_int64),
        ("K", ctypes.c_int64),
        ("row_begin", ctypes.c_int64),
        ("rows", ctypes.c_int64),
        ("nz_begin", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("U", ctypes.c_int64),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("chunk", ctypes.c_int32),
        ("lanes", ctypes.c_int32),
        ("unroll", ctypes.c_int32),
        ("group_rows", ctypes.c_int32),
        ("xcd_remap", ctypes.c_int32),
        ("wg_per_cu", ctypes.c_int32),
        ("lds_rows", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lock = threading.Lock()
_lib = None

_i64, _i32, _u32, _p = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_void_p


def load(path: str = LIB_PATH):
    """Load (once) and return the library; raises if it is not built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise ImportError(
                f"{path} is missing: build it with `python -m paper_2512_20178_amd.build` "
                "(hipcc, gfx950); there is no CPU fallback"
            )
        L = ctypes.CDLL(path)
        L.shiro_version.restype = ctypes.c_int
        L.shiro_last_error.restype = ctypes.c_char_p
        L.shiro_build_hash.restype = ctypes.c_char_p
        L.shiro_partition.argtypes = [_i64, _i64, _i64, _p, _p, _i32, _i32, _u32, _p, ctypes.POINTER(_p)]
        L.shiro_plan_info.argtypes = [_p, ctypes.POINTER(PlanInfo)]
        L.shiro_block_nnz.argtypes = [_p, _p, _p]
        L.shiro_select_rows.argtypes = [_p, _p, ctypes.POINTER(_i64), _p]
        L.shiro_refresh_selection.argtypes = [_p, _p]
        L.shiro_plan_selection.argtypes = [_p, ctypes.POINTER(_p), ctypes.POINTER(_p), ctypes.POINTER(_p)]
        L.shiro_copy_selection.argtypes = [_p, _p, _p, _p, _p]
        L.shiro_pack_B.argtypes = [_p, _p, _i64, _i32, ctypes.c_int, _p, _i64, _p]
        L.shiro_spmm.argtypes = [_p, _p, _p, _i64, _i32, ctypes.c_int, _p, _i64, ctypes.c_int, _u32, _p]
        L.shiro_spmm_backward.argtypes = [_p, _p, _p, _i64, _p, _i64, _i32, ctypes.c_int, _p, _i64, _p, _i64, _p,
                                          ctypes.c_uint32, _p]
        L.shiro_select_c_rows.argtypes = [_p, _p, ctypes.POINTER(_i64), _p]
        L.shiro_copy_c_row_selection.argtypes = [_p, _p, _p, _p]
        L.shiro_partial_c.argtypes = [_p, _p, _p, _i64, _i32, ctypes.c_int, _p, _i64, ctypes.c_int, _p]
        L.shiro_aggregate_c.argtypes = [_p, _p, _i64, _i32, ctypes.c_int, _p, _i64, ctypes.c_int, _u32, _p]
        L.shiro_partition_subset.argtypes = [_i64, _i64, _i64, _p, _p, _p, ctypes.c_uint8, _i32, _i32, _u32, _p,
                                             ctypes.POINTER(_p)]
        L.shiro_mvc_bipartite.argtypes = [_i64, _i64, _i64, _p, _p, _p, _p, _p, _p, ctypes.POINTER(_i64)]
        L.shiro_joint_plan.argtypes = [_p, _p, _p, _p, _p, _i32, _p]
        L.shiro_prepare.argtypes = [_p, _i32, ctypes.c_int, _u32, _p]
        L.shiro_autotune.argtypes = [_p, _i32, ctypes.c_int, _u32, _p]
        L.shiro_get_tuning.argtypes = [_p, _i32, _i32, ctypes.c_int, ctypes.POINTER(Tuning)]
        L.shiro_set_tuning.argtypes = [_p, _i32, _i32, ctypes.c_int, ctypes.POINTER(Tuning)]
        L.shiro_graph_begin.argtypes = [_p, _p]
        L.shiro_graph_end.argtypes = [_p, _p, ctypes.POINTER(_i32)]
        L.shiro_graph_launch.argtypes = [_p, _i32, _p]
        L.shiro_set_allocator.argtypes = [ALLOC_FN, FREE_FN, _p]
        L.shiro_plan_destroy.argtypes = [_p]
        L.shiro_spmm_noalloc.argtypes = [_p, _p, _p, _i64, _i32, ctypes.c_int, _p, _i64, ctypes.c_int, _p]
        for name in EXPORTS:
            if name not in ("shiro_last_error", "shiro_build_hash"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
        return _lib


def build_hash() -> str:
    """Source hash stamped into the loaded library."""
    return load().shiro_build_hash().decode()


def check_build(strict: bool = True) -> bool:
    """True when the loaded library was built from the sources in the tree;
    with strict, a mismatch raises (the library is stale: rebuild it)."""
    from . import build as _build

    ok = build_hash() == _build.source_hash()
    if not ok and strict:
        raise ImportError(f"{LIB_PATH} was built from other sources (stamp {build_hash()}, tree "
                          f"{_build.source_hash()}): rebuild with `python -m paper_2512_20178_amd.build`")
    return ok


def check(rc: int) -> None:
    if rc != SHIRO_OK:
        msg = load().shiro_last_error()
        raise ShiroError(rc, msg.decode() if msg else "")
