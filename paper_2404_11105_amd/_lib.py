"""ctypes loader for libxminer.so (the C ABI of include/xminer.h).

The shared library must have been built (paper_2404_11105_amd.build); this
module never builds it and there is no fallback: every count runs in the
library's HIP kernels.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libxminer.so")

XM_OK = 0
XM_ERR_INVALID = -1
XM_ERR_PATTERN = -2
XM_ERR_OOM = -3
XM_ERR_HIP = -4
XM_ERR_OVERFLOW = -5
XM_ERR_WORKSPACE = -6
XM_ERR_CANCELLED = -7
XM_ERR_GRAPH = -8

XM_MEM_DEVICE = 0x1
XM_MEM_HOST = 0x2
XM_ORDER_BY_DEGREE = 0x8
XM_VALIDATE = 0x4
XM_PLAN_REDUCED = 0x1
XM_PLAN_UNREDUCED = 0x2
XM_PLAN_SYMMETRY = 0x4
XM_PLAN_SYM_BELOW = 0x8


def XM_PLAN_ROOT(v: int) -> int:
    return (v + 1) << 8


def XM_PLAN_ROOT_SHARE(s: int) -> int:
    return (int(s) & 0xFF) << 16


class XmCountOpts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("chunk", ctypes.c_uint32),
        ("split", ctypes.c_uint32),
        ("cap", ctypes.c_uint32),
        ("waves_per_cu", ctypes.c_uint32),
        ("roots_dev", ctypes.c_void_p),
        ("n_roots", ctypes.c_uint32),
        ("reserved0", ctypes.c_uint32),
        ("cancel_dev", ctypes.c_void_p),
        ("split_work", ctypes.c_uint32),
        ("merge_min", ctypes.c_uint32),
        ("merge_ratio", ctypes.c_uint32),
        ("ev_kernel_start", ctypes.c_void_p),
        ("ev_kernel_stop", ctypes.c_void_p),
        ("roots_host", ctypes.c_void_p),
        ("list_dev", ctypes.c_void_p),
        ("list_cap", ctypes.c_uint64),
        ("list_count_dev", ctypes.c_void_p),
    ]


class XminerError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


EXPORTS = [
    "xm_load_graph", "xm_free_graph", "xm_graph_info", "xm_graph_node_order", "xm_graph_dense_rows", "xm_graph_dense_rows_info",
    "xm_plan", "xm_plan_describe",
    "xm_plan_root_vertex", "xm_free_plan", "xm_plan_work", "xm_plan_traffic", "xm_workspace_size", "xm_count",
    "xm_count_static", "xm_count_capture",
    "xm_exec_launch", "xm_free_exec", "xm_strerror", "xm_last_error", "xm_version",
]

_lib = None


def lib():
    """Load libxminer.so once; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2404_11105_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, U32, SZ = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_size_t
        L.xm_load_graph.argtypes = [U32, U32, P, P, P, P, U32, P, ctypes.POINTER(P)]
        L.xm_free_graph.argtypes = [P]
        L.xm_graph_info.argtypes = [P, P, P, P, P]
        L.xm_graph_node_order.argtypes = [P, P]
        L.xm_graph_dense_rows.argtypes = [P, ctypes.c_uint64, U32, P, P]
        L.xm_graph_dense_rows_info.argtypes = [P, P, P, P, P]
        L.xm_plan.argtypes = [U32, U32, P, U32, P, ctypes.POINTER(P)]
        L.xm_plan_describe.argtypes = [P, ctypes.c_char_p, SZ, ctypes.POINTER(SZ)]
        L.xm_plan_root_vertex.argtypes = [P]
        L.xm_free_plan.argtypes = [P]
        L.xm_plan_work.argtypes = [U32, P, P, P, P, P, P, U32, U32, ctypes.c_uint64, P]
        L.xm_plan_traffic.argtypes = [U32, P, P, P, P, P, P, U32, U32, U32, ctypes.c_uint64, P]
        L.xm_workspace_size.argtypes = [P, U32, P, P]
        L.xm_workspace_size.restype = SZ
        L.xm_count.argtypes = [P, U32, P, P, P, SZ, P, P, P]
        L.xm_count_static.argtypes = [P, U32, P, P, P, P, P]
        L.xm_count_capture.argtypes = [P, U32, P, P, P, SZ, P, P, P, ctypes.POINTER(P)]
        L.xm_exec_launch.argtypes = [P, P]
        L.xm_free_exec.argtypes = [P]
        L.xm_strerror.argtypes = [ctypes.c_int]
        L.xm_strerror.restype = ctypes.c_char_p
        L.xm_last_error.restype = ctypes.c_char_p
        L.xm_version.restype = ctypes.c_char_p
        for name in ["xm_load_graph", "xm_free_graph", "xm_graph_info", "xm_graph_dense_rows",
                     "xm_graph_dense_rows_info", "xm_plan",
                     "xm_plan_describe", "xm_plan_root_vertex", "xm_free_plan", "xm_plan_work",
                     "xm_plan_traffic", "xm_count", "xm_count_static",
                     "xm_count_capture", "xm_exec_launch", "xm_free_exec"]:
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(code: int) -> int:
    if code < 0:
        L = lib()
        raise XminerError(code, f"{L.xm_strerror(code).decode()}: {L.xm_last_error().decode()}")
    return code
