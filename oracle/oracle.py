"""ctypes wrapper around oracle/xm_oracle.c (test infrastructure only).

The oracle counts injective, direction-preserving, non-induced maps of a
pattern into a digraph by plain backtracking (the paper, section 2,
Definitions 2.1-2.2; section 5.3).  See the C file's header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "xm_oracle.c")
LIB_PATH = os.path.join(HERE, "libxm_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/libxm_oracle.so."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-Wall", "-shared", "-fPIC", "-pthread",
                               SRC, "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        lib.xmo_count.argtypes = [ctypes.c_uint32, P, P, ctypes.c_int, ctypes.c_int, P,
                                  P, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                  P, P, P, ctypes.c_int, P]
        lib.xmo_count.restype = ctypes.c_int
        lib.xmo_list.argtypes = [ctypes.c_uint32, P, P, ctypes.c_int, ctypes.c_int, P,
                                 P, ctypes.c_uint64, ctypes.c_int, P, ctypes.c_uint64, P, P]
        lib.xmo_list.restype = ctypes.c_int
        lib.xmo_prepare.argtypes = [ctypes.c_uint32, P, P]
        lib.xmo_prepare.restype = ctypes.c_void_p
        lib.xmo_count_prepared.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P, ctypes.c_uint64, ctypes.c_int,
                                           ctypes.c_int, P, P, P, ctypes.c_int, P]
        lib.xmo_count_prepared.restype = ctypes.c_int
        lib.xmo_release.argtypes = [P]
        lib.xmo_release.restype = None
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _call(graph, pattern, roots, mode, threads, per_root, root_vertex=-1):
    lib = _load()
    out_off = np.ascontiguousarray(graph.out_off, dtype=np.uint32)
    out_adj = np.ascontiguousarray(graph.out_adj, dtype=np.uint32)
    if out_adj.size == 0:
        out_adj = np.zeros(1, dtype=np.uint32)
    arcs = np.frombuffer(pattern.arcs_u8(), dtype=np.uint8).copy()
    if arcs.size == 0:
        arcs = np.zeros(2, dtype=np.uint8)
    r = None if roots is None else np.ascontiguousarray(roots, dtype=np.uint32)
    nr = 0 if r is None else int(r.size)
    pr = np.zeros(2 * (nr if r is not None else graph.n), dtype=np.uint64) if per_root else None
    lo = ctypes.c_uint64(0)
    hi = ctypes.c_uint64(0)
    first = ctypes.c_int(-1)
    rc = lib.xmo_count(graph.n, _ptr(out_off), _ptr(out_adj), pattern.k, len(pattern.arcs),
                       _ptr(arcs), _ptr(r), nr, {"A": 0, "B": 1}[mode], threads,
                       ctypes.byref(lo), ctypes.byref(hi), _ptr(pr), int(root_vertex),
                       ctypes.byref(first))
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    total = lo.value | (hi.value << 64)
    return total, pr, first.value


def count(graph, pattern, roots=None, mode: str = "A", threads: int = 1,
          root_vertex: int = -1) -> int:
    """Exact embedding count (Python int).

    roots (optional) restricts the image of the first pattern vertex, which is
    root_vertex when given (>= 0), else the oracle's own choice."""
    return _call(graph, pattern, roots, mode, threads, False, root_vertex)[0]


def count_per_root(graph, pattern, roots=None, mode: str = "A", threads: int = 1,
                   root_vertex: int = -1):
    """(total, per_root list of ints, first pattern vertex in the oracle's order)."""
    total, pr, first = _call(graph, pattern, roots, mode, threads, True, root_vertex)
    per = [int(pr[2 * i]) | (int(pr[2 * i + 1]) << 64) for i in range(pr.size // 2)]
    return total, per, first


def list_embeddings(graph, pattern, cap: int, roots=None, root_vertex: int = -1):
    """(total, array [min(total, cap), k] of embeddings): row = phi of pattern
    vertices 0..k-1, in the oracle's enumeration order."""
    lib = _load()
    out_off = np.ascontiguousarray(graph.out_off, dtype=np.uint32)
    out_adj = np.ascontiguousarray(graph.out_adj, dtype=np.uint32)
    if out_adj.size == 0:
        out_adj = np.zeros(1, dtype=np.uint32)
    arcs = np.frombuffer(pattern.arcs_u8(), dtype=np.uint8).copy()
    if arcs.size == 0:
        arcs = np.zeros(2, dtype=np.uint8)
    r = None if roots is None else np.ascontiguousarray(roots, dtype=np.uint32)
    nr = 0 if r is None else int(r.size)
    out = np.zeros((max(cap, 1), pattern.k), dtype=np.uint32)
    lo, hi = ctypes.c_uint64(0), ctypes.c_uint64(0)
    rc = lib.xmo_list(graph.n, _ptr(out_off), _ptr(out_adj), pattern.k, len(pattern.arcs), _ptr(arcs),
                      _ptr(r), nr, int(root_vertex), _ptr(out), int(cap), ctypes.byref(lo), ctypes.byref(hi))
    if rc != 0:
        raise ValueError(f"oracle rejected the input (code {rc})")
    total = lo.value | (hi.value << 64)
    return total, out[:min(total, cap)]


class Prepared:
    """A graph whose in-lists the oracle built once (graph pre-processing):
    count() gives exactly oracle.count()'s values without rebuilding them.
    The graph's arrays must stay alive while this object is used."""

    def __init__(self, graph):
        lib = _load()
        self.n = graph.n
        self._off = np.ascontiguousarray(graph.out_off, dtype=np.uint32)
        self._adj = np.ascontiguousarray(graph.out_adj, dtype=np.uint32)
        if self._adj.size == 0:
            self._adj = np.zeros(1, dtype=np.uint32)
        self._h = lib.xmo_prepare(graph.n, _ptr(self._off), _ptr(self._adj))
        if not self._h:
            raise MemoryError("oracle could not prepare the graph")

    def count(self, pattern, roots=None, mode: str = "A", threads: int = 1, root_vertex: int = -1) -> int:
        arcs = np.frombuffer(pattern.arcs_u8(), dtype=np.uint8).copy()
        if arcs.size == 0:
            arcs = np.zeros(2, dtype=np.uint8)
        r = None if roots is None else np.ascontiguousarray(roots, dtype=np.uint32)
        nr = 0 if r is None else int(r.size)
        lo, hi = ctypes.c_uint64(0), ctypes.c_uint64(0)
        rc = _load().xmo_count_prepared(ctypes.c_void_p(self._h), pattern.k, len(pattern.arcs), _ptr(arcs),
                                        _ptr(r), nr, {"A": 0, "B": 1}[mode], threads, ctypes.byref(lo),
                                        ctypes.byref(hi), None, int(root_vertex), None)
        if rc != 0:
            raise ValueError(f"oracle rejected the input (code {rc})")
        return lo.value | (hi.value << 64)

    def close(self):
        if getattr(self, "_h", None):
            _load().xmo_release(ctypes.c_void_p(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
