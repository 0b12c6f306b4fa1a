"""Python binding over the C ABI (argument marshalling only).

    g = Graph(digraph)                       # xm_load_graph (device buffers borrowed)
    p = Plan(pattern, reduced=True, graph=g) # xm_plan
    counts = count(g, [p])                   # xm_count -> list of Python ints
"""
from __future__ import annotations

import ctypes
import os
import json

import numpy as np

from . import _lib
from ._lib import check, lib


def _u32_tensor(a, device):
    import torch
    arr = np.ascontiguousarray(a, dtype=np.uint32)
    if arr.size == 0:
        arr = np.zeros(1, dtype=np.uint32)
    return torch.from_numpy(arr.view(np.int32)).to(device)


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Graph:
    """A resident data graph: uint32 out-CSR + in-CSR in device memory.

    The device tensors are owned here and borrowed by the library
    (XM_MEM_DEVICE) until close().  Lists of at least `row_min` elements get
    dense membership rows (xm_graph_dense_rows) within `dense_rows` bytes;
    dense_rows=0 keeps every membership test a sorted-list search.
    """

    DEFAULT_ROW_BYTES = 8 << 30
    DEFAULT_ROW_MIN = 64

    def __init__(self, digraph, device: str = "cuda", validate: bool = False, stream=None,
                 dense_rows: int | None = None, row_min: int | None = None, order_by_degree: bool = False):
        import torch
        self.n = int(digraph.n)
        self.m = int(digraph.m)
        self.device = torch.device(device)
        arrays = (digraph.out_off, digraph.out_adj, digraph.in_off, digraph.in_adj)
        h = ctypes.c_void_p()
        flags = _lib.XM_VALIDATE if validate else 0
        if order_by_degree:
            # the library renumbers and owns the device copy (XM_ORDER_BY_DEGREE)
            if any(isinstance(x, torch.Tensor) for x in arrays):
                raise ValueError("order_by_degree needs host (numpy) CSR arrays")
            host = [np.ascontiguousarray(x, dtype=np.uint32) for x in arrays]
            host = [a if a.size else np.zeros(1, dtype=np.uint32) for a in host]
            self.tensors = []
            flags |= _lib.XM_MEM_HOST | _lib.XM_ORDER_BY_DEGREE
            ptrs = [a.ctypes.data_as(ctypes.c_void_p) for a in host]
        else:
            if all(isinstance(x, torch.Tensor) for x in arrays):
                # already device-resident int32 tensors holding uint32 values
                self.tensors = [x.to(self.device).contiguous() for x in arrays]
            else:
                self.tensors = [_u32_tensor(x, self.device) for x in arrays]
            flags |= _lib.XM_MEM_DEVICE
            ptrs = [ctypes.c_void_p(t.data_ptr()) for t in self.tensors]
        self.nbytes = 4 * (2 * (self.n + 1) + 2 * self.m)
        with torch.cuda.device(self.device):
            check(lib().xm_load_graph(self.n, self.m, *ptrs, flags, _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        self.order_by_degree = order_by_degree
        # host CSR in the stored node order, kept for planning estimates and
        # the host work walk (None for device-only input)
        if order_by_degree:
            self.host = _renumbered(digraph, self.node_order())
        elif all(isinstance(x, torch.Tensor) for x in arrays):
            self.host = None
        else:
            self.host = digraph
        self.set_dense_rows(self.DEFAULT_ROW_BYTES if dense_rows is None else dense_rows,
                            self.DEFAULT_ROW_MIN if row_min is None else row_min, stream)

    def set_dense_rows(self, max_bytes: int, row_min: int = 32, stream=None) -> int:
        """(Re)build dense rows within max_bytes; returns the threshold used (0:
        none).  When the device cannot hold them the budget is halved until it
        can (rows only make membership tests faster)."""
        import torch
        t = ctypes.c_uint32()
        budget = int(max_bytes)
        with torch.cuda.device(self.device):
            while True:
                rc = lib().xm_graph_dense_rows(self.handle, budget, int(row_min), _stream_ptr(stream),
                                               ctypes.byref(t))
                if rc != _lib.XM_ERR_OOM or budget == 0:
                    check(rc)
                    return t.value
                budget //= 2

    def node_order(self) -> np.ndarray:
        """new_of_old: the stored id of every node (the identity unless the
        graph was loaded with order_by_degree)."""
        out = np.empty(self.n, dtype=np.uint32)
        check(lib().xm_graph_node_order(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def dense_rows_info(self) -> dict:
        t, no, ni, b = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint64()
        check(lib().xm_graph_dense_rows_info(self.handle, ctypes.byref(t), ctypes.byref(no), ctypes.byref(ni),
                                             ctypes.byref(b)))
        return {"row_min": t.value, "out_rows": no.value, "in_rows": ni.value, "bytes": b.value}

    def info(self):
        n, m, mo, mi = (ctypes.c_uint32() for _ in range(4))
        check(lib().xm_graph_info(self.handle, ctypes.byref(n), ctypes.byref(m),
                                  ctypes.byref(mo), ctypes.byref(mi)))
        return {"n": n.value, "m": m.value, "max_out": mo.value, "max_in": mi.value}

    def close(self):
        if getattr(self, "handle", None):
            lib().xm_free_graph(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _renumbered(digraph, new_of_old):
    """Host CSR of digraph with node v renamed new_of_old[v] (lists sorted)."""
    import types
    n = int(digraph.n)
    off = np.asarray(digraph.out_off, dtype=np.int64)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    dst = np.asarray(digraph.out_adj, dtype=np.int64)
    new = np.asarray(new_of_old, dtype=np.int64)
    s2, d2 = new[src], new[dst]

    def csr(a, b):
        o = np.lexsort((b, a))
        offs = np.zeros(n + 1, dtype=np.uint32)
        offs[1:] = np.cumsum(np.bincount(a, minlength=n))
        return offs, b[o].astype(np.uint32)

    oo, oa = csr(s2, d2)
    io, ia = csr(d2, s2)
    return types.SimpleNamespace(n=n, m=int(digraph.m), out_off=oo, out_adj=oa, in_off=io, in_adj=ia)


class Plan:
    """A counting plan for one pattern (reduced or unreduced).

    symmetry counts one embedding per orbit of the pattern's automorphisms on
    the enumerated vertices and scales the total by the orbit size (same
    counts, less work); such a plan cannot list embeddings, and counts a root
    subset only with a forced root_vertex (then only automorphisms fixing
    that vertex are used).  "above" keeps, per orbit, the embedding whose first
    conditioned vertex has the smallest image; "below" the largest; True picks
    the one with less estimated work on `graph` (a sampled host walk), or
    "above" without a host copy of the graph.

    root_share = s > 0 counts only the embeddings whose start vertex maps to
    a node with stored id r, r mod 2^s = 2^s - 1: an exact partial count over
    a fixed share of the roots (with symmetry, only automorphisms that fix
    the start vertex are used)."""

    def __init__(self, pattern, reduced: bool = True, graph: Graph | None = None,
                 root_vertex: int | None = None, symmetry=False, root_share: int = 0):
        self.pattern = pattern
        self.reduced = reduced
        self.root_share = int(root_share)
        if symmetry is True:
            symmetry = _choose_direction(pattern, reduced, graph, root_vertex, root_share)
        if symmetry not in (False, "above", "below"):
            raise ValueError("symmetry must be False, True, 'above' or 'below'")
        self.symmetry = symmetry
        arcs = (ctypes.c_uint8 * max(1, 2 * len(pattern.arcs)))(*pattern.arcs_u8())
        flags = _lib.XM_PLAN_REDUCED if reduced else _lib.XM_PLAN_UNREDUCED
        if symmetry:
            flags |= _lib.XM_PLAN_SYMMETRY
        if symmetry == "below":
            flags |= _lib.XM_PLAN_SYM_BELOW
        if root_vertex is not None:
            flags |= _lib.XM_PLAN_ROOT(root_vertex)
        if root_share:
            flags |= _lib.XM_PLAN_ROOT_SHARE(root_share)
        h = ctypes.c_void_p()
        check(lib().xm_plan(pattern.k, len(pattern.arcs), arcs, flags,
                            graph.handle if graph is not None else None, ctypes.byref(h)))
        self.handle = h

    def describe(self) -> dict:
        return json.loads(plan_json(self))

    @property
    def root_vertex(self) -> int:
        return check(lib().xm_plan_root_vertex(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            lib().xm_free_plan(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_json(plan: Plan) -> str:
    need = ctypes.c_size_t()
    lib().xm_plan_describe(plan.handle, None, 0, ctypes.byref(need))
    buf = ctypes.create_string_buffer(need.value)
    check(lib().xm_plan_describe(plan.handle, buf, need.value, None))
    return buf.value.decode()


def describe_plan(pattern, reduced: bool = True, symmetry=False, root_share: int = 0) -> dict:
    return Plan(pattern, reduced, symmetry=symmetry, root_share=root_share).describe()


SYM_FETCH_COST = 64      # one list fetch weighs as much as this many elements
SYM_SAMPLE_HUBS = 64     # longest-listed nodes always in the sample
SYM_SAMPLE_REST = 4096   # other nodes, strided
SYM_WALK_CAP = 200_000_000  # partial matches per estimate


def _choose_direction(pattern, reduced, graph, root_vertex, root_share=0):
    """The symmetry direction with the smaller estimated work: the host walk
    (elements + SYM_FETCH_COST x list fetches) over the hub roots and a
    strided sample of the others, scaled to all roots.  Patterns without
    symmetry, graphs without a host copy and walks past the cap keep
    "above"."""
    if graph is None or getattr(graph, "host", None) is None:
        return "above"
    g = graph.host
    cand = {d: Plan(pattern, reduced, root_vertex=root_vertex, symmetry=d, root_share=root_share)
            for d in ("above", "below")}
    if cand["above"].describe()["sym_mult"] == 1:
        return "above"
    deg = np.diff(np.asarray(g.out_off, dtype=np.int64)) + np.diff(np.asarray(g.in_off, dtype=np.int64))
    n = deg.size
    hubs = np.argsort(-deg, kind="stable")[:SYM_SAMPLE_HUBS]
    rest = np.setdiff1d(np.arange(0, n, max(1, n // SYM_SAMPLE_REST)), hubs)
    w_rest = (n - hubs.size) / max(1, rest.size)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    cost = {}
    for d, p in cand.items():
        tot = 0.0
        for roots, w in ((hubs, 1.0), (rest, w_rest)):
            if roots.size == 0:
                continue
            r = plan_work(g, p, roots=roots.astype(np.uint32), threads=threads, max_partial=SYM_WALK_CAP)
            if r["exceeded"]:
                return "above"
            tot += w * (r["elements"] + SYM_FETCH_COST * r["fetches"])
        cost[d] = tot
    return "below" if cost["below"] < cost["above"] else "above"


def make_opts(chunk=0, split=0, cap=0, waves_per_cu=0, roots=None, cancel=None, events=None,
              merge_min=0, merge_ratio=0, split_work=0, roots_host=None, listing=None):
    """xm_count_opts; roots is a device tensor, roots_host (optional) a
    contiguous uint32 numpy copy the caller keeps alive."""
    o = _lib.XmCountOpts()
    o.struct_size = ctypes.sizeof(_lib.XmCountOpts)
    o.chunk, o.split, o.cap, o.waves_per_cu = chunk, split, cap, waves_per_cu
    o.merge_min, o.merge_ratio, o.split_work = merge_min, merge_ratio, split_work
    if roots is not None:
        o.roots_dev = roots.data_ptr()
        o.n_roots = roots.numel()
        if roots_host is not None:
            o.roots_host = roots_host.ctypes.data
    if cancel is not None:
        o.cancel_dev = cancel.data_ptr()
    if listing is not None:
        buf, cap_rows, cnt = listing
        o.list_dev = buf.data_ptr()
        o.list_cap = int(cap_rows)
        o.list_count_dev = cnt.data_ptr()
    if events is not None:
        o.ev_kernel_start = events[0].cuda_event
        o.ev_kernel_stop = events[1].cuda_event
    return o


class Counter:
    """One reusable xm_count call: fixed graph, plans and options.

    Owns the workspace, count and status tensors; run() enqueues on a
    stream, results() waits and converts the (lo, hi) pairs to ints.
    """

    def __init__(self, graph: Graph, plans, chunk=0, split=0, cap=0, waves_per_cu=0,
                 roots=None, cancel=None, kernel_events: bool = False, stream=None,
                 merge_min=0, merge_ratio=0, split_work=0, workspace=None, list_cap: int = 0):
        import torch
        self.graph = graph
        self.plans = list(plans)
        dev = graph.device
        self.roots = self.roots_host = None
        if roots is not None:
            self.roots_host = np.ascontiguousarray(roots, dtype=np.uint32)
            self.roots = _u32_tensor(self.roots_host, dev)
        self.cancel = cancel
        self.events = None
        if kernel_events:
            # events around the count kernel itself; recording once creates them
            with torch.cuda.device(dev):
                s = stream if stream is not None else torch.cuda.current_stream()
                self.events = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                for ev in self.events:
                    ev.record(s)
        self.list = self.list_count = None
        listing = None
        if list_cap > 0:
            # every embedding written out: rows of k node ids (one plan, one leaf)
            k = self.plans[0].pattern.k
            self.list = torch.empty(int(list_cap) * k, dtype=torch.int32, device=dev)
            self.list_count = torch.zeros(1, dtype=torch.int64, device=dev)
            listing = (self.list, int(list_cap), self.list_count)
        self.opts = make_opts(chunk, split, cap, waves_per_cu, self.roots, cancel, self.events,
                              merge_min, merge_ratio, split_work, self.roots_host, listing)
        self._parr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        ws = lib().xm_workspace_size(graph.handle, len(self.plans), self._parr, ctypes.byref(self.opts))
        if ws == 0:
            check(_lib.XM_ERR_INVALID if lib().xm_last_error() else _lib.XM_ERR_INVALID)
        self.ws_bytes = int(ws)
        if workspace is not None:
            # a caller-shared buffer: launches that use it must not overlap in time
            if workspace.numel() * workspace.element_size() < self.ws_bytes:
                raise ValueError("shared workspace is smaller than xm_workspace_size")
            self.workspace = workspace
            self.ws_bytes = workspace.numel() * workspace.element_size()
        else:
            self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.counts = torch.zeros(2 * len(self.plans), dtype=torch.int64, device=dev)
        self.status = torch.zeros(len(self.plans), dtype=torch.int32, device=dev)
        self.exec = None
        # the fills and copies above run on torch's current stream; a launch on
        # another stream must wait for them
        self._ready = torch.cuda.Event()
        self._ready.record(torch.cuda.current_stream(dev))
        self._streams = set()

    def _order(self, stream):
        """Make `stream` wait for this object's set-up, and tell torch's
        allocator that its buffers are used there."""
        import torch
        if stream is None:
            return
        cur = torch.cuda.current_stream(self.graph.device)
        if stream == cur:
            return
        stream.wait_event(self._ready)
        key = stream.cuda_stream
        if key not in self._streams:
            self._streams.add(key)
            for t in (self.workspace, self.counts, self.status, self.roots, self.list, self.list_count):
                if t is not None:
                    t.record_stream(stream)

    def _args(self):
        return (self.graph.handle, len(self.plans), self._parr, ctypes.byref(self.opts),
                ctypes.c_void_p(self.workspace.data_ptr()), self.ws_bytes,
                ctypes.c_void_p(self.counts.data_ptr()), ctypes.c_void_p(self.status.data_ptr()))

    def run(self, stream=None):
        import torch
        with torch.cuda.device(self.graph.device):
            self._order(stream)
            if self.exec is not None:
                check(lib().xm_exec_launch(self.exec, _stream_ptr(stream)))
            else:
                check(lib().xm_count(*self._args(), _stream_ptr(stream)))

    def capture(self, stream):
        """Record this call once as a HIP graph; later run() calls replay it."""
        import torch
        h = ctypes.c_void_p()
        with torch.cuda.device(self.graph.device):
            # set-up must be complete before the recorded launches read it
            self._ready.synchronize()
            self._order(stream)
            check(lib().xm_count_capture(*self._args(), _stream_ptr(stream), ctypes.byref(h)))
        self.exec = h

    def results(self, sync: bool = True):
        import torch
        if sync:
            torch.cuda.synchronize(self.graph.device)
        c = self.counts.cpu().numpy().view(np.uint64)
        st = self.status.cpu().numpy()
        out = [int(c[2 * i]) | (int(c[2 * i + 1]) << 64) for i in range(len(self.plans))]
        return out, [int(s) for s in st]

    def listed(self, sync: bool = True):
        """(number of embeddings found, array [min(found, list_cap), k] of rows in
        pattern-vertex order); sync waits for the device first."""
        import torch
        if sync:
            torch.cuda.synchronize(self.graph.device)
        n = int(self.list_count.cpu().numpy().view(np.uint64)[0])
        k = self.plans[0].pattern.k
        rows = self.list.cpu().numpy().view(np.uint32).reshape(-1, k)
        return n, rows[:min(n, rows.shape[0])]

    def kernel_ms(self) -> float:
        """Duration of the last count kernel (call after the stream completed)."""
        return self.events[0].elapsed_time(self.events[1])

    def close(self):
        if self.exec is not None:
            lib().xm_free_exec(self.exec)
            self.exec = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_work(digraph, plan: Plan, roots=None, threads: int = 1, max_partial: int = 0) -> dict:
    """Algorithmic work of a plan on a host graph (statistics only, no count).

    With max_partial > 0 the walk stops after that many partial matches and
    the result has exceeded=True."""
    arrs = [np.ascontiguousarray(a, dtype=np.uint32) for a in
            (digraph.out_off, digraph.out_adj, digraph.in_off, digraph.in_adj)]
    arrs = [a if a.size else np.zeros(1, dtype=np.uint32) for a in arrs]
    out = (ctypes.c_uint64 * 4)()
    r, nr = None, 0
    if roots is not None:
        r = np.ascontiguousarray(roots, dtype=np.uint32)
        nr = int(r.size)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    rc = check(lib().xm_plan_work(int(digraph.n), *[ptr(a) for a in arrs], plan.handle,
                                  ptr(r) if r is not None else None, nr, threads, max_partial, out))
    return dict(elements=out[0], fetches=out[1], partial_matches=out[2], roots=out[3],
                exceeded=rc == 1)


TRAFFIC_KEYS = ("base_elements", "offset_pairs", "degree_pairs", "row_words", "searches", "search_words",
                "partial_matches", "chain_words", "roots", "elements_merge")


def plan_traffic(digraph, plan: Plan, row_min: int = 0, roots=None, threads: int = 1,
                 max_partial: int = 0) -> dict:
    """Memory operations the count kernel issues for `plan` on a host graph
    (xm_plan_traffic; statistics only, no count).  row_min: the graph's dense
    row threshold (0: no rows).  The dict also holds `bytes`: 4 B per base
    element, row word, search word and chain word, 8 B per offset pair and
    partial match written, 1 B per degree class read."""
    arrs = [np.ascontiguousarray(a, dtype=np.uint32) for a in
            (digraph.out_off, digraph.out_adj, digraph.in_off, digraph.in_adj)]
    arrs = [a if a.size else np.zeros(1, dtype=np.uint32) for a in arrs]
    out = (ctypes.c_uint64 * len(TRAFFIC_KEYS))()
    r, nr = None, 0
    if roots is not None:
        r = np.ascontiguousarray(roots, dtype=np.uint32)
        nr = int(r.size)
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
    rc = check(lib().xm_plan_traffic(int(digraph.n), *[ptr(a) for a in arrs], plan.handle,
                                     ptr(r) if r is not None else None, nr, int(row_min), threads,
                                     max_partial, out))
    d = {k: int(v) for k, v in zip(TRAFFIC_KEYS, out)}
    d["bytes"] = traffic_bytes(d)
    d["exceeded"] = rc == 1
    return d


def traffic_bytes(d: dict) -> int:
    """Bytes of the issued model: what the kernel's tests read and write."""
    return (4 * (d["base_elements"] + d["row_words"] + d["search_words"] + d["chain_words"])
            + 8 * (d["offset_pairs"] + d["partial_matches"]) + d["degree_pairs"])


class Watchdog:
    """A cancel flag in pinned host memory and a host timer that raises it.

    Pass `flag` as Counter(cancel=...); `arm(seconds)` before a launch,
    `disarm()` after it completed.  A launch that outlives the budget stops
    at its next poll and reports XM_ERR_CANCELLED."""

    def __init__(self):
        import torch
        self.flag = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        self._timer = None
        # the device reads the flag through the mapped alias of the pinned page
        hip = ctypes.CDLL("libamdhip64.so")
        dptr = ctypes.c_void_p()
        rc = hip.hipHostGetDevicePointer(ctypes.byref(dptr), ctypes.c_void_p(self.flag.data_ptr()), 0)
        if rc != 0 or not dptr.value:
            raise RuntimeError(f"pinned flag is not mapped for the device (hip error {rc})")
        self._dev = dptr.value

    def data_ptr(self) -> int:
        """Device address of the flag (what the kernel polls)."""
        return self._dev

    def arm(self, seconds: float):
        import threading
        self.disarm()
        self.flag[0] = 0
        self._timer = threading.Timer(seconds, self._fire)
        self._timer.daemon = True
        self._timer.start()

    def _fire(self):
        self.flag[0] = 1

    def disarm(self):
        if self._timer is not None:
            self._timer.cancel()
            self._timer = None
        self.flag[0] = 0

    @property
    def fired(self) -> bool:
        return bool(self.flag[0].item())


def workspace_bytes(graph: Graph, plans, **opts) -> int:
    """xm_workspace_size for these plans and options."""
    o = make_opts(**opts)
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    ws = lib().xm_workspace_size(graph.handle, len(plans), arr, ctypes.byref(o))
    if ws == 0:
        check(_lib.XM_ERR_INVALID)
    return int(ws)


def count_anchored(graph: Graph, pattern, vertex: int, nodes, reduced: bool = True, stream=None,
                   symmetry=False, **opts):
    """Embeddings of `pattern` that map pattern vertex `vertex` to each data
    node in `nodes` (a constant pattern vertex, Definition 2.2's vertex
    constraints): the plan starts at `vertex` and each node is a one-root
    subset.  Returns one count per node.  With symmetry, only automorphisms
    that fix `vertex` are used, so every count stays exact per node."""
    import numpy as np
    plan = Plan(pattern, reduced=reduced, graph=graph, root_vertex=vertex, symmetry=symmetry)
    out = []
    for x in np.asarray(nodes, dtype=np.uint32).reshape(-1):
        c = Counter(graph, [plan], roots=np.array([x], dtype=np.uint32), **opts)
        c.run(stream)
        counts, status = c.results()
        check(status[0])
        out.append(counts[0])
    return out


def list_embeddings(graph: Graph, pattern, cap: int, reduced: bool = False, roots=None, root_vertex=None,
                    stream=None, **opts):
    """Write out the embeddings of `pattern`: (total found, array [min(total,
    cap), k] of node ids in pattern-vertex order, rows in no particular
    order).  The plan is unreduced by default (its last vertex is the only
    leaf); a reduced plan works when its leaf group is one vertex."""
    plan = Plan(pattern, reduced=reduced, graph=graph, root_vertex=root_vertex)
    c = Counter(graph, [plan], roots=roots, list_cap=cap, **opts)
    c.run(stream)
    counts, status = c.results()
    check(status[0])
    n, rows = c.listed()
    assert n == counts[0]
    return n, rows


def count(graph: Graph, plans, stream=None, **opts):
    """Count every plan against graph in one batched launch; returns ints."""
    c = Counter(graph, plans, **opts)
    c.run(stream)
    counts, status = c.results()
    for s in status:
        if s != 0:
            check(s)
    return counts
