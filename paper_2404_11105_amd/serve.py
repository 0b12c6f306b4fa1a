"""Continuous-batching server for (graph, pattern) count queries.

Graphs stay resident; plans are cached per (graph, pattern).  A scheduler
thread keeps up to `slots` micro-batches in flight, each on its own HIP
stream: when a slot is free and memory allows, it takes the oldest pending
request, gathers further pending requests on the same graph (up to
`max_batch`), and launches them as ONE persistent xm_count.  Requests that
arrive while others run are admitted as soon as a slot and HBM budget free
up, so their work overlaps the tail of the running batches on the device.

Admission is by HBM footprint: a micro-batch needs its workspace
(xm_workspace_size) plus 24 bytes per plan; the sum over in-flight batches
never exceeds `hbm_budget`.  A request whose batch could never fit is
rejected at once.  Each request may carry a deadline; one that expires while
still queued is completed with status XM_ERR_CANCELLED without running.

A request may be anchored: pin = (v, x) counts only the embeddings that map
pattern vertex v to data node x (a constant pattern vertex).  Its plan starts
at v and its launch is restricted to the root subset {x}; anchored requests
batch with others on the same graph and node.  A request may also carry a
root subset, roots = (v, nodes): the embeddings that map v into `nodes` (an
exact partial count); it batches with requests on the same graph and the
same node array.  A request may instead carry a root share s: only the
embeddings whose start vertex maps to a stored id r with r mod 2^s = 2^s - 1
(the plan's XM_PLAN_ROOT_SHARE); the share is part of the plan, so such
requests batch with any other on the same graph.

Order: policy "fifo" takes the oldest pending request first; policy "sjf"
takes the request with the smallest estimated cost first (the backend's
estimate; for the GPU, the planner's work model on the graph's degree
statistics), except that a request waiting longer than `age_s` goes first in
arrival order, so heavy requests are delayed, never starved.

Latency = completion time - submission time (host clock).  `stats()` gives
p50 / p99 latency and counts/s over the completed requests.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time
from concurrent.futures import Future

XM_ERR_CANCELLED = -7
XM_ERR_ADMISSION = -9  # serving-level status: the request can never fit the budget
XM_ERR_SERVER = -10    # serving-level status: planning, sizing or launching raised


@dataclasses.dataclass
class Request:
    rid: int
    graph_id: object
    pattern: object
    submitted: float
    deadline: float | None
    future: Future
    pin: tuple | None = None      # (pattern vertex, data node)
    roots: tuple | None = None    # (pattern vertex, uint32 node array)
    share: int = 0                # root share exponent (0: every root)
    done: float = 0.0
    status: int = 0
    count: int | None = None


class GpuBackend:
    """Runs micro-batches with the HIP library on torch streams."""

    def __init__(self, graphs: dict, opts: dict | None = None, symmetry: bool = True):
        import torch
        self.torch = torch
        self.graphs = graphs
        self.opts = dict(opts or {})
        self.plans = {}
        # requests count with symmetry-broken plans (same counts; a pinned
        # request's plan only uses automorphisms that fix the pinned vertex);
        # the fixed side keeps planning free of host walks per request
        self.symmetry = symmetry

    def plan(self, graph_id, pattern, pin_vertex=None, share=0):
        from .api import Plan
        key = (graph_id, pattern.k, pattern.arcs, pin_vertex, share)
        p = self.plans.get(key)
        if p is None:
            sym = "above" if self.symmetry else False
            p = Plan(pattern, reduced=True, graph=self.graphs[graph_id], root_vertex=pin_vertex, symmetry=sym,
                     root_share=share)
            self.plans[key] = p
        return p

    def footprint(self, graph_id, plans, node=None) -> int:
        import ctypes
        from ._lib import XminerError, lib
        from .api import make_opts
        # an anchored launch (node given) needs at most the full-graph workspace
        o = make_opts(**self.opts)
        arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
        ws = lib().xm_workspace_size(self.graphs[graph_id].handle, len(plans), arr, ctypes.byref(o))
        if ws == 0:
            raise XminerError(-1, lib().xm_last_error().decode())
        return int(ws) + 24 * len(plans)

    def cost(self, graph_id, pattern, pin_vertex=None, share=0) -> float:
        """The planner's work estimate for this request (cached with the plan)."""
        p = self.plan(graph_id, pattern, pin_vertex, share)
        c = getattr(p, "_est_cost", None)
        if c is None:
            c = float(p.describe().get("est_cost", 0.0))
            p._est_cost = c
        return c

    def new_slot(self):
        return self.torch.cuda.Stream()

    def launch(self, slot, graph_id, plans, node=None, roots=None):
        import numpy as np
        from .api import Counter
        if roots is None and node is not None:
            roots = np.array([node], dtype=np.uint32)
        c = Counter(self.graphs[graph_id], plans, roots=roots, **self.opts)
        c.run(slot)
        ev = self.torch.cuda.Event()
        ev.record(slot)
        return (c, ev)

    def poll(self, handle) -> bool:
        return handle[1].query()

    def results(self, handle):
        c, ev = handle
        ev.synchronize()
        return c.results(sync=False)


class Server:
    def __init__(self, backend, hbm_budget: int, slots: int = 4, max_batch: int = 32,
                 poll_s: float = 0.0002, policy: str = "fifo", age_s: float = 2.0):
        if policy not in ("fifo", "sjf"):
            raise ValueError("policy must be 'fifo' or 'sjf'")
        self.policy = policy
        self.age_s = age_s
        self.backend = backend
        self.hbm_budget = int(hbm_budget)
        self.max_batch = max_batch
        self.poll_s = poll_s
        self.slots = [backend.new_slot() for _ in range(slots)]
        self.busy = {}  # slot index -> (handle, requests, footprint)
        self.pending = collections.deque()
        self.completed = []
        self.in_use = 0
        self.lock = threading.Condition()
        self.next_id = 0
        self.stop = False
        self.launches = 0
        self.max_inflight = 0
        self.thread = threading.Thread(target=self._loop, daemon=True)
        self.thread.start()

    # ---- client side
    def submit(self, graph_id, pattern, deadline_s: float | None = None, pin=None, roots=None,
               share: int = 0) -> Future:
        """Queue a count of `pattern` on graph `graph_id`; pin = (v, x) anchors
        pattern vertex v at data node x; roots = (v, nodes) counts only the
        embeddings that map v into the uint32 array `nodes`; share = s > 0
        counts only those whose start vertex maps to the root share s.  The
        future gives (count, status)."""
        if (pin is not None) + (roots is not None) + (int(share) != 0) > 1:
            raise ValueError("a request takes one of pin, roots and share")
        if not 0 <= int(share) <= 31:
            raise ValueError("share must be in 0..31")
        now = time.perf_counter()
        f = Future()
        with self.lock:
            r = Request(self.next_id, graph_id, pattern, now,
                        now + deadline_s if deadline_s is not None else None, f,
                        pin=tuple(pin) if pin is not None else None,
                        roots=(int(roots[0]), roots[1]) if roots is not None else None, share=int(share))
            self.next_id += 1
            self.pending.append(r)
            self.lock.notify()
        return f

    def close(self):
        with self.lock:
            self.stop = True
            self.lock.notify()
        self.thread.join()

    def drain(self, timeout_s: float = 600.0):
        t0 = time.perf_counter()
        while True:
            with self.lock:
                if not self.pending and not self.busy:
                    return
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError("server did not drain")
            time.sleep(0.001)

    # ---- scheduler
    def _finish(self, r: Request, status: int, count):
        r.done = time.perf_counter()
        r.status = status
        r.count = count
        self.completed.append(r)
        r.future.set_result((count, status))

    @staticmethod
    def _vertex(r):
        """The pattern vertex a request fixes the start of its plan at."""
        return r.pin[0] if r.pin else (r.roots[0] if r.roots else None)

    @staticmethod
    def _target(r):
        """Requests batch together only with the same anchor node or the
        same root array."""
        return ("pin", r.pin[1]) if r.pin else (("roots", id(r.roots[1])) if r.roots else None)

    @staticmethod
    def _code(exc) -> int:
        code = getattr(exc, "code", None)
        return code if isinstance(code, int) and code < 0 else XM_ERR_SERVER

    def _reap(self):
        for si in list(self.busy):
            handle, reqs, fp = self.busy[si]
            try:
                if not self.backend.poll(handle):
                    continue
                counts, status = self.backend.results(handle)
            except Exception as exc:  # a failed launch ends its requests, not the loop
                counts, status = [None] * len(reqs), [self._code(exc)] * len(reqs)
            for r, c, s in zip(reqs, counts, status):
                self._finish(r, s, c if s == 0 else None)
            self.in_use -= fp
            del self.busy[si]

    def _admit(self):
        free = [i for i in range(len(self.slots)) if i not in self.busy]
        now = time.perf_counter()
        while free and self.pending:
            head = self.pending[0]
            if head.deadline is not None and now > head.deadline:
                self.pending.popleft()
                self._finish(head, XM_ERR_CANCELLED, None)
                continue
            sjf = self.policy == "sjf"

            def est(r):
                # a request that cannot be planned sorts last and fails below
                try:
                    return self.backend.cost(r.graph_id, r.pattern, self._vertex(r), share=r.share)
                except Exception:
                    return float("inf")
            if sjf and now - head.submitted <= self.age_s:
                # the cheapest pending request leads; the rest keep arrival order
                head = min(self.pending, key=lambda r: (est(r), r.rid))
                self.pending.remove(head)
                self.pending.appendleft(head)
            # gather requests on the same graph (and anchor node) in arrival
            # order; under sjf only those within 8x of the head's cost, so a
            # light launch is not held up by a heavy plan in it
            node = head.pin[1] if head.pin else None
            roots = head.roots[1] if head.roots else None
            target = self._target(head)
            head_est = est(head) if sjf else 0.0
            batch, rest = [], collections.deque()
            while self.pending:
                r = self.pending.popleft()
                similar = not sjf or r is head or (head_est / 8 <= est(r) <= head_est * 8)
                if r.graph_id == head.graph_id and self._target(r) == target and len(batch) < self.max_batch and similar and (
                        r.deadline is None or now <= r.deadline):
                    batch.append(r)
                else:
                    rest.append(r)
            # plan every request; one that cannot be planned fails on its own
            plans, ok = [], []
            for r in batch:
                try:
                    plans.append(self.backend.plan(r.graph_id, r.pattern, self._vertex(r), share=r.share))
                    ok.append(r)
                except Exception as exc:
                    self._finish(r, self._code(exc), None)
            batch = ok
            if not batch:
                self.pending = collections.deque(sorted(rest, key=lambda q: q.rid))
                continue
            # shrink the batch until it fits the free budget
            try:
                fp = self.backend.footprint(head.graph_id, plans, node)
                while fp > self.hbm_budget - self.in_use and len(batch) > 1:
                    rest.appendleft(batch.pop())
                    plans.pop()
                    fp = self.backend.footprint(head.graph_id, plans, node)
            except Exception as exc:
                for r in batch:
                    self._finish(r, self._code(exc), None)
                self.pending = collections.deque(sorted(rest, key=lambda q: q.rid))
                continue
            if fp > self.hbm_budget:
                # even alone this request can never fit
                self._finish(batch[0], XM_ERR_ADMISSION, None)
                self.pending = collections.deque(sorted(list(rest) + batch[1:], key=lambda q: q.rid))
                continue
            if fp > self.hbm_budget - self.in_use:
                # wait for memory; everything goes back in arrival order
                self.pending = collections.deque(sorted(list(rest) + batch, key=lambda q: q.rid))
                break
            self.pending = collections.deque(sorted(rest, key=lambda q: q.rid))
            si = free[0]
            try:
                handle = (self.backend.launch(self.slots[si], head.graph_id, plans, node) if roots is None
                          else self.backend.launch(self.slots[si], head.graph_id, plans, roots=roots))
            except Exception as exc:
                for r in batch:
                    self._finish(r, self._code(exc), None)
                continue
            free.pop(0)
            self.busy[si] = (handle, batch, fp)
            self.in_use += fp
            self.launches += 1
            self.max_inflight = max(self.max_inflight, len(self.busy))

    def _loop(self):
        while True:
            with self.lock:
                if self.stop and not self.pending and not self.busy:
                    return
                self._reap()
                self._admit()
                idle = not self.pending and not self.busy
                if idle:
                    self.lock.wait(timeout=0.01)
            if not idle:
                time.sleep(self.poll_s)

    # ---- reporting
    def stats(self) -> dict:
        ok = [r for r in self.completed if r.status == 0]
        lat = sorted((r.done - r.submitted) * 1e3 for r in ok)
        if not lat:
            return {"completed": 0}
        span = max(r.done for r in ok) - min(r.submitted for r in ok)
        pick = lambda q: lat[min(len(lat) - 1, int(q * len(lat)))]  # noqa: E731
        return {"completed": len(ok), "failed": len(self.completed) - len(ok),
                "p50_ms": pick(0.50), "p99_ms": pick(0.99), "max_ms": lat[-1],
                "requests_per_s": len(ok) / span if span > 0 else None,
                "embeddings_per_s": sum(r.count for r in ok) / span if span > 0 else None,
                "launches": self.launches, "max_inflight_batches": self.max_inflight}
