"""Serving loop (CPU): admission by footprint, continuous batching, deadlines,
and results identical alone and in the mix.  A fake backend stands in for the
GPU: its launches take simulated time and its counts come from the oracle."""
import threading
import time

import pytest

import oracle
import xmgen
from paper_2404_11105_amd.serve import XM_ERR_ADMISSION, XM_ERR_CANCELLED, Server


class FakeBackend:
    def __init__(self, graphs, secs_per_plan=0.002, ws_bytes=1000, scale_by_cost=False):
        self.graphs = graphs
        self.scale_by_cost = scale_by_cost
        self.secs = secs_per_plan
        self.ws = ws_bytes
        self.launched = []
        self.inflight = 0
        self.max_inflight = 0
        self.mu = threading.Lock()

    def plan(self, graph_id, pattern, pin_vertex=None, share=0):
        return (pattern, pin_vertex)

    def cost(self, graph_id, pattern, pin_vertex=None, share=0):
        return float(len(pattern.arcs))

    def footprint(self, graph_id, plans, node=None):
        return self.ws + 24 * len(plans)

    def new_slot(self):
        return object()

    def launch(self, slot, graph_id, plans, node=None, roots=None):
        g = self.graphs[graph_id]
        if roots is not None:
            counts = [oracle.count(g, p, roots=roots, root_vertex=v) for p, v in plans]
        elif node is None:
            counts = [oracle.count(g, p) for p, _ in plans]
        else:
            counts = [oracle.count(g, p, roots=[node], root_vertex=v) for p, v in plans]
        with self.mu:
            self.inflight += 1
            self.max_inflight = max(self.max_inflight, self.inflight)
            self.launched.append((graph_id, len(plans)))
        secs = sum(self.secs * (self.cost(graph_id, p) if self.scale_by_cost else 1.0) for p, _ in plans)
        return {"t": time.perf_counter() + secs, "counts": counts, "done": False}

    def poll(self, h):
        if time.perf_counter() >= h["t"]:
            if not h["done"]:
                with self.mu:
                    self.inflight -= 1
                h["done"] = True
            return True
        return False

    def results(self, h):
        return h["counts"], [0] * len(h["counts"])


def graphs():
    return {"u": xmgen.uniform_digraph(200, 1500, 1), "r": xmgen.rmat(8, seed=2)}


def pats():
    return [xmgen.named(n) for n in ["ffl", "c3", "bifan", "c4", "path3", "outstar3"]]


def test_results_alone_and_in_the_mix_are_identical():
    G = graphs()
    P = pats()
    alone = {}
    for gid in G:
        for i, p in enumerate(P):
            s = Server(FakeBackend(G), hbm_budget=10 ** 6, slots=1, max_batch=1)
            alone[(gid, i)] = s.submit(gid, p).result(timeout=60)[0]
            s.close()
    be = FakeBackend(G, secs_per_plan=0.01)
    s = Server(be, hbm_budget=10 ** 6, slots=3, max_batch=8)
    futs = []
    for rep in range(4):
        for gid in G:
            for i, p in enumerate(P):
                futs.append(((gid, i), s.submit(gid, p)))
        time.sleep(0.003)  # arrivals while earlier batches run
    mixed = [(k, f.result(timeout=60)) for k, f in futs]
    s.close()
    for k, (c, st) in mixed:
        assert st == 0 and c == alone[k]
    st = s.stats()
    assert st["completed"] == len(futs) and st["p99_ms"] >= st["p50_ms"] > 0
    assert be.max_inflight >= 2, "batches must overlap"
    assert any(n > 1 for _, n in be.launched), "requests must be batched"


def test_admission_respects_hbm_budget():
    G = graphs()
    be = FakeBackend(G, secs_per_plan=0.02, ws_bytes=1000)
    # room for exactly one batch at a time
    s = Server(be, hbm_budget=1000 + 24 * 4, slots=4, max_batch=4)
    futs = [s.submit("u", p) for p in pats() * 2]
    for f in futs:
        assert f.result(timeout=60)[1] == 0
    s.close()
    assert be.max_inflight == 1


def test_request_that_can_never_fit_is_rejected():
    G = graphs()
    s = Server(FakeBackend(G, ws_bytes=10 ** 6), hbm_budget=1000, slots=2)
    c, st = s.submit("u", xmgen.named("c3")).result(timeout=60)
    s.close()
    assert st == XM_ERR_ADMISSION and c is None


def test_expired_deadline_is_cancelled_without_running():
    G = graphs()
    be = FakeBackend(G, secs_per_plan=0.2)
    s = Server(be, hbm_budget=10 ** 6, slots=1, max_batch=1)
    f1 = s.submit("u", xmgen.named("c3"))
    f2 = s.submit("u", xmgen.named("ffl"), deadline_s=0.01)  # expires while f1 runs
    assert f1.result(timeout=60)[1] == 0
    c, st = f2.result(timeout=60)
    s.close()
    assert st == XM_ERR_CANCELLED and c is None
    assert len(be.launched) == 1


def test_anchored_requests_batch_by_node_and_sum_to_the_total():
    """Anchored requests (pattern vertex v at node x) count the embeddings
    with that image; over all x they sum to the unanchored count."""
    G = {"u": xmgen.uniform_digraph(40, 200, 3)}
    be = FakeBackend(G, secs_per_plan=0.001)
    s = Server(be, hbm_budget=10 ** 6, slots=2, max_batch=8)
    p = xmgen.named("ffl")
    total = s.submit("u", p).result(timeout=60)[0]
    futs = {(v, x): s.submit("u", p, pin=(v, x)) for x in range(40) for v in range(p.k)}
    for v in range(p.k):
        assert sum(futs[(v, x)].result(timeout=60)[0] for x in range(40)) == total
    s.close()
    # anchored requests on the same node share launches
    assert any(n > 1 for _, n in be.launched[1:])


def test_sjf_runs_cheap_requests_first_without_starving_heavy_ones():
    """Policy sjf: with one slot busy, queued cheap requests run before a
    heavier one that arrived earlier; once a request has waited age_s it
    goes first; every count is unchanged."""
    G = {"u": xmgen.uniform_digraph(100, 600, 2)}
    heavy, light = xmgen.named("c5chord"), xmgen.named("arc")
    be = FakeBackend(G, secs_per_plan=0.01, scale_by_cost=True)
    s = Server(be, hbm_budget=10 ** 6, slots=1, max_batch=1, policy="sjf", age_s=30.0)
    first = s.submit("u", light)          # occupies the slot
    time.sleep(0.002)
    fh = s.submit("u", heavy)
    fl = [s.submit("u", light) for _ in range(3)]
    for f in [first, fh] + fl:
        f.result(timeout=60)
    done = {r.rid: r.done for r in s.completed}
    s.close()
    assert all(done[i] < done[1] for i in (2, 3, 4)), "cheap requests should overtake the heavy one"
    assert fh.result()[0] == oracle.count(G["u"], heavy)
    # aging: with age_s = 0 the order is arrival order
    be = FakeBackend(G, secs_per_plan=0.01, scale_by_cost=True)
    s = Server(be, hbm_budget=10 ** 6, slots=1, max_batch=1, policy="sjf", age_s=0.0)
    futs = [s.submit("u", light)]
    time.sleep(0.002)
    futs += [s.submit("u", heavy)] + [s.submit("u", light) for _ in range(3)]
    for f in futs:
        f.result(timeout=60)
    done = {r.rid: r.done for r in s.completed}
    s.close()
    assert all(done[1] < done[i] for i in (2, 3, 4))


class FailingBackend(FakeBackend):
    """Raises from plan (patterns with 4 vertices), footprint (graph "r" with
    2 or more plans) or launch (a c3 in the batch), like a library error or
    an out-of-memory during set-up would."""

    def plan(self, graph_id, pattern, pin_vertex=None, share=0):
        if pattern.k == 4:
            from paper_2404_11105_amd._lib import XminerError
            raise XminerError(-2, "pattern rejected")
        return super().plan(graph_id, pattern, pin_vertex)

    def cost(self, graph_id, pattern, pin_vertex=None, share=0):
        self.plan(graph_id, pattern, pin_vertex)
        return super().cost(graph_id, pattern, pin_vertex)

    def footprint(self, graph_id, plans, node=None):
        if graph_id == "r" and len(plans) >= 2:
            raise MemoryError("workspace sizing failed")
        return super().footprint(graph_id, plans, node)

    def launch(self, slot, graph_id, plans, node=None, roots=None):
        if any(p.name == "c3" for p, _ in plans):
            raise RuntimeError("launch failed")
        return super().launch(slot, graph_id, plans, node, roots)


@pytest.mark.parametrize("policy", ["fifo", "sjf"])
def test_backend_errors_fail_their_requests_and_keep_serving(policy):
    gs = graphs()
    be = FailingBackend(gs)
    srv = Server(be, hbm_budget=10_000, slots=2, max_batch=4, policy=policy)
    reqs = [("u", xmgen.named(n)) for n in ["ffl", "bifan", "c3", "path3", "ffl"]]
    reqs += [("r", xmgen.named("ffl")), ("r", xmgen.named("path3"))]
    futs = [srv.submit(g, p) for g, p in reqs]
    res = [f.result(timeout=30) for f in futs]
    # the loop is still alive: a later request on a healthy batch completes
    late = srv.submit("u", xmgen.named("path3")).result(timeout=30)
    srv.close()
    for (gid, p), (c, s) in zip(reqs, res):
        if p.k == 4:
            assert s == -2 and c is None  # the plan's own error code
        elif gid == "r" or s != 0:
            assert s < 0 and c is None
        else:
            assert c == oracle.count(gs[gid], p)
    assert res[1][1] == -2
    assert late == (oracle.count(gs["u"], xmgen.named("path3")), 0)
    # every request on graph "r" shares a batch whose sizing raised, unless
    # it ran alone; none of them hangs
    assert all(s in (0, -10) for (gid, _), (_, s) in zip(reqs, res) if gid == "r")


def test_root_subset_requests_batch_by_array_and_are_exact():
    """Requests with a root subset (v, nodes) count the embeddings that map
    v into nodes; they batch only with requests on the same array, and the
    counts are the oracle's partial sums."""
    import numpy as np
    gs = graphs()
    be = FakeBackend(gs, secs_per_plan=0.001)
    srv = Server(be, hbm_budget=10_000, slots=2, max_batch=8)
    a = np.arange(0, 200, 7, dtype=np.uint32)
    b = np.arange(3, 200, 11, dtype=np.uint32)
    reqs = [(xmgen.named(n), (0, a)) for n in ["ffl", "c3", "bifan"]] + [(xmgen.named("c4"), (1, b)),
                                                                          (xmgen.named("path3"), (0, b))]
    futs = [srv.submit("u", p, roots=r) for p, r in reqs]
    res = [f.result(timeout=30) for f in futs]
    srv.close()
    for (p, (v, nodes)), (c, s) in zip(reqs, res):
        assert s == 0 and c == oracle.count(gs["u"], p, roots=nodes, root_vertex=v)
    # the three requests on array a went out together at most in one launch each way
    assert srv.launches <= 4


class ShareBackend(FakeBackend):
    """Plans carry the request's root share; a plan starts at pattern vertex 0."""

    def plan(self, graph_id, pattern, pin_vertex=None, share=0):
        return (pattern, pin_vertex, share)

    def launch(self, slot, graph_id, plans, node=None, roots=None):
        import numpy as np
        g = self.graphs[graph_id]
        counts = []
        for p, _, s in plans:
            share = np.arange((1 << s) - 1, g.n, 1 << s, dtype=np.uint32)
            counts.append(oracle.count(g, p, roots=share, root_vertex=0) if s else oracle.count(g, p))
        with self.mu:
            self.inflight += 1
            self.launched.append((graph_id, len(plans)))
        return {"t": time.perf_counter() + self.secs, "counts": counts, "done": False}


def test_root_share_requests_reach_the_plan_and_batch_with_others():
    """A request's root share is part of its plan: requests with different
    shares on one graph go out in one launch, each with its own partial
    count; a share with a pin or a root array, or past 31, is refused."""
    gs = graphs()
    be = ShareBackend(gs, secs_per_plan=0.001)
    srv = Server(be, hbm_budget=10_000, slots=1, max_batch=8)
    reqs = [(xmgen.named("ffl"), 0), (xmgen.named("ffl"), 2), (xmgen.named("c4"), 3), (xmgen.named("path3"), 1)]
    with srv.lock:  # queue all four before the scheduler looks
        futs = [srv.submit("u", p, share=s) for p, s in reqs]
    res = [f.result(timeout=30) for f in futs]
    srv.close()
    import numpy as np
    n = gs["u"].n
    for (p, s), (c, st) in zip(reqs, res):
        want = oracle.count(gs["u"], p, roots=np.arange((1 << s) - 1, n, 1 << s, dtype=np.uint32),
                            root_vertex=0) if s else oracle.count(gs["u"], p)
        assert st == 0 and c == want
    assert be.launched == [("u", 4)]
    srv = Server(be, hbm_budget=10_000)
    for kw in ({"share": 2, "pin": (0, 1)}, {"share": 1, "roots": (0, np.arange(3, dtype=np.uint32))},
               {"share": 32}):
        with pytest.raises(ValueError):
            srv.submit("u", xmgen.named("ffl"), **kw)
    srv.close()
