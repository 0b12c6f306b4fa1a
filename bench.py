#!/usr/bin/env python3
"""Benchmark: exact directed-pattern counting on one MI355X.

Workload (default): R-MAT scale 16 (65,536 nodes, ~955K arcs after removing
repeats and loops, (a,b,c,d) = (.57,.19,.19,.05), seed 0), uint32 out+in CSR
resident in HBM, and four patterns: feed-forward triangle, directed 3-cycle,
bi-fan, directed 4-cycle.  The graph is stored with its nodes renumbered by
decreasing degree (load time, untimed).  One step counts all four with their
reduced, symmetry-broken plans (one embedding per automorphism orbit, scaled
by the orbit size: the same labelled counts) in one persistent launch,
replayed as a HIP graph.  The same step is also timed without symmetry
breaking, as plain per-pattern launches and with unreduced plans.

Prints one JSON line (see the repository's benchmark contract).  Only the
`cpu_baseline` leg calls the oracle, on a bounded root sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("embeddings counted/sec + adjacency elems intersected/s (HBM GB/s %), "
          "batched vs plain")
HBM_PEAK_GBPS = 8000.0
PATTERNS = ["ffl", "c3", "bifan", "c4"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def lib_hash() -> str:
    from paper_2404_11105_amd._lib import LIB_PATH
    h = hashlib.sha256()
    with open(LIB_PATH, "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def timed_steps(counter, stream, steps, warmup, progress=None):
    """Wall time per step, and the GPU time of each launch from HIP events
    recorded on the launch stream around it (these also cover the three
    microsecond-scale set-up/status kernels next to the count kernel).
    progress(msg), if given, is called after every launch."""
    import torch
    for i in range(warmup):
        counter.run(stream)
        stream.synchronize()
        if progress:
            progress(f"  warm-up launch {i} done")
    stream.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (e0, e1) in enumerate(evs):
        e0.record(stream)
        counter.run(stream)
        e1.record(stream)
        stream.synchronize()
        if progress:
            progress(f"  step {i}: {e0.elapsed_time(e1):.1f} ms")
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    gpu = sum(e0.elapsed_time(e1) for e0, e1 in evs) / steps
    return wall, gpu


def timed_plain(counters, stream, steps, warmup, progress=None):
    import torch
    for _ in range(warmup):
        for c in counters:
            c.run(stream)
        stream.synchronize()
        if progress:
            progress("  plain warm-up done")
    stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        for c in counters:
            c.run(stream)
        stream.synchronize()
        if progress:
            progress(f"  plain step {i} done")
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps * 1e3


def cpu_baseline(g, pats, target_s=4.0):
    """The oracle as it stands, on a seeded uniform sample of roots."""
    import numpy as np

    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    threads = max(1, min(16, cores))
    rng = np.random.default_rng(12345)
    total_c, total_t, parts = 0, 0.0, []
    for p in pats:
        frac = 0.002
        while True:
            k = max(1, int(frac * g.n))
            roots = np.sort(rng.choice(g.n, size=k, replace=False)).astype(np.uint32)
            t = time.perf_counter()
            c = oracle.count(g, p, roots=roots, threads=threads)
            dt = time.perf_counter() - t
            if dt >= target_s / 4 or frac >= 1.0:
                break
            frac = min(1.0, frac * max(2.0, min(50.0, target_s / max(dt, 1e-3))))
        total_c += c
        total_t += dt
        parts.append(f"{p.name}:{k}/{g.n} roots")
    return {"value": total_c / total_t, "unit": "embeddings/s", "cores": threads, "kind": "oracle",
            "sample": "seeded uniform root samples per pattern (" + ", ".join(parts) +
                      f"), {total_c} embeddings in {total_t:.2f} s"}


def traffic_from_profile(workload):
    path = os.path.join(ROOT, "profiles", "count_kernel_rmat16_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        # counters of this build and this workload only
        if rec.get("lib_sha256_16") != lib_hash() or rec.get("workload_id") != workload:
            return None
        return rec.get("hbm_bytes_per_launch")
    except Exception:
        return None


def copy_probe(mib: int, reps: int):
    """Plain device-to-device copies of `mib` MiB: reads and writes are known
    exactly, so the HBM counters of the same run calibrate the count kernel's."""
    import torch
    torch.cuda.set_device(0)
    n = mib * (1 << 20) // 4
    a = torch.arange(n, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "reps": reps}), flush=True)


def bench_batch256(args):
    """256 capped random patterns on one resident R-MAT scale 22 graph: one
    persistent batched launch (HIP graph, autotuned) against 256 plain
    launches of the same plans; batched == plain for every count, and oracle
    root-subset parity on a sample of patterns."""
    import numpy as np
    import torch

    import oracle
    from paper_2404_11105_amd import Counter, Graph, Plan, workloads
    from paper_2404_11105_amd.api import workspace_bytes
    from paper_2404_11105_amd.tune import tune

    torch.cuda.set_device(0)
    log("[batch] generating R-MAT scale 22")
    g = workloads.batch_graph()
    pats = workloads.batch_patterns()
    order = not args.generated_order
    log("[batch] loading" + (" (nodes in degree order)" if order else ""))
    G = Graph(g, order_by_degree=order)
    sym = not args.no_symmetry
    log("[batch] planning" + (" (symmetry directions from a sampled host walk)" if sym else ""))
    t_plan = time.time()
    plans = [Plan(p, reduced=True, graph=G, symmetry=sym) for p in pats]
    t_plan = time.time() - t_plan
    n_sym = sum(1 for p in plans if p.describe()["sym_mult"] > 1)
    log(f"[batch] {n_sym} plans with symmetry breaking, planned in {t_plan:.1f} s")
    s = torch.cuda.Stream()
    log("[batch] autotuning")
    rows_info = G.dense_rows_info()
    log(f"[batch] dense rows {rows_info}")
    opts, trec = tune(G, plans, stream=s, reps=1, budget_s=120, log=log)
    log(f"[batch] tuned {opts} ({trec['ms']:.1f} ms vs default {trec['default_ms']:.1f} ms)")
    cb = Counter(G, plans, **opts)
    cb.capture(s)
    log("[batch] batched launches (HIP graph)")
    ms_b, gpu_b = timed_steps(cb, s, args.steps, args.warmup, progress=log)
    counts, status = cb.results()
    assert all(x == 0 for x in status), status
    log("[batch] 256 plain launches")
    ws = torch.empty(max(workspace_bytes(G, [p], **opts) for p in plans), dtype=torch.uint8,
                     device="cuda")
    plain = [Counter(G, [p], workspace=ws, **opts) for p in plans]
    steps_plain = max(1, args.steps // 2)
    ms_p = timed_plain(plain, s, steps_plain, 1, progress=log)
    plain_counts = [c.results()[0][0] for c in plain]
    assert plain_counts == counts, "batched and plain counts differ"
    ms_nosym = None
    if sym and n_sym:
        # every embedding enumerated: the same counts
        log("[batch] batched launch without symmetry breaking")
        cn = Counter(G, [Plan(p, reduced=True, graph=G) for p in pats], **opts)
        cn.capture(s)
        ms_nosym, _ = timed_steps(cn, s, 1, 1, progress=log)
        assert cn.results()[0] == counts, "symmetry-broken and plain plans differ"
        del cn
    # oracle parity on root subsets of a sample of patterns (plans without
    # symmetry breaking on the graph in its generated order: a subset count
    # is per root, in the caller's node ids)
    log("[batch] oracle root-subset parity")
    del cb, plain, ws
    if order:
        G = Graph(g)
    rng = np.random.default_rng(7)
    sample_ids = rng.choice(len(pats), size=12, replace=False)
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    parity = True
    for i in sample_ids:
        roots = np.sort(rng.choice(g.n, size=256, replace=False)).astype(np.uint32)
        pi = Plan(pats[i], reduced=True, graph=G)
        c = Counter(G, [pi], roots=roots, **opts)
        c.run(s)
        s.synchronize()
        got = c.results()[0][0]
        want = oracle.count(g, pats[i], roots=roots, root_vertex=pi.root_vertex,
                            threads=threads, mode="B")
        parity = parity and got == want
    total = sum(counts)
    rec = {
        "metric": METRIC, "value": total / (ms_b / 1e3), "unit": "embeddings/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_b, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "batch256_rmat22", "n": g.n, "m": g.m, "patterns": len(pats),
                   "pattern_sizes": {k: sum(1 for p in pats if p.k == k) for k in (3, 4, 5, 6)},
                   "plan": "reduced, symmetry breaking" if sym else "reduced",
                   "node_order": "by decreasing degree (load time)" if order else "as generated",
                   "launch": "one persistent launch, HIP graph, autotuned",
                   "tuned": opts, "dense_rows": rows_info},
        "batched_gpu_ms": round(gpu_b, 3), "plain_ms_per_step": round(ms_p, 3),
        "batched_vs_plain_speedup": round(ms_p / ms_b, 3),
        "plans_with_symmetry_breaking": n_sym, "planning_s": round(t_plan, 1),
        "no_symmetry_ms_per_step": None if ms_nosym is None else round(ms_nosym, 3),
        "tune": trec, "counts_sum": str(total), "batched_equals_plain": True,
        "oracle_root_subset_parity": parity, "oracle_parity_patterns": len(sample_ids),
    }
    print(json.dumps(rec), flush=True)


def bench_fraction(args):
    """Exploration of a growing share of start nodes (the paper's experiment on
    the percentage of start nodes, here on the R-MAT scale 16 workload): a
    seeded permutation of the nodes is cut into ten deciles; the batched launch
    of the four patterns runs on the first 10%, 20%, ..., 100% of it, and the
    ten disjoint deciles' counts must sum to the full counts."""
    import numpy as np
    import torch

    import xmgen
    from paper_2404_11105_amd import Counter, Graph, Plan

    torch.cuda.set_device(0)
    log("[fraction] generating R-MAT scale 16")
    g = xmgen.rmat(16, seed=0)
    pats = [xmgen.named(n) for n in PATTERNS]
    G = Graph(g)
    # every plan of a root-subset launch starts at the same pattern vertex
    # symmetry breaking with the start vertex fixed keeps subset counts exact
    plans = [Plan(p, reduced=True, graph=G, root_vertex=0, symmetry=True) for p in pats]
    perm = np.random.default_rng(16).permutation(g.n).astype(np.uint32)
    cuts = [round(g.n * i / 10) for i in range(11)]
    s = torch.cuda.Stream()
    full = Counter(G, plans)
    full.run(s)
    want = full.results()[0]
    sums = [0] * len(plans)
    for i in range(10):
        c = Counter(G, plans, roots=np.sort(perm[cuts[i]:cuts[i + 1]]))
        c.run(s)
        got, st = c.results()
        assert st == [0] * len(plans)
        sums = [a + b for a, b in zip(sums, got)]
    points = []
    for i in range(1, 11):
        c = Counter(G, plans, roots=np.sort(perm[:cuts[i]]))
        c.capture(s)
        ms, _ = timed_steps(c, s, max(2, args.steps // 4), 1)
        counts, st = c.results()
        points.append({"fraction": i / 10, "ms": round(ms, 3), "counts": [str(x) for x in counts]})
        log(f"[fraction] {i * 10}% of start nodes: {ms:.2f} ms")
    rec = {
        "metric": METRIC, "value": sum(want) / (points[-1]["ms"] / 1e3), "unit": "embeddings/s",
        "n_gpus": 1, "steps": max(2, args.steps // 4), "warmup": 1, "ms_per_step": points[-1]["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "rmat16_start_node_fraction", "patterns": PATTERNS, "start_vertex": 0, "symmetry": "automorphisms fixing the start vertex",
                   "root_order": "seeded permutation, numpy default_rng(16)"},
        "points": points, "deciles_sum_to_full": sums == want, "full_counts": [str(x) for x in want],
    }
    print(json.dumps(rec), flush=True)


def bench_listing(args):
    """Listing mode on the R-MAT scale 16 graph: the unreduced plans of the
    feed-forward triangle and the 3-cycle write every embedding (3 node ids
    each) into HBM; rows/s and bytes written/s, against the counting launch of
    the same plans, and the rows checked against the oracle's listing on a
    seeded root sample."""
    import numpy as np
    import torch

    import oracle
    import xmgen
    from paper_2404_11105_amd import Counter, Graph, Plan

    torch.cuda.set_device(0)
    log("[listing] generating R-MAT scale 16")
    g = xmgen.rmat(16, seed=0)
    G = Graph(g)
    s = torch.cuda.Stream()
    out = []
    for name in ("ffl", "c3"):
        p = xmgen.named(name)
        plan = Plan(p, reduced=False, graph=G)
        cnt = Counter(G, [plan])
        cnt.capture(s)
        ms_count, _ = timed_steps(cnt, s, max(3, args.steps // 4), 1)
        total = cnt.results()[0][0]
        lst = Counter(G, [plan], list_cap=total)
        lst.capture(s)
        ms_list, _ = timed_steps(lst, s, max(3, args.steps // 4), 1)
        n, rows = lst.listed()
        assert n == total
        # oracle parity on the rows of a seeded root sample
        roots = np.sort(np.random.default_rng(3).choice(g.n, size=2048, replace=False)).astype(np.uint32)
        rv = plan.root_vertex
        sub = Counter(G, [Plan(p, reduced=False, graph=G, root_vertex=rv)], roots=roots, list_cap=total)
        sub.run(s)
        sn, srows = sub.listed()
        on, orows = oracle.list_embeddings(g, p, cap=total, roots=roots, root_vertex=rv)
        key = lambda a: a[np.lexsort(a.astype(np.int64).T[::-1])]  # noqa: E731
        same = sn == on and np.array_equal(key(srows), key(orows))
        log(f"[listing] {name}: {n} rows, {ms_list:.2f} ms listing vs {ms_count:.2f} ms counting")
        out.append({"pattern": name, "rows": str(n), "ms_listing": round(ms_list, 3),
                    "ms_counting": round(ms_count, 3), "rows_per_s": n / (ms_list / 1e3),
                    "bytes_written_per_s": n * 3 * 4 / (ms_list / 1e3),
                    "oracle_rows_equal_on_root_sample": bool(same), "sample_rows": str(sn)})
    rows_total = sum(int(o["rows"]) for o in out)
    ms_total = sum(o["ms_listing"] for o in out)
    rec = {"metric": METRIC, "value": rows_total / (ms_total / 1e3), "unit": "embeddings listed/s", "n_gpus": 1,
           "steps": max(3, args.steps // 4), "warmup": 1, "ms_per_step": round(ms_total, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
           "data": "synthetic", "config": {"workload": "rmat16_listing_ffl_c3_unreduced"}, "patterns": out}
    print(json.dumps(rec), flush=True)


def bench_serve(args):
    """Continuous batching over 8 resident R-MAT graphs (scales 18-24, built
    on the device); Poisson arrivals at two fixed rates set from the measured
    capacity; p50/p99 latency and counts/s; results alone == in the mix."""
    import numpy as np
    import torch

    import xmgen
    from paper_2404_11105_amd import Graph, workloads
    from paper_2404_11105_amd.serve import GpuBackend, Server

    torch.cuda.set_device(0)
    scales = [18, 19, 20, 21, 22, 23, 24, 24]
    graphs = {}
    for i, sc in enumerate(scales):
        log(f"[serve] building R-MAT scale {sc} on the device")
        dg = xmgen.rmat_device(sc, seed=i)
        graphs[i] = Graph(dg)
    resident = sum(G.nbytes for G in graphs.values())
    pool = workloads.batch_patterns()
    rng = np.random.default_rng(5)

    def draw(nreq):
        return [(int(rng.integers(0, len(scales))), pool[int(rng.integers(0, len(pool)))])
                for _ in range(nreq)]

    backend = GpuBackend(graphs)
    budget = 64 << 30
    # capacity: back-to-back requests, everything queued at once
    log("[serve] measuring capacity")
    warm = draw(64)
    srv = Server(backend, budget, slots=4, max_batch=16)
    t0 = time.perf_counter()
    futs = [srv.submit(gid, p) for gid, p in warm]
    for f in futs:
        f.result()
    cap_rps = len(warm) / (time.perf_counter() - t0)
    srv.close()
    levels = []
    for frac in (0.5, 0.8):
        qps = frac * cap_rps
        reqs = draw(args.requests)
        gaps = rng.exponential(1.0 / qps, size=len(reqs))
        for policy in ("fifo", "sjf"):
            log(f"[serve] {len(reqs)} requests at {qps:.1f}/s, policy {policy}")
            srv = Server(backend, budget, slots=4, max_batch=16, policy=policy)
            futs = []
            t_next = time.perf_counter()
            for (gid, p), gap in zip(reqs, gaps):
                t_next += gap
                d = t_next - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                futs.append(srv.submit(gid, p))
                if len(futs) % 50 == 0:
                    log(f"[serve]   submitted {len(futs)}")
            res = []
            for f in futs:
                res.append(f.result())
                if len(res) % 50 == 0:
                    log(f"[serve]   completed {len(res)}")
            srv.close()
            st = srv.stats()
            st.update(qps=qps, load=frac, policy=policy)
            levels.append((st, reqs, res))
    # alone vs in the mix, on a sample of the last level's requests
    log("[serve] alone vs mix")
    st_last, reqs, res = levels[-1]
    same = True
    for i in rng.choice(len(reqs), size=16, replace=False):
        srv = Server(backend, budget, slots=1, max_batch=1)
        alone = srv.submit(*reqs[i]).result()
        srv.close()
        same = same and alone == res[i]
    st = levels[-1][0]
    rec = {
        "metric": METRIC, "value": st["embeddings_per_s"], "unit": "embeddings/s", "n_gpus": 1,
        "steps": args.requests, "warmup": len(warm), "ms_per_step": st["p50_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "serve_rmat18-24x8", "graph_scales": scales,
                   "resident_bytes": resident, "pattern_pool": len(pool),
                   "arrivals": "Poisson", "hbm_budget_bytes": budget, "slots": 4, "max_batch": 16,
                   "policies": ["fifo", "sjf"]},
        "capacity_requests_per_s": cap_rps,
        "levels": [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in l[0].items()}
                   for l in levels],
        "alone_equals_mix": same,
    }
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip plain/unreduced timings")
    ap.add_argument("--no-symmetry", action="store_true",
                    help="plans without symmetry breaking (every embedding enumerated)")
    ap.add_argument("--generated-order", action="store_true",
                    help="store the graph in the generator's node order (default: nodes "
                         "renumbered by decreasing degree at load, untimed)")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--split", type=int, default=0)
    ap.add_argument("--split-work", type=int, default=0)
    ap.add_argument("--cap", type=int, default=0)
    ap.add_argument("--waves-per-cu", type=int, default=0)
    ap.add_argument("--row-min", type=int, default=None,
                    help="shortest list with a dense membership row (default: the library's)")
    ap.add_argument("--dense-rows", type=int, default=None,
                    help="byte budget of the dense rows (0: none; default: the library's)")
    ap.add_argument("--workload", default="rmat16",
                    choices=["rmat16", "batch256", "serve", "fraction", "listing"],
                    help="rmat16: the contract line (default); batch256 / serve: the batched "
                         "and serving workloads, each printing its own JSON line")
    ap.add_argument("--requests", type=int, default=150, help="serve: requests per load level and policy")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run plain device copies of this size (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib, args.steps)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(roots would shard across GPUs with one final 128-bit sum; not built).",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch256":
        bench_batch256(args)
        return
    if args.workload == "serve":
        bench_serve(args)
        return
    if args.workload == "fraction":
        bench_fraction(args)
        return
    if args.workload == "listing":
        bench_listing(args)
        return

    import numpy as np
    import torch

    import xmgen
    from paper_2404_11105_amd import Counter, Graph, Plan, plan_work

    torch.cuda.set_device(0)
    log("[bench] generating R-MAT scale 16")
    g = xmgen.rmat(16, seed=0)
    pats = [xmgen.named(n) for n in PATTERNS]
    G = Graph(g, dense_rows=args.dense_rows, row_min=args.row_min, order_by_degree=not args.generated_order)
    tune = dict(chunk=args.chunk, split=args.split, split_work=args.split_work, cap=args.cap,
                waves_per_cu=args.waves_per_cu)
    sym = not args.no_symmetry
    red = [Plan(p, reduced=True, graph=G, symmetry=sym) for p in pats]
    unred = [Plan(p, reduced=False, graph=G, symmetry=sym) for p in pats]
    workload = ("rmat16_ffl_c3_bifan_c4_reduced" + ("_sym" if sym else "")
                + ("" if args.generated_order else "_degorder") + "_batched")
    s = torch.cuda.Stream()

    # algorithmic work of the four plans (host walk, untimed; with symmetry
    # breaking only the list parts above each bound count)
    log("[bench] algorithmic work (host walk)")
    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    st = [plan_work(G.host, p, threads=threads) for p in red]
    E = sum(x["elements"] for x in st)
    F = sum(x["fetches"] for x in st)
    B_alg = 4 * E + 8 * F + 8 * g.n * len(pats)

    log("[bench] batched reduced (HIP graph)")
    cb = Counter(G, red, **tune)
    cb.capture(s)
    ms_step, kern_ms = timed_steps(cb, s, args.steps, args.warmup)
    counts, status = cb.results()
    assert status == [0] * len(pats), status

    extras = {}
    if not args.no_extras:
        log("[bench] plain per-pattern launches")
        plain = [Counter(G, [p], **tune) for p in red]
        ms_plain = timed_plain(plain, s, args.steps, args.warmup)
        assert [c.results()[0][0] for c in plain] == counts
        log("[bench] batched unreduced")
        cu = Counter(G, unred, **tune)
        cu.capture(s)
        ms_unred, kern_unred = timed_steps(cu, s, max(3, args.steps // 4), 1)
        assert cu.results()[0] == counts
        E_un = sum(plan_work(G.host, p, threads=threads)["elements"] for p in unred)
        if sym:
            log("[bench] batched reduced without symmetry breaking")
            cn = Counter(G, [Plan(p, reduced=True, graph=G) for p in pats], **tune)
            cn.capture(s)
            ms_nosym, _ = timed_steps(cn, s, max(3, args.steps // 4), 1)
            assert cn.results()[0] == counts
            extras = {"no_symmetry_ms_per_step": round(ms_nosym, 4),
                      "symmetry_speedup": round(ms_nosym / ms_step, 3)}
        extras.update({"plain_ms_per_step": round(ms_plain, 4),
                  "batched_vs_plain_speedup": round(ms_plain / ms_step, 3),
                  "unreduced_ms_per_step": round(ms_unred, 4),
                  "unreduced_kernel_ms": round(kern_unred, 4),
                  "reduced_vs_unreduced_speedup": round(ms_unred / ms_step, 3),
                  "unreduced_elements": E_un})

    gold_ok = None
    gpath = os.path.join(ROOT, "tests", "golden", "rmat16.json")
    if os.path.exists(gpath):
        gold = json.load(open(gpath))["counts"]
        gold_ok = counts == [int(gold[n]) for n in PATTERNS]

    total = sum(counts)
    value = total / (ms_step / 1e3)
    achieved = B_alg / (kern_ms / 1e3) / 1e9
    traffic = traffic_from_profile(workload)
    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] oracle cpu baseline")
        cpu = cpu_baseline(g, pats)

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "embeddings/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": workload,
                   "graph": "R-MAT scale 16, edge factor 16, (.57,.19,.19,.05), seed 0",
                   "n": g.n, "m": g.m, "patterns": PATTERNS,
                   "plan": "reduced, symmetry breaking" if sym else "reduced",
                   "launch": "one persistent launch for 4 patterns, HIP graph replay",
                   "parallelism": "1 GPU", "dense_rows": G.dense_rows_info(),
                   "node_order": "as generated" if args.generated_order else "by decreasing degree (load time)"},
        "counts": [str(c) for c in counts],
        "counts_match_oracle": gold_ok,
        "kernel_ms": round(kern_ms, 4),
        "kernel_ms_note": "HIP events on the launch stream around each HIP-graph replay",
        "elements_intersected": E,
        "list_fetches": F,
        "elements_per_s": E / (kern_ms / 1e3),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic},
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
