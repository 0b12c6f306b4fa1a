#!/usr/bin/env python3
"""Benchmark: exact directed-pattern counting on one MI355X.

Default workload (one JSON line, the repository's benchmark contract): one
resident R-MAT scale 22 graph (4,194,304 nodes, ~65.2M arcs after removing
repeats and loops, (a,b,c,d) = (.57,.19,.19,.05), seed 0; uint32 out+in CSR,
stored with its nodes renumbered by decreasing degree at load, untimed) and
256 seeded random connected directed patterns of 3-6 vertices, 64 of each
size, each counted on its root share (paper_2404_11105_amd/workloads.py).
One step is ONE persistent launch that counts all 256 reduced,
symmetry-broken plans, replayed as a HIP graph with launch options tuned
offline (workloads/batch256_tuned.json).  The same 256 plans are also timed
as 256 plain launches (batched vs plain), and every count must agree.

Also in the line: the roofline of the count kernel (issued bytes from the
host walk stored in workloads/batch256_traffic.json, measured HBM traffic
and VALU issue from the rocprofv3 summaries under profiles/ when they were
taken on this build), the oracle's throughput on a bounded sample of the
same workload (1 core and all cores, 1 warm-up then the median of 5), and
two smaller workloads as extra keys: R-MAT scale 16 with the four motifs
(batched, plain, unreduced) and R-MAT scale 20 with the two 5-vertex
patterns, reduced vs unreduced plans.

Only the `cpu_baseline` leg calls the oracle.
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
SJF_AGE_S = 0.25  # serving: a request waiting longer than this goes first under sjf
N_CU, CLOCK_HZ = 256, 2.4e9   # MI355X: VALU issue capacity = one wave64 instruction per CU per cycle
PATTERNS = ["ffl", "c3", "bifan", "c4"]
C5CHORD_SHARE = 6             # scale-20 extra: the 5-cycle with a chord on 1/64 of the roots
WL_DIR = os.path.join(ROOT, "paper_2404_11105_amd", "workloads")


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


def host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def oracle_timing(prep, work, threads, reps=5):
    """The oracle as it stands on `work` = [(pattern, roots, root_vertex)] over
    a prepared graph (its in-lists built once, untimed, like the device
    graph's load): one warm-up pass, then the median of `reps` timed passes
    (embeddings, seconds).  With threads > 1 the work items run concurrently,
    one oracle call per item on its own host thread (the oracle's own threads
    split a call's roots 64 at a time, too coarse for these samples)."""
    from concurrent.futures import ThreadPoolExecutor

    def item(w):
        p, r, rv = w
        return prep.count(p, roots=r, root_vertex=rv, mode="B")

    def one():
        t = time.perf_counter()
        if threads == 1:
            c = sum(item(w) for w in work)
        else:
            with ThreadPoolExecutor(max_workers=threads) as ex:
                c = sum(ex.map(item, work))
        return c, time.perf_counter() - t

    one()
    runs = sorted((one() for _ in range(reps)), key=lambda x: x[1])
    return runs[len(runs) // 2]


def cpu_baseline(g, work, sample_desc):
    """1 core and all T cores, each 1 warm-up + median of 5; `value` is the
    all-core rate (embeddings/s), the 1-core rate is beside it."""
    import oracle
    T = host_cores()
    prep = oracle.Prepared(g)
    c1, t1 = oracle_timing(prep, work, 1)
    cT, tT = oracle_timing(prep, work, T)
    prep.close()
    assert c1 == cT
    return {"value": cT / tT, "unit": "embeddings/s", "cores": T, "kind": "oracle",
            "sample": sample_desc + f"; {cT} embeddings; median of 5 after 1 warm-up: {tT:.3f} s on {T} "
                                    f"threads, {t1:.3f} s on 1",
            "value_1core": c1 / t1, "seconds_1core": round(t1, 4), "seconds_all_cores": round(tT, 4)}


# hub roots of the oracle's sample, per pattern size: the first root of the
# pattern's share at or above each of these degree ranks (R-MAT 22 in degree
# order: rank 256 ~ degree 9,700, 1,024 ~ 9,400, 4,096 ~ 3,100, 16,384 ~
# 1,000, 65,536 ~ 320).  A six-vertex pattern on a root of rank 65,536 took
# the oracle 68 s, so six-vertex patterns get no hub root.
SAMPLE_HUB_RANKS = {3: (256, 1024, 4096), 4: (256, 1024, 4096), 5: (16384, 65536), 6: ()}


def write_cpu_sample(n_patterns=16, per_pattern=128, chunks=8):
    """The oracle's sample of the batch workload (stored in
    workloads/batch256_cpu_sample.json; chosen from the stored batch without
    running anything): every 16th pattern (four of each size), each on 128
    seeded roots of its own root share of degree rank [n/16, n/4) (all of
    them when the share has fewer there; lists of a few to ten arcs: the
    bulk of the roots a launch walks) split into 8 work items, plus the hub
    roots SAMPLE_HUB_RANKS names, one work item each; roots in the
    generated ids."""
    import numpy as np

    from paper_2404_11105_amd import workloads
    rec = json.load(open(workloads.BATCH_PATH))["accepted"]
    g = workloads.batch_graph()
    new_of_old = workloads.degree_order(g)
    old_of_new = np.empty_like(new_of_old)
    old_of_new[new_of_old] = np.arange(g.n, dtype=np.uint32)
    rng = np.random.default_rng(64)
    plans = workloads.batch_plans()
    work = []
    n_hubs = 0
    for i in range(0, len(rec), len(rec) // n_patterns):
        share = workloads.share_roots(g.n, rec[i]["share"])
        sh = share[(share >= g.n // 16) & (share < g.n // 4)]
        roots = np.sort(old_of_new[rng.choice(sh, size=min(per_pattern, sh.size), replace=False)])
        rv = plans[i].describe()["root_vertex"]
        for c in np.array_split(roots, chunks):
            work.append([i, c.tolist(), rv])
        for rank in SAMPLE_HUB_RANKS[rec[i]["k"]]:
            hub = share[share >= rank]
            if hub.size:
                work.append([i, [int(old_of_new[hub[0]])], rv])
                n_hubs += 1
    desc = (f"{n_patterns} of the 256 patterns (every 16th), up to {per_pattern} roots each from its root share "
            f"at degree ranks [n/16, n/4) in {chunks} work items, plus {n_hubs} hub roots (the first of the "
            f"share at degree rank >= 256, >= 1024 and >= 4096 for 3-4-vertex patterns, >= 16384 and >= 65536 "
            f"for 5-vertex ones), one work item each; generated ids")
    out = {"description": desc, "work": work}
    with open(os.path.join(WL_DIR, "batch256_cpu_sample.json"), "w") as f:
        json.dump(out, f)
        f.write("\n")
    return out


def profile_record(name, workload_id):
    """A counter summary under profiles/ taken on this library build and
    workload, else None."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        if rec.get("lib_sha256_16") != lib_hash() or rec.get("workload_id") != workload_id:
            return None
        return rec
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


def load_json(name):
    path = os.path.join(WL_DIR, name)
    return json.load(open(path)) if os.path.exists(path) else None


def batch_setup():
    """The scale-22 graph (degree order, dense rows), its 256 plans on their
    root shares, and the stored launch options."""
    from paper_2404_11105_amd import Graph, workloads
    log("[batch] generating R-MAT scale 22")
    t = time.time()
    g = workloads.batch_graph()
    log(f"[batch]   {time.time() - t:.1f} s; loading in degree order with dense rows")
    t = time.time()
    G = Graph(g, order_by_degree=True, dense_rows=workloads.ROW_BYTES)
    log(f"[batch]   {time.time() - t:.1f} s, rows {G.dense_rows_info()}")
    pats = workloads.batch_patterns()
    shares = workloads.batch_shares()
    t = time.time()
    plans = workloads.batch_plans()
    t_plan = time.time() - t
    tuned = load_json("batch256_tuned.json") or {"opts": {}}
    return g, G, pats, shares, plans, t_plan, tuned


def bench_batch256(args):
    """The contract line: one persistent launch of 256 plans against 256
    plain launches on the resident scale-22 graph."""
    import numpy as np
    import torch

    from paper_2404_11105_amd import Counter, workloads
    from paper_2404_11105_amd.api import workspace_bytes

    torch.cuda.set_device(0)
    g, G, pats, shares, plans, t_plan, tuned = batch_setup()
    opts = dict(tuned["opts"])
    row_min = G.dense_rows_info()["row_min"]
    key = workloads.plans_key(plans, row_min)
    n_sym = sum(1 for p in plans if p.describe()["sym_mult"] > 1)
    log(f"[batch] 256 plans in {t_plan:.1f} s ({n_sym} symmetry-broken), options {opts}")
    s = torch.cuda.Stream()
    cb = Counter(G, plans, **opts)
    cb.capture(s)
    log("[batch] batched launches (HIP graph replays)")
    ms_b, gpu_b = timed_steps(cb, s, args.steps, args.warmup, progress=log)
    counts, status = cb.results()
    assert all(x == 0 for x in status), status
    extras = {}
    if not args.no_extras:
        # 256 plain launches, each captured as its own HIP graph like the
        # batched one, with the batch's tuned options and with the defaults
        steps_plain = max(1, args.steps // 4)
        ms_plain = {}
        for label, o in (("batch_options", opts), ("default_options", {})):
            log(f"[batch] 256 plain launches ({label})")
            ws = torch.empty(max(workspace_bytes(G, [p], **o) for p in plans), dtype=torch.uint8, device="cuda")
            plain = [Counter(G, [p], workspace=ws, **o) for p in plans]
            for c in plain:
                c.capture(s)
            ms_plain[label] = timed_plain(plain, s, steps_plain, 1, progress=log)
            plain_counts = [c.results()[0][0] for c in plain]
            assert plain_counts == counts, "batched and plain counts differ"
            del plain, ws
        ms_p = min(ms_plain.values())
        extras.update({"plain_ms_per_step": round(ms_p, 3), "plain_steps": steps_plain,
                       "plain_ms_by_options": {k: round(v, 3) for k, v in ms_plain.items()},
                       "batched_vs_plain_speedup": round(ms_p / ms_b, 3), "batched_equals_plain": True,
                       "plain_note": "each plain launch a HIP-graph replay; plain_ms_per_step is the faster "
                                     "of the two option sets"})
    # issued bytes of the launch (host walk stored per plan set and row threshold)
    tr = load_json("batch256_traffic.json") or {}
    roofline, elements = None, None
    if tr.get("key") == key:
        B = tr["total"]["bytes"]
        elements = tr["total"]["elements_merge"]
        achieved = B / (gpu_b / 1e3) / 1e9
        wl = "batch256_rmat22"
        prof = profile_record("count_kernel_batch256_traffic.json", wl)
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 4),
                    "traffic": prof["hbm_bytes_per_launch"] if prof else None}
        cnt = profile_record("count_kernel_batch256_counters.json", wl)
        if cnt:
            extras["issue"] = {"valu_instructions": cnt["SQ_INSTS_VALU"],
                               "frac": round(cnt["SQ_INSTS_VALU"] / (N_CU * CLOCK_HZ * gpu_b / 1e3), 4),
                               "note": "SQ_INSTS_VALU / (256 CUs x 2.4 GHz x launch time), one wave64 VALU "
                                       "instruction per CU per cycle"}
        extras["issued_bytes_per_launch"] = B
        extras["elements_intersected"] = elements
        extras["elements_per_s"] = elements / (gpu_b / 1e3)
    else:
        log("[batch] stored traffic does not match these plans; roofline not reported")
    cpu = None
    smp = load_json("batch256_cpu_sample.json")
    if not args.no_cpu_baseline and smp:
        log("[batch] oracle cpu baseline")
        work = [(pats[i], np.array(r, dtype=np.uint32), rv) for i, r, rv in smp["work"]]
        cpu = cpu_baseline(g, work, smp["description"])
    if not args.no_extras:
        extras["rmat16_motifs"] = extra_rmat16(args)
        extras["rmat20_reduction"] = extra_rmat20(args)
    total = sum(counts)
    sizes = {k: sum(1 for p in pats if p.k == k) for k in (3, 4, 5, 6)}
    rec = {
        "metric": METRIC, "value": total / (ms_b / 1e3), "unit": "embeddings/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_b, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "batch256_rmat22",
                   "graph": "R-MAT scale 22, edge factor 16, (.57,.19,.19,.05), seed 0",
                   "n": g.n, "m": g.m, "patterns": len(pats), "pattern_sizes": sizes,
                   "root_shares": {str(sh): sum(1 for x in shares if x == sh) for sh in sorted(set(shares))},
                   "plan": "reduced, symmetry breaking (side stored per pattern), unit cover weights",
                   "node_order": "by decreasing degree (load time)",
                   "launch": "one persistent launch of 256 plans, HIP graph replay",
                   "options": opts, "options_tuned_for_these_plans": tuned.get("key") == key,
                   "dense_rows": G.dense_rows_info(), "parallelism": "1 GPU"},
        "kernel_ms": round(gpu_b, 3),
        "kernel_ms_note": "HIP events on the launch stream around each HIP-graph replay",
        "counts_sum": str(total), "plans_with_symmetry_breaking": n_sym, "planning_s": round(t_plan, 2),
        "roofline": roofline, "cpu_baseline": cpu, **extras,
    }
    print(json.dumps(rec), flush=True)


def extra_rmat16(args):
    """Beside the line: R-MAT scale 16, four motifs, reduced
    symmetry-broken plans in one batched launch; plain launches; unreduced
    plans; counts checked against the stored oracle values."""
    import torch

    import xmgen
    from paper_2404_11105_amd import Counter, Graph, Plan
    log("[rmat16] generating R-MAT scale 16")
    g = xmgen.rmat(16, seed=0)
    pats = [xmgen.named(n) for n in PATTERNS]
    G = Graph(g, order_by_degree=True)
    s = torch.cuda.Stream()
    red = [Plan(p, reduced=True, graph=G, symmetry=True) for p in pats]
    cb = Counter(G, red)
    cb.capture(s)
    steps = max(3, args.steps // 2)
    ms_b, _ = timed_steps(cb, s, steps, 2)
    counts = cb.results()[0]
    plain = [Counter(G, [p]) for p in red]
    ms_p = timed_plain(plain, s, steps, 1)
    assert [c.results()[0][0] for c in plain] == counts
    cu = Counter(G, [Plan(p, reduced=False, graph=G, symmetry=True) for p in pats])
    cu.capture(s)
    ms_u, _ = timed_steps(cu, s, steps, 1)
    assert cu.results()[0] == counts
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "rmat16.json")))["counts"]
    return {"graph": "R-MAT scale 16, seed 0", "patterns": PATTERNS, "counts": [str(c) for c in counts],
            "counts_match_oracle": counts == [int(gold[n]) for n in PATTERNS],
            "batched_ms": round(ms_b, 3), "plain_ms": round(ms_p, 3),
            "batched_vs_plain_speedup": round(ms_p / ms_b, 3), "unreduced_ms": round(ms_u, 3),
            "reduced_vs_unreduced_speedup": round(ms_u / ms_b, 3),
            "embeddings_per_s": sum(counts) / (ms_b / 1e3)}


def extra_rmat20(args):
    """Beside the line: R-MAT scale 20, transitive tournament on 4
    vertices plus a pendant in-arc (every root) and the 5-cycle with a chord
    (root share 1/64), each as the reduced plan (leaf groups counted by
    product, included arcs taken from the including arc's candidates)
    against the unreduced plan (every level fetches all its lists, only the
    last vertex counted); a launch past the limit is cancelled."""
    import torch

    import xmgen
    from paper_2404_11105_amd import Counter, Graph, Plan
    from paper_2404_11105_amd import Watchdog
    log("[rmat20] generating R-MAT scale 20")
    g = xmgen.rmat(20, seed=0)
    G = Graph(g, order_by_degree=True)
    s = torch.cuda.Stream()
    wd = Watchdog()
    limit_s = float(getattr(args, "rmat20_limit_s", 60.0))
    out = {"cancel_after_s": limit_s}
    # the 5-cycle with a chord has ~10^14 embeddings and does not finish
    # within the limit on every root: it is counted on a root share
    shares = {"tt4p": 0, "c5chord": C5CHORD_SHARE}
    for name in ("tt4p", "c5chord"):
        p = xmgen.named(name)
        row = {"root_share": shares[name]}
        for kind, red in (("reduced", True), ("unreduced", False)):
            plan = Plan(p, reduced=red, graph=G, symmetry=True, root_share=shares[name])
            c = Counter(G, [plan], cancel=wd, kernel_events=True, stream=s)
            ms = []
            for _ in range(2):
                wd.arm(limit_s)
                c.run(s)
                s.synchronize()
                wd.disarm()
                cnt, st = c.results()
                if st != [0]:
                    break
                ms.append(c.kernel_ms())
            d = plan.describe()
            row[kind] = {"ms": round(min(ms), 3) if ms and st == [0] else None, "count": str(cnt[0]) if st == [0] else None,
                         "status": st[0], "e": d["e"], "leaves": d["t"], "removed_arcs": d["removed_edges"],
                         "fetched_arcs": len(d["cover"]["fetched"])}
            log(f"[rmat20] {name} {kind}: {row[kind]['ms']} ms (status {st[0]})")
        if row["reduced"]["ms"] and row["unreduced"]["ms"]:
            assert row["reduced"]["count"] == row["unreduced"]["count"]
            row["reduced_vs_unreduced_speedup"] = round(row["unreduced"]["ms"] / row["reduced"]["ms"], 3)
        out[name] = row
    return out


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
    on the device, generated node order); each request draws a graph and a
    pattern of 3-7 vertices from the serving pool, counted on the pattern's
    root share of that graph; Poisson arrivals at two fixed rates set from
    the measured capacity; p50/p99 latency and counts/s; results alone ==
    in the mix."""
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
    pool = workloads.serve_pool()
    rng = np.random.default_rng(5)

    def draw(nreq):
        return [(int(rng.integers(0, len(scales))), pool[int(rng.integers(0, len(pool)))])
                for _ in range(nreq)]

    backend = GpuBackend(graphs)
    budget = 64 << 30
    # warm-up: every (graph, pool entry) planned and launched once, untimed
    log("[serve] warm-up: every pool entry on every graph")
    srv = Server(backend, budget, slots=4, max_batch=16)
    for f in [srv.submit(gid, p, share=sh) for gid in range(len(scales)) for p, sh in pool]:
        f.result()
    srv.close()
    # capacity: back-to-back requests, everything queued at once; the median
    # of three draws of 256
    log("[serve] measuring capacity")
    caps = []
    for _ in range(3):
        warm = draw(256)
        srv = Server(backend, budget, slots=4, max_batch=16)
        t0 = time.perf_counter()
        futs = [srv.submit(gid, p, share=sh) for gid, (p, sh) in warm]
        for f in futs:
            f.result()
        caps.append(len(warm) / (time.perf_counter() - t0))
        srv.close()
    cap_rps = sorted(caps)[1]
    levels = []
    for frac in (0.5, 0.8):
        qps = frac * cap_rps
        reqs = draw(args.requests)
        gaps = rng.exponential(1.0 / qps, size=len(reqs))
        for policy in ("fifo", "sjf"):
            log(f"[serve] {len(reqs)} requests at {qps:.1f}/s, policy {policy}")
            srv = Server(backend, budget, slots=4, max_batch=16, policy=policy, age_s=SJF_AGE_S)
            futs = []
            t_next = time.perf_counter()
            for (gid, (p, sh)), gap in zip(reqs, gaps):
                t_next += gap
                d = t_next - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                futs.append(srv.submit(gid, p, share=sh))
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
        gid, (p, sh) = reqs[i]
        alone = srv.submit(gid, p, share=sh).result()
        srv.close()
        same = same and alone == res[i]
    st = levels[-1][0]
    rec = {
        "metric": METRIC, "value": st["embeddings_per_s"], "unit": "embeddings/s", "n_gpus": 1,
        "steps": args.requests, "warmup": len(scales) * len(pool), "ms_per_step": st["p50_ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "serve_rmat18-24x8", "graph_scales": scales,
                   "resident_bytes": resident, "pattern_pool": len(pool),
                   "pool_sizes": {str(k): sum(1 for p, _ in pool if p.k == k) for k in range(3, 8)},
                   "pool_shares": {str(sh): sum(1 for _, x in pool if x == sh) for sh in sorted({x for _, x in pool})},
                   "arrivals": "Poisson", "hbm_budget_bytes": budget, "slots": 4, "max_batch": 16,
                   "sjf_age_s": SJF_AGE_S,
                   "policies": ["fifo", "sjf"]},
        "capacity_requests_per_s": cap_rps,
        "capacity_draws_requests_per_s": [round(c, 1) for c in caps],
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
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the plain launches and the scale-16 / scale-20 extras")
    ap.add_argument("--workload", default="batch256",
                    choices=["batch256", "rmat16", "rmat20", "serve", "fraction", "listing"],
                    help="batch256: the contract line (default); the others print their own JSON line")
    ap.add_argument("--requests", type=int, default=150, help="serve: requests per load level and policy")
    ap.add_argument("--rmat20-limit-s", type=float, default=60.0,
                    help="R-MAT 20 reduced vs unreduced: cancel a launch after this many seconds")
    ap.add_argument("--write-cpu-sample", action="store_true",
                    help="write the oracle's sample of the batch workload and time it (host only)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run plain device copies of this size (counter calibration)")
    args = ap.parse_args()
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib, args.steps)
        return
    if args.write_cpu_sample:
        import numpy as np

        from paper_2404_11105_amd import workloads
        smp = write_cpu_sample()
        g = workloads.batch_graph()
        pats = workloads.batch_patterns()
        work = [(pats[i], np.array(r, dtype=np.uint32), rv) for i, r, rv in smp["work"]]
        print(json.dumps(cpu_baseline(g, work, smp["description"])), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(roots would shard across GPUs with one final 128-bit sum; not built).",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch256":
        bench_batch256(args)
    elif args.workload == "rmat16":
        import torch
        torch.cuda.set_device(0)
        r = extra_rmat16(args)
        print(json.dumps({"metric": METRIC, "value": r["embeddings_per_s"], "unit": "embeddings/s", "n_gpus": 1,
                          "steps": max(3, args.steps // 2), "warmup": 2, "ms_per_step": r["batched_ms"],
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
                          "data": "synthetic", "config": {"workload": "rmat16_motifs_batched"}, **r}), flush=True)
    elif args.workload == "rmat20":
        import torch
        torch.cuda.set_device(0)
        r = extra_rmat20(args)
        print(json.dumps({"workload": "rmat20_reduction", **r}), flush=True)
    elif args.workload == "serve":
        bench_serve(args)
    elif args.workload == "fraction":
        bench_fraction(args)
    elif args.workload == "listing":
        bench_listing(args)


if __name__ == "__main__":
    main()
