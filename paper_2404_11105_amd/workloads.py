"""Workload definitions for the batched and serving benchmarks.

batch256: 256 seeded random connected patterns of 3-6 vertices (xmgen's
random_pattern recipe) counted against one resident R-MAT scale 22 graph.
Random sparse patterns on a graph with ~10^5-degree hubs can have 10^15 or
more partial matches, which no launch can enumerate, so candidates pass a
work cap: the plan's algorithmic work (xm_plan_work) is estimated from roots
sampled by degree rank -- all of the 16 largest, then 16 seeded roots from
each rank stratum [16,64), [64,256), ..., [262144, n), each weighted by its
stratum size -- and must stay under CAP_ELEMENTS, with no walk passing
WALK_BUDGET partial matches; the estimates of the accepted heavy patterns
(above HEAVY elements) together stay under TOTAL_CAP (a heavy candidate that
would pass it is rejected), which keeps one batched launch at a few seconds.  Sizes are drawn round-robin (3, 4, 5, 6) with a
quota of 64 each; a size whose candidates run out (MAX_DRAWS) is backfilled
by smaller sizes.  The accepted seeds are stored in workloads/batch256.json
with the counts of rejected draws.

    python -m paper_2404_11105_amd.workloads batch256
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
BATCH_PATH = os.path.join(HERE, "workloads", "batch256.json")
CAP_ELEMENTS = 3e11
TOTAL_CAP = 4e12
HEAVY = 1e10
WALK_BUDGET = 2_000_000
STRATA = [0, 16, 64, 256, 1024, 4096, 16384, 65536, 262144]
MAX_DRAWS = 1000
SEED_BASE = {3: 300000, 4: 400000, 5: 500000, 6: 600000}


def batch_graph():
    import xmgen
    return xmgen.rmat(22, seed=0)


def batch_patterns():
    """The 256 accepted patterns (list of xmgen.Pattern) from the stored file."""
    import xmgen
    rec = json.load(open(BATCH_PATH))
    return [xmgen.random_pattern(k, s) for k, s in rec["accepted"]]


def select_batch(threads: int = 8):
    import xmgen
    from .api import Plan, plan_work
    t0 = time.time()
    g = batch_graph()
    deg = np.maximum(g.out_deg(), g.in_deg())
    order = np.argsort(-deg, kind="stable").astype(np.uint32)
    rng = np.random.default_rng(22)
    strata = []  # (roots, weight)
    bounds = STRATA + [g.n]
    for a, b in zip(bounds[:-1], bounds[1:]):
        idx = order[a:b]
        if b - a <= 16:
            strata.append((np.sort(idx), 1.0))
        else:
            strata.append((np.sort(rng.choice(idx, size=16, replace=False)), (b - a) / 16.0))
    quota = {3: 64, 4: 64, 5: 64, 6: 64}
    accepted, rejected, draws, est = [], {k: 0 for k in quota}, {k: 0 for k in quota}, []
    exhausted = set()
    while len(accepted) < 256:
        progressed = False
        for k in (3, 4, 5, 6):
            if k in exhausted or quota[k] == 0:
                continue
            seed = SEED_BASE[k] + draws[k]
            draws[k] += 1
            if draws[k] > MAX_DRAWS:
                exhausted.add(k)
                continue
            progressed = True
            p = xmgen.random_pattern(k, seed)
            plan = Plan(p, True)
            e, exceeded = 0.0, False
            for roots, w in strata:
                r = plan_work(g, plan, roots=roots, threads=threads, max_partial=WALK_BUDGET)
                e += r["elements"] * w
                if r["exceeded"] or e > CAP_ELEMENTS:
                    exceeded = True
                    break
            if exceeded or (e > HEAVY and sum(x for x in est if x > HEAVY) + e > TOTAL_CAP):
                rejected[k] += 1
                continue
            accepted.append((k, seed))
            est.append(e)
            quota[k] -= 1
            print(f"k={k} seed={seed} est={e:.3g} accepted={len(accepted)}", flush=True)
            if len(accepted) == 256:
                break
        if not progressed:
            # backfill the missing quota from the smallest sizes
            missing = 256 - len(accepted)
            for k in (3, 4, 5, 6):
                if k not in exhausted:
                    quota[k] += missing
                    break
            else:
                break
    rec = {"graph": "rmat(scale=22, edge_factor=16, abcd=(.57,.19,.19,.05), seed=0)",
           "recipe": "random_pattern(k, seed); work cap from a degree-stratified root sample",
           "cap_elements": CAP_ELEMENTS, "total_cap": TOTAL_CAP, "heavy": HEAVY, "walk_budget": WALK_BUDGET,
           "accepted": accepted, "estimated_elements": est,
           "rejected_per_k": rejected, "draws_per_k": draws,
           "selection_seconds": round(time.time() - t0, 1)}
    os.makedirs(os.path.dirname(BATCH_PATH), exist_ok=True)
    with open(BATCH_PATH, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return rec


if __name__ == "__main__":
    if sys.argv[1:] == ["batch256"]:
        r = select_batch()
        print({k: v for k, v in r.items() if k not in ("accepted", "estimated_elements")})
