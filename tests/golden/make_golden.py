"""Write expected counts for the parity tests by calling only the oracle.

    python tests/golden/make_golden.py uniform2000 rmat16 rmat20_subset

Each workload writes tests/golden/<name>.json with the generator recipe, the
patterns and the oracle's counts (decimal strings: they can exceed 2**64).
No value here comes from the HIP path.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import xmgen  # noqa: E402

THREADS = int(os.environ.get("XM_ORACLE_THREADS", os.cpu_count() or 1))


def _write(name, rec):
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")


def cases():
    """Every case of tests/cases.py: oracle counts (and root-subset sums)."""
    from tests.cases import CASES
    out = {}
    for name, c in CASES.items():
        t = time.time()
        g = c["graph"]()
        pats = c["patterns"]()
        if "roots" in c:
            vals = [str(oracle.count(g, p, roots=c["roots"], root_vertex=rv, threads=THREADS, mode="B"))
                    for p, rv in zip(pats, c["root_vertex"])]
        else:
            vals = [str(oracle.count(g, p, threads=THREADS, mode="B")) for p in pats]
        out[name] = {"graph": g.name, "m": g.m, "patterns": [list(map(list, p.arcs)) for p in pats],
                     "k": [p.k for p in pats], "counts": vals}
        print(name, round(time.time() - t, 2), flush=True)
    _write("cases", out)


def uniform2000():
    g = xmgen.uniform_digraph(2000, 20000, 0)
    out = {}
    for p in ["bifan", "ffl", "c3", "c4", "tt4p", "c5chord", "outstar3", "mixed_star", "p7hub"]:
        out[p] = str(oracle.count(g, xmgen.named(p), threads=THREADS))
    _write("uniform2000", {"graph": "uniform_digraph(n=2000, m=20000, seed=0)", "m": g.m,
                           "counts": out})


def rmat16():
    g = xmgen.rmat(16, seed=0)
    out, secs = {}, {}
    for p in ["ffl", "c3", "bifan", "c4"]:
        t = time.time()
        out[p] = str(oracle.count(g, xmgen.named(p), threads=THREADS))
        secs[p] = round(time.time() - t, 2)
        print(p, out[p], secs[p], flush=True)
    _write("rmat16", {"graph": "rmat(scale=16, edge_factor=16, abcd=(.57,.19,.19,.05), seed=0)",
                      "m": g.m, "counts": out, "oracle_seconds": secs, "threads": THREADS})


def rmat20_subset():
    """Root-subset parity at scale 20: exact partial sums over listed roots."""
    g = xmgen.rmat(20, seed=0)
    deg = g.out_deg() + g.in_deg()
    # mid-degree roots (ranks 2000-2015) plus a seeded uniform sample; the
    # largest hubs (~40K arcs) would take the oracle hours per pattern
    order = np.argsort(-deg, kind="stable")
    mids = order[2000:2016]
    rng = np.random.default_rng(20)
    sample = rng.choice(g.n, size=512, replace=False)
    roots = np.unique(np.concatenate([mids, sample])).astype(np.uint32)
    sample_only = np.sort(sample[:256]).astype(np.uint32)
    res = {}
    # c5chord enumerates four levels from its start vertex: the mid-degree
    # roots alone would take the oracle hours, so it uses the uniform sample
    for p, rv, rr in [("tt4p", 0, roots), ("c5chord", 0, sample_only)]:
        t = time.time()
        c = oracle.count(g, xmgen.named(p), roots=rr, root_vertex=rv, threads=THREADS, mode="B")
        res[p] = {"root_vertex": rv, "count": str(c), "seconds": round(time.time() - t, 2),
                  "roots": rr.tolist()}
        print(p, {k: v for k, v in res[p].items() if k != "roots"}, flush=True)
    _write("rmat20_subset", {"graph": "rmat(scale=20, edge_factor=16, abcd=(.57,.19,.19,.05), seed=0)",
                             "m": g.m, "results": res})


def _per_root(g, pat, roots, root_vertex, workers):
    """Oracle counts of one pattern per root, one root per oracle call, the
    calls spread over `workers` host threads (the oracle runs single-threaded
    per call and releases the interpreter while it counts)."""
    from concurrent.futures import ThreadPoolExecutor

    prep = oracle.Prepared(g)  # in-lists built once for every root

    def one(r):
        t = time.time()
        c = prep.count(pat, roots=np.array([r], dtype=np.uint32), root_vertex=root_vertex, mode="B")
        print(pat.name, int(r), c, round(time.time() - t, 1), flush=True)
        return str(c), round(time.time() - t, 1)

    with ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(one, [int(r) for r in roots]))
    return [c for c, _ in res], [s for _, s in res]


def rmat20_hubs():
    """Per-root oracle counts on R-MAT scale 20 hub roots (generated ids).

    tt4p: the 16 nodes of largest total degree (ranks 0-15, degree ~31K-40K);
    the oracle takes 20-60 minutes per such root.  c5chord enumerates three
    levels below its start vertex in the oracle's order: a root of degree
    ~450 (rank ~8,000) already takes ~4 minutes, one of rank 4,000 (degree
    ~1,300) did not finish in 25 minutes; it gets the eight roots of ranks
    8000-8007, the highest-ranked ones within a budget of ~5 minutes each."""
    g = xmgen.rmat(20, seed=0)
    deg = g.out_deg() + g.in_deg()
    order = np.argsort(-deg, kind="stable")
    res = {}
    for name, ranks in [("c5chord", range(8000, 8008)), ("tt4p", range(0, 16))]:
        roots = order[list(ranks)].astype(np.uint32)
        t = time.time()
        counts, secs = _per_root(g, xmgen.named(name), roots, 0, THREADS)
        res[name] = {"root_vertex": 0, "ranks": list(ranks), "roots": roots.tolist(),
                     "degrees": deg[roots].tolist(), "counts": counts, "seconds": secs,
                     "wall_seconds": round(time.time() - t, 1)}
        _write("rmat20_hubs", {"graph": "rmat(scale=20, edge_factor=16, abcd=(.57,.19,.19,.05), seed=0)",
                               "m": g.m, "mode": "B (last vertex with one constraint counted from |L|)",
                               "threads": THREADS, "results": res})


SUBSET_HUB_RANK = {3: 0, 4: 256, 5: 4096, 6: 65536}
SUBSET_OTHER_RANK = {3: 0, 4: 0, 5: 16384, 6: 262144}


def batch_subsets(workers=None):
    """Root-subset parity for 16 of the 256 batch patterns on R-MAT scale 22:
    per size 3-6 the two with the longest plain launch and two seeded others.
    Each is counted on roots of its own root share (the roots the batch
    counts), mapped back to the generated ids, one oracle count per root:
    the two of largest degree in the share at or above degree rank
    SUBSET_HUB_RANK[k] and 30 seeded others at or above SUBSET_OTHER_RANK[k]
    (stored ids are degree ranks).  The floors keep the oracle within
    minutes per pattern: a 4-vertex pattern on a rank-15 hub took it 12
    minutes, a 5-vertex one on a rank-1,087 root 70 s, a 6-vertex one on a
    rank-65,599 root 68 s.  The plan's start vertex (root_vertex) is the one
    the batch's plan uses; it only selects which per-root count is stored."""
    from paper_2404_11105_amd import workloads
    rec = json.load(open(workloads.BATCH_PATH))
    acc = rec["accepted"]
    rng = np.random.default_rng(256)
    pick = []
    for k in (3, 4, 5, 6):
        idx = [i for i, e in enumerate(acc) if e["k"] == k]
        heavy = sorted(idx, key=lambda i: -acc[i]["plain_ms"])[:2]
        rest = [i for i in idx if i not in heavy]
        pick += heavy + [int(x) for x in rng.choice(rest, size=2, replace=False)]
    g = workloads.batch_graph()
    new_of_old = workloads.degree_order(g)
    old_of_new = np.empty_like(new_of_old)
    old_of_new[new_of_old] = np.arange(g.n, dtype=np.uint32)
    pats = workloads.batch_patterns()
    def stored_roots(i):
        e = acc[i]
        share = workloads.share_roots(g.n, e["share"])
        hubs = share[share >= SUBSET_HUB_RANK[e["k"]]][:2]
        others = np.setdiff1d(share[share >= SUBSET_OTHER_RANK[e["k"]]], hubs)
        ri = np.random.default_rng(2560 + i)
        return np.concatenate([hubs, np.sort(ri.choice(others, size=min(30, others.size), replace=False))])

    out = []
    path = os.path.join(HERE, "batch256_subsets.json")
    if os.path.exists(path):  # continue a run that stopped: keep the patterns done with these roots
        out = [r for r in json.load(open(path))["patterns"]
               if r["index"] in pick and r["stored_roots"] == stored_roots(r["index"]).tolist()]
    for i in pick:
        if any(r["index"] == i for r in out):
            continue
        e = acc[i]
        stored = stored_roots(i)
        roots = old_of_new[stored]
        from paper_2404_11105_amd.api import Plan
        rv = Plan(pats[i], reduced=True, symmetry=e["symmetry"], root_share=e["share"]).describe()["root_vertex"]
        t = time.time()
        counts, secs = _per_root(g, pats[i], roots, rv, workers or THREADS)
        out.append({"index": i, "k": e["k"], "seed": e["seed"], "share": e["share"], "symmetry": e["symmetry"],
                    "plain_ms": e["plain_ms"], "root_vertex": rv, "stored_roots": stored.tolist(),
                    "roots": roots.tolist(), "counts": counts, "oracle_seconds": round(sum(secs), 1),
                    "wall_seconds": round(time.time() - t, 1)})
        print("pattern", i, e["k"], e["share"], sum(int(c) for c in counts), out[-1]["wall_seconds"], flush=True)
        _write("batch256_subsets", {"graph": "rmat(scale=22, edge_factor=16, abcd=(.57,.19,.19,.05), seed=0)",
                                    "m": g.m, "mode": "B", "patterns": out})


SERVE_REQUESTS = [  # (R-MAT scale, seed, pattern): one request per serving graph
    (18, 0, "p7hub"), (19, 1, "rand6"), (20, 2, "c5chord"), (21, 3, "rand5"),
    (22, 4, "bifan"), (23, 5, "rand4"), (24, 6, "ffl"), (24, 7, "c3"),
]


def serve_pattern(name):
    return {"rand6": lambda: xmgen.random_pattern(6, 777), "rand5": lambda: xmgen.random_pattern(5, 555),
            "rand4": lambda: xmgen.random_pattern(4, 444)}.get(name, lambda: xmgen.named(name))()


def serve_roots(g, seed, hubs: bool):
    """64 roots in the generated ids: with hubs, degree ranks 1000-1003 (lists
    of hundreds to thousands of arcs) and 60 seeded nodes below degree rank
    10,000; without, 64 seeded nodes below degree rank 50,000 (the oracle
    enumerates every level but the last one, which is out of its reach on the
    largest hubs, and for patterns of 5 or more vertices on any hub)."""
    deg = g.out_deg() + g.in_deg()
    order = np.argsort(-deg, kind="stable")
    rng = np.random.default_rng(1000 + seed)
    if not hubs:
        # below the 50,000 largest: generator ids are skewed, low ids are hubs
        return np.sort(rng.choice(order[50000:], size=64, replace=False)).astype(np.uint32)
    uni = rng.choice(order[10000:], size=60, replace=False)
    return np.unique(np.concatenate([order[1000:1004], uni])).astype(np.uint32)


def serve_scales():
    """Per-root oracle counts of one request per serving graph (R-MAT scales
    18-24, 16 arcs per node, seeds 0-7), start vertex 0, on 64 roots each
    (with four hubs for the patterns of at most 4 vertices).  A 4-cycle on
    the scale-24 graph ran over 40 minutes without finishing a root, so that
    graph's second request is a 3-cycle."""
    out = []
    path = os.path.join(HERE, "serve_scales.json")
    if os.path.exists(path):  # continue a run that stopped: keep the requests done
        out = [r for r in json.load(open(path))["requests"]
               if (r["scale"], r["seed"], r["pattern"]) in SERVE_REQUESTS]
    for scale, seed, name in SERVE_REQUESTS:
        if any((r["scale"], r["seed"], r["pattern"]) == (scale, seed, name) for r in out):
            continue
        t = time.time()
        g = xmgen.rmat(scale, seed=seed)
        pat = serve_pattern(name)
        roots = serve_roots(g, seed, hubs=pat.k <= 4)
        counts, secs = _per_root(g, pat, roots, 0, THREADS)
        out.append({"scale": scale, "seed": seed, "pattern": name, "arcs": [list(a) for a in pat.arcs],
                    "k": pat.k, "m": g.m, "root_vertex": 0, "roots": roots.tolist(), "counts": counts,
                    "oracle_seconds": round(sum(secs), 1), "wall_seconds": round(time.time() - t, 1)})
        print(scale, name, sum(int(c) for c in counts), out[-1]["wall_seconds"], flush=True)
        del g
        _write("serve_scales", {"recipe": "rmat(scale, edge_factor=16, abcd=(.57,.19,.19,.05), seed)",
                                "mode": "B", "requests": out})


if __name__ == "__main__":
    for name in sys.argv[1:] or ["cases", "uniform2000", "rmat16", "rmat20_subset"]:
        globals()[name]()
