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


if __name__ == "__main__":
    for name in sys.argv[1:] or ["cases", "uniform2000", "rmat16", "rmat20_subset"]:
        globals()[name]()
