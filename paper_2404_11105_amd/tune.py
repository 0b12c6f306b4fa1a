"""Autotuner for xm_count launch parameters.

For one resident graph and one batch of plans it searches the launch
parameters that only change speed, never the counts:

  split_work  target work of a stealable first-level task (hub splitting)
  split       largest first-level sub-range of a split root
  chunk       roots per root task (0: sized from the task count)
  waves_per_cu resident waves (0 = from occupancy)
  merge_min   cooperative merge threshold (0xFFFFFFFF = off)

by coordinate descent from the library defaults: each parameter in turn is
set to every value of its list with the others fixed, the batched launch is
timed with HIP events on the launch stream (one warm-up, then the median of
`reps` launches), and the fastest value is kept.  Every configuration must
return the same counts, else the tuner raises.  Results are cached in a
JSON file keyed by the graph's size and the plans' descriptions.

Every launch runs under a Watchdog: a trial that has not finished within a
few times the best time so far is cancelled on the device and counted as
slower; the default configuration gets `first_budget_s`, and the tuner
raises if it does not finish within it.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

SPACE = [
    ("split_work", [4096, 16384, 65536]),
    ("split", [64, 128, 512]),
    ("chunk", [0, 1, 4, 16, 64]),
    ("waves_per_cu", [0, 12, 16, 32]),
    ("merge_min", [0xFFFFFFFF, 64]),
]
DEFAULTS = dict(split_work=4096, split=64, chunk=0, waves_per_cu=0, merge_min=0xFFFFFFFF)


def signature(graph, plans) -> str:
    from .api import plan_json
    h = hashlib.sha256()
    h.update(f"{graph.n}:{graph.m}".encode())
    for p in plans:
        h.update(plan_json(p).encode())
    return h.hexdigest()[:24]


def time_launch(graph, plans, stream, reps: int = 3, watchdog=None, budget_s: float = 0.0,
                log=None, **opts):
    """Median GPU milliseconds of one batched launch, and its counts.

    One untimed launch, then `reps` timed ones; with a watchdog every launch
    is cancelled after budget_s seconds, and then (inf, None) is returned."""
    import torch
    from .api import Counter
    c = Counter(graph, plans, cancel=watchdog, **opts)
    ms = []
    for i in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        if watchdog is not None:
            watchdog.arm(budget_s)
        e0.record(stream)
        c.run(stream)
        e1.record(stream)
        stream.synchronize()
        if watchdog is not None:
            watchdog.disarm()
        counts, status = c.results()
        if any(s == -7 for s in status):
            return float("inf"), None
        if any(s != 0 for s in status):
            raise RuntimeError(f"launch status {status} with {opts}")
        if log:
            log(f"[tune]   launch {i}: {e0.elapsed_time(e1):.1f} ms")
        if i:
            ms.append(e0.elapsed_time(e1))
    ms.sort()
    return ms[len(ms) // 2], counts


def tune(graph, plans, stream=None, cache_path: str | None = None, reps: int = 3,
         budget_s: float = 120.0, log=None, first_budget_s: float = 60.0):
    """Best launch options for (graph, plans); returns (opts, record)."""
    import torch
    from .api import Watchdog
    key = signature(graph, plans)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
        if key in cache:
            return dict(cache[key]["opts"]), cache[key]
    stream = stream or torch.cuda.Stream()
    t0 = time.time()
    best = dict(DEFAULTS)
    wd = Watchdog()
    if log:
        log(f"[tune] default {best}")
    best_ms, ref_counts = time_launch(graph, plans, stream, reps, wd, first_budget_s, log, **best)
    if ref_counts is None:
        raise RuntimeError(f"default launch did not finish within {first_budget_s} s")
    trials = [(dict(best), best_ms)]
    for name, values in SPACE:
        for v in values:
            if v == best[name] or time.time() - t0 > budget_s:
                continue
            cand = dict(best, **{name: v})
            ms, counts = time_launch(graph, plans, stream, reps, wd,
                                     max(1.0, 4e-3 * best_ms), None, **cand)
            if counts is None:
                if log:
                    log(f"[tune] {name}={v}: cancelled after {max(1.0, 4e-3 * best_ms):.1f} s")
                trials.append((cand, ms))
                continue
            if counts != ref_counts:
                raise RuntimeError(f"counts changed with {cand}")
            trials.append((cand, ms))
            if log:
                log(f"[tune] {name}={v}: {ms:.2f} ms (best {best_ms:.2f})")
            if ms < best_ms:
                best, best_ms = cand, ms
    rec = {"opts": best, "ms": best_ms, "default_ms": trials[0][1], "trials": len(trials),
           "seconds": round(time.time() - t0, 1)}
    if cache_path:
        cache[key] = rec
        d = os.path.dirname(cache_path)
        if d:
            os.makedirs(d, exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return dict(best), rec
