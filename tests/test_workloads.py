"""The stored benchmark workloads (CPU): the 256-pattern batch and the
serving pool have the stated composition, every pattern is the seeded draw
its entry names, and the helpers that pick roots and row thresholds follow
their definitions."""
import json

import numpy as np

import xmgen
from paper_2404_11105_amd import workloads


def test_batch_has_64_patterns_of_each_size_on_stated_shares():
    rec = json.load(open(workloads.BATCH_PATH))
    acc = rec["accepted"]
    assert len(acc) == 256
    for k in (3, 4, 5, 6):
        mine = [e for e in acc if e["k"] == k]
        assert len(mine) == 64
        # seeds are the size's draw order: accepted ones increase, rejected ones fill the gaps
        seeds = [e["seed"] for e in mine]
        assert seeds == sorted(seeds) and seeds[0] >= workloads.SEED_BASE[k]
        assert seeds[-1] < workloads.SEED_BASE[k] + rec["draws_per_k"][str(k)]
        assert len(mine) + rec["rejected_per_k"][str(k)] == rec["draws_per_k"][str(k)]
    assert all(e["share"] in rec["shares"] and e["plain_ms"] <= rec["cap_ms"] for e in acc)
    pats = workloads.batch_patterns()
    for e, p in zip(acc, pats):
        q = xmgen.random_pattern(e["k"], e["seed"])
        assert (p.k, p.arcs) == (q.k, q.arcs)


def test_serving_pool_has_16_patterns_of_each_size_3_to_7():
    pool = workloads.serve_pool()
    sizes = [p.k for p, _ in pool]
    assert all(sizes.count(k) == workloads.SERVE_PER_SIZE for k in (3, 4, 5, 6, 7))
    rec = json.load(open(workloads.SERVE7_PATH))
    assert all(0 <= sh <= 31 for _, sh in pool)
    assert [sh for p, sh in pool if p.k == 7] == [e["share"] for e in rec["accepted"]]


def test_share_roots_are_the_ids_with_low_bits_set():
    n = 1000
    for s in (0, 1, 3, 6):
        r = workloads.share_roots(n, s)
        want = [x for x in range(n) if (x + 1) % (1 << s) == 0]
        assert r.tolist() == want


def test_degree_order_is_a_permutation_by_decreasing_degree():
    g = xmgen.rmat(8, seed=1)
    new_of_old = workloads.degree_order(g)
    assert np.array_equal(np.sort(new_of_old), np.arange(g.n))
    deg = g.out_deg() + g.in_deg()
    by_new = np.empty(g.n, dtype=np.int64)
    by_new[new_of_old] = deg
    assert np.all(np.diff(by_new) <= 0)


def test_row_threshold_fits_the_budget():
    g = xmgen.rmat(10, seed=2)
    row_bytes = (g.n + 31) // 32 * 4
    lens = np.concatenate([np.diff(g.out_off.astype(np.int64)), np.diff(g.in_off.astype(np.int64))])
    for budget in (row_bytes * 3, row_bytes * 40, 1 << 30):
        t = workloads.row_threshold(g, budget, 32)
        if t:
            assert (lens >= t).sum() * row_bytes <= budget
            assert t >= 32
