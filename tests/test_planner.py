"""Planner tests (CPU): plan validity, paper pins, and plan semantics vs the oracle."""
import numpy as np
import pytest

import oracle
import xmgen
from paper_2404_11105_amd import Plan, describe_plan
from paper_2404_11105_amd._lib import XminerError, lib
from tests import pins
from tests.plan_sim import simulate

NAMES = ["arc", "pair2", "ffl", "c3", "bifan", "c4", "path3", "outstar3", "instar3", "outstar5",
         "tt4p", "tt4p_t3", "tt4p_out", "c5chord", "mixed_star", "p7hub"]


def small_graphs():
    gs = []
    for seed in range(3):
        rng = np.random.default_rng(40 + seed)
        n = 8
        A = rng.random((n, n)) < 0.4
        np.fill_diagonal(A, False)
        u, v = np.nonzero(A)
        gs.append(xmgen.from_arcs(n, u, v))
    gs.append(xmgen.rmat(6, edge_factor=4, seed=1))
    return gs


def patterns():
    pats = [xmgen.named(x) for x in NAMES]
    for k in range(3, 8):
        for s in range(5):
            pats.append(xmgen.random_pattern(k, 500 + 10 * k + s))
    return pats


def test_cycles_are_irreducible():
    # directed cycles: every inclusion group is a single edge, so the cover keeps all
    for name, k in [("c3", 3), ("c4", 4)]:
        d = describe_plan(xmgen.named(name), True)
        assert len(d["min_cover"]) == k and len(d["greedy_cover"]) == k
        assert d["removed_edges"] == 0
        assert all(L["reuse"] < 0 for L in d["levels"])
        assert d["t"] == 1


def test_start_vertex_has_max_degree():
    for pat in patterns():
        d = describe_plan(pat, True)
        deg = [0] * pat.k
        for a, b in pat.arcs:
            deg[a] += 1
            deg[b] += 1
        assert deg[d["root_vertex"]] == max(deg)


def test_min_cover_not_larger_than_greedy_and_covers():
    for pat in patterns():
        d = describe_plan(pat, True)
        arcs = [tuple(a) for a in d["arcs"]]
        cover = [tuple(a) for a in d["min_cover"]]
        covered = set()
        for (u, w) in cover:
            covered |= {a for a in arcs if a[0] == u or a[1] == w}
        assert covered == set(arcs)
        assert len(d["min_cover"]) <= len(d["greedy_cover"])


def test_reduced_plan_not_larger():
    # the reduced plan never enumerates more levels than the unreduced one
    for pat in patterns():
        r = describe_plan(pat, True)
        u = describe_plan(pat, False)
        assert r["e"] <= u["e"]
        assert r["k"] == u["k"] == pat.k


@pytest.mark.parametrize("reduced", [True, False])
def test_plan_semantics_match_oracle(reduced):
    graphs = small_graphs()
    for pat in patterns():
        d = describe_plan(pat, reduced)
        for g in graphs:
            if g.n < pat.k:
                continue
            assert simulate(d, g) == oracle.count(g, pat), (pat.name, reduced)


def test_forced_root_vertex():
    g = small_graphs()[0]
    pat = xmgen.named("c4")
    for v in range(4):
        p = Plan(pat, True, root_vertex=v)
        assert p.root_vertex == v
        assert simulate(p.describe(), g) == oracle.count(g, pat)


def test_leaf_terms_are_falling_factorial_for_one_signature():
    d = describe_plan(xmgen.named("outstar5"), True)
    assert d["e"] == 1 and d["t"] == 5 and len(d["leaf_sigs"]) == 1
    # sum of coef * s^(#blocks) must equal s(s-1)(s-2)(s-3)(s-4)
    for s in range(0, 12):
        val = sum(t["coef"] * s ** len(t["masks"]) for t in d["terms"])
        assert val == pins.falling(s, 5)


@pytest.mark.parametrize("bad", [
    (1, [(0, 0)]), (3, [(0, 1)]), (2, [(0, 2)]), (8, [(i, i + 1) for i in range(7)]), (3, []),
])
def test_bad_patterns_rejected(bad):
    k, arcs = bad
    with pytest.raises(XminerError) as ei:
        Plan(xmgen.Pattern(k, tuple(arcs)) if arcs else _Raw(k), True)
    assert ei.value.code == -2


class _Raw:
    def __init__(self, k):
        self.k = k
        self.arcs = ()
        self.name = "raw"

    def arcs_u8(self):
        return b""


def test_plan_work_complete_digraph_closed_form():
    """xm_plan_work on K_n: every list holds n-1 nodes and every candidate survives
    except the bound ones, so the partial matches of level i are n!/(n-i-1)!."""
    from paper_2404_11105_amd import plan_work
    n = 7
    g = xmgen.complete_digraph(n)
    for name in ["c4", "bifan", "tt4p", "c5chord", "p7hub"]:
        for reduced in (True, False):
            p = Plan(xmgen.named(name), reduced)
            d = p.describe()
            w = plan_work(g, p)
            e = d["e"]
            assert w["roots"] == n
            partial = sum(pins.complete_count(n, i + 1) for i in range(1, e))
            assert w["partial_matches"] == partial, (name, reduced)
            # every fetched list has n-1 entries; reused candidate sets hold the survivors
            assert w["elements"] > 0 and w["fetches"] >= partial
            assert w["elements"] <= (n - 1) * w["fetches"]


def test_plan_work_reduced_reads_less_on_stars():
    from paper_2404_11105_amd import plan_work
    g = xmgen.rmat(9, seed=1)
    pat = xmgen.named("mixed_star")
    red = plan_work(g, Plan(pat, True))
    unred = plan_work(g, Plan(pat, False))
    assert red["elements"] < unred["elements"]
    assert red["partial_matches"] == 0 < unred["partial_matches"]
