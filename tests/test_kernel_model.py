"""CPU model of the count kernel's control flow: termination and parity.

Runs tests/kernel_model.py (which follows count.hip step by step and
asserts every buffer index) under extreme tunings that force hub splitting,
partial windows and reuse fallbacks, and compares with the oracle.
"""
import pytest

import oracle
import xmgen
from paper_2404_11105_amd import describe_plan
from tests.cases import symmetric_patterns, symmetric_patterns_large
from tests.kernel_model import Model

TUNINGS = [dict(chunk=1, split=64, cap=64), dict(chunk=64, split=64, cap=128, split_work=4096),
           dict(chunk=7, split=100, cap=4096)]


@pytest.mark.parametrize("tune", TUNINGS, ids=lambda t: f"c{t['chunk']}s{t['split']}k{t['cap']}")
def test_model_terminates_and_matches_oracle(tune):
    g = xmgen.rmat(7, seed=7)  # hubs of degree > 64 exist, so roots get split
    assert max(g.out_deg().max(), g.in_deg().max()) > 64
    for name in ["bifan", "c4", "tt4p", "ffl", "c3", "mixed_star"]:
        pat = xmgen.named(name)
        want = oracle.count(g, pat)
        for reduced in (True, False):
            m = Model(describe_plan(pat, reduced), g, **tune, max_windows=200000)
            assert m.run() == want, (name, reduced)


def test_model_random_patterns_small_cap():
    g = xmgen.uniform_digraph(60, 500, 3)
    pat = xmgen.named("p7hub")
    for reduced in (True, False):
        assert Model(describe_plan(pat, reduced), g, chunk=3, split=64, cap=64).run() == oracle.count(g, pat)
    for k in range(3, 7):
        for s in range(3):
            pat = xmgen.random_pattern(k, 700 + 10 * k + s)
            want = oracle.count(g, pat)
            for reduced in (True, False):
                m = Model(describe_plan(pat, reduced), g, chunk=3, split=64, cap=64)
                assert m.run() == want, (k, s, reduced)


def test_symmetry_multiplier_is_the_orbit_size():
    """With one counted leaf every vertex is conditioned, so the multiplier is
    |Aut(P)| (counted here by brute force); in general it divides it."""
    for pat in symmetric_patterns() + symmetric_patterns_large():
        aut = pat.automorphisms()
        for reduced in (True, False):
            d = describe_plan(pat, reduced, symmetry=True)
            assert aut % d["sym_mult"] == 0, (pat.name, reduced)
            # the reversed conditions: same orbits, same bound levels
            e = describe_plan(pat, reduced, symmetry="below")
            assert e["sym_mult"] == d["sym_mult"]
            assert [L["gt"] for L in e["levels"]] == [L["gt"] for L in d["levels"]]
            assert all(L["lt"] == 1 for L in e["levels"] + e["leaf_sigs"])
            assert all(L["lt"] == 0 for L in d["levels"] + d["leaf_sigs"])
            if d["t"] == 1:
                assert d["sym_mult"] == aut, (pat.name, reduced)
            # a bound only ever refers to earlier levels
            for i, L in enumerate(d["levels"], start=1):
                assert L["gt"] < (1 << i)
        assert describe_plan(pat, True)["sym_mult"] == 1  # off unless asked for


@pytest.mark.parametrize("tune,direction", [(TUNINGS[0], "above"), (TUNINGS[1], "below")],
                         ids=["c1s64k64-above", "c64s64k128-below"])
def test_model_symmetry_broken_plans_match_oracle(tune, direction):
    """Counting one embedding per orbit and scaling gives the oracle's
    labelled count, with hub splits and partial windows forced."""
    hub = xmgen.rmat(7, seed=7)  # lists longer than a split: hub roots are split
    small = xmgen.uniform_digraph(40, 420, 11)
    for g in (hub, small):
        for pat in symmetric_patterns() + (symmetric_patterns_large() if g is small else []):
            if g is hub and (pat.k > 4 or pat.name == "mixed_star") and pat.name not in ("k23", "c5"):
                continue  # the pure-Python model is slow on these there
            want = oracle.count(g, pat)
            for reduced in (True, False):
                m = Model(describe_plan(pat, reduced, symmetry=direction), g, **tune, max_windows=400000)
                assert m.run() == want, (pat.name, reduced)


def test_symmetry_with_forced_root_fixes_it():
    """With a forced start vertex v only automorphisms fixing v are used: the
    multiplier of an unreduced plan (every vertex conditioned) is the size of
    v's stabiliser, counted here by brute force, and the plan's total still
    equals the oracle's."""
    import itertools
    g = xmgen.uniform_digraph(40, 420, 11)
    for pat in symmetric_patterns()[:5] + symmetric_patterns()[7:9]:
        arcs = set(pat.arcs)
        auts = [q for q in itertools.permutations(range(pat.k))
                if {(q[a], q[b]) for a, b in arcs} == arcs]
        want = oracle.count(g, pat)
        for v in range(pat.k):
            d = describe_plan_forced(pat, v)
            assert d["sym_fixes_root"] == 1 and d["root_vertex"] == v
            assert d["sym_mult"] == sum(1 for q in auts if q[v] == v), (pat.name, v)
            assert Model(d, g, chunk=3, split=64, cap=64).run() == want, (pat.name, v)


def describe_plan_forced(pat, v):
    from paper_2404_11105_amd import Plan
    return Plan(pat, reduced=False, root_vertex=v, symmetry="above").describe()
