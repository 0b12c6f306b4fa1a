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


def _read_arcs(plan: dict, pattern, reads, fallback: bool):
    """Pattern arcs whose data lists the model read, attributed from the plan
    description alone: a level's constraint (j, dir) is the arc between its
    vertex and the vertex bound at level j; a leaf descriptor's constraint
    belongs to the first leaf (in plan order) of the first signature of the
    descriptor's mask that has that constraint."""
    order, e = plan["order"], plan["e"]
    leaves = order[e:]
    arcs = set(pattern.arcs)

    def arc(u, x, d):  # d = 0: x in out(u) (u -> x); d = 1: x in in(u) (x -> u)
        a = (u, x) if d == 0 else (x, u)
        assert a in arcs, (a, plan)
        return a

    def leaf_cons(v):
        return {(j, 0) for j in range(e) if (order[j], v) in arcs} | {(j, 1) for j in range(e) if (v, order[j]) in arcs}

    sig_cons = [{tuple(c) for c in S["cons"]} for S in plan["leaf_sigs"]]
    rep = {}
    for g, sc in enumerate(sig_cons):
        rep[g] = next(v for v in leaves if leaf_cons(v) == sc)
    out = set()
    for (kind, idx), c, fb in reads:
        if fb != fallback:
            continue
        if kind == "lvl":
            j, d = plan["levels"][idx - 1]["cons"][c]
            out.add(arc(order[j], order[idx], d))
        elif kind == "sig":
            j, d = plan["leaf_sigs"][idx]["cons"][c]
            out.add(arc(order[j], rep[idx], d))
        else:
            M = plan["masks"][idx]
            j, d = M["cons"][c]
            if plan["linear"]:
                out.add(arc(order[j], rep[0], d))
                continue
            g = next(g for g in range(len(sig_cons)) if (M["mask"] >> g) & 1 and (j, d) in sig_cons[g])
            out.add(arc(order[j], rep[g], d))
    return out


def _cover_patterns():
    pats = [xmgen.named(n) for n in ["ffl", "c3", "bifan", "c4", "tt4p", "tt4p_t3", "tt4p_out", "c5chord",
                                     "outstar3", "instar3", "outstar5", "path3", "mixed_star", "p7hub"]]
    pats += [xmgen.random_pattern(k, 900 + 7 * k + s) for k in range(3, 8) for s in range(4)]
    return pats


def test_removed_arcs_are_the_lists_the_kernel_never_fetches():
    """The plan's realized cover (section 4.2) is what runs: with whole
    windows (no hub splits or window slices) the kernel model reads exactly
    the lists of the plan's fetched arcs, never those of a removed arc, whose
    candidates come from the including arc's result (section 5.2); the
    fetched arcs are a constraint cover (every removed arc shares a source or
    a destination with a fetched arc that reaches it, Theorem 2.1); and the
    unconstrained minimum cover is never heavier in arcs than the realized
    one.  Unreduced plans fetch every arc."""
    # every pattern embeds in a complete digraph, so every descriptor runs
    g = xmgen.complete_digraph(8)
    n_removed = 0
    for pat in _cover_patterns():
        for reduced in (True, False):
            plan = describe_plan(pat, reduced)
            fetched = {tuple(a) for a in plan["cover"]["fetched"]}
            removed = {tuple(a) for a in plan["cover"]["removed"]}
            assert fetched | removed == set(pat.arcs) and not fetched & removed
            assert plan["removed_edges"] == len(removed)
            if not reduced:
                assert not removed, pat
            m = Model(plan, g, chunk=64, split=1 << 16, cap=1 << 16, split_work=1 << 30)
            assert m.run() == oracle.count(g, pat), pat
            assert _read_arcs(plan, pat, m.reads, False) == fetched, (pat, plan["order"])
            assert not _read_arcs(plan, pat, m.reads, True), pat  # no fallback with whole windows
            for a, b in removed:
                assert any(a == u or b == w for u, w in fetched), ((a, b), pat)
            assert len(plan["min_cover"]) <= len(fetched)
            n_removed += len(removed)
    assert n_removed > 20


def test_reuse_fallback_reads_only_lists_of_the_same_inclusion_group():
    """When a window holds only part of a reuse source's candidates (hub
    sub-ranges, slices), a reusing level fetches its own lists instead; every
    such list is the list of an arc in the same inclusion group as a fetched
    arc (same bound endpoint, same direction), so the data touched is the
    including arc's."""
    g = xmgen.rmat(7, seed=7)  # hubs of degree > 64: split roots and partial windows
    fallbacks = 0
    for pat in _cover_patterns()[:8]:
        plan = describe_plan(pat, True)
        fetched = {tuple(a) for a in plan["cover"]["fetched"]}
        m = Model(plan, g, chunk=1, split=64, cap=64, split_work=4096, max_windows=200000)
        assert m.run() == oracle.count(g, pat), pat
        fb = _read_arcs(plan, pat, m.reads, True)
        fallbacks += len(fb)
        for a, b in fb - fetched:
            assert any(a == u for u, w in fetched) or any(b == w for u, w in fetched), ((a, b), pat)
    assert fallbacks > 0


@pytest.mark.parametrize("share", [1, 2, 3])
def test_root_share_counts_the_share_exactly(share):
    """A plan with a root share counts exactly the embeddings whose start
    vertex maps into the share (stored id r with r mod 2^s = 2^s - 1): the
    kernel model equals the oracle restricted to those roots, with and
    without symmetry breaking (only automorphisms fixing the start vertex)."""
    g = xmgen.rmat(7, seed=7)
    roots = [r for r in range(g.n) if (r + 1) % (1 << share) == 0]
    for name in ["bifan", "c4", "tt4p", "ffl", "mixed_star"]:
        pat = xmgen.named(name)
        for sym in (False, "above"):
            plan = describe_plan(pat, True, symmetry=sym, root_share=share)
            assert plan["root_share"] == share
            if sym:
                assert plan["sym_fixes_root"] == 1
            want = oracle.count(g, pat, roots=roots, root_vertex=plan["order"][0])
            m = Model(plan, g, chunk=3, split=64, cap=128, split_work=4096)
            assert m.run() == want, (name, sym, share)
