"""GPU parity: the HIP path through the C ABI against the oracle, bit-exact.

Every expected value comes from the oracle (at test time, or stored under
tests/golden/ by make_golden.py, which calls only the oracle) or from a
closed form written out in tests/pins.py.
"""
import json
import os

import numpy as np
import pytest

import oracle
import xmgen
from tests import pins

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

from tests.cases import NAMED_ALL as NAMED


@pytest.fixture(scope="module")
def xa():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_11105_amd as xa
    return xa


def run(xa, g, pats, reduced=True, G=None, symmetry=False, **opts):
    G = G or xa.Graph(g)
    plans = [xa.Plan(p, reduced=reduced, graph=G, symmetry=symmetry) for p in pats]
    c = xa.Counter(G, plans, **opts)
    c.run()
    counts, status = c.results()
    assert all(s == 0 for s in status), status
    return counts


def banner(msg):
    print(f"[case] {msg}", flush=True)


def golden_case(name):
    from tests.cases import CASES
    gold = json.load(open(os.path.join(HERE, "golden", "cases.json")))[name]
    c = CASES[name]
    g = c["graph"]()
    pats = c["patterns"]()
    assert [list(map(list, p.arcs)) for p in pats] == gold["patterns"], "case drifted from its golden"
    return c, g, pats, [int(x) for x in gold["counts"]]


def test_config1_bifan_reduced(xa):
    banner("uniform 2000/20000 seed 0, bifan reduced")
    g = xmgen.uniform_digraph(2000, 20000, 0)
    pat = xmgen.named("bifan")
    assert run(xa, g, [pat]) == [oracle.count(g, pat)]


@pytest.mark.parametrize("case", ["uniform2000_named", "rmat11_named", "rand_uniform300", "rand_rmat8"])
@pytest.mark.parametrize("reduced", [True, False])
def test_cases_vs_oracle(xa, case, reduced):
    banner(f"{case} reduced={reduced}")
    _, g, pats, want = golden_case(case)
    assert run(xa, g, pats, reduced=reduced) == want


@pytest.mark.parametrize("tune", [dict(chunk=1, split=64, cap=64), dict(chunk=64, split=64, cap=128, split_work=4096),
                                  dict(chunk=7, split=100, cap=4096, waves_per_cu=4),
                                  dict(split=512, split_work=1 << 20, merge_min=64, merge_ratio=16)])
def test_tunings_exercise_splits_and_partial_windows(xa, tune):
    banner(f"rmat 11 tunings {tune}")
    _, g, pats, want = golden_case("tune_rmat11")
    G = xa.Graph(g)
    for p, w in zip(pats, want):
        for reduced in (True, False):
            if not reduced and p.name == "mixed_star":
                continue  # enumerates ~5e8 partial matches unreduced; covered at default tuning
            banner(f"  {p.name} reduced={reduced}")
            assert run(xa, g, [p], G=G, reduced=reduced, **tune) == [w]


@pytest.mark.parametrize("rows", [dict(dense_rows=0), dict(row_min=64, dense_rows=1 << 20),
                                  dict(row_min=32, dense_rows=40 * 256)])
def test_dense_rows_do_not_change_counts(xa, rows):
    banner(f"rmat 11 named patterns with dense rows {rows}")
    _, g, pats, want = golden_case("rmat11_named")
    G = xa.Graph(g, **rows)
    info = G.dense_rows_info()
    t = info["row_min"]
    if rows["dense_rows"] == 0:
        assert t == 0 and info["bytes"] == 0
    else:
        # every list at least t long has a row, within the byte budget
        assert t >= rows["row_min"]
        n_out = int((np.diff(g.out_off.astype(np.int64)) >= t).sum())
        n_in = int((np.diff(g.in_off.astype(np.int64)) >= t).sum())
        assert (info["out_rows"], info["in_rows"]) == (n_out, n_in) and n_out + n_in > 0
        assert info["bytes"] == (n_out + n_in) * ((g.n + 31) // 32) * 4 <= rows["dense_rows"]
    for reduced in (True, False):
        assert run(xa, g, pats, G=G, reduced=reduced) == want


def test_batched_equals_plain(xa):
    banner("batched vs plain, 24 random patterns on rmat 10")
    _, g, pats, want = golden_case("batch_rmat10")
    G = xa.Graph(g)
    batched = run(xa, g, pats, G=G)
    plain = [run(xa, g, [p], G=G)[0] for p in pats]
    assert batched == plain == want


def test_tiny_and_degenerate_graphs(xa):
    banner("tiny and degenerate graphs")
    cases = [xmgen.complete_digraph(2), xmgen.complete_digraph(5), xmgen.from_arcs(3, [0], [1]),
             xmgen.from_arcs(6, [], []), xmgen.star_hub(3, extra_nodes=2)]
    for g in cases:
        pats = [xmgen.named(n) for n in ["arc", "pair2", "ffl", "c3", "bifan", "outstar3", "c4"]]
        want = [oracle.count(g, p) for p in pats]
        assert run(xa, g, pats) == want, g.name
        assert run(xa, g, pats, reduced=False) == want, g.name
        # the same with the graph in degree order and symmetry breaking
        Gd = xa.Graph(g, order_by_degree=True)
        assert run(xa, g, pats, G=Gd, symmetry=True) == want, g.name
        assert run(xa, g, pats, G=Gd, reduced=False, symmetry="below") == want, g.name


def test_complete_digraph_closed_form(xa):
    banner("complete digraph 9: n!/(n-k)!")
    g = xmgen.complete_digraph(9)
    pats = [xmgen.named(n) for n in NAMED] + [xmgen.random_pattern(k, 77 + k) for k in range(3, 8)]
    want = [pins.complete_count(9, p.k) for p in pats]
    assert run(xa, g, pats) == want
    assert run(xa, g, pats, reduced=False) == want


def test_u128_star_hub_closed_form(xa):
    banner("out-star hub D=100000, 5 leaves: falling factorial > 2^64")
    D = 100000
    g = xmgen.star_hub(D)
    pat = xmgen.named("outstar5")
    want = pins.falling(D, 5)
    assert want > 2 ** 64
    assert run(xa, g, [pat]) == [want]
    want3 = pins.falling(D, 3)
    assert run(xa, g, [xmgen.named("outstar3")]) == [want3]


def test_root_subset_partial_sums(xa):
    banner("root subset partial sums, rmat 11")
    c, g, pats, want = golden_case("subset_rmat11")
    G = xa.Graph(g)
    for pat, rv, w in zip(pats, c["root_vertex"], want):
        for reduced in (True, False):
            # with symmetry breaking a forced start vertex keeps subset counts exact
            for symmetry in (False, "above", "below"):
                p = xa.Plan(pat, reduced=reduced, graph=G, root_vertex=rv, symmetry=symmetry)
                cnt = xa.Counter(G, [p], roots=c["roots"])
                cnt.run()
                got, st = cnt.results()
                assert got == [w] and st == [0], (pat.name, reduced, symmetry)


@pytest.mark.skip(reason="the device statistics launch (a second kernel variant) went silent on "
                         "its only GPU run with no cause found; it was removed and work statistics "
                         "now come from the host walk xm_plan_work")
def test_stats_mode_same_counts(xa):
    banner("stats mode")


def test_graph_replay_matches_eager(xa):
    import torch
    banner("hip graph capture and replays")
    _, g, pats, want = golden_case("replay_rmat10")
    G = xa.Graph(g)
    plans = [xa.Plan(p, graph=G) for p in pats]
    s = torch.cuda.Stream()
    c = xa.Counter(G, plans)
    c.capture(s)
    for _ in range(4):
        c.run(s)
        s.synchronize()
        got, st = c.results()
        assert got == want and st == [0] * len(pats)
        torch.zeros(1000, device="cuda").sum().item()  # eager work between replays


def test_config2_full_size(xa):
    banner("rmat 16 full size, 4 patterns x reduced/unreduced vs stored oracle counts")
    gold = json.load(open(os.path.join(HERE, "golden", "rmat16.json")))["counts"]
    g = xmgen.rmat(16, seed=0)
    G = xa.Graph(g)
    names = list(gold)
    pats = [xmgen.named(n) for n in names]
    want = [int(gold[n]) for n in names]
    assert run(xa, g, pats, G=G, reduced=True) == want
    assert run(xa, g, pats, G=G, reduced=False) == want
    for direction in ("above", "below"):
        banner(f"  symmetry-broken plans, {direction}")
        assert run(xa, g, pats, G=G, reduced=True, symmetry=direction) == want
        assert run(xa, g, pats, G=G, reduced=False, symmetry=direction) == want
    banner("  graph in degree order, symmetry side chosen by the sampled walk")
    Gd = xa.Graph(g, order_by_degree=True)
    assert run(xa, g, pats, G=Gd, reduced=True, symmetry=True) == want
    assert run(xa, g, pats, G=Gd, reduced=True) == want



def test_root_deciles_sum_to_full_counts(xa):
    """Disjoint root subsets (deciles of a seeded permutation, queue sized
    from the subsets' own degrees) add up to the full counts."""
    banner("rmat 11 named patterns: ten disjoint root subsets sum to the full counts")
    _, g, pats, want = golden_case("rmat11_named")
    G = xa.Graph(g)
    plans = [xa.Plan(p, graph=G, root_vertex=0) for p in pats]
    perm = np.random.default_rng(3).permutation(g.n).astype(np.uint32)
    cuts = [round(g.n * i / 10) for i in range(11)]
    sums = [0] * len(plans)
    for i in range(10):
        c = xa.Counter(G, plans, roots=np.sort(perm[cuts[i]:cuts[i + 1]]))
        c.run()
        got, st = c.results()
        assert st == [0] * len(plans)
        sums = [a + b for a, b in zip(sums, got)]
    assert sums == want


def _sorted_rows(a):
    a = np.asarray(a, dtype=np.int64)
    return a[np.lexsort(a.T[::-1])] if a.size else a.reshape(0, a.shape[1] if a.ndim == 2 else 0)


def test_listing_equals_oracle_embeddings(xa):
    """Listing mode: the rows written are exactly the oracle's embeddings
    (pattern-vertex order), with the exact total, for unreduced plans and a
    reduced plan whose leaf group is one vertex; a small capacity keeps the
    total and writes distinct true embeddings."""
    banner("listing: uniform 60/400 and rmat 6, unreduced and one-leaf reduced plans")
    for g in (xmgen.uniform_digraph(60, 400, 12), xmgen.rmat(6, seed=8)):
        G = xa.Graph(g)
        for name in ["arc", "ffl", "c3", "bifan", "c4", "tt4p", "c5chord"]:
            p = xmgen.named(name)
            total, want = oracle.list_embeddings(g, p, cap=2_000_000)
            assert total == len(want)
            for reduced in (False, True):
                if reduced and xa.Plan(p).describe()["t"] != 1:
                    continue
                n, rows = xa.list_embeddings(G, p, cap=2_000_000, reduced=reduced)
                assert n == total and len(rows) == total, (name, reduced)
                assert np.array_equal(_sorted_rows(rows), _sorted_rows(want)), (name, reduced)
        p = xmgen.named("c4")
        total = oracle.count(g, p)
        if total > 10:
            n, rows = xa.list_embeddings(G, p, cap=10)
            assert n == total and len(rows) == 10
            allw = {tuple(r) for r in oracle.list_embeddings(g, p, cap=2_000_000)[1].tolist()}
            got = [tuple(r) for r in rows.tolist()]
            assert len(set(got)) == 10 and all(r in allw for r in got)


def test_listing_rejects_multi_leaf_plans(xa):
    banner("listing needs one plan with a one-vertex leaf group")
    g = xmgen.uniform_digraph(60, 400, 12)
    G = xa.Graph(g)
    with pytest.raises(Exception):
        xa.list_embeddings(G, xmgen.named("outstar3"), cap=100, reduced=True)


@pytest.mark.parametrize("direction", ["above", "below"])
@pytest.mark.parametrize("tune", [dict(), dict(chunk=1, split=64, cap=64),
                                  dict(chunk=64, split=64, cap=128, split_work=4096)])
def test_symmetry_broken_plans_vs_oracle(xa, tune, direction):
    """Plans that count one embedding per automorphism orbit and scale by the
    orbit size give the oracle's labelled counts: all patterns in one batched
    launch (mixed multipliers), reduced and unreduced, with hub splits and
    partial windows forced by the small tunings."""
    from tests.cases import symmetric_patterns
    pats = symmetric_patterns()
    for g in (xmgen.rmat(9, seed=3), xmgen.uniform_digraph(300, 2400, 5)):
        banner(f"symmetry-broken plans ({direction}) on {g.name}, {len(pats)} patterns, tuning {tune}")
        G = xa.Graph(g)
        want = [oracle.count(g, p, threads=8, mode="B") for p in pats]
        for reduced in (True, False):
            assert run(xa, g, pats, G=G, reduced=reduced, symmetry=direction, **tune) == want, reduced


def test_symmetry_large_groups_vs_oracle(xa):
    """Groups of order 6 and 24 and patterns of up to 7 vertices, on a graph
    small enough for the oracle: both sides, reduced and unreduced, in the
    generated and the degree order."""
    from tests.cases import symmetric_patterns_large
    pats = symmetric_patterns_large()
    g = xmgen.uniform_digraph(50, 900, 21)  # dense enough for reciprocal arcs
    banner(f"symmetry-broken plans, large groups, {g.name}")
    want = [oracle.count(g, p, threads=8) for p in pats]
    for G in (xa.Graph(g), xa.Graph(g, order_by_degree=True)):
        for reduced in (True, False):
            for direction in ("above", "below"):
                assert run(xa, g, pats, G=G, reduced=reduced, symmetry=direction) == want, (reduced, direction)


def test_symmetry_closed_forms(xa):
    """Complete digraph: n!/(n-k)! for every pattern.  Out-star hub: the
    falling factorial above 2^64 with the reduced plan (its leaf group holds
    every leaf, so the multiplier is 1: an unreduced plan there would
    enumerate ~10^18 prefixes even with symmetry breaking)."""
    banner("symmetry-broken plans: complete digraph 9 and the out-star hub")
    g = xmgen.complete_digraph(9)
    pats = [xmgen.named(n) for n in NAMED] + [xmgen.random_pattern(k, 77 + k) for k in range(3, 8)]
    want = [pins.complete_count(9, p.k) for p in pats]
    for direction in ("above", "below"):
        assert run(xa, g, pats, symmetry=direction) == want
        assert run(xa, g, pats, reduced=False, symmetry=direction) == want
    D = 100000
    g = xmgen.star_hub(D)
    for name, k in (("outstar5", 5), ("outstar3", 3)):
        assert run(xa, g, [xmgen.named(name)], symmetry=True) == [pins.falling(D, k)]


def test_symmetry_rejects_root_subsets_and_listing(xa):
    banner("symmetry-broken plans refuse root subsets and listing")
    g = xmgen.uniform_digraph(60, 400, 12)
    G = xa.Graph(g)
    p = xa.Plan(xmgen.named("c4"), graph=G, symmetry=True)
    assert p.describe()["sym_mult"] == 4
    with pytest.raises(Exception):
        c = xa.Counter(G, [p], roots=np.arange(10, dtype=np.uint32))
        c.run()
    with pytest.raises(Exception):
        c = xa.Counter(G, [p], list_cap=100)
        c.run()
    # a forced start vertex: only automorphisms fixing it, subsets allowed
    # (bi-fan from a: the swap of c and d fixes a, so the multiplier is 2)
    pr = xa.Plan(xmgen.named("bifan"), graph=G, symmetry="above", root_vertex=0)
    d = pr.describe()
    assert d["sym_fixes_root"] == 1 and d["sym_mult"] == 2
    roots = np.arange(10, dtype=np.uint32)
    c = xa.Counter(G, [pr], roots=roots)
    c.run()
    got, st = c.results()
    assert st == [0] and got == [oracle.count(g, xmgen.named("bifan"), roots=roots.tolist(), root_vertex=0)]
    # a pattern without symmetry keeps a plain plan: subsets still work
    q = xa.Plan(xmgen.named("ffl"), graph=G, symmetry=True)
    assert q.describe()["sym_mult"] == 1
    c = xa.Counter(G, [q], roots=np.arange(g.n, dtype=np.uint32))
    c.run()
    got, st = c.results()
    assert got == [oracle.count(g, xmgen.named("ffl"))] and st == [0]


def test_root_share_counts_vs_oracle(xa):
    """Plans on a root share (XM_PLAN_ROOT_SHARE: only stored ids r with
    r mod 2^s = 2^s - 1 as images of the start vertex) against the oracle on
    the same roots, in generated and in degree order, reduced and unreduced,
    with and without symmetry breaking (then only automorphisms fixing the
    start vertex), batched, with chunks that leave a share's last chunk part
    full."""
    pats = [xmgen.named(n) for n in ["ffl", "c3", "bifan", "c4", "tt4p", "c5chord"]]
    pats += [xmgen.random_pattern(5, 51), xmgen.random_pattern(6, 61)]
    g = xmgen.rmat(8, seed=3)
    memo = {}

    def oracle_count(i, roots, rv):
        key = (i, roots.tobytes(), rv)
        if key not in memo:
            memo[key] = oracle.count(g, pats[i], roots=roots, root_vertex=rv, mode="B")
        return memo[key]
    for order in (False, True):
        G = xa.Graph(g, order_by_degree=order)
        old_of_new = np.arange(g.n, dtype=np.uint32)
        if order:
            old_of_new[G.node_order()] = np.arange(g.n, dtype=np.uint32)
        for share in (2, 3, 5):
            stored = np.arange((1 << share) - 1, g.n, 1 << share, dtype=np.uint32)
            banner(f"root share {share} ({stored.size} roots), degree order {order}")
            for reduced in (True, False):
                for symmetry in (False, True):
                    plans = [xa.Plan(p, reduced=reduced, graph=G, symmetry=symmetry, root_share=share)
                             for p in pats]
                    want = [oracle_count(i, np.sort(old_of_new[stored]), pl.root_vertex)
                            for i, pl in enumerate(plans)]
                    for chunk in (0, 1, 3):
                        c = xa.Counter(G, plans, chunk=chunk)
                        c.run()
                        assert c.results() == (want, [0] * len(pats)), (order, share, reduced, symmetry, chunk)


def test_root_items_past_32_bits_are_refused(xa):
    """Root items (plan, chunk) are numbered in 32 bits: a launch whose
    ceil(n / chunk) x n_plans reaches 2^32 is refused before anything runs
    (2^22 nodes, 1,024 plans, chunk 1), one with half as many items is
    accepted."""
    from paper_2404_11105_amd._lib import XminerError
    banner("root items: 2^22 nodes x 1024 plans at chunk 1 and 2")
    g = xmgen.uniform_digraph(1 << 22, 64, 1)
    G = xa.Graph(g, dense_rows=0)
    plans = [xa.Plan(xmgen.named("ffl"), graph=G)] * 1024
    with pytest.raises(XminerError, match="root items"):
        xa.Counter(G, plans, chunk=1)
    xa.Counter(G, plans, chunk=2)


def test_degree_order_keeps_counts(xa):
    """A graph stored with its nodes renumbered by decreasing degree gives the
    oracle's counts with and without symmetry breaking (either direction),
    and refuses root subsets and listing."""
    from tests.cases import symmetric_patterns
    pats = [xmgen.named(n) for n in ["ffl", "c3", "bifan", "c4", "tt4p", "c5chord", "mixed_star"]]
    pats += symmetric_patterns()[7:13]
    for g in (xmgen.rmat(9, seed=3), xmgen.uniform_digraph(300, 2400, 5)):
        banner(f"degree order on {g.name}, {len(pats)} patterns")
        G = xa.Graph(g, order_by_degree=True)
        new = G.node_order()
        assert np.array_equal(np.sort(new), np.arange(g.n, dtype=np.uint32))
        deg = np.diff(g.out_off.astype(np.int64)) + np.diff(g.in_off.astype(np.int64))
        by_new = np.empty(g.n, dtype=np.int64)
        by_new[new] = deg
        assert np.all(np.diff(by_new) <= 0), "stored ids are not in decreasing degree order"
        want = [oracle.count(g, p, threads=8, mode="B") for p in pats]
        for reduced in (True, False):
            for symmetry in (False, "above", "below", True):
                assert run(xa, g, pats, G=G, reduced=reduced, symmetry=symmetry) == want, (reduced, symmetry)
        p = xa.Plan(xmgen.named("ffl"), graph=G)
        with pytest.raises(Exception):
            c = xa.Counter(G, [p], roots=np.arange(10, dtype=np.uint32))
            c.run()
        with pytest.raises(Exception):
            c = xa.Counter(G, [xa.Plan(xmgen.named("ffl"), reduced=False, graph=G)], list_cap=100)
            c.run()
