"""Pins for the oracle: brute force, closed forms, invariants (CPU only).

The paper prints no embedding counts (its worked example's figure is not in
the text), so the oracle is pinned to mathematics: the definition evaluated
by brute force on tiny graphs, adjacency-matrix closed forms, the complete
digraph's n!/(n-k)!, and invariants that any correct count satisfies.
"""
import itertools

import numpy as np
import pytest

import oracle
import xmgen
from tests import pins


def tiny_graphs():
    out = []
    for seed in range(12):
        rng = np.random.default_rng(100 + seed)
        n = int(rng.integers(4, 9))
        p = float(rng.uniform(0.2, 0.6))
        A = rng.random((n, n)) < p
        np.fill_diagonal(A, False)
        u, v = np.nonzero(A)
        out.append(xmgen.from_arcs(n, u, v, name=f"tiny{seed}"))
    return out


SMALL_PATTERNS = [xmgen.named(x) for x in
                  ["arc", "pair2", "ffl", "c3", "bifan", "c4", "path3", "outstar3",
                   "instar3", "tt4p", "c5chord", "mixed_star"]]


@pytest.mark.parametrize("pat", SMALL_PATTERNS, ids=lambda p: p.name)
def test_oracle_equals_brute_force_named(pat):
    for g in tiny_graphs():
        bf = pins.brute_force(g, pat)
        assert oracle.count(g, pat) == bf, (g.name, pat.name)
        assert oracle.count(g, pat, mode="B") == bf


def test_oracle_equals_brute_force_random_patterns():
    graphs = tiny_graphs()
    for k in range(3, 8):
        for seed in range(6):
            pat = xmgen.random_pattern(k, 1000 + 10 * k + seed)
            for g in graphs[: 6 if k < 7 else 3]:
                if g.n < k:
                    continue
                assert oracle.count(g, pat) == pins.brute_force(g, pat), (k, seed, g.name)


def test_oracle_p7_example_shape_brute_force():
    # dense tiny graph so that a 7-vertex, 11-arc pattern has embeddings
    rng = np.random.default_rng(7)
    A = rng.random((8, 8)) < 0.75
    np.fill_diagonal(A, False)
    u, v = np.nonzero(A)
    g = xmgen.from_arcs(8, u, v)
    pat = xmgen.named("p7hub")
    bf = pins.brute_force(g, pat)
    assert bf > 0
    assert oracle.count(g, pat) == bf


@pytest.mark.parametrize("n", [3, 5, 7, 9])
def test_complete_digraph_closed_form(n):
    g = xmgen.complete_digraph(n)
    pats = SMALL_PATTERNS + [xmgen.random_pattern(k, 5 + k) for k in range(3, 8)]
    for pat in pats:
        assert oracle.count(g, pat) == pins.complete_count(n, pat.k), (n, pat.name)


def test_matrix_closed_forms_uniform_2000():
    g = xmgen.uniform_digraph(2000, 20000, 0)
    A = pins.adjacency(g)
    assert oracle.count(g, xmgen.named("c3")) == pins.closed_c3(A)
    assert oracle.count(g, xmgen.named("ffl")) == pins.closed_ffl(A)
    assert oracle.count(g, xmgen.named("c4")) == pins.closed_c4(A)
    assert oracle.count(g, xmgen.named("bifan")) == pins.closed_bifan(A)


def test_matrix_closed_forms_dense_reciprocal():
    # many reciprocal arcs exercise the degenerate-walk corrections in the C4 form
    rng = np.random.default_rng(3)
    n = 60
    A = rng.random((n, n)) < 0.3
    np.fill_diagonal(A, False)
    u, v = np.nonzero(A)
    g = xmgen.from_arcs(n, u, v)
    M = pins.adjacency(g)
    assert oracle.count(g, xmgen.named("c3")) == pins.closed_c3(M)
    assert oracle.count(g, xmgen.named("ffl")) == pins.closed_ffl(M)
    assert oracle.count(g, xmgen.named("c4")) == pins.closed_c4(M)
    assert oracle.count(g, xmgen.named("bifan")) == pins.closed_bifan(M)
    r = (M * M.T).sum()
    assert oracle.count(g, xmgen.named("pair2")) == r


def test_stars_closed_form():
    g = xmgen.rmat(10, seed=1)
    assert oracle.count(g, xmgen.named("arc")) == g.m
    assert oracle.count(g, xmgen.named("outstar3")) == pins.closed_outstar(g, 3)
    assert oracle.count(g, xmgen.named("instar3"), mode="B") == pins.closed_instar(g, 3)
    s = xmgen.star_hub(40)
    assert oracle.count(s, xmgen.named("outstar5"), mode="B") == pins.falling(40, 5)


def test_relabel_reverse_and_automorphism_invariants():
    g = xmgen.uniform_digraph(400, 4000, 2)
    perm = np.random.default_rng(5).permutation(g.n)
    gp = g.relabeled(perm)
    gr = g.reversed()
    for name in ["ffl", "c3", "bifan", "c4", "tt4p", "c5chord", "mixed_star"]:
        pat = xmgen.named(name)
        c = oracle.count(g, pat)
        assert oracle.count(gp, pat) == c
        assert oracle.count(gr, pat.reversed()) == c
        ppat = pat.relabeled(list(np.random.default_rng(1).permutation(pat.k)))
        assert oracle.count(g, ppat) == c
        assert c % pat.automorphisms() == 0


def test_root_decomposition_and_subsets():
    g = xmgen.rmat(9, seed=3)
    pat = xmgen.named("c4")
    total, per, first = oracle.count_per_root(g, pat)
    assert sum(per) == total
    roots = np.array([0, 3, 7, 100, 511], dtype=np.uint32)
    sub = oracle.count(g, pat, roots=roots, root_vertex=first)
    assert sub == sum(per[r] for r in roots)
    # a different root vertex partitions the same total differently
    t2, per2, _ = oracle.count_per_root(g, pat, root_vertex=2)
    assert t2 == total and sum(per2) == total


def test_threads_do_not_change_counts():
    g = xmgen.rmat(10, seed=4)
    for name in ["bifan", "c4", "tt4p"]:
        pat = xmgen.named(name)
        assert oracle.count(g, pat, threads=4) == oracle.count(g, pat)


def test_oracle_rejects_bad_patterns():
    g = xmgen.complete_digraph(4)
    with pytest.raises(ValueError):
        oracle.count(g, xmgen.Pattern(3, ((0, 1),)))  # vertex 2 isolated
    with pytest.raises(ValueError):
        oracle.count(g, xmgen.Pattern(2, ((0, 0),)))  # self-loop


@pytest.mark.parametrize("name", ["arc", "ffl", "c3", "bifan", "c4", "tt4p", "outstar3"])
def test_oracle_listing_equals_brute_force_maps(name):
    """Listing mode writes exactly the set of embeddings brute force finds
    (pattern-vertex order), and caps without changing the total."""
    pat = xmgen.named(name)
    for seed in range(3):
        g = xmgen.uniform_digraph(9, 30, 40 + seed)
        want = pins.brute_force_maps(g, pat)
        total, rows = oracle.list_embeddings(g, pat, cap=10 ** 6)
        assert total == len(want)
        got = rows.astype(np.int64)
        got = got[np.lexsort(got.T[::-1])] if got.size else got
        assert np.array_equal(got, want)
        # a small capacity keeps the exact total and writes a subset
        total2, part = oracle.list_embeddings(g, pat, cap=3)
        assert total2 == total and len(part) == min(3, total)
        assert all(any((r == w).all() for w in want) for r in part.astype(np.int64))


def test_prepared_graph_gives_the_same_counts():
    """Counting on a graph whose in-lists were built once (graph
    pre-processing kept out of timings) gives the plain call's counts."""
    g = xmgen.rmat(7, seed=3)
    pr = oracle.Prepared(g)
    roots = np.arange(1, g.n, 7, dtype=np.uint32)
    for name in ["ffl", "bifan", "tt4p", "c5chord", "mixed_star"]:
        p = xmgen.named(name)
        for mode in ("A", "B"):
            assert pr.count(p, mode=mode) == oracle.count(g, p, mode=mode)
            assert pr.count(p, roots=roots, mode=mode, root_vertex=1, threads=3) == \
                oracle.count(g, p, roots=roots, mode=mode, root_vertex=1)
    pr.close()
