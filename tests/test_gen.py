"""Generators: determinism, simplicity, CSR invariants (CPU)."""
import numpy as np
import pytest

import xmgen


def _check_simple(g):
    assert g.out_off.dtype == np.uint32 and g.in_adj.dtype == np.uint32
    assert g.out_off[0] == 0 and g.out_off[-1] == g.m and g.in_off[-1] == g.m
    a = g.arcs()
    assert np.all(a[:, 0] != a[:, 1]), "self-loop"
    key = a[:, 0] * g.n + a[:, 1]
    assert np.all(np.diff(key) > 0), "out lists sorted and distinct"
    # in-CSR is the transpose of the out-CSR
    src_in = np.repeat(np.arange(g.n), g.in_deg())
    tkey = np.sort(g.in_adj.astype(np.int64) * g.n + src_in)
    assert np.array_equal(np.sort(key), tkey)
    ikey = src_in * g.n + g.in_adj.astype(np.int64)
    assert np.all(np.diff(ikey) > 0), "in lists sorted and distinct"


def test_uniform_exact_and_seeded():
    g1 = xmgen.uniform_digraph(2000, 20000, 0)
    g2 = xmgen.uniform_digraph(2000, 20000, 0)
    assert g1.m == 20000
    assert np.array_equal(g1.out_adj, g2.out_adj) and np.array_equal(g1.out_off, g2.out_off)
    _check_simple(g1)
    g3 = xmgen.uniform_digraph(2000, 20000, 1)
    assert not np.array_equal(g1.out_adj, g3.out_adj)


def test_rmat_small_scale():
    g = xmgen.rmat(10, seed=0)
    _check_simple(g)
    g2 = xmgen.rmat(10, seed=0)
    assert np.array_equal(g.out_adj, g2.out_adj)
    assert g.n == 1024 and 0.6 * 16 * 1024 < g.m <= 16 * 1024
    # skew: low ids are hubs for (a,b,c,d) = (.57,.19,.19,.05)
    assert g.out_deg()[:8].mean() > 10 * g.out_deg().mean()


def test_complete_and_star():
    g = xmgen.complete_digraph(5)
    _check_simple(g)
    assert g.m == 20
    s = xmgen.star_hub(10)
    assert s.m == 10 and s.out_deg()[0] == 10


def test_random_pattern_connected_and_seeded():
    for k in range(3, 8):
        for seed in range(20):
            p = xmgen.random_pattern(k, seed)
            assert p.k == k and p.is_connected()
            assert all(a != b and 0 <= a < k and 0 <= b < k for a, b in p.arcs)
            assert p == xmgen.random_pattern(k, seed)
