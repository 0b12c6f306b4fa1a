"""CPU: host-side helpers of the Python binding (no device work)."""
import types

import numpy as np

import oracle
import xmgen
from paper_2404_11105_amd import api


def test_renumbered_host_csr_is_the_relabelled_graph():
    """The host copy kept for planning a degree-ordered graph: node v becomes
    new[v], lists sorted; same counts as the original (relabel invariance)."""
    g = xmgen.rmat(8, seed=5)
    n = g.n
    deg = np.diff(g.out_off.astype(np.int64)) + np.diff(g.in_off.astype(np.int64))
    order = np.argsort(-deg, kind="stable")
    new = np.empty(n, dtype=np.int64)
    new[order] = np.arange(n)
    h = api._renumbered(g, new)
    src = np.repeat(np.arange(n), np.diff(g.out_off.astype(np.int64)))
    ref = xmgen.from_arcs(n, new[src], new[g.out_adj.astype(np.int64)])
    for a in ("out_off", "out_adj", "in_off", "in_adj"):
        assert np.array_equal(np.asarray(getattr(h, a), dtype=np.int64), np.asarray(getattr(ref, a), dtype=np.int64)), a
    hdeg = np.diff(h.out_off.astype(np.int64)) + np.diff(h.in_off.astype(np.int64))
    assert np.all(np.diff(hdeg) <= 0)
    for name in ("ffl", "c4"):
        p = xmgen.named(name)
        assert oracle.count(h, p) == oracle.count(g, p)


def test_symmetry_direction_choice():
    """The sampled-walk estimate picks a side, and the plan on that side keeps
    the pattern's orbit multiplier; without a host copy of the graph the
    default side is kept.  (That both sides count the same is checked against
    the oracle by the kernel model on the CPU and by the GPU parity tests.)"""
    g = xmgen.rmat(9, seed=2)
    G = types.SimpleNamespace(host=g)
    for name in ("c3", "bifan", "c4", "ffl"):
        d = api._choose_direction(xmgen.named(name), True, G, None)
        assert d in ("above", "below")
        m = api.Plan(xmgen.named(name), symmetry=d).describe()["sym_mult"]
        assert m == {"c3": 3, "bifan": 4, "c4": 4, "ffl": 1}[name]
    # no host copy: the default side
    assert api._choose_direction(xmgen.named("c4"), True, types.SimpleNamespace(host=None), None) == "above"
