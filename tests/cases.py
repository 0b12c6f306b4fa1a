"""Parity cases shared by the golden writer (oracle side) and the GPU tests.

Each case names a seeded graph recipe, a list of patterns and optionally a
root subset with the pattern vertex whose images it restricts.  Only input
generation lives here.
"""
from __future__ import annotations

import numpy as np

import xmgen

NAMED_ALL = ["arc", "pair2", "ffl", "c3", "bifan", "c4", "path3", "outstar3", "instar3",
             "outstar5", "tt4p", "tt4p_t3", "tt4p_out", "c5chord", "mixed_star", "p7hub"]


def _rand(ks, per, base):
    return [xmgen.random_pattern(k, base + 7 * k + s) for k in ks for s in range(per)]


CASES = {
    "uniform2000_named": dict(graph=lambda: xmgen.uniform_digraph(2000, 20000, 0),
                              patterns=lambda: [xmgen.named(n) for n in NAMED_ALL]),
    "rmat11_named": dict(graph=lambda: xmgen.rmat(11, seed=3),
                         patterns=lambda: [xmgen.named(n) for n in NAMED_ALL
                                           if n not in ("outstar5", "p7hub", "mixed_star")]),
    "rand_uniform300": dict(graph=lambda: xmgen.uniform_digraph(300, 2400, 5),
                            patterns=lambda: _rand(range(3, 8), 6, 900)),
    "rand_rmat8": dict(graph=lambda: xmgen.rmat(8, edge_factor=6, seed=5),
                       patterns=lambda: _rand(range(3, 8), 6, 900)),
    "tune_rmat11": dict(graph=lambda: xmgen.rmat(11, seed=7),
                        patterns=lambda: [xmgen.named(n) for n in
                                          ["bifan", "c4", "tt4p", "c5chord", "ffl", "mixed_star"]]),
    "batch_rmat10": dict(graph=lambda: xmgen.rmat(10, seed=11),
                         patterns=lambda: [xmgen.random_pattern(3 + (i % 4), 3000 + i)
                                           for i in range(24)]),
    "replay_rmat10": dict(graph=lambda: xmgen.rmat(10, seed=4),
                          patterns=lambda: [xmgen.named(n) for n in ["bifan", "c4", "tt4p", "c5chord"]]),
    "subset_rmat11": dict(graph=lambda: xmgen.rmat(11, seed=13),
                          patterns=lambda: [xmgen.named(n) for n in ["c4", "tt4p", "bifan", "c5chord"]],
                          roots=np.array([0, 1, 2, 5, 17, 100, 1000, 2047], dtype=np.uint32),
                          root_vertex=[0, 0, 2, 1]),
}


def symmetric_patterns():
    """Patterns with non-trivial automorphism groups: named ones, a few built
    by hand and the first random draws (k = 3..6) that have any."""
    P = xmgen.Pattern
    out = [xmgen.named(n) for n in ["c3", "c4", "bifan", "outstar3", "instar3", "mixed_star", "pair2"]]
    out += [P(3, ((0, 1), (1, 0), (1, 2), (2, 1), (0, 2), (2, 0)), "bitri"),
            P(4, tuple((a, b) for a in range(4) for b in range(4) if a != b), "k4"),
            P(5, ((0, 1), (1, 2), (2, 3), (3, 4), (4, 0)), "c5"),
            P(4, ((0, 1), (1, 0), (1, 2), (2, 1), (2, 3), (3, 2), (3, 0), (0, 3)), "bic4"),
            P(5, ((0, 2), (0, 3), (0, 4), (1, 2), (1, 3), (1, 4)), "k23"),
            P(5, ((0, 1), (1, 2), (0, 2), (0, 3), (3, 4), (0, 4)), "two_ffl")]
    for k in range(3, 7):
        got = 0
        for s in range(400):
            pat = xmgen.random_pattern(k, 9000 + 100 * k + s)
            if pat.automorphisms() > 1:
                out.append(pat)
                got += 1
                if got == 2:
                    break
    return out


def symmetric_patterns_large():
    """Larger groups and k up to 7: a directed 6-cycle (|Aut| 6), three
    2-paths from one vertex (|Aut| 6) and a star of four bidirected edges
    (|Aut| 24).  The oracle is slow on them beyond small graphs."""
    P = xmgen.Pattern
    return [P(6, ((0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0)), "c6"),
            P(7, ((0, 1), (1, 2), (0, 3), (3, 4), (0, 5), (5, 6)), "windmill3"),
            P(5, tuple(x for i in range(1, 5) for x in ((0, i), (i, 0))), "bistar4")]
