"""Small directed pattern graphs (k <= 7 vertices) and a seeded random draw.

A pattern is k vertices 0..k-1 and a list of arcs (src, dst), src != dst.
A bidirected pattern edge is two arcs.  Patterns are weakly connected.
"""
from __future__ import annotations

import dataclasses
import itertools
import numpy as np


@dataclasses.dataclass(frozen=True)
class Pattern:
    k: int
    arcs: tuple  # tuple of (src, dst)
    name: str = ""

    def __post_init__(self):
        object.__setattr__(self, "arcs", tuple(sorted({(int(a), int(b)) for a, b in self.arcs})))

    def arcs_u8(self) -> bytes:
        return bytes(x for ab in self.arcs for x in ab)

    def reversed(self) -> "Pattern":
        return Pattern(self.k, tuple((b, a) for a, b in self.arcs), self.name + "^T")

    def relabeled(self, perm) -> "Pattern":
        return Pattern(self.k, tuple((perm[a], perm[b]) for a, b in self.arcs), self.name + "^perm")

    def is_connected(self) -> bool:
        adj = {v: set() for v in range(self.k)}
        for a, b in self.arcs:
            adj[a].add(b)
            adj[b].add(a)
        seen, stack = {0}, [0]
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if y not in seen:
                    seen.add(y)
                    stack.append(y)
        return len(seen) == self.k

    def automorphisms(self) -> int:
        """Number of vertex permutations that map the arc set onto itself."""
        s = set(self.arcs)
        return sum(1 for p in itertools.permutations(range(self.k))
                   if {(p[a], p[b]) for a, b in s} == s)


def _p(k, arcs, name):
    return Pattern(k, tuple(arcs), name)


# Named patterns of the workloads.  Letters map to ids in order a=0, b=1, ...
NAMED = {
    # single arc and reciprocal pair
    "arc": _p(2, [(0, 1)], "arc"),
    "pair2": _p(2, [(0, 1), (1, 0)], "pair2"),
    # feed-forward triangle a->b, b->c, a->c
    "ffl": _p(3, [(0, 1), (1, 2), (0, 2)], "ffl"),
    # directed 3-cycle a->b->c->a
    "c3": _p(3, [(0, 1), (1, 2), (2, 0)], "c3"),
    # bi-fan a->c, b->c, a->d, b->d
    "bifan": _p(4, [(0, 2), (1, 2), (0, 3), (1, 3)], "bifan"),
    # directed 4-cycle a->b->c->d->a
    "c4": _p(4, [(0, 1), (1, 2), (2, 3), (3, 0)], "c4"),
    # transitive tournament t0..t3 (t_i -> t_j for i < j) plus vertex p=4 with
    # the single arc p -> t0 (an in-arc of the tournament's source)
    "tt4p": _p(5, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (4, 0)], "tt4p"),
    # alternative pendant readings of the same workload name
    "tt4p_t3": _p(5, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (4, 3)], "tt4p_t3"),
    "tt4p_out": _p(5, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (0, 4)], "tt4p_out"),
    # directed 5-cycle a->b->c->d->e->a with one chord a->c
    "c5chord": _p(5, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (0, 2)], "c5chord"),
    # stars
    "outstar3": _p(4, [(0, 1), (0, 2), (0, 3)], "outstar3"),
    "instar3": _p(4, [(1, 0), (2, 0), (3, 0)], "instar3"),
    "outstar5": _p(6, [(0, i) for i in range(1, 6)], "outstar5"),
    # 2-path and wedge shapes
    "path3": _p(3, [(0, 1), (1, 2)], "path3"),
    "mixed_star": _p(5, [(0, 1), (0, 2), (3, 0), (4, 0)], "mixed_star"),
    # a 7-vertex pattern with 11 arcs: hub c with three in-arcs and two out-arcs
    # (the shape the paper's running example describes in words)
    "p7hub": _p(7, [(0, 2), (1, 2), (5, 2), (2, 4), (2, 3), (0, 1), (1, 4),
                    (4, 5), (5, 6), (3, 6), (0, 3)], "p7hub"),
}


def named(name: str) -> Pattern:
    return NAMED[name]


PATTERN_RECIPES = {
    "random": "k drawn by the caller; undirected G(k, 1/2) redrawn until connected; "
              "each edge oriented by a fair coin; each edge bidirected with p = 0.1; "
              "one numpy PCG64 stream per seed",
}


def random_pattern(k: int, seed: int, p_edge: float = 0.5, p_bidir: float = 0.1) -> Pattern:
    """Random weakly connected directed pattern on k vertices (seeded)."""
    rng = np.random.default_rng(seed)
    pairs = list(itertools.combinations(range(k), 2))
    while True:
        take = rng.random(len(pairs)) < p_edge
        orient = rng.random(len(pairs)) < 0.5
        bid = rng.random(len(pairs)) < p_bidir
        arcs = []
        for (a, b), t, o, bd in zip(pairs, take, orient, bid):
            if not t:
                continue
            if bd:
                arcs += [(a, b), (b, a)]
            elif o:
                arcs.append((a, b))
            else:
                arcs.append((b, a))
        pat = Pattern(k, tuple(arcs), f"rand(k={k},seed={seed})")
        if arcs and pat.is_connected():
            return pat
