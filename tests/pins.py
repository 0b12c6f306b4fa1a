"""Independent checks that pin the oracle to mathematics (test helpers).

* brute force: every injective map of the pattern into a tiny graph;
* closed forms from adjacency-matrix algebra for cycles, feed-forward loops,
  bi-fans and stars; the complete digraph's n!/(n-k)!.
None of this shares code with the oracle or the HIP library.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def adjacency(graph) -> np.ndarray:
    A = np.zeros((graph.n, graph.n), dtype=np.int64)
    a = graph.arcs()
    A[a[:, 0], a[:, 1]] = 1
    return A


def brute_force(graph, pattern) -> int:
    """Count injective maps phi with every pattern arc mapped onto a data arc."""
    A = adjacency(graph).astype(bool)
    n, k = graph.n, pattern.k
    if k > n:
        return 0
    perms = np.array(list(itertools.permutations(range(n), k)), dtype=np.int64).reshape(-1, k)
    ok = np.ones(perms.shape[0], dtype=bool)
    for s, d in pattern.arcs:
        ok &= A[perms[:, s], perms[:, d]]
    return int(ok.sum())


def brute_force_maps(graph, pattern) -> np.ndarray:
    """Every injective map with every pattern arc on a data arc, one row of
    phi(0..k-1) per map, rows sorted."""
    A = adjacency(graph).astype(bool)
    n, k = graph.n, pattern.k
    if k > n:
        return np.zeros((0, k), dtype=np.int64)
    perms = np.array(list(itertools.permutations(range(n), k)), dtype=np.int64).reshape(-1, k)
    ok = np.ones(perms.shape[0], dtype=bool)
    for s, d in pattern.arcs:
        ok &= A[perms[:, s], perms[:, d]]
    rows = perms[ok]
    return rows[np.lexsort(rows.T[::-1])] if rows.size else rows


def falling(x: int, s: int) -> int:
    r = 1
    for i in range(s):
        r *= max(0, x - i)
    return r


def complete_count(n: int, k: int) -> int:
    return math.factorial(n) // math.factorial(n - k) if k <= n else 0


def _mm(X, Y):
    """Integer matrix product through float64 BLAS.

    Exact while every partial sum stays below 2**53 (true for the 0/1
    adjacency matrices of graphs with at most a few thousand nodes used
    here); the assertion guards that bound."""
    Z = np.asarray(X, dtype=np.float64) @ np.asarray(Y, dtype=np.float64)
    assert np.abs(Z).max(initial=0) < 2 ** 52
    return np.rint(Z).astype(np.int64)


def closed_c3(A) -> int:
    return int(np.trace(_mm(_mm(A, A), A)))


def closed_ffl(A) -> int:
    return int((_mm(A, A) * A).sum())


def closed_c4(A) -> int:
    r = (A * A.T).sum(axis=1)
    A2 = _mm(A, A)
    return int((A2 * A2.T).sum() - 2 * (r * r).sum() + r.sum())


def closed_bifan(A) -> int:
    M = _mm(A.T, A)
    np.fill_diagonal(M, 0)
    return int((M * (M - 1)).sum())


def closed_outstar(graph, s: int) -> int:
    return sum(falling(int(d), s) for d in graph.out_deg())


def closed_instar(graph, s: int) -> int:
    return sum(falling(int(d), s) for d in graph.in_deg())
