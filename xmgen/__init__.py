"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This package holds only input generation (graphs, patterns, request
streams).  It contains none of the counting method's arithmetic, so the
oracle and the GPU path can both draw from it without sharing any code
that computes a count.
"""
from .graphs import (Digraph, DeviceDigraph, uniform_digraph, rmat, rmat_device, complete_digraph,
                     from_arcs, star_hub)
from .patterns import Pattern, NAMED, named, random_pattern, PATTERN_RECIPES

__all__ = [
    "Digraph", "DeviceDigraph", "uniform_digraph", "rmat", "rmat_device", "complete_digraph",
    "from_arcs", "star_hub",
    "Pattern", "NAMED", "named", "random_pattern", "PATTERN_RECIPES",
]
