"""Theorem 2.2 (path-level inclusion) against the plans that run.

Theorem 2.2: for paths <e1, e2> and <e3, e4> (e1 = (u, v1), e2 leaving v1,
e3 = (u, v2), e4 leaving v2 in the same direction), if e1 is included in e3
then e2 is included in e4: the data arcs that match the second hop of one
path are among those of the other, so a system that stores per-arc matches
could derive one from the other.  In this engine a second hop's list is
read per partial match, and it could be shared between partial matches
only when the hop's destination w depends on its first vertex v alone:
  * w is a leaf with the single constraint (v, dir): the plan counts it from
    the list length (no element of the list is scanned), so there is nothing
    to share;
  * w has constraints on other bound vertices too: its candidate set
    differs between partial matches that agree on v;
  * w is enumerated with v as its only bound neighbour: the level reads
    v's list (and for a bidirected edge probes v's other list), so every
    element read that passes is a candidate that
    becomes a partial match of the next level (or fails injectivity or the
    degree filter); reusing the set of a partial match that agrees on v
    would copy as many elements as the list read takes, and every one of
    those partial matches must still be extended.
This test walks every plan of the scale-20 patterns and of the 256-pattern
batch, finds every pair of paths the theorem's premise relates, and checks
that each second hop falls in one of these three cases -- i.e. path-level
reuse would cut no list element the kernel reads beyond what it would
copy."""
import json
import os

import xmgen
from paper_2404_11105_amd import describe_plan, workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def path_pairs(pat):
    """(v1, w1, v2, w2, d) for paths u -> v1 -> w1 and u -> v2 -> w2 (or the
    mirror with in-arcs), v1 != v2, w1 != w2, every vertex distinct from u,
    second hops in the same direction d (0: v -> w, 1: w -> v)."""
    arcs = set(pat.arcs)
    out = []
    for u in range(pat.k):
        for first in (0, 1):
            heads = [v for v in range(pat.k) if ((u, v) in arcs if first == 0 else (v, u) in arcs)]
            for v1 in heads:
                for v2 in heads:
                    if v1 == v2:
                        continue
                    for d in (0, 1):
                        w1s = [w for w in range(pat.k) if w not in (u, v1) and ((v1, w) if d == 0 else (w, v1)) in arcs]
                        w2s = [w for w in range(pat.k) if w not in (u, v2) and ((v2, w) if d == 0 else (w, v2)) in arcs]
                        out += [(v1, w1, v2, w2, d) for w1 in w1s for w2 in w2s if w1 != w2]
    return out


def classify(plan, pat, v, w):
    """'leaf1' (w a leaf whose only constraint is v), 'multi' (w has
    constraints on bound vertices other than v), or 'alone' (w enumerated
    with v as its only constraint)."""
    order, e = plan["order"], plan["e"]
    arcs = set(pat.arcs)
    pos = order.index(w)
    bound = order[:pos] if pos < e else order[:e]
    cons = [b for b in bound if (b, w) in arcs or (w, b) in arcs]
    if pos >= e:  # leaf
        return "leaf1" if cons == [v] and sum(((v, w) in arcs, (w, v) in arcs)) == 1 else "multi"
    if any(b != v for b in cons):
        return "multi"
    return "alone" if cons == [v] else "other"


def test_path_level_reuse_would_cut_no_element():
    pats = [xmgen.named("tt4p"), xmgen.named("c5chord")] + workloads.batch_patterns()
    shares = [0, 0] + workloads.batch_shares()
    seen = {"leaf1": 0, "multi": 0, "alone": 0}
    for pat, sh in zip(pats, shares):
        plan = describe_plan(pat, True, root_share=sh)
        for v1, w1, v2, w2, d in path_pairs(pat):
            for v, w in ((v1, w1), (v2, w2)):
                if v not in plan["order"] or w not in plan["order"]:
                    continue
                # only hops whose destination is bound after v share a list read from phi(v)
                if plan["order"].index(w) < plan["order"].index(v):
                    continue
                c = classify(plan, pat, v, w)
                assert c in seen, (pat, plan["order"], v, w, c)
                if c == "alone":
                    # every constraint is on v's level (one list, or v's out- and in-list for a
                    # bidirected edge): the set depends on phi(v) alone
                    lvl = plan["levels"][plan["order"].index(w) - 1]
                    assert {j for j, _ in lvl["cons"]} == {plan["order"].index(v)}, (pat, plan["order"], w)
                seen[c] += 1
    assert seen["leaf1"] > 0 and seen["multi"] > 0
    print(seen)
