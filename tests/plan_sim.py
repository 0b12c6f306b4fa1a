"""Test-only executor of a plan description (the JSON of xm_plan_describe).

It runs the plan's semantics in plain Python on tiny graphs so the planner's
choices (reuse sources, degree filters, injectivity masks, leaf-group
product terms) can be checked against the oracle without a GPU.  It mirrors
what the count kernel must compute, not how.
"""
from __future__ import annotations


def simulate(plan: dict, graph) -> int:
    n = graph.n
    outl = [set(graph.out_adj[graph.out_off[v]:graph.out_off[v + 1]].tolist()) for v in range(n)]
    inl = [set(graph.in_adj[graph.in_off[v]:graph.in_off[v + 1]].tolist()) for v in range(n)]
    lists = (outl, inl)
    dout = [len(s) for s in outl]
    din = [len(s) for s in inl]
    e = plan["e"]
    levels = [None] + plan["levels"]
    sigs = plan["leaf_sigs"]
    terms = plan["terms"]
    rdo, rdi = plan["root_dmin"]

    def cand(L, phi, mem):
        cons = L["cons"]
        if L["reuse"] >= 0:
            base = mem[L["reuse"]]
            chk = [c for i, c in enumerate(cons) if (L["extra"] >> i) & 1]
        else:
            base = None
            chk = cons
        out = []
        if base is None:
            sets = [lists[d][phi[j]] for j, d in cons]
            base = sorted(set.intersection(*sets))
            chk = []
        for x in base:
            ok = all(x != phi[j] for j in range(len(phi)) if (L["inj"] >> j) & 1)
            ok = ok and dout[x] >= L["dmin"][0] and din[x] >= L["dmin"][1]
            ok = ok and all(x in lists[d][phi[j]] for j, d in chk)
            if ok:
                out.append(x)
        return out

    def leaves(phi, mem):
        nsig = len(sigs)
        S = [set(cand(s, phi, mem)) for s in sigs]
        total = 0
        full = (1 << nsig) - 1
        I = {}
        for m in range(1, full + 1):
            inter = None
            for s in range(nsig):
                if (m >> s) & 1:
                    inter = S[s] if inter is None else inter & S[s]
            I[m] = len(inter)
        for t in terms:
            prod = t["coef"]
            for b in t["masks"]:
                prod *= I[b]
            total += prod
        return total

    def rec(lv, phi, mem):
        if lv == e:
            return leaves(phi, mem)
        c = cand(levels[lv], phi, mem)
        mem[lv] = c
        tot = 0
        for x in c:
            tot += rec(lv + 1, phi + [x], mem)
        return tot

    total = 0
    for r in range(n):
        if dout[r] < rdo or din[r] < rdi:
            continue
        total += rec(1, [r], {})
    return total
