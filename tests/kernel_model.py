"""A host model of the count kernel's control flow (test infrastructure).

It follows count.hip's per-task logic (split items and strided root chunks,
windowed level expansion with partial windows, child segments, reuse with
fallback, leaf-group counting: single-signature passes and per-mask
intersection sizes) on numpy arrays, one simulated wave at a time, so that
termination, cursor arithmetic and buffer bounds can be checked on the CPU
for any tuning.  It asserts every buffer index it uses.  It runs the tasks in
order on one wave: the XCD-local split queues, work donation between waves
and the dense-row representation of probe lists change which wave does a
task and how a membership is tested, not what a task computes, and are not
modelled.
"""
from __future__ import annotations

SKIP = 0xFFFFFFFF
# the kernel's base choice below the first level (kFreshBaseRatio in
# kernels.h): the deepest bound vertex's list when at most this many times
# longer than the shortest
FRESH_BASE_RATIO = 2


class Model:
    def __init__(self, plan: dict, graph, chunk: int, split: int, cap: int, max_windows=10**7,
                 split_work: int = 32768):
        self.P = plan
        self.g = graph
        self.chunk, self.split, self.cap = chunk, split, cap
        self.split_work = split_work
        self.out_off = graph.out_off.astype(int)
        self.in_off = graph.in_off.astype(int)
        self.out_adj = graph.out_adj.astype(int)
        self.in_adj = graph.in_adj.astype(int)
        self.sets = ([set(self.out_adj[self.out_off[v]:self.out_off[v + 1]].tolist()) for v in range(graph.n)],
                     [set(self.in_adj[self.in_off[v]:self.in_off[v + 1]].tolist()) for v in range(graph.n)])
        self.windows = 0
        self.max_windows = max_windows
        # lists read from the data graph: (descriptor, constraint index,
        # whether the read replaced an unavailable reuse source)
        self.reads = set()
        e = plan["e"]
        self.F = [dict(node=[0] * cap, parent=[0] * cap, segb=[0] * cap, segc=[0] * cap, aux=[0] * cap)
                  for _ in range(max(e, 1))]
        self.total = 0

    def lst(self, node, d):
        off = self.in_off if d else self.out_off
        return off[node], off[node + 1] - off[node]

    def adj(self, d):
        return self.in_adj if d else self.out_adj

    def level1_len(self, r):
        L = self.P["levels"][0]
        return min(self.lst(r, d)[1] for j, d in L["cons"])

    def item_size(self, L1):
        split, split_work = self.split, self.split_work
        if self.P["e"] == 2:
            # one level below the root: larger sub-ranges (at most cap)
            split = split * 8 if split <= self.cap // 8 else max(self.cap, split)
            split_work = min(split_work * 16, 0xFFFFFFFF)
        s = split_work // L1 if L1 else split
        s = max(1, min(s, split))
        return max(s, -(-L1 // 4096))

    def deg(self, x):
        return self.out_off[x + 1] - self.out_off[x], self.in_off[x + 1] - self.in_off[x]

    # ---- phase A for one parent p of level lv (or prefix p of level lv-1 for sigs)
    def phase_a(self, D, lv, p, is_sig, bound, anc, tag=None):
        meta = {}
        fetched = False
        if D["reuse"] >= 0:
            r = D["reuse"]
            ai = anc[r - 1]
            Fr1 = self.F[r - 1]
            assert 0 <= ai < self.cap
            sc = Fr1["segc"][ai]
            if sc & 0x80000000:
                meta["kind"] = 2
                meta["off"] = Fr1["segb"][ai]
                ln = sc & 0x7FFFFFFF
                chk = []
                for c, (j, d) in enumerate(D["cons"]):
                    if (D["extra"] >> c) & 1:
                        chk.append((d,) + self.lst(bound[j], d) + (bound[j],))
                        self.reads.add((tag, c, False))
                meta["chk"] = chk
                fetched = True
        if not fetched:
            for c in range(len(D["cons"])):
                self.reads.add((tag, c, D["reuse"] >= 0))
            lists = [(d,) + self.lst(bound[j], d) + (bound[j],) for j, d in D["cons"]]
            bi = min(range(len(lists)), key=lambda i: (lists[i][2], i))
            if FRESH_BASE_RATIO and (is_sig or lv >= 2):
                # the deepest bound vertex's list when within the ratio of the shortest
                dc = min(range(len(lists)), key=lambda i: (-D["cons"][i][0], lists[i][2], i))
                if D["cons"][bi][0] < D["cons"][dc][0] and lists[dc][2] <= FRESH_BASE_RATIO * lists[bi][2]:
                    bi = dc
            meta["kind"] = lists[bi][0]
            meta["off"] = lists[bi][1]
            ln = lists[bi][2]
            meta["chk"] = [x for i, x in enumerate(lists) if i != bi]
            if not is_sig and lv == 1:
                F0 = self.F[0]
                lo, hi = F0["parent"][p], F0["aux"][p]
                hi = min(hi, ln)
                lo = min(lo, hi)
                meta["off"] += lo
                ln = hi - lo
        meta["len"] = ln
        if D.get("gt", 0):
            # symmetry breaking: the sorted base's range beyond the bounds
            bs = [bound[l] for l in range(lv) if (D["gt"] >> l) & 1]
            elems = [self.base_elem(meta, i, D["reuse"]) for i in range(ln)]
            assert all(x < y for x, y in zip(elems, elems[1:])), "unsorted base"
            if D["lt"]:
                meta["len"] = sum(1 for x in elems if x < min(bs))
            else:
                skip = sum(1 for x in elems if x <= max(bs))
                meta["off"] += skip
                meta["len"] = ln - skip
        return meta

    def base_elem(self, meta, local, reuse):
        if meta["kind"] == 2:
            assert 0 <= meta["off"] + local < self.cap
            return self.F[reuse]["node"][meta["off"] + local]
        return self.adj(meta["kind"])[meta["off"] + local]

    def check(self, D, lv, bound, meta, x):
        for l in range(lv):
            if (D["inj"] >> l) & 1 and x == bound[l]:
                return False
        do, di = self.deg(x)
        if do < D["dmin"][0] or di < D["dmin"][1]:
            return False
        for d, off, ln, node in meta["chk"]:
            if x not in self.sets[d][node]:
                return False
        return True

    def chain(self, lv_top, p):
        """bound nodes and ancestor indices of entry p of level lv_top."""
        bound, anc = {}, {}
        idx = p
        for l in range(lv_top, -1, -1):
            F = self.F[l]
            bound[l] = F["node"][idx]
            anc[l] = idx
            if l > 0:
                idx = F["parent"][idx]
        return bound, anc

    def expand(self, lv, st):
        self.windows += 1
        assert self.windows < self.max_windows, "window budget exceeded (no progress?)"
        D = self.P["levels"][lv - 1]
        nparents = st["n"][lv - 1]
        cur, pofs = st["cur"][lv], st["pofs"][lv]
        metas, lens = [], []
        for lane in range(64):
            p = cur + lane
            if p >= nparents:
                lens.append(0)
                metas.append(None)
                continue
            bound, anc = self.chain(lv - 1, p)
            m = self.phase_a(D, lv, p, False, bound, anc, tag=("lvl", lv))
            m["bound"] = bound
            ln = m["len"] - (pofs if lane == 0 else 0)
            assert ln >= 0, "negative remaining length"
            lens.append(ln)
            metas.append(m)
        incl, acc = [], 0
        for ln in lens:
            acc += ln
            incl.append(acc)
        np_ = sum(1 for lane in range(64) if cur + lane < nparents and incl[lane] <= self.cap)
        partial = False
        if np_ == 0:
            T, partial, np_ = self.cap, True, 1
            incl[0] = self.cap
        else:
            T = incl[np_ - 1]
        seg = (self.P["seg_src"] >> lv) & 1
        Fo = self.F[lv]
        nout = 0
        segcnt = [0] * 64
        for gi in range(T):
            j = next(i for i in range(np_) if incl[i] > gi)
            local = gi - (incl[j - 1] if j else 0) + (pofs if j == 0 else 0)
            m = metas[j]
            assert local < m["len"], "base index out of range"
            x = self.base_elem(m, local, D["reuse"])
            if self.check(D, lv, m["bound"], m, x):
                assert nout < self.cap, "level buffer overflow"
                Fo["node"][nout] = x
                Fo["parent"][nout] = cur + j
                segcnt[j] += 1
                nout += 1
        if seg:
            ex = 0
            for lane in range(np_):
                complete = not (lane == 0 and (pofs > 0 or partial))
                if lv == 1:
                    F0 = self.F[0]
                    complete = complete and F0["parent"][cur + lane] == 0 and F0["aux"][cur + lane] == SKIP
                Fi = self.F[lv - 1]
                Fi["segb"][cur + lane] = ex
                Fi["segc"][cur + lane] = segcnt[lane] | (0x80000000 if complete else 0)
                ex += segcnt[lane]
        if partial:
            st["pofs"][lv] = pofs + self.cap
        else:
            st["cur"][lv] = cur + np_
            st["pofs"][lv] = 0
        st["n"][lv] = nout
        return nout

    def count_leaves(self, lv, nprefix):
        P = self.P
        sigs = P["leaf_sigs"]
        nsig = len(sigs)
        for w0 in range(0, nprefix, 64):
            for p in range(w0, min(nprefix, w0 + 64)):
                bound, anc = self.chain(lv, p)
                S0 = sigs[0]
                if P["linear"] and len(S0["cons"]) == 1 and S0["reuse"] < 0:
                    self.reads.add((("sig", 0), 0, False))
                    j, d = S0["cons"][0]
                    lo, hi = self._rng(bound[j], d)
                    L = self.sets[d][bound[j]]
                    keep = lambda x: True  # noqa: E731
                    if S0.get("gt", 0):
                        bs = [bound[l] for l in range(lv + 1) if (S0["gt"] >> l) & 1]
                        if S0["lt"]:
                            keep = lambda x: x < min(bs)  # noqa: E731
                        else:
                            keep = lambda x: x > max(bs)  # noqa: E731
                    n_in = sum(1 for i in range(lo, hi) if keep(self.adj(d)[i]))
                    self.total += n_in - sum(1 for b in range(lv + 1)
                                             if (S0["inj"] >> b) & 1 and bound[b] in L and keep(bound[b]))
                    continue
                # several signatures: h[M] = |intersection of the sets in M| for
                # every mask the terms use, then the inclusion-exclusion terms
                hist = [0] * 16
                for mi, M in enumerate(P["masks"]):
                    if len(M["cons"]) == 1 and M["reuse"] < 0:
                        self.reads.add((("mask", mi), 0, False))
                        j, d = M["cons"][0]
                        L = self.sets[d][bound[j]]
                        lo, hi = self._rng(bound[j], d)
                        for mm in M["mask_set"]:
                            hist[mm] = (hi - lo) - sum(1 for b in range(lv + 1)
                                                       if (M["inj"] >> b) & 1 and bound[b] in L)
                        continue
                    m = self.phase_a(M, lv + 1, p, True, bound, anc, tag=("mask", mi))
                    cnt = 0
                    for local in range(m["len"]):
                        x = self.base_elem(m, local, M["reuse"])
                        if self.check(M, lv + 1, bound, m, x):
                            cnt += 1
                    for mm in M["mask_set"]:
                        hist[mm] = cnt
                val = 0
                for t in P["terms"]:
                    prod = t["coef"]
                    for b in t["masks"]:
                        prod *= hist[b]
                    val += prod
                self.total += val

    def _rng(self, node, d):
        off = self.in_off if d else self.out_off
        return off[node], off[node + 1]

    def explore(self, n0):
        e = self.P["e"]
        if e == 1:
            self.count_leaves(0, n0)
            return
        st = {"cur": [0] * 8, "pofs": [0] * 8, "n": [0] * 8}
        st["n"][0] = n0
        lv = 1
        while True:
            if st["cur"][lv] >= st["n"][lv - 1]:
                if lv == 1:
                    break
                lv -= 1
                continue
            nout = self.expand(lv, st)
            if lv == e - 1:
                if nout:
                    self.count_leaves(lv, nout)
            elif nout:
                lv += 1
                st["cur"][lv] = 0
                st["pofs"][lv] = 0

    def run(self):
        P, g = self.P, self.g
        rdo, rdi = P["root_dmin"]
        items = []
        share = P.get("root_share", 0)
        in_share = lambda r: (r + 1) % (1 << share) == 0  # noqa: E731
        if P["e"] >= 2:
            for r in range(g.n):
                if not in_share(r):
                    continue
                do, di = self.deg(r)
                if do < rdo or di < rdi:
                    continue
                ln = self.level1_len(r)
                sz = self.item_size(ln)
                if ln > sz:
                    for q in range((ln + sz - 1) // sz):
                        items.append((r, q * sz, min(ln, (q + 1) * sz)))
        F0 = self.F[0]
        for r, lo, hi in items:
            F0["node"][0], F0["parent"][0], F0["aux"][0] = r, lo, hi
            self.explore(1)
        # a plan on a root share chunks the share's ids (j + 1) 2^s - 1 only
        ids = range((1 << share) - 1, g.n, 1 << share)
        n_chunks = -(-len(ids) // self.chunk)
        for c0 in range(n_chunks):
            n0 = 0
            # chunk c0 takes the roots c0, c0 + n_chunks, ... (strided)
            for r in ids[c0::n_chunks][: self.chunk]:
                if not in_share(r):
                    continue
                do, di = self.deg(r)
                if do < rdo or di < rdi:
                    continue
                if P["e"] >= 2:
                    ln = self.level1_len(r)
                    if not (0 < ln <= self.item_size(ln)):
                        continue
                F0["node"][n0], F0["parent"][n0], F0["aux"][n0] = r, 0, SKIP
                n0 += 1
            if n0:
                self.explore(n0)
        return self.total * P.get("sym_mult", 1)
