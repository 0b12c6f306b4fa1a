// work.cpp — algorithmic work of a plan on a graph, measured on the host.
//
// Walks the plan's partial matches level by level exactly as the plan
// defines them (the candidate sets of the enumerated levels are built; leaf
// groups only contribute the lengths of the lists they read) and sums, per
// partial match and level, the length of the base list plus the lengths of
// the lists probed for membership.  This is the algorithmic element count of
// the plan, independent of how a launch is tuned (hub splits, window sizes).
// It is a statistic for roofline accounting: it returns no embedding count.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "kernels.h"

namespace xm {

namespace {

struct Walker {
    const HostCsr& G;
    const PlanDesc& P;
    WorkOut w;
    std::atomic<uint64_t>* shared_partial = nullptr;  // budget accounting across threads
    uint64_t budget = 0;
    uint64_t reported = 0;
    bool stop = false;
    uint32_t phi[kMaxK] = {0};
    std::vector<uint32_t> cand[kMaxK];

    Walker(const HostCsr& g, const PlanDesc& p) : G(g), P(p) {}

    void list(uint32_t node, uint32_t dir, const uint32_t*& a, uint32_t& len) const {
        const uint32_t* off = dir ? G.in_off : G.out_off;
        a = (dir ? G.in_adj : G.out_adj) + off[node];
        len = off[node + 1] - off[node];
    }

    static bool has(const uint32_t* a, uint32_t len, uint32_t x) {
        return std::binary_search(a, a + len, x);
    }

    // Symmetry breaking: keep the part of a sorted list above the largest
    // (D.lt = 0) or below the smallest (D.lt = 1) image of the levels in D.gt.
    void trim(const LevelDesc& D, const uint32_t*& a, uint32_t& len) const {
        uint32_t lo = 0xFFFFFFFFu, hi = 0;
        for (uint32_t l = 0; l < kMaxK; l++)
            if ((D.gt >> l) & 1u) {
                lo = std::min(lo, phi[l]);
                hi = std::max(hi, phi[l]);
            }
        if (D.lt) {
            len = (uint32_t)(std::lower_bound(a, a + len, lo) - a);
        } else {
            const uint32_t skip = (uint32_t)(std::upper_bound(a, a + len, hi) - a);
            a += skip;
            len -= skip;
        }
    }

    // Base and probe lists of level desc D at depth lv (levels < lv bound).
    // With a symmetry bound, only the parts on its side are counted:
    // candidates are a range of the base, and a merge would read only that
    // range of each probe list.
    void lists(const LevelDesc& D, bool& from_level, const uint32_t*& base, uint32_t& blen,
               const uint32_t* probe[kMaxCons], uint32_t plen[kMaxCons], int& np) {
        lists_all(D, from_level, base, blen, probe, plen, np);
        if (!D.gt) return;
        trim(D, base, blen);
        for (int i = 0; i < np; i++) trim(D, probe[i], plen[i]);
    }

    void lists_all(const LevelDesc& D, bool& from_level, const uint32_t*& base, uint32_t& blen,
                   const uint32_t* probe[kMaxCons], uint32_t plen[kMaxCons], int& np) {
        np = 0;
        from_level = D.reuse != kNoReuse;
        if (from_level) {
            base = cand[D.reuse].data();
            blen = (uint32_t)cand[D.reuse].size();
            for (int c = 0; c < D.n_cons; c++)
                if ((D.extra >> c) & 1u) {
                    list(phi[D.cons_lvl[c]], D.cons_dir[c], probe[np], plen[np]);
                    np++;
                }
            return;
        }
        int bc = 0;
        const uint32_t* a[kMaxCons];
        uint32_t l[kMaxCons];
        for (int c = 0; c < D.n_cons; c++) {
            list(phi[D.cons_lvl[c]], D.cons_dir[c], a[c], l[c]);
            if (l[c] < l[bc]) bc = c;
        }
        base = a[bc];
        blen = l[bc];
        for (int c = 0; c < D.n_cons; c++)
            if (c != bc) {
                probe[np] = a[c];
                plen[np++] = l[c];
            }
    }

    void leaves(uint32_t nb) {
        const LevelDesc& S0 = P.sig[0];
        if (P.linear && S0.n_cons == 1 && S0.reuse == kNoReuse) {
            const uint32_t* a;
            uint32_t l;
            list(phi[S0.cons_lvl[0]], S0.cons_dir[0], a, l);
            if (S0.gt) trim(S0, a, l);
            w.elements += l;
            w.fetches += 1;
            return;
        }
        (void)nb;
        // one leaf: its signature's lists; several: the lists of every
        // signature mask the inclusion-exclusion terms measure
        const uint32_t nd = P.linear ? 1u : P.n_masks;
        for (uint32_t s = 0; s < nd; s++) {
            const LevelDesc& L = P.linear ? P.sig[0] : P.mdesc[s];
            if (!P.linear && L.n_cons == 1 && L.reuse == kNoReuse) {
                // a single list counts with its length (the kernel reads the
                // length and searches the list only for the bound nodes)
                const uint32_t* a;
                uint32_t l;
                list(phi[L.cons_lvl[0]], L.cons_dir[0], a, l);
                w.elements += l;
                w.fetches += 1;
                continue;
            }
            bool fl;
            const uint32_t* base;
            uint32_t blen;
            const uint32_t* probe[kMaxCons];
            uint32_t plen[kMaxCons];
            int np;
            lists(L, fl, base, blen, probe, plen, np);
            w.elements += blen;
            w.fetches += 1;
            for (int i = 0; i < np; i++) {
                w.elements += plen[i];
                w.fetches += 1;
            }
        }
    }

    void level(uint32_t lv) {
        if (stop) return;
        if (lv == P.e) {
            leaves(lv);
            return;
        }
        const LevelDesc& D = P.lvl[lv];
        bool fl;
        const uint32_t* base;
        uint32_t blen;
        const uint32_t* probe[kMaxCons];
        uint32_t plen[kMaxCons];
        int np;
        lists(D, fl, base, blen, probe, plen, np);
        w.elements += blen;
        w.fetches += 1;
        for (int i = 0; i < np; i++) {
            w.elements += plen[i];
            w.fetches += 1;
        }
        std::vector<uint32_t>& out = cand[lv];
        out.clear();
        for (uint32_t i = 0; i < blen; i++) {
            uint32_t x = base[i];
            bool ok = true;
            for (uint32_t j = 0; j < lv && ok; j++)
                if (((D.inj >> j) & 1u) && x == phi[j]) ok = false;
            if (ok && D.deg_check) {
                uint32_t dout = G.out_off[x + 1] - G.out_off[x], din = G.in_off[x + 1] - G.in_off[x];
                ok = dout >= D.dmin_out && din >= D.dmin_in;
            }
            for (int c = 0; c < np && ok; c++) ok = has(probe[c], plen[c], x);
            if (ok) out.push_back(x);
        }
        w.partial += out.size();
        if (budget && w.partial - reported >= 4096) {
            uint64_t tot = shared_partial->fetch_add(w.partial - reported) + (w.partial - reported);
            reported = w.partial;
            if (tot > budget) stop = true;
        }
        // deeper levels only write cand[> lv], so cand[lv] stays valid for reuse
        for (size_t i = 0; i < cand[lv].size(); i++) {
            phi[lv] = cand[lv][i];
            level(lv + 1);
        }
    }

    void root(uint32_t r) {
        uint32_t dout = G.out_off[r + 1] - G.out_off[r], din = G.in_off[r + 1] - G.in_off[r];
        if (dout < P.root_dout || din < P.root_din) return;
        w.roots += 1;
        phi[0] = r;
        level(1);
    }
};

}  // namespace

bool plan_work(const HostCsr& g, const PlanDesc& p, const uint32_t* roots, uint32_t n_roots,
               unsigned threads, uint64_t max_partial, WorkOut& out) {
    std::atomic<uint64_t> cursor{0};
    std::atomic<uint64_t> partial{0};
    std::atomic<bool> exceeded{false};
    uint64_t total = roots ? n_roots : g.n;
    threads = std::max(1u, threads);
    std::vector<WorkOut> parts(threads);
    // small root lists (a sample of hubs) spread one root at a time
    const uint64_t step = std::max<uint64_t>(1, std::min<uint64_t>(64, total / (16ull * threads)));
    std::vector<std::thread> ts;
    for (unsigned t = 0; t < threads; t++) {
        ts.emplace_back([&, t]() {
            Walker wk(g, p);
            wk.shared_partial = &partial;
            wk.budget = max_partial;
            for (;;) {
                uint64_t b = cursor.fetch_add(step);
                if (b >= total || wk.stop || exceeded.load()) break;
                uint64_t e = std::min<uint64_t>(total, b + step);
                for (uint64_t i = b; i < e && !wk.stop; i++) {
                    uint32_t r = roots ? roots[i] : (uint32_t)i;
                    if (r < g.n) wk.root(r);
                }
            }
            if (wk.stop) exceeded.store(true);
            parts[t] = wk.w;
        });
    }
    for (auto& th : ts) th.join();
    out = WorkOut();
    for (auto& w : parts) {
        out.elements += w.elements;
        out.fetches += w.fetches;
        out.partial += w.partial;
        out.roots += w.roots;
    }
    return exceeded.load();
}

}  // namespace xm
