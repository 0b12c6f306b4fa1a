// work.cpp — algorithmic work of a plan on a graph, measured on the host.
//
// Walks the plan's partial matches level by level exactly as the plan
// defines them (the candidate sets of the enumerated levels are built; leaf
// groups are measured, not enumerated) and sums two accounts.
//
// The merge model (the metric's "adjacency elements intersected"): per
// partial match and level, the length of the base list plus the lengths of
// the lists probed for membership, as a merge of sorted lists would read
// them.  It is independent of how a test is carried out.
//
// The issued model (what the count kernel reads and writes for the same
// partial matches): every base element scanned, every offset pair read to
// find a list, every degree pair read by a degree filter, every membership
// test as issued -- one word of a dense row for a list at least row_min
// long, else a branch-free binary search whose loads are counted -- with
// the kernel's order and short-circuit (injectivity, degree, then the probe
// slots in order, stopping at the first failure), the searches that cut a
// sorted base at a symmetry bound and the bound-node checks of leaf counts,
// the partial matches written to the level buffers and the ancestor chains
// read back.  It assumes every window holds whole candidate sets (no hub
// sub-ranges, donated prefixes or window slices), as in a launch whose
// tasks are whole roots.
//
// Both are statistics for roofline accounting: no count is returned.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <thread>
#include <vector>

#include "kernels.h"

namespace xm {

namespace {

// Loads of the kernel's branch-free search of a sorted list of len elements
// (halving until one element is left, then one compare load).
inline uint64_t search_loads(uint32_t len) {
    if (len == 0) return 0;
    uint64_t k = 1;
    for (uint32_t n = len; n > 1; n -= n >> 1) k++;
    return k;
}

// Loads of the kernel's lower-bound search (count of elements <= x).
inline uint64_t bound_loads(uint32_t len) {
    uint64_t k = 0;
    for (uint32_t n = len; n > 0; n >>= 1) k++;
    return k;
}

struct Walker {
    const HostCsr& G;
    const PlanDesc& P;
    uint32_t row_min;
    WorkOut w;
    std::atomic<uint64_t>* shared_partial = nullptr;  // budget accounting across threads
    uint64_t budget = 0;
    uint64_t reported = 0;
    bool stop = false;
    uint32_t phi[kMaxK] = {0};
    std::vector<uint32_t> cand[kMaxK];

    Walker(const HostCsr& g, const PlanDesc& p, uint32_t rm) : G(g), P(p), row_min(rm) {}

    void list(uint32_t node, uint32_t dir, const uint32_t*& a, uint32_t& len) const {
        const uint32_t* off = dir ? G.in_off : G.out_off;
        a = (dir ? G.in_adj : G.out_adj) + off[node];
        len = off[node + 1] - off[node];
    }

    static bool has(const uint32_t* a, uint32_t len, uint32_t x) {
        return std::binary_search(a, a + len, x);
    }

    // One membership test as the kernel issues it: a dense-row word, or a
    // binary search of the sorted list (an empty list answers at once).
    bool probe(const uint32_t* a, uint32_t len, uint32_t x) {
        if (len >= row_min) {
            w.row_probes += 1;
        } else if (len > 0) {
            w.searches += 1;
            w.search_words += search_loads(len);
        }
        return len > 0 && has(a, len, x);
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

    // Base and probe lists of level desc D (levels < its depth bound).  With
    // a symmetry bound the base is cut to its range on the kept side (one
    // search, issued model); the merge model also counts only the parts of
    // the probe lists on that side, which is what a merge would read.
    void lists(const LevelDesc& D, const uint32_t*& base, uint32_t& blen, const uint32_t* probe[kMaxCons],
               uint32_t plen[kMaxCons], int& np, bool fresh_ok) {
        np = 0;
        if (D.reuse != kNoReuse) {
            base = cand[D.reuse].data();
            blen = (uint32_t)cand[D.reuse].size();
            for (int c = 0; c < D.n_cons; c++)
                if ((D.extra >> c) & 1u) {
                    list(phi[D.cons_lvl[c]], D.cons_dir[c], probe[np], plen[np]);
                    np++;
                }
            w.offset_pairs += (uint64_t)np;
        } else {
            int bc = 0, dc = 0;
            const uint32_t* a[kMaxCons];
            uint32_t l[kMaxCons];
            for (int c = 0; c < D.n_cons; c++) {
                list(phi[D.cons_lvl[c]], D.cons_dir[c], a[c], l[c]);
                if (l[c] < l[bc]) bc = c;
                if (D.cons_lvl[c] > D.cons_lvl[dc] || (D.cons_lvl[c] == D.cons_lvl[dc] && l[c] < l[dc])) dc = c;
            }
            // the kernel's choice: the deepest bound vertex's list when it is
            // within kFreshBaseRatio of the shortest (not on the first level)
            if (kFreshBaseRatio && fresh_ok && D.cons_lvl[bc] < D.cons_lvl[dc] &&
                (uint64_t)l[dc] <= (uint64_t)kFreshBaseRatio * l[bc])
                bc = dc;
            base = a[bc];
            blen = l[bc];
            for (int c = 0; c < D.n_cons; c++)
                if (c != bc) {
                    probe[np] = a[c];
                    plen[np++] = l[c];
                }
            w.offset_pairs += (uint64_t)D.n_cons;
        }
        w.fetches += 1 + (uint64_t)np;  // merge model: the base (a list or a reused set) and each probed list
        if (D.gt) {
            w.search_words += bound_loads(blen);
            w.searches += 1;
            trim(D, base, blen);
        }
        w.elements += blen;
        for (int i = 0; i < np; i++) {
            const uint32_t* pa = probe[i];
            uint32_t pl = plen[i];
            if (D.gt) trim(D, pa, pl);
            w.elements += pl;
        }
        w.base += blen;
    }

    // Candidate test of x (issued model order): injectivity over `inj`,
    // degree thresholds, then the probes in order.
    bool test(const LevelDesc& D, uint32_t inj, uint32_t nb, const uint32_t* const plist[], const uint32_t plen[],
              int np, uint32_t x) {
        for (uint32_t j = 0; j < nb; j++)
            if (((inj >> j) & 1u) && x == phi[j]) return false;
        if (D.deg_check) {
            w.deg_reads += 1;
            const uint32_t dout = G.out_off[x + 1] - G.out_off[x], din = G.in_off[x + 1] - G.in_off[x];
            if (dout < D.dmin_out || din < D.dmin_in) return false;
        }
        for (int c = 0; c < np; c++)
            if (!probe(plist[c], plen[c], x)) return false;
        return true;
    }

    // |L| minus the bound nodes of `inj` found in L (one list, no scan).
    void single_list(const LevelDesc& L, uint32_t nb, bool sym) {
        const uint32_t* a;
        uint32_t l;
        list(phi[L.cons_lvl[0]], L.cons_dir[0], a, l);
        w.fetches += 1;
        w.offset_pairs += 1;
        if (sym && L.gt) {
            w.searches += 1;
            w.search_words += bound_loads(l);
            trim(L, a, l);
        }
        w.elements += l;
        for (uint32_t b = 0; b < nb; b++)
            if ((L.inj >> b) & 1u) {
                w.searches += 1;
                w.search_words += search_loads(l);
            }
    }

    // A flattened leaf pass over descriptor L: the set's size per partial
    // match (elements tested without injectivity, then the bound nodes the
    // set may not hold checked one by one).
    void leaf_pass(const LevelDesc& L, uint32_t nb) {
        const uint32_t* base;
        uint32_t blen;
        const uint32_t* probe_l[kMaxCons];
        uint32_t plen[kMaxCons];
        int np;
        lists(L, base, blen, probe_l, plen, np, true);
        for (uint32_t i = 0; i < blen; i++) test(L, 0u, nb, probe_l, plen, np, base[i]);
        for (uint32_t b = 0; b < nb; b++) {
            if (!((L.inj >> b) & 1u)) continue;
            w.searches += 1;
            w.search_words += search_loads(blen);
            if (has(base, blen, phi[b]))
                for (int c = 0; c < np; c++)
                    if (!probe(probe_l[c], plen[c], phi[b])) break;
        }
    }

    void leaves(uint32_t nb) {
        // the kernel walks each prefix's chain once: node and parent per level
        w.chain_words += 2ull * nb;
        const LevelDesc& S0 = P.sig[0];
        if (P.linear) {
            if (S0.n_cons == 1 && S0.reuse == kNoReuse) {
                single_list(S0, nb, true);
                return;
            }
            leaf_pass(S0, nb);
            return;
        }
        // several signatures: every signature mask the inclusion-exclusion
        // terms measure
        for (uint32_t s = 0; s < P.n_masks; s++) {
            const LevelDesc& L = P.mdesc[s];
            if (L.n_cons == 1 && L.reuse == kNoReuse) {
                single_list(L, nb, false);
                continue;
            }
            leaf_pass(L, nb);
        }
    }

    // Budget accounting: partial matches plus merge-model elements / 256 (a
    // leaf pass over hub lists does much work per partial match).
    void charge() {
        const uint64_t units = w.partial + w.elements / 256;
        if (budget && units - reported >= 4096) {
            uint64_t tot = shared_partial->fetch_add(units - reported) + (units - reported);
            reported = units;
            if (tot > budget) stop = true;
        }
    }

    void level(uint32_t lv) {
        if (stop) return;
        if (lv == P.e) {
            leaves(lv);
            return;
        }
        const LevelDesc& D = P.lvl[lv];
        const uint32_t* base;
        uint32_t blen;
        const uint32_t* probe_l[kMaxCons];
        uint32_t plen[kMaxCons];
        int np;
        // the parent's chain: node and parent per bound level
        w.chain_words += 2ull * lv;
        lists(D, base, blen, probe_l, plen, np, lv >= 2);
        std::vector<uint32_t>& out = cand[lv];
        out.clear();
        for (uint32_t i = 0; i < blen; i++) {
            const uint32_t x = base[i];
            if (test(D, D.inj, lv, probe_l, plen, np, x)) out.push_back(x);
        }
        w.partial += out.size();
        charge();
        // deeper levels only write cand[> lv], so cand[lv] stays valid for reuse
        for (size_t i = 0; i < cand[lv].size() && !stop; i++) {
            phi[lv] = cand[lv][i];
            level(lv + 1);
            charge();
        }
    }

    void root(uint32_t r) {
        if (!in_root_share(r, P.root_share)) return;
        uint32_t dout = G.out_off[r + 1] - G.out_off[r], din = G.in_off[r + 1] - G.in_off[r];
        w.deg_reads += 1;
        if (dout < P.root_dout || din < P.root_din) return;
        w.roots += 1;
        phi[0] = r;
        level(1);
    }
};

}  // namespace

bool plan_work(const HostCsr& g, const PlanDesc& p, const uint32_t* roots, uint32_t n_roots,
               unsigned threads, uint64_t max_partial, uint32_t row_min, WorkOut& out) {
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
            Walker wk(g, p, row_min);
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
        out.base += w.base;
        out.deg_reads += w.deg_reads;
        out.offset_pairs += w.offset_pairs;
        out.row_probes += w.row_probes;
        out.searches += w.searches;
        out.search_words += w.search_words;
        out.chain_words += w.chain_words;
    }
    return exceeded.load();
}

}  // namespace xm
