// planner.cpp — host-side pattern reduction and plan generation.
//
// Section 4.1 (finding constraint inclusion): edges that share a source, or
// share a destination, are related by inclusion (Theorem 2.1); for each
// vertex the in-edge from its smallest-degree in-neighbour includes the other
// in-edges, and likewise for out-edges.  Section 4.2 (reducing the pattern):
// the edges kept form a constraint cover (Definition "Constraint Cover"); its
// weighted minimum is the objective argmin sum ||A_e||; Algorithm 1 is the
// paper's greedy for it.  Section 5.1 (plan generation): start at the
// reduction's start vertex, materialise it, then extend to the vertex
// adjacent to the visited ones that is most constrained.
//
// The plan emitted here (plan_ir.h) is what the count kernel executes:
//   reduced   - siblings with included constraint sets reuse the candidate
//               set already materialised for the including level (section
//               5.2), and the trailing independent vertices are counted by
//               product (section 5.3) with an exact inclusion-exclusion
//               correction for injectivity;
//   unreduced - every level materialises all of its constraints from the data
//               graph; only the last vertex is counted instead of enumerated.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "planner.h"

namespace xm {

namespace {

inline int popc(uint32_t x) { return __builtin_popcount(x); }

struct Pat {
    int k = 0;
    uint32_t out[kMaxK] = {0};  // bit w: arc v -> w
    uint32_t in[kMaxK] = {0};   // bit u: arc u -> v
    std::vector<std::pair<int, int>> arcs;  // distinct, sorted
    int dout(int v) const { return popc(out[v]); }
    int din(int v) const { return popc(in[v]); }
    int deg(int v) const { return dout(v) + din(v); }
    uint32_t nbr(int v) const { return out[v] | in[v]; }
};

bool connected(const Pat& p, uint32_t vmask) {
    if (!vmask) return true;
    int s = __builtin_ctz(vmask);
    uint32_t seen = 1u << s, frontier = seen;
    while (frontier) {
        uint32_t nxt = 0;
        for (int v = 0; v < p.k; v++)
            if (frontier & (1u << v)) nxt |= p.nbr(v) & vmask;
        nxt &= ~seen;
        seen |= nxt;
        frontier = nxt;
    }
    return seen == vmask;
}

// ---------------------------------------------------------------------------
// Inclusion analysis and constraint covers (reported in the plan JSON).
// ---------------------------------------------------------------------------
struct CoverReport {
    std::vector<int> groups_in_rep, groups_out_rep;  // representative arc index per vertex, -1 if none
    std::vector<int> min_cover;                       // arc indices
    double min_cover_weight = 0;
    std::vector<int> greedy_cover;                    // Algorithm 1's split queue
    int greedy_start = -1;
};

// Arc e = (u, w) includes every arc leaving u and every arc entering w
// (Theorem 2.1 applied to shared sources and shared destinations).
uint64_t inclusion_set(const Pat& p, int e) {
    uint64_t s = 0;
    int u = p.arcs[e].first, w = p.arcs[e].second;
    for (size_t f = 0; f < p.arcs.size(); f++)
        if (p.arcs[f].first == u || p.arcs[f].second == w) s |= 1ull << f;
    return s;
}

void min_cover_bb(const std::vector<uint64_t>& inc, const std::vector<double>& w, uint64_t all,
                  uint64_t covered, double cost, std::vector<int>& cur, double& best,
                  std::vector<int>& best_set) {
    if (cost >= best - 1e-12) return;
    if (covered != all) {
        // every further arc covers at most max_inc uncovered arcs and costs >= min_w
        int left = __builtin_popcountll(all & ~covered), max_inc = 1;
        double min_w = 1e300;
        for (size_t e = 0; e < inc.size(); e++) {
            max_inc = std::max(max_inc, __builtin_popcountll(inc[e] & ~covered));
            min_w = std::min(min_w, w[e]);
        }
        if (cost + ((left + max_inc - 1) / max_inc) * min_w >= best - 1e-12) return;
    }
    if (covered == all) {
        best = cost;
        best_set = cur;
        return;
    }
    int first = __builtin_ctzll(all & ~covered);
    for (size_t e = 0; e < inc.size(); e++) {
        if (!(inc[e] & (1ull << first))) continue;
        cur.push_back((int)e);
        min_cover_bb(inc, w, all, covered | inc[e], cost + w[e], cur, best, best_set);
        cur.pop_back();
    }
}

CoverReport analyse_cover(const Pat& p, const GraphStats* gs, int start) {
    CoverReport r;
    int na = (int)p.arcs.size();
    r.groups_in_rep.assign(p.k, -1);
    r.groups_out_rep.assign(p.k, -1);
    // Section 4.1: the smallest-degree in-neighbour's edge represents the
    // in-group (ties: lowest vertex id); same for out-neighbours.
    for (int v = 0; v < p.k; v++) {
        int best_in = -1, best_out = -1;
        for (int e = 0; e < na; e++) {
            int a = p.arcs[e].first, b = p.arcs[e].second;
            if (b == v && (best_in < 0 || p.deg(a) < p.deg(p.arcs[best_in].first))) best_in = e;
            if (a == v && (best_out < 0 || p.deg(b) < p.deg(p.arcs[best_out].second))) best_out = e;
        }
        r.groups_in_rep[v] = best_in;
        r.groups_out_rep[v] = best_out;
    }
    // Weights ||A_e||: expected arcs of the data graph that satisfy the degree
    // constraints of both endpoints (unit weights without a graph).
    std::vector<double> w(na, 1.0);
    if (gs && gs->m > 0) {
        for (int e = 0; e < na; e++) {
            int a = p.arcs[e].first, b = p.arcs[e].second;
            int ta = std::min(p.dout(a), 7), tb = std::min(p.din(b), 7);
            w[e] = std::max(1e-9, (double)gs->m * gs->frac_out_ge[ta] * gs->frac_in_ge[tb]);
        }
    }
    std::vector<uint64_t> inc(na);
    for (int e = 0; e < na; e++) inc[e] = inclusion_set(p, e);
    uint64_t all = (na == 64) ? ~0ull : ((1ull << na) - 1);
    double best = 1e300;
    std::vector<int> cur;
    min_cover_bb(inc, w, all, 0, 0.0, cur, best, r.min_cover);
    std::sort(r.min_cover.begin(), r.min_cover.end());
    r.min_cover_weight = best;

    // Algorithm 1 (greedy), readings: the outer loop takes the lowest-index
    // unvisited arc and restarts from its larger-degree endpoint;
    // findMaxECoverage picks the unvisited arc at v that covers the most
    // unvisited arcs (ties: smaller degree of its other endpoint, then lowest
    // index); Neighbor_MaxDegree is the max-degree vertex that still has an
    // unvisited arc and is adjacent to a vertex already reached.
    uint64_t visited = 0;
    uint32_t reached = 1u << start;
    r.greedy_start = start;
    auto search_split = [&](int u) {
        int v = u;
        while (v >= 0) {
            reached |= 1u << v;
            for (;;) {
                int mec = -1, mec_cov = -1;
                for (int e = 0; e < na; e++) {
                    if (visited & (1ull << e)) continue;
                    int a = p.arcs[e].first, b = p.arcs[e].second;
                    if (a != v && b != v) continue;
                    int cov = __builtin_popcountll(inc[e] & ~visited);
                    int other = (a == v) ? b : a;
                    int mo = mec >= 0 ? ((p.arcs[mec].first == v) ? p.arcs[mec].second : p.arcs[mec].first) : 0;
                    if (cov > mec_cov || (cov == mec_cov && p.deg(other) < p.deg(mo))) {
                        mec = e;
                        mec_cov = cov;
                    }
                }
                if (mec < 0) break;
                r.greedy_cover.push_back(mec);
                visited |= inc[mec];  // updateVInclusion: included arcs are removed
                int a = p.arcs[mec].first, b = p.arcs[mec].second;
                reached |= (1u << a) | (1u << b);
            }
            int nv = -1;
            for (int x = 0; x < p.k; x++) {
                bool has = false;
                for (int e = 0; e < na; e++)
                    if (!(visited & (1ull << e)) && (p.arcs[e].first == x || p.arcs[e].second == x)) has = true;
                if (!has) continue;
                bool adj = (reached & (1u << x)) || (p.nbr(x) & reached);
                if (!adj) continue;
                if (nv < 0 || p.deg(x) > p.deg(nv)) nv = x;
            }
            v = nv;
        }
    };
    search_split(start);
    while (visited != all) {
        int e = __builtin_ctzll(all & ~visited);
        int a = p.arcs[e].first, b = p.arcs[e].second;
        search_split(p.deg(a) <= p.deg(b) ? b : a);
    }
    std::sort(r.greedy_cover.begin(), r.greedy_cover.end());
    return r;
}

// ---------------------------------------------------------------------------
// Plan construction
// ---------------------------------------------------------------------------
struct LeafSig {
    uint32_t in_mask, out_mask;  // pattern vertices u with u -> leaf / leaf -> u
    bool operator<(const LeafSig& o) const {
        int a = popc(in_mask) + popc(out_mask), b = popc(o.in_mask) + popc(o.out_mask);
        if (a != b) return a < b;
        if (in_mask != o.in_mask) return in_mask < o.in_mask;
        return out_mask < o.out_mask;
    }
    bool operator==(const LeafSig& o) const { return in_mask == o.in_mask && out_mask == o.out_mask; }
    bool subset_of(const LeafSig& o) const {
        return (in_mask & ~o.in_mask) == 0 && (out_mask & ~o.out_mask) == 0;
    }
};

// Set partitions of `t` leaves -> merged Moebius terms.
// injective tuples = sum over partitions pi of prod_{B in pi} (-1)^{|B|-1} (|B|-1)!
//                    * |intersection of the sets of the leaves in B|
bool leaf_terms(const std::vector<int>& leaf_sig, std::vector<Term>& out) {
    int t = (int)leaf_sig.size();
    std::map<std::vector<uint8_t>, long long> acc;
    std::vector<int> rgs(t, 0);
    // restricted growth strings enumerate set partitions
    for (;;) {
        int nb = 0;
        for (int i = 0; i < t; i++) nb = std::max(nb, rgs[i] + 1);
        std::vector<uint8_t> masks(nb, 0);
        std::vector<int> sz(nb, 0);
        for (int i = 0; i < t; i++) {
            masks[rgs[i]] |= (uint8_t)(1u << leaf_sig[i]);
            sz[rgs[i]]++;
        }
        long long coef = 1;
        for (int b = 0; b < nb; b++) {
            long long f = 1;
            for (int x = 2; x < sz[b]; x++) f *= x;
            coef *= ((sz[b] - 1) % 2 ? -1 : 1) * f;
        }
        std::sort(masks.begin(), masks.end());
        acc[masks] += coef;
        // next restricted growth string
        int i = t - 1;
        while (i > 0) {
            int mx = 0;
            for (int j = 0; j < i; j++) mx = std::max(mx, rgs[j]);
            if (rgs[i] <= mx) {
                rgs[i]++;
                for (int j = i + 1; j < t; j++) rgs[j] = 0;
                break;
            }
            i--;
        }
        if (i == 0) break;
    }
    out.clear();
    for (auto& kv : acc) {
        if (kv.second == 0) continue;
        Term tm;
        std::memset(&tm, 0, sizeof(tm));
        tm.coef = (int32_t)kv.second;
        tm.nb = (uint8_t)kv.first.size();
        for (size_t b = 0; b < kv.first.size(); b++) tm.mask[b] = kv.first[b];
        out.push_back(tm);
    }
    return (int)out.size() <= kMaxTerms;
}

struct Cand {
    std::vector<int> order;   // enumerated vertices (level order)
    std::vector<int> leaves;  // leaf vertices
    double cost = 0;
};

// Greedy order of the enumerated vertices (section 5.1): start vertex, then
// repeatedly the unvisited vertex adjacent to the visited ones with the most
// arcs to them (ties: larger degree, then lowest id).
std::vector<int> enum_order(const Pat& p, int start, uint32_t emask) {
    std::vector<int> ord{start};
    uint32_t bound = 1u << start;
    while ((int)ord.size() < popc(emask)) {
        int best = -1, bc = -1;
        for (int v = 0; v < p.k; v++) {
            if (!(emask & (1u << v)) || (bound & (1u << v))) continue;
            int c = popc(p.out[v] & bound) + popc(p.in[v] & bound);
            if (c == 0) continue;
            if (c > bc || (c == bc && p.deg(v) > p.deg(best))) {
                best = v;
                bc = c;
            }
        }
        if (best < 0) break;
        ord.push_back(best);
        bound |= 1u << best;
    }
    return ord;
}

// Rough work model on a random graph with n nodes and average degree d:
// a level with c constraints keeps d * (d/n)^(c-1) candidates per partial
// match and costs about d element reads per partial match.
double model_cost(const Pat& p, const std::vector<int>& ord, int n_scan, const GraphStats* gs) {
    double n = (gs && gs->n) ? (double)gs->n : 1e6;
    double d = (gs && gs->n) ? std::max(1.0, (double)gs->m / (double)gs->n) : 16.0;
    double P = n, cost = n;
    uint32_t bound = 1u << ord[0];
    for (size_t i = 1; i < ord.size(); i++) {
        int v = ord[i];
        int c = popc(p.out[v] & bound) + popc(p.in[v] & bound);
        cost += P * d;
        P *= d * std::pow(d / n, c - 1);
        bound |= 1u << v;
    }
    cost += P * d * n_scan;
    return cost;
}

void fill_level(const Pat& p, const std::vector<int>& lvl_of, int v, int nlv_limit,
                uint32_t later_mask, LevelDesc& L) {
    std::memset(&L, 0, sizeof(L));
    L.reuse = kNoReuse;
    uint32_t cons_lv = 0;
    for (int j = 0; j < nlv_limit; j++) {
        int u = -1;
        for (int x = 0; x < p.k; x++)
            if (lvl_of[x] == j) u = x;
        if (u < 0) continue;
        if (p.out[u] & (1u << v)) {  // u -> v: v in out(phi(u))
            L.cons_lvl[L.n_cons] = (uint8_t)j;
            L.cons_dir[L.n_cons++] = 0;
            cons_lv |= 1u << j;
        }
        if (p.out[v] & (1u << u)) {  // v -> u: v in in(phi(u))
            L.cons_lvl[L.n_cons] = (uint8_t)j;
            L.cons_dir[L.n_cons++] = 1;
            cons_lv |= 1u << j;
        }
    }
    uint32_t all_lv = (nlv_limit >= 32) ? ~0u : ((1u << nlv_limit) - 1);
    L.inj = (uint8_t)(all_lv & ~cons_lv);
    // Degree thresholds only prune when some arc of v goes to a later vertex.
    bool out_later = (p.out[v] & later_mask) != 0;
    bool in_later = (p.in[v] & later_mask) != 0;
    L.dmin_out = out_later ? (uint32_t)p.dout(v) : 0;
    L.dmin_in = in_later ? (uint32_t)p.din(v) : 0;
    L.deg_check = (L.dmin_out || L.dmin_in) ? 1 : 0;
}

// Candidate test of a leaf with in-neighbours `in_mask` and out-neighbours
// `out_mask` (pattern vertices), all of them bound at levels < nlv_limit.
void fill_level_sig(const Pat& p, const std::vector<int>& lvl_of, uint32_t in_mask, uint32_t out_mask,
                    int nlv_limit, LevelDesc& L) {
    std::memset(&L, 0, sizeof(L));
    L.reuse = kNoReuse;
    uint32_t cons_lv = 0;
    for (int j = 0; j < nlv_limit; j++) {
        int u = -1;
        for (int x = 0; x < p.k; x++)
            if (lvl_of[x] == j) u = x;
        if (u < 0) continue;
        if (in_mask & (1u << u)) {  // u -> leaf: leaf in out(phi(u))
            L.cons_lvl[L.n_cons] = (uint8_t)j;
            L.cons_dir[L.n_cons++] = 0;
            cons_lv |= 1u << j;
        }
        if (out_mask & (1u << u)) {  // leaf -> u: leaf in in(phi(u))
            L.cons_lvl[L.n_cons] = (uint8_t)j;
            L.cons_dir[L.n_cons++] = 1;
            cons_lv |= 1u << j;
        }
    }
    uint32_t all_lv = (nlv_limit >= 32) ? ~0u : ((1u << nlv_limit) - 1);
    L.inj = (uint8_t)(all_lv & ~cons_lv);
}

uint32_t cons_mask_bits(const LevelDesc& L, int c) { return (uint32_t)L.cons_lvl[c] * 2 + L.cons_dir[c]; }

// True (and fills `extra`) when every constraint of src is a constraint of dst.
bool cons_subset(const LevelDesc& src, const LevelDesc& dst, uint16_t& extra) {
    uint32_t have = 0;
    for (int c = 0; c < src.n_cons; c++) have |= 1u << cons_mask_bits(src, c);
    uint32_t covered = 0;
    extra = 0;
    for (int c = 0; c < dst.n_cons; c++) {
        uint32_t b = 1u << cons_mask_bits(dst, c);
        if (have & b) covered |= b;
        else extra |= (uint16_t)(1u << c);
    }
    return covered == have;
}

// Lower the degree filter of level r (and of the levels it reuses from, whose
// candidates it inherits) so that no candidate a reuser needs is dropped.
void weaken(PlanDesc& D, int r, uint32_t need_out, uint32_t need_in) {
    LevelDesc& S = D.lvl[r];
    S.dmin_out = std::min(S.dmin_out, need_out);
    S.dmin_in = std::min(S.dmin_in, need_in);
    S.deg_check = (S.dmin_out || S.dmin_in) ? 1 : 0;
    if (S.reuse != kNoReuse) weaken(D, S.reuse, S.dmin_out, S.dmin_in);
}

void choose_reuse(PlanDesc& D, LevelDesc& L, int max_src_level, uint32_t need_out, uint32_t need_in) {
    int best = -1;
    uint16_t best_extra = 0;
    for (int r = 1; r <= max_src_level; r++) {
        LevelDesc& S = D.lvl[r];
        uint16_t extra;
        if (!cons_subset(S, L, extra)) continue;
        bool weaker = S.dmin_out <= need_out && S.dmin_in <= need_in;
        // a one-list source is only worth reusing when its filter is kept
        if (!weaker && S.n_cons < 2) continue;
        if (best < 0 || S.n_cons >= D.lvl[best].n_cons) {
            best = r;
            best_extra = extra;
        }
    }
    if (best < 0) return;
    // the source keeps only the degree filter every reuser can accept
    weaken(D, best, need_out, need_in);
    L.reuse = (uint8_t)best;
    L.extra = best_extra;
    D.seg_src |= 1u << best;
}

// ---------------------------------------------------------------------------
// Symmetry breaking over the conditioned vertices (the enumerated levels, and
// the leaf when the leaf group is one vertex).
// ---------------------------------------------------------------------------
using Perm = std::array<uint8_t, kMaxK>;

// All automorphisms of the pattern (arc-preserving permutations), by brute
// force over the at most 7! permutations.
std::vector<Perm> automorphisms(const Pat& p) {
    std::vector<Perm> out;
    Perm s{};
    for (int i = 0; i < p.k; i++) s[i] = (uint8_t)i;
    do {
        bool ok = true;
        for (int a = 0; a < p.k && ok; a++) {
            uint32_t img = 0;
            for (int b = 0; b < p.k; b++)
                if (p.out[a] & (1u << b)) img |= 1u << s[b];
            ok = img == p.out[s[a]];
        }
        if (ok) out.push_back(s);
    } while (std::next_permutation(s.begin(), s.begin() + p.k));
    return out;
}

// Sets D.sym_mult and the `gt` masks; drops a reuse whose source was trimmed
// by a bound the reusing descriptor does not have.
void apply_symmetry(const Pat& p, PlanDesc& D, bool below, bool fix_root) {
    const int nc = (int)D.e + (D.t == 1 ? 1 : 0);  // conditioned positions in level order
    uint32_t cmask = 0;
    int pos_of[kMaxK];
    for (int i = 0; i < kMaxK; i++) pos_of[i] = -1;
    for (int i = 0; i < nc; i++) {
        cmask |= 1u << D.order[i];
        pos_of[D.order[i]] = i;
    }
    // H restricted to the conditioned vertices: distinct restrictions of the
    // automorphisms that map that set onto itself
    std::vector<Perm> grp;
    for (const Perm& s : automorphisms(p)) {
        // with a forced start vertex only automorphisms fixing it: then every
        // orbit keeps one root image and counts per root stay exact
        if (fix_root && s[D.order[0]] != D.order[0]) continue;
        uint32_t img = 0;
        for (int v = 0; v < p.k; v++)
            if (cmask & (1u << v)) img |= 1u << s[v];
        if (img != cmask) continue;
        Perm r{};
        for (int v = 0; v < p.k; v++) r[v] = (cmask & (1u << v)) ? s[v] : (uint8_t)v;
        if (std::find(grp.begin(), grp.end(), r) == grp.end()) grp.push_back(r);
    }
    D.sym_mult = (uint32_t)grp.size();
    D.sym_fixes_root = fix_root ? 1 : 0;
    uint8_t gt[kMaxK + 1] = {0};  // by position
    for (int i = 0; i < nc && grp.size() > 1; i++) {
        const int v = D.order[i];
        uint32_t orbit = 0;
        for (const Perm& s : grp) orbit |= 1u << s[v];
        orbit &= ~(1u << v);
        // every vertex of the orbit comes later: the earlier ones are fixed
        for (int u = 0; u < p.k; u++)
            if (orbit & (1u << u)) gt[pos_of[u]] |= (uint8_t)(1u << i);
        std::vector<Perm> stab;
        for (const Perm& s : grp)
            if (s[v] == v) stab.push_back(s);
        grp.swap(stab);
    }
    const uint8_t lt = below ? 1 : 0;
    for (uint32_t l = 1; l < D.e; l++) D.lvl[l].lt = lt;
    for (uint32_t g = 0; g < D.n_sig; g++) D.sig[g].lt = lt;
    for (uint32_t i = 0; i < D.n_masks; i++) D.mdesc[i].lt = lt;
    for (uint32_t l = 1; l < D.e; l++) D.lvl[l].gt = gt[l];
    if (D.t == 1) {
        // one leaf: its signature and the one mask that measures its set
        D.sig[0].gt = gt[D.e];
        for (uint32_t i = 0; i < D.n_masks; i++) D.mdesc[i].gt = gt[D.e];
    }
    auto fix_reuse = [&](LevelDesc& L) {
        if (L.reuse == kNoReuse) return;
        if (D.lvl[L.reuse].gt & ~L.gt) {
            L.reuse = kNoReuse;
            L.extra = 0;
        }
    };
    for (uint32_t l = 2; l < D.e; l++) fix_reuse(D.lvl[l]);
    for (uint32_t g = 0; g < D.n_sig; g++) fix_reuse(D.sig[g]);
    for (uint32_t i = 0; i < D.n_masks; i++) fix_reuse(D.mdesc[i]);
}

// ---------------------------------------------------------------------------
// Plan candidates and their realized constraint covers
// ---------------------------------------------------------------------------
struct Built {
    PlanDesc D;
    std::vector<int> order, leaves, leaf_sig;  // leaf_sig[i]: signature index of leaves[i]
    double cost = 0, cover_w = 0;
};

// Every order of the enumerated vertices E that starts at `start` and binds
// each next vertex next to an already bound one (section 5.1: the plan
// extends from the visited vertices).
std::vector<std::vector<int>> enum_orders(const Pat& p, int start, uint32_t emask) {
    std::vector<std::vector<int>> out;
    std::vector<int> cur{start};
    const int want = popc(emask);
    std::function<void(uint32_t)> rec = [&](uint32_t bound) {
        if ((int)cur.size() == want) {
            out.push_back(cur);
            return;
        }
        for (int v = 0; v < p.k; v++) {
            if (!(emask & (1u << v)) || (bound & (1u << v))) continue;
            if (!(p.nbr(v) & bound)) continue;
            cur.push_back(v);
            rec(bound | (1u << v));
            cur.pop_back();
        }
    };
    rec(1u << start);
    return out;
}

// Levels, leaf signatures, inclusion-exclusion terms and per-mask tests of
// the plan with this vertex order and leaf group.  Returns false when the
// leaf group needs more terms than the descriptor holds.
bool build_desc(const Pat& p, const std::vector<int>& order, const std::vector<int>& leaves, bool reduced, Built& B) {
    PlanDesc& D = B.D;
    std::memset(&D, 0, sizeof(D));
    B.order = order;
    B.leaves = leaves;
    B.leaf_sig.clear();
    D.k = (uint32_t)p.k;
    D.e = (uint32_t)order.size();
    std::vector<int> lvl_of(p.k, -1);
    for (size_t i = 0; i < order.size(); i++) lvl_of[order[i]] = (int)i;
    for (size_t i = 0; i < order.size(); i++) D.order[i] = (uint8_t)order[i];
    D.root_dout = (uint32_t)p.dout(order[0]);
    D.root_din = (uint32_t)p.din(order[0]);
    uint32_t leaf_mask = 0;
    for (int v : leaves) leaf_mask |= 1u << v;
    for (uint32_t i = 1; i < D.e; i++) {
        int v = order[i];
        uint32_t later = leaf_mask;
        for (size_t j = i + 1; j < order.size(); j++) later |= 1u << order[j];
        fill_level(p, lvl_of, v, (int)i, later, D.lvl[i]);
        if (reduced && i >= 2) choose_reuse(D, D.lvl[i], (int)i - 1, D.lvl[i].dmin_out, D.lvl[i].dmin_in);
    }
    // leaf signatures
    std::vector<LeafSig> sigs;
    for (int v : leaves) {
        LeafSig s{p.in[v], p.out[v]};
        if (std::find(sigs.begin(), sigs.end(), s) == sigs.end()) sigs.push_back(s);
    }
    std::sort(sigs.begin(), sigs.end());
    D.n_sig = (uint32_t)sigs.size();
    D.t = (uint32_t)leaves.size();
    for (int v : leaves) {
        LeafSig s{p.in[v], p.out[v]};
        int g = (int)(std::find(sigs.begin(), sigs.end(), s) - sigs.begin());
        B.leaf_sig.push_back(g);
        D.sig_mult[g]++;
    }
    for (uint32_t g = 0; g < D.n_sig; g++) {
        // any leaf of this signature gives the same constraint set
        int v = -1;
        for (size_t i = 0; i < leaves.size(); i++)
            if (B.leaf_sig[i] == (int)g) v = leaves[i];
        fill_level(p, lvl_of, v, (int)D.e, 0u, D.sig[g]);
        D.sig[g].dmin_out = D.sig[g].dmin_in = 0;  // implied by the constraints of a leaf
        D.sig[g].deg_check = 0;
        if (reduced && D.e >= 2)
            choose_reuse(D, D.sig[g], (int)D.e - 1, (uint32_t)p.dout(v), (uint32_t)p.din(v));
    }
    std::vector<Term> terms;
    if (!leaf_terms(B.leaf_sig, terms)) return false;
    D.n_terms = (uint32_t)terms.size();
    for (size_t i = 0; i < terms.size(); i++) D.terms[i] = terms[i];
    D.linear = (D.t == 1) ? 1 : 0;
    for (size_t i = 0; i < leaves.size(); i++) D.order[D.e + i] = (uint8_t)leaves[i];
    // one candidate test per signature mask the terms use
    uint32_t used = 0;
    for (uint32_t i = 0; i < D.n_terms; i++)
        for (int b = 0; b < D.terms[i].nb; b++) used |= 1u << D.terms[i].mask[b];
    D.n_masks = 0;
    for (uint32_t M = 1; M < 16; M++) {
        if (!((used >> M) & 1u)) continue;
        uint32_t in = 0, out = 0;
        for (uint32_t g = 0; g < D.n_sig; g++)
            if ((M >> g) & 1u) {
                in |= sigs[g].in_mask;
                out |= sigs[g].out_mask;
            }
        LevelDesc L;
        std::memset(&L, 0, sizeof L);
        fill_level_sig(p, lvl_of, in, out, (int)D.e, L);
        // a node in every set of M has all of M's arcs to bound nodes
        if (reduced && D.e >= 2) choose_reuse(D, L, (int)D.e - 1, (uint32_t)popc(out), (uint32_t)popc(in));
        // a mask whose test equals an earlier one's has the same set
        uint32_t j = 0;
        while (j < D.n_masks && std::memcmp(&D.mdesc[j], &L, sizeof L) != 0) j++;
        if (j == D.n_masks) {
            D.mdesc[j] = L;
            D.mask_id[j] = (uint8_t)M;
            D.mask_set[j] = 0;
            D.n_masks++;
        }
        D.mask_set[j] |= (uint16_t)(1u << M);
    }
    return true;
}

// The arcs the plan reads from the data graph (its realized constraint
// cover).  A level fetches every constraint list it does not take from a
// reused candidate set (section 5.2: an included arc is materialised from
// the including arc's result); the leaf passes the kernel runs (the one
// signature of a one-leaf plan, else every signature mask) fetch the same
// way, and a list read for several leaves of one signature is attributed to
// the first of them, the other leaves' arcs being included by its arc
// (shared endpoint, Theorem 2.1).  Bit i stands for p.arcs[i].
uint64_t fetched_arcs(const Pat& p, const Built& B) {
    const PlanDesc& D = B.D;
    auto arc_index = [&](int a, int b) -> int {
        for (size_t i = 0; i < p.arcs.size(); i++)
            if (p.arcs[i].first == a && p.arcs[i].second == b) return (int)i;
        return -1;
    };
    uint64_t f = 0;
    // dir 0: x in out(phi(u)), arc u -> x; dir 1: x in in(phi(u)), arc x -> u
    auto mark = [&](int u, int x, int dir) {
        const int i = dir ? arc_index(x, u) : arc_index(u, x);
        if (i >= 0) f |= 1ull << i;
    };
    auto read = [&](const LevelDesc& L, int c) { return L.reuse == kNoReuse || ((L.extra >> c) & 1u); };
    for (uint32_t i = 1; i < D.e; i++) {
        const LevelDesc& L = D.lvl[i];
        for (int c = 0; c < L.n_cons; c++)
            if (read(L, c)) mark(B.order[L.cons_lvl[c]], B.order[i], L.cons_dir[c]);
    }
    auto rep = [&](uint32_t g) {
        for (size_t i = 0; i < B.leaves.size(); i++)
            if (B.leaf_sig[i] == (int)g) return B.leaves[i];
        return -1;
    };
    auto has_cons = [](const LevelDesc& L, int lvl, int dir) {
        for (int c = 0; c < L.n_cons; c++)
            if (L.cons_lvl[c] == lvl && L.cons_dir[c] == dir) return true;
        return false;
    };
    if (D.linear) {
        const LevelDesc& L = D.sig[0];
        for (int c = 0; c < L.n_cons; c++)
            if (read(L, c)) mark(B.order[L.cons_lvl[c]], rep(0), L.cons_dir[c]);
    } else {
        for (uint32_t mi = 0; mi < D.n_masks; mi++) {
            const LevelDesc& L = D.mdesc[mi];
            const uint32_t M = D.mask_id[mi];
            for (int c = 0; c < L.n_cons; c++) {
                if (!read(L, c)) continue;
                for (uint32_t g = 0; g < D.n_sig; g++)
                    if (((M >> g) & 1u) && has_cons(D.sig[g], L.cons_lvl[c], L.cons_dir[c])) {
                        mark(B.order[L.cons_lvl[c]], rep(g), L.cons_dir[c]);
                        break;
                    }
            }
        }
    }
    return f;
}

// Weight of the realized cover: for every list read, the estimated number of
// partial matches that read it times the mean list length (unit graph of
// 10^6 nodes and mean degree 16 without statistics).  Partial matches grow
// by d (d/n)^(c-1) per level with c constraints.
double cover_weight(const Pat& p, const Built& B, const GraphStats* gs) {
    const PlanDesc& D = B.D;
    const double n = (gs && gs->n) ? (double)gs->n : 1e6;
    const double d = (gs && gs->n) ? std::max(1.0, (double)gs->m / (double)gs->n) : 16.0;
    double P[kMaxK + 1];
    P[0] = n;
    for (uint32_t i = 1; i < D.e; i++) P[i] = P[i - 1] * d * std::pow(d / n, (double)D.lvl[i].n_cons - 1.0);
    auto reads = [](const LevelDesc& L) {
        int r = 0;
        for (int c = 0; c < L.n_cons; c++) r += (L.reuse == kNoReuse || ((L.extra >> c) & 1u)) ? 1 : 0;
        return r;
    };
    double w = 0;
    for (uint32_t i = 1; i < D.e; i++) w += P[i - 1] * d * reads(D.lvl[i]);
    if (D.linear) {
        w += P[D.e - 1] * d * reads(D.sig[0]);
    } else {
        for (uint32_t mi = 0; mi < D.n_masks; mi++) w += P[D.e - 1] * d * reads(D.mdesc[mi]);
    }
    (void)p;
    return w;
}

}  // namespace

// ---------------------------------------------------------------------------
std::string plan_json(const Pat& p, const PlanDesc& D, const CoverReport& cr, bool reduced,
                      double cost, uint64_t fetched, double cover_w) {
    std::string s;
    char buf[256];
    auto arcstr = [&](int e) {
        std::snprintf(buf, sizeof buf, "[%d,%d]", p.arcs[e].first, p.arcs[e].second);
        return std::string(buf);
    };
    s += "{\"kind\":\"";
    s += reduced ? "reduced" : "unreduced";
    std::snprintf(buf, sizeof buf, "\",\"k\":%u,\"e\":%u,\"n_arcs\":%zu,\"root_vertex\":%d,", D.k, D.e,
                  p.arcs.size(), D.order[0]);
    s += buf;
    std::snprintf(buf, sizeof buf, "\"root_dmin\":[%u,%u],\"est_cost\":%.6g,\"order\":[", D.root_dout,
                  D.root_din, cost);
    s += buf;
    for (uint32_t i = 0; i < D.k; i++) {
        std::snprintf(buf, sizeof buf, "%s%d", i ? "," : "", D.order[i]);
        s += buf;
    }
    s += "],\"levels\":[";
    auto lvl_json = [&](const LevelDesc& L) {
        std::string o = "{\"cons\":[";
        for (int c = 0; c < L.n_cons; c++) {
            std::snprintf(buf, sizeof buf, "%s[%d,%d]", c ? "," : "", L.cons_lvl[c], L.cons_dir[c]);
            o += buf;
        }
        std::snprintf(buf, sizeof buf, "],\"reuse\":%d,\"extra\":%u,\"inj\":%u,\"dmin\":[%u,%u],\"gt\":%u,\"lt\":%u}",
                      L.reuse == kNoReuse ? -1 : (int)L.reuse, (unsigned)L.extra, (unsigned)L.inj,
                      L.dmin_out, L.dmin_in, (unsigned)L.gt, (unsigned)L.lt);
        o += buf;
        return o;
    };
    for (uint32_t i = 1; i < D.e; i++) {
        if (i > 1) s += ",";
        s += lvl_json(D.lvl[i]);
    }
    s += "],\"leaf_sigs\":[";
    for (uint32_t g = 0; g < D.n_sig; g++) {
        if (g) s += ",";
        std::string o = lvl_json(D.sig[g]);
        o.pop_back();
        std::snprintf(buf, sizeof buf, ",\"mult\":%u}", D.sig_mult[g]);
        o += buf;
        s += o;
    }
    std::snprintf(buf, sizeof buf,
                  "],\"t\":%u,\"linear\":%u,\"seg_src\":%u,\"sym_mult\":%u,\"sym_fixes_root\":%u,\"root_share\":%u,"
                  "\"terms\":[",
                  D.t, D.linear, D.seg_src, D.sym_mult ? D.sym_mult : 1u, (unsigned)D.sym_fixes_root,
                  (unsigned)D.root_share);
    s += buf;
    for (uint32_t i = 0; i < D.n_terms; i++) {
        std::snprintf(buf, sizeof buf, "%s{\"coef\":%d,\"masks\":[", i ? "," : "", D.terms[i].coef);
        s += buf;
        for (int b = 0; b < D.terms[i].nb; b++) {
            std::snprintf(buf, sizeof buf, "%s%u", b ? "," : "", D.terms[i].mask[b]);
            s += buf;
        }
        s += "]}";
    }
    s += "],\"masks\":[";
    for (uint32_t i = 0; i < D.n_masks; i++) {
        if (i) s += ",";
        std::string o = lvl_json(D.mdesc[i]);
        o.pop_back();
        std::snprintf(buf, sizeof buf, ",\"mask\":%u,\"mask_set\":[", D.mask_id[i]);
        o += buf;
        bool first = true;
        for (uint32_t M = 1; M < 16; M++)
            if ((D.mask_set[i] >> M) & 1u) {
                std::snprintf(buf, sizeof buf, "%s%u", first ? "" : ",", M);
                o += buf;
                first = false;
            }
        o += "]}";
        s += o;
    }
    s += "],\"arcs\":[";
    for (size_t e = 0; e < p.arcs.size(); e++) s += (e ? "," : "") + arcstr((int)e);
    s += "],\"inclusion_groups\":{\"in\":[";
    for (int v = 0; v < p.k; v++) {
        std::snprintf(buf, sizeof buf, "%s%d", v ? "," : "", cr.groups_in_rep[v]);
        s += buf;
    }
    s += "],\"out\":[";
    for (int v = 0; v < p.k; v++) {
        std::snprintf(buf, sizeof buf, "%s%d", v ? "," : "", cr.groups_out_rep[v]);
        s += buf;
    }
    s += "]},\"min_cover\":[";
    for (size_t i = 0; i < cr.min_cover.size(); i++) s += (i ? "," : "") + arcstr(cr.min_cover[i]);
    std::snprintf(buf, sizeof buf, "],\"min_cover_weight\":%.6g,\"greedy_cover\":[", cr.min_cover_weight);
    s += buf;
    for (size_t i = 0; i < cr.greedy_cover.size(); i++) s += (i ? "," : "") + arcstr(cr.greedy_cover[i]);
    // the plan's realized cover: arcs read from the data graph, and arcs whose
    // candidates come from an including arc's result
    s += "],\"cover\":{\"fetched\":[";
    bool first = true;
    for (size_t e = 0; e < p.arcs.size(); e++)
        if ((fetched >> e) & 1ull) {
            s += (first ? "" : ",") + arcstr((int)e);
            first = false;
        }
    s += "],\"removed\":[";
    first = true;
    size_t removed = 0;
    for (size_t e = 0; e < p.arcs.size(); e++)
        if (!((fetched >> e) & 1ull)) {
            s += (first ? "" : ",") + arcstr((int)e);
            first = false;
            removed++;
        }
    std::snprintf(buf, sizeof buf, "],\"weight\":%.6g},\"removed_edges\":%zu}", cover_w, removed);
    s += buf;
    return s;
}

int build_plan(uint32_t k, uint32_t n_arcs, const uint8_t* arcs, uint32_t flags, const GraphStats* gs,
               PlanDesc& D, std::string& json, std::string& err) {
    if (k < 2 || k > (uint32_t)kMaxK) {
        err = "pattern must have 2..7 vertices";
        return -2;
    }
    if (n_arcs == 0 || !arcs) {
        err = "pattern has no arcs";
        return -2;
    }
    Pat p;
    p.k = (int)k;
    for (uint32_t i = 0; i < n_arcs; i++) {
        int a = arcs[2 * i], b = arcs[2 * i + 1];
        if (a >= (int)k || b >= (int)k) {
            err = "arc endpoint out of range";
            return -2;
        }
        if (a == b) {
            err = "self-loop arc in pattern";
            return -2;
        }
        p.out[a] |= 1u << b;
        p.in[b] |= 1u << a;
    }
    for (int a = 0; a < p.k; a++)
        for (int b = 0; b < p.k; b++)
            if (p.out[a] & (1u << b)) p.arcs.push_back({a, b});
    uint32_t allv = (1u << k) - 1;
    if (!connected(p, allv)) {
        err = "pattern is not weakly connected";
        return -2;
    }
    bool reduced = (flags & 0x3u) == 0x1u;
    if ((flags & 0x3u) != 0x1u && (flags & 0x3u) != 0x2u) {
        err = "exactly one of XM_PLAN_REDUCED / XM_PLAN_UNREDUCED";
        return -1;
    }
    int forced = (int)((flags >> 8) & 0xFu) - 1;
    const uint32_t share = (flags >> 16) & 0xFFu;
    if (share > 31) {
        err = "root share exponent must be at most 31";
        return -1;
    }
    if (forced >= p.k) {
        err = "forced root vertex out of range";
        return -1;
    }
    // Start vertex (Algorithm 1: maximal degree; ties: larger out-degree, then lowest id).
    int start = 0;
    for (int v = 1; v < p.k; v++)
        if (p.deg(v) > p.deg(start) || (p.deg(v) == p.deg(start) && p.dout(v) > p.dout(start))) start = v;
    if (forced >= 0) start = forced;

    CoverReport cr = analyse_cover(p, gs, start);

    // Candidate plans: a leaf group (trailing independent vertices counted by
    // product, section 5.3) and an order of the enumerated vertices (section
    // 5.1).  Each candidate's descriptors decide which arcs the kernel reads
    // from the data graph (its realized constraint cover, section 4.2) and
    // which it takes from an including arc's candidate set (section 5.2).
    // The reduced plan keeps the most leaves, then the smallest weight of
    // its realized cover (the paper's objective argmin sum ||A_e|| with each
    // ||A_e|| the estimated list reads of that arc in the plan's context),
    // then the smaller enumeration estimate.
    Cand best;
    bool have = false;
    Built bb;
    if (reduced) {
        for (uint32_t L = 0; L <= allv; L++) {
            if (L & (1u << start)) continue;
            if (L == 0) continue;
            int t = popc(L);
            if (t > kMaxLeaves || t >= p.k) continue;
            if (have && t < (int)best.leaves.size()) continue;
            bool indep = true;
            for (int v = 0; v < p.k && indep; v++)
                if ((L & (1u << v)) && (p.nbr(v) & L)) indep = false;
            if (!indep) continue;
            uint32_t E = allv & ~L;
            if (!connected(p, E)) continue;
            std::vector<LeafSig> sigs;
            for (int v = 0; v < p.k; v++)
                if (L & (1u << v)) {
                    LeafSig s{p.in[v], p.out[v]};
                    if (std::find(sigs.begin(), sigs.end(), s) == sigs.end()) sigs.push_back(s);
                }
            if ((int)sigs.size() > kMaxSig) continue;
            std::vector<int> leaves;
            for (int v = 0; v < p.k; v++)
                if (L & (1u << v)) leaves.push_back(v);
            for (const std::vector<int>& ord : enum_orders(p, start, E)) {
                Built c;
                if (!build_desc(p, ord, leaves, true, c)) continue;  // term budget
                c.cost = model_cost(p, ord, (int)sigs.size(), gs);
                c.cover_w = cover_weight(p, c, gs);
                const bool better =
                    !have || leaves.size() > best.leaves.size() ||
                    (leaves.size() == best.leaves.size() &&
                     (c.cover_w < bb.cover_w * (1 - 1e-9) ||
                      (c.cover_w <= bb.cover_w * (1 + 1e-9) && c.cost < best.cost * (1 - 1e-9))));
                if (better) {
                    best.order = ord;
                    best.leaves = leaves;
                    best.cost = c.cost;
                    bb = c;
                    have = true;
                }
            }
        }
    }
    if (!have) {
        // unreduced: all vertices in greedy order, the last one counted
        std::vector<int> ord = enum_order(p, start, allv);
        best.order.assign(ord.begin(), ord.end() - 1);
        best.leaves = {ord.back()};
        best.cost = model_cost(p, best.order, 1, gs);
        build_desc(p, best.order, best.leaves, false, bb);
        bb.cover_w = cover_weight(p, bb, gs);
    }
    D = bb.D;
    D.sym_mult = 1;
    D.root_share = (uint8_t)share;
    // a root share is a root subset: symmetry breaking then keeps only the
    // automorphisms that fix the start vertex, so every orbit stays in it
    if (flags & 0x4u) apply_symmetry(p, D, (flags & 0x8u) != 0, forced >= 0 || share > 0);
    // packed constraint fields read by the kernel
    auto pack = [](LevelDesc& L) {
        L.dir_mask = 0;
        L.lvl_bits = 0;
        for (int c = 0; c < L.n_cons; c++) {
            L.dir_mask |= (uint16_t)((L.cons_dir[c] & 1u) << c);
            L.lvl_bits |= (uint64_t)(L.cons_lvl[c] & 7u) << (3 * c);
        }
    };
    for (uint32_t i = 1; i < D.e; i++) pack(D.lvl[i]);
    for (uint32_t g = 0; g < D.n_sig; g++) pack(D.sig[g]);
    for (uint32_t i = 0; i < D.n_masks; i++) pack(D.mdesc[i]);
    // the realized cover after symmetry breaking (which may drop a reuse)
    bb.D = D;
    const uint64_t fetched = fetched_arcs(p, bb);
    json = plan_json(p, D, cr, reduced, best.cost, fetched, cover_weight(p, bb, gs));
    return 0;
}

}  // namespace xm
