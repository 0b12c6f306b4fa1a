// count.hip — gfx950 kernels that execute counting plans.
//
// Algorithm 2 (plan execution) run by wavefronts.  Each wave is a worker
// that takes tasks from two device queues: first-level sub-ranges of hub
// roots (split by the split kernel so that other waves can take them, the
// work-stealing of Algorithm 2's parallel loop), then chunks of ordinary
// roots.  A task is explored depth-first, one level buffer per plan level;
// each buffer holds a window of partial matches, and every expansion is
// flattened across the window so that the 64 lanes stay busy even when
// adjacency lists are short (power-law graphs have mostly short lists).
//
// Per element of a base list a lane checks, in order: injectivity against
// the bound nodes (visited marks), the degree thresholds, and membership in
// every other constraint list: one bit test when the list is long enough to
// have a dense row (an n-bit membership row built at graph load, the HBM
// analogue of staging a hub's list), else a binary search of the sorted
// uint32 list.  The
// survivors are compacted with a 64-bit ballot and a popcount.  The leaf
// group of a plan is counted, not enumerated: with one leaf the count is a
// popcount sum; with several, each partial match builds a membership
// histogram in LDS and evaluates the planner's inclusion-exclusion terms in
// 128-bit integers.  Totals are unsigned 128-bit, kept as (lo, hi) uint64
// pairs updated with 64-bit atomics and an explicit carry.
//
// Nothing here is a dense contraction, so no matrix cores are used; the
// kernels are bound by memory latency and bandwidth of list reads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"
#include "u128.h"

namespace xm {

static_assert(sizeof(PlanDesc) % 4 == 0, "plan descriptors are copied in 32-bit words");

constexpr uint32_t kSkip = 0xFFFFFFFFu;
constexpr uint32_t kIdlePolls = 1u << 13;  // polls a waiting wave makes for donated work (at most ~28 us apart)
constexpr uint32_t kMaxWaiters = 512;      // waves that wait for donated work; the others leave
constexpr uint32_t kDonateAfter = 256;     // windows a task runs before it may donate
constexpr uint32_t kComplete = 0x80000000u;

__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// Make this wave's global and LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Wave-wide inclusive scans (sum, max) over the 64 lanes with DPP row
// shifts and row broadcasts: 6 VALU steps, no LDS traffic.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}
__device__ __forceinline__ uint32_t scan_incl(uint32_t v, uint32_t) {
    v += dpp_<0x111, 0xf>(v);  // row_shr:1
    v += dpp_<0x112, 0xf>(v);  // row_shr:2
    v += dpp_<0x114, 0xf>(v);  // row_shr:4
    v += dpp_<0x118, 0xf>(v);  // row_shr:8
    v += dpp_<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}
__device__ __forceinline__ uint32_t scan_max(uint32_t v) {
    v = max(v, dpp_<0x111, 0xf>(v));
    v = max(v, dpp_<0x112, 0xf>(v));
    v = max(v, dpp_<0x114, 0xf>(v));
    v = max(v, dpp_<0x118, 0xf>(v));
    v = max(v, dpp_<0x142, 0xa>(v));
    v = max(v, dpp_<0x143, 0xc>(v));
    return v;
}

// Sorted-list membership: branchless search for the last element <= x.
__device__ __forceinline__ bool contains(const uint32_t* __restrict__ a, uint32_t len, uint32_t x) {
    if (len == 0) return false;
    uint32_t base = 0, n = len;
    while (n > 1) {
        uint32_t h = n >> 1;
        base = (a[base + h] <= x) ? base + h : base;
        n -= h;
    }
    return a[base] == x;
}

__device__ __forceinline__ const uint32_t* adj_of(const DevGraph& g, uint32_t dir) {
    return dir ? g.in_adj : g.out_adj;
}
__device__ __forceinline__ const uint32_t* off_of(const DevGraph& g, uint32_t dir) {
    return dir ? g.in_off : g.out_off;
}

// The probe of list (dir, node nd) at adjacency offset o with length l: the
// list itself, or its dense row (length kRowLen) when it has one.
__device__ __forceinline__ const uint32_t* probe_ref(const DevGraph& g, uint32_t dir, uint32_t nd, uint32_t o,
                                                     uint32_t& l) {
    if (l >= g.row_min) {
        const uint2 r = g.row_of[nd];
        const uint32_t row = dir ? r.y : r.x;
        if (row != kSkip) {
            l = kRowLen;
            return g.rows + (uint64_t)row * g.row_words;
        }
    }
    return adj_of(g, dir) + o;
}

__device__ __forceinline__ const uint32_t* join_ptr(uint32_t lo, uint32_t hi) {
    return reinterpret_cast<const uint32_t*>(((uint64_t)hi << 32) | lo);
}

// Any address that may be read (a lane with nothing to probe reads it and
// ignores the value).
__device__ __forceinline__ const uint32_t* safe_ptr(const DevGraph& g) {
    return reinterpret_cast<const uint32_t*>(g.deg);
}

// Per-level constraint fields, loaded once into scalar registers.
struct LK {
    uint32_t n_cons, reuse, inj, deg_check, extra, dirm, dmin_out, dmin_in, gt, lt;
    uint64_t lvlb;
    __device__ __forceinline__ uint32_t lvl(uint32_t c) const { return (uint32_t)(lvlb >> (3 * c)) & 7u; }
    __device__ __forceinline__ uint32_t dir(uint32_t c) const { return (dirm >> c) & 1u; }
};
__device__ __forceinline__ LK load_lk(const LevelDesc& D, const KArgs& a) {
    LK k;
    k.n_cons = uni(D.n_cons);
    if (k.n_cons > a.maxc) {
        // the per-wave probe arrays hold maxc constraints: never index past them
        atomicOr(&a.ctl[kCtlBadPlan], 1u);
        k.n_cons = a.maxc;
    }
    k.reuse = uni(D.reuse);
    k.inj = uni(D.inj);
    k.deg_check = uni(D.deg_check);
    k.extra = uni(D.extra);
    k.dirm = uni(D.dir_mask);
    k.dmin_out = uni(D.dmin_out);
    k.dmin_in = uni(D.dmin_in);
    k.gt = uni(D.gt);
    k.lt = uni(D.lt);
    k.lvlb = ((uint64_t)uni((uint32_t)(D.lvl_bits >> 32)) << 32) | uni((uint32_t)D.lvl_bits);
    return k;
}

// Unsigned 128-bit atomic add into (lo, hi) with an overflow flag.
__device__ void add_u128(unsigned long long* c, unsigned long long lo, unsigned long long hi,
                         uint32_t* flag) {
    if (lo) {
        unsigned long long old = atomicAdd(c, lo);
        if (old + lo < old) {
            hi += 1;
            if (hi == 0) atomicOr(flag, 1u);
        }
    }
    if (hi) {
        unsigned long long old = atomicAdd(c + 1, hi);
        if (old + hi < old) atomicOr(flag, 1u);
    }
}

// Per-wave LDS carve-out.
struct Lds {
    uint32_t* bound;     // [kMaxK][64]
    uint32_t* anc;       // [kMaxK][64]
    uint32_t* base_lo;   // [64]: address of the parent's base list (low word)
    uint32_t* base_len;  // [64]
    uint32_t* base_hi;   // [64]: (high word)
    uint32_t* incl;      // [64]
    uint32_t* segcnt;    // [64]
    uint32_t* mark;      // [128]: tile parent marks
    uint32_t* slot_len;  // [maxc][64]: probe k of the parent: list length, kRowLen, or kSkip
    uint32_t* slot_lo;   // [maxc][64]: address of the list or of the dense row (low word)
    uint32_t* slot_hi;   // [maxc][64]: (high word)
    uint32_t* hist;      // [64][16]
    uint32_t* st;        // wave state: cur[8], pofs[8], n[8]
    uint32_t* mbuf;      // [kMergeChunk]: probe-list chunk of the cooperative merge
};

__device__ __forceinline__ Lds carve(uint32_t* w, uint32_t rows, uint32_t maxc, bool merge) {
    Lds s;
    s.bound = w;
    s.anc = w + rows * 64;
    uint32_t* q = w + 2 * rows * 64;
    s.base_lo = q;
    s.base_len = q + 64;
    s.base_hi = q + 128;
    s.incl = q + 192;
    s.segcnt = q + 256;
    s.mark = q + 320;
    q += 7 * 64;
    s.slot_len = q;
    s.slot_lo = q + maxc * 64;
    s.slot_hi = q + 2 * maxc * 64;
    q += 3 * maxc * 64;
    s.mbuf = q;
    q += merge ? kMergeChunk : 0;
    s.st = q;
    s.hist = q + 32;
    return s;
}

struct Lvl {
    uint32_t* node;
    uint32_t* parent;  // level 0: first-level range start
    uint32_t* segb;
    uint32_t* segc;    // child count | kComplete
    uint32_t* aux;     // level 0: first-level range end
};

__device__ __forceinline__ Lvl lvl_arrays(uint32_t* scr, uint32_t cap, uint32_t l) {
    uint32_t* b = scr + (size_t)l * kLvlArrays * cap;
    return {b, b + cap, b + 2 * cap, b + 3 * cap, b + 4 * cap};
}

struct Ctx {
    const KArgs* a;
    const PlanDesc* P;
    uint32_t pi;
    Lds s;
    uint32_t* scr;
    uint32_t lane;
    unsigned long long acc_lo, acc_hi;  // per-lane 128-bit partial (leaf groups)
    bool ovf;                           // this lane's partial or a leaf-group term left the 128-bit range
    bool donated;                       // this wave has handed off work (it then always waits)
    bool stop;                          // the cancel flag was seen: leave the task
    uint32_t polls;                     // leaf blocks since the last look at the cancel flag
};

// First-level base list length of root r for plan P (shortest constraint list).
__device__ __forceinline__ uint32_t level1_len(const DevGraph& g, const PlanDesc* P, uint32_t r) {
    const LevelDesc& D = P->lvl[1];
    uint32_t best = kSkip;
    for (uint32_t c = 0; c < D.n_cons; c++) {
        const uint32_t* off = off_of(g, D.cons_dir[c]);
        uint32_t l = off[r + 1] - off[r];
        best = l < best ? l : best;
    }
    return best;
}

// Number of elements <= x in the sorted list a[0, n).
__device__ __forceinline__ uint32_t count_le(const uint32_t* __restrict__ a, uint32_t n, uint32_t x) {
    uint32_t lo = 0;
    while (n > 0) {
        const uint32_t h = n >> 1;
        if (a[lo + h] <= x) {
            lo += h + 1;
            n -= h + 1;
        } else {
            n = h;
        }
    }
    return lo;
}

// Symmetry breaking: the part of the sorted list a[0, len) that lies above
// the largest (lt = 0) or below the smallest (lt = 1) bound image among the
// levels in gt (levels < lv) of this lane's partial match.
__device__ __forceinline__ void sym_trim(const Lds& s, uint32_t gt, uint32_t lt, uint32_t lv, uint32_t lane,
                                         const uint32_t*& a, uint32_t& len) {
    uint32_t lo = 0xFFFFFFFFu, hi = 0;
    for (uint32_t l = 0; l < lv; l++)
        if ((gt >> l) & 1u) {
            const uint32_t b = s.bound[l * 64 + lane];
            lo = b < lo ? b : lo;
            hi = b > hi ? b : hi;
        }
    if (lt) {
        len = lo ? count_le(a, len, lo - 1u) : 0u;
    } else {
        const uint32_t skip = count_le(a, len, hi);
        a += skip;
        len -= skip;
    }
}

// Phase A of a level: lane = one partial match (parent) of the window.  Walks
// the parent chain into LDS (bound nodes, ancestor indices), picks the base
// list and writes the probes (the other constraint lists, long ones as their
// dense rows) into the parent's probe slots.  Returns the base length.
template <bool IS_SIG>
__device__ uint32_t phase_a(Ctx& C, const LK& D, uint32_t lv, uint32_t p, bool pv, bool walk) {
    const KArgs& a = *C.a;
    const DevGraph& g = a.g;
    const uint32_t lane = C.lane;
    uint32_t len = 0;
    if (!pv) {
        C.s.base_len[lane] = 0;
        return 0;
    }
    if (walk) {
        uint32_t idx = p;
        for (int l = (int)lv - 1; l >= 0; --l) {
            Lvl F = lvl_arrays(C.scr, a.cap, (uint32_t)l);
            C.s.bound[l * 64 + lane] = F.node[idx];
            C.s.anc[l * 64 + lane] = idx;
            if (l > 0) idx = F.parent[idx];
        }
    }
    auto put = [&](uint32_t k, const uint32_t* ptr, uint32_t l) {
        const uint64_t v = reinterpret_cast<uint64_t>(ptr);
        C.s.slot_len[k * 64 + lane] = l;
        C.s.slot_lo[k * 64 + lane] = (uint32_t)v;
        C.s.slot_hi[k * 64 + lane] = (uint32_t)(v >> 32);
    };
    const uint32_t* base = nullptr;
    uint32_t k = 0;
    bool fetched = false;
    if (D.reuse != kNoReuse) {
        uint32_t r = D.reuse;
        uint32_t ai = C.s.anc[(r - 1) * 64 + lane];
        Lvl F = lvl_arrays(C.scr, a.cap, r - 1);
        uint32_t sc = F.segc[ai];
        if (sc & kComplete) {
            base = lvl_arrays(C.scr, a.cap, r).node + F.segb[ai];
            len = sc & ~kComplete;
            for (uint32_t c = 0; c < D.n_cons; c++) {
                if (!((D.extra >> c) & 1u)) continue;
                const uint32_t nd = C.s.bound[D.lvl(c) * 64 + lane];
                const uint32_t* off = off_of(g, D.dir(c));
                const uint32_t o = off[nd];
                uint32_t l = off[nd + 1] - o;
                const uint32_t* ptr = probe_ref(g, D.dir(c), nd, o, l);
                put(k++, ptr, l);
            }
            fetched = true;
        }
    }
    if (!fetched) {
        // the shortest list is the base; the others are probed
        uint32_t best = kSkip, bc = 0, bo = 0;
        uint32_t dbest = kSkip, dc = 0, dof = 0, dlv = 0;  // shortest list at the deepest bound level
        for (uint32_t c = 0; c < D.n_cons; c++) {
            const uint32_t nd = C.s.bound[D.lvl(c) * 64 + lane];
            const uint32_t* off = off_of(g, D.dir(c));
            const uint32_t o = off[nd], l = off[nd + 1] - o;
            if (l < best) {
                best = l;
                bc = c;
                bo = o;
            }
            if (D.lvl(c) > dlv || (D.lvl(c) == dlv && l < dbest)) {
                dlv = D.lvl(c);
                dbest = l;
                dc = c;
                dof = o;
            }
        }
        // the first level keeps the shortest: root sub-ranges index into it
        if (kFreshBaseRatio && (IS_SIG || lv >= 2) && D.lvl(bc) < dlv &&
            (uint64_t)dbest <= (uint64_t)kFreshBaseRatio * best) {
            best = dbest;
            bc = dc;
            bo = dof;
        }
        for (uint32_t c = 0; c < D.n_cons; c++) {
            if (c == bc) continue;
            const uint32_t nd = C.s.bound[D.lvl(c) * 64 + lane];
            const uint32_t* off = off_of(g, D.dir(c));
            const uint32_t o = off[nd];
            uint32_t l = off[nd + 1] - o;
            const uint32_t* ptr = probe_ref(g, D.dir(c), nd, o, l);
            put(k++, ptr, l);
        }
        base = adj_of(g, D.dir(bc)) + bo;
        len = best;
        if (!IS_SIG && lv == 1) {
            // a root carries its first-level range [lo, hi)
            Lvl F0 = lvl_arrays(C.scr, a.cap, 0);
            uint32_t lo = F0.parent[p], hi = F0.aux[p];
            hi = hi < len ? hi : len;
            lo = lo < hi ? lo : hi;
            base += lo;
            len = hi - lo;
        }
    }
    for (; k < D.n_cons; k++) put(k, safe_ptr(g), kSkip);
    // symmetry breaking: the base is sorted, so its candidates are a range
    if (D.gt) sym_trim(C.s, D.gt, D.lt, lv, lane, base, len);
    const uint64_t bv = reinterpret_cast<uint64_t>(base);
    C.s.base_lo[lane] = (uint32_t)bv;
    C.s.base_hi[lane] = (uint32_t)(bv >> 32);
    C.s.base_len[lane] = len;
    return len;
}

// Probe slots a level uses: all but the base constraint, or (when reusing a
// complete candidate set) the extra constraints; lanes with fewer pad with
// kSkip.
__device__ __forceinline__ uint32_t n_slots(const LK& D) {
    return D.reuse == kNoReuse ? (D.n_cons ? D.n_cons - 1 : 0) : D.n_cons;
}

// Base element `local` of window parent j.
__device__ __forceinline__ uint32_t base_elem(const Ctx& C, uint32_t j, uint32_t local) {
    return join_ptr(C.s.base_lo[j], C.s.base_hi[j])[local];
}

// Window parents of the elements t0 + lane (tile a) and t0 + 64 + lane (tile
// b) of a flattened pass.  Lane j (a window parent) owns the elements
// [start, start + len); parents that own elements mark their first one, and a
// max-scan carries each mark forward.  `carry` is the parent of the last
// element of the previous step (0 before the first).
__device__ __forceinline__ void tile_parents(const Lds& s, uint32_t lane, uint32_t t0, uint32_t start, bool owns,
                                             uint32_t& carry, uint32_t& ja, uint32_t& jb) {
    s.mark[lane] = 0;
    s.mark[64 + lane] = 0;
    wave_sync();
    if (owns && start >= t0 && start - t0 < 128u) s.mark[start - t0] = lane + 1;
    wave_sync();
    const uint32_t ma = scan_max(s.mark[lane]);
    const uint32_t mb = scan_max(s.mark[64 + lane]);
    ja = ma ? ma - 1 : carry;
    const uint32_t last_a = uni(__shfl(ja, 63, 64));
    jb = mb ? mb - 1 : last_a;
    carry = uni(__shfl(jb, 63, 64));
}

// Two sorted-list searches per lane (one per element), both loads of a step
// issued together.  A lane without a search passes n = 0 and a readable
// pointer (its value is ignored).
__device__ __forceinline__ void search2(const uint32_t* __restrict__ A, uint32_t na, uint32_t xa, bool& fa,
                                        const uint32_t* __restrict__ B, uint32_t nb, uint32_t xb, bool& fb) {
    uint32_t ba = 0, bb = 0, ra = na, rb = nb;
    while (__ballot(ra > 1 || rb > 1)) {
        const uint32_t ha = ra >> 1, hb = rb >> 1;
        const uint32_t va = A[ba + ha], vb = B[bb + hb];
        ba = (va <= xa) ? ba + ha : ba;
        bb = (vb <= xb) ? bb + hb : bb;
        ra -= ha;
        rb -= hb;
    }
    const uint32_t ea = A[ba], eb = B[bb];
    fa = na > 0 && ea == xa;
    fb = nb > 0 && eb == xb;
}

// Membership of x in probe (ptr, len) for one lane: a dense-row bit or a
// sorted-list search (no test when len is kSkip: returns true).
__device__ __forceinline__ bool probe_one(const uint32_t* ptr, uint32_t len, uint32_t x) {
    if (len == kSkip) return true;
    if (len == kRowLen) return (ptr[x >> 5] >> (x & 31u)) & 1u;
    return contains(ptr, len, x);
}

// Candidate tests of two elements (xa of window parent ja, xb of jb) against
// level D: injectivity (levels in `inj`), degree thresholds, then each probe
// slot as a dense-row bit test or a sorted-list search.  oka / okb: in =
// element valid, out = element passes.
__device__ __forceinline__ void check_pair(const Ctx& C, const LK& D, uint32_t inj, uint32_t lv, uint32_t ns,
                                           uint32_t ja, uint32_t xa, bool& oka, uint32_t jb, uint32_t xb,
                                           bool& okb) {
    const DevGraph& g = C.a->g;
    for (uint32_t l = 0; l < lv; l++)
        if ((inj >> l) & 1u) {
            oka = oka && (xa != C.s.bound[l * 64 + ja]);
            okb = okb && (xb != C.s.bound[l * 64 + jb]);
        }
    if (D.deg_check) {
        // one byte per node: in degree order the frequent candidates (hubs)
        // share a few cache lines
        const uint32_t da = g.degc[oka ? xa : 0u], db = g.degc[okb ? xb : 0u];
        oka = oka && (da & 15u) >= D.dmin_out && (da >> 4) >= D.dmin_in;
        okb = okb && (db & 15u) >= D.dmin_out && (db >> 4) >= D.dmin_in;
    }
    const uint32_t* safe = safe_ptr(g);
    for (uint32_t k = 0; k < ns; k++) {
        const uint32_t lA = C.s.slot_len[k * 64 + ja], lB = C.s.slot_len[k * 64 + jb];
        const uint32_t* pA = join_ptr(C.s.slot_lo[k * 64 + ja], C.s.slot_hi[k * 64 + ja]);
        const uint32_t* pB = join_ptr(C.s.slot_lo[k * 64 + jb], C.s.slot_hi[k * 64 + jb]);
        const bool rA = oka && lA == kRowLen, rB = okb && lB == kRowLen;
        if (__ballot(rA || rB)) {
            const uint32_t wa = (rA ? pA : safe)[rA ? (xa >> 5) : 0u];
            const uint32_t wb = (rB ? pB : safe)[rB ? (xb >> 5) : 0u];
            if (rA) oka = (wa >> (xa & 31u)) & 1u;
            if (rB) okb = (wb >> (xb & 31u)) & 1u;
        }
        // an empty list holds nothing
        if (lA == 0) oka = false;
        if (lB == 0) okb = false;
        const bool sa = oka && lA < kRowLen, sb = okb && lB < kRowLen;
        if (__ballot(sa || sb)) {
            bool fa, fb;
            search2(sa ? pA : safe, sa ? lA : 0u, xa, fa, sb ? pB : safe, sb ? lB : 0u, xb, fb);
            if (sa) oka = fa;
            if (sb) okb = fb;
        }
    }
}

// Whether bound node y of this lane's partial match lies in the lane's base
// list and passes all its probes: then a flattened pass without injectivity
// counted it once.
__device__ __forceinline__ bool bound_in_set(const Ctx& C, uint32_t ns, uint32_t y) {
    const uint32_t lane = C.lane;
    const uint32_t len = C.s.base_len[lane];
    if (!contains(join_ptr(C.s.base_lo[lane], C.s.base_hi[lane]), len, y)) return false;
    for (uint32_t k = 0; k < ns; k++)
        if (!probe_one(join_ptr(C.s.slot_lo[k * 64 + lane], C.s.slot_hi[k * 64 + lane]),
                       C.s.slot_len[k * 64 + lane], y))
            return false;
    return true;
}

// Expand one window of level lv from the parents in level lv-1.  Returns the
// number of children written to level lv's buffer.
__device__ uint32_t expand(Ctx& C, uint32_t lv) {
    const KArgs& a = *C.a;
    const LK D = load_lk(C.P->lvl[lv], a);
    const uint32_t lane = C.lane;
    uint32_t* st = C.s.st;
    const uint32_t nparents = uni(st[16 + lv - 1]);
    const uint32_t cur = uni(st[lv]);
    const uint32_t pofs = uni(st[8 + lv]);
    const uint32_t p = cur + lane;
    const bool pv = p < nparents;
    uint32_t len = phase_a<false>(C, D, lv, p, pv, true);
    if (pv && lane == 0) len -= pofs;
    uint32_t incl = scan_incl(len, lane);
    C.s.incl[lane] = incl;
    const bool seg = (C.P->seg_src >> lv) & 1u;
    if (seg) C.s.segcnt[lane] = 0;
    const uint32_t cap = a.cap;
    uint32_t np = uni((uint32_t)__popcll(__ballot(pv && incl <= cap)));
    uint32_t T;
    bool partial = false;
    if (np == 0) {
        // the first parent alone exceeds the buffer: take a slice of it
        T = cap;
        partial = true;
        np = 1;
        if (lane == 0) incl = len = cap;
        C.s.incl[0] = cap;
    } else {
        T = uni(__shfl(incl, (int)np - 1, 64));
    }
    // lane j < np owns the elements [incl - len, incl)
    const bool owns = lane < np && len > 0;
    const uint32_t start = incl - len;
    wave_sync();
    Lvl Fo = lvl_arrays(C.scr, cap, lv);
    uint32_t nout = 0, carry = 0;
    const uint32_t ns = n_slots(D);
    // two tiles per step: survivors of tile a are written before those of
    // tile b, so each parent's children stay contiguous and in order
    for (uint32_t t0 = 0; t0 < T; t0 += 128) {
        const uint32_t ga = t0 + lane, gb = t0 + 64 + lane;
        uint32_t ja, jb;
        tile_parents(C.s, lane, t0, start, owns, carry, ja, jb);
        bool oka = ga < T, okb = gb < T;
        uint32_t xa = 0, xb = 0;
        const uint32_t la = ga - (ja ? C.s.incl[ja - 1] : 0u) + (ja == 0 ? pofs : 0u);
        const uint32_t lb = gb - (jb ? C.s.incl[jb - 1] : 0u) + (jb == 0 ? pofs : 0u);
        oka = oka && la < C.s.base_len[ja];
        okb = okb && lb < C.s.base_len[jb];
        if (oka) xa = base_elem(C, ja, la);
        if (okb) xb = base_elem(C, jb, lb);
        check_pair(C, D, D.inj, lv, ns, ja, xa, oka, jb, xb, okb);
        const uint64_t ma = __ballot(oka);
        if (oka) {
            const uint32_t pos = nout + rank_below(ma);
            Fo.node[pos] = xa;
            Fo.parent[pos] = cur + ja;
            if (seg) atomicAdd(&C.s.segcnt[ja], 1u);
        }
        nout += (uint32_t)__popcll(ma);
        const uint64_t mb = __ballot(okb);
        if (okb) {
            const uint32_t pos = nout + rank_below(mb);
            Fo.node[pos] = xb;
            Fo.parent[pos] = cur + jb;
            if (seg) atomicAdd(&C.s.segcnt[jb], 1u);
        }
        nout += (uint32_t)__popcll(mb);
    }
    wave_sync();
    if (seg) {
        // children of each parent are contiguous in output order
        uint32_t cnt = (lane < np) ? C.s.segcnt[lane] : 0;
        uint32_t ex = scan_incl(cnt, lane) - cnt;
        if (lane < np) {
            Lvl Fi = lvl_arrays(C.scr, cap, lv - 1);
            bool complete = !(lane == 0 && (pofs > 0 || partial));
            if (lv == 1) {
                // a root split into first-level sub-ranges never has all its children here
                Lvl F0 = lvl_arrays(C.scr, cap, 0);
                complete = complete && F0.parent[cur + lane] == 0 && F0.aux[cur + lane] == kSkip;
            }
            Fi.segb[cur + lane] = ex;
            Fi.segc[cur + lane] = cnt | (complete ? kComplete : 0u);
        }
    }
    // advance the cursor of this level
    if (lane == 0) {
        if (partial) {
            st[8 + lv] = pofs + cap;
        } else {
            st[lv] = cur + np;
            st[8 + lv] = 0;
        }
        st[16 + lv] = nout;
    }
    wave_sync();
    return nout;
}

// |A intersect B| minus the listed bound nodes, for one partial match, by the
// whole wave: both sorted lists are walked in chunks of kMergeChunk elements
// (A in registers, B staged in LDS); each A element is looked up in the B
// chunk, and the chunk with the smaller maximum advances (both on a tie), so
// every matching pair is seen exactly once.  Reads are coalesced and no
// dependent global search is needed (merge path for balanced list sizes).
__device__ uint32_t merge_count(const Lds& s, const uint32_t* __restrict__ A, uint32_t na,
                                const uint32_t* __restrict__ B, uint32_t nb, uint32_t inj, uint32_t nbound,
                                uint32_t j, uint32_t lane) {
    constexpr uint32_t U = kMergeChunk / 64;
    uint32_t ia = 0, ib = 0, cnt = 0;
    while (ia < na && ib < nb) {
        uint32_t av[U];
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            uint32_t i = ia + u * 64 + lane;
            av[u] = i < na ? A[i] : 0xFFFFFFFFu;
            uint32_t k = ib + u * 64 + lane;
            s.mbuf[u * 64 + lane] = k < nb ? B[k] : 0xFFFFFFFFu;
        }
        const uint32_t alast = (ia + kMergeChunk < na ? ia + kMergeChunk : na) - 1;
        const uint32_t blast = (ib + kMergeChunk < nb ? ib + kMergeChunk : nb) - 1;
        const uint32_t amax = A[alast], bmax = B[blast];
        const uint32_t nbc = blast - ib + 1;
        wave_sync();
#pragma unroll
        for (uint32_t u = 0; u < U; u++) {
            uint32_t x = av[u];
            if (ia + u * 64 + lane < na) {
                uint32_t base = 0, n = nbc;
                while (n > 1) {
                    uint32_t h = n >> 1;
                    base = (s.mbuf[base + h] <= x) ? base + h : base;
                    n -= h;
                }
                bool ok = s.mbuf[base] == x;
                for (uint32_t t = 0; t < nbound; t++)
                    if ((inj >> t) & 1u) ok = ok && (x != s.bound[t * 64 + j]);
                cnt += ok ? 1u : 0u;
            }
        }
        if (amax <= bmax) ia += kMergeChunk;
        if (bmax <= amax) ib += kMergeChunk;
        wave_sync();
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
    return cnt;
}

// Survivors of this step's two tiles that belong to the parent owning the
// elements [start, start + len).
__device__ __forceinline__ uint32_t own_count(uint64_t ballot, uint32_t start, uint32_t len, uint32_t base) {
    const uint32_t lo = start > base ? start : base;
    const uint32_t end = start + len, top = base + 64;
    const uint32_t hi = end < top ? end : top;
    if (hi <= lo) return 0;
    const uint32_t a = lo - base, b = hi - base;
    const uint64_t m = (b == 64 ? ~0ull : ((1ull << b) - 1ull)) & ~((1ull << a) - 1ull);
    return (uint32_t)__popcll(ballot & m);
}

// Leaf group with several signatures: for every signature mask M the terms
// use, h[M] = |intersection over s in M of S_s| is measured per partial match
// (one flattened pass over the shortest list of M's constraints, or list
// length minus bound hits when M has a single constraint list), then the
// inclusion-exclusion terms over set partitions of the leaves are summed in
// 128-bit integers.  The 64 lanes hold the 64 partial matches [w0, w0 + 64).
__device__ void leaf_masks(Ctx& C, uint32_t nb, uint32_t p, bool pv) {
    const KArgs& a = *C.a;
    const PlanDesc* P = C.P;
    const uint32_t lane = C.lane;
    const uint32_t n_masks = uni(P->n_masks);
    for (uint32_t mi = 0; mi < n_masks; mi++) {
        const LK K = load_lk(P->mdesc[mi], a);
        uint32_t h = 0;
        if (K.n_cons == 1 && K.reuse == kNoReuse) {
            // one list L: |L| minus the bound nodes found in L
            if (pv) {
                const DevGraph& g = a.g;
                const uint32_t nd = C.s.bound[K.lvl(0) * 64 + lane];
                const uint32_t* off = off_of(g, K.dir(0));
                const uint32_t o = off[nd], l = off[nd + 1] - o;
                const uint32_t* L = adj_of(g, K.dir(0)) + o;
                h = l;
                for (uint32_t b = 0; b < nb; b++)
                    if (((K.inj >> b) & 1u) && contains(L, l, C.s.bound[b * 64 + lane])) h -= 1;
            }
        } else {
            const uint32_t len = phase_a<true>(C, K, nb, p, pv, false);
            const uint32_t ns = n_slots(K);
            const uint32_t incl = scan_incl(len, lane);
            C.s.incl[lane] = incl;
            const uint32_t T = uni(__shfl(incl, 63, 64));
            const bool owns = len > 0;
            const uint32_t start = incl - len;
            wave_sync();
            uint32_t carry = 0;
            for (uint32_t t0 = 0; t0 < T; t0 += 128) {
                const uint32_t ga = t0 + lane, gb = t0 + 64 + lane;
                uint32_t ja, jb;
                tile_parents(C.s, lane, t0, start, owns, carry, ja, jb);
                const uint32_t la = ga - (ja ? C.s.incl[ja - 1] : 0u);
                const uint32_t lb = gb - (jb ? C.s.incl[jb - 1] : 0u);
                bool oka = ga < T && la < C.s.base_len[ja];
                bool okb = gb < T && lb < C.s.base_len[jb];
                uint32_t xa = 0, xb = 0;
                if (oka) xa = base_elem(C, ja, la);
                if (okb) xb = base_elem(C, jb, lb);
                // injectivity is settled per partial match below
                check_pair(C, K, 0u, nb, ns, ja, xa, oka, jb, xb, okb);
                const uint64_t ba = __ballot(oka), bb = __ballot(okb);
                if (owns) h += own_count(ba, start, len, t0) + own_count(bb, start, len, t0 + 64);
            }
            // the bound nodes the set may not contain were counted if present
            if (pv)
                for (uint32_t b = 0; b < nb; b++)
                    if (((K.inj >> b) & 1u) && bound_in_set(C, ns, C.s.bound[b * 64 + lane])) h -= 1;
            wave_sync();
        }
        // every mask whose test is this entry's takes its size
        for (uint32_t ms = uni(P->mask_set[mi]) & 0xFFFEu; ms; ms &= ms - 1)
            C.s.hist[lane * 16 + (uint32_t)__builtin_ctz(ms)] = h;
    }
    wave_sync();
    if (pv) {
        // inclusion-exclusion over set partitions of the leaves; a term whose
        // magnitude could pass 2^120 marks the plan as overflowed
        const uint32_t* h = C.s.hist + lane * 16;
        __int128 val = 0;
        bool big = false;
        const uint32_t n_terms = uni(P->n_terms);
        for (uint32_t t = 0; t < n_terms; t++) {
            const Term& tm = P->terms[t];
            uint32_t hv[kMaxBlocks];
            const uint32_t nb = tm.nb < kMaxBlocks ? tm.nb : kMaxBlocks;
            for (uint32_t b = 0; b < nb; b++) hv[b] = h[tm.mask[b] & 15u];
            val += ie_term(tm.coef, hv, nb, &big);
        }
        // the injective count of one partial match is never negative
        const unsigned __int128 v = (unsigned __int128)(val < 0 ? (__int128)0 : val);
        if (big || val < 0) C.ovf = true;
        if (u128_add(C.acc_lo, C.acc_hi, (unsigned long long)v, (unsigned long long)(v >> 64))) C.ovf = true;
    }
    wave_sync();
}

// Listing: the survivors of a tile pair are whole embeddings (bound levels
// 0..nb-1 of their parent plus the leaf); one 64-bit atomic per step reserves
// their rows, written in pattern-vertex order while they fit the capacity.
__device__ __forceinline__ void write_rows(const Ctx& C, uint32_t nb, uint64_t ma, uint64_t mb, uint32_t ja,
                                           uint32_t xa, bool oka, uint32_t jb, uint32_t xb, bool okb) {
    const KArgs& a = *C.a;
    const uint32_t na = (uint32_t)__popcll(ma), nbb = (uint32_t)__popcll(mb);
    if (na + nbb == 0) return;
    unsigned long long base = 0;
    if (C.lane == 0) base = atomicAdd(a.list_count, (unsigned long long)(na + nbb));
    base = __shfl(base, 0, 64);
    const PlanDesc* P = C.P;
    const uint32_t k = P->k;
    auto put = [&](unsigned long long row, uint32_t j, uint32_t x) {
        if (row >= a.list_cap) return;
        uint32_t* out = a.list + row * k;
        for (uint32_t l = 0; l < nb; l++) out[P->order[l]] = C.s.bound[l * 64 + j];
        out[P->order[nb]] = x;
    };
    if (oka) put(base + rank_below(ma), ja, xa);
    if (okb) put(base + na + rank_below(mb), jb, xb);
}

// Count the leaf group for every partial match in level `lv` (= e - 1).
template <bool NONLIN>
__device__ void count_leaves(Ctx& C, uint32_t lv, uint32_t nprefix) {
    const KArgs& a = *C.a;
    const PlanDesc* P = C.P;
    const uint32_t lane = C.lane;
    const uint32_t nsig = uni(P->n_sig);
    const bool linear = !NONLIN || P->linear != 0;
    const uint32_t nb = lv + 1;  // bound levels 0..lv
    const LK S0 = load_lk(P->sig[0], a);
    for (uint32_t w0 = 0; w0 < nprefix; w0 += 64) {
        // a leaf pass over hub lists can run long: look at the cancel flag
        // every 8 blocks of 64 prefixes
        if (a.cancel && (++C.polls & 7u) == 0) {
            uint32_t stop = 0;
            if (lane == 0) stop = __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0;
            if (uni(__shfl(stop, 0, 64))) {
                if (lane == 0) atomicOr(&a.ctl[kCtlCancelled], 1u);
                C.stop = true;
                return;
            }
        }
        const uint32_t p = w0 + lane;
        const bool pv = p < nprefix;
        // walk the chain once: bound nodes of levels 0..lv
        if (pv) {
            uint32_t idx = p;
            for (int l = (int)lv; l >= 0; --l) {
                Lvl F = lvl_arrays(C.scr, a.cap, (uint32_t)l);
                C.s.bound[l * 64 + lane] = F.node[idx];
                C.s.anc[l * 64 + lane] = idx;
                if (l > 0) idx = F.parent[idx];
            }
        }
        unsigned long long lin = 0;
        if (!linear) {
            leaf_masks(C, nb, p, pv);
            continue;
        }
        const bool listing = a.list != nullptr;
        if (!listing && S0.n_cons == 1 && S0.reuse == kNoReuse) {
            // one leaf drawn from one list L: |L| minus the bound nodes found in L
            uint32_t v = 0;
            if (pv) {
                const DevGraph& g = a.g;
                uint32_t nd = C.s.bound[S0.lvl(0) * 64 + lane];
                const uint32_t* off = off_of(g, S0.dir(0));
                uint32_t o = off[nd];
                uint32_t l = off[nd + 1] - o;
                const uint32_t* L = adj_of(g, S0.dir(0)) + o;
                if (S0.gt) sym_trim(C.s, S0.gt, S0.lt, nb, lane, L, l);
                v = l;
                for (uint32_t b = 0; b < nb; b++)
                    if (((S0.inj >> b) & 1u) && contains(L, l, C.s.bound[b * 64 + lane])) v -= 1;
            }
            if (u128_add(C.acc_lo, C.acc_hi, v, 0ull)) C.ovf = true;
            wave_sync();
            continue;
        }
        {
            // one leaf signature
            const LK& S = S0;
            uint32_t len = phase_a<true>(C, S, nb, p, pv, false);
            // one leaf whose set is a base list and one probe list: balanced big
            // pairs leave the flattened pass for the cooperative merge
            uint32_t probe_c = kSkip;
            bool big = false;
            const uint32_t ns = n_slots(S);
            if (linear && pv && !listing) {
                uint32_t nprobe = 0;
                for (uint32_t c = 0; c < ns; c++)
                    if (C.s.slot_len[c * 64 + lane] != kSkip) {
                        probe_c = c;
                        nprobe++;
                    }
                if (nprobe == 1 && C.s.slot_len[probe_c * 64 + lane] != kRowLen) {
                    uint32_t pl = C.s.slot_len[probe_c * 64 + lane];
                    uint32_t mn = len < pl ? len : pl, mx = len < pl ? pl : len;
                    big = mn >= a.merge_min && (uint64_t)mx <= (uint64_t)a.merge_ratio * mn;
                }
            }
            uint64_t bigmask = __ballot(big);
            if (big) len = 0;
            (void)nsig;
            const uint32_t incl = scan_incl(len, lane);
            C.s.incl[lane] = incl;
            const uint32_t T = uni(__shfl(incl, 63, 64));
            const bool owns = len > 0;
            const uint32_t start = incl - len;
            wave_sync();
            uint32_t carry = 0;
            // two tiles per step
            for (uint32_t t0 = 0; t0 < T; t0 += 128) {
                const uint32_t ga = t0 + lane, gb = t0 + 64 + lane;
                uint32_t ja, jb;
                tile_parents(C.s, lane, t0, start, owns, carry, ja, jb);
                const uint32_t la = ga - (ja ? C.s.incl[ja - 1] : 0u);
                const uint32_t lb = gb - (jb ? C.s.incl[jb - 1] : 0u);
                bool oka = ga < T && la < C.s.base_len[ja];
                bool okb = gb < T && lb < C.s.base_len[jb];
                uint32_t xa = 0, xb = 0;
                if (oka) xa = base_elem(C, ja, la);
                if (okb) xb = base_elem(C, jb, lb);
                // injectivity is settled per partial match below (per element
                // when every embedding is written out)
                check_pair(C, S, listing ? S.inj : 0u, nb, ns, ja, xa, oka, jb, xb, okb);
                // one leaf: survivors are only counted
                const uint64_t ma = __ballot(oka), mb = __ballot(okb);
                lin += (unsigned long long)(__popcll(ma) + __popcll(mb));
                if (listing) write_rows(C, nb, ma, mb, ja, xa, oka, jb, xb, okb);
            }
            // bound nodes the leaf may not take were counted if they are in the set
            for (uint32_t b = 0; b < nb && !listing; b++) {
                if (!((S.inj >> b) & 1u)) continue;
                const bool hit = pv && !big && bound_in_set(C, ns, C.s.bound[b * 64 + lane]);
                lin -= (unsigned long long)__popcll(__ballot(hit));
            }
            wave_sync();
            // balanced big pairs, one partial match at a time
            while (bigmask) {
                const uint32_t j = (uint32_t)__builtin_ctzll(bigmask);
                bigmask &= bigmask - 1;
                const uint32_t blen = uni(C.s.base_len[j]);
                uint32_t pc = 0;
                for (uint32_t c = 0; c < ns; c++)
                    if (C.s.slot_len[c * 64 + j] != kSkip) pc = c;
                pc = uni(pc);
                const uint32_t plen = uni(C.s.slot_len[pc * 64 + j]);
                const uint32_t* A = join_ptr(uni(C.s.base_lo[j]), uni(C.s.base_hi[j]));
                const uint32_t* B = join_ptr(uni(C.s.slot_lo[pc * 64 + j]), uni(C.s.slot_hi[pc * 64 + j]));
                lin += merge_count(C.s, A, blen, B, plen, S.inj, nb, j, lane);
            }
        }
        if (lane == 0 && u128_add(C.acc_lo, C.acc_hi, lin, 0ull)) C.ovf = true;
        wave_sync();
    }
}

__device__ void flush(Ctx& C) {
    unsigned long long lo = C.acc_lo, hi = C.acc_hi;
    bool ovf = C.ovf;
    // wave reduction of 128-bit partials
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        unsigned long long olo = __shfl_xor(lo, d, 64);
        unsigned long long ohi = __shfl_xor(hi, d, 64);
        if (u128_add(lo, hi, olo, ohi)) ovf = true;
    }
    const bool any_ovf = __ballot(ovf) != 0;
    if (C.lane == 0 && (lo | hi))
        add_u128(C.a->counts + 2 * C.pi, lo, hi, C.a->plan_flags + C.pi);
    if (C.lane == 0 && any_ovf) atomicOr(C.a->plan_flags + C.pi, 1u);
    C.acc_lo = C.acc_hi = 0;
    C.ovf = false;
}

// Work donation.  While some waves are idle (all queues drained), a wave that
// has spent at least kDonateAfter windows in one task (a straggler: most tasks
// take a few windows, and a donated subtree is explored less efficiently than
// in a full window) hands off unstarted partial matches: at the shallowest
// level l >= 2 with at least two parents at level l-1 not yet expanded, the
// last half of them (at most 64) become donated tasks, each carrying its
// prefix phi(v_0..v_{l-1}); the donor drops them from its window.  A donated
// task is explored from level l by another wave.  Slots are reserved with a
// CAS on the tail (never past the capacity) and published with a ready flag.
__device__ void maybe_donate(Ctx& C, uint32_t start, uint32_t lv) {
    const KArgs& a = *C.a;
    uint32_t* st = C.s.st;
    uint32_t idle = 0;
    if (C.lane == 0) idle = __atomic_load_n(&a.ctl[kCtlIdle], __ATOMIC_RELAXED);
    if (uni(__shfl(idle, 0, 64)) == 0) return;
    for (uint32_t l = (start > 2 ? start : 2); l <= lv; l++) {
        const uint32_t n = uni(st[16 + l - 1]);
        uint32_t first = uni(st[l]);
        if (l == lv && uni(st[8 + l]) > 0) first += 1;  // a parent in the middle of a slice stays
        if (first >= n || n - first < 2) continue;
        uint32_t k = (n - first) / 2;
        k = k < 64 ? k : 64;
        // reserve k slots
        uint32_t base = kSkip;
        if (C.lane == 0) {
            uint32_t t = __atomic_load_n(&a.ctl[kCtlDonTail], __ATOMIC_RELAXED);
            while (t + k <= a.don_cap) {
                const uint32_t seen = atomicCAS(&a.ctl[kCtlDonTail], t, t + k);
                if (seen == t) {
                    base = t;
                    break;
                }
                t = seen;
            }
        }
        base = uni(__shfl(base, 0, 64));
        if (base == kSkip) return;  // no room: keep the work
        C.donated = true;
        if (C.lane < k) {
            uint32_t* ent = a.don + (uint64_t)(base + C.lane) * kDonWords;
            uint32_t idx = n - k + C.lane;
            for (int j = (int)l - 1; j >= 0; --j) {
                Lvl F = lvl_arrays(C.scr, a.cap, (uint32_t)j);
                ent[2 + j] = F.node[idx];
                if (j > 0) idx = F.parent[idx];
            }
            ent[0] = C.pi | (l << 16);
            __threadfence();
            __atomic_store_n(&ent[1], 1u, __ATOMIC_RELEASE);
        }
        if (C.lane == 0) st[16 + l - 1] = n - k;
        wave_sync();
        return;
    }
}

// Depth-first exploration of the n0 partial matches held in level start-1
// (start = 1: roots in level 0).
template <bool NONLIN>
__device__ void explore(Ctx& C, uint32_t n0, uint32_t start) {
    const uint32_t e = C.P->e;
    uint32_t* st = C.s.st;
    if (e == 1) {
        count_leaves<NONLIN>(C, 0, n0);
        return;
    }
    if (C.lane == 0) {
        st[16 + start - 1] = n0;
        st[start] = 0;
        st[8 + start] = 0;
    }
    wave_sync();
    uint32_t lv = start;
    uint32_t windows = 0;
    for (;;) {
        uint32_t nparents = uni(st[16 + lv - 1]);
        uint32_t cur = uni(st[lv]);
        if (cur >= nparents) {
            if (lv == start) break;
            lv -= 1;
            continue;
        }
        ++windows;
        // a long task still notices the cancel flag (counts are then partial)
        if (C.a->cancel && (windows & 15u) == 0) {
            uint32_t stop = 0;
            if (C.lane == 0) stop = __atomic_load_n(C.a->cancel, __ATOMIC_RELAXED) != 0;
            if (uni(__shfl(stop, 0, 64))) {
                if (C.lane == 0) atomicOr(&C.a->ctl[kCtlCancelled], 1u);
                break;
            }
        }
        if (windows >= kDonateAfter && (windows & 7u) == 0 && lv >= 2) maybe_donate(C, start, lv);
        uint32_t nout = expand(C, lv);
        if (lv == e - 1) {
            if (nout) count_leaves<NONLIN>(C, lv, nout);
            if (C.stop) break;
        } else if (nout) {
            lv += 1;
            if (C.lane == 0) {
                st[lv] = 0;
                st[8 + lv] = 0;
            }
            wave_sync();
        }
    }
}

// Two register budgets.  MINB resident blocks per CU: 8 (8 waves per SIMD,
// 64 VGPRs, some state spilled to scratch) for launches of more than
// kRoomyBlocksPerCu blocks per CU, and kRoomyBlocksPerCu (3 waves per SIMD,
// the whole kernel in registers) for launches of at most that many.
template <bool NONLIN, int MINB>
__global__ void __launch_bounds__(kBlockThreads, MINB) count_kernel(KArgs a) {
    extern __shared__ uint32_t smem[];
    Ctx C;
    C.a = &a;
    C.lane = lane_id();
    const uint32_t wid = threadIdx.x >> 6;
    C.s = carve(smem + wid * a.lds_words, a.lds_rows, a.maxc, a.merge_min != 0xFFFFFFFFu);
    const uint64_t gw = (uint64_t)blockIdx.x * kWavesPerBlock + wid;
    C.scr = a.scratch + gw * (uint64_t)a.wave_words;
    C.acc_lo = C.acc_hi = 0;
    C.ovf = false;
    C.pi = 0;
    C.P = a.plans;
    C.donated = false;
    C.stop = false;
    C.polls = 0;
    // this wave's home split queue: the XCD its block runs on (blocks go to
    // the 8 XCDs round-robin), so a hub's sub-range tasks share one L2
    const uint32_t home = blockIdx.x % kQueues;
    bool split_left = true;
    // 64-bit: the host keeps the product below 2^32 (root items are 32-bit)
    const uint64_t chunks_per_plan = ((uint64_t)a.n_src + a.chunk - 1) / a.chunk;
    const uint64_t total_chunks = chunks_per_plan * a.n_plans;
    Lvl F0 = lvl_arrays(C.scr, a.cap, 0);
    uint32_t taken = 0;
    // root items (item = chunk index x n_plans + plan) come from kQueues
    // cursors, so the grabs spread over several words and every cursor still
    // walks its items in order; a wave starts at its home cursor (its XCD's)
    // and moves on once one runs dry
    uint32_t rq = home, rtried = 0;
    // a wave counts as active from its first task until the queues run dry
    // (and again while it runs a donated task), not per task
    bool active = true;
    if (C.lane == 0) atomicAdd(&a.ctl[kCtlActive], 1u);
    for (;;) {
        // ---- take a task
        uint32_t kind = 2, item = 0;
        bool stop = false;
        if (C.lane == 0) {
            // the flag may sit in host memory: poll it on every 32nd task only
            if (a.cancel && (taken++ & 31u) == 0 && __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0) {
                atomicOr(&a.ctl[kCtlCancelled], 1u);
                stop = true;
            }
            // split queues: the home queue first, then the others (stealing);
            // the split kernel has finished, so an empty queue stays empty
            if (!stop && split_left) {
                split_left = false;
                for (uint32_t t = 0; t < kQueues; t++) {
                    const uint32_t q = (home + t) % kQueues;
                    const uint32_t qcap = a.qbase[q + 1] - a.qbase[q];
                    uint32_t cnt = __atomic_load_n(&a.ctl[kCtlSplitCount0 + q], __ATOMIC_RELAXED);
                    cnt = cnt < qcap ? cnt : qcap;
                    if (__atomic_load_n(&a.ctl[kCtlSplitHead0 + q], __ATOMIC_RELAXED) >= cnt) continue;
                    const uint32_t it = atomicAdd(&a.ctl[kCtlSplitHead0 + q], 1u);
                    if (it < cnt) {
                        kind = 0;
                        item = a.qbase[q] + it;
                        split_left = true;
                        break;
                    }
                }
            }
            while (!stop && kind == 2 && rtried < kQueues) {
                const uint32_t c = atomicAdd(&a.ctl[kCtlRootCursor0 + 32 * rq], 1u);
                uint64_t it;
                if (a.n_plans > kQueues) {
                    // chunk-major: cursor q walks the chunk indices q, q + kQueues, ...
                    // with all plans of one index in a row, so the plans whose
                    // chunks hold the same roots run on one XCD and share its L2
                    const uint64_t ci = (uint64_t)rq + (uint64_t)kQueues * (c / a.n_plans);
                    it = ci * a.n_plans + c % a.n_plans;
                } else {
                    // plan-major: with few plans, cursor q keeps to the plans q mod
                    // n_plans, so a wave's counts stay in its lanes between tasks
                    it = (uint64_t)rq + (uint64_t)kQueues * c;
                }
                if (it < total_chunks) {
                    kind = 1;
                    item = (uint32_t)it;
                } else {
                    rq = (rq + 1) % kQueues;
                    rtried++;
                }
            }
        }
        if (C.lane == 0 && kind == 2 && active) {
            atomicSub(&a.ctl[kCtlActive], 1u);
            active = false;
        }
        if (C.lane == 0 && kind == 2 && !stop) {
            // queues drained: wait for donated work while any wave still holds a
            // task.  At most kMaxWaiters waves wait (the others leave at once),
            // and they poll with growing pauses, so waiting waves do not crowd
            // the cache lines the working waves update.
            // A wave that donated always waits: a waiter that read the queue
            // just before a donation was published and the active count just
            // after its donor finished would leave without it, and the donor
            // itself then takes its entries (the poll checks the queue first).
            if (atomicAdd(&a.ctl[kCtlIdle], 1u) < kMaxWaiters || C.donated) {
                uint32_t nap = 1;
                for (uint32_t polls = 0; polls < kIdlePolls; polls++) {
                    const uint32_t h = __atomic_load_n(&a.ctl[kCtlDonHead], __ATOMIC_RELAXED);
                    const uint32_t t = __atomic_load_n(&a.ctl[kCtlDonTail], __ATOMIC_RELAXED);
                    if (h < t) {
                        if (atomicCAS(&a.ctl[kCtlDonHead], h, h + 1) == h) {
                            kind = 3;
                            item = h;
                            break;
                        }
                        continue;
                    }
                    if ((polls & 7u) == 7u && __atomic_load_n(&a.ctl[kCtlActive], __ATOMIC_RELAXED) == 0) break;
                    if (a.cancel && (polls & 63u) == 0 && __atomic_load_n(a.cancel, __ATOMIC_RELAXED) != 0) break;
                    for (uint32_t z = 0; z < nap; z++) __builtin_amdgcn_s_sleep(64);  // ~4K cycles each
                    nap = nap < 16 ? nap * 2 : 16;
                }
            }
            atomicSub(&a.ctl[kCtlIdle], 1u);
        }
        if (C.lane == 0 && kind == 3) {
            atomicAdd(&a.ctl[kCtlActive], 1u);
            active = true;
        }
        kind = uni(__shfl(kind, 0, 64));
        item = uni(__shfl(item, 0, 64));
        if (kind == 2) break;
        uint32_t n0 = 0, start = 1;
        // counts of consecutive tasks of one plan stay in the lanes'
        // accumulators: flush only when the plan changes (and at the end)
        auto set_plan = [&](uint32_t pi) {
            if (pi != C.pi) {
                flush(C);
                C.pi = pi;
            }
            C.P = a.plans + C.pi;
        };
        if (kind == 0) {
            uint4 it = a.split_items[item];
            set_plan(uni(it.x));
            if (C.lane == 0) {
                F0.node[0] = it.y;
                F0.parent[0] = it.z;
                F0.aux[0] = it.w;
            }
            n0 = 1;
        } else if (kind == 3) {
            // a donated prefix: bind levels 0..d-1 as single entries and explore from level d
            uint32_t* ent = a.don + (uint64_t)item * kDonWords;
            uint32_t ready = 0;
            if (C.lane == 0) {
                for (uint32_t spin = 0; spin < kIdlePolls; spin++) {
                    ready = __atomic_load_n(&ent[1], __ATOMIC_ACQUIRE);
                    if (ready) break;
                    __builtin_amdgcn_s_sleep(1);
                }
                if (!ready) atomicOr(&a.ctl[kCtlBadPlan], 1u);  // a reserved slot never published
            }
            ready = uni(__shfl(ready, 0, 64));
            __atomic_thread_fence(__ATOMIC_ACQUIRE);  // every lane reads the entry after its ready flag
            const uint32_t head = ready ? uni(__atomic_load_n(&ent[0], __ATOMIC_RELAXED)) : (1u << 16);
            set_plan(head & 0xFFFFu);
            start = head >> 16;
            if (ready && C.lane < start) {
                Lvl F = lvl_arrays(C.scr, a.cap, C.lane);
                F.node[0] = __atomic_load_n(&ent[2 + C.lane], __ATOMIC_RELAXED);
                F.parent[0] = 0;
                F.segc[0] = 0;  // no complete child segments: reusers fetch their lists
                F.aux[0] = kSkip;
            }
            n0 = ready ? 1u : 0u;
        } else {
            // interleave plans so that all of them start on the low (hub) ids
            set_plan(uni(item % a.n_plans));
            const uint32_t ci = item / a.n_plans;
            // without a root list, a plan on a root share counts the ids
            // (j + 1) 2^s - 1 only: its chunks run over j, so that every lane
            // of a chunk gets a root of the share (n >> s of them)
            const uint32_t sh = C.P->root_share;
            const bool compact = a.roots == nullptr && sh > 0;
            const uint64_t n_p = compact ? ((uint64_t)a.n_src >> sh) : (uint64_t)a.n_src;
            const uint64_t cpp = compact ? (n_p + a.chunk - 1) / a.chunk : chunks_per_plan;
            // chunk ci takes the roots ci, ci + chunks, ci + 2 chunks, ...: long
            // lists cluster at low ids on power-law generators, and striding
            // spreads them over many tasks
            const uint64_t idx64 = (uint64_t)ci + (uint64_t)C.lane * cpp;
            const uint32_t idx = (uint32_t)(idx64 < n_p ? idx64 : n_p);
            bool ok = C.lane < a.chunk && ci < cpp && idx64 < n_p;
            uint32_t r = 0;
            if (ok) {
                r = compact ? (uint32_t)(((idx64 + 1) << sh) - 1) : (a.roots ? a.roots[idx] : idx);
                ok = r < a.g.n && in_root_share(r, sh);
            }
            if (ok) {
                uint2 d = a.g.deg[r];
                ok = d.x >= C.P->root_dout && d.y >= C.P->root_din;
            }
            if (ok && C.P->e >= 2) {
                uint32_t l = level1_len(a.g, C.P, r);
                // longer lists were queued as sub-ranges by the split kernel
                ok = l > 0 && l <= plan_item_size(l, C.P->e, a.split, a.split_work, a.cap);
            }
            uint64_t m = __ballot(ok);
            if (ok) {
                uint32_t pos = rank_below(m);
                F0.node[pos] = r;
                F0.parent[pos] = 0;
                F0.aux[pos] = kSkip;
            }
            n0 = (uint32_t)__popcll(m);
        }
        wave_sync();
        if (n0) explore<NONLIN>(C, n0, start);
        if (C.stop) break;
    }
    // a wave that was counted as active must not stay so after a cancel
    if (C.lane == 0 && C.stop && active) atomicSub(&a.ctl[kCtlActive], 1u);
    flush(C);
}

// Hub roots whose first-level list is longer than `split` become several
// queued sub-range tasks.  Must agree with the root filter of count_kernel.
__global__ void split_kernel(KArgs a) {
    const uint32_t nsrc = a.roots ? a.n_src : a.n_hubs;
    const uint64_t total = (uint64_t)nsrc * a.n_plans;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        // root-major: the tasks of all plans on one hub are pushed together,
        // so the waves of its XCD work on that hub's lists side by side
        const uint32_t pi = (uint32_t)(i % a.n_plans);
        const uint32_t h = (uint32_t)(i / a.n_plans);
        const PlanDesc* P = a.plans + pi;
        if (P->e < 2) continue;
        uint32_t r = a.roots ? a.roots[h] : a.hubs[h];
        if (r >= a.g.n || !in_root_share(r, P->root_share)) continue;
        uint2 d = a.g.deg[r];
        if (d.x < P->root_dout || d.y < P->root_din) continue;
        uint32_t len = level1_len(a.g, P, r);
        const uint32_t sz = plan_item_size(len, P->e, a.split, a.split_work, a.cap);
        if (len <= sz) continue;
        uint32_t nit = (len + sz - 1) / sz;
        // all tasks of one root go to one queue (one XCD's L2)
        const uint32_t qu = h % kQueues;
        const uint32_t qcap = a.qbase[qu + 1] - a.qbase[qu];
        uint32_t base = atomicAdd(&a.ctl[kCtlSplitCount0 + qu], nit);
        if (base + nit > qcap) {
            atomicOr(&a.ctl[kCtlQueueFull], 1u);
            continue;
        }
        for (uint32_t q = 0; q < nit; q++) {
            uint32_t lo = q * sz;
            uint32_t hi = lo + sz < len ? lo + sz : len;
            a.split_items[a.qbase[qu] + base + q] = make_uint4(pi, r, lo, hi);
        }
    }
}

// Copy plan descriptors into the workspace table and clear control state.
__global__ void init_kernel(InitArgs a) {
    const uint32_t words = sizeof(PlanDesc) / 4;
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t nthr = gridDim.x * blockDim.x;
    for (uint32_t i = tid; i < a.count * words; i += nthr) {
        uint32_t pl = i / words, w = i % words;
        reinterpret_cast<uint32_t*>(a.table + a.first + pl)[w] =
            reinterpret_cast<const uint32_t*>(a.src[pl])[w];
    }
    if (a.zero_ctl) {
        for (uint32_t i = tid; i < kCtlWords; i += nthr) a.ctl[i] = 0;
        for (uint32_t i = tid; i < a.n_plans; i += nthr) a.plan_flags[i] = 0;
        for (uint32_t i = tid; i < 2 * a.n_plans; i += nthr) a.counts[i] = 0;
        // the workspace is reused across launches (and by the caller's
        // allocator): a slot is ready only once this launch publishes it
        for (uint32_t i = tid; i < a.don_cap; i += nthr) a.don[(uint64_t)i * kDonWords + 1] = 0;
        if (a.list_count && tid == 0) *a.list_count = 0;
    }
}

// Per-plan status from the flags the count kernel raised.
__global__ void finalize_kernel(KArgs a) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n_plans; i += gridDim.x * blockDim.x) {
        int32_t st = 0;
        if (a.ctl[kCtlBadPlan]) st = -1;
        else if (a.ctl[kCtlQueueFull]) st = -6;
        else if (a.ctl[kCtlCancelled]) st = -7;
        else if (a.plan_flags[i] & 1u) st = -5;
        const uint32_t m = a.plans[i].sym_mult;
        if (m > 1 && st == 0) {
            // one embedding per orbit was counted: scale the 128-bit total
            unsigned long long* c = a.counts + 2 * i;
            unsigned long long lo = c[0], hi = c[1];
            if (u128_scale(lo, hi, m)) st = -5;
            c[0] = lo;
            c[1] = hi;
        }
        a.status[i] = st;
    }
}

// Workspace of xm_count_static: a fixed array in device memory, one copy per
// device, so that launches need no allocation.  Host code never uses this
// name as an address: the address comes from hipGetSymbolAddress.
static __device__ __align__(256) uint8_t g_static_scratch[kStaticScratchBytes];

hipError_t static_scratch_address(void** ptr) {
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(g_static_scratch));
}

__global__ void desc_chunk_kernel(DescChunk c) {
    for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) c.dst[i] = c.w[i];
}

hipError_t copy_desc(PlanDesc* dst, const PlanDesc& src, hipStream_t stream) {
    const uint32_t words = sizeof(PlanDesc) / 4;
    const uint32_t* s = reinterpret_cast<const uint32_t*>(&src);
    for (uint32_t o = 0; o < words; o += kDescChunkWords) {
        DescChunk c;
        c.dst = reinterpret_cast<uint32_t*>(dst) + o;
        c.n = words - o < kDescChunkWords ? words - o : kDescChunkWords;
        for (uint32_t i = 0; i < c.n; i++) c.w[i] = s[o + i];
        hipLaunchKernelGGL(desc_chunk_kernel, dim3(1), dim3(256), 0, stream, c);
    }
    return hipGetLastError();
}

int count_blocks_per_cu(bool nonlin, size_t lds_bytes) {
    int nb = 0;
    hipError_t e;
    if (nonlin)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, count_kernel<true, 8>, kBlockThreads, lds_bytes);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, count_kernel<false, 8>, kBlockThreads, lds_bytes);
    return e == hipSuccess ? nb : 0;
}

// One block per dense row: set the bit of every list element.
__global__ void rows_kernel(DevGraph g, const uint32_t* row_node, uint32_t n_out_rows, uint32_t n_rows,
                            uint32_t* rows) {
    for (uint32_t r = blockIdx.x; r < n_rows; r += gridDim.x) {
        const uint32_t dir = r >= n_out_rows ? 1u : 0u;
        const uint32_t v = row_node[r];
        const uint32_t* off = off_of(g, dir);
        const uint32_t* adj = adj_of(g, dir);
        uint32_t* row = rows + (uint64_t)r * g.row_words;
        for (uint32_t i = off[v] + threadIdx.x; i < off[v + 1]; i += blockDim.x) {
            const uint32_t x = adj[i];
            atomicOr(&row[x >> 5], 1u << (x & 31u));
        }
    }
}

hipError_t build_rows(const DevGraph& g, const uint32_t* row_node, uint32_t n_out_rows, uint32_t n_rows,
                      uint32_t* rows, hipStream_t stream) {
    if (n_rows == 0) return hipSuccess;
    uint32_t blocks = n_rows < 65535u ? n_rows : 65535u;
    hipLaunchKernelGGL(rows_kernel, dim3(blocks), dim3(256), 0, stream, g, row_node, n_out_rows, n_rows, rows);
    return hipGetLastError();
}

hipError_t launch_count(const InitArgs* inits, int n_inits, const KArgs& a, uint32_t n_blocks,
                        hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_stop) {
    for (int i = 0; i < n_inits; i++) {
        hipLaunchKernelGGL(init_kernel, dim3(64), dim3(256), 0, stream, inits[i]);
    }
    uint32_t nsrc = a.roots ? a.n_src : a.n_hubs;
    uint64_t total = (uint64_t)nsrc * a.n_plans;
    uint32_t sb = (uint32_t)((total + 255) / 256);
    sb = sb < 1 ? 1 : (sb > 4096 ? 4096 : sb);
    hipLaunchKernelGGL(split_kernel, dim3(sb), dim3(256), 0, stream, a);
    size_t lds = (size_t)a.lds_words * 4 * kWavesPerBlock;
    if (ev_start) {
        hipError_t e = hipEventRecord(ev_start, stream);
        if (e != hipSuccess) return e;
    }
    // the whole kernel in registers when the launch asks for few enough waves
    const bool roomy = n_blocks <= (uint64_t)a.n_cu * kRoomyBlocksPerCu;
    if (a.nonlinear && roomy)
        hipLaunchKernelGGL((count_kernel<true, kRoomyBlocksPerCu>), dim3(n_blocks), dim3(kBlockThreads), lds, stream, a);
    else if (a.nonlinear)
        hipLaunchKernelGGL((count_kernel<true, 8>), dim3(n_blocks), dim3(kBlockThreads), lds, stream, a);
    else if (roomy)
        hipLaunchKernelGGL((count_kernel<false, kRoomyBlocksPerCu>), dim3(n_blocks), dim3(kBlockThreads), lds, stream, a);
    else
        hipLaunchKernelGGL((count_kernel<false, 8>), dim3(n_blocks), dim3(kBlockThreads), lds, stream, a);
    if (ev_stop) {
        hipError_t e = hipEventRecord(ev_stop, stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(256), 0, stream, a);
    return hipGetLastError();
}

}  // namespace xm
