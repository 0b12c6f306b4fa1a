// runtime.cpp — the C ABI (include/xminer.h): graph residency, planning,
// workspace layout and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <atomic>
#include <functional>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/xminer.h"
#include "kernels.h"
#include "planner.h"

using xm::PlanDesc;

static_assert(xm::kStaticScratchBytes == XM_STATIC_SCRATCH_BYTES, "static scratch size differs from the header's");

struct xm_graph_s {
    int device = 0;
    uint32_t n = 0, m = 0;
    const uint32_t *out_off = nullptr, *out_adj = nullptr, *in_off = nullptr, *in_adj = nullptr;
    bool owns_csr = false;
    uint2* deg = nullptr;         // device, owned
    uint8_t* degc = nullptr;      // device, owned: per node min(out, 15) | min(in, 15) << 4
    uint32_t* hubs = nullptr;     // device, owned
    uint32_t n_hubs = 0;
    std::vector<uint32_t> hub_len;  // host: longest list of each hub (queue sizing)
    std::vector<uint2> hub_deg;     // host: (out, in) degree of each hub
    std::vector<uint32_t> hub_id;   // host: node id of each hub
    uint32_t max_out = 0, max_in = 0;
    std::vector<uint2> hdeg;        // host: (out, in) degree per node
    std::vector<uint32_t> new_of_old;  // XM_ORDER_BY_DEGREE: the renumbering (empty: none)
    // dense membership rows of long lists (xm_graph_dense_rows)
    uint32_t* rows = nullptr;       // device, owned: out rows, then in rows
    uint2* row_of = nullptr;        // device, owned: per node (out row, in row)
    uint32_t row_min = xm::kNoRows, n_rows_out = 0, n_rows_in = 0;
    uint64_t row_words = 0;
    mutable std::atomic<int> execs{0};  // captured launches that hold this graph's pointers
    int n_cu = 0;
    size_t max_lds_block = 65536;
    xm::GraphStats stats;
};

struct xm_plan_s {
    PlanDesc desc;
    std::string json;
    std::mutex mu;
    std::vector<void*> dev;  // per device copy of desc (lazy)
};

struct xm_exec_s {
    const xm_graph_s* g = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return XM_ERR_HIP;
}

#define HIP_TRY(call, what)                         \
    do {                                            \
        hipError_t _e = (call);                     \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

// Device copy of a plan's descriptor (uploaded once per device).
int plan_device_desc(xm_plan_t* p, int dev, const PlanDesc** out) {
    std::lock_guard<std::mutex> lk(p->mu);
    if ((int)p->dev.size() <= dev) p->dev.resize(dev + 1, nullptr);
    if (!p->dev[dev]) {
        void* d = nullptr;
        HIP_TRY(hipMalloc(&d, sizeof(PlanDesc)), "hipMalloc(plan)");
        hipError_t e = hipMemcpy(d, &p->desc, sizeof(PlanDesc), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            return hip_fail(e, "hipMemcpy(plan)");
        }
        p->dev[dev] = d;
    }
    *out = static_cast<const PlanDesc*>(p->dev[dev]);
    return XM_OK;
}

struct Layout {
    uint32_t chunk, split, split_work, cap, waves_per_cu, n_waves, n_blocks, e_max, maxc, merge_min, don_cap;
    bool nonlinear;
    size_t off_ctl, off_flags, off_table, off_split, off_don, off_scratch, total;
    uint32_t split_cap, wave_words, lds_words;
    uint32_t qbase[xm::kQueues + 1];
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

constexpr uint64_t kMaxQueueBytes = 2ull << 30;  // split task queue, at most
constexpr uint64_t kMaxRootItems = 0xFFFFFFFFull - 64;  // root items per launch (32-bit item ids)

// Defaults of launches on the static scratch array (xm_count_static): fewer
// resident waves and smaller level windows, so that the workspace of most
// launches fits the array.
constexpr uint32_t kStaticCap = 256, kStaticWavesPerCu = 4;

int make_layout(const xm_graph_t* g, uint32_t n_plans, const xm_plan_t* const* plans,
                const xm_count_opts* o, Layout& L, bool on_static = false) {
    if (!g) return fail(XM_ERR_INVALID, "graph is NULL");
    if (n_plans == 0 || !plans) return fail(XM_ERR_INVALID, "no plans");
    if (n_plans > 65535) return fail(XM_ERR_INVALID, "at most 65535 plans per launch");
    // struct_size: 0 or at least the layout before roots_host (fields added
    // later are read only when struct_size covers them)
    if (o && o->struct_size != 0 && o->struct_size < offsetof(xm_count_opts, roots_host))
        return fail(XM_ERR_INVALID, "xm_count_opts.struct_size too small");
    const bool full_opts = o && (o->struct_size == 0 || o->struct_size >= sizeof(xm_count_opts));
    const uint32_t* roots_host =
        (o && o->roots_dev && (o->struct_size == 0 || o->struct_size >= offsetof(xm_count_opts, list_dev)))
            ? o->roots_host
            : nullptr;
    if (full_opts && o->list_dev) {
        if (n_plans != 1) return fail(XM_ERR_INVALID, "listing needs exactly one plan");
        if (!plans[0] || plans[0]->desc.t != 1)
            return fail(XM_ERR_INVALID, "listing needs a plan whose leaf group is one vertex (e.g. unreduced)");
        if (!o->list_count_dev) return fail(XM_ERR_INVALID, "listing needs list_count_dev");
    }
    L.chunk = (o && o->chunk) ? o->chunk : 0;  // 0: sized below from the task count
    L.split = (o && o->split) ? o->split : 64;
    L.split_work = (o && o->split_work) ? o->split_work : 4096;
    L.cap = (o && o->cap) ? o->cap : (on_static ? kStaticCap : 4096);
    L.waves_per_cu = (o && o->waves_per_cu) ? o->waves_per_cu : (on_static ? kStaticWavesPerCu : 0);  // 0: from occupancy
    L.don_cap = on_static ? xm::kDonCapStatic : xm::kDonCap;
    if (L.chunk > 64) return fail(XM_ERR_INVALID, "chunk must be <= 64");
    if (L.split < xm::kHubMin) return fail(XM_ERR_INVALID, "split must be >= 64");
    if (L.split_work < xm::kHubMin * xm::kHubMin) return fail(XM_ERR_INVALID, "split_work must be >= 4096");
    if (on_static && !(o && o->split) && L.cap < L.split) L.split = L.cap;
    if (L.cap < L.split || L.cap < 64) return fail(XM_ERR_INVALID, "cap must be >= split and >= 64");
    if (L.cap > (1u << 24)) return fail(XM_ERR_INVALID, "cap too large");
    if (L.waves_per_cu != 0 && (L.waves_per_cu < 4 || L.waves_per_cu > 32))
        return fail(XM_ERR_INVALID, "waves_per_cu must be in 4..32");
    uint32_t max_list = std::max(g->max_out, g->max_in);
    if ((uint64_t)max_list * 64 >= (1ull << 32))
        return fail(XM_ERR_INVALID, "adjacency lists too long for 32-bit window offsets");
    L.e_max = 1;
    L.maxc = 1;
    L.nonlinear = false;
    uint32_t splittable = 0;
    for (uint32_t i = 0; i < n_plans; i++) {
        if (!plans[i]) return fail(XM_ERR_INVALID, "plan is NULL");
        const PlanDesc& D = plans[i]->desc;
        L.e_max = std::max(L.e_max, D.e);
        for (uint32_t l = 1; l < D.e; l++) L.maxc = std::max<uint32_t>(L.maxc, D.lvl[l].n_cons);
        for (uint32_t s = 0; s < D.n_sig; s++) L.maxc = std::max<uint32_t>(L.maxc, D.sig[s].n_cons);
        // a signature mask unites the constraints of several signatures
        for (uint32_t i = 0; i < D.n_masks; i++) L.maxc = std::max<uint32_t>(L.maxc, D.mdesc[i].n_cons);
        if (!D.linear) L.nonlinear = true;
        if (D.e >= 2) splittable++;
        // a symmetry-broken plan counts one embedding per orbit: neither the
        // embeddings of a root subset nor a listing can be read from it
        if (!g->new_of_old.empty() && o && o->roots_dev)
            return fail(XM_ERR_INVALID, "root subsets need a graph loaded without XM_ORDER_BY_DEGREE");
        if (!g->new_of_old.empty() && full_opts && o->list_dev)
            return fail(XM_ERR_INVALID, "listing needs a graph loaded without XM_ORDER_BY_DEGREE");
        if (D.sym_mult > 1 && !D.sym_fixes_root && o && o->roots_dev)
            return fail(XM_ERR_INVALID,
                        "root subsets need plans without XM_PLAN_SYMMETRY or with a forced start vertex");
        if (D.sym_mult > 1 && full_opts && o->list_dev)
            return fail(XM_ERR_INVALID, "listing needs a plan without XM_PLAN_SYMMETRY");
    }
    L.merge_min = (o && o->merge_min) ? o->merge_min : xm::kMergeMin;
    L.lds_words = xm::lds_words_for(L.e_max, L.maxc, L.nonlinear, L.merge_min != 0xFFFFFFFFu);
    if (L.waves_per_cu == 0) {
        // as many waves as can be resident at once: the kernel is persistent.
        // When LDS leaves room for fewer than 6 blocks of the 64-VGPR kernel,
        // its extra occupancy does not pay for its spills: take the kernel
        // that keeps everything in registers at its kRoomyBlocksPerCu blocks
        // (measured: 256 plans on R-MAT 22 1,340 ms at 3 blocks against
        // 1,374 ms at 4; TT4 + pendant on R-MAT 20 2,199 ms against 2,787 ms)
        int bpc = xm::count_blocks_per_cu(L.nonlinear, (size_t)L.lds_words * 4 * xm::kWavesPerBlock);
        if (bpc < 6) bpc = std::min(bpc, xm::kRoomyBlocksPerCu);
        L.waves_per_cu = (uint32_t)std::max(1, std::min(bpc, 8)) * xm::kWavesPerBlock;
    }
    L.n_waves = (uint32_t)g->n_cu * L.waves_per_cu;
    L.n_waves = (L.n_waves + xm::kWavesPerBlock - 1) / xm::kWavesPerBlock * xm::kWavesPerBlock;
    L.n_blocks = L.n_waves / xm::kWavesPerBlock;
    if (L.chunk == 0) {
        // about 64 root tasks per wave: one root per task on small batches,
        // up to 64 roots per task when plans x roots is large (each task has a
        // fixed cost: a queue grab, the root filter, a flush)
        const uint64_t n_src = (o && o->roots_dev) ? o->n_roots : g->n;
        const uint64_t per = (uint64_t)L.n_waves * 64;
        L.chunk = (uint32_t)std::min<uint64_t>(64, std::max<uint64_t>(1, (n_src * n_plans + per - 1) / per));
    }
    {
        // root items (plan, chunk) are numbered in 32 bits
        const uint64_t n_src = (o && o->roots_dev) ? o->n_roots : g->n;
        const uint64_t items = (n_src + L.chunk - 1) / L.chunk * n_plans;
        if (items > kMaxRootItems)
            return fail(XM_ERR_INVALID, "too many root items (roots x plans / chunk >= 2^32); raise chunk");
    }
    if ((size_t)L.lds_words * 4 * xm::kWavesPerBlock > g->max_lds_block)
        return fail(XM_ERR_INVALID, "plans need more LDS than a workgroup may use");
    // split task queue capacity
    uint64_t items = 0;
    // Exact count of sub-range tasks the split kernel will emit: per plan and
    // hub, the root filter and the first-level list length (the shortest list
    // of the level-1 constraints).  When the queue would pass kMaxQueueBytes
    // the task size target split_work doubles for this launch.
    auto pieces = [&](uint32_t len, uint32_t sw, uint32_t e) -> uint64_t {
        uint32_t sz = xm::plan_item_size(len, e, L.split, sw, L.cap);
        return len > sz ? (len + sz - 1) / sz : 0;
    };
    // per queue: a root's tasks go to queue (its index in the hub list or
    // the subset) mod kQueues
    uint64_t qc[xm::kQueues];
    auto count_items = [&](uint32_t sw) -> uint64_t {
        uint64_t tot = 0;
        for (uint32_t q = 0; q < xm::kQueues; q++) qc[q] = 0;
        if (o && o->roots_dev && roots_host) {
            // exact, from the subset's degrees
            for (uint32_t i = 0; i < n_plans; i++) {
                const PlanDesc& D = plans[i]->desc;
                if (D.e < 2) continue;
                for (uint32_t k = 0; k < o->n_roots; k++) {
                    const uint32_t r = roots_host[k];
                    if (r >= g->n) continue;
                    const uint2 d = g->hdeg[r];
                    if (std::max(d.x, d.y) <= xm::kHubMin) continue;  // the split kernel's cut
                    if (d.x < D.root_dout || d.y < D.root_din) continue;
                    if (!xm::in_root_share(r, D.root_share)) continue;
                    uint32_t L1 = 0xFFFFFFFFu;
                    for (int c = 0; c < D.lvl[1].n_cons; c++) L1 = std::min(L1, D.lvl[1].cons_dir[c] ? d.y : d.x);
                    const uint64_t pc = pieces(L1, sw, D.e);
                    tot += pc;
                    qc[k % xm::kQueues] += pc;
                }
            }
            return tot;
        }
        if (o && o->roots_dev) {  // subset degrees are not known on the host: bound them
            // the smaller sub-ranges (deeper plans) bound every plan's count
            const uint64_t per = pieces(max_list, sw, 3) * splittable;
            for (uint32_t q = 0; q < xm::kQueues; q++)
                qc[q] = (o->n_roots > q ? ((uint64_t)o->n_roots - q + xm::kQueues - 1) / xm::kQueues : 0) * per;
            return (uint64_t)o->n_roots * per;
        }
        for (uint32_t i = 0; i < n_plans; i++) {
            const PlanDesc& D = plans[i]->desc;
            if (D.e < 2) continue;
            for (size_t h = 0; h < g->hub_deg.size(); h++) {
                uint2 d = g->hub_deg[h];
                if (d.x < D.root_dout || d.y < D.root_din) continue;
                if (!xm::in_root_share(g->hub_id[h], D.root_share)) continue;
                uint32_t L1 = 0xFFFFFFFFu;
                for (int c = 0; c < D.lvl[1].n_cons; c++) L1 = std::min(L1, D.lvl[1].cons_dir[c] ? d.y : d.x);
                const uint64_t pc = pieces(L1, sw, D.e);
                tot += pc;
                qc[h % xm::kQueues] += pc;
            }
        }
        return tot;
    };
    items = count_items(L.split_work);
    while (items * 16 > kMaxQueueBytes && L.split_work < (1u << 30)) {
        L.split_work *= 2;
        items = count_items(L.split_work);
    }
    if (items > 0xFFFFFFF0ull) return fail(XM_ERR_INVALID, "split queue too large; raise split_work");
    L.split_cap = (uint32_t)std::max<uint64_t>(items, 1);
    L.qbase[0] = 0;
    for (uint32_t q = 0; q < xm::kQueues; q++) L.qbase[q + 1] = L.qbase[q] + (uint32_t)qc[q];
    L.wave_words = L.e_max * xm::kLvlArrays * L.cap;
    size_t off = 0;
    L.off_ctl = off;
    off = align256(off + xm::kCtlWords * 4);
    L.off_flags = off;
    off = align256(off + (size_t)n_plans * 4);
    L.off_table = off;
    off = align256(off + (size_t)n_plans * sizeof(PlanDesc));
    L.off_split = off;
    off = align256(off + (size_t)L.split_cap * 16);
    L.off_don = off;
    off = align256(off + (size_t)L.don_cap * xm::kDonWords * 4);
    L.off_scratch = off;
    off = align256(off + (size_t)L.n_waves * L.wave_words * 4);
    L.total = off;
    return XM_OK;
}

// Device address of the static scratch array on the current device, looked
// up once per device (each device holds its own copy).
int static_scratch(int dev, void** out) {
    static std::mutex mu;
    static std::vector<void*> addr;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
    if (!addr[dev]) {
        void* p = nullptr;
        HIP_TRY(xm::static_scratch_address(&p), "hipGetSymbolAddress(static scratch)");
        if (!p) return fail(XM_ERR_HIP, "hipGetSymbolAddress(static scratch) returned NULL");
        addr[dev] = p;
    }
    *out = addr[dev];
    return XM_OK;
}

int enqueue_count(const xm_graph_t* g, uint32_t n_plans, const xm_plan_t* const* plans,
                  const xm_count_opts* o, void* ws, size_t ws_bytes, uint64_t* counts,
                  int32_t* status, hipStream_t stream, bool on_static = false) {
    Layout L;
    int rc = make_layout(g, n_plans, plans, o, L, on_static);
    if (rc) return rc;
    if (on_static) {
        if (L.total > xm::kStaticScratchBytes)
            return fail(XM_ERR_WORKSPACE, "launch needs " + std::to_string(L.total) +
                                              " bytes of workspace, more than the static scratch array holds (" +
                                              std::to_string(xm::kStaticScratchBytes) +
                                              "); lower cap or waves_per_cu, or use xm_count");
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
        rc = static_scratch(dev, &ws);
        if (rc) return rc;
        ws_bytes = xm::kStaticScratchBytes;
    }
    if (!ws || ws_bytes < L.total) return fail(XM_ERR_WORKSPACE, "workspace missing or too small");
    if (!counts || !status) return fail(XM_ERR_INVALID, "counts/status buffers are NULL");
    if (o && o->flags != 0) return fail(XM_ERR_INVALID, "unknown xm_count_opts flag");
    if (o && o->roots_dev && o->n_roots == 0) return fail(XM_ERR_INVALID, "empty root subset");
    int cur_dev = 0;
    HIP_TRY(hipGetDevice(&cur_dev), "hipGetDevice");
    if (cur_dev != g->device) return fail(XM_ERR_INVALID, "current device differs from the graph's");
    char* base = static_cast<char*>(ws);
    xm::KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g.out_off = g->out_off;
    a.g.out_adj = g->out_adj;
    a.g.in_off = g->in_off;
    a.g.in_adj = g->in_adj;
    a.g.deg = g->deg;
    a.g.degc = g->degc;
    a.g.n = g->n;
    a.g.row_min = g->rows ? g->row_min : xm::kNoRows;
    a.g.rows = g->rows;
    a.g.row_of = g->row_of;
    a.g.row_words = (uint32_t)g->row_words;
    a.plans = reinterpret_cast<const PlanDesc*>(base + L.off_table);
    a.n_plans = n_plans;
    a.chunk = L.chunk;
    a.split = L.split;
    a.split_work = L.split_work;
    a.cap = L.cap;
    a.ctl = reinterpret_cast<uint32_t*>(base + L.off_ctl);
    a.plan_flags = reinterpret_cast<uint32_t*>(base + L.off_flags);
    a.split_items = reinterpret_cast<uint4*>(base + L.off_split);
    a.split_cap = L.split_cap;
    a.don = reinterpret_cast<uint32_t*>(base + L.off_don);
    a.don_cap = L.don_cap;
    for (uint32_t q = 0; q <= xm::kQueues; q++) a.qbase[q] = L.qbase[q];
    a.roots = (o && o->roots_dev) ? o->roots_dev : nullptr;
    a.n_src = a.roots ? o->n_roots : g->n;
    a.hubs = g->hubs;
    a.n_hubs = g->n_hubs;
    a.lds_words = L.lds_words;
    a.lds_rows = L.e_max;
    a.maxc = L.maxc;
    a.merge_min = L.merge_min;
    a.merge_ratio = (o && o->merge_ratio) ? o->merge_ratio : xm::kMergeRatio;
    a.nonlinear = L.nonlinear ? 1u : 0u;
    a.n_cu = (uint32_t)g->n_cu;
    a.wave_words = L.wave_words;
    a.scratch = reinterpret_cast<uint32_t*>(base + L.off_scratch);
    a.counts = reinterpret_cast<unsigned long long*>(counts);
    a.status = status;
    a.cancel = o ? o->cancel_dev : nullptr;
    const bool listing = o && (o->struct_size == 0 || o->struct_size >= sizeof(xm_count_opts)) && o->list_dev;
    a.list = listing ? o->list_dev : nullptr;
    a.list_count = listing ? o->list_count_dev : nullptr;
    a.list_cap = listing ? o->list_cap : 0;

    std::vector<xm::InitArgs> inits;
    if (on_static) {
        // descriptors travel in kernel arguments: no device copy of a plan is
        // allocated; one set-up launch clears the control words
        PlanDesc* table = reinterpret_cast<PlanDesc*>(base + L.off_table);
        for (uint32_t i = 0; i < n_plans; i++) {
            hipError_t e = xm::copy_desc(table + i, plans[i]->desc, stream);
            if (e != hipSuccess) return hip_fail(e, "descriptor copy launch");
        }
        xm::InitArgs ia;
        std::memset(&ia, 0, sizeof(ia));
        ia.table = table;
        ia.count = 0;
        ia.n_plans = n_plans;
        ia.zero_ctl = 1;
        ia.ctl = a.ctl;
        ia.plan_flags = a.plan_flags;
        ia.counts = a.counts;
        ia.don = a.don;
        ia.don_cap = a.don_cap;
        ia.list_count = a.list_count;
        inits.push_back(ia);
    }
    for (uint32_t first = 0; first < n_plans && !on_static; first += xm::kMaxPlansPerInit) {
        xm::InitArgs ia;
        std::memset(&ia, 0, sizeof(ia));
        ia.table = reinterpret_cast<PlanDesc*>(base + L.off_table);
        ia.first = first;
        ia.count = std::min<uint32_t>(xm::kMaxPlansPerInit, n_plans - first);
        for (uint32_t i = 0; i < ia.count; i++) {
            const PlanDesc* d = nullptr;
            int r2 = plan_device_desc(const_cast<xm_plan_t*>(plans[first + i]), g->device, &d);
            if (r2) return r2;
            ia.src[i] = d;
        }
        ia.n_plans = n_plans;
        ia.zero_ctl = (first == 0) ? 1 : 0;
        ia.ctl = a.ctl;
        ia.plan_flags = a.plan_flags;
        ia.counts = a.counts;
        ia.don = a.don;
        ia.don_cap = a.don_cap;
        ia.list_count = a.list_count;
        inits.push_back(ia);
    }
    hipEvent_t ev0 = o ? static_cast<hipEvent_t>(o->ev_kernel_start) : nullptr;
    hipEvent_t ev1 = o ? static_cast<hipEvent_t>(o->ev_kernel_stop) : nullptr;
    hipError_t e = xm::launch_count(inits.data(), (int)inits.size(), a, L.n_blocks, stream, ev0, ev1);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return XM_OK;
}

}  // namespace

extern "C" {

const char* xm_version(void) { return "xminer-gfx950 0.1"; }

const char* xm_last_error(void) { return g_err.c_str(); }

const char* xm_strerror(int code) {
    switch (code) {
        case XM_OK: return "ok";
        case XM_ERR_INVALID: return "invalid argument";
        case XM_ERR_PATTERN: return "pattern rejected";
        case XM_ERR_OOM: return "out of memory";
        case XM_ERR_HIP: return "HIP runtime error";
        case XM_ERR_OVERFLOW: return "count exceeded 2^128-1";
        case XM_ERR_WORKSPACE: return "workspace too small";
        case XM_ERR_CANCELLED: return "cancelled";
        case XM_ERR_GRAPH: return "graph failed validation";
        default: return "unknown status";
    }
}

int xm_load_graph(uint32_t n, uint32_t m, const uint32_t* out_off, const uint32_t* out_adj,
                  const uint32_t* in_off, const uint32_t* in_adj, uint32_t flags, void* hip_stream,
                  xm_graph_t** out) {
    if (!out) return fail(XM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n == 0 || n >= 0xFFFFFFFFu) return fail(XM_ERR_INVALID, "n must be in 1..2^32-2");
    if (!out_off || !in_off || (m > 0 && (!out_adj || !in_adj)))
        return fail(XM_ERR_INVALID, "CSR array is NULL");
    bool dev_mem = (flags & XM_MEM_DEVICE) != 0, host_mem = (flags & XM_MEM_HOST) != 0;
    if (dev_mem == host_mem) return fail(XM_ERR_INVALID, "set exactly one of XM_MEM_DEVICE / XM_MEM_HOST");
    if (flags & ~(XM_MEM_DEVICE | XM_MEM_HOST | XM_VALIDATE | XM_ORDER_BY_DEGREE))
        return fail(XM_ERR_INVALID, "unknown flag");
    const bool reorder = (flags & XM_ORDER_BY_DEGREE) != 0;
    if (reorder && !host_mem) return fail(XM_ERR_INVALID, "XM_ORDER_BY_DEGREE needs XM_MEM_HOST");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    xm_graph_t* g = new (std::nothrow) xm_graph_s;
    if (!g) return fail(XM_ERR_OOM, "host allocation");
    g->n = n;
    g->m = m;
    HIP_TRY(hipGetDevice(&g->device), "hipGetDevice");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, g->device), "hipGetDeviceProperties");
    g->n_cu = prop.multiProcessorCount;
    g->max_lds_block = prop.sharedMemPerBlock;
    // host copies of the offsets (and lists when validating)
    std::vector<uint32_t> ho(n + 1), hi(n + 1), hoa, hia;
    auto to_host = [&](std::vector<uint32_t>& dst, const uint32_t* src, size_t cnt) -> hipError_t {
        dst.resize(cnt);
        if (cnt == 0) return hipSuccess;
        if (host_mem) {
            std::memcpy(dst.data(), src, cnt * 4);
            return hipSuccess;
        }
        return hipMemcpy(dst.data(), src, cnt * 4, hipMemcpyDeviceToHost);
    };
    auto cleanup = [&]() {
        if (g->owns_csr) {
            (void)hipFree((void*)g->out_off);
            (void)hipFree((void*)g->out_adj);
            (void)hipFree((void*)g->in_off);
            (void)hipFree((void*)g->in_adj);
        }
        if (g->deg) (void)hipFree(g->deg);
        if (g->degc) (void)hipFree(g->degc);
        if (g->hubs) (void)hipFree(g->hubs);
        delete g;
    };
    hipError_t e;
    if ((e = to_host(ho, out_off, n + 1)) != hipSuccess || (e = to_host(hi, in_off, n + 1)) != hipSuccess) {
        cleanup();
        return hip_fail(e, "copy offsets");
    }
    if (ho[0] != 0 || hi[0] != 0 || ho[n] != m || hi[n] != m) {
        cleanup();
        return fail(XM_ERR_GRAPH, "offsets must start at 0 and end at m");
    }
    for (uint32_t v = 0; v < n; v++)
        if (ho[v + 1] < ho[v] || hi[v + 1] < hi[v]) {
            cleanup();
            return fail(XM_ERR_GRAPH, "offsets must be non-decreasing");
        }
    if (flags & XM_VALIDATE) {
        if ((e = to_host(hoa, out_adj, m)) != hipSuccess || (e = to_host(hia, in_adj, m)) != hipSuccess) {
            cleanup();
            return hip_fail(e, "copy lists");
        }
        std::vector<uint32_t> cnt(n, 0);
        for (uint32_t u = 0; u < n; u++)
            for (uint32_t k = ho[u]; k < ho[u + 1]; k++) {
                uint32_t v = hoa[k];
                if (v >= n || v == u || (k > ho[u] && hoa[k - 1] >= v)) {
                    cleanup();
                    return fail(XM_ERR_GRAPH, "out-lists must be sorted, distinct, in range, loop-free");
                }
                cnt[v]++;
            }
        for (uint32_t v = 0; v < n; v++)
            if (cnt[v] != hi[v + 1] - hi[v]) {
                cleanup();
                return fail(XM_ERR_GRAPH, "in-CSR is not the transpose of the out-CSR");
            }
        std::vector<uint32_t> fill(n, 0);
        for (uint32_t u = 0; u < n; u++)
            for (uint32_t k = ho[u]; k < ho[u + 1]; k++) {
                uint32_t v = hoa[k];
                if (hia[hi[v] + fill[v]++] != u) {
                    cleanup();
                    return fail(XM_ERR_GRAPH, "in-CSR is not the transpose of the out-CSR");
                }
            }
    }
    std::vector<uint32_t> roa, ria;  // renumbered lists (XM_ORDER_BY_DEGREE)
    if (reorder) {
        // new ids by decreasing total degree (ties: lower old id first); each
        // list is renumbered and sorted again
        std::vector<uint32_t> by_deg(n);
        for (uint32_t v = 0; v < n; v++) by_deg[v] = v;
        auto tot = [&](uint32_t v) { return (uint64_t)(ho[v + 1] - ho[v]) + (hi[v + 1] - hi[v]); };
        std::stable_sort(by_deg.begin(), by_deg.end(), [&](uint32_t a, uint32_t b) { return tot(a) > tot(b); });
        g->new_of_old.assign(n, 0);
        for (uint32_t i = 0; i < n; i++) g->new_of_old[by_deg[i]] = i;
        const std::vector<uint32_t>& nw = g->new_of_old;
        auto renumber = [&](const std::vector<uint32_t>& off, const uint32_t* adj, std::vector<uint32_t>& noff,
                            std::vector<uint32_t>& nadj) {
            noff.assign(n + 1, 0);
            for (uint32_t i = 0; i < n; i++) noff[i + 1] = noff[i] + (off[by_deg[i] + 1] - off[by_deg[i]]);
            nadj.resize(std::max<uint32_t>(m, 1));
            for (uint32_t i = 0; i < n; i++) {
                const uint32_t v = by_deg[i];
                uint32_t* d = nadj.data() + noff[i];
                for (uint32_t k = off[v]; k < off[v + 1]; k++) *d++ = nw[adj[k]];
                std::sort(nadj.data() + noff[i], nadj.data() + noff[i + 1]);
            }
        };
        std::vector<uint32_t> no, ni;
        renumber(ho, out_adj, no, roa);
        renumber(hi, in_adj, ni, ria);
        ho.swap(no);
        hi.swap(ni);
    }
    if (host_mem) {
        void* p[4] = {nullptr, nullptr, nullptr, nullptr};
        size_t sz[4] = {(size_t)(n + 1) * 4, (size_t)std::max<uint32_t>(m, 1) * 4, (size_t)(n + 1) * 4,
                        (size_t)std::max<uint32_t>(m, 1) * 4};
        const void* src[4] = {out_off, out_adj, in_off, in_adj};
        if (reorder) {
            src[0] = ho.data();
            src[1] = roa.data();
            src[2] = hi.data();
            src[3] = ria.data();
        }
        size_t cp[4] = {(size_t)(n + 1) * 4, (size_t)m * 4, (size_t)(n + 1) * 4, (size_t)m * 4};
        g->owns_csr = true;
        for (int i = 0; i < 4; i++) {
            if ((e = hipMalloc(&p[i], sz[i])) != hipSuccess) {
                for (int j = 0; j < i; j++) (void)hipFree(p[j]);
                g->owns_csr = false;
                cleanup();
                return fail(XM_ERR_OOM, "hipMalloc(csr)");
            }
        }
        g->out_off = (uint32_t*)p[0];
        g->out_adj = (uint32_t*)p[1];
        g->in_off = (uint32_t*)p[2];
        g->in_adj = (uint32_t*)p[3];
        for (int i = 0; i < 4; i++)
            if (cp[i] && (e = hipMemcpyAsync(p[i], src[i], cp[i], hipMemcpyHostToDevice, stream)) != hipSuccess) {
                cleanup();
                return hip_fail(e, "hipMemcpyAsync(csr)");
            }
    } else {
        g->out_off = out_off;
        g->out_adj = out_adj;
        g->in_off = in_off;
        g->in_adj = in_adj;
    }
    // degrees, hub candidates and statistics
    std::vector<uint2> deg(n);
    std::vector<std::pair<uint32_t, uint32_t>> hubs;
    uint64_t ge_out[8] = {0}, ge_in[8] = {0};
    for (uint32_t v = 0; v < n; v++) {
        uint32_t dout = ho[v + 1] - ho[v], din = hi[v + 1] - hi[v];
        deg[v] = make_uint2(dout, din);
        g->max_out = std::max(g->max_out, dout);
        g->max_in = std::max(g->max_in, din);
        uint32_t mx = std::max(dout, din);
        if (mx > xm::kHubMin) hubs.push_back({mx, v});
        for (int t = 0; t < 8; t++) {
            ge_out[t] += dout >= (uint32_t)t;
            ge_in[t] += din >= (uint32_t)t;
        }
    }
    std::sort(hubs.begin(), hubs.end(), [](auto& x, auto& y) { return x.first > y.first || (x.first == y.first && x.second < y.second); });
    g->n_hubs = (uint32_t)hubs.size();
    g->hub_len.resize(hubs.size());
    g->hub_deg.resize(hubs.size());
    g->hub_id.resize(hubs.size());
    std::vector<uint32_t> hub_ids(std::max<size_t>(hubs.size(), 1), 0);
    for (size_t i = 0; i < hubs.size(); i++) {
        g->hub_len[i] = hubs[i].first;
        g->hub_deg[i] = deg[hubs[i].second];
        g->hub_id[i] = hubs[i].second;
        hub_ids[i] = hubs[i].second;
    }
    g->stats.n = n;
    g->stats.m = m;
    for (int t = 0; t < 8; t++) {
        g->stats.frac_out_ge[t] = (double)ge_out[t] / n;
        g->stats.frac_in_ge[t] = (double)ge_in[t] / n;
    }
    g->hdeg = deg;
    // degree classes for the candidate tests: thresholds never pass 6 (a
    // pattern vertex has at most 6 out- and 6 in-neighbours), so degrees
    // capped at 15 decide them exactly, one byte per node
    std::vector<uint8_t> degc(n);
    for (uint32_t v = 0; v < n; v++)
        degc[v] = (uint8_t)(std::min<uint32_t>(deg[v].x, 15u) | (std::min<uint32_t>(deg[v].y, 15u) << 4));
    if ((e = hipMalloc(&g->deg, (size_t)n * sizeof(uint2))) != hipSuccess ||
        (e = hipMalloc(&g->degc, (size_t)n)) != hipSuccess ||
        (e = hipMalloc(&g->hubs, hub_ids.size() * 4)) != hipSuccess) {
        cleanup();
        return fail(XM_ERR_OOM, "hipMalloc(degrees)");
    }
    if ((e = hipMemcpyAsync(g->deg, deg.data(), (size_t)n * sizeof(uint2), hipMemcpyHostToDevice, stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(g->degc, degc.data(), (size_t)n, hipMemcpyHostToDevice, stream)) != hipSuccess ||
        (e = hipMemcpyAsync(g->hubs, hub_ids.data(), hub_ids.size() * 4, hipMemcpyHostToDevice, stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess) {
        cleanup();
        return hip_fail(e, "upload degrees");
    }
    *out = g;
    return XM_OK;
}

int xm_plan_work(uint32_t n, const uint32_t* out_off, const uint32_t* out_adj, const uint32_t* in_off,
                 const uint32_t* in_adj, const xm_plan_t* p, const uint32_t* roots, uint32_t n_roots,
                 uint32_t threads, uint64_t max_partial, uint64_t out[4]) {
    if (!p || !out || !out_off || !in_off || n == 0) return fail(XM_ERR_INVALID, "NULL argument");
    if ((out_off[n] > 0 && !out_adj) || (in_off[n] > 0 && !in_adj))
        return fail(XM_ERR_INVALID, "NULL adjacency array");
    xm::HostCsr h{out_off, out_adj, in_off, in_adj, n};
    xm::WorkOut w;
    bool exceeded = xm::plan_work(h, p->desc, roots, n_roots, threads ? threads : 1, max_partial, xm::kNoRows, w);
    out[0] = w.elements;
    out[1] = w.fetches;
    out[2] = w.partial;
    out[3] = w.roots;
    return exceeded ? 1 : XM_OK;
}

int xm_plan_traffic(uint32_t n, const uint32_t* out_off, const uint32_t* out_adj, const uint32_t* in_off,
                    const uint32_t* in_adj, const xm_plan_t* p, const uint32_t* roots, uint32_t n_roots,
                    uint32_t row_min, uint32_t threads, uint64_t max_partial, uint64_t out[XM_TRAFFIC_WORDS]) {
    if (!p || !out || !out_off || !in_off || n == 0) return fail(XM_ERR_INVALID, "NULL argument");
    if ((out_off[n] > 0 && !out_adj) || (in_off[n] > 0 && !in_adj))
        return fail(XM_ERR_INVALID, "NULL adjacency array");
    xm::HostCsr h{out_off, out_adj, in_off, in_adj, n};
    xm::WorkOut w;
    bool exceeded = xm::plan_work(h, p->desc, roots, n_roots, threads ? threads : 1, max_partial,
                                  row_min ? row_min : xm::kNoRows, w);
    out[0] = w.base;
    out[1] = w.offset_pairs;
    out[2] = w.deg_reads;
    out[3] = w.row_probes;
    out[4] = w.searches;
    out[5] = w.search_words;
    out[6] = w.partial;
    out[7] = w.chain_words;
    out[8] = w.roots;
    out[9] = w.elements;
    return exceeded ? 1 : XM_OK;
}

int xm_free_graph(xm_graph_t* g) {
    if (!g) return XM_OK;
    if (g->execs.load() != 0) return fail(XM_ERR_INVALID, "graph has captured launches; free them first");
    if (g->owns_csr) {
        (void)hipFree((void*)g->out_off);
        (void)hipFree((void*)g->out_adj);
        (void)hipFree((void*)g->in_off);
        (void)hipFree((void*)g->in_adj);
    }
    if (g->deg) (void)hipFree(g->deg);
    if (g->degc) (void)hipFree(g->degc);
    if (g->hubs) (void)hipFree(g->hubs);
    if (g->rows) (void)hipFree(g->rows);
    if (g->row_of) (void)hipFree(g->row_of);
    delete g;
    return XM_OK;
}

int xm_graph_dense_rows(xm_graph_t* g, uint64_t max_bytes, uint32_t min_len, void* hip_stream,
                        uint32_t* out_min_len) {
    if (!g) return fail(XM_ERR_INVALID, "graph is NULL");
    if (out_min_len) *out_min_len = 0;
    if (g->execs.load() != 0) return fail(XM_ERR_INVALID, "graph has captured launches; free them first");
    int cur_dev = 0;
    HIP_TRY(hipGetDevice(&cur_dev), "hipGetDevice");
    if (cur_dev != g->device) return fail(XM_ERR_INVALID, "current device differs from the graph's");
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    // launches in flight may read the old rows
    HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (g->rows) (void)hipFree(g->rows);
    if (g->row_of) (void)hipFree(g->row_of);
    g->rows = nullptr;
    g->row_of = nullptr;
    g->row_min = xm::kNoRows;
    g->n_rows_out = g->n_rows_in = 0;
    g->row_words = 0;
    if (max_bytes == 0 || g->n >= 0x80000000u) return XM_OK;
    max_bytes = std::min<uint64_t>(max_bytes, xm::kMaxRowBytes);
    const uint64_t words = ((uint64_t)g->n + 31) / 32;
    const uint64_t row_bytes = words * 4;
    // rows go to the longest lists first: the threshold is the smallest list
    // length (at least max(min_len, 32)) such that every list at least that
    // long, in both directions, has a row within max_bytes
    const uint64_t fit = max_bytes / row_bytes;
    const uint32_t lo = std::max<uint32_t>(min_len, 32);
    std::vector<uint32_t> lens;
    for (const uint2& d : g->hdeg) {
        if (d.x >= lo) lens.push_back(d.x);
        if (d.y >= lo) lens.push_back(d.y);
    }
    if (lens.empty() || fit == 0) return XM_OK;
    std::sort(lens.begin(), lens.end(), std::greater<uint32_t>());
    uint64_t t = lo;
    if (lens.size() > fit) {
        // lens[fit] must stay below the threshold (ties included)
        t = (uint64_t)lens[fit] + 1;
        if (t > lens[0]) return XM_OK;
    }
    uint64_t n_out = 0, n_in = 0;
    for (const uint2& d : g->hdeg) {
        n_out += d.x >= t;
        n_in += d.y >= t;
    }
    if (n_out + n_in == 0) return XM_OK;
    std::vector<uint2> row_of(g->n, make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu));
    std::vector<uint32_t> row_node;
    row_node.reserve(n_out + n_in);
    for (uint32_t v = 0; v < g->n; v++)
        if (g->hdeg[v].x >= t) {
            row_of[v].x = (uint32_t)row_node.size();
            row_node.push_back(v);
        }
    for (uint32_t v = 0; v < g->n; v++)
        if (g->hdeg[v].y >= t) {
            row_of[v].y = (uint32_t)row_node.size();  // in rows follow the out rows
            row_node.push_back(v);
        }
    uint32_t* rn = nullptr;
    hipError_t e;
    if ((e = hipMalloc(&g->rows, (n_out + n_in) * row_bytes)) != hipSuccess ||
        (e = hipMalloc(&g->row_of, (size_t)g->n * sizeof(uint2))) != hipSuccess ||
        (e = hipMalloc(&rn, row_node.size() * 4)) != hipSuccess) {
        if (g->rows) (void)hipFree(g->rows);
        if (g->row_of) (void)hipFree(g->row_of);
        g->rows = nullptr;
        g->row_of = nullptr;
        return fail(XM_ERR_OOM, "hipMalloc(dense rows)");
    }
    g->row_words = words;
    g->n_rows_out = (uint32_t)n_out;
    g->n_rows_in = (uint32_t)n_in;
    g->row_min = (uint32_t)t;
    xm::DevGraph dg{};
    dg.out_off = g->out_off;
    dg.out_adj = g->out_adj;
    dg.in_off = g->in_off;
    dg.in_adj = g->in_adj;
    dg.n = g->n;
    dg.row_words = (uint32_t)words;
    if ((e = hipMemsetAsync(g->rows, 0, (n_out + n_in) * row_bytes, stream)) != hipSuccess ||
        (e = hipMemcpyAsync(g->row_of, row_of.data(), (size_t)g->n * sizeof(uint2), hipMemcpyHostToDevice,
                            stream)) != hipSuccess ||
        (e = hipMemcpyAsync(rn, row_node.data(), row_node.size() * 4, hipMemcpyHostToDevice, stream)) !=
            hipSuccess ||
        (e = xm::build_rows(dg, rn, (uint32_t)n_out, (uint32_t)(n_out + n_in), g->rows, stream)) != hipSuccess ||
        (e = hipStreamSynchronize(stream)) != hipSuccess) {
        (void)hipStreamSynchronize(stream);
        (void)hipFree(rn);
        (void)hipFree(g->rows);
        (void)hipFree(g->row_of);
        g->rows = nullptr;
        g->row_of = nullptr;
        g->row_min = xm::kNoRows;
        g->n_rows_out = g->n_rows_in = 0;
        g->row_words = 0;
        return hip_fail(e, "build dense rows");
    }
    (void)hipFree(rn);
    if (out_min_len) *out_min_len = (uint32_t)t;
    return XM_OK;
}

int xm_graph_dense_rows_info(const xm_graph_t* g, uint32_t* min_len, uint32_t* n_out_rows, uint32_t* n_in_rows,
                             uint64_t* bytes) {
    if (!g) return fail(XM_ERR_INVALID, "graph is NULL");
    const bool on = g->rows != nullptr;
    if (min_len) *min_len = on ? g->row_min : 0;
    if (n_out_rows) *n_out_rows = on ? g->n_rows_out : 0;
    if (n_in_rows) *n_in_rows = on ? g->n_rows_in : 0;
    if (bytes) *bytes = on ? (uint64_t)(g->n_rows_out + g->n_rows_in) * g->row_words * 4 : 0;
    return XM_OK;
}

int xm_graph_node_order(const xm_graph_t* g, uint32_t* new_of_old) {
    if (!g || !new_of_old) return fail(XM_ERR_INVALID, "NULL argument");
    for (uint32_t v = 0; v < g->n; v++) new_of_old[v] = g->new_of_old.empty() ? v : g->new_of_old[v];
    return XM_OK;
}

int xm_graph_info(const xm_graph_t* g, uint32_t* n, uint32_t* m, uint32_t* max_out, uint32_t* max_in) {
    if (!g) return fail(XM_ERR_INVALID, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (max_out) *max_out = g->max_out;
    if (max_in) *max_in = g->max_in;
    return XM_OK;
}

int xm_plan(uint32_t k, uint32_t n_arcs, const uint8_t* arcs, uint32_t flags, const xm_graph_t* g,
            xm_plan_t** out) {
    if (!out) return fail(XM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (flags & ~(0xFu | 0xF00u | 0xFF0000u)) return fail(XM_ERR_INVALID, "unknown plan flag");
    xm_plan_t* p = new (std::nothrow) xm_plan_s;
    if (!p) return fail(XM_ERR_OOM, "host allocation");
    std::string err;
    int rc = xm::build_plan(k, n_arcs, arcs, flags, g ? &g->stats : nullptr, p->desc, p->json, err);
    if (rc) {
        delete p;
        return fail(rc == -1 ? XM_ERR_INVALID : XM_ERR_PATTERN, err);
    }
    *out = p;
    return XM_OK;
}

int xm_plan_describe(const xm_plan_t* p, char* json, size_t cap, size_t* needed) {
    if (!p) return fail(XM_ERR_INVALID, "plan is NULL");
    if (needed) *needed = p->json.size() + 1;
    if (!json || cap < p->json.size() + 1) return fail(XM_ERR_INVALID, "buffer too small");
    std::memcpy(json, p->json.c_str(), p->json.size() + 1);
    return XM_OK;
}

int xm_plan_root_vertex(const xm_plan_t* p) {
    if (!p) return fail(XM_ERR_INVALID, "plan is NULL");
    return p->desc.order[0];
}

int xm_free_plan(xm_plan_t* p) {
    if (!p) return XM_OK;
    for (size_t d = 0; d < p->dev.size(); d++)
        if (p->dev[d]) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            (void)hipSetDevice((int)d);
            (void)hipFree(p->dev[d]);
            (void)hipSetDevice(cur);
        }
    delete p;
    return XM_OK;
}

size_t xm_workspace_size(const xm_graph_t* g, uint32_t n_plans, const xm_plan_t* const* plans,
                         const xm_count_opts* opts) {
    Layout L;
    if (make_layout(g, n_plans, plans, opts, L)) return 0;
    return L.total;
}

int xm_count(const xm_graph_t* g, uint32_t n_plans, const xm_plan_t* const* plans, const xm_count_opts* opts,
             void* workspace, size_t ws_bytes, uint64_t* counts_dev, int32_t* status_dev, void* hip_stream) {
    return enqueue_count(g, n_plans, plans, opts, workspace, ws_bytes, counts_dev, status_dev,
                         static_cast<hipStream_t>(hip_stream));
}

int xm_count_static(const xm_graph_t* g, uint32_t n_plans, const xm_plan_t* const* plans,
                    const xm_count_opts* opts, uint64_t* counts_dev, int32_t* status_dev, void* hip_stream) {
    return enqueue_count(g, n_plans, plans, opts, nullptr, 0, counts_dev, status_dev,
                         static_cast<hipStream_t>(hip_stream), true);
}

int xm_count_capture(const xm_graph_t* g, uint32_t n_plans, const xm_plan_t* const* plans,
                     const xm_count_opts* opts, void* workspace, size_t ws_bytes, uint64_t* counts_dev,
                     int32_t* status_dev, void* hip_stream, xm_exec_t** out) {
    if (!out) return fail(XM_ERR_INVALID, "out is NULL");
    *out = nullptr;
    Layout L;
    int rc = make_layout(g, n_plans, plans, opts, L);
    if (rc) return rc;
    if (!hip_stream) return fail(XM_ERR_INVALID, "capture needs a non-null stream");
    // plan uploads happen outside the capture
    for (uint32_t i = 0; i < n_plans; i++) {
        const PlanDesc* d = nullptr;
        rc = plan_device_desc(const_cast<xm_plan_t*>(plans[i]), g->device, &d);
        if (rc) return rc;
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    xm_exec_t* x = new (std::nothrow) xm_exec_s;
    if (!x) return fail(XM_ERR_OOM, "host allocation");
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        delete x;
        return hip_fail(e, "hipStreamBeginCapture");
    }
    rc = enqueue_count(g, n_plans, plans, opts, workspace, ws_bytes, counts_dev, status_dev, s);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        delete x;
        return rc;
    }
    if (e != hipSuccess) {
        delete x;
        return hip_fail(e, "hipStreamEndCapture");
    }
    x->graph = graph;
    e = hipGraphInstantiate(&x->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        delete x;
        return hip_fail(e, "hipGraphInstantiate");
    }
    x->g = g;
    g->execs.fetch_add(1);
    *out = x;
    return XM_OK;
}

int xm_exec_launch(xm_exec_t* x, void* hip_stream) {
    if (!x) return fail(XM_ERR_INVALID, "exec is NULL");
    HIP_TRY(hipGraphLaunch(x->exec, static_cast<hipStream_t>(hip_stream)), "hipGraphLaunch");
    return XM_OK;
}

int xm_free_exec(xm_exec_t* x) {
    if (!x) return XM_OK;
    if (x->exec) (void)hipGraphExecDestroy(x->exec);
    if (x->graph) (void)hipGraphDestroy(x->graph);
    if (x->g) x->g->execs.fetch_sub(1);
    delete x;
    return XM_OK;
}

}  // extern "C"
