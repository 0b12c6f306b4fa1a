// kernels.h — launch interface between the host runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "plan_ir.h"

namespace xm {

constexpr int kWavesPerBlock = 4;
constexpr int kBlockThreads = 64 * kWavesPerBlock;
constexpr uint32_t kHubMin = 64;    // nodes with a list longer than this are hub candidates
constexpr int kMaxPlansPerInit = 240;
constexpr int kLvlArrays = 5;       // node, parent, seg_begin, seg_count, aux per level
constexpr uint32_t kMergeChunk = 256; // elements per list chunk in the cooperative merge
constexpr uint32_t kMergeMin = 0xFFFFFFFFu;  // default: merge off (see xm_count_opts.merge_min)
constexpr uint32_t kMergeRatio = 16;  // ... and within this length ratio -> merge

// Control words at the start of the workspace.
constexpr uint32_t kQueues = 8;  // split-task queues, one per XCD (8 XCDs on MI355X)
constexpr uint32_t kDonWords = 8;  // donated task: plan | depth << 16, ready flag, prefix nodes [6]
constexpr uint32_t kDonCap = 1u << 18;  // donated-task slots per launch
constexpr uint32_t kDonCapStatic = 1u << 14;  // ... in launches on the static scratch array

// The static scratch array of xm_count_static (file scope in count.hip): one
// copy per device, held until the process ends.
constexpr uint64_t kStaticScratchBytes = 64ull << 20;
// Device address of this device's copy (hipGetSymbolAddress; call with the
// device current).
hipError_t static_scratch_address(void** ptr);

// Copy one plan descriptor from host memory into dst through kernel
// arguments (no staging allocation): words of the descriptor in chunks.
constexpr uint32_t kDescChunkWords = 480;
struct DescChunk {
    uint32_t* dst;
    uint32_t n;
    uint32_t w[kDescChunkWords];
};
hipError_t copy_desc(PlanDesc* dst, const PlanDesc& src, hipStream_t stream);

enum Ctl : uint32_t {
    kCtlCancelled = 3,    // a wave saw the cancel flag
    kCtlQueueFull = 4,    // split queue overflow (cannot happen with a sized workspace)
    kCtlBadPlan = 5,      // a level had more constraints than the layout holds (cannot happen)
    kCtlSplitHead0 = 8,   // [kQueues]: next item of split queue q
    kCtlSplitCount0 = 16, // [kQueues]: items the split kernel wrote to queue q
    // the words idle waves poll sit on cache lines of their own
    kCtlActive = 64,      // waves in a work phase (from their first task until the queues ran dry)
    kCtlIdle = 96,        // waves waiting for donated tasks
    kCtlDonHead = 128,    // next donated task to take
    kCtlDonTail = 160,    // donated-task slots reserved
    kCtlRootCursor0 = 192,  // [kQueues], 32 words apart: cursor q hands out root items q, q + 8, ...
    kCtlWords = 192 + 32 * kQueues
};

struct DevGraph {
    const uint32_t* out_off;
    const uint32_t* out_adj;
    const uint32_t* in_off;
    const uint32_t* in_adj;
    const uint2* deg;   // (out-degree, in-degree)
    const uint8_t* degc;  // min(out-degree, 15) | min(in-degree, 15) << 4
    uint32_t n;
    uint32_t row_min;   // lists at least this long have a dense row (kNoRows: none)
    // dense membership rows of long lists: row r is row_words uint32 words at
    // word offset r * row_words, computed in 64 bits (out rows first, then in
    // rows), bit x set iff node x is in the list
    const uint32_t* rows;
    const uint2* row_of;  // per node: (out row, in row), 0xFFFFFFFF = no row
    uint32_t row_words;
    uint32_t pad;
};

constexpr uint32_t kNoRows = 0xFFFFFFFFu;
constexpr uint32_t kRowLen = 0xFFFFFFFEu;  // probe-list length marker: test a dense row

constexpr uint64_t kMaxRowBytes = 256ull << 30;  // rows budget, at most (row ids are 32-bit)

// Set the bits of dense rows [0, n_rows): row r holds the out-list (r <
// n_out_rows) or in-list of node row_node[r].  Rows must be zeroed first.
hipError_t build_rows(const DevGraph& g, const uint32_t* row_node, uint32_t n_out_rows, uint32_t n_rows,
                      uint32_t* rows, hipStream_t stream);

struct KArgs {
    DevGraph g;
    const PlanDesc* plans;      // table in the workspace
    uint32_t n_plans;
    uint32_t chunk;             // roots per root work item (<= 64)
    uint32_t split;             // largest first-level sub-range of a split root
    uint32_t split_work;        // target (sub-range length x first-level length) per task
    uint32_t cap;               // entries per level buffer
    uint32_t* ctl;              // control words
    uint32_t* plan_flags;       // per plan: bit 0 overflow
    uint4* split_items;         // (plan, root, lo, hi); queue q holds [qbase[q], qbase[q+1])
    uint32_t split_cap;
    uint32_t qbase[kQueues + 1];
    uint32_t* don;              // donated tasks: kDonWords words each
    uint32_t don_cap;
    uint32_t* list;             // listing: rows of k node ids (NULL: counting only)
    unsigned long long* list_count;
    unsigned long long list_cap;
    uint32_t n_src;             // roots: subset size or n
    const uint32_t* roots;      // subset or NULL (then root i is node i)
    const uint32_t* hubs;       // hub candidates for the split kernel (when roots == NULL)
    uint32_t n_hubs;
    uint32_t lds_words;         // LDS words per wave
    uint32_t lds_rows;          // bound / ancestor rows (largest enumerated depth)
    uint32_t maxc;              // largest constraint count over plans and signatures
    uint32_t nonlinear;         // some plan counts a leaf group of several vertices
    uint32_t n_cu;              // compute units of the device (picks the register budget)
    uint32_t merge_min;         // cooperative merge thresholds
    uint32_t merge_ratio;
    uint32_t wave_words;        // scratch words per wave
    uint32_t* scratch;          // n_waves * wave_words
    unsigned long long* counts; // 2 per plan
    int32_t* status;            // 1 per plan
    const int32_t* cancel;      // nullable
};

struct InitArgs {
    PlanDesc* table;
    const PlanDesc* src[kMaxPlansPerInit];
    uint32_t first, count;      // plans [first, first+count) of the table
    uint32_t n_plans;
    uint32_t zero_ctl;          // 1: also clear control words, flags and counts
    uint32_t* ctl;
    uint32_t* plan_flags;
    unsigned long long* counts;
    uint32_t* don;              // donated-task slots: their ready words are cleared
    uint32_t don_cap;
    unsigned long long* list_count;  // listing counter (NULL: none)
};

// First-level sub-range length for a root whose first-level list has L1
// entries: the task size shrinks as the list grows, because each first-level
// candidate of a long list usually carries a long list below it.
constexpr uint32_t kMaxPieces = 4096;  // sub-range tasks per root and plan, at most
// launches of at most this many resident blocks per CU use the count kernel
// compiled for that occupancy, which keeps all its state in registers
constexpr int kRoomyBlocksPerCu = 3;

// The base list of a level below the first (and of a leaf pass): the
// shortest constraint list, except that when the shortest belongs to an
// earlier bound vertex than the deepest constraint's, the deepest vertex's
// list is taken if it is at most kFreshBaseRatio times longer (0: never).
// The deepest bound vertex changes from parent to parent while the earlier
// ones are shared by the siblings of a window: scanning the fresh list reads
// it line by line, and the candidate tests then land on the shared lists'
// lines (dense-row words) that stay in L2, instead of one fresh line each.
// Measured on the 256-plan R-MAT 22 batch: ratio 2 cuts the launch by 2%,
// ratios 4 and 8 lengthen it by 21-22% (more elements to test).
#ifndef XM_FRESH_BASE_RATIO
#define XM_FRESH_BASE_RATIO 2
#endif
constexpr uint32_t kFreshBaseRatio = XM_FRESH_BASE_RATIO;

__host__ __device__ inline uint32_t item_size(uint32_t L1, uint32_t split, uint32_t split_work) {
    uint32_t s = L1 ? split_work / L1 : split;
    s = s < split ? s : split;
    s = s < 1 ? 1 : s;
    const uint32_t floor_s = (L1 + kMaxPieces - 1) / kMaxPieces;
    return s > floor_s ? s : floor_s;
}

// Sub-range size for a plan with e enumerated levels (root included).  A
// plan with one level below the root spends one leaf count per first-level
// candidate, so its sub-ranges are larger (8x the candidates, 16x the work
// target, at most cap) than those of deeper plans, whose candidates each
// carry a subtree.  The split kernel, the count kernel's root filter and the
// host's queue sizing all use this.
__host__ __device__ inline uint32_t plan_item_size(uint32_t L1, uint32_t e, uint32_t split, uint32_t split_work,
                                                   uint32_t cap) {
    if (e == 2) {
        split = split <= cap / 8 ? split * 8 : (cap > split ? cap : split);
        split_work = split_work <= (0xFFFFFFFFu >> 4) ? split_work << 4 : 0xFFFFFFFFu;
    }
    return item_size(L1, split, split_work);
}

// Whether root r belongs to a plan's root share s: r mod 2^s = 2^s - 1
// (every root when s = 0).  The residue 2^s - 1 keeps node 0 -- on a graph
// stored in degree order, the largest hub -- out of every proper share.
__host__ __device__ inline bool in_root_share(uint32_t r, uint32_t s) {
    const uint32_t mask = s >= 32 ? 0xFFFFFFFFu : ((1u << s) - 1u);
    return ((r + 1u) & mask) == 0u;
}

// LDS words per wave: `rows` bound levels (the largest enumerated depth of
// the batch), the largest constraint count, and the optional parts.
inline uint32_t lds_words_for(uint32_t rows, uint32_t maxc, bool nonlinear, bool merge) {
    return 2 * rows * 64       // bound values, ancestor indices
           + 7 * 64            // base address (2 words) and length, inclusive scan, segment
                               // counts, tile parent marks (2 x 64)
           + 3 * maxc * 64     // probe slots: length, address (two words) per constraint
           + (merge ? kMergeChunk : 0)  // merge chunk
           + (nonlinear ? 16 * 64 : 0)  // leaf-group histograms
           + 32;               // wave state
}

// Resident 256-thread blocks per compute unit for the count kernel variant.
int count_blocks_per_cu(bool nonlin, size_t lds_bytes);

hipError_t launch_count(const InitArgs* inits, int n_inits, const KArgs& a, uint32_t n_blocks,
                        hipStream_t stream, hipEvent_t ev_start, hipEvent_t ev_stop);

// Host-side algorithmic work of a plan (work.cpp).
struct HostCsr {
    const uint32_t *out_off, *out_adj, *in_off, *in_adj;
    uint32_t n;
};
struct WorkOut {
    // merge model: every element of every list a partial match intersects
    uint64_t elements = 0, fetches = 0, partial = 0, roots = 0;
    // what the count kernel reads and writes per partial match (its
    // candidate tests as issued: base elements scanned, offset pairs,
    // degree pairs, dense-row words, sorted-list searches and the words
    // they read, partial matches written and the chains read back)
    uint64_t base = 0, offset_pairs = 0, deg_reads = 0, row_probes = 0, searches = 0, search_words = 0,
             chain_words = 0;
};
// Returns true when the walk stopped early because it passed max_partial
// partial matches (0 = no limit); the figures are then partial sums.
// row_min: lists at least this long are tested through dense rows
// (kNoRows: none).
bool plan_work(const HostCsr& g, const PlanDesc& p, const uint32_t* roots, uint32_t n_roots,
               unsigned threads, uint64_t max_partial, uint32_t row_min, WorkOut& out);

}  // namespace xm
