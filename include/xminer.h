/*
 * xminer.h — C ABI of the MI355X (gfx950) exact directed-pattern counter.
 *
 * The library counts the embeddings of a small directed pattern graph in a
 * large directed data graph: the number of injective maps phi from pattern
 * vertices to data nodes such that every pattern arc (u, w) lands on a data
 * arc (phi(u), phi(w)), oriented the same (the paper, section 2: Definitions
 * 2.1 Digraph and 2.2 Pattern Graph, with constraint set C = vertices u
 * edges; counting by multiplying candidate-set sizes, section 5.3).  Matches
 * are non-induced and labelled: they are not divided by the pattern's
 * automorphism count.
 *
 * The work runs in three calls:
 *   xm_load_graph  registers a resident data graph (uint32 out-CSR + in-CSR);
 *   xm_plan        reduces the pattern and emits a level-by-level plan on the
 *                  host (section 4: inclusion sets, Theorem 2.1, minimum
 *                  constraint cover, Algorithm 1; section 5.1 plan generation);
 *   xm_count       executes one or many plans on the GPU (Algorithm 2 plan
 *                  execution, section 5.2 intermediate-result reuse, section
 *                  5.3 result generation by product) and writes exact counts.
 *
 * Conventions
 *   - Every call returns int: XM_OK (0) or a negative xm_status.  Argument
 *     errors are found on the host before anything is enqueued and leave no
 *     side effects.  xm_last_error() gives a message for the calling thread.
 *   - Ownership: the library never frees caller memory.  It owns xm_graph_t,
 *     xm_plan_t and xm_exec_t objects, which the caller frees with xm_free_*.
 *   - Streams: void* hip_stream is a hipStream_t (NULL = the null stream).
 *     xm_count is asynchronous on that stream.
 *   - Device: all device pointers must belong to the device that was current
 *     when the graph was loaded.
 */
#ifndef XMINER_H
#define XMINER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XM_MAX_K 7 /* largest pattern (vertices) */

typedef enum xm_status {
    XM_OK = 0,
    XM_ERR_INVALID = -1,   /* bad argument: NULL, size out of range, unknown flag */
    XM_ERR_PATTERN = -2,   /* pattern rejected: k outside 2..7, arc endpoint >= k,
                              self-loop arc, no arcs, not weakly connected */
    XM_ERR_OOM = -3,       /* host or device allocation failed */
    XM_ERR_HIP = -4,       /* a HIP runtime call failed (see xm_last_error) */
    XM_ERR_OVERFLOW = -5,  /* status only: a total exceeded 2^128 - 1 */
    XM_ERR_WORKSPACE = -6, /* workspace NULL or smaller than xm_workspace_size */
    XM_ERR_CANCELLED = -7, /* status only: stopped through the cancel flag */
    XM_ERR_GRAPH = -8      /* graph failed validation (XM_VALIDATE) */
} xm_status;

typedef struct xm_graph_s xm_graph_t; /* immutable after load; shareable between threads */
typedef struct xm_plan_s xm_plan_t; /* immutable; host-side plan + compact descriptor */
typedef struct xm_exec_s xm_exec_t; /* an instantiated HIP graph of one xm_count call */

/* ----------------------------------------------------------------------------
 * Graph residency (Definition 2.1; the paper keeps the data graph resident
 * and excludes loading from timing, section 6.1).
 *
 * n nodes 0..n-1 (1 <= n < 2^32 - 1), m arcs (m < 2^32).
 * out_off[n+1], out_adj[m]: out-CSR, each list sorted ascending, no repeats,
 *                           no self-loops.
 * in_off[n+1],  in_adj[m]:  in-CSR, the transpose of the out-CSR, same rules.
 * flags:
 *   XM_MEM_DEVICE  the four arrays are device pointers; the library BORROWS
 *                  them: the caller keeps them alive and unchanged until
 *                  xm_free_graph.
 *   XM_MEM_HOST    the four arrays are host pointers; the library copies them
 *                  to device memory it owns.
 *   XM_VALIDATE    check the rules above on the host (copies device arrays
 *                  back when XM_MEM_DEVICE); failure returns XM_ERR_GRAPH.
 *   XM_ORDER_BY_DEGREE  (with XM_MEM_HOST) store the graph with its nodes
 *                  renumbered by decreasing total degree, ties by lower id
 *                  (xm_graph_node_order gives the renumbering).  Counts do not
 *                  change; symmetry-broken plans (XM_PLAN_SYMMETRY) compare
 *                  node ids, and in this order their bounds cut more work.
 *                  Node ids at the boundary would be the new ones, so
 *                  xm_count refuses root subsets and listing on such a graph
 *                  (XM_ERR_INVALID).
 * Exactly one of XM_MEM_DEVICE / XM_MEM_HOST must be set.  The call also
 * builds per-node degree pairs and a hub list on the device (library-owned),
 * and synchronises hip_stream before returning.
 * ------------------------------------------------------------------------- */
#define XM_MEM_DEVICE 0x1u
#define XM_MEM_HOST 0x2u
#define XM_VALIDATE 0x4u
#define XM_ORDER_BY_DEGREE 0x8u
int xm_load_graph(uint32_t n, uint32_t m,
                  const uint32_t* out_off, const uint32_t* out_adj,
                  const uint32_t* in_off, const uint32_t* in_adj,
                  uint32_t flags, void* hip_stream, xm_graph_t** out);
/* Frees the graph; fails with XM_ERR_INVALID while captured launches
 * (xm_exec_t) of it exist. */
int xm_free_graph(xm_graph_t* g);
/* The node renumbering of a graph loaded with XM_ORDER_BY_DEGREE: writes n
 * entries to the host array new_of_old (new_of_old[v] = stored id of the
 * caller's node v); the identity for any other graph. */
int xm_graph_node_order(const xm_graph_t* g, uint32_t* new_of_old);
/* Dense membership rows for long adjacency lists.
 *
 * Every candidate test of Algorithm 2 asks whether a node x lies in the out-
 * or in-list of a bound node (the set intersections that build candidate
 * sets).  For lists of at least min_len elements this call stores an n-bit
 * row per list (bit x set iff x is in the list) in device memory the library
 * owns, and xm_count then answers such a test with one load instead of a
 * search of the sorted list.  Counts do not change.
 *
 * max_bytes bounds the rows' total size: the threshold is the smallest
 * list length, at least max(min_len, 32), such that every out- and in-list
 * at least that long gets a row within max_bytes (the longest lists first).
 * *out_min_len (nullable) receives the threshold used, 0 if no row was
 * built.  max_bytes = 0 removes the rows; budgets above 256 GiB are treated
 * as that.  Graphs with n >= 2^31 get no rows.  The call synchronises the device (launches in
 * flight may read the old rows) and fails with XM_ERR_INVALID while captured
 * launches (xm_exec_t) of this graph exist.  Rows cost ceil(n/32)*4 bytes
 * each; XM_ERR_OOM leaves the graph without rows. */
int xm_graph_dense_rows(xm_graph_t* g, uint64_t max_bytes, uint32_t min_len, void* hip_stream,
                        uint32_t* out_min_len);
/* Current rows: threshold (0 = none), rows per direction, bytes. */
int xm_graph_dense_rows_info(const xm_graph_t* g, uint32_t* min_len, uint32_t* n_out_rows,
                             uint32_t* n_in_rows, uint64_t* bytes);

/* Graph facts: n, m, max out-degree, max in-degree (any pointer may be NULL). */
int xm_graph_info(const xm_graph_t* g, uint32_t* n, uint32_t* m,
                  uint32_t* max_out, uint32_t* max_in);

/* ----------------------------------------------------------------------------
 * Planning (section 4.1 constraint inclusion; section 4.2 / Algorithm 1
 * reduction and minimum constraint cover; section 5.1 plan generation).
 *
 * k pattern vertices (2..XM_MAX_K), n_arcs arcs given as k-bounded byte pairs
 * arcs[2*i] -> arcs[2*i+1].  Repeated arcs are ignored; a bidirected edge is
 * two arcs.  flags: exactly one of
 *   XM_PLAN_REDUCED    pattern-reduced plan: sibling vertices share one
 *                      fetched candidate set, included constraints are
 *                      materialised from the including one, trailing
 *                      independent vertices are counted by product;
 *   XM_PLAN_UNREDUCED  every level materialises its own constraints from the
 *                      data graph; only the last vertex is counted, not
 *                      enumerated;
 * optionally OR'ed with XM_PLAN_ROOT(v) to force pattern vertex v as the
 * plan's start vertex (needed for root-subset counting), and with
 *   XM_PLAN_SYMMETRY   symmetry breaking (the symmetry destruction that the
 *                      related-work section says XMiner uses, made exact):
 *                      with H the automorphisms of the pattern that map the
 *                      enumerated vertices (plus the counted leaf when the
 *                      leaf group is one vertex) onto themselves, the plan
 *                      counts one partial match per H-orbit and the launch
 *                      scales the total by the orbit size, so counts are the
 *                      same labelled counts; a pattern without such
 *                      automorphisms gets a plain plan.  With XM_PLAN_ROOT(v)
 *                      only automorphisms that fix v are used, so each orbit
 *                      keeps one image of v and root-subset counts stay
 *                      exact; without it xm_count refuses such a plan with a
 *                      root subset.  Listing refuses both;
 *   XM_PLAN_ROOT_SHARE(s)  (s <= 31) count only the embeddings whose start
 *                      vertex (xm_plan_root_vertex) maps to a node whose
 *                      stored id r has r mod 2^s = 2^s - 1: an exact partial
 *                      count over a fixed 1/2^s share of the roots, for
 *                      patterns too heavy to count on every root (on a graph
 *                      stored in degree order the share takes every 2^s-th
 *                      node by degree rank, never the largest hub); with
 *                      XM_PLAN_SYMMETRY only automorphisms that fix the
 *                      start vertex are used, as with XM_PLAN_ROOT;
 *   XM_PLAN_SYM_BELOW  with XM_PLAN_SYMMETRY: keep per orbit the partial
 *                      match whose first conditioned vertex has the largest
 *                      image instead of the smallest (both exact; which
 *                      enumerates less depends on the graph).
 * g (nullable) supplies degree statistics used as cover weights; with g NULL
 * the plan uses unit weights.  No device work is done.
 * ------------------------------------------------------------------------- */
#define XM_PLAN_REDUCED 0x1u
#define XM_PLAN_UNREDUCED 0x2u
#define XM_PLAN_SYMMETRY 0x4u
#define XM_PLAN_SYM_BELOW 0x8u
#define XM_PLAN_ROOT(v) ((((uint32_t)(v)) + 1u) << 8)
#define XM_PLAN_ROOT_SHARE(s) (((uint32_t)(s) & 0xFFu) << 16)
int xm_plan(uint32_t k, uint32_t n_arcs, const uint8_t* arcs, uint32_t flags,
            const xm_graph_t* g, xm_plan_t** out);
/* JSON description: vertex order, levels and their constraints, reuse
 * sources, leaf groups and product terms, inclusion groups, the exact
 * minimum constraint cover and Algorithm 1's greedy cover.  Writes at most
 * cap bytes including the terminating NUL; *needed (nullable) receives the
 * full length + 1.  Returns XM_ERR_INVALID if cap is too small. */
int xm_plan_describe(const xm_plan_t* p, char* json, size_t cap, size_t* needed);
/* The pattern vertex the plan starts from (images of it are the roots). */
int xm_plan_root_vertex(const xm_plan_t* p);
int xm_free_plan(xm_plan_t* p);

/* Algorithmic work of plan p on a graph given as HOST CSR arrays (same rules
 * as xm_load_graph): a host computation for statistics only, it returns no
 * count.  It walks the plan's partial matches and sums, per partial match
 * and level, the length of the base list and of every list probed for
 * membership (with section 5.2's reuse the reused candidate set is the
 * base).  out[0] = adjacency elements intersected, out[1] = list fetches,
 * out[2] = partial matches of the enumerated levels, out[3] = roots that
 * pass the start vertex's degree constraint.  roots (nullable, host array)
 * limits the start vertex's images.  threads: host worker threads (0 = 1).
 * max_partial > 0 stops the walk once the partial matches seen plus the
 * elements counted / 256 pass it; the call then returns 1 (figures are
 * partial sums) instead of XM_OK. */
int xm_plan_work(uint32_t n, const uint32_t* out_off, const uint32_t* out_adj,
                 const uint32_t* in_off, const uint32_t* in_adj, const xm_plan_t* p,
                 const uint32_t* roots, uint32_t n_roots, uint32_t threads,
                 uint64_t max_partial, uint64_t out[4]);

/* Memory operations the count kernel issues for plan p on a graph given as
 * HOST CSR arrays (same rules as xm_load_graph), for roofline accounting: a
 * host computation that returns no count.  It walks the same partial matches
 * as xm_plan_work (Algorithm 2's exploration with section 5.2's reuse and
 * section 5.3's leaf counting) and counts, per partial match, what the
 * kernel's candidate tests read as issued: the elements of each scanned
 * base list, offset pairs, degree pairs, one word per membership test in a
 * list of at least row_min elements (a dense row; 0 = no rows), the loads of
 * a binary search otherwise (tests stop at the first failing list), and the
 * partial matches written and their ancestor chains read back.  It assumes
 * every window holds whole candidate sets (no hub sub-ranges or donated
 * prefixes).  out[XM_TRAFFIC_WORDS]:
 *   [0] base elements scanned (4 B each)     [1] offset pairs read (8 B)
 *   [2] degree classes read (1 B)             [3] dense-row words tested (4 B)
 *   [4] sorted-list searches                  [5] words those searches load (4 B)
 *   [6] partial matches written (8 B: node, parent)
 *   [7] words of ancestor chains read back (4 B)
 *   [8] roots passing the start vertex's degree filter
 *   [9] adjacency elements intersected (merge model, as xm_plan_work out[0])
 * roots, threads, max_partial and the return value as for xm_plan_work. */
#define XM_TRAFFIC_WORDS 10
int xm_plan_traffic(uint32_t n, const uint32_t* out_off, const uint32_t* out_adj,
                    const uint32_t* in_off, const uint32_t* in_adj, const xm_plan_t* p,
                    const uint32_t* roots, uint32_t n_roots, uint32_t row_min, uint32_t threads,
                    uint64_t max_partial, uint64_t out[XM_TRAFFIC_WORDS]);

/* ----------------------------------------------------------------------------
 * Counting (Algorithm 2; sections 5.2-5.3).
 *
 * Counts every plan in plans[0..n_plans) against g in ONE persistent kernel
 * launch (batched form) on hip_stream.  n_plans = 1 is the plain form;
 * n_plans is at most 65535.  While some waves have run out of queued work,
 * waves in the middle of a task hand unstarted partial matches (with their
 * bound prefix) to them through a device queue (work donation), so one heavy
 * root does not leave the rest of the device idle.
 *
 * counts_dev: caller device buffer of 2*n_plans uint64: (lo, hi) of the
 *             unsigned 128-bit count of plan i at [2i], [2i+1].
 * status_dev: caller device buffer of n_plans int32: XM_OK, XM_ERR_OVERFLOW
 *             (total exceeded 2^128 - 1; counts then wrap),
 *             XM_ERR_CANCELLED, or XM_ERR_INVALID (an internal consistency
 *             check of the launch failed; counts are then not valid).
 * workspace:  caller device buffer of at least xm_workspace_size(...) bytes,
 *             same n_plans, plans and opts.  Its contents are scratch; the
 *             call initialises what it needs on the stream.  Calls that share
 *             one workspace must not overlap in time.
 * opts (nullable): see xm_count_opts.  Fields left 0 take defaults.
 * Returns after enqueueing; results are ready when hip_stream completes.
 * ------------------------------------------------------------------------- */
typedef struct xm_count_opts {
    uint32_t struct_size;   /* sizeof(xm_count_opts) */
    uint32_t flags;         /* reserved, must be 0 */
    uint32_t chunk;         /* roots taken per work grab (<= 64; default 0: about
                               64 root tasks per resident wave, i.e.
                               ceil(roots x plans / (waves x 64)) clamped to 1..64) */
    uint32_t split;         /* a root whose first-level candidate list has L1
                               entries is split into stealable sub-ranges of
                               min(split, split_work / L1) entries (at least 1)
                               when L1 exceeds that size (default 64, >= 64);
                               for a plan with one enumerated level below the
                               root, 8 x split (at most cap) and 16 x split_work */
    uint32_t cap;           /* per-level candidate buffer entries (default 4096,
                               at least split) */
    uint32_t waves_per_cu;  /* resident waves per compute unit, 4..32 (default:
                               as many as LDS allows, at most 32; when that is
                               fewer than 24, 12 or as many as LDS allows).
                               Launches of at most 12 waves per CU run a build
                               of the count kernel that keeps all its state in
                               registers; larger ones a build limited to 64
                               VGPRs that spills some of it. */
    /* root subset: device array of n_roots node ids (< n, distinct); when
       non-NULL only these nodes are tried as images of the plan's start
       vertex (xm_plan_root_vertex).  Counts are then exact partial sums.
       Plans with symmetry breaking are refused here (XM_ERR_INVALID) unless
       they were built with a forced start vertex (XM_PLAN_ROOT). */
    const uint32_t* roots_dev;
    uint32_t n_roots;
    uint32_t reserved0;
    /* cancel flag: int32 the device can read (device memory, or pinned host
       memory to raise it while the launch runs); each wave polls it on every
       32nd task it takes and every 16 level windows of a task, and stops
       once it is nonzero.  Every plan of
       the launch then reports XM_ERR_CANCELLED and its count is partial. */
    const int32_t* cancel_dev;
    uint32_t split_work;    /* see split (default 4096, >= 4096) */
    /* single-leaf intersections whose two lists are both at least merge_min
       long (default 0xFFFFFFFF: off) and within merge_ratio of each
       other (default 16) are counted by a wave-cooperative merge instead of
       per-element binary search. */
    uint32_t merge_min;
    uint32_t merge_ratio;
    /* Profiling (nullable hipEvent_t): recorded on hip_stream immediately
       before and after the count kernel itself, so its duration excludes the
       small set-up and status kernels. */
    void* ev_kernel_start;
    void* ev_kernel_stop;
    /* Host copy of roots_dev (nullable; read only when struct_size covers
       it).  With it the split-task queue is sized from the subset's own
       degrees; without it every subset root is assumed to have the longest
       list in the graph, which can coarsen the hub splits. */
    const uint32_t* roots_host;
    /* Listing (section 5.3's result generation, written out): when list_dev
       is non-NULL, every embedding found is also written as k uint32 node
       ids in pattern-vertex order (row i at list_dev[i*k .. i*k+k)), rows in
       no particular order, up to list_cap rows; *list_count_dev (device,
       zeroed by the launch) receives the number of embeddings found, which
       may exceed list_cap (then only list_cap rows were written).  Needs
       n_plans = 1 and a plan whose leaf group is a single vertex (every
       XM_PLAN_UNREDUCED plan) without symmetry breaking; XM_ERR_INVALID
       otherwise.  Counts are written as usual. */
    uint32_t* list_dev;
    uint64_t list_cap;
    unsigned long long* list_count_dev;
} xm_count_opts;

size_t xm_workspace_size(const xm_graph_t* g, uint32_t n_plans,
                         const xm_plan_t* const* plans, const xm_count_opts* opts);
int xm_count(const xm_graph_t* g, uint32_t n_plans, const xm_plan_t* const* plans,
             const xm_count_opts* opts, void* workspace, size_t ws_bytes,
             uint64_t* counts_dev, int32_t* status_dev, void* hip_stream);

/* xm_count without a workspace, for callers that cannot allocate device
 * memory (code under HIP-graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The workspace is a fixed array of
 * XM_STATIC_SCRATCH_BYTES in device memory that the library holds on every
 * device it runs on until the process ends; the call allocates nothing (plan
 * descriptors travel to the device in kernel arguments).  Same arguments and
 * results as xm_count otherwise; fields of opts left 0 take smaller defaults
 * here (cap 256, 4 waves per compute unit).  A launch whose workspace
 * (xm_workspace_size with those defaults) would pass the array fails with
 * XM_ERR_WORKSPACE before anything is enqueued.  Every call on one device
 * shares that device's array: calls that overlap in time on one device race
 * and give wrong counts; the call itself clears what must start at zero. */
#define XM_STATIC_SCRATCH_BYTES (64ull << 20)
int xm_count_static(const xm_graph_t* g, uint32_t n_plans, const xm_plan_t* const* plans,
                    const xm_count_opts* opts, uint64_t* counts_dev, int32_t* status_dev, void* hip_stream);

/* ----------------------------------------------------------------------------
 * HIP-graph form of xm_count: records the same launches once (captured on
 * hip_stream) and instantiates them; xm_exec_launch replays them with the
 * arguments given at capture (same workspace, counts, status, plans).  The
 * caller keeps every buffer alive until xm_free_exec.
 * ------------------------------------------------------------------------- */
int xm_count_capture(const xm_graph_t* g, uint32_t n_plans, const xm_plan_t* const* plans,
                     const xm_count_opts* opts, void* workspace, size_t ws_bytes,
                     uint64_t* counts_dev, int32_t* status_dev, void* hip_stream,
                     xm_exec_t** out);
int xm_exec_launch(xm_exec_t* e, void* hip_stream);
int xm_free_exec(xm_exec_t* e);

const char* xm_strerror(int code);
const char* xm_last_error(void);
/* Library version string. */
const char* xm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* XMINER_H */
