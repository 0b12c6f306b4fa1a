/*
 * The oracle: plain, slow, obviously correct counting of pattern embeddings.
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may call it.  It shares no code with the HIP library.
 *
 * What it computes (the paper, section 2, Definitions 2.1 and 2.2 and the
 * constraint set C = V u E; result generation, section 5.3):
 *
 *   count(P, G) = #{ phi : V_P -> V  injective  |  for every pattern arc (u, w):
 *                    (phi(u), phi(w)) is an arc of G }
 *
 * i.e. non-induced, direction-preserving, labelled embeddings, not divided by
 * the automorphism count of P.  Matches must be oriented the same as the
 * pattern (section 2, opening paragraph); the only constraints are vertices
 * and edges, so extra data arcs are allowed; a visited mark per bound node
 * makes maps injective (Algorithm 2, the recursion with visited checks).
 *
 * Method: single-threaded depth-first backtracking over all injective maps with
 * no pattern reduction.  Vertex order: the pattern vertex of largest total
 * degree first (ties: lowest id), then repeatedly the unbound vertex with the
 * most arcs to bound vertices (ties: larger degree, then lowest id).  Level i
 * draws candidates from the adjacency list of its first bound neighbour in the
 * required direction, rejects nodes already used, and checks every other arc
 * to a bound vertex by binary search.  Totals are unsigned 128-bit.
 *
 * Mode A counts one per complete map.  Mode B is allowed only where mode A is
 * too slow: at the last vertex, when it has exactly one arc to the bound
 * vertices, it adds |L| minus the bound nodes found in L instead of walking L.
 *
 * Threads only split the list of root images (images of the first vertex)
 * for timing; the per-root algorithm is the same.
 *
 * Listing (xmo_list) walks the same maps in mode A, single-threaded, and
 * writes each one as phi(0), ..., phi(k-1) in pattern-vertex order (the
 * embeddings of section 5.3's result generation, written out instead of
 * counted), up to a capacity; the total is always exact.
 *
 * The oracle reads only the out-CSR and builds its own sorted in-lists.
 *
 * Parity unpinned: the 128-bit accumulation of totals above 2^64 (no
 * enumeration reaches such a total in reasonable time, and no stored value
 * depends on it; the GPU's 128-bit path is pinned by a closed form instead).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

typedef unsigned __int128 u128;

#define MAXK 7

typedef struct {
    uint32_t n;
    const uint32_t *out_off, *out_adj;
    uint32_t *in_off, *in_adj;   /* built here */
} ograph;

typedef struct {
    int k;
    int order[MAXK];           /* level -> pattern vertex */
    /* for level i: list of (j, dir) constraints to earlier levels j.
       dir 0: candidate must be in out(phi(v_j)); dir 1: in in(phi(v_j)). */
    int ncons[MAXK];
    int cons_j[MAXK][2 * MAXK];
    int cons_dir[MAXK][2 * MAXK];
} oplan;

static int has_arc(const uint32_t *off, const uint32_t *adj, uint32_t u, uint32_t x) {
    uint32_t lo = off[u], hi = off[u + 1];
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (adj[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo < off[u + 1] && adj[lo] == x;
}

static int build_in(ograph *g) {
    uint32_t n = g->n;
    uint64_t m = g->out_off[n];
    g->in_off = (uint32_t *)calloc((size_t)n + 1, sizeof(uint32_t));
    g->in_adj = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    uint32_t *fill = (uint32_t *)calloc((size_t)n + 1, sizeof(uint32_t));
    if (!g->in_off || !g->in_adj || !fill) { free(fill); return -1; }
    for (uint64_t e = 0; e < m; e++) g->in_off[g->out_adj[e] + 1]++;
    for (uint32_t v = 0; v < n; v++) g->in_off[v + 1] += g->in_off[v];
    /* sources visited in increasing order => each in-list comes out sorted */
    for (uint32_t u = 0; u < n; u++)
        for (uint32_t e = g->out_off[u]; e < g->out_off[u + 1]; e++) {
            uint32_t v = g->out_adj[e];
            g->in_adj[g->in_off[v] + fill[v]++] = u;
        }
    free(fill);
    return 0;
}

static int make_plan(int k, int n_arcs, const uint8_t *arcs, int root_vertex, oplan *p) {
    int adj_out[MAXK][MAXK] = {{0}};
    int deg[MAXK] = {0};
    if (k < 1 || k > MAXK) return -1;
    for (int a = 0; a < n_arcs; a++) {
        int s = arcs[2 * a], d = arcs[2 * a + 1];
        if (s >= k || d >= k || s == d) return -1;
        if (!adj_out[s][d]) { adj_out[s][d] = 1; deg[s]++; deg[d]++; }
    }
    int bound[MAXK] = {0};
    int first = 0;
    for (int v = 1; v < k; v++) if (deg[v] > deg[first]) first = v;
    if (root_vertex >= 0) {
        if (root_vertex >= k) return -1;
        first = root_vertex;
    }
    p->k = k;
    p->order[0] = first;
    bound[first] = 1;
    for (int i = 1; i < k; i++) {
        int best = -1, best_c = -1;
        for (int v = 0; v < k; v++) {
            if (bound[v]) continue;
            int c = 0;
            for (int u = 0; u < k; u++)
                if (bound[u]) c += adj_out[u][v] + adj_out[v][u];
            if (c > best_c || (c == best_c && deg[v] > deg[best])) { best = v; best_c = c; }
        }
        if (best_c <= 0) return -2; /* not connected */
        p->order[i] = best;
        bound[best] = 1;
    }
    for (int i = 0; i < k; i++) {
        int v = p->order[i];
        p->ncons[i] = 0;
        for (int j = 0; j < i; j++) {
            int u = p->order[j];
            if (adj_out[u][v]) { p->cons_j[i][p->ncons[i]] = j; p->cons_dir[i][p->ncons[i]++] = 0; }
            if (adj_out[v][u]) { p->cons_j[i][p->ncons[i]] = j; p->cons_dir[i][p->ncons[i]++] = 1; }
        }
    }
    return 0;
}

typedef struct {
    const ograph *g;
    const oplan *p;
    int mode;
    uint32_t phi[MAXK];
    /* listing: complete maps go to out[cap][k] (pattern-vertex order) */
    uint32_t *out;
    uint64_t cap, listed;
} ostate;

static u128 extend(ostate *s, int i) {
    const ograph *g = s->g;
    const oplan *p = s->p;
    if (i == p->k) {
        if (s->out) {
            if (s->listed < s->cap)
                for (int t = 0; t < p->k; t++) s->out[s->listed * (uint64_t)p->k + p->order[t]] = s->phi[t];
            s->listed++;
        }
        return 1;
    }
    /* candidate list from the first constraint */
    int j0 = p->cons_j[i][0], d0 = p->cons_dir[i][0];
    uint32_t a = s->phi[j0];
    const uint32_t *off = d0 ? g->in_off : g->out_off;
    const uint32_t *adj = d0 ? g->in_adj : g->out_adj;
    uint32_t lo = off[a], hi = off[a + 1];
    if (s->mode == 1 && i == p->k - 1 && p->ncons[i] == 1) {
        u128 c = hi - lo;
        for (int t = 0; t < i; t++)
            if (has_arc(off, adj, a, s->phi[t])) c -= 1;
        return c;
    }
    u128 total = 0;
    for (uint32_t e = lo; e < hi; e++) {
        uint32_t x = adj[e];
        int ok = 1;
        for (int t = 0; t < i && ok; t++) if (s->phi[t] == x) ok = 0;
        for (int c = 1; c < p->ncons[i] && ok; c++) {
            uint32_t b = s->phi[p->cons_j[i][c]];
            if (p->cons_dir[i][c] == 0) ok = has_arc(g->out_off, g->out_adj, b, x);
            else ok = has_arc(g->out_off, g->out_adj, x, b);
        }
        if (!ok) continue;
        s->phi[i] = x;
        total += extend(s, i + 1);
    }
    return total;
}

typedef struct {
    const ograph *g;
    const oplan *p;
    int mode;
    const uint32_t *roots;
    uint64_t n_roots;
    uint64_t *per_root;
    volatile uint64_t *cursor;
    u128 sum;
} oworker;

static void *worker(void *arg) {
    oworker *w = (oworker *)arg;
    ostate s;
    s.g = w->g; s.p = w->p; s.mode = w->mode;
    s.out = NULL; s.cap = s.listed = 0;
    w->sum = 0;
    for (;;) {
        uint64_t base = __atomic_fetch_add(w->cursor, 64, __ATOMIC_RELAXED);
        if (base >= w->n_roots) break;
        uint64_t end = base + 64 < w->n_roots ? base + 64 : w->n_roots;
        for (uint64_t r = base; r < end; r++) {
            uint32_t x = w->roots ? w->roots[r] : (uint32_t)r;
            u128 c = 0;
            if (x < w->g->n) {
                s.phi[0] = x;
                c = extend(&s, 1);
            }
            w->sum += c;
            if (w->per_root) {
                w->per_root[2 * r] = (uint64_t)c;
                w->per_root[2 * r + 1] = (uint64_t)(c >> 64);
            }
        }
    }
    return NULL;
}

/*
 * Count the embeddings of the pattern (k vertices, n_arcs arcs as (src, dst)
 * byte pairs) in the graph given by its out-CSR.  roots (nullable) restricts
 * the image of the first pattern vertex in the oracle's own order to the
 * listed nodes; the sum over all nodes is the full count, so per-root counts
 * of any subset are exact parts of it.  The first vertex is reported through
 * first_vertex (nullable); root_vertex >= 0 forces which pattern vertex is
 * first (the one the roots list restricts).  Returns 0, or -1 on bad input, -2 if the pattern
 * is not connected, -3 on allocation failure.
 */
static int count_on(const ograph *g, int k, int n_arcs, const uint8_t *arcs,
                    const uint32_t *roots, uint64_t n_roots, int mode, int threads,
                    uint64_t *total_lo, uint64_t *total_hi,
                    uint64_t *per_root, int root_vertex, int *first_vertex) {
    oplan p;
    int rc = make_plan(k, n_arcs, arcs, root_vertex, &p);
    if (rc) return rc;
    if (first_vertex) *first_vertex = p.order[0];
    if (!roots) n_roots = g->n;
    if (threads < 1) threads = 1;
    volatile uint64_t cursor = 0;
    oworker *ws = (oworker *)calloc((size_t)threads, sizeof(oworker));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    if (!ws || !tid) { free(ws); free(tid); return -3; }
    for (int t = 0; t < threads; t++) {
        ws[t].g = g; ws[t].p = &p; ws[t].mode = mode;
        ws[t].roots = roots; ws[t].n_roots = n_roots;
        ws[t].per_root = per_root; ws[t].cursor = &cursor;
    }
    if (threads == 1) {
        worker(&ws[0]);
    } else {
        for (int t = 0; t < threads; t++) pthread_create(&tid[t], NULL, worker, &ws[t]);
        for (int t = 0; t < threads; t++) pthread_join(tid[t], NULL);
    }
    u128 total = 0;
    for (int t = 0; t < threads; t++) total += ws[t].sum;
    *total_lo = (uint64_t)total;
    *total_hi = (uint64_t)(total >> 64);
    free(ws); free(tid);
    return 0;
}

int xmo_count(uint32_t n, const uint32_t *out_off, const uint32_t *out_adj,
              int k, int n_arcs, const uint8_t *arcs,
              const uint32_t *roots, uint64_t n_roots,
              int mode, int threads,
              uint64_t *total_lo, uint64_t *total_hi,
              uint64_t *per_root, int root_vertex, int *first_vertex) {
    ograph g;
    g.n = n; g.out_off = out_off; g.out_adj = out_adj;
    if (build_in(&g)) return -3;
    int rc = count_on(&g, k, n_arcs, arcs, roots, n_roots, mode, threads, total_lo, total_hi, per_root,
                      root_vertex, first_vertex);
    free(g.in_off); free(g.in_adj);
    return rc;
}

/*
 * The same counts on a graph prepared once: xmo_prepare builds the in-lists
 * of the out-CSR (which must stay alive and unchanged) and returns a handle
 * (NULL on allocation failure); xmo_count_prepared counts exactly as
 * xmo_count with the in-lists built already (graph pre-processing, excluded
 * from timings); xmo_release frees the handle.
 */
void *xmo_prepare(uint32_t n, const uint32_t *out_off, const uint32_t *out_adj) {
    ograph *g = (ograph *)calloc(1, sizeof(ograph));
    if (!g) return NULL;
    g->n = n; g->out_off = out_off; g->out_adj = out_adj;
    if (build_in(g)) { free(g->in_off); free(g->in_adj); free(g); return NULL; }
    return g;
}

int xmo_count_prepared(const void *h, int k, int n_arcs, const uint8_t *arcs,
                       const uint32_t *roots, uint64_t n_roots, int mode, int threads,
                       uint64_t *total_lo, uint64_t *total_hi,
                       uint64_t *per_root, int root_vertex, int *first_vertex) {
    if (!h) return -1;
    return count_on((const ograph *)h, k, n_arcs, arcs, roots, n_roots, mode, threads, total_lo, total_hi,
                    per_root, root_vertex, first_vertex);
}

void xmo_release(void *h) {
    ograph *g = (ograph *)h;
    if (!g) return;
    free(g->in_off); free(g->in_adj); free(g);
}

/*
 * List the embeddings: out (nullable when cap is 0) receives up to cap maps,
 * k uint32 each, phi of pattern vertex 0..k-1; *total receives the exact
 * number of embeddings (lo, hi).  roots / root_vertex as in xmo_count.
 * Returns as xmo_count.
 */
int xmo_list(uint32_t n, const uint32_t *out_off, const uint32_t *out_adj,
             int k, int n_arcs, const uint8_t *arcs,
             const uint32_t *roots, uint64_t n_roots, int root_vertex,
             uint32_t *out, uint64_t cap, uint64_t *total_lo, uint64_t *total_hi) {
    oplan p;
    int rc = make_plan(k, n_arcs, arcs, root_vertex, &p);
    if (rc) return rc;
    ograph g;
    g.n = n; g.out_off = out_off; g.out_adj = out_adj;
    if (build_in(&g)) return -3;
    if (!roots) n_roots = n;
    ostate s;
    s.g = &g; s.p = &p; s.mode = 0;
    s.out = out; s.cap = out ? cap : 0; s.listed = 0;
    u128 total = 0;
    for (uint64_t r = 0; r < n_roots; r++) {
        uint32_t x = roots ? roots[r] : (uint32_t)r;
        if (x >= n) continue;
        s.phi[0] = x;
        total += extend(&s, 1);
    }
    *total_lo = (uint64_t)total;
    *total_hi = (uint64_t)(total >> 64);
    free(g.in_off); free(g.in_adj);
    return 0;
}
