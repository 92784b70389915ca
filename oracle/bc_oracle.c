/*
 * bc_oracle.c -- CPU oracle for Brandes betweenness centrality.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * reference the GPU library is checked against.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header or table with the GPU library.
 *
 * What it computes (paper, Section "Background"):
 *   Eq. 1    BC[v] = sum over s != v != t of sigma_st(v) / sigma_st
 *   Eq. 2    delta_s(v) = sum over u with v in P_s(u) of
 *                         sigma_sv / sigma_su * (1 + delta_s(u))
 *            BC[v] = sum over s != v of delta_s(v)
 * written out from those definitions, one source at a time:
 *   1. distances d(s, .) by breadth-first search along arcs (the graphs are
 *      unweighted);
 *   2. path counts from the recurrence sigma_ss = 1 and, for t != s,
 *      sigma_st = sum of sigma_sv over the in-neighbours v of t (arcs v -> t)
 *      with d(s, v) = d(s, t) - 1 (every shortest s-t path enters t from such
 *      a v, and each of them continues exactly the sigma_sv shortest s-v
 *      paths), taking vertices in non-decreasing distance;
 *   3. Eq. 2 for each vertex v as a sum over its successors u (out-neighbours
 *      with d(s, u) = d(s, v) + 1), taking vertices in non-increasing
 *      distance so that every delta_s(u) on the right is final;
 *   4. BC[v] += delta_s(v) for every reached v != s.
 * An undirected graph is the directed graph with both arcs of every edge
 * (the paper converts every input to that form, Section "Experiments and
 * Results"): its adjacency serves as both the out- and the in-adjacency.
 *
 * Readings where the paper is silent or loose (each one is listed in the
 * design notes of the repository):
 *   - Sums are over ordered pairs, so for an undirected graph every unordered
 *     pair is counted twice.  The raw sum over the given sources is returned.
 *   - v = s is excluded from BC (Eq. 2's outer sum has s != v); vertices not
 *     reached from s receive nothing (pairs with sigma_st = 0 contribute 0).
 *   - The predecessor set P_s(u) of Eq. 2 is the set of neighbours v of u
 *     with d(s, v) = d(s, u) - 1; it is not stored.
 *   - Path counts use uint64.  A source whose exact count exceeds 2^64 - 1 is
 *     flagged F64 and recomputed entirely in x87 long double (64-bit
 *     mantissa, 15-bit exponent); its dependencies are rounded to double at
 *     the end.  Every partial sum of a path count is a sum of non-negative
 *     terms no larger than the final count, so a carry out of 64 bits occurs
 *     exactly when some count exceeds 2^64 - 1.
 *   - Each term of Eq. 2 is evaluated as (sigma_sv / sigma_su) *
 *     (1 + delta_s(u)) and the terms of one vertex are added in adjacency
 *     order, in double (U64 mode) or long double (F64 mode).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_MEM 2

typedef struct {
    int32_t n;
    const int64_t *row_ptr; /* out-arcs: int64 copy for uniform indexing */
    const int32_t *col;
    const int64_t *in_row_ptr; /* in-arcs (the same arrays for an undirected graph) */
    const int32_t *in_col;
    int32_t *dist;           /* d(s, v), -1 = not reached */
    int32_t *order;          /* reached vertices in breadth-first order (non-decreasing d) */
    int64_t n_reached;
    uint64_t *sig_u;         /* sigma_sv, U64 mode */
    long double *sig_l;      /* sigma_sv, F64 mode */
    double *dep_d;           /* delta_s(v), U64 mode */
    long double *dep_l;      /* delta_s(v), F64 mode */
} orc_ws;

/* Step 1: breadth-first search from s.  The FIFO order is kept: it lists
 * the reached vertices by non-decreasing distance. */
static void distances(orc_ws *w, int32_t s)
{
    for (int32_t i = 0; i < w->n; ++i) w->dist[i] = -1;
    int64_t head = 0, tail = 0;
    w->order[tail++] = s;
    w->dist[s] = 0;
    while (head < tail) {
        const int32_t v = w->order[head++];
        for (int64_t e = w->row_ptr[v]; e < w->row_ptr[v + 1]; ++e) {
            const int32_t x = w->col[e];
            if (w->dist[x] < 0) {
                w->dist[x] = w->dist[v] + 1;
                w->order[tail++] = x;
            }
        }
    }
    w->n_reached = tail;
}

/* Step 2: sigma_st = sum over the neighbours one step closer to s.  Returns
 * 1 when a count does not fit in uint64 (use_ld == 0 only). */
static int path_counts(orc_ws *w, int use_ld)
{
    int overflow = 0;
    for (int64_t k = 0; k < w->n_reached; ++k) {
        const int32_t t = w->order[k];
        if (k == 0) { /* t = s */
            if (use_ld) w->sig_l[t] = 1.0L; else w->sig_u[t] = 1;
            continue;
        }
        uint64_t su = 0;
        long double sl = 0.0L;
        for (int64_t e = w->in_row_ptr[t]; e < w->in_row_ptr[t + 1]; ++e) {
            const int32_t v = w->in_col[e];
            if (w->dist[v] != w->dist[t] - 1) continue;
            if (use_ld) {
                sl += w->sig_l[v];
            } else if (__builtin_add_overflow(su, w->sig_u[v], &su)) {
                overflow = 1;
            }
        }
        if (use_ld) w->sig_l[t] = sl; else w->sig_u[t] = su;
    }
    return overflow;
}

/* Step 3: Eq. 2, delta_s(v) = sum over successors u of
 * sigma_sv / sigma_su * (1 + delta_s(u)), vertices by non-increasing distance. */
static void dependencies(orc_ws *w, int use_ld)
{
    for (int64_t k = w->n_reached - 1; k >= 0; --k) {
        const int32_t v = w->order[k];
        double dd = 0.0;
        long double dl = 0.0L;
        for (int64_t e = w->row_ptr[v]; e < w->row_ptr[v + 1]; ++e) {
            const int32_t u = w->col[e];
            if (w->dist[u] != w->dist[v] + 1) continue; /* u is not a successor of v */
            if (use_ld) dl += (w->sig_l[v] / w->sig_l[u]) * (1.0L + w->dep_l[u]);
            else dd += ((double)w->sig_u[v] / (double)w->sig_u[u]) * (1.0 + w->dep_d[u]);
        }
        if (use_ld) w->dep_l[v] = dl; else w->dep_d[v] = dd;
    }
}

static int64_t *rp_copy(int32_t n, const int32_t *rp32, const int64_t *rp64)
{
    int64_t *rp = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (rp)
        for (int64_t i = 0; i <= n; ++i) rp[i] = rp64 ? rp64[i] : (int64_t)rp32[i];
    return rp;
}

/* in_* == NULL: undirected, the out-adjacency is also the in-adjacency. */
static int ws_init(orc_ws *w, int32_t n, const int32_t *row_ptr32, const int64_t *row_ptr64,
                   const int32_t *col, const int32_t *in_rp32, const int64_t *in_rp64, const int32_t *in_col)
{
    memset(w, 0, sizeof(*w));
    w->n = n;
    w->row_ptr = rp_copy(n, row_ptr32, row_ptr64);
    if (!w->row_ptr) return ORC_ERR_MEM;
    w->col = col;
    if (in_rp32 || in_rp64) {
        w->in_row_ptr = rp_copy(n, in_rp32, in_rp64);
        if (!w->in_row_ptr) return ORC_ERR_MEM;
        w->in_col = in_col;
    } else {
        w->in_row_ptr = w->row_ptr;
        w->in_col = col;
    }
    const size_t m = (size_t)(n > 0 ? n : 1);
    w->dist = (int32_t *)malloc(sizeof(int32_t) * m);
    w->order = (int32_t *)malloc(sizeof(int32_t) * m);
    w->sig_u = (uint64_t *)calloc(m, sizeof(uint64_t));
    w->sig_l = (long double *)calloc(m, sizeof(long double));
    w->dep_d = (double *)calloc(m, sizeof(double));
    w->dep_l = (long double *)calloc(m, sizeof(long double));
    if (!w->dist || !w->order || !w->sig_u || !w->sig_l || !w->dep_d || !w->dep_l) return ORC_ERR_MEM;
    return ORC_OK;
}

static void ws_free(orc_ws *w)
{
    if (w->in_row_ptr != w->row_ptr) free((void *)w->in_row_ptr);
    free((void *)w->row_ptr);
    free(w->dist); free(w->order);
    free(w->sig_u); free(w->sig_l); free(w->dep_d); free(w->dep_l);
}

/* One source: distances, path counts (uint64, else long double), Eq. 2.
 * Returns the mode (0 = U64, 1 = F64). */
static int one_source(orc_ws *w, int32_t s)
{
    distances(w, s);
    int mode = 0;
    if (path_counts(w, 0)) {
        mode = 1;
        path_counts(w, 1);
    }
    dependencies(w, mode);
    return mode;
}

/*
 * BC over a source list of a directed graph: out-arcs (row_ptr*, col) and
 * in-arcs (in_row_ptr*, in_col, the transpose; both NULL for an undirected
 * graph, whose adjacency is used for both).  sources == NULL means every
 * vertex 0..n-1 in order.  bc[0..n) receives the raw ordered-pair sums (it
 * is overwritten, not accumulated), sources taken in list order.  modes
 * (nullable) receives 0/1 per source.  Row offsets are given either as int32
 * or int64; pass NULL for the other.
 */
int oracle_bc_dir(int32_t n, const int32_t *row_ptr32, const int64_t *row_ptr64, const int32_t *col,
                  const int32_t *in_rp32, const int64_t *in_rp64, const int32_t *in_col,
                  const int32_t *sources, int64_t n_sources, double *bc, int32_t *modes)
{
    if (n < 0 || (!row_ptr32 && !row_ptr64) || !bc) return ORC_ERR_ARG;
    orc_ws w;
    if (ws_init(&w, n, row_ptr32, row_ptr64, col, in_rp32, in_rp64, in_col) != ORC_OK) { ws_free(&w); return ORC_ERR_MEM; }
    for (int32_t i = 0; i < n; ++i) bc[i] = 0.0;
    const int64_t ns = sources ? n_sources : n;
    for (int64_t k = 0; k < ns; ++k) {
        const int32_t s = sources ? sources[k] : (int32_t)k;
        if (s < 0 || s >= n) { ws_free(&w); return ORC_ERR_ARG; }
        const int mode = one_source(&w, s);
        if (modes) modes[k] = mode;
        for (int64_t i = 1; i < w.n_reached; ++i) { /* order[0] is s itself */
            const int32_t v = w.order[i];
            bc[v] += mode ? (double)w.dep_l[v] : w.dep_d[v];
        }
    }
    ws_free(&w);
    return ORC_OK;
}

/* Undirected graphs: the adjacency is both the out- and the in-adjacency. */
int oracle_bc(int32_t n, const int32_t *row_ptr32, const int64_t *row_ptr64, const int32_t *col,
              const int32_t *sources, int64_t n_sources, double *bc, int32_t *modes)
{
    return oracle_bc_dir(n, row_ptr32, row_ptr64, col, NULL, NULL, NULL, sources, n_sources, bc, modes);
}

/*
 * Per-source detail (in-arcs as in oracle_bc_dir; NULL = undirected).
 * d: int32[n] (-1 = unreached).  sigma_u64: uint64[n]
 * (valid in U64 mode; zero in F64 mode).  sigma_ld: long double[n] (the F64
 * mode counts; in U64 mode the exact counts converted).  delta: double[n],
 * delta_s(v) from Eq. 2 for reached v (for v = s the same sum over its
 * successors, which BC excludes), 0 for unreached v.  n_levels: number of
 * distinct distances (largest d + 1).  Any output pointer may be NULL.
 * Returns the mode (0/1) or a negative error.
 */
int oracle_source_dir(int32_t n, const int32_t *row_ptr32, const int64_t *row_ptr64, const int32_t *col,
                      const int32_t *in_rp32, const int64_t *in_rp64, const int32_t *in_col,
                      int32_t s, int32_t *d, uint64_t *sigma_u64, long double *sigma_ld, double *delta,
                      int32_t *n_levels)
{
    if (n <= 0 || s < 0 || s >= n || (!row_ptr32 && !row_ptr64)) return -ORC_ERR_ARG;
    orc_ws w;
    if (ws_init(&w, n, row_ptr32, row_ptr64, col, in_rp32, in_rp64, in_col) != ORC_OK) { ws_free(&w); return -ORC_ERR_MEM; }
    const int mode = one_source(&w, s);
    for (int32_t v = 0; v < n; ++v) {
        const int reached = w.dist[v] >= 0;
        if (d) d[v] = w.dist[v];
        if (sigma_u64) sigma_u64[v] = (mode || !reached) ? 0 : w.sig_u[v];
        if (sigma_ld) sigma_ld[v] = !reached ? 0.0L : (mode ? w.sig_l[v] : (long double)w.sig_u[v]);
        if (delta) delta[v] = !reached ? 0.0 : (mode ? (double)w.dep_l[v] : w.dep_d[v]);
    }
    if (n_levels) *n_levels = w.dist[w.order[w.n_reached - 1]] + 1;
    ws_free(&w);
    return mode;
}

int oracle_source(int32_t n, const int32_t *row_ptr32, const int64_t *row_ptr64, const int32_t *col,
                  int32_t s, int32_t *d, uint64_t *sigma_u64, long double *sigma_ld, double *delta,
                  int32_t *n_levels)
{
    return oracle_source_dir(n, row_ptr32, row_ptr64, col, NULL, NULL, NULL, s, d, sigma_u64, sigma_ld, delta,
                             n_levels);
}

/* ------------------------------------------------------------------------
 * Weighted graphs.  The paper's forward phase is "a BFS traversal or SSSP
 * calculation" (Section "Background"), and its graph layout keeps edge
 * weights (Section "Space Complexity").  Arc weights here are positive
 * integers (int32 >= 1, aligned with col), so distances are exact int64 and
 * equal-length paths are recognised exactly.  Written out from the same
 * definitions as above, with "one step closer to s" read as
 * d(s, v) + w(v, t) = d(s, t):
 *   1. distances by Dijkstra's method (a binary heap of tentative
 *      distances; a vertex is settled when it leaves the heap with its
 *      final distance), which lists the reached vertices by non-decreasing
 *      distance;
 *   2. sigma_st = sum of sigma_sv over arcs v -> t with d(s, v) + w(v, t) =
 *      d(s, t) (such v are strictly closer, weights being >= 1);
 *   3. Eq. 2 over the arcs v -> u with d(s, v) + w(v, u) = d(s, u), vertices
 *      by non-increasing distance; same mode rule and evaluation order as
 *      the unweighted oracle.
 * ---------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    const int64_t *row_ptr;
    const int32_t *col, *wt;
    const int64_t *in_row_ptr;
    const int32_t *in_col, *in_wt;
    int64_t *dist;           /* -1 = not reached */
    int32_t *order;
    int64_t n_reached;
    unsigned char *done;
    int64_t *heap_d;         /* binary heap of (distance, vertex) pairs, with stale copies */
    int32_t *heap_v;
    int64_t heap_cap;
    uint64_t *sig_u;
    long double *sig_l;
    double *dep_d;
    long double *dep_l;
} orc_wws;

static void heap_push(orc_wws *w, int64_t *size, int64_t d, int32_t v)
{
    int64_t i = (*size)++;
    while (i > 0) {
        const int64_t p = (i - 1) / 2;
        if (w->heap_d[p] < d || (w->heap_d[p] == d && w->heap_v[p] <= v)) break;
        w->heap_d[i] = w->heap_d[p];
        w->heap_v[i] = w->heap_v[p];
        i = p;
    }
    w->heap_d[i] = d;
    w->heap_v[i] = v;
}

static void heap_pop(orc_wws *w, int64_t *size, int64_t *d, int32_t *v)
{
    *d = w->heap_d[0];
    *v = w->heap_v[0];
    const int64_t ld = w->heap_d[--(*size)];
    const int32_t lv = w->heap_v[*size];
    int64_t i = 0;
    for (;;) {
        int64_t c = 2 * i + 1;
        if (c >= *size) break;
        if (c + 1 < *size && (w->heap_d[c + 1] < w->heap_d[c] ||
                              (w->heap_d[c + 1] == w->heap_d[c] && w->heap_v[c + 1] < w->heap_v[c]))) ++c;
        if (ld < w->heap_d[c] || (ld == w->heap_d[c] && lv <= w->heap_v[c])) break;
        w->heap_d[i] = w->heap_d[c];
        w->heap_v[i] = w->heap_v[c];
        i = c;
    }
    w->heap_d[i] = ld;
    w->heap_v[i] = lv;
}

static void wdistances(orc_wws *w, int32_t s)
{
    for (int32_t i = 0; i < w->n; ++i) {
        w->dist[i] = -1;
        w->done[i] = 0;
    }
    int64_t size = 0, k = 0;
    w->dist[s] = 0;
    heap_push(w, &size, 0, s);
    while (size > 0) {
        int64_t d;
        int32_t v;
        heap_pop(w, &size, &d, &v);
        if (w->done[v] || d != w->dist[v]) continue; /* a stale copy */
        w->done[v] = 1;
        w->order[k++] = v;
        for (int64_t e = w->row_ptr[v]; e < w->row_ptr[v + 1]; ++e) {
            const int32_t x = w->col[e];
            const int64_t nd = d + (int64_t)w->wt[e];
            if (!w->done[x] && (w->dist[x] < 0 || nd < w->dist[x])) {
                w->dist[x] = nd;
                heap_push(w, &size, nd, x);
            }
        }
    }
    w->n_reached = k;
}

static int wpath_counts(orc_wws *w, int use_ld)
{
    int overflow = 0;
    for (int64_t k = 0; k < w->n_reached; ++k) {
        const int32_t t = w->order[k];
        if (k == 0) {
            if (use_ld) w->sig_l[t] = 1.0L; else w->sig_u[t] = 1;
            continue;
        }
        uint64_t su = 0;
        long double sl = 0.0L;
        for (int64_t e = w->in_row_ptr[t]; e < w->in_row_ptr[t + 1]; ++e) {
            const int32_t v = w->in_col[e];
            if (w->dist[v] < 0 || w->dist[v] + (int64_t)w->in_wt[e] != w->dist[t]) continue;
            if (use_ld) sl += w->sig_l[v];
            else if (__builtin_add_overflow(su, w->sig_u[v], &su)) overflow = 1;
        }
        if (use_ld) w->sig_l[t] = sl; else w->sig_u[t] = su;
    }
    return overflow;
}

static void wdependencies(orc_wws *w, int use_ld)
{
    for (int64_t k = w->n_reached - 1; k >= 0; --k) {
        const int32_t v = w->order[k];
        double dd = 0.0;
        long double dl = 0.0L;
        for (int64_t e = w->row_ptr[v]; e < w->row_ptr[v + 1]; ++e) {
            const int32_t u = w->col[e];
            if (w->dist[u] != w->dist[v] + (int64_t)w->wt[e]) continue; /* not a successor */
            if (use_ld) dl += (w->sig_l[v] / w->sig_l[u]) * (1.0L + w->dep_l[u]);
            else dd += ((double)w->sig_u[v] / (double)w->sig_u[u]) * (1.0 + w->dep_d[u]);
        }
        if (use_ld) w->dep_l[v] = dl; else w->dep_d[v] = dd;
    }
}

static void wws_free(orc_wws *w)
{
    if (w->in_row_ptr != w->row_ptr) free((void *)w->in_row_ptr);
    free((void *)w->row_ptr);
    free(w->dist); free(w->order); free(w->done); free(w->heap_d); free(w->heap_v);
    free(w->sig_u); free(w->sig_l); free(w->dep_d); free(w->dep_l);
}

static int wws_init(orc_wws *w, int32_t n, const int32_t *rp32, const int64_t *rp64, const int32_t *col,
                    const int32_t *wt, const int32_t *in_rp32, const int64_t *in_rp64, const int32_t *in_col,
                    const int32_t *in_wt)
{
    memset(w, 0, sizeof(*w));
    w->n = n;
    w->row_ptr = rp_copy(n, rp32, rp64);
    if (!w->row_ptr) return ORC_ERR_MEM;
    w->col = col;
    w->wt = wt;
    if (in_rp32 || in_rp64) {
        w->in_row_ptr = rp_copy(n, in_rp32, in_rp64);
        if (!w->in_row_ptr) return ORC_ERR_MEM;
        w->in_col = in_col;
        w->in_wt = in_wt;
    } else {
        w->in_row_ptr = w->row_ptr;
        w->in_col = col;
        w->in_wt = wt;
    }
    const int64_t nnz = w->row_ptr[n];
    for (int64_t e = 0; e < nnz; ++e)
        if (wt[e] < 1) return ORC_ERR_ARG;
    const size_t m = (size_t)(n > 0 ? n : 1);
    w->heap_cap = nnz + 1;
    w->dist = (int64_t *)malloc(sizeof(int64_t) * m);
    w->order = (int32_t *)malloc(sizeof(int32_t) * m);
    w->done = (unsigned char *)malloc(m);
    w->heap_d = (int64_t *)malloc(sizeof(int64_t) * (size_t)w->heap_cap);
    w->heap_v = (int32_t *)malloc(sizeof(int32_t) * (size_t)w->heap_cap);
    w->sig_u = (uint64_t *)calloc(m, sizeof(uint64_t));
    w->sig_l = (long double *)calloc(m, sizeof(long double));
    w->dep_d = (double *)calloc(m, sizeof(double));
    w->dep_l = (long double *)calloc(m, sizeof(long double));
    if (!w->dist || !w->order || !w->done || !w->heap_d || !w->heap_v || !w->sig_u || !w->sig_l || !w->dep_d ||
        !w->dep_l)
        return ORC_ERR_MEM;
    return ORC_OK;
}

static int wone_source(orc_wws *w, int32_t s)
{
    wdistances(w, s);
    int mode = 0;
    if (wpath_counts(w, 0)) {
        mode = 1;
        wpath_counts(w, 1);
    }
    wdependencies(w, mode);
    return mode;
}

/* BC over a source list of a weighted graph (arguments as oracle_bc_dir,
 * plus the weights wt aligned with col and in_wt aligned with in_col; in_*
 * all NULL for an undirected graph whose weights are symmetric). */
int oracle_bc_w(int32_t n, const int32_t *row_ptr32, const int64_t *row_ptr64, const int32_t *col,
                const int32_t *wt, const int32_t *in_rp32, const int64_t *in_rp64, const int32_t *in_col,
                const int32_t *in_wt, const int32_t *sources, int64_t n_sources, double *bc, int32_t *modes)
{
    if (n < 0 || (!row_ptr32 && !row_ptr64) || !bc || !wt) return ORC_ERR_ARG;
    orc_wws w;
    const int r = wws_init(&w, n, row_ptr32, row_ptr64, col, wt, in_rp32, in_rp64, in_col, in_wt);
    if (r != ORC_OK) { wws_free(&w); return r; }
    for (int32_t i = 0; i < n; ++i) bc[i] = 0.0;
    const int64_t ns = sources ? n_sources : n;
    for (int64_t k = 0; k < ns; ++k) {
        const int32_t s = sources ? sources[k] : (int32_t)k;
        if (s < 0 || s >= n) { wws_free(&w); return ORC_ERR_ARG; }
        const int mode = wone_source(&w, s);
        if (modes) modes[k] = mode;
        for (int64_t i = 1; i < w.n_reached; ++i) {
            const int32_t v = w.order[i];
            bc[v] += mode ? (double)w.dep_l[v] : w.dep_d[v];
        }
    }
    wws_free(&w);
    return ORC_OK;
}

/* Per-source detail of a weighted graph; d is int64 (-1 = unreached),
 * other outputs as in oracle_source_dir.  Returns the mode or -error. */
int oracle_source_w(int32_t n, const int32_t *row_ptr32, const int64_t *row_ptr64, const int32_t *col,
                    const int32_t *wt, const int32_t *in_rp32, const int64_t *in_rp64, const int32_t *in_col,
                    const int32_t *in_wt, int32_t s, int64_t *d, uint64_t *sigma_u64, long double *sigma_ld,
                    double *delta)
{
    if (n <= 0 || s < 0 || s >= n || (!row_ptr32 && !row_ptr64) || !wt) return -ORC_ERR_ARG;
    orc_wws w;
    const int r = wws_init(&w, n, row_ptr32, row_ptr64, col, wt, in_rp32, in_rp64, in_col, in_wt);
    if (r != ORC_OK) { wws_free(&w); return -r; }
    const int mode = wone_source(&w, s);
    for (int32_t v = 0; v < n; ++v) {
        const int reached = w.dist[v] >= 0;
        if (d) d[v] = w.dist[v];
        if (sigma_u64) sigma_u64[v] = (mode || !reached) ? 0 : w.sig_u[v];
        if (sigma_ld) sigma_ld[v] = !reached ? 0.0L : (mode ? w.sig_l[v] : (long double)w.sig_u[v]);
        if (delta) delta[v] = !reached ? 0.0 : (mode ? (double)w.dep_l[v] : w.dep_d[v]);
    }
    wws_free(&w);
    return mode;
}

/* Size of long double in the compiled oracle, so the loader can check it
 * matches numpy's longdouble. */
int oracle_sizeof_long_double(void) { return (int)sizeof(long double); }

/*
 * Path-length excess per source: excess[k] = sum over vertices t reached from
 * sources[k] (along out-arcs), t != s, of (d(s, t) - 1).  A shortest s-t path has d(s, t) - 1
 * interior vertices and every interior vertex v of the sigma_st paths takes
 * the share sigma_st(v) / sigma_st, so these shares sum to d(s, t) - 1 and,
 * summed over t, sum_v delta_s(v) = excess (Eq. 1 and 2 with the readings
 * above).  Plain queue BFS; it touches no path count, so it checks the
 * dependency sums of any size of run independently.  Reentrant: every call
 * owns its buffers, so disjoint source slices may run on several threads.
 */
int oracle_path_excess(int32_t n, const int32_t *row_ptr32, const int64_t *row_ptr64, const int32_t *col,
                       const int32_t *sources, int64_t n_sources, int64_t *excess)
{
    if (n <= 0 || (!row_ptr32 && !row_ptr64) || !sources || !excess) return ORC_ERR_ARG;
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!d || !queue) { free(d); free(queue); return ORC_ERR_MEM; }
    for (int32_t i = 0; i < n; ++i) d[i] = -1;
    for (int64_t k = 0; k < n_sources; ++k) {
        const int32_t s = sources[k];
        if (s < 0 || s >= n) { free(d); free(queue); return ORC_ERR_ARG; }
        int64_t head = 0, tail = 0, sum = 0;
        queue[tail++] = s;
        d[s] = 0;
        while (head < tail) {
            const int32_t v = queue[head++];
            const int64_t e0 = row_ptr64 ? row_ptr64[v] : (int64_t)row_ptr32[v];
            const int64_t e1 = row_ptr64 ? row_ptr64[v + 1] : (int64_t)row_ptr32[v + 1];
            for (int64_t e = e0; e < e1; ++e) {
                const int32_t x = col[e];
                if (d[x] == -1) {
                    d[x] = d[v] + 1;
                    sum += d[x] - 1;
                    queue[tail++] = x;
                }
            }
        }
        excess[k] = sum;
        for (int64_t i = 0; i < tail; ++i) d[queue[i]] = -1; /* reset only what was reached */
    }
    free(d);
    free(queue);
    return ORC_OK;
}
