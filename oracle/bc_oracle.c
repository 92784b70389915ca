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
 *   Algorithm "Betweenness Centrality Algorithm" (Fig. seq-BC): a
 *   level-synchronous forward phase that records level sets, distances and
 *   path counts, and a backward phase over the levels in descending order.
 *
 * Readings where the paper is silent or loose (each one is listed in the
 * design notes of the repository):
 *   - Sums are over ordered pairs, so for an undirected graph every unordered
 *     pair is counted twice.  The raw sum over the given sources is returned.
 *   - v = s is excluded from BC (Eq. 2's outer sum has s != v); vertices not
 *     reached from s receive nothing (pairs with sigma_st = 0 contribute 0).
 *   - Predecessor sets are not stored: v is a predecessor of u exactly when
 *     (v, u) is an edge and d[v] = d[u] - 1, which is the set the forward
 *     phase would have built.
 *   - Path counts use uint64.  A source whose exact count exceeds 2^64 - 1 is
 *     flagged F64 and recomputed entirely in x87 long double (64-bit
 *     mantissa, 15-bit exponent); its dependencies are rounded to double at
 *     the end.  Since all partial sums of a path count are non-negative and
 *     increasing, the first carry out of 64 bits is detected exactly.
 *   - The backward update is evaluated as written,
 *     delta[v] = delta[v] + sigma[v] / sigma[u] * (1 + delta[u]),
 *     left to right, in double (U64 mode) or long double (F64 mode).
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
    const int64_t *row_ptr; /* int64 copy for uniform indexing */
    const int32_t *col;
    int32_t *d;
    int32_t *queue;          /* all levels, concatenated in discovery order */
    int64_t *level_start;    /* level l occupies queue[level_start[l] .. level_start[l+1]) */
    int32_t n_levels;        /* number of non-empty levels */
    uint64_t *sig_u;
    long double *sig_l;
    double *del_d;
    long double *del_l;
} orc_ws;

/* Forward phase (Algorithm, forward loop).  Returns 1 when a path count
 * overflowed uint64 (only possible when use_ld == 0). */
static int forward(orc_ws *w, int32_t s, int use_ld)
{
    const int32_t n = w->n;
    for (int32_t i = 0; i < n; ++i) w->d[i] = -1;
    if (use_ld) { for (int32_t i = 0; i < n; ++i) w->sig_l[i] = 0.0L; }
    else        { for (int32_t i = 0; i < n; ++i) w->sig_u[i] = 0; }
    int64_t tail = 0;
    w->queue[tail++] = s;
    w->d[s] = 0;
    if (use_ld) w->sig_l[s] = 1.0L; else w->sig_u[s] = 1;
    w->level_start[0] = 0;
    w->level_start[1] = 1;
    int32_t cur = 0;
    int overflow = 0;
    while (w->level_start[cur + 1] > w->level_start[cur]) {
        const int64_t lo = w->level_start[cur], hi = w->level_start[cur + 1];
        for (int64_t qi = lo; qi < hi; ++qi) {
            const int32_t v = w->queue[qi];
            for (int64_t e = w->row_ptr[v]; e < w->row_ptr[v + 1]; ++e) {
                const int32_t x = w->col[e];
                if (w->d[x] == -1) {
                    w->queue[tail++] = x;
                    w->d[x] = w->d[v] + 1;
                }
                if (w->d[x] == w->d[v] + 1) {
                    if (use_ld) {
                        w->sig_l[x] = w->sig_l[x] + w->sig_l[v];
                    } else {
                        uint64_t r;
                        if (__builtin_add_overflow(w->sig_u[x], w->sig_u[v], &r)) overflow = 1;
                        w->sig_u[x] = r;
                    }
                }
            }
        }
        ++cur;
        w->level_start[cur + 1] = tail;
    }
    w->n_levels = cur; /* levels 0 .. cur-1 are non-empty */
    return overflow;
}

/* Backward phase (Algorithm, backward loop): levels L..1 in descending
 * order, every vertex u of the level pushes into its predecessors. */
static void backward(orc_ws *w, int use_ld)
{
    const int32_t n = w->n;
    if (use_ld) { for (int32_t i = 0; i < n; ++i) w->del_l[i] = 0.0L; }
    else        { for (int32_t i = 0; i < n; ++i) w->del_d[i] = 0.0; }
    for (int32_t l = w->n_levels - 1; l > 0; --l) {
        for (int64_t qi = w->level_start[l]; qi < w->level_start[l + 1]; ++qi) {
            const int32_t u = w->queue[qi];
            for (int64_t e = w->row_ptr[u]; e < w->row_ptr[u + 1]; ++e) {
                const int32_t v = w->col[e];
                if (w->d[v] != l - 1) continue; /* v not in pred[u] */
                if (use_ld)
                    w->del_l[v] = w->del_l[v] + w->sig_l[v] / w->sig_l[u] * (1.0L + w->del_l[u]);
                else
                    w->del_d[v] = w->del_d[v] + (double)w->sig_u[v] / (double)w->sig_u[u] * (1.0 + w->del_d[u]);
            }
        }
    }
}

static int ws_init(orc_ws *w, int32_t n, const int32_t *row_ptr32, const int64_t *row_ptr64,
                   const int32_t *col)
{
    memset(w, 0, sizeof(*w));
    w->n = n;
    int64_t *rp = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!rp) return ORC_ERR_MEM;
    for (int64_t i = 0; i <= n; ++i) rp[i] = row_ptr64 ? row_ptr64[i] : (int64_t)row_ptr32[i];
    w->row_ptr = rp;
    w->col = col;
    w->d = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    w->queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    w->level_start = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 2));
    w->sig_u = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    w->sig_l = (long double *)malloc(sizeof(long double) * (size_t)(n > 0 ? n : 1));
    w->del_d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    w->del_l = (long double *)malloc(sizeof(long double) * (size_t)(n > 0 ? n : 1));
    if (!w->d || !w->queue || !w->level_start || !w->sig_u || !w->sig_l || !w->del_d || !w->del_l)
        return ORC_ERR_MEM;
    return ORC_OK;
}

static void ws_free(orc_ws *w)
{
    free((void *)w->row_ptr);
    free(w->d); free(w->queue); free(w->level_start);
    free(w->sig_u); free(w->sig_l); free(w->del_d); free(w->del_l);
}

/* One source: forward, overflow fallback, backward.  Returns the mode
 * (0 = U64, 1 = F64). */
static int one_source(orc_ws *w, int32_t s)
{
    int mode = 0;
    if (forward(w, s, 0)) {
        mode = 1;
        forward(w, s, 1);
    }
    backward(w, mode);
    return mode;
}

/*
 * BC over a source list.  sources == NULL means every vertex 0..n-1 in
 * order.  bc[0..n) receives the raw ordered-pair sums (it is overwritten, not
 * accumulated).  modes (nullable) receives 0/1 per source.  row_ptr is given
 * either as int32 (row_ptr32) or int64 (row_ptr64); pass NULL for the other.
 */
int oracle_bc(int32_t n, const int32_t *row_ptr32, const int64_t *row_ptr64, const int32_t *col,
              const int32_t *sources, int64_t n_sources, double *bc, int32_t *modes)
{
    if (n < 0 || (!row_ptr32 && !row_ptr64) || !bc) return ORC_ERR_ARG;
    orc_ws w;
    if (ws_init(&w, n, row_ptr32, row_ptr64, col) != ORC_OK) { ws_free(&w); return ORC_ERR_MEM; }
    for (int32_t i = 0; i < n; ++i) bc[i] = 0.0;
    const int64_t ns = sources ? n_sources : n;
    for (int64_t k = 0; k < ns; ++k) {
        const int32_t s = sources ? sources[k] : (int32_t)k;
        if (s < 0 || s >= n) { ws_free(&w); return ORC_ERR_ARG; }
        const int mode = one_source(&w, s);
        if (modes) modes[k] = mode;
        for (int32_t v = 0; v < n; ++v) {
            if (w.d[v] <= 0) continue; /* unreached, or v == s */
            bc[v] += mode ? (double)w.del_l[v] : w.del_d[v];
        }
    }
    ws_free(&w);
    return ORC_OK;
}

/*
 * Per-source detail.  d: int32[n] (-1 = unreached).  sigma_u64: uint64[n]
 * (valid in U64 mode; zero in F64 mode).  sigma_ld: long double[n] (the F64
 * mode counts; in U64 mode the exact counts converted).  delta: double[n],
 * the backward loop's values; the source's own entry is what the loop leaves
 * there (BC excludes it).  Any output pointer may be NULL.  Returns the mode
 * (0/1) or a negative error.
 */
int oracle_source(int32_t n, const int32_t *row_ptr32, const int64_t *row_ptr64, const int32_t *col,
                  int32_t s, int32_t *d, uint64_t *sigma_u64, long double *sigma_ld, double *delta,
                  int32_t *n_levels)
{
    if (n <= 0 || s < 0 || s >= n || (!row_ptr32 && !row_ptr64)) return -ORC_ERR_ARG;
    orc_ws w;
    if (ws_init(&w, n, row_ptr32, row_ptr64, col) != ORC_OK) { ws_free(&w); return -ORC_ERR_MEM; }
    const int mode = one_source(&w, s);
    for (int32_t v = 0; v < n; ++v) {
        if (d) d[v] = w.d[v];
        if (sigma_u64) sigma_u64[v] = mode ? 0 : w.sig_u[v];
        if (sigma_ld) sigma_ld[v] = mode ? w.sig_l[v] : (long double)w.sig_u[v];
        if (delta) delta[v] = mode ? (double)w.del_l[v] : w.del_d[v];
    }
    if (n_levels) *n_levels = w.n_levels;
    ws_free(&w);
    return mode;
}

/* Size of long double in the compiled oracle, so the loader can check it
 * matches numpy's longdouble. */
int oracle_sizeof_long_double(void) { return (int)sizeof(long double); }

/*
 * Path-length excess per source: excess[k] = sum over vertices t reached from
 * sources[k], t != s, of (d(s, t) - 1).  A shortest s-t path has d(s, t) - 1
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
