// bc_api.hip -- the C ABI of libbc (include/bc.h): graph handles, device
// validation, the host driver of the device-resident level state machine
// (direct launches or captured hipGraph chunks), FP64 fallback, detail dumps,
// statistics and the policy weights.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "../../include/bc.h"
#include "bc_common.h"
#include "bc_wbatch.h"

namespace bcx {
template <int MODE> __global__ void plain_step(PlainArgs a);
template <int MODE> __global__ void batch_step(BatchArgs a);
template <int MODE> __global__ void block_run(BlockArgs a);
template <int MODE> __global__ void weighted_run(WeightedArgs a);
template <int MODE> __global__ void wbatch_run(WeightedArgs a);
}  // namespace bcx

using namespace bcx;

// ------------------------------------------------------------------ errors
static thread_local std::string g_last_error;

// 64-bit FNV-1a over bytes (keys of the tune cache; not a security hash).
struct Fnv64 {
    uint64_t v = 0xcbf29ce484222325ull;
    void add(const void *p, size_t bytes) {
        const unsigned char *c = (const unsigned char *)p;
        for (size_t i = 0; i < bytes; ++i) {
            v ^= c[i];
            v *= 0x100000001b3ull;
        }
    }
};

static bc_status fail(bc_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

bc_status bc_set_error(bc_status s, const char *msg) { return fail(s, msg ? msg : ""); }

static bc_status hip_fail(hipError_t e, const char *what);

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess) return hip_fail(_e, #expr);                                     \
    } while (0)

// ----------------------------------------------------------- small kernels
namespace {

__global__ void fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

enum : unsigned {
    VAL_NONMONO = 1, VAL_RANGE = 2, VAL_SELF = 4, VAL_UNSORTED = 8, VAL_ASYM = 16, VAL_CROSS = 32
};

// Pass 1: row pointers are monotone and inside [0, nnz]; count non-isolated.
__global__ void validate_rows(int32_t n, int64_t nnz, const int32_t *rp, unsigned *err,
                              unsigned long long *nonisolated) {
    unsigned long long cnt = 0;
    unsigned e = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = rp[v], b = rp[v + 1];
        if (a > b || a < 0 || (int64_t)b > nnz) e |= VAL_NONMONO;
        else if (b > a) ++cnt;
    }
    if (e) atomicOr(err, e);
    cnt = wave_sum_u64(cnt);
    if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(nonisolated, cnt);
}

// Pass 2 (only after pass 1 is clean): one wavefront per vertex checks every
// arc: range, self-loop, strict order, block membership, symmetry.
__global__ void validate_arcs(int32_t n, const int32_t *rp, const int32_t *col, const int32_t *voff,
                              int32_t n_graphs, int check_sym, unsigned *err) {
    const int lane = threadIdx.x & 63;
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    unsigned e = 0;
    for (int64_t vv = gw; vv < n; vv += nw) {
        const int32_t v = (int32_t)vv;
        int glo = 0, ghi = n_graphs;  // block of v: voff[g] <= v < voff[g+1]
        while (ghi - glo > 1) {
            const int mid = (glo + ghi) >> 1;
            if (voff[mid] <= v) glo = mid;
            else ghi = mid;
        }
        const int32_t blo = voff[glo], bhi = voff[glo + 1];
        const int32_t e0 = rp[v], e1 = rp[v + 1];
        for (int32_t k = e0 + lane; k < e1; k += 64) {
            const int32_t w = col[k];
            if (w < 0 || w >= n) { e |= VAL_RANGE; continue; }
            if (w == v) e |= VAL_SELF;
            if (k > e0 && col[k - 1] >= w) e |= VAL_UNSORTED;
            if (w < blo || w >= bhi) e |= VAL_CROSS;
            if (check_sym) {
                int32_t lo = rp[w], hi = rp[w + 1];
                bool found = false;
                while (lo < hi) {
                    const int32_t mid = lo + ((hi - lo) >> 1);
                    const int32_t x = col[mid];
                    if (x == v) { found = true; break; }
                    if (x < v) lo = mid + 1;
                    else hi = mid;
                }
                if (!found) e |= VAL_ASYM;
            }
        }
    }
    if (e) atomicOr(err, e);
}

}  // namespace

// ------------------------------------------------------------------ handle
// Device bytes a handle holds and its cap (bc_set_device_limit; 0 = none).
struct ByteAcct {
    size_t bytes = 0;
    size_t limit = 0;
};
static thread_local bool t_cap_refused = false;  // the last refusal came from the cap, not the device

static bool over_cap(const ByteAcct *a, size_t more) { return a && a->limit && a->bytes + more > a->limit; }

static bc_status hip_fail(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory && t_cap_refused) {
        t_cap_refused = false;
        return fail(BC_ERR_OUT_OF_MEMORY, std::string(what) + ": over the handle's max_device_bytes");
    }
    return fail(e == hipErrorOutOfMemory ? BC_ERR_OUT_OF_MEMORY : BC_ERR_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

template <typename T>
static hipError_t dalloc(T **p, size_t count, ByteAcct *acc) {
    *p = nullptr;
    if (count == 0) count = 1;
    const size_t bytes = count * sizeof(T);
    t_cap_refused = false;
    if (over_cap(acc, bytes)) {  // refused before any device memory is requested
        t_cap_refused = true;
        return hipErrorOutOfMemory;
    }
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e == hipSuccess && acc) acc->bytes += bytes;
    return e;
}

struct CachedGraph {
    std::vector<unsigned char> key;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

struct SubPart;

struct bc_graph {
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t n_graphs = 1;
    std::vector<int32_t> voff;     // host copy of vertex offsets
    std::vector<int32_t> vgraph;   // not kept (large); block lookups use voff
    int32_t *row_ptr = nullptr, *col = nullptr;
    // directed graphs: row_ptr / col are the out-arcs, these the in-arcs
    bool directed = false;
    int32_t *in_row_ptr = nullptr, *in_col = nullptr;
    // weighted graphs: arc weights aligned with col and with in_col (the
    // same array for an undirected graph); the weighted engine's state
    bool weighted = false;
    int32_t *wt = nullptr, *in_wt = nullptr;
    int w_lanes = 0;                  // sources per workgroup of the allocated state (1 or kWL)
    int w_wg = 0;                     // workgroups whose state is allocated
    size_t w_stride = 0;
    char *w_scratch = nullptr;
    unsigned long long *w_ctr = nullptr;  // [0] work queue, [1] overflow count, [2] error bits, [4..14] statistics
    int32_t *w_chunk = nullptr;       // s0, s1, order
    int64_t w_chunk_cap = 0;
    int64_t *w_pos = nullptr;
    int64_t w_pos_cap = 0;
    double *w_partials = nullptr;
    int64_t w_partials_cap = 0;
    int64_t nonisolated = 0;
    // vertices of degree > kSegBatched (ascending) and their segment prefix
    // sums; p_*: the same for the plain engine's kSegPlain
    int32_t *hv_vtx = nullptr, *hv_seg = nullptr;
    int32_t n_heavy = 0;
    int64_t heavy_segs = 0;
    int32_t *p_hv_vtx = nullptr, *p_hv_seg = nullptr;
    int32_t p_n_heavy = 0;
    int64_t p_heavy_segs = 0;
    int64_t cost_units = 0;         // sum of entry_cost over all vertices
    double clock_khz = 100000.0;
    int grid_plain = 1024, grid_batch = 1024;  // resident workgroups of the step kernels
    double *bc = nullptr;
    LevelRec *lvl = nullptr;       // per-level records of the last run [kLevelRecs]
    bool last_parts = false;       // the last run ran on concurrent parts
    ByteAcct acct;                 // device bytes held by this handle itself, and the cap
    size_t create_bytes = 0;       // bytes held right after creation
    hipStream_t cap_stream = nullptr;  // private non-blocking capture stream, created on first capture
    Ctl *ctl = nullptr;
    Ctl *ctl_host = nullptr;       // pinned
    int32_t *flag_host = nullptr;  // pinned: {phase, err} polled after chunks
    // plain engine
    bool plain_ready = false, plain_dirty = false;
    int32_t *p_d = nullptr, *p_queue = nullptr, *p_level_off = nullptr, *p_shift = nullptr;
    unsigned long long *p_sig = nullptr;
    double *p_chat = nullptr;
    HeavyQ p_hq{};
    // batched engine
    bool batch_ready = false;
    VisNext *b_vn = nullptr;
    Tagged *b_fw0 = nullptr, *b_fw1 = nullptr;
    int32_t *b_lq_vtx = nullptr;
    unsigned long long *b_lq_mask = nullptr;
    uint32_t b_lq_cap = 0;
    int32_t *b_level_off = nullptr;
    int32_t b_max_levels = 0;
    unsigned long long *b_sigma = nullptr;
    double *b_chat = nullptr, *b_delta = nullptr;
    uint32_t *b_gstart = nullptr, *b_gbase = nullptr;
    uint32_t b_gcap = 0;
    int32_t *b_shift = nullptr, *b_maxexp = nullptr, *b_lane_src = nullptr;
    HeavyQ b_hq{};
    // per-run buffers (grown on demand)
    int32_t *srcs = nullptr;
    int64_t srcs_cap = 0;
    int64_t *ovf = nullptr;
    int64_t ovf_cap = 0;
    int64_t *bstart = nullptr;
    int32_t *blo = nullptr, *bhi = nullptr;
    int64_t bcap[3] = {0, 0, 0};   // capacities of bstart, blo, bhi
    // policy
    float *mlp = nullptr;
    bool has_mlp = false;
    // hub-first relabelling (empty = identity): perm[new] = old, inv[old] = new
    std::vector<int32_t> perm, inv;
    int32_t *inv_dev = nullptr;
    double *bc_out = nullptr;  // scores gathered back to the caller's order
    // rank of each internal vertex as a source (empty = keep the caller's
    // order; see source_ranks)
    std::vector<int32_t> srank;
    // autotuner result (bc_autotune), used by bc_run with BC_RUN_TUNED
    bool has_tuned = false;
    bc_run_options tuned{};
    // sizes, flags, block offsets and degree sequence (caller's order) of the
    // graph: the key of its autotuner results in the tune cache
    uint64_t fingerprint = 0;
    // unions of many graphs: sub-unions run concurrently (see run_parts)
    std::vector<struct SubPart> parts;
    std::vector<int32_t> part_of_graph, local_base;  // per parent graph
    bool replicas = false;  // parts are full copies of a single graph (see ensure_replicas)
    bool parts_refused = false;  // concurrent parts would not fit under the cap (see parts_fit)
    // block engine (graphs of at most kBlockMaxN vertices; see run_block)
    bool blk_sized = false;            // per-graph facts below are computed
    int32_t blk_nmax = 0;              // largest graph
    int64_t blk_cost_max = 0, blk_heavy_max = 0, blk_segs_max = 0;
    int blk_wg = 0;                    // workgroups whose state is allocated
    size_t blk_stride = 0;
    BlockArgs blk_dims{};              // capacities of one workgroup's state
    char *blk_scratch = nullptr;
    Ctl *blk_ctls = nullptr;
    int32_t *blk_chunk = nullptr;      // b0, b1, order (3 x n_chunks), grown per run
    int64_t blk_chunk_cap = 0;
    int64_t *blk_part_off = nullptr;
    int64_t blk_part_off_cap = 0;
    double *blk_partials = nullptr;
    int64_t blk_partials_cap = 0;
    int32_t *blk_gsum = nullptr;       // per graph: lo, hi, first chunk, end chunk
    int64_t blk_gsum_cap = 0;
    uint32_t *blk_next = nullptr;
    // graph cache
    std::vector<CachedGraph> graphs;
    bc_stats stats{};
};

// One sub-union of a many-graph handle: a handle of its own over some of
// the graphs (vertices renumbered consecutively), its stream, and the map
// back to the parent's vertex ids.
struct SubPart {
    bc_graph *h = nullptr;
    int32_t *to_parent = nullptr;           // device int32[h->n]
    std::vector<int32_t> to_parent_host;
    hipStream_t stream = nullptr;
};

static void free_graphs(bc_graph *g) {
    for (auto &cg : g->graphs) {
        if (cg.exec) (void)hipGraphExecDestroy(cg.exec);
        if (cg.graph) (void)hipGraphDestroy(cg.graph);
    }
    g->graphs.clear();
}

static void free_parts(bc_graph *g);

extern "C" void bc_destroy(bc_graph *g) {
    if (!g) return;
    (void)hipDeviceSynchronize();
    free_parts(g);
    free_graphs(g);
    void *dev[] = {g->row_ptr, g->col, g->in_row_ptr, g->in_col, g->wt,
                   g->in_wt == g->wt ? nullptr : g->in_wt, g->w_scratch, g->w_ctr, g->w_chunk, g->w_pos,
                   g->w_partials, g->bc, g->ctl, g->p_d, g->p_queue, g->p_level_off, g->p_shift,
                   g->p_sig, g->p_chat, g->b_vn, g->b_fw0, g->b_fw1, g->b_lq_vtx, g->b_lq_mask,
                   g->b_level_off, g->b_delta, g->b_chat, g->b_shift, g->b_maxexp, g->b_lane_src,
                   g->b_sigma, g->b_gstart, g->b_gbase, g->inv_dev, g->bc_out,
                   g->srcs, g->ovf, g->bstart, g->blo, g->bhi, g->mlp, g->hv_vtx, g->hv_seg, g->p_hv_vtx, g->p_hv_seg,
                   g->p_hq.pos, g->p_hq.seg, g->p_hq.cnt, g->p_hq.off, g->p_hq.nseg, g->p_hq.part_lo,
                   g->p_hq.part_hi, g->b_hq.pos, g->b_hq.seg, g->b_hq.cnt, g->b_hq.off, g->b_hq.nseg,
                   g->b_hq.part_lo, g->b_hq.part_hi, g->lvl, g->blk_scratch, g->blk_ctls, g->blk_chunk,
                   g->blk_part_off, g->blk_partials, g->blk_gsum, g->blk_next};
    for (void *p : dev)
        if (p) (void)hipFree(p);
    if (g->ctl_host) (void)hipHostFree(g->ctl_host);
    if (g->flag_host) (void)hipHostFree(g->flag_host);
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    delete g;
}

extern "C" const char *bc_last_error(void) { return g_last_error.c_str(); }

extern "C" const char *bc_status_string(bc_status s) {
    switch (s) {
    case BC_OK: return "BC_OK";
    case BC_ERR_INVALID_ARG: return "BC_ERR_INVALID_ARG";
    case BC_ERR_INVALID_GRAPH: return "BC_ERR_INVALID_GRAPH";
    case BC_ERR_OUT_OF_MEMORY: return "BC_ERR_OUT_OF_MEMORY";
    case BC_ERR_DEVICE: return "BC_ERR_DEVICE";
    case BC_ERR_SIGMA_RANGE: return "BC_ERR_SIGMA_RANGE";
    case BC_ERR_NOT_SUPPORTED: return "BC_ERR_NOT_SUPPORTED";
    }
    return "BC_ERR_UNKNOWN";
}

static int grid_for(int64_t work, int per_block, int cap) {
    int64_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

// Rank of every vertex as a source.  Within each graph, sources are taken
// by hop distance from the graph's vertex of largest degree (the hub), then
// by their parent in the hub's BFS tree (the neighbour one hop closer, of
// largest degree; parents of larger degree first), then by decreasing
// degree.  Sources equally far from the hub that hang off the same parent
// reach most vertices at the same depth, so a batch of them shares frontier
// entries: fewer level-queue entries, and neighbour rows read for more lanes
// at once.
static void source_ranks(int32_t n_graphs, const std::vector<int32_t> &voff, const std::vector<int32_t> &rp,
                         const std::vector<int32_t> &col, std::vector<int32_t> *rank) {
    const int32_t n = (int32_t)rp.size() - 1;
    const int32_t kFar = INT32_MAX;
    std::vector<int32_t> dist((size_t)n, kFar), par((size_t)n, -1), q;
    q.reserve((size_t)n);
    auto deg = [&](int32_t v) { return v < 0 ? INT32_MAX : rp[v + 1] - rp[v]; };
    for (int gi = 0; gi < n_graphs; ++gi) {
        const int32_t lo = voff[gi], hi = voff[gi + 1];
        if (lo == hi) continue;
        int32_t hub = lo;
        for (int32_t v = lo; v < hi; ++v)
            if (deg(v) > deg(hub)) hub = v;
        q.clear();
        q.push_back(hub);
        dist[hub] = 0;
        for (size_t h = 0; h < q.size(); ++h) {
            const int32_t v = q[h];
            for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
                if (dist[col[e]] == kFar) {
                    dist[col[e]] = dist[v] + 1;
                    q.push_back(col[e]);
                }
        }
        for (int32_t v : q) {
            if (v == hub) continue;
            int32_t p = -1;
            for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
                const int32_t u = col[e];
                if (dist[u] == dist[v] - 1 && (p < 0 || deg(u) > deg(p))) p = u;
            }
            par[v] = p;
        }
    }
    std::vector<int32_t> order((size_t)n), gidx((size_t)n);
    for (int gi = 0; gi < n_graphs; ++gi)
        for (int32_t v = voff[gi]; v < voff[gi + 1]; ++v) gidx[v] = gi;
    for (int32_t v = 0; v < n; ++v) order[v] = v;
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (gidx[a] != gidx[b]) return gidx[a] < gidx[b];
        if (dist[a] != dist[b]) return dist[a] < dist[b];
        const int32_t pa = par[a], pb = par[b];
        if (pa != pb) {
            if (deg(pa) != deg(pb)) return deg(pa) > deg(pb);
            return pa < pb;
        }
        if (deg(a) != deg(b)) return deg(a) > deg(b);
        return a < b;
    });
    rank->assign((size_t)n, 0);
    for (int32_t i = 0; i < n; ++i) (*rank)[order[i]] = i;
}

static bc_status create_impl(int32_t n_graphs, const int32_t *voff_in, int32_t n, int64_t nnz,
                             const int32_t *row_ptr, const int32_t *col_idx, uint32_t flags, bc_graph **out,
                             const int32_t *weights = nullptr) {
    if (!out) return fail(BC_ERR_INVALID_ARG, "out is NULL");
    if (n < 0 || n >= INT32_MAX - 2) return fail(BC_ERR_INVALID_ARG, "n out of range");
    if (nnz < 0 || nnz > INT32_MAX) return fail(BC_ERR_INVALID_ARG, "nnz out of range (must be <= 2^31-1)");
    if (!row_ptr || (nnz > 0 && !col_idx)) return fail(BC_ERR_INVALID_ARG, "NULL CSR array");
    if (n_graphs < 1) return fail(BC_ERR_INVALID_ARG, "n_graphs < 1");
    std::vector<int32_t> voff;
    if (voff_in) {
        voff.assign(voff_in, voff_in + n_graphs + 1);
        if (voff[0] != 0 || voff[n_graphs] != n) return fail(BC_ERR_INVALID_ARG, "vtx_offsets must run from 0 to n");
        for (int i = 0; i < n_graphs; ++i)
            if (voff[i] > voff[i + 1]) return fail(BC_ERR_INVALID_ARG, "vtx_offsets not non-decreasing");
    } else {
        voff = {0, n};
    }
    const bool on_dev = flags & BC_INPUT_DEVICE;
    const bool directed = flags & BC_DIRECTED;
    if (directed && n_graphs > 1)
        return fail(BC_ERR_NOT_SUPPORTED, "directed graphs are supported one per handle (bc_graph_create)");
    const bool keep_sources = flags & BC_KEEP_ORDER;  // the caller's own request
    if (directed) flags |= BC_SKIP_SYMMETRY_CHECK | BC_KEEP_ORDER;
    if (weights && n_graphs > 1)
        return fail(BC_ERR_NOT_SUPPORTED, "weighted graphs are supported one per handle (bc_graph_create_weighted)");
    if (weights) flags |= BC_KEEP_ORDER;  // weights stay aligned with the caller's arcs
    bc_graph *g = new bc_graph();
    g->directed = directed;
    g->weighted = weights != nullptr;
    g->n = n;
    g->nnz = nnz;
    g->n_graphs = n_graphs;
    g->voff = voff;
    auto bail = [&](bc_status st) {
        bc_destroy(g);
        return st;
    };
    hipError_t e;
    unsigned *derr = nullptr;
    unsigned long long *dcnt = nullptr;
    int32_t *dvoff = nullptr;
#define CR_TRY(expr)                                                                           \
    do {                                                                                       \
        e = (expr);                                                                            \
        if (e != hipSuccess) {                                                                 \
            if (derr) (void)hipFree(derr);                                                     \
            if (dcnt) (void)hipFree(dcnt);                                                     \
            if (dvoff) (void)hipFree(dvoff);                                                   \
            return bail(hip_fail(e, #expr));                                                   \
        }                                                                                      \
    } while (0)
    CR_TRY(dalloc(&g->row_ptr, (size_t)n + 1, &g->acct));
    CR_TRY(dalloc(&g->col, (size_t)nnz, &g->acct));
    const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    CR_TRY(hipMemcpy(g->row_ptr, row_ptr, sizeof(int32_t) * ((size_t)n + 1), kind));
    if (nnz) CR_TRY(hipMemcpy(g->col, col_idx, sizeof(int32_t) * (size_t)nnz, kind));
    int32_t ends[2];
    CR_TRY(hipMemcpy(&ends[0], g->row_ptr, sizeof(int32_t), hipMemcpyDeviceToHost));
    CR_TRY(hipMemcpy(&ends[1], g->row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (ends[0] != 0 || (int64_t)ends[1] != nnz) {
        fail(BC_ERR_INVALID_GRAPH, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
        return bail(BC_ERR_INVALID_GRAPH);
    }
    CR_TRY(hipMalloc((void **)&derr, sizeof(unsigned)));
    CR_TRY(hipMalloc((void **)&dcnt, sizeof(unsigned long long)));
    CR_TRY(hipMalloc((void **)&dvoff, sizeof(int32_t) * voff.size()));
    CR_TRY(hipMemcpy(dvoff, voff.data(), sizeof(int32_t) * voff.size(), hipMemcpyHostToDevice));
    CR_TRY(hipMemset(derr, 0, sizeof(unsigned)));
    CR_TRY(hipMemset(dcnt, 0, sizeof(unsigned long long)));
    if (n > 0) {
        validate_rows<<<grid_for(n, 256, 4096), 256>>>(n, nnz, g->row_ptr, derr, dcnt);
        CR_TRY(hipGetLastError());
    }
    unsigned herr = 0;
    unsigned long long hcnt = 0;
    CR_TRY(hipMemcpy(&herr, derr, sizeof(unsigned), hipMemcpyDeviceToHost));
    CR_TRY(hipMemcpy(&hcnt, dcnt, sizeof(unsigned long long), hipMemcpyDeviceToHost));
    if (!herr && n > 0 && nnz > 0) {
        validate_arcs<<<grid_for((int64_t)n * 64, 256, 8192), 256>>>(
            n, g->row_ptr, g->col, dvoff, n_graphs, (flags & BC_SKIP_SYMMETRY_CHECK) ? 0 : 1, derr);
        CR_TRY(hipGetLastError());
        CR_TRY(hipMemcpy(&herr, derr, sizeof(unsigned), hipMemcpyDeviceToHost));
    }
    (void)hipFree(derr);
    (void)hipFree(dcnt);
    (void)hipFree(dvoff);
    derr = nullptr;
    dcnt = nullptr;
    dvoff = nullptr;
    if (herr) {
        std::string m = "invalid CSR:";
        if (herr & VAL_NONMONO) m += " row_ptr not monotone / outside [0, nnz];";
        if (herr & VAL_RANGE) m += " column index outside [0, n);";
        if (herr & VAL_SELF) m += " self-loop;";
        if (herr & VAL_UNSORTED) m += " row not strictly ascending (unsorted or duplicate arc);";
        if (herr & VAL_ASYM) m += " arcs not symmetric;";
        if (herr & VAL_CROSS) m += " arc crosses a graph boundary;";
        fail(BC_ERR_INVALID_GRAPH, m);
        return bail(BC_ERR_INVALID_GRAPH);
    }
    g->nonisolated = (int64_t)hcnt;
    {
        std::vector<int32_t> rp((size_t)n + 1);
        CR_TRY(hipMemcpy(rp.data(), g->row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost));
        {
            Fnv64 h;
            const int64_t head[5] = {n, nnz, n_graphs, directed ? 1 : 0, weights ? 1 : 0};
            h.add(head, sizeof(head));
            h.add(voff.data(), sizeof(int32_t) * voff.size());
            h.add(rp.data(), sizeof(int32_t) * rp.size());
            g->fingerprint = h.v;
        }
        // directed: the in-arcs (transpose), rows ascending; a vertex is
        // classified by the larger of its out- and in-degree
        std::vector<int32_t> cdeg((size_t)n);
        for (int32_t v = 0; v < n; ++v) cdeg[v] = rp[v + 1] - rp[v];
        if (directed) {
            std::vector<int32_t> col((size_t)nnz), irp((size_t)n + 1, 0), icol((size_t)nnz);
            if (nnz) CR_TRY(hipMemcpy(col.data(), g->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost));
            for (int64_t k = 0; k < nnz; ++k) ++irp[(size_t)col[k] + 1];
            for (int32_t v = 0; v < n; ++v) irp[v + 1] += irp[v];
            std::vector<int32_t> fill(irp.begin(), irp.end() - 1);
            for (int32_t u = 0; u < n; ++u)  // sources in ascending order: every in-row comes out sorted
                for (int32_t k = rp[u]; k < rp[u + 1]; ++k) icol[fill[col[k]]++] = u;
            for (int32_t v = 0; v < n; ++v) cdeg[v] = std::max(cdeg[v], irp[v + 1] - irp[v]);
            if (weights) {  // the in-arcs carry the weight of the same arc
                std::vector<int32_t> w((size_t)nnz), iw((size_t)nnz);
                if (nnz) CR_TRY(hipMemcpy(w.data(), weights, sizeof(int32_t) * (size_t)nnz,
                                          on_dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
                std::vector<int32_t> fill2(irp.begin(), irp.end() - 1);
                for (int32_t u = 0; u < n; ++u)
                    for (int32_t k = rp[u]; k < rp[u + 1]; ++k) iw[fill2[col[k]]++] = w[k];
                CR_TRY(dalloc(&g->in_wt, (size_t)nnz, &g->acct));
                if (nnz) CR_TRY(hipMemcpy(g->in_wt, iw.data(), sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice));
            }
            CR_TRY(dalloc(&g->in_row_ptr, (size_t)n + 1, &g->acct));
            CR_TRY(dalloc(&g->in_col, (size_t)nnz, &g->acct));
            CR_TRY(hipMemcpy(g->in_row_ptr, irp.data(), sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice));
            if (nnz) CR_TRY(hipMemcpy(g->in_col, icol.data(), sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice));
        }
        if (!(flags & BC_KEEP_ORDER) && n > 0 && nnz > 0) {
            // hub-first renumbering inside each graph: vertices of degree at
            // least twice the graph's mean (over vertices with arcs) first, by
            // decreasing degree, the rest in their order
            std::vector<int32_t> order((size_t)n);
            bool moved = false, any_hubs = false;
            for (int gi = 0; gi < n_graphs; ++gi) {
                const int32_t lo = voff[gi], hi = voff[gi + 1];
                int64_t arcs = 0, with = 0;
                for (int32_t v = lo; v < hi; ++v) {
                    const int32_t d = rp[v + 1] - rp[v];
                    arcs += d;
                    with += d > 0;
                }
                const double thr = with ? 2.0 * (double)arcs / (double)with : 1e300;
                std::vector<int32_t> hubs, rest;
                for (int32_t v = lo; v < hi; ++v) ((double)(rp[v + 1] - rp[v]) >= thr ? hubs : rest).push_back(v);
                std::stable_sort(hubs.begin(), hubs.end(),
                                 [&](int32_t a, int32_t b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
                any_hubs = any_hubs || !hubs.empty();
                int32_t k = lo;
                for (int32_t v : hubs) order[k++] = v;
                for (int32_t v : rest) order[k++] = v;
                for (int32_t i = lo; i < hi && !moved; ++i) moved = order[i] != i;
            }
            if (moved) {
                std::vector<int32_t> col((size_t)nnz), ncol((size_t)nnz), nrp((size_t)n + 1);
                CR_TRY(hipMemcpy(col.data(), g->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost));
                g->perm = order;
                g->inv.assign((size_t)n, 0);
                for (int32_t i = 0; i < n; ++i) g->inv[order[i]] = i;
                nrp[0] = 0;
                for (int32_t i = 0; i < n; ++i) nrp[i + 1] = nrp[i] + (rp[order[i] + 1] - rp[order[i]]);
                // rows are independent: renumber and sort them on a few host threads
                const int nt = (int)std::min<int64_t>(16, std::max<int64_t>(1, nnz >> 20));
                std::vector<std::thread> pool;
                for (int t = 0; t < nt; ++t)
                    pool.emplace_back([&, t] {
                        for (int32_t i = (int32_t)((int64_t)n * t / nt); i < (int32_t)((int64_t)n * (t + 1) / nt); ++i) {
                            const int32_t v = order[i];
                            int32_t *dst = ncol.data() + nrp[i];
                            const int32_t d = rp[v + 1] - rp[v];
                            for (int32_t e = 0; e < d; ++e) dst[e] = g->inv[col[rp[v] + e]];
                            std::sort(dst, dst + d);
                        }
                    });
                for (std::thread &th : pool) th.join();
                rp = nrp;
                CR_TRY(hipMemcpy(g->row_ptr, rp.data(), sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice));
                CR_TRY(hipMemcpy(g->col, ncol.data(), sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice));
                CR_TRY(dalloc(&g->inv_dev, (size_t)n, &g->acct));
                CR_TRY(hipMemcpy(g->inv_dev, g->inv.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice));
                CR_TRY(dalloc(&g->bc_out, (size_t)n, &g->acct));
                source_ranks(n_graphs, voff, rp, ncol, &g->srank);
            } else if (any_hubs) {  // hubs already first: keep the numbering, still order the sources
                std::vector<int32_t> col((size_t)nnz);
                CR_TRY(hipMemcpy(col.data(), g->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost));
                source_ranks(n_graphs, voff, rp, col, &g->srank);
            }
        }
        if ((weights || directed) && !keep_sources && n > 0 && nnz > 0) {
            // the vertex numbering stays, the sources are still ranked (hop
            // distance along out-arcs from the vertex of largest out-degree):
            // a batch then holds sources near each other
            std::vector<int32_t> col((size_t)nnz);
            CR_TRY(hipMemcpy(col.data(), g->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost));
            source_ranks(n_graphs, voff, rp, col, &g->srank);
        }
        // vertices heavier than one segment, for the split load balancing
        // (one list per engine segment size)
        if (!directed)  // after any renumbering
            for (int32_t v = 0; v < n; ++v) cdeg[v] = rp[v + 1] - rp[v];
        if (weights) {
            // every weight >= 1; an undirected graph carries the same weight on
            // both arcs of an edge
            std::vector<int32_t> w((size_t)nnz), col((size_t)nnz);
            if (nnz) {
                CR_TRY(hipMemcpy(w.data(), weights, sizeof(int32_t) * (size_t)nnz,
                                 on_dev ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
                CR_TRY(hipMemcpy(col.data(), g->col, sizeof(int32_t) * (size_t)nnz, hipMemcpyDeviceToHost));
            }
            bool ok = true;
            for (int64_t k = 0; k < nnz && ok; ++k) ok = w[k] >= 1;
            if (!ok) {
                fail(BC_ERR_INVALID_GRAPH, "invalid weights: every arc weight must be >= 1");
                return bail(BC_ERR_INVALID_GRAPH);
            }
            if (!directed) {
                for (int32_t u = 0; u < n && ok; ++u)
                    for (int32_t k = rp[u]; k < rp[u + 1] && ok; ++k) {
                        const int32_t v = col[k];
                        const int32_t *b0 = col.data() + rp[v], *b1 = col.data() + rp[v + 1];
                        const int32_t *f = std::lower_bound(b0, b1, u);
                        ok = f != b1 && *f == u && w[(size_t)(f - col.data())] == w[k];
                    }
                if (!ok) {
                    fail(BC_ERR_INVALID_GRAPH, "invalid weights: the two arcs of an undirected edge differ");
                    return bail(BC_ERR_INVALID_GRAPH);
                }
            }
            CR_TRY(dalloc(&g->wt, (size_t)nnz, &g->acct));
            if (nnz) CR_TRY(hipMemcpy(g->wt, w.data(), sizeof(int32_t) * (size_t)nnz, hipMemcpyHostToDevice));
            if (!directed) g->in_wt = g->wt;
        }
        int64_t cost_units = 0;
        for (int32_t v = 0; v < n; ++v) cost_units += entry_cost(cdeg[v]);
        g->cost_units = cost_units;
        for (int which = 0; which < 2; ++which) {
            const int seg = which == 0 ? kSegBatched : kSegPlain;
            std::vector<int32_t> hv, hs(1, 0);
            int64_t segs = 0;
            for (int32_t v = 0; v < n; ++v) {
                const int32_t deg = cdeg[v];
                if (deg > seg) {
                    hv.push_back(v);
                    segs += (deg + seg - 1) / seg;
                    hs.push_back((int32_t)segs);
                }
            }
            int32_t **pv = which == 0 ? &g->hv_vtx : &g->p_hv_vtx, **ps = which == 0 ? &g->hv_seg : &g->p_hv_seg;
            (which == 0 ? g->n_heavy : g->p_n_heavy) = (int32_t)hv.size();
            (which == 0 ? g->heavy_segs : g->p_heavy_segs) = segs;
            CR_TRY(dalloc(pv, hv.size(), &g->acct));
            CR_TRY(dalloc(ps, hs.size(), &g->acct));
            if (!hv.empty()) CR_TRY(hipMemcpy(*pv, hv.data(), sizeof(int32_t) * hv.size(), hipMemcpyHostToDevice));
            CR_TRY(hipMemcpy(*ps, hs.data(), sizeof(int32_t) * hs.size(), hipMemcpyHostToDevice));
        }
        int dev = 0, khz = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            g->clock_khz = khz;
        // one full wave of workgroups: every CU holds as many as occupancy allows
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
            int bp = 0, bb = 0;
            // the plain engine's levels are small: half a wave of workgroups
            // keeps the per-step arrival count (and idle launches) down
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bp, (const void *)plain_step<0>, kBlock, 0) == hipSuccess &&
                bp > 0)
                g->grid_plain = std::max(cus, cus * bp / 2);
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bb, (const void *)batch_step<0>, kBlock, 0) == hipSuccess &&
                bb > 0)
                g->grid_batch = cus * bb;
        }
    }
    CR_TRY(dalloc(&g->bc, (size_t)n, &g->acct));
    CR_TRY(hipMemset(g->bc, 0, sizeof(double) * (size_t)(n > 0 ? n : 1)));
    CR_TRY(dalloc(&g->ctl, 1, &g->acct));
    CR_TRY(hipHostMalloc((void **)&g->ctl_host, sizeof(Ctl), hipHostMallocDefault));
    CR_TRY(hipHostMalloc((void **)&g->flag_host, 64 * sizeof(int32_t), hipHostMallocDefault));
    CR_TRY(dalloc(&g->mlp, (size_t)kMlpParams, &g->acct));
    CR_TRY(dalloc(&g->lvl, (size_t)kLevelRecs, &g->acct));
    CR_TRY(hipMemset(g->lvl, 0, sizeof(LevelRec) * kLevelRecs));
#undef CR_TRY
    g->create_bytes = g->acct.bytes;
    *out = g;
    return BC_OK;
}

extern "C" bc_status bc_graph_create(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                     uint32_t flags, bc_graph **out) {
    return create_impl(1, nullptr, n, nnz, row_ptr, col_idx, flags, out);
}

extern "C" bc_status bc_graph_create_weighted(int32_t n, int64_t nnz, const int32_t *row_ptr,
                                              const int32_t *col_idx, const int32_t *weights, uint32_t flags,
                                              bc_graph **out) {
    if (!weights && nnz > 0) return fail(BC_ERR_INVALID_ARG, "NULL weights");
    static const int32_t one = 1;
    return create_impl(1, nullptr, n, nnz, row_ptr, col_idx, flags, out, weights ? weights : &one);
}

extern "C" bc_status bc_graph_create_multi(int32_t n_graphs, const int32_t *vtx_offsets, int32_t n, int64_t nnz,
                                           const int32_t *row_ptr, const int32_t *col_idx, uint32_t flags,
                                           bc_graph **out) {
    if (!vtx_offsets) return fail(BC_ERR_INVALID_ARG, "vtx_offsets is NULL");
    return create_impl(n_graphs, vtx_offsets, n, nnz, row_ptr, col_idx, flags, out);
}

// Device bytes of the handle and of the concurrent parts it created.
static size_t total_bytes(const bc_graph *g) {
    size_t t = g->acct.bytes;
    for (const SubPart &pt : g->parts) t += total_bytes(pt.h) + pt.to_parent_host.size() * sizeof(int32_t);
    return t;
}

extern "C" bc_status bc_graph_info(const bc_graph *g, int32_t *n, int64_t *nnz, int32_t *n_graphs,
                                   int64_t *device_bytes) {
    if (!g) return fail(BC_ERR_INVALID_ARG, "NULL handle");
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    if (n_graphs) *n_graphs = g->n_graphs;
    if (device_bytes) *device_bytes = (int64_t)total_bytes(g);
    return BC_OK;
}

extern "C" bc_status bc_set_device_limit(bc_graph *g, int64_t max_device_bytes) {
    if (!g) return fail(BC_ERR_INVALID_ARG, "NULL handle");
    if (max_device_bytes < 0) return fail(BC_ERR_INVALID_ARG, "max_device_bytes < 0");
    g->acct.limit = (size_t)max_device_bytes;
    g->parts_refused = false;  // decided again at the next run
    if (g->acct.limit && !g->parts.empty() && total_bytes(g) > g->acct.limit) {
        // the parts already made do not fit under the new cap: drop them
        (void)hipDeviceSynchronize();
        free_parts(g);
        g->replicas = false;
    }
    return BC_OK;
}

extern "C" void bc_run_options_init(bc_run_options *opt) {
    if (opt) std::memset(opt, 0, sizeof(*opt));
}

// ------------------------------------------------------------ engine setup
static bc_status alloc_hq(bc_graph *g, HeavyQ *q, int64_t entries, int64_t levels, int lanes, int64_t heavy_segs) {
    HIP_TRY(dalloc(&q->pos, (size_t)entries, &g->acct));
    HIP_TRY(dalloc(&q->seg, (size_t)entries, &g->acct));
    HIP_TRY(dalloc(&q->cnt, (size_t)entries, &g->acct));
    HIP_TRY(dalloc(&q->off, (size_t)levels, &g->acct));
    HIP_TRY(dalloc(&q->nseg, (size_t)levels, &g->acct));
    const int64_t segs = heavy_segs + 1;
    HIP_TRY(dalloc(&q->part_lo, (size_t)segs * lanes, &g->acct));
    HIP_TRY(dalloc(&q->part_hi, (size_t)segs * lanes, &g->acct));
    q->cap = (uint32_t)std::min<int64_t>(entries, UINT32_MAX);
    q->part_cap = (uint32_t)std::min<int64_t>(segs, UINT32_MAX);
    return BC_OK;
}

static bc_status ensure_plain(bc_graph *g, hipStream_t st) {
    const int64_t n = g->n;
    if (!g->plain_ready) {
        const size_t need = (size_t)(g->p_n_heavy + 1) * 12 + (size_t)(n + 3) * 8 + (size_t)(g->p_heavy_segs + 1) * 16 +
                            (size_t)std::max<int64_t>(n, 1) * 24 + (size_t)(n + 2) * 8;
        if (over_cap(&g->acct, need))
            return fail(BC_ERR_OUT_OF_MEMORY, "per-source engine state (" + std::to_string(need) +
                                                  " bytes) is over the handle's max_device_bytes");
        // each heavy vertex enters a source's level queues once
        bc_status s = alloc_hq(g, &g->p_hq, (int64_t)g->p_n_heavy + 1, n + 3, 1, g->p_heavy_segs);
        if (s != BC_OK) return s;
        HIP_TRY(dalloc(&g->p_d, (size_t)n, &g->acct));
        HIP_TRY(dalloc(&g->p_queue, (size_t)n, &g->acct));
        HIP_TRY(dalloc(&g->p_level_off, (size_t)n + 2, &g->acct));
        HIP_TRY(dalloc(&g->p_shift, (size_t)n + 2, &g->acct));
        HIP_TRY(dalloc(&g->p_sig, (size_t)n, &g->acct));
        HIP_TRY(dalloc(&g->p_chat, (size_t)n, &g->acct));
        g->plain_ready = true;
        g->plain_dirty = true;
    }
    if (g->plain_dirty && n > 0) {
        // invariant between sources: d = -1, sig = 0 everywhere
        fill_i32<<<grid_for(n, 256, 4096), 256, 0, st>>>(g->p_d, n, -1);
        fill_u64<<<grid_for(n, 256, 4096), 256, 0, st>>>(g->p_sig, n, 0ull);
        HIP_TRY(hipGetLastError());
        g->plain_dirty = false;
    }
    return BC_OK;
}

// Sizes of the batched engine's state for a graph (shared by the allocation
// and by the estimates the device-memory cap is checked against).
struct BatchedSizes {
    int64_t lq_cap, max_levels, gcap, hq_entries, hq_levels;
    size_t bytes;
};
static BatchedSizes batched_sizes(int64_t n, int64_t cost_units, int64_t n_heavy, int64_t heavy_segs) {
    BatchedSizes z;
    // every (vertex, lane) pair enters the level queues at most once
    z.lq_cap = std::min<int64_t>((int64_t)kLanes * std::max<int64_t>(n, 1) + 64, (int64_t)INT32_MAX);
    z.max_levels = std::max<int64_t>(std::min<int64_t>(n + 2, 65536), 4);
    // work groups: a vertex is on at most 64 levels of a batch; each level
    // has cost / kBudget + 1 groups and one closing slot
    z.gcap = std::min<int64_t>((int64_t)kLanes * cost_units / kBudget + 2 * (z.max_levels + 2) + 64,
                               (int64_t)UINT32_MAX);
    // a heavy vertex sits on at most 64 distinct levels of a batch (one per lane)
    z.hq_entries = n_heavy * kLanes + kLanes;
    z.hq_levels = z.max_levels + 3;
    const size_t nn = (size_t)std::max<int64_t>(n, 1);
    z.bytes = nn * (sizeof(VisNext) + 2 * sizeof(Tagged)) + (size_t)z.lq_cap * (sizeof(int32_t) + 8) +
              (size_t)(z.max_levels + 2) * sizeof(int32_t) * 3 + nn * kLanes * 3 * 8 + (size_t)z.gcap * 4 +
              (size_t)(z.max_levels + 2) * kLanes * 4 + (size_t)2 * kSlots * kLanes * 4 + kLanes * 4 +
              (size_t)z.hq_entries * 12 + (size_t)z.hq_levels * 8 + (size_t)(heavy_segs + 1) * kLanes * 16;
    return z;
}

static bc_status ensure_batched(bc_graph *g) {
    if (g->batch_ready) return BC_OK;
    const int64_t n = g->n;
    // level cost prefixes are 32-bit; a level holds each vertex at most once
    if (g->cost_units >= (int64_t)UINT32_MAX)
        return fail(BC_ERR_NOT_SUPPORTED, "graph too large for the batched engine: use batch = 1");
    const BatchedSizes z = batched_sizes(n, g->cost_units, g->n_heavy, g->heavy_segs);
    if (over_cap(&g->acct, z.bytes))
        return fail(BC_ERR_OUT_OF_MEMORY, "batched engine state (" + std::to_string(z.bytes) +
                                              " bytes) is over the handle's max_device_bytes");
    HIP_TRY(dalloc(&g->b_vn, (size_t)n, &g->acct));
    HIP_TRY(dalloc(&g->b_fw0, (size_t)n, &g->acct));
    HIP_TRY(dalloc(&g->b_fw1, (size_t)n, &g->acct));
    g->b_lq_cap = (uint32_t)z.lq_cap;
    HIP_TRY(dalloc(&g->b_lq_vtx, (size_t)z.lq_cap, &g->acct));
    HIP_TRY(dalloc(&g->b_lq_mask, (size_t)z.lq_cap, &g->acct));
    g->b_max_levels = (int32_t)z.max_levels;
    HIP_TRY(dalloc(&g->b_level_off, (size_t)g->b_max_levels + 2, &g->acct));
    // per-(vertex, lane) slabs of path counts, c and delta
    HIP_TRY(dalloc(&g->b_sigma, (size_t)n * kLanes, &g->acct));
    HIP_TRY(dalloc(&g->b_chat, (size_t)n * kLanes, &g->acct));
    HIP_TRY(dalloc(&g->b_delta, (size_t)n * kLanes, &g->acct));
    g->b_gcap = (uint32_t)z.gcap;
    HIP_TRY(dalloc(&g->b_gstart, (size_t)z.gcap, &g->acct));
    // group bases, then the summation options chosen at each level
    HIP_TRY(dalloc(&g->b_gbase, 2 * ((size_t)g->b_max_levels + 2), &g->acct));
    HIP_TRY(dalloc(&g->b_shift, ((size_t)g->b_max_levels + 2) * kLanes, &g->acct));
    HIP_TRY(dalloc(&g->b_maxexp, (size_t)2 * kSlots * kLanes, &g->acct));
    HIP_TRY(dalloc(&g->b_lane_src, (size_t)kLanes, &g->acct));
    bc_status s = alloc_hq(g, &g->b_hq, z.hq_entries, z.hq_levels, kLanes, g->heavy_segs);
    if (s != BC_OK) return s;
    g->batch_ready = true;
    return BC_OK;
}

template <typename T>
static bc_status grow(T **p, int64_t *cap, int64_t need, ByteAcct *acct) {
    if (need <= *cap && *p) return BC_OK;
    if (*p) {
        HIP_TRY(hipFree(*p));
        *p = nullptr;
        acct->bytes -= (size_t)(*cap) * sizeof(T);
        *cap = 0;
    }
    int64_t c = std::max<int64_t>(need, 16);
    HIP_TRY(dalloc(p, (size_t)c, acct));
    *cap = c;
    return BC_OK;
}

// ------------------------------------------------------------------ driver
struct RunCfg {
    int engine;   // 1 = plain, 64 = batched
    int lanes;    // batched: sources per batch (8 .. 64)
    int mode;     // 0 / 1
    int policy;   // POL_*
    int grid;
    int chunk;
    bool use_graphs;
    bool f64_check = false;  // batched FP64 pass: lanes whose counts stay below 2^65 are handed back
};

template <typename Args>
static bc_status get_graph(bc_graph *g, const Args &args, void (*kern)(Args), const RunCfg &cfg,
                           hipStream_t launch_st, hipGraphExec_t *out) {
    std::vector<unsigned char> key(sizeof(Args) + 3 * sizeof(int));
    std::memcpy(key.data(), &args, sizeof(Args));
    int extra[3] = {cfg.grid, cfg.chunk, cfg.engine * 2 + cfg.mode};
    std::memcpy(key.data() + sizeof(Args), extra, sizeof(extra));
    for (auto &cg : g->graphs)
        if (cg.key == key) {
            *out = cg.exec;
            return BC_OK;
        }
    CachedGraph cg;
    cg.key = key;
    // capture on a private non-blocking stream: capturing a blocking stream
    // would forbid legacy-stream work in other threads (concurrent parts)
    (void)launch_st;
    if (!g->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = g->cap_stream;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    Args argcopy = args;
    void *kargs[] = {(void *)&argcopy};
    for (int i = 0; i < cfg.chunk; ++i)
        (void)hipLaunchKernel((const void *)kern, dim3(cfg.grid), dim3(kBlock), kargs, 0, cs);
    // flag readback at the end of the chunk
    (void)hipMemcpyAsync(g->flag_host, g->ctl, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, cs);
    hipError_t e = hipStreamEndCapture(cs, &cg.graph);
    if (e != hipSuccess) return fail(BC_ERR_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&cg.exec, cg.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(cg.graph);
        return fail(BC_ERR_DEVICE, std::string("graph instantiate failed: ") + hipGetErrorString(e));
    }
    if (g->graphs.size() >= 16) {
        (void)hipGraphExecDestroy(g->graphs.front().exec);
        (void)hipGraphDestroy(g->graphs.front().graph);
        g->graphs.erase(g->graphs.begin());
    }
    g->graphs.push_back(cg);
    *out = cg.exec;
    return BC_OK;
}

// Launch chunks of step kernels until the device state machine reports done.
template <typename Args>
static bc_status drive(bc_graph *g, const Args &args, void (*kern)(Args), const RunCfg &cfg, hipStream_t st,
                       int64_t max_steps, int64_t *launches, double *dev_ms) {
    hipGraphExec_t exec = nullptr;
    if (cfg.use_graphs) {
        bc_status s = get_graph(g, args, kern, cfg, st, &exec);
        if (s != BC_OK) return s;
    }
    const int kRing = 4;
    hipEvent_t ev[kRing];
    for (int i = 0; i < kRing; ++i) HIP_TRY(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
    // device time of the whole pass: from before the first step launch to
    // after the last, on the launch stream
    hipEvent_t t_ev[2];
    HIP_TRY(hipEventCreate(&t_ev[0]));
    HIP_TRY(hipEventCreate(&t_ev[1]));
    HIP_TRY(hipEventRecord(t_ev[0], st));
    int64_t issued = 0, chunks = 0;
    bc_status result = BC_OK;
    g->flag_host[0] = PH_IDLE;
    g->flag_host[1] = 0;
    const auto t0 = std::chrono::steady_clock::now();
    double max_seconds = 900.0;
    if (const char *s = std::getenv("BC_MAX_SECONDS")) max_seconds = std::atof(s);
    for (;;) {
        if (chunks >= kRing) {
            hipError_t e = hipEventSynchronize(ev[chunks % kRing]);
            if (e != hipSuccess) { result = fail(BC_ERR_DEVICE, std::string("step sync: ") + hipGetErrorString(e)); break; }
            const int32_t ph = ((volatile int32_t *)g->flag_host)[0];
            const int32_t er = ((volatile int32_t *)g->flag_host)[1];
            if (er) break;  // reported by the caller from the control block
            if (ph == PH_DONE) break;
        }
        if (issued >= max_steps) {
            result = fail(BC_ERR_DEVICE, "level state machine did not finish within its step bound");
            break;
        }
        if (std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() > max_seconds) {
            result = fail(BC_ERR_DEVICE, "run exceeded BC_MAX_SECONDS");
            break;
        }
        if (exec) {
            hipError_t e = hipGraphLaunch(exec, st);
            if (e != hipSuccess) { result = fail(BC_ERR_DEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e)); break; }
        } else {
            Args argcopy = args;
            void *kargs[] = {(void *)&argcopy};
            for (int i = 0; i < cfg.chunk; ++i)
                (void)hipLaunchKernel((const void *)kern, dim3(cfg.grid), dim3(kBlock), kargs, 0, st);
            hipError_t e = hipMemcpyAsync(g->flag_host, g->ctl, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, st);
            if (e != hipSuccess) { result = fail(BC_ERR_DEVICE, std::string("flag copy: ") + hipGetErrorString(e)); break; }
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) { result = fail(BC_ERR_DEVICE, std::string("step launch: ") + hipGetErrorString(e)); break; }
        e = hipEventRecord(ev[chunks % kRing], st);
        if (e != hipSuccess) { result = fail(BC_ERR_DEVICE, std::string("event record: ") + hipGetErrorString(e)); break; }
        issued += cfg.chunk;
        ++chunks;
    }
    (void)hipEventRecord(t_ev[1], st);
    hipError_t e = hipStreamSynchronize(st);
    float pass_ms = 0.0f;
    if (e == hipSuccess && hipEventElapsedTime(&pass_ms, t_ev[0], t_ev[1]) == hipSuccess) *dev_ms += pass_ms;
    (void)hipEventDestroy(t_ev[0]);
    (void)hipEventDestroy(t_ev[1]);
    for (int i = 0; i < kRing; ++i) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess && result == BC_OK) result = fail(BC_ERR_DEVICE, std::string("stream sync: ") + hipGetErrorString(e));
    *launches += issued;
    return result;
}

static void init_ctl(Ctl *c) {
    std::memset(c, 0, sizeof(*c));
    c->dump_pos = -1;
    c->dump_lane = -1;
    c->maxexp = INT_MIN;
    c->minexp = INT_MAX;
}

static PolicyArgs policy_args(const bc_graph *g, const bc_run_options &o) {
    PolicyArgs p;
    p.alpha = o.alpha > 0 ? o.alpha : 14.0f;
    p.beta = o.beta > 0 ? o.beta : 24.0f;
    p.wpv_degree = o.wpv_degree > 0 ? o.wpv_degree : 24.0f;
    p.item_lanes = o.lanes_per_entry > 0 ? o.lanes_per_entry : (o.lanes_per_entry < 0 ? -1.0f : 4.0f);
    p.margin = o.policy_margin > 0 ? o.policy_margin : (o.policy_margin < 0 ? 0.0f : kPolicyMargin);
    p.has_mlp = g->has_mlp ? 1 : 0;
    p.mlp = g->mlp;
    return p;
}

struct DumpBufs {
    int32_t *d = nullptr;
    unsigned long long *sig = nullptr;
    double *delta = nullptr;
    int32_t *shift = nullptr;
    int64_t *d64 = nullptr;  // weighted graphs: distances
};

// Algorithmic bytes: every scanned arc reads its column index and a 4-8 byte
// word of the neighbour (8 B + 8 B), every DAG (arc, source) pair moves one
// 8-byte path count or c value, every level-queue entry costs its row
// offsets, queue slots and per-vertex words (32 B), and every reached
// (vertex, source) pair moves five 8-byte slab values: its path count written
// (forward) and read (backward), c and delta written (backward), delta read
// (score accumulation).  algo_bytes_arcs leaves the last term out.
static double algo_bytes_arcs(const bc_stats &s) {
    return 16.0 * (double)s.arcs_scanned + 8.0 * (double)s.lane_arcs + 32.0 * (double)s.queue_entries;
}
static double algo_bytes(const bc_stats &s) { return algo_bytes_arcs(s) + 40.0 * (double)s.reached_pairs; }
// Weighted engine: 16 B per arc visit (target or source id, weight, the
// other end's 64-bit distance) in the relaxation rounds and in the four
// passes over the reached vertices' arcs (DAG in-arc counts, path counts,
// release of successors, dependencies); 64 B per reached (vertex, source)
// pair (distance set and reset, path count, c and delta written, delta read
// into the partial scores, the partial's read-modify-write).
static double algo_bytes_weighted(double relax_bytes, double dag_arcs, double reached) {
    return relax_bytes + 16.0 * dag_arcs + 64.0 * reached;
}

// Lane-batched weighted engine: 8 B per arc read by a round's entry (far end
// and weight, once for all sources of the entry), 8 B per (arc, source) pair
// (the far end's 64-bit distance, path count or c of that source), 64 B per
// reached (vertex, source) pair as above.
static double algo_bytes_wbatch(double entry_arcs, double lane_arcs, double reached) {
    return 8.0 * entry_arcs + 8.0 * lane_arcs + 64.0 * reached;
}

static void accumulate_stats(bc_stats *s, const Ctl &c, double clock_khz) {
    for (int i = 0; i < kPhases; ++i) s->phase_ms[i] += (double)c.st_ticks[i] / clock_khz;
    for (int i = 0; i < 3; ++i) s->variant_ms[i] += (double)c.st_vticks[i] / clock_khz;
    for (int i = 0; i < kPhases; ++i) {
        s->phase_arcs[i] += (int64_t)c.st_parcs[i];
        s->phase_lane_arcs[i] += (int64_t)c.st_plarcs[i];
        s->phase_pairs[i] += (int64_t)c.st_ppairs[i];
    }
    s->steps += (int64_t)c.st_steps;
    s->forward_levels += (int64_t)c.st_fwd_levels;
    for (int i = 0; i < 3; ++i) s->variant_levels[i] += (int64_t)c.st_var[i];
    s->arcs_scanned += (int64_t)c.st_arcs;
    s->lane_arcs += (int64_t)c.st_lane_arcs;
    s->queue_entries += (int64_t)c.st_qentries;
    s->reached_pairs += (int64_t)c.st_lane_entries;
    s->max_levels = std::max<int64_t>(s->max_levels, (int64_t)c.st_max_levels);
    s->n_batches += (int64_t)c.st_batches;
}

static bc_status ctl_error(const Ctl &c) {
    if (c.err & ERR_SIGMA_RANGE)
        return fail(BC_ERR_SIGMA_RANGE, "scaled FP64 path counts left the double range");
    if (c.err & ERR_LEVEL_CAP) return fail(BC_ERR_NOT_SUPPORTED, "more BFS levels than the batched engine holds (65534)");
    if (c.err) return fail(BC_ERR_DEVICE, "device capacity error (queue / overflow list)");
    return BC_OK;
}

// One pass of one engine over a device source list.  Overflowed source
// positions (mode 0) are returned in *ovf_positions.
struct CollectBufs {
    float *X = nullptr, *Y = nullptr;  // device
    float *F = nullptr;                // device: per-level features of the current batch
    uint32_t cap = 0;
};

static bc_status run_pass(bc_graph *g, const RunCfg &cfg, const bc_run_options &o, const int32_t *h_srcs,
                          int64_t ns, int64_t dump_pos, DumpBufs *dump, hipStream_t st,
                          std::vector<int64_t> *ovf_positions, int *dump_done, Ctl *ctl_out,
                          const CollectBufs *col = nullptr) {
    bc_status s;
    // engine state first: it is by far the largest allocation, so a run
    // refused under the device-memory cap allocates nothing
    s = cfg.engine == 1 ? ensure_plain(g, st) : ensure_batched(g);
    if (s != BC_OK) return s;
    s = grow(&g->srcs, &g->srcs_cap, ns, &g->acct);
    if (s != BC_OK) return s;
    s = grow(&g->ovf, &g->ovf_cap, ns, &g->acct);
    if (s != BC_OK) return s;
    if (ns) HIP_TRY(hipMemcpyAsync(g->srcs, h_srcs, sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
    Ctl *hc = g->ctl_host;
    init_ctl(hc);
    hc->policy = cfg.policy;
    hc->mode = cfg.mode;
    hc->f64_check = cfg.f64_check ? 1 : 0;
    hc->dump_pos = dump_pos;
    const unsigned long long limit = o.sigma_limit > 0 ? (unsigned long long)o.sigma_limit : ~0ull;
    GraphArgs ga;
    ga.n = g->n;
    ga.nnz_lo = (int32_t)g->nnz;
    ga.row_ptr = g->row_ptr;
    ga.col = g->col;
    ga.directed = g->directed ? 1 : 0;
    ga.in_row_ptr = g->directed ? g->in_row_ptr : g->row_ptr;
    ga.in_col = g->directed ? g->in_col : g->col;
    ga.nonisolated = g->nonisolated;
    ga.hv_vtx = g->hv_vtx;
    ga.hv_seg = g->hv_seg;
    ga.n_heavy = g->n_heavy;
    int64_t launches = 0;
    double dev_ms = 0.0;
    if (cfg.engine == 1) {
        ga.hv_vtx = g->p_hv_vtx;
        ga.hv_seg = g->p_hv_seg;
        ga.n_heavy = g->p_n_heavy;
        hc->phase = PH_FIN;
        hc->pos = -1;
        hc->n_items = ns;
        hc->total_queued = 0;
        HIP_TRY(hipMemcpyAsync(g->ctl, hc, sizeof(Ctl), hipMemcpyHostToDevice, st));
        PlainArgs a;
        std::memset(&a, 0, sizeof(a));
        a.g = ga;
        a.p = policy_args(g, o);
        a.ctl = g->ctl;
        a.d = g->p_d;
        a.sig = g->p_sig;
        a.chat = g->p_chat;
        a.bc = g->bc;
        a.queue = g->p_queue;
        a.level_off = g->p_level_off;
        a.shift = g->p_shift;
        a.srcs = g->srcs;
        a.ovf_list = g->ovf;
        a.ovf_cap = (uint32_t)std::min<int64_t>(g->ovf_cap, UINT32_MAX);
        a.sigma_limit = limit;
        a.hq = g->p_hq;
        a.lvl = g->lvl;
        if (dump) {
            a.dump_d = dump->d;
            a.dump_sig = dump->sig;
            a.dump_delta = dump->delta;
            a.dump_shift = dump->shift;
        }
        const double bound = (double)ns * (2.0 * (double)g->n + 6.0) + 64.0;
        const int64_t max_steps = bound > 4e18 ? (int64_t)4e18 : (int64_t)bound;
        s = drive(g, a, cfg.mode ? plain_step<1> : plain_step<0>, cfg, st, max_steps, &launches, &dev_ms);
        if (s != BC_OK) g->plain_dirty = true;
    } else {
        // batches of up to 64 sources that never cross a graph boundary
        std::vector<int64_t> bs;
        std::vector<int32_t> lo, hi;
        int64_t i = 0;
        while (i < ns) {
            const int32_t v = h_srcs[i];
            const int gi = (int)(std::upper_bound(g->voff.begin(), g->voff.end(), v) - g->voff.begin()) - 1;
            const int32_t glo = g->voff[gi], ghi = g->voff[gi + 1];
            int64_t j = i + 1;
            while (j < ns && j - i < cfg.lanes && h_srcs[j] >= glo && h_srcs[j] < ghi) ++j;
            bs.push_back(i);
            lo.push_back(glo);
            hi.push_back(ghi);
            i = j;
        }
        bs.push_back(ns);
        const int64_t nb = (int64_t)lo.size();
        s = grow(&g->bstart, &g->bcap[0], nb + 1, &g->acct);
        if (s != BC_OK) return s;
        s = grow(&g->blo, &g->bcap[1], nb + 1, &g->acct);
        if (s != BC_OK) return s;
        s = grow(&g->bhi, &g->bcap[2], nb + 1, &g->acct);
        if (s != BC_OK) return s;
        HIP_TRY(hipMemcpyAsync(g->bstart, bs.data(), sizeof(int64_t) * bs.size(), hipMemcpyHostToDevice, st));
        if (nb) {
            HIP_TRY(hipMemcpyAsync(g->blo, lo.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
            HIP_TRY(hipMemcpyAsync(g->bhi, hi.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
        }
        // fresh tags and visited words for this run
        const int64_t n = g->n;
        if (n > 0) {
            fill_u64<<<grid_for(2 * n, 256, 4096), 256, 0, st>>>((unsigned long long *)g->b_vn, 2 * n, 0ull);
            fill_u64<<<grid_for(2 * n, 256, 4096), 256, 0, st>>>((unsigned long long *)g->b_fw0, 2 * n, 0ull);
            fill_u64<<<grid_for(2 * n, 256, 4096), 256, 0, st>>>((unsigned long long *)g->b_fw1, 2 * n, 0ull);
        }
        fill_i32<<<8, 256, 0, st>>>(g->b_maxexp, kSlots * kLanes, INT_MIN);
        fill_i32<<<8, 256, 0, st>>>(g->b_maxexp + kSlots * kLanes, kSlots * kLanes, INT_MAX);
        HIP_TRY(hipGetLastError());
        hc->phase = PH_BC;
        hc->pos = -1;
        hc->n_items = nb;
        hc->collect = col ? 1 : 0;
        hc->range_lo = 0;
        hc->range_hi = 0;
        hc->epoch_b = 0;
        hc->n_levels = 0;
        HIP_TRY(hipMemcpyAsync(g->ctl, hc, sizeof(Ctl), hipMemcpyHostToDevice, st));
        BatchArgs a;
        std::memset(&a, 0, sizeof(a));
        a.g = ga;
        a.p = policy_args(g, o);
        a.ctl = g->ctl;
        a.vn = g->b_vn;
        a.fw0 = g->b_fw0;
        a.fw1 = g->b_fw1;
        a.lq_vtx = g->b_lq_vtx;
        a.lq_mask = g->b_lq_mask;
        a.lq_cap = g->b_lq_cap;
        a.level_off = g->b_level_off;
        a.max_levels = g->b_max_levels;
        a.delta = g->b_delta;
        a.sigma = g->b_sigma;
        a.chat = g->b_chat;
        a.gstart = g->b_gstart;
        a.gbase = g->b_gbase;
        a.lbsel = (int32_t *)(g->b_gbase + g->b_max_levels + 2);
        a.gcap = g->b_gcap;
        a.shift = g->b_shift;
        a.maxexp = g->b_maxexp;
        a.bc = g->bc;
        a.srcs = g->srcs;
        a.batch_start = g->bstart;
        a.batch_lo = g->blo;
        a.batch_hi = g->bhi;
        a.lane_src = g->b_lane_src;
        a.hq = g->b_hq;
        a.lvl = g->lvl;
        if (col) {
            a.col_X = col->X;
            a.col_Y = col->Y;
            a.col_F = col->F;
            a.col_cap = col->cap;
        }
        a.ovf_list = g->ovf;
        a.ovf_cap = (uint32_t)std::min<int64_t>(g->ovf_cap, UINT32_MAX);
        a.sigma_limit = limit;
        if (dump) {
            a.dump_d = dump->d;
            a.dump_sig = dump->sig;
            a.dump_delta = dump->delta;
            a.dump_shift = dump->shift;
        }
        const int64_t maxl = std::min<int64_t>(g->n, g->b_max_levels) + 2;
        const int64_t max_steps = (nb + 1) * ((col ? 7 : 3) * maxl + 8) + 64;
        s = drive(g, a, cfg.mode ? batch_step<1> : batch_step<0>, cfg, st, max_steps, &launches, &dev_ms);
    }
    g->stats.launches += launches;
    if (s != BC_OK) return s;
    HIP_TRY(hipMemcpyAsync(hc, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *ctl_out = *hc;
    const double bytes0 = algo_bytes(g->stats);
    accumulate_stats(&g->stats, *hc, g->clock_khz);
    const int mi = cfg.mode ? 1 : 0;
    g->stats.mode_launches[mi] += launches;
    g->stats.mode_ms[mi] += dev_ms;
    g->stats.mode_algo_bytes[mi] += algo_bytes(g->stats) - bytes0;
    if (hc->err) {
        g->plain_dirty = true;
        return ctl_error(*hc);
    }
    if (hc->phase != PH_DONE) return fail(BC_ERR_DEVICE, "run ended before the state machine finished");
    if (dump_done) *dump_done = hc->dump_state == 2;
    if (ovf_positions && hc->n_ovf) {
        std::vector<int64_t> tmp(hc->n_ovf);
        HIP_TRY(hipMemcpyAsync(tmp.data(), g->ovf, sizeof(int64_t) * hc->n_ovf, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        std::sort(tmp.begin(), tmp.end());
        *ovf_positions = tmp;
    }
    return BC_OK;
}

static bc_status resolve_cfg(const bc_graph *g, const bc_run_options &o, int64_t ns, RunCfg *cfg) {
    if (o.batch != 0 && o.batch != 1 && o.batch != 8 && o.batch != 16 && o.batch != 32 && o.batch != 64)
        return fail(BC_ERR_INVALID_ARG, "batch must be 0, 1, 8, 16, 32 or 64");
    cfg->engine = o.batch == 1 ? 1 : 64;
    if (o.batch == 0) cfg->engine = ns >= 2 ? 64 : 1;
    cfg->lanes = (o.batch >= 8) ? o.batch : 64;
    if (g->directed && cfg->engine == 1) {  // one source per traversal on the batched engine
        cfg->engine = 64;
        cfg->lanes = 1;
    }
    switch (o.policy) {
    case BC_POLICY_AUTO: cfg->policy = g->has_mlp ? POL_MLP : POL_HEUR; break;
    case BC_POLICY_HEURISTIC: cfg->policy = POL_HEUR; break;
    case BC_POLICY_MLP:
        if (!g->has_mlp) return fail(BC_ERR_INVALID_ARG, "BC_POLICY_MLP without loaded weights");
        cfg->policy = POL_MLP;
        break;
    case BC_POLICY_FORCE_PUSH_TPV: cfg->policy = POL_FORCE_TPV; break;
    case BC_POLICY_FORCE_PUSH_WPV: cfg->policy = POL_FORCE_WPV; break;
    case BC_POLICY_FORCE_PULL: cfg->policy = POL_FORCE_PULL; break;
    default: return fail(BC_ERR_INVALID_ARG, "unknown policy");
    }
    if (o.grid_blocks < 0 || o.grid_blocks > 65536) return fail(BC_ERR_INVALID_ARG, "grid_blocks out of range");
    if (o.chunk_steps < 0 || o.chunk_steps > 4096) return fail(BC_ERR_INVALID_ARG, "chunk_steps out of range");
    cfg->grid = o.grid_blocks ? o.grid_blocks : (cfg->engine == 1 ? g->grid_plain : g->grid_batch);
    cfg->chunk = o.chunk_steps ? o.chunk_steps : 16;
    cfg->use_graphs = !(o.flags & BC_RUN_NO_GRAPHS);
    cfg->mode = 0;
    return BC_OK;
}

// ------------------------------------------------ concurrent sub-unions
// A handle over many graphs (block-diagonal union) runs its batched work as
// up to 16 sub-unions (environment BC_PARTS overrides, at least two graphs
// per part), each a handle of its own on its own stream with a dedicated
// hardware queue, driven from its own host thread, so the level steps of
// different graphs overlap on the device (one level state machine leaves
// the GPU idle during the small steps of small graphs).  Graphs are dealt
// by size; a part keeps its graphs in the parent's order and a graph's
// sources in list order, so every score is accumulated in the same order as
// by one handle and the results are identical bit for bit.
// 16 by default: on 512 BA graphs (64 sources each) 16 parts ran 22 % faster
// than 8 (26.5 vs 21.7 GTEPS); on every 64th source of the 512 graphs, 16
// parts 36.3 GTEPS, 24 or 32 parts 29.0.  BC_PARTS overrides (2 .. 32).
static int n_parts() {
    static const int np = [] {
        const char *e = std::getenv("BC_PARTS");
        const int v = e ? std::atoi(e) : 16;
        return std::min(32, std::max(2, v));
    }();
    return np;
}

__global__ void gather_f64(double *dst, const double *src, const int32_t *map, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[map[i]];
}
__global__ void scatter_f64(double *dst, const double *src, const int32_t *map, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[map[i]] = src[i];
}

struct PartScores {
    const double *p[16];
    int n;
};
// dst[v] = (acc ? dst[v] : 0) + the parts' scores added in part order
__global__ void sum_parts_f64(double *dst, PartScores ps, int acc, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double t = ps.p[0][i];
        for (int k = 1; k < ps.n; ++k) t += ps.p[k][i];
        dst[i] = acc ? dst[i] + t : t;
    }
}

// ------------------------------------------------------------ block engine
// Graphs of at most kBlockMaxN vertices: one persistent launch of block_run
// in which every workgroup owns a level state machine and works through
// chunks of consecutive batches of one graph (see bc_dev.h).  A chunk's
// scores go to a partial vector; block_sum then adds, for every vertex, the
// partials of its graph's chunks in batch order.  The result is
// deterministic for a given run (the chunking depends only on the graph
// sizes, the source list and the number of workgroups), but the additions
// are grouped per chunk, so it agrees with one level state machine to
// rounding only.  Capacities of a workgroup's state are sized for the
// largest graph with a margin; a run that exceeds one (or overflows a
// workgroup's list of 64-bit overflows) is run again by the general engine.

// dst[v] += partial scores of v's graph, chunk by chunk in batch order.
// gsum: per graph with chunks {lo, hi, first, end} into lst (part offsets).
__global__ void block_sum(double *dst, const double *partials, const int32_t *gsum, int32_t n_gsum,
                          const int64_t *lst) {
    for (int32_t k = blockIdx.y; k < n_gsum; k += gridDim.y) {
        const int32_t lo = gsum[4 * k], hi = gsum[4 * k + 1], c0 = gsum[4 * k + 2], c1 = gsum[4 * k + 3];
        for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < hi - lo; i += gridDim.x * blockDim.x) {
            double t = dst[lo + i];
            for (int32_t c = c0; c < c1; ++c) t += partials[lst[c] + i];
            dst[lo + i] = t;
        }
    }
}

// Zero the two tagged frontier arrays of every workgroup (tags restart each run).
__global__ void block_clear_tags(char *scratch, size_t stride, size_t off, size_t bytes, int nwg) {
    const size_t words = bytes / 8;
    for (int w = blockIdx.y; w < nwg; w += gridDim.y) {
        unsigned long long *p = (unsigned long long *)(scratch + (size_t)w * stride + off);
        for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
            p[i] = 0ull;
    }
}

// Largest graph, cost units, heavy vertices and segments over the handle's
// graphs (entries classified by the larger of out- and in-degree).
static bc_status block_facts(bc_graph *g) {
    if (g->blk_sized) return BC_OK;
    const int32_t n = g->n;
    std::vector<int32_t> rp((size_t)n + 1), irp;
    HIP_TRY(hipMemcpy(rp.data(), g->row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost));
    if (g->directed) {
        irp.resize((size_t)n + 1);
        HIP_TRY(hipMemcpy(irp.data(), g->in_row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost));
    }
    int32_t nmax = 0;
    int64_t cmax = 0, hmax = 0, smax = 0;
    for (int gi = 0; gi < g->n_graphs; ++gi) {
        const int32_t lo = g->voff[gi], hi = g->voff[gi + 1];
        int64_t cost = 0, heavy = 0, segs = 0;
        for (int32_t v = lo; v < hi; ++v) {
            int32_t d = rp[v + 1] - rp[v];
            if (g->directed) d = std::max(d, irp[v + 1] - irp[v]);
            cost += entry_cost(d);
            if (d > kSegBatched) {
                ++heavy;
                segs += (d + kSegBatched - 1) / kSegBatched;
            }
        }
        nmax = std::max(nmax, hi - lo);
        cmax = std::max(cmax, cost);
        hmax = std::max(hmax, heavy);
        smax = std::max(smax, segs);
    }
    g->blk_nmax = nmax;
    g->blk_cost_max = cmax;
    g->blk_heavy_max = hmax;
    g->blk_segs_max = smax;
    g->blk_sized = true;
    return BC_OK;
}

// Capacities of one workgroup's state (once per handle) and how many
// workgroups can run: resident ones (occupancy) that fit in the memory
// budget (half the free device memory, at most 96 GiB, under the handle's
// cap).  Returns 0 workgroups when not even one fits.
static bc_status block_dims(bc_graph *g, int *resident) {
    BlockArgs &d = g->blk_dims;
    const int64_t nmax = std::max<int32_t>(g->blk_nmax, 1);
    d.nmax = (int32_t)nmax;
    d.max_levels = (int32_t)std::min<int64_t>(nmax + 2, 4096);
    // every (vertex, lane) pair enters a batch's queues at most once: small
    // graphs get that bound, larger ones 16 entries per vertex
    d.lq_cap = (uint32_t)std::min<int64_t>(std::max<int64_t>(16 * nmax + 4096, (int64_t)1 << 20),
                                           (int64_t)kLanes * nmax + 64);
    d.gcap = (uint32_t)((int64_t)kLanes * g->blk_cost_max / kBudget + 2 * ((int64_t)d.max_levels + 2) + 64);
    d.hq_entries = (uint32_t)(g->blk_heavy_max * kLanes + kLanes);
    d.hq_levels = (uint32_t)d.max_levels + 3;
    d.part_cap = (uint32_t)(g->blk_segs_max + 1);
    d.ovf_cap = 4096;
    const BlockLayout L((size_t)d.nmax, d.lq_cap, (size_t)d.max_levels, d.gcap, d.hq_entries, d.hq_levels,
                        d.part_cap, d.ovf_cap);
    g->blk_stride = L.bytes;
    int dev = 0, cus = 0, per_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)block_run<0>, kBlock, 0));
    int64_t want = (int64_t)std::max(1, cus) * std::max(1, per_cu);
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    // what this handle already holds for the block engine counts as free
    free_b += (size_t)g->blk_wg * (g->blk_stride + sizeof(Ctl));
    size_t budget = std::min<size_t>(free_b / 4 * 3, (size_t)192 << 30);
    if (g->acct.limit) {
        const size_t held = (size_t)g->blk_wg * (g->blk_stride + sizeof(Ctl));
        const size_t room = g->acct.limit > g->acct.bytes - held ? g->acct.limit - (g->acct.bytes - held) : 0;
        budget = std::min(budget, room);
    }
    want = std::min<int64_t>(want, (int64_t)(budget / (g->blk_stride + sizeof(Ctl))));
    *resident = (int)std::max<int64_t>(want, 0);
    return BC_OK;
}

// State for `need` workgroups (kept and grown across runs).
static bc_status ensure_block(bc_graph *g, int need) {
    if (g->blk_wg >= need) return BC_OK;
    if (g->blk_scratch) {
        HIP_TRY(hipStreamSynchronize(nullptr));
        (void)hipFree(g->blk_scratch);
        (void)hipFree(g->blk_ctls);
        g->acct.bytes -= (size_t)g->blk_wg * (g->blk_stride + sizeof(Ctl));
        g->blk_scratch = nullptr;
        g->blk_ctls = nullptr;
        g->blk_wg = 0;
    }
    HIP_TRY(dalloc(&g->blk_scratch, (size_t)need * g->blk_stride, &g->acct));
    HIP_TRY(dalloc(&g->blk_ctls, (size_t)need, &g->acct));
    if (!g->blk_next) HIP_TRY(dalloc(&g->blk_next, 1, &g->acct));
    g->blk_wg = need;
    return BC_OK;
}

// The block engine is used for runs of the batched engine without a detail
// dump over handles whose graphs all have at most kBlockMaxN vertices, always
// with BC_RUN_BLOCKS, never with BC_RUN_NO_BLOCKS or BC_RUN_ONE_QUEUE, and by
// default when every graph has at most kBlockDefaultN vertices and the list
// fills 8 batches.  (A workgroup holds fewer wavefronts than a CU can run,
// so on larger graphs, whose level steps keep the whole GPU busy, the
// general engine is faster: 38.0 against 29.4 GTEPS on the BA union
// sample; on ER(2000) the block engine is faster, 2.36 against 1.65.)
constexpr int kBlockDefaultN = 16384;
static bool use_block(bc_graph *g, const bc_run_options &o, int64_t ns, bool detail) {
    if (g->weighted || detail || o.batch == 1 || (o.flags & (BC_RUN_NO_BLOCKS | BC_RUN_ONE_QUEUE | BC_RUN_FORCE_F64)))
        return false;
    if (o.batch == 0 && ns < 2) return false;
    if (block_facts(g) != BC_OK || g->blk_nmax > kBlockMaxN || g->blk_nmax < 1) return false;
    if (o.flags & BC_RUN_BLOCKS) return true;
    const int K = o.batch >= 8 ? o.batch : 64;
    return g->blk_nmax <= kBlockDefaultN && ns >= 8 * (int64_t)K;
}

// One 64-bit pass over h_srcs on the block engine.  *fallback = true when a
// workgroup's capacity was exceeded or its state does not fit: nothing was
// added to the scores and the caller runs the general engine instead.
static bc_status run_block(bc_graph *g, const RunCfg &cfg, const bc_run_options &o, const int32_t *h_srcs,
                           int64_t ns, hipStream_t st, std::vector<int64_t> *ovf_positions, bool *fallback) {
    *fallback = false;
    ovf_positions->clear();
    if (ns == 0) return BC_OK;
    int resident = 0;
    bc_status s = block_dims(g, &resident);
    if (s != BC_OK) return s;
    if (resident < 1) {
        *fallback = true;
        return BC_OK;
    }
    const BlockArgs &dm = g->blk_dims;
    s = grow(&g->srcs, &g->srcs_cap, ns, &g->acct);
    if (s != BC_OK) return s;
    HIP_TRY(hipMemcpyAsync(g->srcs, h_srcs, sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
    // batches of up to K sources of one graph (as in the general engine)
    std::vector<int64_t> bs;
    std::vector<int32_t> blo, bhi, bg;
    for (int64_t i = 0; i < ns;) {
        const int32_t v = h_srcs[i];
        const int gi = (int)(std::upper_bound(g->voff.begin(), g->voff.end(), v) - g->voff.begin()) - 1;
        const int32_t glo = g->voff[gi], ghi = g->voff[gi + 1];
        int64_t j = i + 1;
        while (j < ns && j - i < cfg.lanes && h_srcs[j] >= glo && h_srcs[j] < ghi) ++j;
        bs.push_back(i);
        blo.push_back(glo);
        bhi.push_back(ghi);
        bg.push_back(gi);
        i = j;
    }
    bs.push_back(ns);
    const int64_t nb = (int64_t)blo.size();
    // chunks: runs of at most C consecutive batches of one graph, about four
    // per resident workgroup
    const int64_t C =
        std::min<int64_t>(64, std::max<int64_t>(1, (nb + 4 * (int64_t)resident - 1) / (4 * (int64_t)resident)));
    std::vector<int32_t> cb0, cb1;
    for (int64_t b = 0; b < nb;) {
        int64_t e = b + 1;
        while (e < nb && e - b < C && bg[e] == bg[b]) ++e;
        cb0.push_back((int32_t)b);
        cb1.push_back((int32_t)e);
        b = e;
    }
    const int64_t nc = (int64_t)cb0.size();
    const int nwg = (int)std::min<int64_t>(resident, nc);
    s = ensure_block(g, nwg);
    if (s == BC_ERR_OUT_OF_MEMORY) {  // the general engine needs less: let it run
        *fallback = true;
        return BC_OK;
    }
    if (s != BC_OK) return s;
    std::vector<int64_t> part_off((size_t)nc);
    int64_t tot = 0;
    for (int64_t t = 0; t < nc; ++t) {
        part_off[t] = tot;
        tot += bhi[cb0[t]] - blo[cb0[t]];
    }
    // per graph, its chunks in batch order (the summation order)
    std::vector<std::vector<int64_t>> per_graph((size_t)g->n_graphs);
    for (int64_t t = 0; t < nc; ++t) per_graph[bg[cb0[t]]].push_back(t);
    std::vector<int32_t> gsum;
    std::vector<int64_t> lst;
    for (int gi = 0; gi < g->n_graphs; ++gi) {
        if (per_graph[gi].empty()) continue;
        gsum.push_back(g->voff[gi]);
        gsum.push_back(g->voff[gi + 1]);
        gsum.push_back((int32_t)lst.size());
        for (int64_t t : per_graph[gi]) lst.push_back(part_off[t]);
        gsum.push_back((int32_t)lst.size());
    }
    // dispatch order: largest work (vertices x sources of the chunk) first
    std::vector<int32_t> order((size_t)nc);
    for (int64_t t = 0; t < nc; ++t) order[t] = (int32_t)t;
    std::vector<double> work((size_t)nc);
    for (int64_t t = 0; t < nc; ++t)
        work[t] = (double)(bhi[cb0[t]] - blo[cb0[t]]) * (double)(bs[cb1[t]] - bs[cb0[t]]);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a_, int32_t b_) { return work[a_] > work[b_]; });
    // device copies
    s = grow(&g->bstart, &g->bcap[0], nb + 1, &g->acct);
    if (s == BC_OK) s = grow(&g->blo, &g->bcap[1], nb + 1, &g->acct);
    if (s == BC_OK) s = grow(&g->bhi, &g->bcap[2], nb + 1, &g->acct);
    if (s == BC_OK) s = grow(&g->blk_chunk, &g->blk_chunk_cap, 3 * nc, &g->acct);
    if (s == BC_OK) s = grow(&g->blk_part_off, &g->blk_part_off_cap, std::max<int64_t>(nc, (int64_t)lst.size()) * 2, &g->acct);
    if (s == BC_OK) s = grow(&g->blk_partials, &g->blk_partials_cap, std::max<int64_t>(tot, 1), &g->acct);
    if (s == BC_OK) s = grow(&g->blk_gsum, &g->blk_gsum_cap, std::max<int64_t>((int64_t)gsum.size(), 4), &g->acct);
    if (s != BC_OK) {
        if (s == BC_ERR_OUT_OF_MEMORY) {  // the general engine needs less: let it run
            *fallback = true;
            return BC_OK;
        }
        return s;
    }
    std::vector<int32_t> chunk_host;
    chunk_host.insert(chunk_host.end(), cb0.begin(), cb0.end());
    chunk_host.insert(chunk_host.end(), cb1.begin(), cb1.end());
    chunk_host.insert(chunk_host.end(), order.begin(), order.end());
    std::vector<int64_t> offs(part_off);
    offs.insert(offs.end(), lst.begin(), lst.end());
    HIP_TRY(hipMemcpyAsync(g->bstart, bs.data(), sizeof(int64_t) * bs.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(g->blo, blo.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(g->bhi, bhi.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(g->blk_chunk, chunk_host.data(), sizeof(int32_t) * chunk_host.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(g->blk_part_off, offs.data(), sizeof(int64_t) * offs.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(g->blk_gsum, gsum.data(), sizeof(int32_t) * gsum.size(), hipMemcpyHostToDevice, st));
    // control blocks and tags
    std::vector<Ctl> hc((size_t)nwg);
    for (Ctl &c : hc) {
        init_ctl(&c);
        c.policy = cfg.policy;
        c.mode = 0;
    }
    HIP_TRY(hipMemcpyAsync(g->blk_ctls, hc.data(), sizeof(Ctl) * hc.size(), hipMemcpyHostToDevice, st));
    {
        const BlockLayout L((size_t)dm.nmax, dm.lq_cap, (size_t)dm.max_levels, dm.gcap, dm.hq_entries, dm.hq_levels,
                            dm.part_cap, dm.ovf_cap);
        dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (int64_t)dm.nmax * 4 / 256 + 1)),
                  (unsigned)std::min(nwg, 65535));
        block_clear_tags<<<grid, 256, 0, st>>>(g->blk_scratch, g->blk_stride, L.fw0, L.fw1 - L.fw0 + (size_t)dm.nmax * sizeof(Tagged), nwg);
    }
    fill_u64<<<1, 64, 0, st>>>((unsigned long long *)g->blk_next, 1, 0ull);
    HIP_TRY(hipGetLastError());
    BlockArgs ra = dm;
    std::memset(&ra.a, 0, sizeof(ra.a));
    GraphArgs ga;
    ga.n = g->n;
    ga.nnz_lo = (int32_t)g->nnz;
    ga.row_ptr = g->row_ptr;
    ga.col = g->col;
    ga.directed = g->directed ? 1 : 0;
    ga.in_row_ptr = g->directed ? g->in_row_ptr : g->row_ptr;
    ga.in_col = g->directed ? g->in_col : g->col;
    ga.nonisolated = g->nonisolated;
    ga.hv_vtx = g->hv_vtx;
    ga.hv_seg = g->hv_seg;
    ga.n_heavy = g->n_heavy;
    ra.a.g = ga;
    ra.a.p = policy_args(g, o);
    ra.a.srcs = g->srcs;
    ra.a.batch_start = g->bstart;
    ra.a.batch_lo = g->blo;
    ra.a.batch_hi = g->bhi;
    ra.a.sigma_limit = o.sigma_limit > 0 ? (unsigned long long)o.sigma_limit : ~0ull;
    ra.scratch = g->blk_scratch;
    ra.stride = g->blk_stride;
    ra.ctls = g->blk_ctls;
    ra.c_b0 = g->blk_chunk;
    ra.c_b1 = g->blk_chunk + nc;
    ra.order = g->blk_chunk + 2 * nc;
    ra.c_part = g->blk_part_off;
    ra.n_chunks = (int32_t)nc;
    ra.next = g->blk_next;
    ra.partials = g->blk_partials;
    ra.max_steps = 3 * ((int64_t)dm.max_levels + 2) + 16;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
    block_run<0><<<(unsigned)nwg, kBlock, 0, st>>>(ra);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(e1, st));
    HIP_TRY(hipMemcpyAsync(hc.data(), g->blk_ctls, sizeof(Ctl) * hc.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const int used = nwg;
    for (int w = 0; w < used; ++w)
        if (hc[w].err) {
            *fallback = true;
            return BC_OK;
        }
    // scores: partials of every graph, chunk by chunk
    if (!gsum.empty()) {
        const int32_t ng = (int32_t)(gsum.size() / 4);
        dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(256, (int64_t)dm.nmax / 256 + 1)),
                  (unsigned)std::min(ng, 65535));
        block_sum<<<grid, 256, 0, st>>>(g->bc, g->blk_partials, g->blk_gsum, ng, g->blk_part_off + nc);
        HIP_TRY(hipGetLastError());
    }
    const double bytes0 = algo_bytes(g->stats);
    for (int w = 0; w < used; ++w) {
        accumulate_stats(&g->stats, hc[w], g->clock_khz);
        if (hc[w].n_ovf) {
            std::vector<int64_t> tmp(hc[w].n_ovf);
            const BlockLayout L((size_t)dm.nmax, dm.lq_cap, (size_t)dm.max_levels, dm.gcap, dm.hq_entries,
                                dm.hq_levels, dm.part_cap, dm.ovf_cap);
            HIP_TRY(hipMemcpy(tmp.data(), g->blk_scratch + (size_t)w * g->blk_stride + L.ovf,
                              sizeof(int64_t) * tmp.size(), hipMemcpyDeviceToHost));
            ovf_positions->insert(ovf_positions->end(), tmp.begin(), tmp.end());
        }
    }
    std::sort(ovf_positions->begin(), ovf_positions->end());
    g->stats.launches += 1;
    g->stats.mode_launches[0] += 1;
    g->stats.mode_ms[0] += ms;
    g->stats.mode_algo_bytes[0] += algo_bytes(g->stats) - bytes0;
    g->stats.block_workgroups = used;
    g->stats.block_chunks = nc;
    HIP_TRY(hipStreamSynchronize(st));
    return BC_OK;
}

// --------------------------------------------------------- weighted engine
// Graphs with arc weights: one persistent launch of weighted_run per pass,
// every workgroup computing whole sources (chunks of consecutive positions)
// on a private copy of the per-vertex state; a chunk's scores go to a
// partial vector, added in chunk order by sum_partials.  First a 64-bit pass
// over every source, then an FP64 pass over the sources whose path counts
// overflowed.

// dst[v] += sum over chunks t (in order) of partials[t * n + v]
__global__ void sum_partials(double *dst, const double *partials, int64_t n, int64_t n_chunks) {
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
        double t = dst[v];
        for (int64_t c = 0; c < n_chunks; ++c) t += partials[c * n + v];
        dst[v] = t;
    }
}

// Sources one workgroup runs together on a weighted graph: the run option,
// else kWL; one when the lane batches' round records (n * kWL entries,
// 32-bit offsets) would not fit.
static int weighted_lanes(const bc_graph *g, const bc_run_options &o) {
    if (o.weighted_lanes == 1 || (int64_t)g->n * kWL > (int64_t)INT32_MAX) return 1;
    return kWL;
}

static bc_status ensure_weighted(bc_graph *g, int lanes) {
    if (g->w_wg > 0 && g->w_lanes == lanes) return BC_OK;
    if (g->w_scratch) {  // the other engine's state
        (void)hipFree(g->w_scratch);
        g->acct.bytes -= std::min(g->acct.bytes, (size_t)g->w_wg * g->w_stride);
        g->w_scratch = nullptr;
        g->w_wg = 0;
    }
    const size_t n = (size_t)std::max<int32_t>(g->n, 1);
    g->w_stride = lanes == 1 ? WeightedLayout(n).bytes : WBLayout(n).bytes;
    int dev = 0, cus = 0, per_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    if (lanes == 1)
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)weighted_run<0>, kBlock, 0));
    else
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)wbatch_run<0>, kWBatchBlock, 0));
    // as many workgroups as the CUs hold (each works through its sources
    // alone, so resident workgroups are what hides memory latency), within
    // the memory budget
    int64_t want = (int64_t)std::max(1, cus) * std::max(1, std::min(per_cu, 8));
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    size_t budget = std::min<size_t>(free_b / 2, (size_t)64 << 30);
    if (g->acct.limit) budget = std::min(budget, g->acct.limit > g->acct.bytes ? g->acct.limit - g->acct.bytes : 0);
    want = std::min<int64_t>(want, (int64_t)(budget / g->w_stride));
    if (want < 1) return fail(BC_ERR_OUT_OF_MEMORY, "the weighted engine's per-workgroup state does not fit");
    HIP_TRY(dalloc(&g->w_scratch, (size_t)want * g->w_stride, &g->acct));
    if (!g->w_ctr) HIP_TRY(dalloc(&g->w_ctr, 16, &g->acct));
    g->w_wg = (int)want;
    g->w_lanes = lanes;
    return BC_OK;
}

// One pass over the run positions `pos` (sources h_srcs[pos[i]]) with the
// given path-count mode; overflowed positions (mode 0) are returned.
static bc_status weighted_pass(bc_graph *g, int mode, const bc_run_options &o, const int32_t *h_srcs,
                               const std::vector<int64_t> &pos, int64_t dump_pos_run, DumpBufs *dump, hipStream_t st,
                               std::vector<int64_t> *ovf, bool *dumped) {
    ovf->clear();
    if (pos.empty()) return BC_OK;
    const int lanes = weighted_lanes(g, o);
    bc_status s = ensure_weighted(g, lanes);
    if (s != BC_OK) return s;
    const int64_t ns = (int64_t)pos.size(), n = std::max<int32_t>(g->n, 1);
    // chunks of consecutive positions, whole batches of `lanes` sources: up
    // to two per workgroup, and at most 8 GiB of partial scores
    const int64_t nbatch = (ns + lanes - 1) / lanes;
    int64_t nc = std::min<int64_t>(nbatch, 2 * (int64_t)g->w_wg);
    nc = std::max<int64_t>(1, std::min<int64_t>(nc, ((int64_t)8 << 30) / (8 * n)));
    const int nwg = (int)std::min<int64_t>(g->w_wg, nc);
    std::vector<int32_t> ch(3 * (size_t)nc), list((size_t)ns);
    for (int64_t t = 0; t < nc; ++t) {
        ch[t] = (int32_t)std::min<int64_t>(ns, lanes * (nbatch * t / nc));
        ch[nc + t] = (int32_t)std::min<int64_t>(ns, lanes * (nbatch * (t + 1) / nc));
        ch[2 * nc + t] = (int32_t)t;
    }
    int64_t pdump = -1;
    for (int64_t i = 0; i < ns; ++i) {
        list[i] = h_srcs[pos[i]];
        if (pos[i] == dump_pos_run) pdump = i;
    }
    s = grow(&g->srcs, &g->srcs_cap, ns, &g->acct);
    if (s == BC_OK) s = grow(&g->w_chunk, &g->w_chunk_cap, 3 * nc, &g->acct);
    if (s == BC_OK) s = grow(&g->w_pos, &g->w_pos_cap, ns, &g->acct);
    if (s == BC_OK) s = grow(&g->ovf, &g->ovf_cap, ns, &g->acct);
    if (s == BC_OK) s = grow(&g->w_partials, &g->w_partials_cap, nc * n, &g->acct);
    if (s != BC_OK) return s;
    HIP_TRY(hipMemcpyAsync(g->srcs, list.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(g->w_chunk, ch.data(), sizeof(int32_t) * ch.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(g->w_pos, pos.data(), sizeof(int64_t) * ns, hipMemcpyHostToDevice, st));
    fill_u64<<<1, 64, 0, st>>>(g->w_ctr, 16, 0ull);
    HIP_TRY(hipGetLastError());
    WeightedArgs a;
    std::memset(&a, 0, sizeof(a));
    a.g.n = g->n;
    a.g.nnz_lo = (int32_t)g->nnz;
    a.g.row_ptr = g->row_ptr;
    a.g.col = g->col;
    a.g.directed = g->directed ? 1 : 0;
    a.g.in_row_ptr = g->directed ? g->in_row_ptr : g->row_ptr;
    a.g.in_col = g->directed ? g->in_col : g->col;
    a.wt = g->wt;
    a.in_wt = g->in_wt;
    a.srcs = g->srcs;
    a.pos = g->w_pos;
    a.c_s0 = g->w_chunk;
    a.c_s1 = g->w_chunk + nc;
    a.order = g->w_chunk + 2 * nc;
    a.n_chunks = (int32_t)nc;
    a.next = (uint32_t *)&g->w_ctr[0];
    a.ovf_count = (uint32_t *)&g->w_ctr[1];
    a.err = (int32_t *)&g->w_ctr[2];
    a.st = &g->w_ctr[4];
    a.partials = g->w_partials;
    a.scratch = g->w_scratch;
    a.stride = g->w_stride;
    a.ovf_list = g->ovf;
    a.ovf_cap = (uint32_t)std::min<int64_t>(g->ovf_cap, UINT32_MAX);
    a.sigma_limit = o.sigma_limit > 0 ? (unsigned long long)o.sigma_limit : ~0ull;
    a.dump_pos = (dump && pdump >= 0) ? pdump : -1;
    if (dump) {
        a.dump_d = dump->d64;
        a.dump_sig = dump->sig;
        a.dump_delta = dump->delta;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, st));
    if (lanes == 1) {
        if (mode) weighted_run<1><<<nwg, kBlock, 0, st>>>(a);
        else weighted_run<0><<<nwg, kBlock, 0, st>>>(a);
    } else {
        if (mode) wbatch_run<1><<<nwg, kWBatchBlock, 0, st>>>(a);
        else wbatch_run<0><<<nwg, kWBatchBlock, 0, st>>>(a);
    }
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(e1, st));
    sum_partials<<<grid_for(n, 256, 4096), 256, 0, st>>>(g->bc, g->w_partials, n, nc);
    HIP_TRY(hipGetLastError());
    unsigned long long ctr[16];
    HIP_TRY(hipMemcpyAsync(ctr, g->w_ctr, sizeof(ctr), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const int32_t err = (int32_t)(uint32_t)ctr[2];
    if (err & ERR_SIGMA_RANGE) return fail(BC_ERR_SIGMA_RANGE, "FP64 path counts left the double range");
    if (err) return fail(BC_ERR_DEVICE, "weighted engine capacity error");
    const uint32_t no = (uint32_t)ctr[1];
    if (no) {
        ovf->resize(no);
        HIP_TRY(hipMemcpy(ovf->data(), g->ovf, sizeof(int64_t) * no, hipMemcpyDeviceToHost));
        std::sort(ovf->begin(), ovf->end());
    }
    if (pdump >= 0 && dump) *dumped = std::find(ovf->begin(), ovf->end(), dump_pos_run) == ovf->end();
    g->stats.launches += 1;
    g->stats.mode_launches[mode] += 1;
    g->stats.mode_ms[mode] += ms;
    g->stats.forward_levels += (int64_t)ctr[4];
    g->stats.arcs_scanned += (int64_t)ctr[5];
    g->stats.max_levels = std::max<int64_t>(g->stats.max_levels, 0);
    g->stats.steps += (int64_t)ctr[6];
    g->stats.reached_pairs += (int64_t)ctr[7];
    if (lanes == 1) {
        g->stats.lane_arcs += (int64_t)ctr[8];
        g->stats.mode_algo_bytes[mode] += algo_bytes_weighted(16.0 * (double)ctr[5], (double)ctr[8], (double)ctr[7]);
    } else {
        g->stats.lane_arcs += (int64_t)ctr[8];
        g->stats.phase_lane_arcs[1] += (int64_t)ctr[9];
        g->stats.phase_lane_arcs[2] += (int64_t)ctr[10];
        for (int i = 0; i < 3; ++i) g->stats.phase_ms[1 + i] += (double)ctr[11 + i] / g->clock_khz;
        g->stats.phase_ms[4] = std::max(g->stats.phase_ms[4], (double)ctr[14] / g->clock_khz);
        g->stats.mode_algo_bytes[mode] +=
            algo_bytes_wbatch((double)(ctr[5] + ctr[8]), (double)(ctr[9] + ctr[10]), (double)ctr[7]);
    }
    return BC_OK;
}

static bc_status run_weighted(bc_graph *g, const int32_t *src, int64_t ns, const bc_run_options &o, hipStream_t st,
                              int64_t dump_index, DumpBufs *db, int *dump_mode) {
    std::vector<int64_t> all((size_t)ns), ovf, none;
    for (int64_t i = 0; i < ns; ++i) all[i] = i;
    bool dumped = false;
    const bool force = (o.flags & BC_RUN_FORCE_F64) != 0;
    bc_status s = weighted_pass(g, force ? 1 : 0, o, src, all, dump_index, db, st, &ovf, &dumped);
    if (s != BC_OK) return s;
    *dump_mode = force ? 1 : 0;
    if (force) {
        g->stats.f64_sources = ns;
        return BC_OK;
    }
    if (!ovf.empty()) {
        bool dumped2 = false;
        s = weighted_pass(g, 1, o, src, ovf, dump_index, db, st, &none, &dumped2);
        if (s != BC_OK) return s;
        if (dumped2) *dump_mode = 1;
    }
    g->stats.f64_sources = (int64_t)ovf.size();
    return BC_OK;
}

static bc_status run_impl(bc_graph *g, const int32_t *sources, int64_t n_sources, const bc_run_options *opt,
                          void *stream, int64_t dump_index, bc_detail *detail);

static void free_parts(bc_graph *g) {
    for (SubPart &pt : g->parts) {
        if (pt.h) bc_destroy(pt.h);
        if (pt.to_parent) (void)hipFree(pt.to_parent);
        if (pt.stream) (void)hipStreamDestroy(pt.stream);
    }
    g->parts.clear();
}

// Replicas of a single graph: the run option, else 8 while one batch's steps
// are small (up to 2^19 vertices), 4 above, where fewer, larger state
// machines measured faster (R-MAT 18: 8 replicas +3 % over 4; R-MAT 22:
// -3 %; the damaged 1024^2 grid, whose levels are many and thin: 8 replicas
// 5.83 GTEPS against 5.42 for 4 and 5.41 for 16, which the autotuner finds).
// BC_REPLICAS overrides both (1 .. 16).
constexpr int kMaxReplicas = 16;
static int n_replicas(const bc_graph *g, const bc_run_options &o) {
    static const int env = [] {
        const char *e = std::getenv("BC_REPLICAS");
        return e ? std::min(kMaxReplicas, std::max(1, std::atoi(e))) : 0;
    }();
    if (env) return env;
    if (o.replicas > 0) return std::min(kMaxReplicas, o.replicas);
    return g->n <= (1 << 19) ? 8 : 4;
}

static bool use_parts(const bc_graph *g, const bc_run_options &o, int64_t ns) {
    if ((o.flags & BC_RUN_ONE_QUEUE) || o.batch == 1 || std::getenv("BC_ONE_QUEUE")) return false;
    if (g->parts_refused) return false;
    if (o.batch == 0 && ns < 2) return false;  // the per-source engine would be chosen
    if (g->n_graphs >= 4) return true;
    const int K = o.batch >= 8 ? o.batch : 64;
    return n_replicas(g, o) >= 2 && ns >= 2 * (int64_t)K;
}

// Single graph: parts are full copies of the graph (own per-vertex state);
// batches of K sources are dealt to them in turn, and the parts' score
// vectors are added in part order.  Deterministic for a given K, but the
// additions are grouped differently from one state machine.
// Under a device-memory cap, concurrent parts are created only when the
// state they would allocate fits beside what the handle holds; otherwise the
// handle runs on its own level state machine (same results to rounding).
static bool parts_fit(bc_graph *g, size_t need) {
    if (!g->acct.limit) return true;
    const size_t have = g->acct.bytes;
    if (have + need <= g->acct.limit) return true;
    g->parts_refused = true;
    return false;
}

// Per-run buffers of a handle running ns sources: source list, overflow
// list, batch bounds.
static size_t run_buffer_bytes(int64_t ns) { return (size_t)(ns + 16) * 12 + (size_t)(ns + 17) * 16; }

static bc_status ensure_replicas(bc_graph *g, int R) {
    if (!g->parts.empty() && (int)g->parts.size() == R) return BC_OK;
    if (!g->parts.empty()) {  // another count was asked for: make them again
        (void)hipDeviceSynchronize();
        free_parts(g);
        g->replicas = false;
    }
    {
        // a replica holds the graph (created with the parent's internal
        // numbering) and its own batched engine state
        const BatchedSizes z = batched_sizes(g->n, g->cost_units, g->n_heavy, g->heavy_segs);
        if (!parts_fit(g, (size_t)R * (g->create_bytes + z.bytes + run_buffer_bytes(g->n))))
            return fail(BC_ERR_OUT_OF_MEMORY, "concurrent replicas do not fit under max_device_bytes");
    }
    int cus = 0, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    std::vector<uint32_t> cu_mask((size_t)std::max(1, (cus + 31) / 32), 0xffffffffu);
    std::vector<float> w;
    if (g->has_mlp) {
        w.resize(kMlpParams);
        HIP_TRY(hipMemcpy(w.data(), g->mlp, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    }
    std::vector<SubPart> parts(R);
    for (int r = 0; r < R; ++r) {
        SubPart &pt = parts[r];
        bc_status s = bc_graph_create(g->n, g->nnz, g->row_ptr, g->col,
                                      BC_INPUT_DEVICE | BC_SKIP_SYMMETRY_CHECK | BC_KEEP_ORDER |
                                          (g->directed ? BC_DIRECTED : 0u),
                                      &pt.h);
        if (s == BC_OK && !w.empty()) s = bc_load_policy(pt.h, w.data(), kMlpParams);
        if (s == BC_OK && hipExtStreamCreateWithCUMask(&pt.stream, (uint32_t)cu_mask.size(), cu_mask.data()) != hipSuccess)
            pt.stream = nullptr;
        if (s == BC_OK && !pt.stream && hipStreamCreateWithFlags(&pt.stream, hipStreamNonBlocking) != hipSuccess)
            s = fail(BC_ERR_DEVICE, "replica stream");
        if (s != BC_OK) {
            g->parts = std::move(parts);
            free_parts(g);
            return s;
        }
    }
    g->parts = std::move(parts);
    g->replicas = true;
    return BC_OK;
}

static bc_status ensure_parts(bc_graph *g) {
    if (!g->parts.empty()) return BC_OK;
    const int32_t n = g->n;
    std::vector<int32_t> rp((size_t)n + 1), col((size_t)g->nnz);
    HIP_TRY(hipMemcpy(rp.data(), g->row_ptr, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToHost));
    if (g->nnz) HIP_TRY(hipMemcpy(col.data(), g->col, sizeof(int32_t) * (size_t)g->nnz, hipMemcpyDeviceToHost));
    // graphs by decreasing size (vertices x arcs), dealt to the parts in
    // snake order (0 1 2 3 3 2 1 0 ...): every part gets about the same
    // number of graphs (batches) and the same total size
    const int G = g->n_graphs;
    const int P = std::min(n_parts(), G / 2);  // at least two graphs per part
    std::vector<int32_t> order(G);
    std::vector<double> work(G);
    for (int i = 0; i < G; ++i) {
        order[i] = i;
        const int32_t lo = g->voff[i], hi = g->voff[i + 1];
        work[i] = (double)(hi - lo) * (double)(rp[hi] - rp[lo] + (hi - lo));
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
    g->part_of_graph.assign(G, 0);
    for (int r = 0; r < G; ++r) {
        const int k = r % (2 * P);
        g->part_of_graph[order[r]] = k < P ? k : 2 * P - 1 - k;
    }
    if (g->acct.limit) {
        // what the parts would hold: their graphs and batched engine state
        std::vector<int64_t> pn(P, 0), pnnz(P, 0), pcost(P, 0), pheavy(P, 0), psegs(P, 0);
        for (int i = 0; i < G; ++i) {
            const int p = g->part_of_graph[i];
            for (int32_t v = g->voff[i]; v < g->voff[i + 1]; ++v) {
                const int32_t d = rp[v + 1] - rp[v];
                pn[p] += 1;
                pnnz[p] += d;
                pcost[p] += entry_cost(d);
                if (d > kSegBatched) {
                    pheavy[p] += 1;
                    psegs[p] += (d + kSegBatched - 1) / kSegBatched;
                }
            }
        }
        size_t need = 0;
        for (int p = 0; p < P; ++p)
            need += (size_t)(pn[p] + 1) * 24 + (size_t)pnnz[p] * 4 + sizeof(Ctl) + (size_t)kLevelRecs * sizeof(LevelRec) +
                    (size_t)pheavy[p] * 16 + 4096 + batched_sizes(pn[p], pcost[p], pheavy[p], psegs[p]).bytes +
                    run_buffer_bytes(pn[p]);
        if (!parts_fit(g, need)) {
            g->part_of_graph.clear();
            return fail(BC_ERR_OUT_OF_MEMORY, "concurrent sub-unions do not fit under max_device_bytes");
        }
    }
    g->local_base.assign(G, 0);
    std::vector<float> w;
    if (g->has_mlp) {
        w.resize(kMlpParams);
        HIP_TRY(hipMemcpy(w.data(), g->mlp, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    }
    std::vector<SubPart> parts(P);
    // each part needs a hardware queue of its own: ordinary streams share the
    // device's few queues with other streams of the process, a stream with
    // a CU mask gets a dedicated queue (here the mask enables every CU)
    int cus = 0, dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    std::vector<uint32_t> cu_mask((size_t)std::max(1, (cus + 31) / 32), 0xffffffffu);
    for (int p = 0; p < P; ++p) {
        std::vector<int32_t> srp(1, 0), scol, svoff(1, 0), map;
        for (int i = 0; i < G; ++i) {
            if (g->part_of_graph[i] != p) continue;
            const int32_t lo = g->voff[i], hi = g->voff[i + 1];
            const int32_t base = (int32_t)map.size();
            g->local_base[i] = base;
            for (int32_t v = lo; v < hi; ++v) {
                map.push_back(v);
                for (int32_t e = rp[v]; e < rp[v + 1]; ++e) scol.push_back(col[e] - lo + base);
                srp.push_back((int32_t)scol.size());
            }
            svoff.push_back((int32_t)map.size());
        }
        SubPart &pt = parts[p];
        bc_status s = bc_graph_create_multi((int32_t)svoff.size() - 1, svoff.data(), (int32_t)map.size(),
                                            (int64_t)scol.size(), srp.data(), scol.data(),
                                            BC_SKIP_SYMMETRY_CHECK | BC_KEEP_ORDER, &pt.h);
        if (s == BC_OK && !w.empty()) s = bc_load_policy(pt.h, w.data(), kMlpParams);
        if (s == BC_OK && hipMalloc((void **)&pt.to_parent, sizeof(int32_t) * std::max<size_t>(map.size(), 1)) != hipSuccess)
            s = fail(BC_ERR_OUT_OF_MEMORY, "part vertex map");
        if (s == BC_OK && !map.empty() &&
            hipMemcpy(pt.to_parent, map.data(), sizeof(int32_t) * map.size(), hipMemcpyHostToDevice) != hipSuccess)
            s = fail(BC_ERR_DEVICE, "part vertex map copy");
        if (s == BC_OK && std::getenv("BC_PART_PLAIN_STREAMS") == nullptr &&
            hipExtStreamCreateWithCUMask(&pt.stream, (uint32_t)cu_mask.size(), cu_mask.data()) != hipSuccess)
            pt.stream = nullptr;
        if (s == BC_OK && !pt.stream && hipStreamCreateWithFlags(&pt.stream, hipStreamNonBlocking) != hipSuccess)
            s = fail(BC_ERR_DEVICE, "part stream");
        pt.to_parent_host = std::move(map);
        if (s != BC_OK) {
            g->parts = std::move(parts);
            free_parts(g);
            return s;
        }
    }
    g->parts = std::move(parts);
    return BC_OK;
}

static bc_status run_parts(bc_graph *g, const int32_t *sources, int64_t n_sources, const bc_run_options &o,
                           void *stream, int64_t dump_index, bc_detail *detail) {
    bc_status s = g->n_graphs >= 4 ? ensure_parts(g) : ensure_replicas(g, n_replicas(g, o));
    if (s != BC_OK) return s;
    const bool repl = g->replicas;
    const int64_t K = o.batch >= 8 ? o.batch : 64;
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    const int64_t ns = sources ? n_sources : g->n;
    if (ns < 0) return fail(BC_ERR_INVALID_ARG, "n_sources < 0");
    if (detail && (dump_index < 0 || dump_index >= ns)) return fail(BC_ERR_INVALID_ARG, "dump_index out of range");
    const int P = (int)g->parts.size();
    std::vector<std::vector<int32_t>> lists(P);
    int dump_part = -1;
    int64_t dump_local = -1;
    for (int64_t i = 0; i < ns; ++i) {
        const int32_t v = sources ? sources[i] : (int32_t)i;
        if (v < 0 || v >= g->n) return fail(BC_ERR_INVALID_ARG, "source id outside [0, n)");
        int p;
        int32_t local;
        if (repl) {
            p = (int)((i / K) % P);
            local = v;
        } else {
            const int gi = (int)(std::upper_bound(g->voff.begin(), g->voff.end(), v) - g->voff.begin()) - 1;
            p = g->part_of_graph[gi];
            local = g->local_base[gi] + (v - g->voff[gi]);
        }
        if (detail && i == dump_index) {
            dump_part = p;
            dump_local = (int64_t)lists[p].size();
        }
        lists[p].push_back(local);
    }
    const bool acc = (o.flags & BC_RUN_ACCUMULATE) != 0;
    if (!acc && g->n > 0 && !repl) {
        fill_u64<<<grid_for(g->n, 256, 4096), 256, 0, st>>>((unsigned long long *)g->bc, g->n, 0ull);
        HIP_TRY(hipGetLastError());
    }
    for (SubPart &pt : g->parts) {
        if (acc && pt.h->n > 0 && !repl) {  // the parts continue from the parent's scores
            gather_f64<<<grid_for(pt.h->n, 256, 4096), 256, 0, st>>>(pt.h->bc, g->bc, pt.to_parent, pt.h->n);
            HIP_TRY(hipGetLastError());
        }
    }
    hipEvent_t ev0;
    HIP_TRY(hipEventCreateWithFlags(&ev0, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ev0, st));
    for (SubPart &pt : g->parts) HIP_TRY(hipStreamWaitEvent(pt.stream, ev0, 0));
    (void)hipEventDestroy(ev0);
    // sub-detail buffers for the part that holds the dumped source
    const size_t dn = dump_part >= 0 ? (size_t)std::max<int32_t>(g->parts[dump_part].h->n, 1) : 0;
    std::vector<int32_t> sd(dn), sexp(dn);
    std::vector<uint64_t> su(dn);
    std::vector<double> smant(dn), sdel(dn);
    bc_detail sub_det{};
    sub_det.d = sd.data();
    sub_det.sigma_u64 = su.data();
    sub_det.sigma_mant = smant.data();
    sub_det.sigma_exp = sexp.data();
    sub_det.delta = sdel.data();
    std::vector<bc_status> res(P, BC_OK);
    std::vector<std::string> msg(P);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::vector<std::thread> th;
    for (int p = 0; p < P; ++p) {
        if (lists[p].empty()) continue;
        th.emplace_back([&, p]() {
            (void)hipSetDevice(dev);
            bc_run_options po = o;
            if (!acc || repl) po.flags &= ~BC_RUN_ACCUMULATE;
            po.flags |= BC_RUN_ONE_QUEUE;
            SubPart &pt = g->parts[p];
            if (p == dump_part)
                res[p] = run_impl(pt.h, lists[p].data(), (int64_t)lists[p].size(), &po, pt.stream, dump_local, &sub_det);
            else
                res[p] = run_impl(pt.h, lists[p].data(), (int64_t)lists[p].size(), &po, pt.stream, -1, nullptr);
            if (res[p] != BC_OK) msg[p] = bc_last_error();
        });
    }
    for (std::thread &t : th) t.join();
    for (int p = 0; p < P; ++p)
        if (res[p] != BC_OK) return fail(res[p], msg[p]);
    // scores back to the parent, then the caller's stream waits for every part
    PartScores ps{};
    for (int p = 0; p < P; ++p) {
        SubPart &pt = g->parts[p];
        if (repl) {
            if (!lists[p].empty()) ps.p[ps.n++] = pt.h->bc;
        } else if (!(lists[p].empty() && !acc) && pt.h->n > 0) {
            scatter_f64<<<grid_for(pt.h->n, 256, 4096), 256, 0, pt.stream>>>(g->bc, pt.h->bc, pt.to_parent, pt.h->n);
            HIP_TRY(hipGetLastError());
        }
        hipEvent_t ev;
        HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIP_TRY(hipEventRecord(ev, pt.stream));
        HIP_TRY(hipStreamWaitEvent(st, ev, 0));
        (void)hipEventDestroy(ev);
    }
    if (repl && g->n > 0 && ps.n > 0) {
        sum_parts_f64<<<grid_for(g->n, 256, 4096), 256, 0, st>>>(g->bc, ps, acc ? 1 : 0, g->n);
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(st));
    // statistics: sums over the parts (device times overlap), wall time of the whole
    std::memset(&g->stats, 0, sizeof(g->stats));
    bc_stats &S = g->stats;
    for (int p = 0; p < P; ++p) {
        if (lists[p].empty()) continue;
        const bc_stats &x = g->parts[p].h->stats;
        S.n_sources += x.n_sources;
        S.n_batches += x.n_batches;
        S.batch = x.batch;
        S.policy = x.policy;
        S.grid_blocks = x.grid_blocks;
        S.chunk_steps = x.chunk_steps;
        S.steps += x.steps;
        S.launches += x.launches;
        S.forward_levels += x.forward_levels;
        S.max_levels = std::max(S.max_levels, x.max_levels);
        for (int k = 0; k < 3; ++k) S.variant_levels[k] += x.variant_levels[k];
        S.f64_sources += x.f64_sources;
        S.arcs_scanned += x.arcs_scanned;
        S.lane_arcs += x.lane_arcs;
        S.queue_entries += x.queue_entries;
        S.algo_bytes += x.algo_bytes;
        S.algo_bytes_arcs += x.algo_bytes_arcs;
        S.reached_pairs += x.reached_pairs;
        for (int k = 0; k < 10; ++k) {
            S.phase_ms[k] += x.phase_ms[k];
            S.phase_arcs[k] += x.phase_arcs[k];
            S.phase_lane_arcs[k] += x.phase_lane_arcs[k];
            S.phase_pairs[k] += x.phase_pairs[k];
        }
        for (int k = 0; k < 3; ++k) S.variant_ms[k] += x.variant_ms[k];
        for (int k = 0; k < 2; ++k) {
            S.mode_launches[k] += x.mode_launches[k];
            S.mode_ms[k] += x.mode_ms[k];
            S.mode_algo_bytes[k] += x.mode_algo_bytes[k];
        }
    }
    S.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (detail) {
        // the dumped source's graph lies in one part; every other vertex is unreached
        const SubPart &pt = g->parts[dump_part];
        if (repl) {
            for (int32_t v = 0; v < g->n; ++v) {
                if (detail->d) detail->d[v] = sd[v];
                if (detail->sigma_u64) detail->sigma_u64[v] = su[v];
                if (detail->sigma_mant) detail->sigma_mant[v] = smant[v];
                if (detail->sigma_exp) detail->sigma_exp[v] = sexp[v];
                if (detail->delta) detail->delta[v] = sdel[v];
            }
        }
        for (int32_t v = 0; v < g->n && !repl; ++v) {
            if (detail->d) detail->d[v] = -1;
            if (detail->sigma_u64) detail->sigma_u64[v] = 0;
            if (detail->sigma_mant) detail->sigma_mant[v] = 0.0;
            if (detail->sigma_exp) detail->sigma_exp[v] = 0;
            if (detail->delta) detail->delta[v] = 0.0;
        }
        for (size_t i = 0; i < pt.to_parent_host.size() && !repl; ++i) {
            const int32_t v = pt.to_parent_host[i];
            if (detail->d) detail->d[v] = sd[i];
            if (detail->sigma_u64) detail->sigma_u64[v] = su[i];
            if (detail->sigma_mant) detail->sigma_mant[v] = smant[i];
            if (detail->sigma_exp) detail->sigma_exp[v] = sexp[i];
            if (detail->delta) detail->delta[v] = sdel[i];
        }
        detail->mode = sub_det.mode;
        detail->n_levels = sub_det.n_levels;
    }
    return BC_OK;
}

static bc_status run_impl(bc_graph *g, const int32_t *sources, int64_t n_sources, const bc_run_options *opt,
                          void *stream, int64_t dump_index, bc_detail *detail) {
    if (!g) return fail(BC_ERR_INVALID_ARG, "NULL handle");
    bc_run_options o;
    bc_run_options_init(&o);
    if (opt) o = *opt;
    if (o.flags & BC_RUN_TUNED) {
        if (!g->has_tuned) return fail(BC_ERR_INVALID_ARG, "BC_RUN_TUNED before bc_autotune");
        // fields the caller left automatic (zero) come from the tuner
        if (o.batch == 0) o.batch = g->tuned.batch;
        if (o.policy == BC_POLICY_AUTO) o.policy = g->tuned.policy;
        if (o.grid_blocks == 0) o.grid_blocks = g->tuned.grid_blocks;
        if (o.chunk_steps == 0) o.chunk_steps = g->tuned.chunk_steps;
        if (o.wpv_degree <= 0.0f) o.wpv_degree = g->tuned.wpv_degree;
        if (o.lanes_per_entry == 0.0f) o.lanes_per_entry = g->tuned.lanes_per_entry;
        if (o.replicas == 0) o.replicas = g->tuned.replicas;
        o.flags &= ~BC_RUN_TUNED;
    }
    if (o.weighted_lanes != 0 && o.weighted_lanes != 1 && o.weighted_lanes != kWL)
        return fail(BC_ERR_INVALID_ARG, "weighted_lanes must be 0, 1 or 16");
    const bool blk = use_block(g, o, sources ? n_sources : g->n, detail != nullptr);
    if (!blk && !g->weighted && use_parts(g, o, sources ? n_sources : g->n)) {
        g->last_parts = true;
        const bc_status ps = run_parts(g, sources, n_sources, o, stream, dump_index, detail);
        if (!(ps == BC_ERR_OUT_OF_MEMORY && g->parts_refused)) return ps;
        // the parts were refused under the cap before anything ran: one state machine
    }
    g->last_parts = false;
    std::vector<int32_t> all;
    const int32_t *src = sources;
    int64_t ns = n_sources;
    if (!sources) {
        all.resize(g->n);
        for (int32_t i = 0; i < g->n; ++i) all[i] = i;
        src = all.data();
        ns = g->n;
    } else if (n_sources < 0) {
        return fail(BC_ERR_INVALID_ARG, "n_sources < 0");
    }
    for (int64_t i = 0; i < ns; ++i)
        if (src[i] < 0 || src[i] >= g->n) return fail(BC_ERR_INVALID_ARG, "source id outside [0, n)");
    if (detail && (dump_index < 0 || dump_index >= ns)) return fail(BC_ERR_INVALID_ARG, "dump_index out of range");
    RunCfg cfg;
    bc_status s = resolve_cfg(g, o, ns, &cfg);
    if (s != BC_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    const auto t0 = std::chrono::steady_clock::now();
    std::memset(&g->stats, 0, sizeof(g->stats));
    fill_u64<<<grid_for((int64_t)kLevelRecs * 8, 256, 4096), 256, 0, st>>>((unsigned long long *)g->lvl,
                                                                           (int64_t)kLevelRecs * 8, 0ull);
    HIP_TRY(hipGetLastError());
    g->stats.n_sources = ns;
    g->stats.batch = cfg.engine;
    g->stats.policy = cfg.policy;
    g->stats.grid_blocks = cfg.grid;
    g->stats.chunk_steps = cfg.use_graphs ? cfg.chunk : 0;
    if (!(o.flags & BC_RUN_ACCUMULATE) && g->n > 0) {
        fill_u64<<<grid_for(g->n, 256, 4096), 256, 0, st>>>((unsigned long long *)g->bc, g->n, 0ull);
        HIP_TRY(hipGetLastError());
    }
    DumpBufs db;
    if (detail) {
        const size_t n = (size_t)std::max<int32_t>(g->n, 1);
        if (over_cap(&g->acct, n * 24 + 8))
            return fail(BC_ERR_OUT_OF_MEMORY, "detail buffers are over the handle's max_device_bytes");
        HIP_TRY(hipMalloc((void **)&db.d, n * sizeof(int32_t)));
        HIP_TRY(hipMalloc((void **)&db.sig, n * sizeof(unsigned long long)));
        HIP_TRY(hipMalloc((void **)&db.delta, n * sizeof(double)));
        HIP_TRY(hipMalloc((void **)&db.shift, ((size_t)g->n + 2) * sizeof(int32_t)));
        if (g->weighted) HIP_TRY(hipMalloc((void **)&db.d64, n * sizeof(int64_t)));
        fill_i32<<<grid_for(n, 256, 4096), 256, 0, st>>>(db.d, n, -1);
        fill_u64<<<grid_for(n, 256, 4096), 256, 0, st>>>(db.sig, n, 0ull);
        fill_u64<<<grid_for(n, 256, 4096), 256, 0, st>>>((unsigned long long *)db.delta, n, 0ull);
        fill_i32<<<grid_for(n + 2, 256, 4096), 256, 0, st>>>(db.shift, n + 2, 0);
        HIP_TRY(hipGetLastError());
    }
    auto free_dump = [&]() {
        if (db.d64) (void)hipFree(db.d64);
        if (db.d) (void)hipFree(db.d);
        if (db.sig) (void)hipFree(db.sig);
        if (db.delta) (void)hipFree(db.delta);
        if (db.shift) (void)hipFree(db.shift);
    };
    if (g->weighted) {
        int wmode = 0;
        s = run_weighted(g, src, ns, o, st, detail ? dump_index : -1, detail ? &db : nullptr, &wmode);
        if (s != BC_OK) { free_dump(); return s; }
        if (detail) {
            const size_t n = (size_t)g->n;
            std::vector<int64_t> hd(n);
            std::vector<unsigned long long> hs(n);
            std::vector<double> hdel(n);
            HIP_TRY(hipMemcpyAsync(hd.data(), db.d64, n * sizeof(int64_t), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(hs.data(), db.sig, n * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipMemcpyAsync(hdel.data(), db.delta, n * sizeof(double), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipStreamSynchronize(st));
            free_dump();
            std::vector<int64_t> dvals;
            for (size_t v = 0; v < n; ++v) {
                if (detail->d) detail->d[v] = hd[v] > INT32_MAX ? INT32_MAX : (int32_t)hd[v];
                if (detail->d64) detail->d64[v] = hd[v];
                if (hd[v] >= 0) dvals.push_back(hd[v]);
                double sv;
                if (wmode) std::memcpy(&sv, &hs[v], sizeof(sv));
                else sv = (double)hs[v];
                if (detail->sigma_u64) detail->sigma_u64[v] = wmode ? 0 : hs[v];
                if (detail->sigma_mant) detail->sigma_mant[v] = hd[v] >= 0 ? sv : 0.0;
                if (detail->sigma_exp) detail->sigma_exp[v] = 0;
                if (detail->delta) detail->delta[v] = hdel[v];
            }
            std::sort(dvals.begin(), dvals.end());
            detail->mode = wmode;
            detail->n_levels = (int32_t)(std::unique(dvals.begin(), dvals.end()) - dvals.begin());
        }
        g->stats.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        g->stats.algo_bytes = g->stats.mode_algo_bytes[0] + g->stats.mode_algo_bytes[1];
        g->stats.algo_bytes_arcs = g->stats.algo_bytes - 64.0 * (double)g->stats.reached_pairs;
        return BC_OK;
    }
    int dump_done = 0;
    int dump_mode = 0;
    Ctl last{};
    const bool force_f64 = (o.flags & BC_RUN_FORCE_F64) != 0;
    // One pass over the sources at the given absolute positions; returns (in
    // *back) the positions the pass handed back: overflowed lanes of a 64-bit
    // pass, or lanes of a checked FP64 pass whose counts may fit in 64 bits.
    auto pass = [&](int mode, bool check, const std::vector<int64_t> &pos, std::vector<int64_t> *back) -> bc_status {
        back->clear();
        if (pos.empty()) return BC_OK;
        std::vector<int32_t> list(pos.size());
        int64_t pdump = -1;
        for (size_t i = 0; i < pos.size(); ++i) {
            list[i] = src[pos[i]];
            if (detail && pos[i] == dump_index) pdump = (int64_t)i;
        }
        RunCfg c = cfg;
        c.mode = mode;
        c.f64_check = check;
        std::vector<int64_t> rel;
        int dd = 0;
        bc_status r = run_pass(g, c, o, list.data(), (int64_t)list.size(), pdump, detail ? &db : nullptr, st, &rel,
                               &dd, &last);
        if (r != BC_OK) return r;
        if (pdump >= 0 && dd) {
            dump_done = dd;
            dump_mode = mode;
        }
        for (int64_t q : rel) back->push_back(pos[q]);
        return BC_OK;
    };
    std::vector<int64_t> all_pos((size_t)ns);
    for (int64_t i = 0; i < ns; ++i) all_pos[i] = i;
    std::vector<int64_t> f64_pos;  // sources that end in FP64 mode (sorted)
    bool block_done = false;
    if (!force_f64 && blk) {
        // the block engine: every source in one 64-bit pass; the sources
        // that overflowed run again in FP64 on the general engine
        std::vector<int64_t> ovf;
        bool fb = false;
        s = run_block(g, cfg, o, src, ns, st, &ovf, &fb);
        if (s != BC_OK) { free_dump(); return s; }
        if (!fb) {
            std::vector<int64_t> none;
            s = pass(1, false, ovf, &none);
            if (s != BC_OK) { free_dump(); return s; }
            g->stats.f64_sources = (int64_t)ovf.size();
            block_done = true;
        }
    }
    if (force_f64) {
        std::vector<int64_t> none;
        s = pass(1, false, all_pos, &none);
        if (s != BC_OK) { free_dump(); return s; }
        g->stats.f64_sources = ns;
    } else if (!block_done) {
        // 64-bit counts first.  When most of the first batch overflows, the
        // graph's counts exceed 64 bits as a rule: the rest runs in FP64
        // straight away (checked), and only the lanes whose counts stay below
        // 2^65 go back to a 64-bit pass, which decides their mode exactly.
        const int64_t probe = cfg.engine == 1 ? ns : std::min<int64_t>(ns, cfg.lanes);
        std::vector<int64_t> head(all_pos.begin(), all_pos.begin() + probe), rest(all_pos.begin() + probe, all_pos.end());
        std::vector<int64_t> ovf_a, ovf_b, kept_f64;
        s = pass(0, false, head, &ovf_a);
        if (s != BC_OK) { free_dump(); return s; }
        if (!rest.empty() && 2 * (int64_t)ovf_a.size() >= probe) {
            std::vector<int64_t> small;
            s = pass(1, true, rest, &small);
            if (s != BC_OK) { free_dump(); return s; }
            std::vector<bool> is_small((size_t)ns, false);
            for (int64_t q : small) is_small[q] = true;
            for (int64_t q : rest)
                if (!is_small[q]) kept_f64.push_back(q);
            s = pass(0, false, small, &ovf_b);
        } else {
            s = pass(0, false, rest, &ovf_b);
        }
        if (s != BC_OK) { free_dump(); return s; }
        std::vector<int64_t> redo(ovf_a);
        redo.insert(redo.end(), ovf_b.begin(), ovf_b.end());
        std::sort(redo.begin(), redo.end());
        if (!redo.empty()) {
            // the overflowed sources, in list order, with FP64 path counts
            std::vector<int64_t> none;
            s = pass(1, false, redo, &none);
            if (s != BC_OK) { free_dump(); return s; }
        }
        g->stats.f64_sources = (int64_t)(redo.size() + kept_f64.size());
    }
    if (detail) {
        if (!dump_done) { free_dump(); return fail(BC_ERR_DEVICE, "detail dump did not complete"); }
        const size_t n = (size_t)g->n;
        std::vector<int32_t> hd(n), hsh(n + 2);
        std::vector<unsigned long long> hs(n);
        std::vector<double> hdel(n);
        HIP_TRY(hipMemcpyAsync(hd.data(), db.d, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hs.data(), db.sig, n * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hdel.data(), db.delta, n * sizeof(double), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipMemcpyAsync(hsh.data(), db.shift, (n + 2) * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        free_dump();
        // sigma(v) = raw * 2^(shift_0 + ... + shift_{d-1}) in mode 1
        std::vector<int64_t> E(n + 2, 0);
        int32_t L = 0;
        for (size_t v = 0; v < n; ++v) L = std::max(L, hd[v] + 1);
        for (int32_t l = 1; l <= L && l < (int32_t)(n + 2); ++l) E[l] = E[l - 1] + hsh[l - 1];
        for (size_t v = 0; v < n; ++v) {
            if (detail->d) detail->d[v] = hd[v];
            const bool reached = hd[v] >= 0;
            if (dump_mode == 0) {
                if (detail->sigma_u64) detail->sigma_u64[v] = hs[v];
                if (detail->sigma_mant) detail->sigma_mant[v] = (double)hs[v];
                if (detail->sigma_exp) detail->sigma_exp[v] = 0;
            } else {
                double raw;
                std::memcpy(&raw, &hs[v], sizeof(raw));
                if (detail->sigma_u64) detail->sigma_u64[v] = 0;
                if (detail->sigma_mant) detail->sigma_mant[v] = reached ? raw : 0.0;
                if (detail->sigma_exp) detail->sigma_exp[v] = reached ? (int32_t)E[hd[v]] : 0;
            }
            if (detail->delta) detail->delta[v] = hdel[v];
        }
        detail->mode = dump_mode;
        detail->n_levels = L;
    }
    g->stats.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    g->stats.algo_bytes = algo_bytes(g->stats);
    g->stats.algo_bytes_arcs = algo_bytes_arcs(g->stats);
    return BC_OK;
}

// Caller ids -> internal ids (hub-first renumbering), and the sources in
// the order the run takes them (by source_ranks; stable, so duplicates keep
// the caller's order).  A NULL list means every vertex.  *pos_of (if given)
// receives, for each run position, the caller's position.  Out-of-range ids
// are passed through unchanged (and rejected by the run).
static const int32_t *to_internal(const bc_graph *g, const int32_t *sources, int64_t *n_sources,
                                  std::vector<int32_t> *buf, std::vector<int64_t> *pos_of = nullptr) {
    if (pos_of) pos_of->clear();
    if (!g || (g->perm.empty() && g->srank.empty())) return sources;
    const bool map = !g->perm.empty();
    if (!sources) {
        *n_sources = g->n;
        buf->resize((size_t)g->n);
        for (int32_t v = 0; v < g->n; ++v) (*buf)[v] = map ? g->inv[v] : v;
    } else {
        // an empty list stays as given (an empty vector's data() may be NULL,
        // which would mean "every vertex")
        if (*n_sources <= 0) return sources;
        buf->resize((size_t)*n_sources);
        for (int64_t i = 0; i < *n_sources; ++i) {
            const int32_t v = sources[i];
            if (v < 0 || v >= g->n) return sources;
            (*buf)[i] = map ? g->inv[v] : v;
        }
    }
    if (!g->srank.empty()) {
        const int64_t ns = *n_sources;
        std::vector<int64_t> order((size_t)ns);
        for (int64_t i = 0; i < ns; ++i) order[i] = i;
        const std::vector<int32_t> &b = *buf;
        std::stable_sort(order.begin(), order.end(),
                         [&](int64_t x, int64_t y) { return g->srank[b[x]] < g->srank[b[y]]; });
        std::vector<int32_t> sorted((size_t)ns);
        for (int64_t i = 0; i < ns; ++i) sorted[i] = b[order[i]];
        buf->swap(sorted);
        if (pos_of) pos_of->swap(order);
    }
    return buf->data();
}

extern "C" bc_status bc_run(bc_graph *g, const int32_t *sources, int64_t n_sources, const bc_run_options *opt,
                            void *stream) {
    std::vector<int32_t> buf;
    const int32_t *src = to_internal(g, sources, &n_sources, &buf);
    return run_impl(g, src, n_sources, opt, stream, -1, nullptr);
}

extern "C" bc_status bc_run_detail(bc_graph *g, const int32_t *sources, int64_t n_sources,
                                   const bc_run_options *opt, int64_t dump_index, bc_detail *out, void *stream) {
    if (!out) return fail(BC_ERR_INVALID_ARG, "out is NULL");
    std::vector<int32_t> buf;
    std::vector<int64_t> pos_of;
    const int32_t *src = to_internal(g, sources, &n_sources, &buf, &pos_of);
    if (!pos_of.empty() && dump_index >= 0 && dump_index < n_sources) {
        for (int64_t i = 0; i < n_sources; ++i)
            if (pos_of[i] == dump_index) {
                dump_index = i;
                break;
            }
    }
    bc_status s = run_impl(g, src, n_sources, opt, stream, dump_index, out);
    if (s != BC_OK || !g || g->perm.empty()) return s;
    // per-vertex outputs back to the caller's ids
    const size_t n = (size_t)g->n;
    auto unperm = [&](auto *a) {
        if (!a) return;
        using T = std::remove_reference_t<decltype(a[0])>;
        std::vector<T> t(a, a + n);
        for (size_t v = 0; v < n; ++v) a[v] = t[g->inv[v]];
    };
    unperm(out->d);
    unperm(out->sigma_u64);
    unperm(out->sigma_mant);
    unperm(out->sigma_exp);
    unperm(out->delta);
    return BC_OK;
}

extern "C" bc_status bc_collect_level_times(bc_graph *g, const int32_t *sources, int64_t n_sources,
                                            const bc_run_options *opt, float *X, float *Y, int64_t cap,
                                            int64_t *count, void *stream) {
    if (!g || !X || !Y || !count || cap < 1 || !sources || n_sources < 1)
        return fail(BC_ERR_INVALID_ARG, "NULL argument, empty source list or cap < 1");
    for (int64_t i = 0; i < n_sources; ++i)
        if (sources[i] < 0 || sources[i] >= g->n) return fail(BC_ERR_INVALID_ARG, "source id outside [0, n)");
    std::vector<int32_t> sbuf;
    sources = to_internal(g, sources, &n_sources, &sbuf);
    bc_run_options o;
    bc_run_options_init(&o);
    if (opt) o = *opt;
    o.batch = 64;
    RunCfg cfg;
    bc_status s = resolve_cfg(g, o, n_sources, &cfg);
    if (s != BC_OK) return s;
    cfg.mode = (o.flags & BC_RUN_FORCE_F64) ? 1 : 0;
    hipStream_t st = (hipStream_t)stream;
    s = ensure_batched(g);
    if (s != BC_OK) return s;
    CollectBufs cb;
    cb.cap = (uint32_t)std::min<int64_t>(cap, UINT32_MAX);
    const size_t nf = ((size_t)g->b_max_levels + 2) * kMlpIn;
    if (over_cap(&g->acct, ((size_t)cb.cap * (kMlpIn + kMlpOut) + nf) * sizeof(float)))
        return fail(BC_ERR_OUT_OF_MEMORY, "collection buffers are over the handle's max_device_bytes");
    HIP_TRY(hipMalloc((void **)&cb.X, (size_t)cb.cap * kMlpIn * sizeof(float)));
    hipError_t e = hipMalloc((void **)&cb.Y, (size_t)cb.cap * kMlpOut * sizeof(float));
    if (e == hipSuccess) e = hipMalloc((void **)&cb.F, nf * sizeof(float));
    if (e != hipSuccess) {
        (void)hipFree(cb.X);
        if (cb.Y) (void)hipFree(cb.Y);
        return fail(BC_ERR_OUT_OF_MEMORY, "collection buffers");
    }
    std::memset(&g->stats, 0, sizeof(g->stats));
    g->last_parts = false;
    fill_u64<<<grid_for((int64_t)kLevelRecs * 8, 256, 4096), 256, 0, st>>>((unsigned long long *)g->lvl,
                                                                           (int64_t)kLevelRecs * 8, 0ull);
    if (!(o.flags & BC_RUN_ACCUMULATE) && g->n > 0) {
        fill_u64<<<grid_for(g->n, 256, 4096), 256, 0, st>>>((unsigned long long *)g->bc, g->n, 0ull);
    }
    Ctl last{};
    std::vector<int64_t> ovf;
    RunCfg c0 = cfg;
    c0.use_graphs = false;  // the machine inserts undo steps; keep launches simple
    s = run_pass(g, c0, o, sources, n_sources, -1, nullptr, st, &ovf, nullptr, &last, &cb);
    int64_t n_samples = std::min<int64_t>((int64_t)last.n_samples, (int64_t)cb.cap);
    if (s == BC_OK && !ovf.empty()) {
        // sources whose path counts overflowed 64 bits run again with FP64
        // path counts, so that the scores stay complete; their levels are
        // timed too (deep levels are only ever reached this way)
        std::vector<int32_t> redo(ovf.size());
        for (size_t i = 0; i < ovf.size(); ++i) redo[i] = sources[ovf[i]];
        RunCfg c1 = c0;
        c1.mode = 1;
        CollectBufs cb1;
        cb1.X = cb.X + (size_t)n_samples * kMlpIn;
        cb1.Y = cb.Y + (size_t)n_samples * kMlpOut;
        cb1.F = cb.F;
        cb1.cap = cb.cap - (uint32_t)n_samples;
        s = run_pass(g, c1, o, redo.data(), (int64_t)redo.size(), -1, nullptr, st, nullptr, nullptr, &last,
                     cb1.cap ? &cb1 : nullptr);
        if (cb1.cap) n_samples += std::min<int64_t>((int64_t)last.n_samples, (int64_t)cb1.cap);
        g->stats.f64_sources = (int64_t)redo.size();
    }
    if (s == BC_OK) {
        const int64_t k = n_samples;
        std::vector<float> hy((size_t)k * kMlpOut);
        hipError_t e1 = hipMemcpy(X, cb.X, (size_t)k * kMlpIn * sizeof(float), hipMemcpyDeviceToHost);
        hipError_t e2 = hipMemcpy(hy.data(), cb.Y, (size_t)k * kMlpOut * sizeof(float), hipMemcpyDeviceToHost);
        if (e1 != hipSuccess || e2 != hipSuccess) {
            s = fail(BC_ERR_DEVICE, "copying collected samples");
        } else {
            // device ticks -> log2 microseconds; NaN where not timed
            for (size_t i = 0; i < hy.size(); ++i) {
                const double us = (double)hy[i] / g->clock_khz * 1000.0;
                Y[i] = hy[i] < 0.0f ? std::nanf("") : (float)std::log2(std::max(us, 0.01));
            }
            *count = k;
        }
    }
    (void)hipFree(cb.X);
    (void)hipFree(cb.Y);
    (void)hipFree(cb.F);
    return s;
}

extern "C" bc_status bc_scores(const bc_graph *g, double *out, int64_t len, uint32_t flags, void *stream) {
    if (!g || !out) return fail(BC_ERR_INVALID_ARG, "NULL argument");
    if (len < g->n) return fail(BC_ERR_INVALID_ARG, "len < n");
    if (g->n == 0) return BC_OK;
    hipStream_t st = (hipStream_t)stream;
    const double *src = g->bc;
    if (!g->perm.empty()) {  // back to the caller's ids: out[v] = bc[inv[v]]
        gather_f64<<<grid_for(g->n, 256, 4096), 256, 0, st>>>(g->bc_out, g->bc, g->inv_dev, g->n);
        HIP_TRY(hipGetLastError());
        src = g->bc_out;
    }
    HIP_TRY(hipMemcpyAsync(out, src, sizeof(double) * g->n,
                           (flags & BC_OUT_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return BC_OK;
}

extern "C" bc_status bc_run_stats(const bc_graph *g, bc_stats *out) {
    if (!g || !out) return fail(BC_ERR_INVALID_ARG, "NULL argument");
    *out = g->stats;
    return BC_OK;
}

// Level records of the last run, summed over the concurrent parts it ran on.
static bc_status level_records(const bc_graph *g, std::vector<LevelRec> *acc) {
    if (g->last_parts) {
        for (const SubPart &pt : g->parts) {
            bc_status s = level_records(pt.h, acc);
            if (s != BC_OK) return s;
        }
        return BC_OK;
    }
    std::vector<LevelRec> r((size_t)kLevelRecs);
    HIP_TRY(hipMemcpy(r.data(), g->lvl, sizeof(LevelRec) * kLevelRecs, hipMemcpyDeviceToHost));
    for (int i = 0; i < kLevelRecs; ++i) {
        LevelRec &a = (*acc)[(size_t)i];
        a.visits += r[i].visits;
        a.entries += r[i].entries;
        a.arcs += r[i].arcs;
        for (int k = 0; k < 3; ++k) a.var[k] += r[i].var[k];
        a.ticks += r[i].ticks;
    }
    return BC_OK;
}

extern "C" bc_status bc_run_level_stats(const bc_graph *g, bc_level_stats *out, int64_t cap, int64_t *n_levels) {
    if (!g || !n_levels || cap < 0 || (cap > 0 && !out)) return fail(BC_ERR_INVALID_ARG, "NULL argument or cap < 0");
    std::vector<LevelRec> acc((size_t)kLevelRecs);
    std::memset(acc.data(), 0, sizeof(LevelRec) * acc.size());
    bc_status s = level_records(g, &acc);
    if (s != BC_OK) return s;
    int64_t used = 0;
    for (int i = 0; i < kLevelRecs; ++i)
        if (acc[i].visits || acc[i].entries) used = i + 1;
    *n_levels = used;
    for (int64_t i = 0; i < std::min(cap, used); ++i) {
        bc_level_stats &o = out[i];
        o.visits = (int64_t)acc[i].visits;
        o.entries = (int64_t)acc[i].entries;
        o.arcs = (int64_t)acc[i].arcs;
        for (int k = 0; k < 3; ++k) o.variant[k] = (int64_t)acc[i].var[k];
        o.ms = (double)acc[i].ticks / g->clock_khz;
    }
    return BC_OK;
}

extern "C" bc_status bc_load_policy(bc_graph *g, const float *weights, int64_t len) {
    if (!g) return fail(BC_ERR_INVALID_ARG, "NULL handle");
    if (weights) {
        if (len != kMlpParams) return fail(BC_ERR_INVALID_ARG, "weights length must be BC_MLP_PARAMS");
        for (int64_t i = 0; i < len; ++i)
            if (!std::isfinite(weights[i])) return fail(BC_ERR_INVALID_ARG, "non-finite policy weight");
    }
    for (SubPart &pt : g->parts) {
        bc_status s = bc_load_policy(pt.h, weights, len);
        if (s != BC_OK) return s;
    }
    if (!weights) {
        g->has_mlp = false;  // unload
        return BC_OK;
    }
    HIP_TRY(hipMemcpy(g->mlp, weights, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    g->has_mlp = true;
    free_graphs(g);  // captured args carry has_mlp
    return BC_OK;
}

// ---------------------------------------------------------------- tune cache
// Autotuner results of this process, keyed by device (architecture and CU
// count), graph fingerprint, sample and resolved base options; saved to and
// loaded from a JSON file by bc_tune_cache_save / bc_tune_cache_load.
namespace {
struct TuneEntry {
    std::string device;
    uint64_t graph = 0, sample = 0, base = 0;
    bc_run_options best{};
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

void tune_put(const TuneEntry &e) {  // caller holds g_tune_mu
    for (TuneEntry &x : g_tune)
        if (x.device == e.device && x.graph == e.graph && x.sample == e.sample && x.base == e.base) {
            x.best = e.best;
            return;
        }
    g_tune.push_back(e);
}

std::string hex64(uint64_t v) {
    char b[17];
    std::snprintf(b, sizeof(b), "%016llx", (unsigned long long)v);
    return b;
}

// A small reader for the cache file: one object with an "entries" array of
// flat objects whose values are strings or numbers.
struct JsonIn {
    const char *p, *end;
    std::string err;
    void ws() {
        while (p < end && (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r')) ++p;
    }
    bool eat(char c) {
        ws();
        if (p < end && *p == c) {
            ++p;
            return true;
        }
        return false;
    }
    bool str(std::string *out) {
        ws();
        if (p >= end || *p != '"') return false;
        ++p;
        out->clear();
        while (p < end && *p != '"') {
            if (*p == '\\' && p + 1 < end) ++p;
            out->push_back(*p++);
        }
        if (p >= end) return false;
        ++p;
        return true;
    }
    bool num(double *out) {
        ws();
        char *q = nullptr;
        const double v = std::strtod(p, &q);
        if (q == p || q > end) return false;
        p = q;
        *out = v;
        return true;
    }
    // a scalar or a nested value we do not use
    bool skip() {
        ws();
        if (p >= end) return false;
        if (*p == '"') {
            std::string t;
            return str(&t);
        }
        if (*p == '{' || *p == '[') {
            const char open = *p, close = open == '{' ? '}' : ']';
            int depth = 0;
            bool in_str = false;
            for (; p < end; ++p) {
                if (in_str) {
                    if (*p == '\\') ++p;
                    else if (*p == '"') in_str = false;
                } else if (*p == '"') in_str = true;
                else if (*p == open) ++depth;
                else if (*p == close && --depth == 0) {
                    ++p;
                    return true;
                }
            }
            return false;
        }
        while (p < end && *p != ',' && *p != '}' && *p != ']') ++p;
        return true;
    }
};

bool parse_entry(JsonIn &in, TuneEntry *e) {
    bc_run_options_init(&e->best);
    if (!in.eat('{')) return false;
    bool have[4] = {false, false, false, false};
    if (in.eat('}')) return false;
    do {
        std::string key, sv;
        double x = 0.0;
        if (!in.str(&key) || !in.eat(':')) return false;
        if (key == "device" || key == "graph" || key == "sample" || key == "base") {
            if (!in.str(&sv)) return false;
            if (key == "device") {
                e->device = sv;
                have[0] = true;
            } else {
                char *q = nullptr;
                const uint64_t v = std::strtoull(sv.c_str(), &q, 16);
                if (sv.empty() || *q) return false;
                (key == "graph" ? e->graph : key == "sample" ? e->sample : e->base) = v;
                have[key == "graph" ? 1 : key == "sample" ? 2 : 3] = true;
            }
        } else if (key == "batch" || key == "policy" || key == "grid_blocks" || key == "chunk_steps" ||
                   key == "wpv_degree" || key == "lanes_per_entry" || key == "policy_margin" || key == "replicas" ||
                   key == "flags") {
            if (!in.num(&x)) return false;
            if (key == "batch") e->best.batch = (int32_t)x;
            else if (key == "policy") e->best.policy = (int32_t)x;
            else if (key == "grid_blocks") e->best.grid_blocks = (int32_t)x;
            else if (key == "chunk_steps") e->best.chunk_steps = (int32_t)x;
            else if (key == "wpv_degree") e->best.wpv_degree = (float)x;
            else if (key == "lanes_per_entry") e->best.lanes_per_entry = (float)x;
            else if (key == "policy_margin") e->best.policy_margin = (float)x;
            else if (key == "replicas") e->best.replicas = (int32_t)x;
            else e->best.flags = (uint32_t)x;
        } else if (!in.skip()) {
            return false;
        }
    } while (in.eat(','));
    if (!in.eat('}')) return false;
    return have[0] && have[1] && have[2] && have[3];
}
}  // namespace

static std::string device_tag() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
    return std::string(prop.gcnArchName) + ":" + std::to_string(prop.multiProcessorCount);
}

extern "C" bc_status bc_tune_cache_save(const char *path) {
    if (!path) return fail(BC_ERR_INVALID_ARG, "path is NULL");
    std::string out = "{\"format\": \"bc-autotune-cache\", \"version\": 1, \"entries\": [";
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (size_t i = 0; i < g_tune.size(); ++i) {
            const TuneEntry &e = g_tune[i];
            char buf[512];
            std::snprintf(buf, sizeof(buf),
                          "%s\n  {\"device\": \"%s\", \"graph\": \"%s\", \"sample\": \"%s\", \"base\": \"%s\", "
                          "\"batch\": %d, \"policy\": %d, \"grid_blocks\": %d, \"chunk_steps\": %d, "
                          "\"wpv_degree\": %.9g, \"lanes_per_entry\": %.9g, \"policy_margin\": %.9g, "
                          "\"replicas\": %d, \"flags\": %u}",
                          i ? "," : "", e.device.c_str(), hex64(e.graph).c_str(), hex64(e.sample).c_str(),
                          hex64(e.base).c_str(), e.best.batch, e.best.policy, e.best.grid_blocks, e.best.chunk_steps,
                          (double)e.best.wpv_degree, (double)e.best.lanes_per_entry,
                          (double)e.best.policy_margin, e.best.replicas, e.best.flags);
            out += buf;
        }
    }
    out += "\n]}\n";
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(BC_ERR_INVALID_ARG, std::string("cannot open ") + path + " for writing");
    const bool ok = std::fwrite(out.data(), 1, out.size(), f) == out.size();
    if (std::fclose(f) != 0 || !ok) return fail(BC_ERR_INVALID_ARG, std::string("cannot write ") + path);
    return BC_OK;
}

extern "C" bc_status bc_tune_cache_load(const char *path) {
    if (!path) return fail(BC_ERR_INVALID_ARG, "path is NULL");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(BC_ERR_INVALID_ARG, std::string("cannot open ") + path);
    std::string text;
    char buf[65536];
    size_t k;
    while ((k = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, k);
    std::fclose(f);
    JsonIn in{text.data(), text.data() + text.size(), ""};
    std::vector<TuneEntry> got;
    bool ok = in.eat('{');
    bool seen = false;
    if (ok && !in.eat('}')) {
        do {
            std::string key;
            if (!in.str(&key) || !in.eat(':')) {
                ok = false;
                break;
            }
            if (key == "entries") {
                seen = true;
                if (!in.eat('[')) {
                    ok = false;
                    break;
                }
                if (!in.eat(']')) {
                    do {
                        TuneEntry e;
                        if (!parse_entry(in, &e)) {
                            ok = false;
                            break;
                        }
                        got.push_back(e);
                    } while (in.eat(','));
                    if (!ok || !in.eat(']')) {
                        ok = false;
                        break;
                    }
                }
            } else if (!in.skip()) {
                ok = false;
                break;
            }
        } while (in.eat(','));
        ok = ok && in.eat('}');
    }
    if (!ok || !seen) return fail(BC_ERR_INVALID_ARG, std::string("not a tune cache file: ") + path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const TuneEntry &e : got) tune_put(e);
    return BC_OK;
}

extern "C" void bc_tune_cache_clear(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

extern "C" int64_t bc_tune_cache_size(void) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return (int64_t)g_tune.size();
}

extern "C" bc_status bc_autotune(bc_graph *g, const int32_t *sample, int64_t n_sample, const bc_run_options *base,
                                 bc_run_options *best, void *stream) {
    if (!g || !best || !sample || n_sample < 1) return fail(BC_ERR_INVALID_ARG, "NULL argument or empty sample");
    Fnv64 hs;
    hs.add(&n_sample, sizeof(n_sample));
    hs.add(sample, sizeof(int32_t) * (size_t)n_sample);
    std::vector<int32_t> sbuf;
    sample = to_internal(g, sample, &n_sample, &sbuf);
    bc_run_options cur;
    bc_run_options_init(&cur);
    if (base) cur = *base;
    const bool fresh = (cur.flags & BC_TUNE_FRESH) != 0;
    cur.flags &= ~(BC_RUN_ACCUMULATE | BC_RUN_TUNED | BC_TUNE_FRESH);
    // resolve the automatic fields so every candidate is explicit
    RunCfg c0;
    bc_status s = resolve_cfg(g, cur, n_sample, &c0);
    if (s != BC_OK) return s;
    if (cur.batch == 0) cur.batch = c0.engine == 1 ? 1 : 64;
    if (cur.policy == BC_POLICY_AUTO) cur.policy = g->has_mlp ? BC_POLICY_MLP : BC_POLICY_HEURISTIC;
    if (cur.grid_blocks == 0) cur.grid_blocks = c0.grid;
    if (cur.chunk_steps == 0) cur.chunk_steps = c0.chunk;
    if (cur.wpv_degree <= 0.0f) cur.wpv_degree = 24.0f;
    if (cur.lanes_per_entry == 0.0f) cur.lanes_per_entry = 4.0f;
    const bool single = g->n_graphs < 4 && !g->weighted;  // replicas apply to single graphs
    if (cur.replicas == 0 && single) cur.replicas = n_replicas(g, cur);
    hipStream_t st = (hipStream_t)stream;
    auto reset_scores = [&]() -> bc_status {
        if (g->n > 0) {
            fill_u64<<<grid_for(g->n, 256, 4096), 256, 0, st>>>((unsigned long long *)g->bc, g->n, 0ull);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipStreamSynchronize(st));
        }
        return BC_OK;
    };
    // the cache: same device, graph, sample and resolved base options
    TuneEntry key;
    key.device = device_tag();
    key.graph = g->fingerprint;
    key.sample = hs.v;
    {
        Fnv64 hb;
        const int64_t f[7] = {cur.flags, cur.batch, cur.policy, cur.grid_blocks, cur.chunk_steps,
                              (int64_t)cur.sigma_limit, cur.replicas};
        const float x[5] = {cur.alpha, cur.beta, cur.wpv_degree, cur.lanes_per_entry, cur.policy_margin};
        hb.add(f, sizeof(f));
        hb.add(x, sizeof(x));
        hb.add(&g->has_mlp, sizeof(g->has_mlp));
        key.base = hb.v;
    }
    if (!fresh) {
        bool hit = false;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            for (const TuneEntry &e : g_tune)
                if (e.device == key.device && e.graph == key.graph && e.sample == key.sample && e.base == key.base) {
                    cur = e.best;
                    hit = true;
                    break;
                }
        }
        if (hit && (cur.policy != BC_POLICY_MLP || g->has_mlp)) {
            g->tuned = cur;
            g->has_tuned = true;
            *best = cur;
            return reset_scores();
        }
        if (hit) return fail(BC_ERR_INVALID_ARG, "cached tuning uses the learned policy; load its weights first");
    }
    // Weighted graphs run on their own engine, which has none of these knobs.
    if (g->weighted) {
        g->tuned = cur;
        g->has_tuned = true;
        *best = cur;
        return reset_scores();
    }
    // a warm-up run (builds the captured graphs), then the best of two timed
    // runs; the per-source engine (K = 1) runs its sources one after another,
    // so it is timed on a prefix of the sample and scaled to the whole
    auto time_one = [&](const bc_run_options &o, double *ms) -> bc_status {
        const int64_t m = o.batch == 1 ? std::min<int64_t>(n_sample, 32) : n_sample;
        bc_status r = run_impl(g, sample, m, &o, st, -1, nullptr);
        if (r != BC_OK) return r;
        *ms = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
            const auto t0 = std::chrono::steady_clock::now();
            r = run_impl(g, sample, m, &o, st, -1, nullptr);
            if (r != BC_OK) return r;
            *ms = std::min(*ms, std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        }
        *ms *= (double)n_sample / (double)m;
        return BC_OK;
    };
    const double kGain = 0.98;  // a candidate must be 2 % faster to replace the current choice
    double best_ms = 0.0;
    s = time_one(cur, &best_ms);
    if (s != BC_OK) return s;
    const int dflt_grid = cur.grid_blocks;
    const bool asked_plain = cur.batch == 1;
    const int dflt_repl = cur.replicas;
    for (int dim = 0; dim < 7; ++dim) {
        std::vector<bc_run_options> cand;
        bc_run_options c = cur;
        if (dim == 0) {
            if (asked_plain) continue;  // the per-source engine was asked for
            for (int k : {64, 32, 16, 8, 1}) { c.batch = k; cand.push_back(c); }
        } else if (dim == 1) {
            if (!g->has_mlp) continue;
            for (int p : {BC_POLICY_HEURISTIC, BC_POLICY_MLP}) { c.policy = p; cand.push_back(c); }
        } else if (dim == 2) {
            for (int d : {1, 2, 4}) { c.grid_blocks = std::max(1, dflt_grid / d); cand.push_back(c); }
        } else if (dim == 3) {
            for (int k : {8, 16, 32}) { c.chunk_steps = k; cand.push_back(c); }
        } else if (dim == 4) {
            for (float w : {12.0f, 24.0f, 48.0f}) { c.wpv_degree = w; cand.push_back(c); }
        } else if (dim == 5) {
            if (cur.batch == 1) continue;
            for (float x : {-1.0f, 2.0f, 4.0f, 12.0f}) { c.lanes_per_entry = x; cand.push_back(c); }
        } else {
            if (cur.batch == 1 || !single) continue;
            for (int r : {dflt_repl / 2, dflt_repl, 2 * dflt_repl}) {
                c.replicas = std::max(1, std::min(kMaxReplicas, r));
                cand.push_back(c);
            }
        }
        for (const bc_run_options &x : cand) {
            if (std::memcmp(&x, &cur, sizeof(x)) == 0) continue;
            double ms = 0.0;
            s = time_one(x, &ms);
            if (s != BC_OK) return s;
            if (ms < kGain * best_ms) {
                best_ms = ms;
                cur = x;
            }
        }
    }
    g->tuned = cur;
    g->has_tuned = true;
    *best = cur;
    key.best = cur;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_put(key);
    }
    return reset_scores();
}
