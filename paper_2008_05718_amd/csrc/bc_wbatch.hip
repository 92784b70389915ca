// bc_wbatch.hip -- Brandes on graphs with positive integer arc weights, kWL
// sources per workgroup.
//
// Same three phases as the one-source-per-workgroup engine (bc_weighted.hip),
// following the paper's forward "BFS traversal or SSSP calculation" and its
// dependency sweep (Section "Background", Eq. 2): label-correcting
// relaxation rounds for the distances, Kahn rounds over the shortest-path
// DAG for the path counts, the same rounds in reverse for the dependencies.
// What changes is the data layout: a workgroup runs a batch of kWL sources
// together, and every per-source value of vertex v sits in the row
// [v * kWL, (v + 1) * kWL) of its slab.  A round's queue holds each vertex
// once with a lane mask (the sources for which it is active), so a vertex's
// arcs are read once per round for all of those sources, and the kWL
// distances of an arc's far end arrive in one 128-byte line instead of one
// line per source.
//
// Thread mapping: a wavefront is kWGrp groups of kWL threads; thread k of a
// group handles source (lane) k.  A wavefront takes 64 queue entries at a
// time; each group walks the arcs of its 16 entries as one packed list, one
// arc per step, in CSR order; entries with more than kWBLight arcs are walked
// by all groups of the wavefront (group g takes arcs g, g + 4, ...).
//
// Relaxation, DAG in-arc counts, release of successors and (uint64) path
// counts are integer atomics, exact in any order.  Sums of doubles (FP64 path
// counts, dependencies) are taken per (entry, source) by one thread in CSR
// order, or for the heavy entries as four group partials added in group
// order, so every result is fixed by the graph and the batch: runs are
// bitwise reproducible.
#include "bc_common.h"
#include "bc_wbatch.h"

namespace bcx {

namespace {

constexpr unsigned long long kWInf = ~0ull;
constexpr int kWGrp = kWave / kWL;  // groups per wavefront
constexpr int kWBBlock = kWBatchBlock;
constexpr int kWBWaves = kWBBlock / kWave;
// (A/B on R-MAT 18 with weights, 4096 sources: 8 arcs per load round 1.88 s
// against 2.04 s for 4 and 2.79 s for 2; light entries up to 32 arcs within
// 2 % of 8 and 16, 64 arcs 1.95 s, 256 arcs 2.17 s)
#ifndef BC_WB_LIGHT
#define BC_WB_LIGHT 32
#endif
#ifndef BC_WB_UNROLL
#define BC_WB_UNROLL 8
#endif
// The dependency pass loads c of an arc's far end together with its
// distance, before the DAG test (most of those loads are discarded, but the
// pass waits one memory round trip less per load round): R-MAT 18 with
// weights 1.59 s against 1.62 s, the pass itself 104 s against 108 s
// summed over the batches.
#ifndef BC_WB_SPEC
#define BC_WB_SPEC 1
#endif
constexpr int kWBLight = BC_WB_LIGHT;  // entries with more arcs are walked by a whole wavefront
constexpr int kWU = BC_WB_UNROLL;      // arcs whose loads a group issues together (divides kWL)
static_assert(kWL <= 32 && kWave % kWL == 0, "lane masks are 32-bit words; groups tile a wavefront");
static_assert(kWL % kWU == 0, "a load round must not reach into the next group's lanes");

// Values that other threads of the workgroup change (by atomics, or by stores
// from other wavefronts) are read and written at device scope, in the L2,
// never through a stale line of the compute unit's L1.
__device__ __forceinline__ unsigned long long wb_ld(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t wb_ld32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double wb_ldf(const double *p) {
    return as_f64(wb_ld((const unsigned long long *)p));
}
__device__ __forceinline__ void wb_stf(double *p, double x) {
    __hip_atomic_store((unsigned long long *)p, as_u64(x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier after which every store and atomic issued before it has completed.
__device__ __forceinline__ void wb_sync() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// One arc of a walk: valid flag, wavefront lane of the entry it belongs to,
// far end and weight.
struct WArc {
    bool ok;
    int o;
    int x;
    int w;
};

// Walks the arcs of the light entries of a wavefront batch.  The entry of
// lane j has arcs [e0, e0 + dg) (dg = 0: none).  The 16 entries of a group
// are packed into one arc list walked in order; on every step each group
// hands kWU consecutive arcs of its list to block(r), which runs on every
// thread of the wavefront.  The wavefront must be converged.
template <class Block>
__device__ __forceinline__ void walk_light(const int32_t *__restrict__ col, const int32_t *__restrict__ wt, int e0,
                                           int dg, Block block) {
    const int lane = lane_id(), k = lane & (kWL - 1), gb = lane - k;
    int incl = dg;
#pragma unroll
    for (int o = 1; o < kWL; o <<= 1) {
        const int y = __shfl_up(incl, o, kWL);
        if (k >= o) incl += y;
    }
    const int excl = incl - dg;
    const int tot = __shfl(incl, gb + kWL - 1);
    int tmax = max(tot, __shfl_xor(tot, 16));
    tmax = max(tmax, __shfl_xor(tmax, 32));
    for (int base = 0; base < tmax; base += kWL) {
        const int ai = base + k;
        const bool ok = ai < tot;
        int o = 0;  // first entry of the group whose inclusive prefix exceeds ai
#pragma unroll
        for (int step = kWL / 2; step > 0; step >>= 1) {
            if (__shfl(incl, gb + o + step - 1) <= ai) o += step;
        }
        const int eo = __shfl(e0, gb + o), xo = __shfl(excl, gb + o);
        const int e = eo + (ai - xo);
        const int x = ok ? col[e] : 0;
        const int w = ok ? wt[e] : 0;
        for (int j = 0; j < kWL && base + j < tmax; j += kWU) {
            WArc r[kWU];
#pragma unroll
            for (int q = 0; q < kWU; ++q) {
                const int sl = gb + j + q;
                r[q].ok = base + j + q < tot;
                r[q].o = gb + __shfl(o, sl);
                r[q].x = __shfl(x, sl);
                r[q].w = __shfl(w, sl);
            }
            block(r);
        }
    }
}

// Walks the arcs [e0, e1) of the heavy entry of lane oj with the whole
// wavefront: group g takes arcs e0 + g, e0 + g + kWGrp, ... in order.
template <class Block>
__device__ __forceinline__ void walk_heavy(const int32_t *__restrict__ col, const int32_t *__restrict__ wt, int oj,
                                           int e0, int e1, Block block) {
    const int lane = lane_id(), g = lane / kWL;
    for (int base = e0; base < e1; base += kWave) {
        const int e = base + lane;
        const int x = e < e1 ? col[e] : 0;
        const int w = e < e1 ? wt[e] : 0;
        for (int j = 0; j < kWave / kWGrp && base + j * kWGrp < e1; j += kWU) {
            WArc r[kWU];
#pragma unroll
            for (int q = 0; q < kWU; ++q) {
                const int sl = (j + q) * kWGrp + g;
                r[q].ok = base + sl < e1;
                r[q].o = oj;
                r[q].x = __shfl(x, sl);
                r[q].w = __shfl(w, sl);
            }
            block(r);
        }
    }
}

// Sum over the groups of a wavefront of thread k's value, groups in order.
__device__ __forceinline__ double group_ordered_sum(double v) {
    const int k = lane_id() & (kWL - 1);
    double s = 0.0;
#pragma unroll
    for (int g = 0; g < kWGrp; ++g) s += __shfl(v, g * kWL + k);
    return s;
}

}  // namespace

template <int MODE>
__global__ __launch_bounds__(kWBBlock) void wbatch_run(WeightedArgs a) {
    __shared__ int s_chunk;
    __shared__ uint32_t s_n0, s_n1, s_nr, s_ovf;
    __shared__ int s_off;  // round records written so far (workgroup-uniform)
    __shared__ int s_src[kWL];
    __shared__ int s_ev[kWBWaves][kWave];       // entries of each wavefront's batch
    __shared__ uint32_t s_em[kWBWaves][kWave];  // their lane masks
    // the entries' own values per lane (distance; path count in the release
    // pass), loaded once per entry instead of once per arc
    __shared__ unsigned long long s_ov[kWBWaves][kWave][kWL];
    __shared__ unsigned long long s_os[kWBWaves][kWave][kWL];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int k = lane & (kWL - 1), gb = lane - k;
    const uint32_t kbit = 1u << k;
    const int n = a.g.n;
    const int32_t *__restrict__ rp = a.g.row_ptr;
    const int32_t *__restrict__ col = a.g.col;
    const int32_t *__restrict__ irp = a.g.in_row_ptr;
    const int32_t *__restrict__ icol = a.g.in_col;
    const int32_t *__restrict__ wt = a.wt;
    const int32_t *__restrict__ iwt = a.in_wt;
    char *base = a.scratch + (size_t)blockIdx.x * a.stride;
    const WBLayout L((size_t)n);
    unsigned long long *dist = (unsigned long long *)(base + L.dist);
    unsigned long long *sig = (unsigned long long *)(base + L.sig);
    double *chat = (double *)(base + L.chat);
    double *dep = (double *)(base + L.dep);
    int32_t *cnt = (int32_t *)(base + L.cnt);
    uint32_t *fm0 = (uint32_t *)(base + L.fm0);
    uint32_t *fm1 = (uint32_t *)(base + L.fm1);
    uint32_t *rm = (uint32_t *)(base + L.rm);
    int32_t *reached = (int32_t *)(base + L.reached);
    int32_t *qa = (int32_t *)(base + L.qa);
    int32_t *qb = (int32_t *)(base + L.qb);
    int32_t *lvl = (int32_t *)(base + L.lvl);
    uint32_t *lvlm = (uint32_t *)(base + L.lvlm);
    int32_t *lvl_off = (int32_t *)(base + L.lvl_off);
    unsigned long long st_rounds = 0, st_arcs = 0, st_dag = 0, st_pairs = 0, st_darcs = 0, st_rl = 0, st_dl = 0;
    // device clock per phase (thread 0): relaxation, DAG rounds, dependencies; longest batch
    unsigned long long tk_a = 0, tk_b = 0, tk_c = 0, tk_max = 0, tk0 = 0, tk1 = 0;
    const size_t nk = (size_t)n * kWL;
    for (size_t i = tid; i < nk; i += kWBBlock) {
        dist[i] = kWInf;
        sig[i] = 0ull;
        cnt[i] = 0;
    }
    for (int i = tid; i < n; i += kWBBlock) {
        fm0[i] = 0u;
        fm1[i] = 0u;
        rm[i] = 0u;
    }
    auto row = [](int v) { return (size_t)v * kWL; };
    // after s_ev / s_em of the wavefront's batch are written: thread k of a
    // group loads lane k of its 16 entries' rows (and of the path counts)
    auto own_values = [&](bool with_sig) {
#pragma unroll
        for (int j = 0; j < kWL; ++j) {
            const int e = gb + j;
            if (s_em[wid][e] & kbit) {
                const size_t at = row(s_ev[wid][e]) + k;
                s_ov[wid][e][k] = wb_ld(&dist[at]);
                if (with_sig) s_os[wid][e][k] = wb_ld(&sig[at]);
            }
        }
        __builtin_amdgcn_wave_barrier();
    };
    // appends every vertex whose mask word is non-zero to list (count in
    // *cnt, LDS), one wavefront-wide reservation per 64 vertices
    auto gather = [&](const uint32_t *mask, int32_t *list, uint32_t *cnt) {
        for (int b0 = wid * kWave; b0 < n; b0 += kWBBlock) {
            const int v = b0 + lane;
            const bool on = v < n && wb_ld32(&mask[v]) != 0u;
            const unsigned long long bal = __ballot(on);
            if (!bal) continue;
            uint32_t at = 0;
            if (lane == 0) at = atomicAdd(cnt, (uint32_t)__popcll(bal));
            at = __shfl(at, 0);
            if (on) list[at + __popcll(bal & ((1ull << lane) - 1ull))] = v;
        }
    };
    for (;;) {
        wb_sync();
        if (tid == 0) {
            const uint32_t q = atomicAdd(a.next, 1u);
            s_chunk = (q < (uint32_t)a.n_chunks && ld_agent(a.err) == 0) ? a.order[q] : -1;
        }
        __syncthreads();
        const int t = s_chunk;
        if (t < 0) break;
        double *part = a.partials + (size_t)t * (size_t)n;
        for (int i = tid; i < n; i += kWBBlock) part[i] = 0.0;
        for (int p0 = a.c_s0[t]; p0 < a.c_s1[t]; p0 += kWL) {
            const int nb = min(kWL, a.c_s1[t] - p0);
            // ---------------- A: distances, relaxation rounds over lane masks
            wb_sync();
            if (tid == 0) tk0 = tk1 = wall_clock64();
            if (tid < kWL) s_src[tid] = tid < nb ? a.srcs[p0 + tid] : -1;
            if (tid == 0) {
                s_n0 = 0;
                s_n1 = 0;
                s_nr = 0;
                s_ovf = 0;
            }
            wb_sync();
            if (tid < nb) {
                const int s = s_src[tid];
                __hip_atomic_store(&dist[row(s) + tid], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (atomicOr(&fm0[s], 1u << tid) == 0u) qa[atomicAdd(&s_n0, 1u)] = s;
                (void)atomicOr(&rm[s], 1u << tid);
            }
            wb_sync();
            uint32_t *fc = fm0, *fn = fm1;
            int32_t *cur = qa, *nxt = qb;
            uint32_t round = 0;
            auto relax = [&](const WArc *r) {
                unsigned long long dv[kWU], dx[kWU];
                bool act[kWU];
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    act[q] = r[q].ok && (s_em[wid][r[q].o] & kbit);
                    dv[q] = act[q] ? s_ov[wid][r[q].o][k] : 0ull;
                    dx[q] = act[q] ? wb_ld(&dist[row(r[q].x) + k]) : 0ull;
                }
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    // No atomic here waits for its result: a lane whose tentative
                    // distance was above the candidate is marked for the next
                    // round even if another arc lowered it further meanwhile
                    // (one relaxation more, never a wrong distance), and the
                    // next round's queue is gathered from the marks afterwards.
                    bool dropped = false, first = false;
                    if (act[q]) {
                        ++st_rl;
                        const unsigned long long nd = dv[q] + (unsigned long long)r[q].w;
                        if (nd < dx[q]) {
                            (void)atomicMin(&dist[row(r[q].x) + k], nd);
                            dropped = true;
                            first = dx[q] == kWInf;
                        }
                    }
                    const uint32_t gd = (uint32_t)(__ballot(dropped) >> gb) & ((1u << kWL) - 1u);
                    const uint32_t gf = (uint32_t)(__ballot(first) >> gb) & ((1u << kWL) - 1u);
                    if (k == 0) {
                        if (gd) (void)atomicOr(&fn[r[q].x], gd);
                        if (gf) (void)atomicOr(&rm[r[q].x], gf);
                    }
                }
            };
            for (;;) {
                const uint32_t nc = s_n0;
                if (nc == 0) break;
                if ((int64_t)(++round) > (int64_t)n + 2) {  // cannot happen with positive weights
                    if (tid == 0) atomicOr(a.err, ERR_LEVEL_CAP);
                    break;
                }
                for (uint32_t cb = (uint32_t)wid * kWave; cb < nc; cb += kWBBlock) {
                    const uint32_t i = cb + lane;
                    const int v = i < nc ? cur[i] : -1;
                    const uint32_t m = v >= 0 ? wb_ld32(&fc[v]) : 0u;
                    const int e0 = v >= 0 ? rp[v] : 0;
                    const int dg = v >= 0 ? rp[v + 1] - e0 : 0;
                    const bool heavy = dg > kWBLight;
                    s_ev[wid][lane] = v;
                    s_em[wid][lane] = m;
                    __builtin_amdgcn_wave_barrier();
                    own_values(false);
                    st_arcs += (unsigned)dg;
                    walk_light(col, wt, e0, heavy ? 0 : dg, relax);
                    for (unsigned long long hm = __ballot(heavy); hm; hm &= hm - 1) {
                        const int j = __ffsll(hm) - 1;
                        const int h0 = __builtin_amdgcn_readlane(e0, j), hd = __builtin_amdgcn_readlane(dg, j);
                        walk_heavy(col, wt, j, h0, h0 + hd, relax);
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                wb_sync();
                for (uint32_t i = tid; i < nc; i += kWBBlock) fc[cur[i]] = 0u;
                gather(fn, nxt, &s_n1);
                wb_sync();
                if (tid == 0) {
                    s_n0 = s_n1;
                    s_n1 = 0;
                }
                wb_sync();
                uint32_t *tm = fc;
                fc = fn;
                fn = tm;
                int32_t *tq = cur;
                cur = nxt;
                nxt = tq;
                ++st_rounds;
            }
            gather(rm, reached, &s_nr);
            wb_sync();
            const uint32_t nr = s_nr;
            if (tid == 0) {
                const unsigned long long now = wall_clock64();
                tk_a += now - tk1;
                tk1 = now;
            }
            // ---------------- B: DAG in-arc counts (per reached vertex and lane)
            auto count = [&](const WArc *r) {
                unsigned long long dv[kWU], du[kWU];
                bool act[kWU];
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    act[q] = r[q].ok && (s_em[wid][r[q].o] & kbit);
                    dv[q] = act[q] ? s_ov[wid][r[q].o][k] : 0ull;
                    du[q] = act[q] ? wb_ld(&dist[row(r[q].x) + k]) : 0ull;
                }
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    if (!act[q]) continue;
                    ++st_dl;
                    if (du[q] != kWInf && du[q] + (unsigned long long)r[q].w == dv[q])
                        atomicAdd(&cnt[row(s_ev[wid][r[q].o]) + k], 1);
                }
            };
            for (uint32_t cb = (uint32_t)wid * kWave; cb < nr; cb += kWBBlock) {
                const uint32_t i = cb + lane;
                const int v = i < nr ? reached[i] : -1;
                const uint32_t m = v >= 0 ? wb_ld32(&rm[v]) : 0u;
                const int e0 = v >= 0 ? irp[v] : 0;
                const int dg = v >= 0 ? irp[v + 1] - e0 : 0;
                const bool heavy = dg > kWBLight;
                s_ev[wid][lane] = v;
                s_em[wid][lane] = m;
                __builtin_amdgcn_wave_barrier();
                own_values(false);
                st_darcs += (unsigned)dg;
                st_pairs += (unsigned)__popc(m);
                walk_light(icol, iwt, e0, heavy ? 0 : dg, count);
                for (unsigned long long hm = __ballot(heavy); hm; hm &= hm - 1) {
                    const int j = __ffsll(hm) - 1;
                    const int h0 = __builtin_amdgcn_readlane(e0, j), hd = __builtin_amdgcn_readlane(dg, j);
                    walk_heavy(icol, iwt, j, h0, h0 + hd, count);
                }
                __builtin_amdgcn_wave_barrier();
            }
            wb_sync();
            // ---------------- B: rounds of ready (vertex, lanes)
            if (tid < nb) {
                const int s = s_src[tid];
                __hip_atomic_store(&sig[row(s) + tid], MODE ? as_u64(1.0) : 1ull, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                if (atomicOr(&fm0[s], 1u << tid) == 0u) qa[atomicAdd(&s_n0, 1u)] = s;
            }
            if (tid == 0) {
                lvl_off[0] = 0;
                s_off = 0;
            }
            wb_sync();
            fc = fm0;
            fn = fm1;
            cur = qa;
            nxt = qb;
            int nl = 0;
            // FP64 path counts: ordered pull over the DAG in-arcs
            double acc = 0.0;
            int owner = 0;
            auto sig_fin = [&](int j, double x) {  // entry of lane gb + j (group-local j)
                const uint32_t m = s_em[wid][gb + j];
                if (!(m & kbit)) return;
                const int v = s_ev[wid][gb + j];
                const double sv = (v == s_src[k]) ? 1.0 : x;
                __hip_atomic_store(&sig[row(v) + k], as_u64(sv), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            };
            auto sig_pull = [&](const WArc *r) {
                unsigned long long dv[kWU], du[kWU];
                bool act[kWU];
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    act[q] = r[q].ok && (s_em[wid][r[q].o] & kbit);
                    dv[q] = act[q] ? s_ov[wid][r[q].o][k] : 0ull;
                    du[q] = act[q] ? wb_ld(&dist[row(r[q].x) + k]) : 0ull;
                }
                double x[kWU];
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    const bool dag = act[q] && du[q] != kWInf && du[q] + (unsigned long long)r[q].w == dv[q];
                    x[q] = dag ? as_f64(wb_ld(&sig[row(r[q].x) + k])) : 0.0;
                    if (!dag) act[q] = false;
                }
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    if (!r[q].ok) continue;
                    const int lo = r[q].o - gb;
                    if (lo != owner) {
                        sig_fin(owner, acc);
                        for (int e = owner + 1; e < lo; ++e) sig_fin(e, 0.0);
                        owner = lo;
                        acc = 0.0;
                    }
                    if (act[q]) acc += x[q];
                }
            };
            auto sig_heavy = [&](const WArc *r) {  // group partials in arc order
                unsigned long long dv[kWU], du[kWU];
                bool act[kWU];
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    act[q] = r[q].ok && (s_em[wid][r[q].o] & kbit);
                    dv[q] = act[q] ? s_ov[wid][r[q].o][k] : 0ull;
                    du[q] = act[q] ? wb_ld(&dist[row(r[q].x) + k]) : 0ull;
                }
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    if (act[q] && du[q] != kWInf && du[q] + (unsigned long long)r[q].w == dv[q])
                        acc += as_f64(wb_ld(&sig[row(r[q].x) + k]));
                }
            };
            // release of the DAG successors (and uint64 path counts pushed to them)
            auto release = [&](const WArc *r) {
                unsigned long long dv[kWU], dx[kWU], sv[kWU];
                bool act[kWU];
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    act[q] = r[q].ok && (s_em[wid][r[q].o] & kbit);
                    dv[q] = act[q] ? s_ov[wid][r[q].o][k] : 0ull;
                    sv[q] = (MODE == 0 && act[q]) ? s_os[wid][r[q].o][k] : 0ull;
                    dx[q] = act[q] ? wb_ld(&dist[row(r[q].x) + k]) : 0ull;
                }
                // the successor's lanes touched here are marked; which of them
                // became ready is read from the counts after the round
                unsigned long long old[kWU];
                bool dag[kWU];
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    dag[q] = act[q] && dv[q] + (unsigned long long)r[q].w == dx[q];
                    if (act[q]) ++st_dl;
                    old[q] = 0ull;
                    if (dag[q]) {
                        const size_t rx = row(r[q].x) + k;
                        if (MODE == 0) old[q] = atomicAdd(&sig[rx], sv[q]);
                        (void)atomicSub(&cnt[rx], 1);
                    }
                    const uint32_t gt = (uint32_t)(__ballot(dag[q]) >> gb) & ((1u << kWL) - 1u);
                    if (k == 0 && gt) (void)atomicOr(&fn[r[q].x], gt);
                }
                if (MODE == 0) {  // exact carry test of the uint64 sums
                    bool carry = false;
#pragma unroll
                    for (int q = 0; q < kWU; ++q) carry |= dag[q] && old[q] + sv[q] < old[q];
                    if (carry) atomicOr(&s_ovf, kbit);
                }
            };
            // after a round: a touched (vertex, lane) whose count reached zero is
            // ready; the touched mask becomes the ready mask, and vertices with a
            // ready lane form the next round's queue
            auto gather_ready = [&](uint32_t *mask, int32_t *list, uint32_t *cntr) {
                for (int b0 = wid * kWave; b0 < n; b0 += kWBBlock) {
                    const int v = b0 + lane;
                    const uint32_t m = v < n ? wb_ld32(&mask[v]) : 0u;
                    uint32_t ready = 0u;
                    if (m) {
                        const unsigned long long *cr = (const unsigned long long *)&cnt[row(v)];
                        unsigned long long c2[kWL / 2];
#pragma unroll
                        for (int j = 0; j < kWL / 2; ++j) c2[j] = wb_ld(&cr[j]);
#pragma unroll
                        for (int j = 0; j < kWL; ++j) {
                            const uint32_t c = (uint32_t)(c2[j >> 1] >> (32 * (j & 1)));
                            if (((m >> j) & 1u) && c == 0u) ready |= 1u << j;
                        }
                        __hip_atomic_store(&mask[v], ready, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    const unsigned long long bal = __ballot(ready != 0u);
                    if (!bal) continue;
                    uint32_t at = 0;
                    if (lane == 0) at = atomicAdd(cntr, (uint32_t)__popcll(bal));
                    at = __shfl(at, 0);
                    if (ready) list[at + __popcll(bal & ((1ull << lane) - 1ull))] = v;
                }
            };
            for (;;) {
                const uint32_t nc = s_n0;
                if (nc == 0) break;
                const int off = s_off;
                // capacity of the round records: every (vertex, lane) pair is ready once
                if (nl > n || (size_t)off + nc > nk) {
                    if (tid == 0) atomicOr(a.err, ERR_LEVEL_CAP);
                    break;
                }
                for (uint32_t i = tid; i < nc; i += kWBBlock) {
                    const int v = cur[i];
                    lvl[off + i] = v;
                    lvlm[off + i] = wb_ld32(&fc[v]);
                }
                if (MODE == 1) {
                    for (uint32_t cb = (uint32_t)wid * kWave; cb < nc; cb += kWBBlock) {
                        const uint32_t i = cb + lane;
                        const int v = i < nc ? cur[i] : -1;
                        const uint32_t m = v >= 0 ? wb_ld32(&fc[v]) : 0u;
                        const int e0 = v >= 0 ? irp[v] : 0;
                        const int dg = v >= 0 ? irp[v + 1] - e0 : 0;
                        const bool heavy = dg > kWBLight;
                        s_ev[wid][lane] = v;
                        s_em[wid][lane] = m;
                        __builtin_amdgcn_wave_barrier();
                        own_values(false);
                        s_em[wid][lane] = heavy ? 0u : m;  // heavy entries are finalised below
                        __builtin_amdgcn_wave_barrier();
                        st_darcs += (unsigned)dg;
                        acc = 0.0;
                        owner = 0;
                        walk_light(icol, iwt, e0, heavy ? 0 : dg, sig_pull);
                        sig_fin(owner, acc);
                        for (int e = owner + 1; e < kWL; ++e) sig_fin(e, 0.0);
                        __builtin_amdgcn_wave_barrier();
                        s_em[wid][lane] = m;
                        __builtin_amdgcn_wave_barrier();
                        for (unsigned long long hm = __ballot(heavy); hm; hm &= hm - 1) {
                            const int j = __ffsll(hm) - 1;
                            const int h0 = __builtin_amdgcn_readlane(e0, j), hd = __builtin_amdgcn_readlane(dg, j);
                            acc = 0.0;
                            walk_heavy(icol, iwt, j, h0, h0 + hd, sig_heavy);
                            const double tot = group_ordered_sum(acc);
                            if (lane < kWL && (s_em[wid][j] & kbit)) {
                                const int v2 = s_ev[wid][j];
                                const double sv = (v2 == s_src[k]) ? 1.0 : tot;
                                __hip_atomic_store(&sig[row(v2) + k], as_u64(sv), __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
                            }
                        }
                        __builtin_amdgcn_wave_barrier();
                    }
                    wb_sync();
                }
                for (uint32_t cb = (uint32_t)wid * kWave; cb < nc; cb += kWBBlock) {
                    const uint32_t i = cb + lane;
                    const int v = i < nc ? cur[i] : -1;
                    const uint32_t m = v >= 0 ? wb_ld32(&fc[v]) : 0u;
                    const int e0 = v >= 0 ? rp[v] : 0;
                    const int dg = v >= 0 ? rp[v + 1] - e0 : 0;
                    const bool heavy = dg > kWBLight;
                    s_ev[wid][lane] = v;
                    s_em[wid][lane] = m;
                    __builtin_amdgcn_wave_barrier();
                    own_values(MODE == 0);
                    st_darcs += (unsigned)dg;
                    if (MODE == 0 && a.sigma_limit != ~0ull) {  // a path count above the run's limit
#pragma unroll 1
                        for (int j = 0; j < kWL; ++j) {
                            if ((s_em[wid][gb + j] & kbit) && s_os[wid][gb + j][k] > a.sigma_limit)
                                atomicOr(&s_ovf, kbit);
                        }
                    }
                    walk_light(col, wt, e0, heavy ? 0 : dg, release);
                    for (unsigned long long hm = __ballot(heavy); hm; hm &= hm - 1) {
                        const int j = __ffsll(hm) - 1;
                        const int h0 = __builtin_amdgcn_readlane(e0, j), hd = __builtin_amdgcn_readlane(dg, j);
                        walk_heavy(col, wt, j, h0, h0 + hd, release);
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                wb_sync();
                for (uint32_t i = tid; i < nc; i += kWBBlock) fc[cur[i]] = 0u;
                gather_ready(fn, nxt, &s_n1);
                wb_sync();
                if (tid == 0) {
                    lvl_off[nl + 1] = off + (int)nc;
                    s_off = off + (int)nc;
                    s_n0 = s_n1;
                    s_n1 = 0;
                }
                wb_sync();
                ++nl;
                uint32_t *tm = fc;
                fc = fn;
                fn = tm;
                int32_t *tq = cur;
                cur = nxt;
                nxt = tq;
            }
            st_dag += (unsigned)nl;
            if (tid == 0) {
                const unsigned long long now = wall_clock64();
                tk_b += now - tk1;
                tk1 = now;
            }
            const uint32_t ovf = MODE == 0 ? s_ovf : 0u;
            const uint32_t live = ~ovf;
            // ---------------- C: dependencies, rounds in reverse
            auto dep_fin = [&](int j, double x) {
                const uint32_t m = s_em[wid][gb + j];
                if (!(m & kbit)) return;
                const int v = s_ev[wid][gb + j];
                const unsigned long long sb = wb_ld(&sig[row(v) + k]);
                const double sv = MODE ? as_f64(sb) : (double)sb;
                const double d = sv * x;
                wb_stf(&chat[row(v) + k], (1.0 + d) / sv);
                wb_stf(&dep[row(v) + k], d);
            };
            auto dep_pull = [&](const WArc *r) {
                unsigned long long dv[kWU], dx[kWU];
                bool act[kWU];
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    act[q] = r[q].ok && (s_em[wid][r[q].o] & kbit);
                    dv[q] = act[q] ? s_ov[wid][r[q].o][k] : 0ull;
                    dx[q] = act[q] ? wb_ld(&dist[row(r[q].x) + k]) : 0ull;
                }
                double x[kWU];
#if BC_WB_SPEC
                double cx[kWU];
#pragma unroll
                for (int q = 0; q < kWU; ++q) cx[q] = act[q] ? wb_ldf(&chat[row(r[q].x) + k]) : 0.0;
#endif
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    const bool dag = act[q] && dv[q] + (unsigned long long)r[q].w == dx[q];
#if BC_WB_SPEC
                    x[q] = dag ? cx[q] : 0.0;
#else
                    x[q] = dag ? wb_ldf(&chat[row(r[q].x) + k]) : 0.0;
#endif
                    if (act[q]) ++st_dl;
                    if (!dag) act[q] = false;
                }
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    if (!r[q].ok) continue;
                    const int lo = r[q].o - gb;
                    if (lo != owner) {
                        dep_fin(owner, acc);
                        for (int e = owner + 1; e < lo; ++e) dep_fin(e, 0.0);
                        owner = lo;
                        acc = 0.0;
                    }
                    if (act[q]) acc += x[q];
                }
            };
            auto dep_heavy = [&](const WArc *r) {
                unsigned long long dv[kWU], dx[kWU];
                bool act[kWU];
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    act[q] = r[q].ok && (s_em[wid][r[q].o] & kbit);
                    dv[q] = act[q] ? s_ov[wid][r[q].o][k] : 0ull;
                    dx[q] = act[q] ? wb_ld(&dist[row(r[q].x) + k]) : 0ull;
                }
#pragma unroll
                for (int q = 0; q < kWU; ++q) {
                    if (act[q]) ++st_dl;
                    if (act[q] && dv[q] + (unsigned long long)r[q].w == dx[q]) acc += wb_ldf(&chat[row(r[q].x) + k]);
                }
            };
            for (int l = nl - 1; l >= 0; --l) {
                const int b0 = lvl_off[l], b1 = lvl_off[l + 1];
                for (int cb = b0 + wid * kWave; cb < b1; cb += kWBBlock) {
                    const int i = cb + lane;
                    const int v = i < b1 ? lvl[i] : -1;
                    const uint32_t m = i < b1 ? (lvlm[i] & live) : 0u;
                    const int e0 = v >= 0 ? rp[v] : 0;
                    const int dg = v >= 0 ? rp[v + 1] - e0 : 0;
                    const bool heavy = dg > kWBLight;
                    s_ev[wid][lane] = v;
                    s_em[wid][lane] = m;
                    __builtin_amdgcn_wave_barrier();
                    own_values(false);
                    s_em[wid][lane] = heavy ? 0u : m;  // heavy entries are finalised below
                    __builtin_amdgcn_wave_barrier();
                    st_darcs += (unsigned)dg;
                    acc = 0.0;
                    owner = 0;
                    walk_light(col, wt, e0, heavy ? 0 : dg, dep_pull);
                    dep_fin(owner, acc);
                    for (int e = owner + 1; e < kWL; ++e) dep_fin(e, 0.0);
                    __builtin_amdgcn_wave_barrier();
                    s_em[wid][lane] = m;
                    __builtin_amdgcn_wave_barrier();
                    for (unsigned long long hm = __ballot(heavy); hm; hm &= hm - 1) {
                        const int j = __ffsll(hm) - 1;
                        const int h0 = __builtin_amdgcn_readlane(e0, j), hd = __builtin_amdgcn_readlane(dg, j);
                        acc = 0.0;
                        walk_heavy(col, wt, j, h0, h0 + hd, dep_heavy);
                        const double tot = group_ordered_sum(acc);
                        if (lane < kWL) dep_fin(j, tot);  // gb is 0 on these lanes: entry of lane j
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                wb_sync();
            }
            // the batch's dependencies into the chunk's partial scores, sources in order
            bool bad = false;
            for (uint32_t i = tid; i < nr; i += kWBBlock) {
                const int v = reached[i];
                const uint32_t m = wb_ld32(&rm[v]) & live;
                double pv = part[v];
                for (int kk = 0; kk < nb; ++kk) {
                    if (!((m >> kk) & 1u) || v == s_src[kk]) continue;
                    const double d = wb_ldf(&dep[row(v) + kk]);
                    if (MODE == 1 && !isfinite(d)) bad = true;
                    pv += d;
                }
                part[v] = pv;
            }
            if (bad) atomicOr(a.err, ERR_SIGMA_RANGE);
            if (tid < nb && ((ovf >> tid) & 1u)) {
                const uint32_t q = atomicAdd(a.ovf_count, 1u);
                if (q < a.ovf_cap) a.ovf_list[q] = a.pos[p0 + tid];
                else atomicOr(a.err, ERR_OVF_CAP);
            }
            if (a.dump_pos >= p0 && a.dump_pos < p0 + nb) {  // detail of one source
                const int kd = (int)(a.dump_pos - p0);
                const bool od = (ovf >> kd) & 1u;
                for (int i = tid; i < n; i += kWBBlock) {
                    const unsigned long long d = wb_ld(&dist[row(i) + kd]);
                    a.dump_d[i] = d == kWInf ? -1 : (int64_t)d;
                    a.dump_sig[i] = d == kWInf ? 0ull : wb_ld(&sig[row(i) + kd]);
                    a.dump_delta[i] = (d == kWInf || od || i == s_src[kd]) ? 0.0 : wb_ldf(&dep[row(i) + kd]);
                }
            }
            // reset what the batch touched
            wb_sync();
            for (size_t i = tid; i < (size_t)nr * kWL; i += kWBBlock) {
                const int v = reached[i / kWL];
                const size_t at = row(v) + (i % kWL);
                dist[at] = kWInf;
                sig[at] = 0ull;
                cnt[at] = 0;
            }
            for (uint32_t i = tid; i < nr; i += kWBBlock) rm[reached[i]] = 0u;
            if (tid == 0) {
                const unsigned long long now = wall_clock64();
                tk_c += now - tk1;
                tk_max = max(tk_max, now - tk0);
            }
        }
    }
    if (tid == 0) {
        if (tk_a) atomicAdd(&a.st[7], tk_a);
        if (tk_b) atomicAdd(&a.st[8], tk_b);
        if (tk_c) atomicAdd(&a.st[9], tk_c);
        if (tk_max) atomicMax(&a.st[10], tk_max);
    }
    // statistics (rounds are the same in every thread, the rest per thread)
    const unsigned long long vals[7] = {st_rounds, st_arcs, st_dag, st_pairs, st_darcs, st_rl, st_dl};
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const bool per_thread = !(q == 0 || q == 2);
        const unsigned long long x = per_thread ? wave_sum_u64(vals[q]) : vals[q];
        if (lane == 0 && (per_thread || tid == 0) && x) atomicAdd(&a.st[q], x);
    }
}

template __global__ void wbatch_run<0>(WeightedArgs);
template __global__ void wbatch_run<1>(WeightedArgs);

}  // namespace bcx
