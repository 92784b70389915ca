// bc_common.h -- wavefront helpers and the per-level policy, shared by the
// plain and batched step kernels.  Internal to libbc.
#pragma once

#include <climits>
#include <cmath>

#include "bc_dev.h"

namespace bcx {

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Number of set bits of m below this lane.
__device__ __forceinline__ unsigned lanes_below(unsigned long long m) {
    return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

__device__ __forceinline__ int wave_max_i(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o));
    return x;
}
__device__ __forceinline__ int wave_min_i(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o));
    return x;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}
__device__ __forceinline__ unsigned long long wave_or_u64(unsigned long long x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o);
    return x;
}
// Butterfly sum: a fixed association, so every lane ends with the same bits
// and the result does not depend on anything but the 64 inputs.
__device__ __forceinline__ double wave_sum_f64(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ double as_f64(unsigned long long u) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ unsigned long long as_u64(double x) { return (unsigned long long)__double_as_longlong(x); }

// Append w for every lane with pred to dst (one atomic per wavefront).  The
// wavefront must be converged.  Positions are relative to dst.
__device__ __forceinline__ void wave_append(bool pred, int32_t w, uint32_t *counter, int32_t *dst,
                                            uint32_t cap, int32_t *err) {
    const unsigned long long m = __ballot(pred);
    if (m == 0) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    unsigned base = 0;
    if (lane_id() == leader) base = atomicAdd(counter, (unsigned)__popcll(m));
    base = __shfl(base, leader);
    if (pred) {
        const unsigned p = base + lanes_below(m);
        if (p < cap) dst[p] = w;
        else atomicOr(err, ERR_QUEUE_CAP);
    }
}

// ---------------------------------------------------------------- counters
struct Counters {
    unsigned long long v[kNCnt];
    __device__ Counters() {
#pragma unroll
        for (int k = 0; k < kNCnt; ++k) v[k] = 0ull;
    }
    __device__ void exponent(int e) {
        v[SC_MAXE] = max(v[SC_MAXE], (unsigned long long)(e + 4096));
        v[SC_MINE] = max(v[SC_MINE], (unsigned long long)(4096 - e));
    }
};

__device__ __forceinline__ int cnt_op(int k) {  // 0 sum, 1 or, 2 max
    return k >= SC_PAIRS ? 0 : (k >= SC_MAXE ? 2 : (k >= SC_ACT ? 1 : 0));
}

__device__ __forceinline__ unsigned long long cnt_combine(int k, unsigned long long a, unsigned long long b) {
    const int op = cnt_op(k);
    return op == 0 ? a + b : (op == 1 ? (a | b) : (a > b ? a : b));
}

// Workgroups a step needs for `items` wavefront work items (at least one, at
// most the launched grid).  Workgroups beyond it leave at once.
__device__ __forceinline__ unsigned active_blocks(long long items, unsigned grid) {
    long long b = (items + kWavesPerBlock - 1) / kWavesPerBlock;
    if (b < 1) b = 1;
    if (b > (long long)grid) b = grid;
    return (unsigned)b;
}
__device__ __forceinline__ unsigned active_blocks(long long items) { return active_blocks(items, gridDim.x); }

// Work items of a step, [0, total), are dealt to ncls = min(nblk, kSlots)
// classes k mod ncls; the workgroups of class r (blockIdx.x mod ncls) share
// that class's items: each wavefront takes its first one statically, later
// ones from the class's counter (reset by the last workgroup of the launch),
// so a wavefront that finishes early takes the next item without all
// wavefronts meeting on one address.  Items are independent and each sum
// stays inside one item, so the assignment never changes a result.
struct WorkCursor {
    uint32_t *ctr;
    int r, ncls, nwr, j, jn;
    __device__ __forceinline__ WorkCursor(Ctl *c, unsigned nblk, unsigned bid) {
        ncls = (int)(nblk < (unsigned)kSlots ? nblk : (unsigned)kSlots);
        r = (int)(bid % (unsigned)ncls);
        const int nb = ((int)nblk - r + ncls - 1) / ncls;  // workgroups of class r
        nwr = nb * kWavesPerBlock;
        j = (int)(bid / (unsigned)ncls) * kWavesPerBlock + (int)(threadIdx.x >> 6);
        ctr = &c->work[r][0];
        jn = fetch();
    }
    __device__ __forceinline__ int fetch() {
        int x = 0;
        if ((threadIdx.x & 63) == 0) x = (int)atomicAdd(ctr, 1u);
        return nwr + __shfl(x, 0);
    }
    __device__ __forceinline__ int item() const { return r + ncls * j; }
    __device__ __forceinline__ void next(int total) {
        j = jn;
        if (item() < total) jn = fetch();
    }
};

// End of a step for one workgroup: reduce the counters over the workgroup,
// add them into the workgroup's slot, count the workgroup in (two-level
// arrival so no single address takes one atomic per workgroup).  Returns
// true in exactly one workgroup -- the last -- once every workgroup of the
// launch has arrived.  Workgroups without work (active == false) only count
// themselves in, so the last one cannot move the state machine on while a
// late workgroup still has to read it.
//
// No fences: within a launch, workgroups exchange only device-scope atomics
// here (slot counters, arrival counts, queue counters); plain stores are
// consumed by later launches, which kernel boundaries order.  The last
// workgroup must therefore never store to a word that another workgroup of
// the same launch stored to: each XCD's L2 would hold its own dirty copy
// until the launch ends and write it back in no fixed order.  Device-scope
// atomics that a workgroup issues before calling this (the slot counters
// here, a caller's exponent ranges) must have completed before it counts
// itself in: each wave that issued one waits for its memory counters first.
// s_red needs kWavesPerBlock * kNCnt entries.
__device__ __forceinline__ bool step_epilogue(Ctl *c, Counters &cn, unsigned long long *s_red, int *s_last,
                                              bool active, unsigned bid, unsigned grid) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int slot = bid % kSlots;
    if (active) {
#pragma unroll
        for (int k = 0; k < kNCnt; ++k) {
            unsigned long long x = cn.v[k];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) x = cnt_combine(k, x, __shfl_xor(x, o));
            if (lane == 0) s_red[wid * kNCnt + k] = x;
        }
        __syncthreads();
        if (threadIdx.x < kNCnt) {
            const int k = threadIdx.x;
            unsigned long long t = s_red[k];
            for (int w = 1; w < kWavesPerBlock; ++w) t = cnt_combine(k, t, s_red[w * kNCnt + k]);
            if (t) {
                const int op = cnt_op(k);
                if (op == 0) atomicAdd(&c->slot[slot][k], t);
                else if (op == 1) atomicOr(&c->slot[slot][k], t);
                else atomicMax(&c->slot[slot][k], t);
            }
        }
        // The slot atomics return nothing, so nothing has waited for them;
        // the last workgroup reads the slots once every arrival is counted,
        // so they must have completed before this workgroup arrives.
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int last = 0;
        const unsigned in_slot = (grid - slot + kSlots - 1) / kSlots;
        const unsigned t = atomicAdd(&c->arrive[slot], 1u);
        if (t == in_slot - 1) {
            const unsigned nslots = grid < (unsigned)kSlots ? grid : (unsigned)kSlots;
            const unsigned t2 = atomicAdd(&c->blocks_done, 1u);
            last = (t2 == nslots - 1) ? 1 : 0;
        }
        *s_last = last;
    }
    __syncthreads();
    return *s_last != 0;
}
__device__ __forceinline__ bool step_epilogue(Ctl *c, Counters &cn, unsigned long long *s_red, int *s_last,
                                              bool active) {
    return step_epilogue(c, cn, s_red, s_last, active, blockIdx.x, gridDim.x);
}

// In the last workgroup: totals of all slots into s_tot[kNCnt] (valid after
// the call in every thread); slots and arrival counters are reset.
__device__ __forceinline__ void collect_slots(Ctl *c, unsigned long long *s_tot, unsigned long long *s_tmp /*kSlots*kNCnt*/) {
    const int t = threadIdx.x;
    if (t < kSlots) {
#pragma unroll
        for (int k = 0; k < kNCnt; ++k) {
            s_tmp[t * kNCnt + k] = __hip_atomic_load(&c->slot[t][k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            c->slot[t][k] = 0ull;
        }
        c->arrive[t] = 0u;
        c->work[t][0] = 0u;
    }
    __syncthreads();
    if (t < kNCnt) {
        unsigned long long x = s_tmp[t];
        for (int sl = 1; sl < kSlots; ++sl) x = cnt_combine(t, x, s_tmp[sl * kNCnt + t]);
        s_tot[t] = x;
    }
    if (t == 0) c->blocks_done = 0u;
    __syncthreads();
}

// ----------------------------------------------------------- staged appends
// New level-queue entries are first gathered per wavefront in LDS and
// written in runs, one position atomic per run instead of per append.
constexpr int kStage = 128;
struct Stage {
    int32_t w[kStage];
    int32_t deg[kStage];
};

// Wavefront-inclusive prefix sum of an int.
__device__ __forceinline__ int wave_incl_scan(int x) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    return x;
}

__device__ __forceinline__ unsigned long long shfl_u64(unsigned long long x, int src) {
    const unsigned lo = __shfl((unsigned)x, src), hi = __shfl((unsigned)(x >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ int n_segments(int deg) { return (deg + kSeg - 1) / kSeg; }

// Degree that decides how a level entry is processed (one thread, one
// wavefront, or kSeg-arc segments) and what it costs: the larger of its out-
// and in-degree, so an entry is handled the same way in every phase, whichever
// arcs the phase scans (out-arcs to push and to pull dependencies from
// successors, in-arcs to pull discovery and path counts from predecessors).
// For an undirected graph it is the degree.
__device__ __forceinline__ int class_deg(const GraphArgs &g, int v, int out_deg) {
    return g.directed ? max(out_deg, g.in_row_ptr[v + 1] - g.in_row_ptr[v]) : out_deg;
}


// Write the n staged entries of this wavefront to the level queue (absolute
// positions qbase + counter), heavy ones also to the level's heavy list.
#ifndef BC_BUDGET
#define BC_BUDGET 64
#endif
constexpr int kBudget = BC_BUDGET;  // cost units (8 arcs each) per work group
static_assert(kBudget >= 2 && kBudget <= 128, "a group must fit in one wavefront (every entry costs >= 2 units)");

// Work estimate of a level entry in units of 8 arcs: its adjacency plus a
// fixed part; heavy entries (split into segments elsewhere) count 2.  Every
// entry costs at least 2 units, so a group never holds more than
// kBudget / 2 entries.
static __host__ __device__ __forceinline__ unsigned entry_cost(int deg) {
    return deg > kSeg ? 2u : 1u + (unsigned)(deg + 7) / 8u;
}

// Groups of a level: the entries whose cost prefix (in append order) starts
// in [k * kBudget, (k + 1) * kBudget) form group k, so every group carries
// about the same work.  Groups are found through gstart: gstart[gb + k] is
// the level-relative index of group k's first entry.  An entry whose cost
// range (P, P + c] contains the boundary k * kBudget writes gstart[gb + k] =
// its index + 1; gstart[gb] = 0 and the end are set when the level closes.
struct GroupArgs {
    uint32_t *gstart = nullptr;  // nullptr: no groups (per-source engine)
    uint32_t gb = 0;             // first gstart slot of the level being appended
    uint32_t gcap = 0;
};

__device__ __forceinline__ void stage_flush(Stage &st, int &n, Ctl *c, int32_t *q, uint32_t qbase, uint32_t qcap,
                                            const HeavyQ &hq, uint32_t hq_base, int32_t *err,
                                            const GroupArgs &ga) {
    if (n == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int lane = lane_id();
    // the run's entries and cost units, taken by one 64-bit atomic
    unsigned run_cost = 0;
    if (ga.gstart)
        for (int i = lane; i < n; i += kWave) run_cost += entry_cost(st.deg[i]);
    run_cost = (unsigned)wave_sum_u64(run_cost);
    unsigned long long old = 0;
    if (lane == 0)
        old = atomicAdd(&c->next_qc, (unsigned long long)(unsigned)n | ((unsigned long long)run_cost << 32));
    old = shfl_u64(old, 0);
    const unsigned base = (unsigned)old;
    unsigned cbase = (unsigned)(old >> 32);
    for (int i0 = 0; i0 < n; i0 += kWave) {
        const int i = i0 + lane;
        const bool on = i < n;
        const int w = on ? st.w[i] : 0;
        const int deg = on ? st.deg[i] : 0;
        const uint32_t p = qbase + base + (uint32_t)i;
        if (on) {
            if (p < qcap) q[p] = w;
            else atomicOr(err, ERR_QUEUE_CAP);
        }
        if (ga.gstart) {
            const unsigned ci = on ? entry_cost(deg) : 0u;
            const unsigned incl = (unsigned)wave_incl_scan((int)ci);
            const unsigned P = cbase + incl - ci;
            for (unsigned k = P / kBudget + 1; on && k <= (P + ci) / kBudget; ++k) {
                const unsigned long long at = (unsigned long long)ga.gb + k;
                if (at < ga.gcap) ga.gstart[at] = base + (uint32_t)i + 1u;
                else atomicOr(err, ERR_QUEUE_CAP);
            }
            cbase += (unsigned)__shfl((int)incl, 63);
        }
        const bool heavy = on && deg > kSeg;
        const unsigned long long hm = __ballot(heavy);
        if (hm) {
            const int ns = heavy ? n_segments(deg) : 0;
            const int incl = wave_incl_scan(ns);
            const int total = __shfl(incl, 63);
            const int hl = __ffsll((unsigned long long)hm) - 1;
            unsigned long long hold = 0;
            if (lane == hl)
                hold = atomicAdd(&c->next_hq,
                                 (unsigned long long)__popcll(hm) | ((unsigned long long)(unsigned)total << 32));
            hold = shfl_u64(hold, hl);
            if (heavy) {
                const uint32_t idx = hq_base + (uint32_t)hold + lanes_below(hm);
                if (idx < hq.cap) {
                    hq.pos[idx] = (int32_t)p;
                    hq.seg[idx] = (int32_t)(hold >> 32) + (incl - ns);
                    hq.cnt[idx] = 0;
                } else {
                    atomicOr(err, ERR_QUEUE_CAP);
                }
            }
        }
    }
    n = 0;
}

// Stage w (degree deg) for every lane with pred; flushes once 64 or more are
// waiting.  n is the wavefront-uniform fill count.  The wavefront must be
// converged.
__device__ __forceinline__ void stage_push(bool pred, int32_t w, int32_t deg, Stage &st, int &n, Ctl *c, int32_t *q,
                                           uint32_t qbase, uint32_t qcap, const HeavyQ &hq, uint32_t hq_base,
                                           int32_t *err, const GroupArgs &ga) {
    const unsigned long long m = __ballot(pred);
    if (m == 0) return;
    if (pred) {
        const int pos = n + (int)lanes_below(m);
        st.w[pos] = w;
        st.deg[pos] = deg;
    }
    n += __popcll(m);
    if (n >= kWave) stage_flush(st, n, c, q, qbase, qcap, hq, hq_base, err, ga);
}

// Largest h in [h0, h1) with seg[h] <= t (seg ascending, seg[h0] = 0 <= t).
__device__ __forceinline__ int seg_owner(const int32_t *seg, int h0, int h1, int t) {
    int lo = h0, hi = h1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (seg[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// First index i in [0, n) with a[i] >= x (a ascending).
__device__ __forceinline__ int lower_bound_i32(const int32_t *a, int n, int x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Block-wide sum of one unsigned 64-bit value per thread; result valid in
// thread 0.  Uses the caller's shared scratch of kWavesPerBlock entries.
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long x, unsigned long long *sh) {
    x = wave_sum_u64(x);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if (lane_id() == 0) sh[w] = x;
    __syncthreads();
    unsigned long long t = 0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kWavesPerBlock; ++i) t += sh[i];
    return t;
}

// Features of a level, normalised as documented for the policy network.
struct LevelFeatures {
    float nf, mf, nu, mu;
    int level;
};

__device__ __forceinline__ void mlp_inputs(const LevelFeatures &f, float n, float nnz, float *x) {
    const float ln = log2f(1.0f + n), lm = log2f(1.0f + nnz);
    x[0] = log2f(1.0f + f.nf) / fmaxf(ln, 1.0f);
    x[1] = log2f(1.0f + f.mf) / fmaxf(lm, 1.0f);
    x[2] = log2f(1.0f + f.nu) / fmaxf(ln, 1.0f);
    x[3] = log2f(1.0f + f.mu) / fmaxf(lm, 1.0f);
    x[4] = (float)f.level / 64.0f;
}

// Direction-optimising rule (Beamer, Asanovic, Patterson, SC'12): go
// bottom-up once the frontier's arcs exceed the unvisited arcs / alpha, come
// back top-down once the frontier has fewer than n / beta vertices.  The
// push variants split by mean frontier degree.
__device__ __forceinline__ int heuristic_variant(const PolicyArgs &p, int prev, const LevelFeatures &f,
                                                 float n) {
    bool pull;
    if (prev == V_PULL) pull = !(f.nf < n / p.beta);
    else pull = f.mf > f.mu / p.alpha;
    if (pull) return V_PULL;
    return (f.nf > 0.0f && f.mf / f.nf > p.wpv_degree) ? V_PUSH_WPV : V_PUSH_TPV;
}

// argmin of y[k0 .. k0 + 2] (the first on ties)
__device__ __forceinline__ int argmin3(const float *y, int k0) {
    int best = 0;
    float bv = y[k0];
    if (y[k0 + 1] < bv) { best = 1; bv = y[k0 + 1]; }
    if (y[k0 + 2] < bv) best = 2;
    return best;
}

// Choose the variant of the next level, and (in *lbo) the summation options
// of the path-count step that sums the entries it discovers and of the
// backward step over the level's own entries (option | option << 2).  Called
// by every thread of one workgroup (the MLP spreads its hidden units over
// threads); the result is returned to every thread.  lds needs
// 2 * kMlpH + kMlpOut floats.  Only the learned policy changes the summation
// options; every other policy keeps the sources-per-entry rule.
__device__ __forceinline__ int choose_variant(const PolicyArgs &p, int policy, int prev, const LevelFeatures &f, float n,
                              float nnz, float *lds, int *lbo) {
    *lbo = kLbDefault;
    if (policy == POL_FORCE_TPV) return V_PUSH_TPV;
    if (policy == POL_FORCE_WPV) return V_PUSH_WPV;
    if (policy == POL_FORCE_PULL) return V_PULL;
    if (policy == POL_MLP && p.has_mlp) {
        const float *W1 = p.mlp;
        const float *b1 = W1 + kMlpH * kMlpIn;
        const float *W2 = b1 + kMlpH;
        const float *b2 = W2 + kMlpH * kMlpH;
        const float *W3 = b2 + kMlpH;
        const float *b3 = W3 + kMlpOut * kMlpH;
        float x[kMlpIn];
        mlp_inputs(f, n, nnz, x);
        const int t = threadIdx.x;
        float *h1 = lds, *h2 = lds + kMlpH, *y = lds + 2 * kMlpH;
        if (t < kMlpH) {
            float s = b1[t];
            for (int i = 0; i < kMlpIn; ++i) s += W1[t * kMlpIn + i] * x[i];
            h1[t] = fmaxf(s, 0.0f);
        }
        __syncthreads();
        if (t < kMlpH) {
            float s = b2[t];
            for (int i = 0; i < kMlpH; ++i) s += W2[t * kMlpH + i] * h1[i];
            h2[t] = fmaxf(s, 0.0f);
        }
        __syncthreads();
        if (t < kMlpOut) {
            float s = b3[t];
            for (int i = 0; i < kMlpH; ++i) s += W3[t * kMlpH + i] * h2[i];
            y[t] = s;
        }
        __syncthreads();
        float yy[kMlpOut];
        bool finite = true;
        for (int k = 0; k < kMlpOut; ++k) {
            yy[k] = y[k];
            finite = finite && isfinite(yy[k]);
        }
        __syncthreads();
        if (finite) {
            // the rule's choice stands unless the network predicts a gain of
            // at least p.margin (log2 units) for another one
            const float m = p.margin;
            int v = argmin3(yy, kOutFwd), so = argmin3(yy, kOutSig), bo = argmin3(yy, kOutBwd);
            const int h = heuristic_variant(p, prev, f, n);
            if (yy[kOutFwd + h] - yy[kOutFwd + v] < m) v = h;
            if (yy[kOutSig + LB_RULE] - yy[kOutSig + so] < m) so = LB_RULE;
            if (yy[kOutBwd + LB_RULE] - yy[kOutBwd + bo] < m) bo = LB_RULE;
            *lbo = so | (bo << 2);
            return v;
        }
        // non-finite prediction: fall back to the rules
    }
    return heuristic_variant(p, prev, f, n);
}

// Sources-per-entry threshold of a summation option: groups whose light
// entries carry at most this many sources on average are summed by (entry,
// source) pairs.
__device__ __forceinline__ float lb_item_lanes(const PolicyArgs &p, int opt) {
    return opt == LB_PACKED ? -1.0f : (opt == LB_ITEMS ? 65.0f : p.item_lanes);
}

// Partial sums exchanged between the wavefronts of one launch (segments of
// a heavy vertex): stored and loaded with device-scope relaxed atomics, which
// are written through to, and read from, the point of coherence of all
// XCDs, so no cache-wide fence (L2 write-back / invalidate) is needed.
// seg_arrive waits until this wavefront's partial stores have completed,
// then counts it in; the wavefront that arrives last (returns true) reads
// every partial with part_load.
__device__ __forceinline__ void part_store(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long part_load(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool seg_arrive(int32_t *cnt, int nseg) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);  // every memory operation of this wavefront has completed
    int old = 0;
    if (lane_id() == 0) old = __hip_atomic_fetch_add(cnt, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    old = __shfl(old, 0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return old == nseg - 1;
}

template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace bcx
