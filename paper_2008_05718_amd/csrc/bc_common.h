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

// Choose the variant of the next level.  Called by every thread of one
// workgroup (the MLP spreads its hidden units over threads); the result is
// returned to every thread.  lds needs 2 * kMlpH + 4 floats.
__device__ int choose_variant(const PolicyArgs &p, int policy, int prev, const LevelFeatures &f, float n,
                              float nnz, float *lds) {
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
        const float y0 = y[0], y1 = y[1], y2 = y[2];
        __syncthreads();
        if (isfinite(y0) && isfinite(y1) && isfinite(y2)) {
            int best = 0;
            float bv = y0;
            if (y1 < bv) { best = 1; bv = y1; }
            if (y2 < bv) { best = 2; }
            return best;
        }
        // non-finite prediction: fall back to the rule
    }
    return heuristic_variant(p, prev, f, n);
}

// Last-workgroup detection: every workgroup calls this once at its end; it
// returns true in exactly one workgroup, after all others have arrived, with
// their memory operations visible.
__device__ __forceinline__ bool last_block_arrive(uint32_t *counter, int *s_last) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned t = atomicAdd(counter, 1u);
        *s_last = (t == gridDim.x - 1) ? 1 : 0;
    }
    __syncthreads();
    if (*s_last) __threadfence();
    return *s_last != 0;
}

template <typename T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace bcx
