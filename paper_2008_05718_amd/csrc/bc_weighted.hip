// bc_weighted.hip -- Brandes on graphs with positive integer arc weights.
//
// The paper's forward phase is "a BFS traversal or SSSP calculation"
// (Section "Background") and its graph layout keeps edge weights (Section
// "Space Complexity").  With weights the level structure of a breadth-first
// search is gone, so this engine is organised differently from the batched
// one: a persistent launch in which every workgroup computes whole sources,
// one after another, on a private copy of the per-vertex state.  Per source:
//
//   A  distances: label-correcting relaxation rounds (a vertex whose
//      distance dropped in a round relaxes its out-arcs in the next one,
//      64-bit atomicMin on the tentative distance); with positive weights
//      the rounds end with the exact shortest distances, whatever the order
//      of the relaxations.
//   B  path counts: the arcs v -> t with d(v) + w(v, t) = d(t) form the
//      shortest-path DAG.  Each reached vertex counts its DAG in-arcs; a
//      vertex is "ready" when every DAG predecessor has its count.  Rounds of
//      ready vertices pull sigma(t) = sum of sigma(v) over the DAG in-arcs
//      (CSR order), then release their DAG successors.  The rounds are the
//      levels of the DAG by longest hop count, kept for phase C.
//   C  dependencies: the rounds in reverse; delta(v) = sigma(v) * sum over DAG
//      out-arcs of c(u), c(u) = (1 + delta(u)) / sigma(u) (Eq. 2 with sigma(v)
//      factored out), then the source's delta is added to the workgroup's
//      partial scores.
//
// Arcs of up to 64 list entries (one per lane) are packed into rounds of 64
// arcs, one per lane, so the loads of a round are issued together; a sum over
// a vertex's arcs is then taken by its own lane in CSR order from the
// round's values (readlane, ascending lane = ascending arc).  Vertices of
// degree above kWHeavy are taken by one wavefront, lane-strided then a fixed
// butterfly.  Every result is fixed by the vertex alone and runs are
// bitwise reproducible.  Path counts are uint64 (MODE 0) with exact overflow
// detection; a source that overflows is handed back and computed again with
// FP64 counts (MODE 1).  Chunks of consecutive sources go to one partial
// vector, and the partials are added in chunk order afterwards (host).
#include "bc_common.h"

namespace bcx {

constexpr unsigned long long kInf = ~0ull;

__device__ __forceinline__ unsigned long long ld_dist(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wavefront-wide sum of v over lanes (fixed butterfly; every lane gets it).
__device__ __forceinline__ double wsum_f64(double v) { return wave_sum_f64(v); }

constexpr int kWHeavy = 4096;  // vertices with more arcs go to one wavefront each

__device__ __forceinline__ unsigned long long lane_u64(unsigned long long x, int j) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, j);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), j);
    return ((unsigned long long)hi << 32) | lo;
}

// Lane holding packed arc a: the first lane whose inclusive degree prefix
// exceeds a (binary search over the wavefront).
__device__ __forceinline__ int arc_lane(int incl, int a) {
    int o = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        if (__shfl(incl, o + step - 1) <= a) o += step;
    }
    return o;
}

// The arcs [rp[v], rp[v+1]) of this lane's entry v (v < 0: none; degree above
// kWHeavy: skipped), all lanes' arcs in lane order, handed out 64 per round:
// body(ok, o, e) runs on every lane of every round, with arc e of the entry
// of lane o when ok.  The wavefront must be converged.
template <class Body>
__device__ __forceinline__ void packed_arcs(const int32_t *__restrict__ rp, int v, Body body) {
    const int lane = lane_id();
    const int e0 = v >= 0 ? rp[v] : 0;
    int deg = v >= 0 ? rp[v + 1] - e0 : 0;
    if (deg > kWHeavy) deg = 0;
    const int incl = wave_incl_scan(deg);
    const int total = __shfl(incl, kWave - 1);
    const int excl = incl - deg;
    for (int ab = 0; ab < total; ab += kWave) {
        const int a = ab + lane;
        const bool ok = a < total;
        const int o = arc_lane(incl, ok ? a : total - 1);
        const int e = __shfl(e0, o) + (a - __shfl(excl, o));
        body(ok, o, e);
    }
}

// Workgroup barrier after which every global store and atomic issued before
// it has completed: distances are read with device-scope loads that go to
// the L2, so a plain store still in flight would not be seen.
__device__ __forceinline__ void wg_sync() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void weighted_run(WeightedArgs a) {
    __shared__ int s_chunk;
    __shared__ uint32_t s_n0, s_n1, s_nr, s_ovf;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int n = a.g.n;
    const int32_t *__restrict__ rp = a.g.row_ptr;
    const int32_t *__restrict__ col = a.g.col;
    const int32_t *__restrict__ irp = a.g.in_row_ptr;
    const int32_t *__restrict__ icol = a.g.in_col;
    const int32_t *__restrict__ wt = a.wt;
    const int32_t *__restrict__ iwt = a.in_wt;
    char *base = a.scratch + (size_t)blockIdx.x * a.stride;
    const WeightedLayout L((size_t)n);
    unsigned long long *dist = (unsigned long long *)(base + L.dist);
    unsigned long long *sig = (unsigned long long *)(base + L.sig);
    double *chat = (double *)(base + L.chat);
    double *dep = (double *)(base + L.dep);
    int32_t *cnt = (int32_t *)(base + L.cnt);
    uint32_t *mark = (uint32_t *)(base + L.mark);
    int32_t *reached = (int32_t *)(base + L.reached);
    int32_t *qa = (int32_t *)(base + L.qa);
    int32_t *qb = (int32_t *)(base + L.qb);
    int32_t *lvl = (int32_t *)(base + L.lvl);
    int32_t *lvl_off = (int32_t *)(base + L.lvl_off);
    unsigned long long st_rounds = 0, st_arcs = 0, st_dag = 0, st_reached = 0, st_darcs = 0;
    // the state of a fresh workgroup: every distance unknown, no marks, no counts
    for (int i = tid; i < n; i += kBlock) {
        dist[i] = kInf;
        mark[i] = 0u;
        cnt[i] = 0;
    }
    for (;;) {
        wg_sync();
        if (tid == 0) {
            const uint32_t k = atomicAdd(a.next, 1u);
            s_chunk = (k < (uint32_t)a.n_chunks && ld_agent(a.err) == 0) ? a.order[k] : -1;
        }
        __syncthreads();
        const int t = s_chunk;
        if (t < 0) break;
        double *part = a.partials + (size_t)t * (size_t)n;
        for (int i = tid; i < n; i += kBlock) part[i] = 0.0;
        for (int p = a.c_s0[t]; p < a.c_s1[t]; ++p) {
            const int s = a.srcs[p];
            // ---------------- A: distances
            wg_sync();
            if (tid == 0) {
                dist[s] = 0ull;
                reached[0] = s;
                qa[0] = s;
                mark[s] = 1u;
                s_nr = 1;
                s_n0 = 1;
                s_n1 = 0;
            }
            wg_sync();
            int32_t *cur = qa, *nxt = qb;
            uint32_t round = 1;
            for (;;) {
                const uint32_t nc = s_n0;
                if (nc == 0) break;
                ++round;
                if ((int64_t)round > (int64_t)n + 2) {  // cannot happen with positive weights
                    if (tid == 0) atomicOr(a.err, ERR_LEVEL_CAP);
                    break;
                }
                // packed rounds of 64 arcs per wavefront, heavy vertices one per wavefront
                for (uint32_t cb = (uint32_t)wid * kWave; cb < nc; cb += kBlock) {
                    const uint32_t i = cb + lane;
                    const int v = i < nc ? cur[i] : -1;
                    const unsigned long long dv = v >= 0 ? ld_dist(&dist[v]) : 0ull;
                    if (v >= 0 && rp[v + 1] - rp[v] <= kWHeavy) st_arcs += (unsigned)(rp[v + 1] - rp[v]);
                    packed_arcs(rp, v, [&](bool ok, int o, int e) {
                        const unsigned long long dvo = shfl_u64(dv, o);
                        if (!ok) return;
                        const int x = col[e];
                        const unsigned long long nd = dvo + (unsigned long long)wt[e];
                        if (nd < ld_dist(&dist[x])) {
                            const unsigned long long old = atomicMin(&dist[x], nd);
                            if (nd < old) {
                                if (old == kInf) reached[atomicAdd(&s_nr, 1u)] = x;
                                if (atomicExch(&mark[x], round) != round) nxt[atomicAdd(&s_n1, 1u)] = x;
                            }
                        }
                    });
                }
                for (uint32_t i = wid; i < nc; i += kWavesPerBlock) {
                    const int v = cur[i];
                    const int e0 = rp[v], e1 = rp[v + 1];
                    if (e1 - e0 <= kWHeavy) continue;
                    const unsigned long long dv = ld_dist(&dist[v]);
                    if (lane == 0) st_arcs += (unsigned)(e1 - e0);
                    for (int e = e0 + lane; e < e1; e += kWave) {
                        const int x = col[e];
                        const unsigned long long nd = dv + (unsigned long long)wt[e];
                        if (nd < ld_dist(&dist[x])) {
                            const unsigned long long old = atomicMin(&dist[x], nd);
                            if (nd < old) {
                                if (old == kInf) reached[atomicAdd(&s_nr, 1u)] = x;
                                if (atomicExch(&mark[x], round) != round) nxt[atomicAdd(&s_n1, 1u)] = x;
                            }
                        }
                    }
                }
                wg_sync();
                if (tid == 0) {
                    s_n0 = s_n1;
                    s_n1 = 0;
                }
                wg_sync();
                int32_t *tmp = cur;
                cur = nxt;
                nxt = tmp;
                ++st_rounds;
            }
            const uint32_t nr = s_nr;
            st_reached += nr;
            // ---------------- B: DAG in-arc counts, then rounds of ready vertices
            for (uint32_t cb = (uint32_t)wid * kWave; cb < nr; cb += kBlock) {
                const uint32_t i = cb + lane;
                const int v = i < nr ? reached[i] : -1;
                const bool light = v >= 0 && irp[v + 1] - irp[v] <= kWHeavy;
                const unsigned long long dv = v >= 0 ? ld_dist(&dist[v]) : 0ull;
                if (light) st_darcs += (unsigned)(irp[v + 1] - irp[v]);
                int c = 0;
                packed_arcs(irp, v, [&](bool ok, int o, int e) {
                    const unsigned long long dvo = shfl_u64(dv, o);
                    bool dag = false;
                    if (ok) {
                        const unsigned long long du = ld_dist(&dist[icol[e]]);
                        dag = du != kInf && du + (unsigned long long)iwt[e] == dvo;
                    }
                    // each lane counts the DAG in-arcs that belong to its entry
                    for (unsigned long long bal = __ballot(dag); bal; bal &= bal - 1) {
                        const int j = __ffsll(bal) - 1;
                        if (__builtin_amdgcn_readlane(o, j) == lane) ++c;
                    }
                });
                if (light) cnt[v] = c;
            }
            for (uint32_t i = wid; i < nr; i += kWavesPerBlock) {
                const int v = reached[i];
                if (irp[v + 1] - irp[v] <= kWHeavy) continue;
                const unsigned long long dv = ld_dist(&dist[v]);
                if (lane == 0) st_darcs += (unsigned)(irp[v + 1] - irp[v]);
                int c = 0;
                for (int e = irp[v] + lane; e < irp[v + 1]; e += kWave) {
                    const unsigned long long du = ld_dist(&dist[icol[e]]);
                    if (du != kInf && du + (unsigned long long)iwt[e] == dv) ++c;
                }
                c = (int)wave_sum_u64((unsigned long long)c);
                if (lane == 0) cnt[v] = c;
            }
            wg_sync();
            if (tid == 0) {
                qa[0] = s;
                s_n0 = 1;
                s_n1 = 0;
                s_ovf = 0;
                lvl_off[0] = 0;
            }
            wg_sync();
            cur = qa;
            nxt = qb;
            int nl = 0;
            for (;;) {
                const uint32_t nc = s_n0;
                if (nc == 0) break;
                const int off = lvl_off[nl];
                // path counts of the ready vertices (their predecessors are final)
                for (uint32_t i = tid; i < nc; i += kBlock) lvl[off + i] = cur[i];
                for (uint32_t cb = (uint32_t)wid * kWave; cb < nc; cb += kBlock) {
                    const uint32_t i = cb + lane;
                    const int v0 = i < nc ? cur[i] : -1;
                    const int v = v0 == s ? -1 : v0;  // the source has no predecessors
                    const bool light = v >= 0 && irp[v + 1] - irp[v] <= kWHeavy;
                    const unsigned long long dv = v >= 0 ? ld_dist(&dist[v]) : 0ull;
                    if (light) st_darcs += (unsigned)(irp[v + 1] - irp[v]);
                    unsigned long long lo = 0, hi = 0;
                    double accd = 0.0;
                    packed_arcs(irp, v, [&](bool ok, int o, int e) {
                        const unsigned long long dvo = shfl_u64(dv, o);
                        unsigned long long x = 0;
                        bool dag = false;
                        if (ok) {
                            const int u = icol[e];
                            const unsigned long long du = ld_dist(&dist[u]);
                            dag = du != kInf && du + (unsigned long long)iwt[e] == dvo;
                            if (dag) x = sig[u];
                        }
                        // each lane adds its entry's terms in arc order
                        for (unsigned long long bal = __ballot(dag); bal; bal &= bal - 1) {
                            const int j = __ffsll(bal) - 1;
                            const unsigned long long xj = lane_u64(x, j);
                            if (__builtin_amdgcn_readlane(o, j) == lane) {
                                if (MODE == 0) {
                                    lo += xj;
                                    hi += (lo < xj) ? 1ull : 0ull;
                                } else {
                                    accd += as_f64(xj);
                                }
                            }
                        }
                    });
                    if (v0 == s) {
                        sig[s] = MODE ? as_u64(1.0) : 1ull;
                    } else if (light) {
                        if (MODE == 0) {
                            sig[v] = lo;
                            if (hi != 0 || lo > a.sigma_limit) s_ovf = 1;
                        } else {
                            sig[v] = as_u64(accd);
                        }
                    }
                }
                for (uint32_t i = wid; i < nc; i += kWavesPerBlock) {
                    const int v = cur[i];
                    const int e0 = irp[v], e1 = irp[v + 1];
                    if (v == s || e1 - e0 <= kWHeavy) continue;
                    const unsigned long long dv = ld_dist(&dist[v]);
                    if (lane == 0) st_darcs += (unsigned)(e1 - e0);
                    unsigned long long lo = 0, hi = 0;
                    double accd = 0.0;
                    for (int e = e0 + lane; e < e1; e += kWave) {
                        const int u = icol[e];
                        const unsigned long long du = ld_dist(&dist[u]);
                        if (du == kInf || du + (unsigned long long)iwt[e] != dv) continue;
                        if (MODE == 0) {
                            lo += sig[u];
                            hi += (lo < sig[u]) ? 1ull : 0ull;
                        } else {
                            accd += as_f64(sig[u]);
                        }
                    }
                    if (MODE == 0) {
                        // exact 128-bit wavefront sum
#pragma unroll
                        for (int o = 32; o > 0; o >>= 1) {
                            const unsigned long long ol = shfl_u64(lo, lane ^ o), oh = shfl_u64(hi, lane ^ o);
                            const unsigned long long nl2 = lo + ol;
                            hi = hi + oh + ((nl2 < lo) ? 1ull : 0ull);
                            lo = nl2;
                        }
                        if (lane == 0) {
                            sig[v] = lo;
                            if (hi != 0 || lo > a.sigma_limit) s_ovf = 1;
                        }
                    } else {
                        accd = wsum_f64(accd);
                        if (lane == 0) sig[v] = as_u64(accd);
                    }
                }
                wg_sync();
                // release the DAG successors
                for (uint32_t cb = (uint32_t)wid * kWave; cb < nc; cb += kBlock) {
                    const uint32_t i = cb + lane;
                    const int v = i < nc ? cur[i] : -1;
                    const unsigned long long dv = v >= 0 ? ld_dist(&dist[v]) : 0ull;
                    if (v >= 0 && rp[v + 1] - rp[v] <= kWHeavy) st_darcs += (unsigned)(rp[v + 1] - rp[v]);
                    packed_arcs(rp, v, [&](bool ok, int o, int e) {
                        const unsigned long long dvo = shfl_u64(dv, o);
                        if (!ok) return;
                        const int x = col[e];
                        if (dvo + (unsigned long long)wt[e] == ld_dist(&dist[x]) && atomicSub(&cnt[x], 1) == 1)
                            nxt[atomicAdd(&s_n1, 1u)] = x;
                    });
                }
                for (uint32_t i = wid; i < nc; i += kWavesPerBlock) {
                    const int v = cur[i];
                    if (rp[v + 1] - rp[v] <= kWHeavy) continue;
                    const unsigned long long dv = ld_dist(&dist[v]);
                    if (lane == 0) st_darcs += (unsigned)(rp[v + 1] - rp[v]);
                    for (int e = rp[v] + lane; e < rp[v + 1]; e += kWave) {
                        const int x = col[e];
                        if (dv + (unsigned long long)wt[e] == ld_dist(&dist[x]) && atomicSub(&cnt[x], 1) == 1)
                            nxt[atomicAdd(&s_n1, 1u)] = x;
                    }
                }
                wg_sync();
                if (tid == 0) {
                    lvl_off[nl + 1] = off + (int)nc;
                    s_n0 = s_n1;
                    s_n1 = 0;
                }
                wg_sync();
                ++nl;
                int32_t *tmp = cur;
                cur = nxt;
                nxt = tmp;
            }
            st_dag += (unsigned)nl;
            const bool ovf = MODE == 0 && s_ovf != 0;
            // ---------------- C: dependencies, rounds in reverse
            if (!ovf) {
                for (int l = nl - 1; l >= 0; --l) {
                    const int b0 = lvl_off[l], b1 = lvl_off[l + 1];
                    for (int cb = b0 + wid * kWave; cb < b1; cb += kBlock) {
                        const int i = cb + lane;
                        const int v = i < b1 ? lvl[i] : -1;
                        const bool light = v >= 0 && rp[v + 1] - rp[v] <= kWHeavy;
                        const unsigned long long dv = v >= 0 ? ld_dist(&dist[v]) : 0ull;
                        if (light) st_darcs += (unsigned)(rp[v + 1] - rp[v]);
                        double acc = 0.0;
                        packed_arcs(rp, v, [&](bool ok, int o, int e) {
                            const unsigned long long dvo = shfl_u64(dv, o);
                            double x = 0.0;
                            bool dag = false;
                            if (ok) {
                                const int u = col[e];
                                dag = dvo + (unsigned long long)wt[e] == ld_dist(&dist[u]);
                                if (dag) x = chat[u];
                            }
                            // each lane adds its entry's terms in arc order
                            for (unsigned long long bal = __ballot(dag); bal; bal &= bal - 1) {
                                const int j = __ffsll(bal) - 1;
                                const double xj = as_f64(lane_u64(as_u64(x), j));
                                if (__builtin_amdgcn_readlane(o, j) == lane) acc += xj;
                            }
                        });
                        if (light) {
                            const double sv = MODE ? as_f64(sig[v]) : (double)sig[v];
                            const double delta = sv * acc;
                            chat[v] = (1.0 + delta) / sv;
                            dep[v] = delta;
                        }
                    }
                    for (int i = b0 + wid; i < b1; i += kWavesPerBlock) {
                        const int v = lvl[i];
                        const int e0 = rp[v], e1 = rp[v + 1];
                        if (e1 - e0 <= kWHeavy) continue;
                        const unsigned long long dv = ld_dist(&dist[v]);
                        if (lane == 0) st_darcs += (unsigned)(e1 - e0);
                        double acc = 0.0;
                        for (int e = e0 + lane; e < e1; e += kWave) {
                            const int u = col[e];
                            if (dv + (unsigned long long)wt[e] == ld_dist(&dist[u])) acc += chat[u];
                        }
                        acc = wsum_f64(acc);
                        if (lane == 0) {
                            const double sv = MODE ? as_f64(sig[v]) : (double)sig[v];
                            const double delta = sv * acc;
                            chat[v] = (1.0 + delta) / sv;
                            dep[v] = delta;
                        }
                    }
                    wg_sync();
                }
                // the source's dependencies into the chunk's partial scores
                bool bad = false;
                for (uint32_t i = tid; i < nr; i += kBlock) {
                    const int v = reached[i];
                    if (v != s) part[v] += dep[v];
                    if (MODE == 1 && !isfinite(dep[v])) bad = true;
                }
                if (bad) atomicOr(a.err, ERR_SIGMA_RANGE);
            } else if (tid == 0) {
                const uint32_t q = atomicAdd(a.ovf_count, 1u);
                if (q < a.ovf_cap) a.ovf_list[q] = a.pos[p];
                else atomicOr(a.err, ERR_OVF_CAP);
            }
            if (p == a.dump_pos) {  // detail of one source
                for (int i = tid; i < n; i += kBlock) {
                    const unsigned long long d = ld_dist(&dist[i]);
                    a.dump_d[i] = d == kInf ? -1 : (int64_t)d;
                    a.dump_sig[i] = d == kInf ? 0ull : sig[i];
                    a.dump_delta[i] = (d == kInf || ovf || i == s) ? 0.0 : dep[i];
                }
            }
            // reset what this source touched
            wg_sync();
            for (uint32_t i = tid; i < nr; i += kBlock) {
                const int v = reached[i];
                dist[v] = kInf;
                mark[v] = 0u;
                cnt[v] = 0;
            }
        }
    }
    // statistics
    // (rounds, DAG rounds and reached pairs are the same in every thread;
    // arc counts are per thread)
    const unsigned long long vals[5] = {st_rounds, st_arcs, st_dag, st_reached, st_darcs};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const bool per_thread = k == 1 || k == 4;
        unsigned long long x = per_thread ? wave_sum_u64(vals[k]) : vals[k];
        if (lane == 0 && (per_thread || tid == 0) && x) atomicAdd(&a.st[k], x);
    }
}

template __global__ void weighted_run<0>(WeightedArgs);
template __global__ void weighted_run<1>(WeightedArgs);

}  // namespace bcx
