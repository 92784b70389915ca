// bc_plain.hip -- plain Brandes engine: one source at a time, the whole GPU
// working on each BFS level (paper, Section "Background": the level loop of
// the algorithm figure "Betweenness Centrality Algorithm", parallelised over
// the frontier's vertices and edges as that section describes).
//
// One kernel, plain_step<MODE>, executes the current phase of a device-side
// state machine (forward discover / path counts / backward / reset).  The
// last workgroup of each launch advances the machine, so a run is a stream of
// identical launches that the host can capture in a hipGraph.
//
// MODE 0: path counts in uint64.  Push levels add sigma with 64-bit atomics
//         (order-independent, exact); the atomic that carries past 2^64 - 1
//         (or the test limit) flags the source, which is then skipped and
//         redone in MODE 1.
// MODE 1: path counts in FP64, scaled by one power of two per level:
//         sigma(v) = raw(v) * 2^(E_l), E_l = shift_0 + ... + shift_l.  Counts
//         are pulled in CSR order after discovery, so every summation order
//         is fixed by the vertex alone.
//
// Backward (both modes): delta(v) = sigma(v) * sum over successors w of
// c(w), c(w) = (1 + delta(w)) / sigma(w) -- Eq. 2 with sigma(v) factored
// out.  Each vertex is written by one thread (or one wavefront for degree >
// kLightDeg); no floating-point atomics, so results are bitwise reproducible.
#include "bc_common.h"

namespace bcx {

template <int MODE>
__device__ __forceinline__ double norm_sigma(const PlainArgs &a, int v, int sh) {
    if (MODE == 0) return (double)a.sig[v];
    return ldexp(as_f64(a.sig[v]), -sh);
}

// Transition helpers run by the last workgroup (all threads present).
template <int MODE>
__device__ void plain_begin_source(PlainArgs &a, Ctl *c, int64_t pos, float *lds, LevelFeatures *sf) {
    if (threadIdx.x == 0) {
        const int s = a.srcs[pos];
        a.d[s] = 0;
        a.sig[s] = MODE ? as_u64(1.0) : 1ull;
        a.queue[0] = s;
        a.level_off[0] = 0;
        a.level_off[1] = 1;
        a.shift[0] = 0;
        const int deg = a.g.row_ptr[s + 1] - a.g.row_ptr[s];
        c->pos = pos;
        c->level = 0;
        c->overflow = 0;
        c->next_count = 0;
        c->next_edges = 0;
        c->visited_n = 1;
        c->visited_m = (unsigned long long)deg;
        c->prev_variant = V_PUSH_TPV;
        c->phase = PH_FWD;
        sf->nf = 1.0f;
        sf->mf = (float)deg;
        sf->nu = (float)(a.g.n - 1);
        sf->mu = (float)((long long)a.g.nnz_lo - deg);
        sf->level = 0;
    }
    __syncthreads();
    const int v = choose_variant(a.p, c->policy, V_PUSH_TPV, *sf, (float)a.g.n, (float)a.g.nnz_lo, lds);
    if (threadIdx.x == 0) c->variant = v;
}

template <int MODE>
__device__ void plain_advance_level(PlainArgs &a, Ctl *c, int l, uint32_t cnt, unsigned long long edges,
                                    float *lds, LevelFeatures *sf) {
    if (threadIdx.x == 0) {
        c->level = l + 1;
        c->visited_n += cnt;
        c->visited_m += edges;
        sf->nf = (float)cnt;
        sf->mf = (float)edges;
        sf->nu = (float)((long long)a.g.n - (long long)c->visited_n);
        sf->mu = (float)((long long)a.g.nnz_lo - (long long)c->visited_m);
        sf->level = l + 1;
        c->next_count = 0;
        c->next_edges = 0;
        c->prev_variant = c->variant;
        c->phase = PH_FWD;
    }
    __syncthreads();
    const int v = choose_variant(a.p, c->policy, c->prev_variant, *sf, (float)a.g.n, (float)a.g.nnz_lo, lds);
    if (threadIdx.x == 0) c->variant = v;
}

// After the forward of the current source ended with L levels.
__device__ __forceinline__ void plain_after_forward(PlainArgs &a, Ctl *c, int L) {
    c->n_levels = L;
    if ((unsigned long long)L > c->st_max_levels) c->st_max_levels = L;
    if (c->dump_pos == c->pos && c->dump_state == 0) {
        c->phase = PH_DUMP_FWD;
    } else if (L >= 2) {
        c->phase = PH_BWD;
        c->level = L - 1;
    } else {
        c->phase = PH_FIN;
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void plain_step(PlainArgs a) {
    __shared__ int s_phase, s_level, s_variant, s_last, s_qb, s_qe, s_qn, s_sh0, s_sh1, s_dump;
    __shared__ unsigned long long s_red[kWavesPerBlock];
    __shared__ float s_lds[2 * kMlpH + 4];
    __shared__ LevelFeatures s_feat;
    Ctl *c = a.ctl;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) {
        s_phase = c->phase;
        s_level = c->level;
        s_variant = c->variant;
        s_dump = (c->dump_pos == c->pos && c->dump_state == 1) ? 1 : 0;
        const int l = s_level;
        if (s_phase == PH_FWD || s_phase == PH_SIG || s_phase == PH_BWD) {
            s_qb = a.level_off[l];
            s_qe = a.level_off[l + 1];
            s_qn = (s_phase == PH_SIG) ? a.level_off[l + 2] : 0;
            s_sh0 = MODE ? a.shift[l] : 0;
            s_sh1 = (MODE && s_phase == PH_BWD && l + 1 < c->n_levels) ? a.shift[l + 1] : 0;
        } else if (s_phase == PH_FIN) {
            s_qb = 0;
            s_qe = (int)c->total_queued;
            s_qn = 0;
            s_sh0 = s_sh1 = 0;
        } else {
            s_qb = s_qe = s_qn = s_sh0 = s_sh1 = 0;
        }
    }
    __syncthreads();
    const int phase = s_phase;
    if (phase == PH_DONE || phase == PH_IDLE) return;

    const int gw = blockIdx.x * kWavesPerBlock + wid;
    const int nw = gridDim.x * kWavesPerBlock;
    const int l = s_level;
    const int n = a.g.n;
    const int32_t *__restrict__ rp = a.g.row_ptr;
    const int32_t *__restrict__ col = a.g.col;
    int32_t *d = a.d;
    unsigned long long *sig = a.sig;

    unsigned long long my_edges = 0, my_arcs = 0, my_larcs = 0;
    int my_ovf = 0, my_maxe = INT_MIN, my_mine = INT_MAX;

    if (phase == PH_FWD) {
        const int qb = s_qb, qe = s_qe, cnt = qe - qb;
        const int variant = s_variant;
        const uint32_t cap = (uint32_t)(n - qe);
        int32_t *nq = a.queue + qe;
        if (variant == V_PUSH_TPV) {
            for (int base = gw * kWave; base < cnt; base += nw * kWave) {
                const int i = base + lane;
                const bool valid = i < cnt;
                const int v = valid ? a.queue[qb + i] : 0;
                const int e0 = valid ? rp[v] : 0;
                const int len = valid ? rp[v + 1] - e0 : 0;
                const unsigned long long sv = (MODE == 0 && valid) ? sig[v] : 0ull;
                my_arcs += (unsigned)len;
                const int maxlen = wave_max_i(len);
                for (int t = 0; t < maxlen; ++t) {
                    bool newly = false;
                    int w = 0;
                    if (t < len) {
                        w = col[e0 + t];
                        int dw = d[w];
                        if (dw == -1) {
                            const int old = atomicCAS(&d[w], -1, l + 1);
                            newly = (old == -1);
                            dw = newly ? l + 1 : old;
                        }
                        if (MODE == 0 && dw == l + 1) {
                            const unsigned long long old = atomicAdd(&sig[w], sv);
                            const unsigned long long nv = old + sv;
                            if (nv < old || nv > a.sigma_limit) my_ovf = 1;
                            ++my_larcs;
                        }
                        if (newly) my_edges += (unsigned)(rp[w + 1] - rp[w]);
                    }
                    wave_append(newly, w, &c->next_count, nq, cap, &c->err);
                }
            }
        } else if (variant == V_PUSH_WPV) {
            for (int i = gw; i < cnt; i += nw) {
                const int v = a.queue[qb + i];
                const int e0 = rp[v], e1 = rp[v + 1];
                const unsigned long long sv = MODE == 0 ? sig[v] : 0ull;
                if (lane == 0) my_arcs += (unsigned)(e1 - e0);
                for (int eb = e0; eb < e1; eb += kWave) {
                    const int e = eb + lane;
                    bool newly = false;
                    int w = 0;
                    if (e < e1) {
                        w = col[e];
                        int dw = d[w];
                        if (dw == -1) {
                            const int old = atomicCAS(&d[w], -1, l + 1);
                            newly = (old == -1);
                            dw = newly ? l + 1 : old;
                        }
                        if (MODE == 0 && dw == l + 1) {
                            const unsigned long long old = atomicAdd(&sig[w], sv);
                            const unsigned long long nv = old + sv;
                            if (nv < old || nv > a.sigma_limit) my_ovf = 1;
                            ++my_larcs;
                        }
                        if (newly) my_edges += (unsigned)(rp[w + 1] - rp[w]);
                    }
                    wave_append(newly, w, &c->next_count, nq, cap, &c->err);
                }
            }
        } else {  // V_PULL: every unvisited vertex looks for neighbours on level l
            for (int base = gw * kWave; base < n; base += nw * kWave) {
                const int w = base + lane;
                const bool cand = (w < n) && d[w] == -1;
                const int e0 = cand ? rp[w] : 0;
                const int len = cand ? rp[w + 1] - e0 : 0;
                const int maxlen = wave_max_i(len);
                unsigned long long lo = 0, hi = 0;
                bool found = false;
                int scanned = 0;
                for (int t = 0; t < maxlen; ++t) {
                    const bool scan = (t < len) && !(MODE == 1 && found);
                    if (scan) {
                        ++scanned;
                        const int u = col[e0 + t];
                        if (d[u] == l) {
                            if (MODE == 0) {
                                const unsigned long long s = sig[u];
                                lo += s;
                                hi += (lo < s) ? 1ull : 0ull;
                                ++my_larcs;
                            }
                            found = true;
                        }
                    }
                    if (MODE == 1 && !__any(t + 1 < len && !found)) break;
                }
                my_arcs += (unsigned)scanned;
                if (found) {
                    d[w] = l + 1;
                    if (MODE == 0) {
                        sig[w] = lo;
                        if (hi != 0 || lo > a.sigma_limit) my_ovf = 1;
                    }
                    my_edges += (unsigned)len;
                }
                wave_append(found, w, &c->next_count, nq, cap, &c->err);
            }
        }
    } else if (MODE == 1 && phase == PH_SIG) {
        // FP64 path counts of level l+1, pulled in CSR order.
        const int qs = s_qe, cnt = s_qn - s_qe;
        const int sh = s_sh0;
        for (int base = gw * kWave; base < cnt; base += nw * kWave) {
            const int i = base + lane;
            const bool valid = i < cnt;
            const int w = valid ? a.queue[qs + i] : 0;
            const int e0 = valid ? rp[w] : 0;
            const int len = valid ? rp[w + 1] - e0 : 0;
            const bool heavy = len > kLightDeg;
            const int llen = heavy ? 0 : len;
            const int maxlen = wave_max_i(llen);
            double acc = 0.0;
            for (int t = 0; t < maxlen; ++t) {
                if (t < llen) {
                    const int u = col[e0 + t];
                    if (d[u] == l) { acc += ldexp(as_f64(sig[u]), -sh); ++my_larcs; }
                }
            }
            my_arcs += (unsigned)len;
            unsigned long long hm = __ballot(heavy);
            while (hm) {
                const int j = __ffsll(hm) - 1;
                hm &= hm - 1;
                const int h0 = __shfl(e0, j), h1 = h0 + __shfl(len, j);
                double p = 0.0;
                for (int e = h0 + lane; e < h1; e += kWave) {
                    const int u = col[e];
                    if (d[u] == l) { p += ldexp(as_f64(sig[u]), -sh); ++my_larcs; }
                }
                p = wave_sum_f64(p);
                if (lane == j) acc = p;
            }
            if (valid) {
                sig[w] = as_u64(acc);
                if (acc > 0.0) {
                    int ex;
                    frexp(acc, &ex);
                    my_maxe = max(my_maxe, ex);
                    my_mine = min(my_mine, ex);
                }
            }
        }
    } else if (phase == PH_BWD) {
        const int qb = s_qb, cnt = s_qe - s_qb;
        const int sh = s_sh0, shn = s_sh1;
        const bool dump = s_dump != 0;
        for (int base = gw * kWave; base < cnt; base += nw * kWave) {
            const int i = base + lane;
            const bool valid = i < cnt;
            const int v = valid ? a.queue[qb + i] : 0;
            const int e0 = valid ? rp[v] : 0;
            const int len = valid ? rp[v + 1] - e0 : 0;
            const bool heavy = len > kLightDeg;
            const int llen = heavy ? 0 : len;
            const int maxlen = wave_max_i(llen);
            double acc = 0.0;
            for (int t = 0; t < maxlen; ++t) {
                if (t < llen) {
                    const int w = col[e0 + t];
                    if (d[w] == l + 1) { acc += a.chat[w]; ++my_larcs; }
                }
            }
            my_arcs += (unsigned)len;
            unsigned long long hm = __ballot(heavy);
            while (hm) {
                const int j = __ffsll(hm) - 1;
                hm &= hm - 1;
                const int h0 = __shfl(e0, j), h1 = h0 + __shfl(len, j);
                double p = 0.0;
                for (int e = h0 + lane; e < h1; e += kWave) {
                    const int w = col[e];
                    if (d[w] == l + 1) { p += a.chat[w]; ++my_larcs; }
                }
                p = wave_sum_f64(p);
                if (lane == j) acc = p;
            }
            if (valid) {
                const double sv = norm_sigma<MODE>(a, v, sh);
                double delta = sv * acc;
                if (MODE == 1) delta = ldexp(delta, -shn);
                a.chat[v] = (1.0 + delta) / sv;
                a.bc[v] += delta;
                if (dump) a.dump_delta[v] = delta;
            }
        }
    } else if (phase == PH_FIN) {
        const int total = s_qe;
        for (int i = blockIdx.x * kBlock + tid; i < total; i += gridDim.x * kBlock) {
            const int v = a.queue[i];
            d[v] = -1;
            sig[v] = 0ull;
        }
    } else if (phase == PH_DUMP_FWD) {
        for (int v = blockIdx.x * kBlock + tid; v < n; v += gridDim.x * kBlock) {
            a.dump_d[v] = d[v];
            a.dump_sig[v] = sig[v];
        }
        if (blockIdx.x == 0)
            for (int i = tid; i < c->n_levels; i += kBlock) a.dump_shift[i] = MODE ? a.shift[i] : 0;
    }

    // ---- per-launch statistics and level counters
    {
        const unsigned long long e = block_sum_u64(my_edges, s_red);
        if (tid == 0 && e) atomicAdd(&c->next_edges, e);
        const unsigned long long ar = block_sum_u64(my_arcs, s_red);
        if (tid == 0 && ar) atomicAdd(&c->st_arcs, ar);
        const unsigned long long la = block_sum_u64(my_larcs, s_red);
        if (tid == 0 && la) atomicAdd(&c->st_lane_arcs, la);
        if (MODE == 0 && phase == PH_FWD) {
            if (__any(my_ovf) && lane == 0) atomicOr(&c->overflow, 1);
        }
        if (MODE == 1 && phase == PH_SIG) {
            const int mx = wave_max_i(my_maxe), mn = wave_min_i(my_mine);
            if (lane == 0) {
                if (mx != INT_MIN) atomicMax(&c->maxexp, mx);
                if (mn != INT_MAX) atomicMin(&c->minexp, mn);
            }
        }
    }

    if (!last_block_arrive(&c->blocks_done, &s_last)) return;

    // ---- the last workgroup advances the state machine
    int begin_pos = 0;
    int advance = 0;
    uint32_t cnt_next = 0;
    unsigned long long edges_next = 0;
    if (tid == 0) {
        c->blocks_done = 0;
        c->st_steps += 1;
        if (phase == PH_FWD) {
            const uint32_t cnt = ld_agent(&c->next_count);
            const int qe = a.level_off[l + 1];
            a.level_off[l + 2] = qe + (int)cnt;
            c->st_fwd_levels += 1;
            c->st_var[s_variant] += 1;
            c->st_qentries += cnt;
            if (MODE == 0 && ld_agent(&c->overflow)) {
                const uint32_t k = c->n_ovf;
                if (k < a.ovf_cap) a.ovf_list[k] = c->pos;
                else c->err |= ERR_OVF_CAP;
                c->n_ovf = k + 1;
                c->total_queued = (uint32_t)(qe + (int)cnt);
                c->phase = PH_FIN;
            } else if (cnt == 0) {
                c->total_queued = (uint32_t)qe;
                plain_after_forward(a, c, l + 1);
            } else if (MODE == 1) {
                c->phase = PH_SIG;
                c->maxexp = INT_MIN;
                c->minexp = INT_MAX;
            } else {
                advance = 1;
                cnt_next = cnt;
                edges_next = ld_agent(&c->next_edges);
            }
        } else if (phase == PH_SIG) {
            const int mx = ld_agent(&c->maxexp), mn = ld_agent(&c->minexp);
            int sh = 0;
            if (mx != INT_MIN && mx > 960) sh = mx - 900;
            if (mn != INT_MAX && mn - sh < -1000) c->err |= ERR_SIGMA_RANGE;
            a.shift[l + 1] = sh;
            advance = 1;
            cnt_next = ld_agent(&c->next_count);
            edges_next = ld_agent(&c->next_edges);
        } else if (phase == PH_BWD) {
            if (l - 1 >= 1) {
                c->level = l - 1;
            } else {
                c->total_queued = (uint32_t)a.level_off[c->n_levels];
                c->phase = PH_FIN;
            }
        } else if (phase == PH_DUMP_FWD) {
            c->dump_state = 1;
            const int L = c->n_levels;
            if (L >= 2) {
                c->phase = PH_BWD;
                c->level = L - 1;
            } else {
                c->phase = PH_FIN;
            }
        } else if (phase == PH_FIN) {
            if (c->dump_state == 1 && c->dump_pos == c->pos) c->dump_state = 2;
            const int64_t next = c->pos + 1;
            c->pos = next;
            if (next < c->n_items) begin_pos = 1;
            else c->phase = PH_DONE;
        }
        s_qb = begin_pos;
        s_qe = advance;
        s_qn = (int)cnt_next;
        s_red[0] = edges_next;
    }
    __syncthreads();
    if (s_qb == 1) plain_begin_source<MODE>(a, c, c->pos, s_lds, &s_feat);
    else if (s_qe == 1) plain_advance_level<MODE>(a, c, l, (uint32_t)s_qn, s_red[0], s_lds, &s_feat);
}

template __global__ void plain_step<0>(PlainArgs);
template __global__ void plain_step<1>(PlainArgs);

}  // namespace bcx
