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
// out.  Each vertex's sum is formed by one thread (degree <= kLightDeg), one
// wavefront (<= kSeg) or kSeg-arc segments combined in segment order by the
// last segment to finish; no floating-point atomics, so results are bitwise
// reproducible.
#define BC_PLAIN_TU 1  // this engine's segment size: kSegPlain
#include "bc_common.h"

namespace bcx {

template <int MODE>
__device__ __forceinline__ double norm_sigma(const PlainArgs &a, int v, int sh) {
    if (MODE == 0) return (double)a.sig[v];
    return ldexp(as_f64(a.sig[v]), -sh);
}

// Top-down over arcs [a0, a1) of frontier vertex v (path count sv): claim
// unvisited neighbours, add sv to the neighbours on level l+1 (MODE 0).
template <int MODE>
__device__ __forceinline__ void plain_push_arcs(const PlainArgs &a, int l, unsigned long long sv, int a0, int a1,
                                                uint32_t qe, uint32_t hqb, unsigned long long &my_edges,
                                                unsigned long long &my_larcs, int &my_ovf, Stage &st, int &sn) {
    const int32_t *__restrict__ rp = a.g.row_ptr;
    const int32_t *__restrict__ col = a.g.col;
    Ctl *c = a.ctl;
    for (int eb = a0; eb < a1; eb += kWave) {
        const int e = eb + lane_id();
        bool newly = false;
        int w = 0, dw = 0;
        if (e < a1) {
            w = col[e];
            int dv = a.d[w];
            if (dv == -1) {
                const int old = atomicCAS(&a.d[w], -1, l + 1);
                newly = (old == -1);
                dv = newly ? l + 1 : old;
            }
            if (MODE == 0 && dv == l + 1) {
                const unsigned long long old = atomicAdd(&a.sig[w], sv);
                const unsigned long long nv = old + sv;
                if (nv < old || nv > a.sigma_limit) my_ovf = 1;
                ++my_larcs;
            }
            if (newly) {
                dw = rp[w + 1] - rp[w];
                my_edges += (unsigned)dw;
            }
        }
        stage_push(newly, w, dw, st, sn, c, a.queue, qe, (uint32_t)a.g.n, a.hq, hqb, &c->err, GroupArgs{});
    }
}

// Sum over arcs [a0, a1) of the values of neighbours u with d[u] == want:
// sigma (normalised by 2^-sh, MODE 1) or c.  Lane-strided, then a fixed
// butterfly: every lane returns the same bits.
__device__ __forceinline__ double plain_wave_sum(const PlainArgs &a, int a0, int a1, int want, bool use_chat, int sh,
                                                 unsigned long long &my_larcs) {
    const int32_t *__restrict__ col = a.g.col;
    double p = 0.0;
    for (int e = a0 + lane_id(); e < a1; e += kWave) {
        const int u = col[e];
        if (a.d[u] == want) {
            p += use_chat ? a.chat[u] : ldexp(as_f64(a.sig[u]), -sh);
            ++my_larcs;
        }
    }
    return wave_sum_f64(p);
}


// Exact 128-bit wavefront sum of (lo, hi) pairs; every lane gets the total.
__device__ __forceinline__ void wave_sum_u128(unsigned long long &lo, unsigned long long &hi) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long ol = shfl_u64(lo, lane ^ o), oh = shfl_u64(hi, lane ^ o);
        const unsigned long long nl = lo + ol;
        hi = hi + oh + ((nl < lo) ? 1ull : 0ull);
        lo = nl;
    }
}

// Transition helpers run by the last workgroup (all threads present).
template <int MODE>
__device__ __forceinline__ void plain_begin_source(const PlainArgs &a, Ctl *c, int64_t pos, float *lds, LevelFeatures *sf) {
    if (threadIdx.x == 0) {
        const int s = a.srcs[pos];
        a.d[s] = 0;
        a.sig[s] = MODE ? as_u64(1.0) : 1ull;
        a.queue[0] = s;
        a.level_off[0] = 0;
        a.level_off[1] = 1;
        a.shift[0] = 0;
        const int deg = a.g.row_ptr[s + 1] - a.g.row_ptr[s];
        a.hq.off[0] = 0;
        if (deg > kSeg) {  // heavy source: its level-0 push runs as segments
            a.hq.pos[0] = 0;
            a.hq.seg[0] = 0;
            a.hq.cnt[0] = 0;
            a.hq.off[1] = 1;
            a.hq.nseg[0] = n_segments(deg);
        } else {
            a.hq.off[1] = 0;
            a.hq.nseg[0] = 0;
        }
        c->next_hq = 0;
        c->pos = pos;
        c->level = 0;
        c->overflow = 0;
        c->next_qc = 0ull;
        c->next_edges = 0;
        c->visited_n = 1;
        c->visited_m = (unsigned long long)deg;
        c->prev_variant = V_PUSH_TPV;
        c->phase = PH_FWD;
        level_rec(a.lvl, 0).entries += 1;
        c->st_lane_entries += 1;
        sf->nf = 1.0f;
        sf->mf = (float)deg;
        sf->nu = (float)(a.g.n - 1);
        sf->mu = (float)((long long)a.g.nnz_lo - deg);
        sf->level = 0;
    }
    __syncthreads();
    int lbo;  // one source per entry: no summation options here
    const int v = choose_variant(a.p, c->policy, V_PUSH_TPV, *sf, (float)a.g.n, (float)a.g.nnz_lo, lds, &lbo);
    if (threadIdx.x == 0) c->variant = v;
}

template <int MODE>
__device__ __forceinline__ void plain_advance_level(const PlainArgs &a, Ctl *c, int l, uint32_t cnt, unsigned long long edges,
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
        c->next_qc = 0ull;
        c->next_edges = 0;
        c->prev_variant = c->variant;
        c->phase = PH_FWD;
    }
    __syncthreads();
    int lbo;
    const int v = choose_variant(a.p, c->policy, c->prev_variant, *sf, (float)a.g.n, (float)a.g.nnz_lo, lds, &lbo);
    if (threadIdx.x == 0) c->variant = v;
}

// After the forward of the current source ended with L levels.
__device__ __forceinline__ void plain_after_forward(const PlainArgs &a, Ctl *c, int L) {
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
    __shared__ int s_h0, s_h1, s_hseg, s_hqb;
    __shared__ unsigned s_nblk;
    __shared__ unsigned long long s_red[kSlots * kNCnt];
    __shared__ unsigned long long s_tot[kNCnt];
    __shared__ Stage s_stage[kWavesPerBlock];
    __shared__ float s_lds[2 * kMlpH + kMlpOut + 4];
    __shared__ LevelFeatures s_feat;
    Ctl *c = a.ctl;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) {
        s_phase = c->phase;
        s_level = c->level;
        s_variant = c->variant;
        s_dump = (c->dump_pos == c->pos && c->dump_state == 1) ? 1 : 0;
        const int l = s_level;
        s_qb = s_qe = s_qn = s_sh0 = s_sh1 = 0;
        s_h0 = s_h1 = s_hseg = s_hqb = 0;
        if (s_phase == PH_FWD || s_phase == PH_SIG || s_phase == PH_BWD) {
            s_qb = a.level_off[l];
            s_qe = a.level_off[l + 1];
            s_qn = (s_phase == PH_SIG) ? a.level_off[l + 2] : 0;
            s_sh0 = MODE ? a.shift[l] : 0;
            s_sh1 = (MODE && s_phase == PH_BWD && l + 1 < c->n_levels) ? a.shift[l + 1] : 0;
        } else if (s_phase == PH_FIN) {
            s_qe = (int)c->total_queued;
            // the next source's words are left to the last workgroup, which
            // sets them: a word stored by two workgroups of one launch ends
            // with whichever L2 writes it back last
            s_sh0 = c->pos + 1 < c->n_items ? a.srcs[c->pos + 1] : -1;
        }
        if (s_phase == PH_FWD) {
            if (s_variant == V_PULL) {  // static heavy vertices
                s_h0 = 0;
                s_h1 = a.g.n_heavy;
                s_hseg = a.g.hv_seg[a.g.n_heavy];
            } else {                    // heavy frontier vertices of level l
                s_h0 = a.hq.off[l];
                s_h1 = a.hq.off[l + 1];
                s_hseg = a.hq.nseg[l];
            }
            s_hqb = a.hq.off[l + 1];
        } else if (s_phase == PH_SIG) {
            s_h0 = a.hq.off[l + 1];
            s_h1 = a.hq.off[l + 2];
            s_hseg = a.hq.nseg[l + 1];
        } else if (s_phase == PH_BWD) {
            s_h0 = a.hq.off[l];
            s_h1 = a.hq.off[l + 1];
            s_hseg = a.hq.nseg[l];
        }
        // wavefront work items of this step -> workgroups taking part
        long long items = 1;
        const int cnt = s_qe - s_qb;
        if (s_phase == PH_FWD) {
            if (s_variant == V_PUSH_TPV) items = (cnt + kWave - 1) / kWave + s_hseg;
            else if (s_variant == V_PUSH_WPV) items = cnt + s_hseg;
            else items = (a.g.n + kWave - 1) / kWave + s_hseg;
        } else if (s_phase == PH_SIG) {
            items = (s_qn - s_qe + kWave - 1) / kWave + s_hseg;
        } else if (s_phase == PH_BWD) {
            items = (cnt + kWave - 1) / kWave + s_hseg;
        } else if (s_phase == PH_FIN) {
            items = (s_qe + kWave - 1) / kWave;
        } else if (s_phase == PH_DUMP_FWD) {
            items = (a.g.n + kWave - 1) / kWave;
        }
        s_nblk = active_blocks(items);
    }
    __syncthreads();
    const int phase = s_phase;
    if (phase == PH_DONE || phase == PH_IDLE) return;
    const unsigned nblk = s_nblk;
    const bool active = blockIdx.x < nblk;  // workgroups beyond nblk only count in

    const int gw = blockIdx.x * kWavesPerBlock + wid;
    const int nw = (int)nblk * kWavesPerBlock;
    const int l = s_level;
    const int n = a.g.n;
    const int32_t *__restrict__ rp = a.g.row_ptr;
    const int32_t *__restrict__ col = a.g.col;
    int32_t *d = a.d;
    unsigned long long *sig = a.sig;
    const int h0 = s_h0, h1 = s_h1, hseg = s_hseg;

    unsigned long long my_edges = 0, my_arcs = 0, my_larcs = 0;
    int my_ovf = 0, my_maxe = INT_MIN, my_mine = INT_MAX;

    if (!active) {
    } else if (phase == PH_FWD) {
        const int qb = s_qb, qe = s_qe, cnt = qe - qb;
        const int variant = s_variant;
        const uint32_t hqb = (uint32_t)s_hqb;
        Stage &st = s_stage[wid];
        int sn = 0;
        if (variant == V_PUSH_TPV || variant == V_PUSH_WPV) {
            const int n_light = variant == V_PUSH_TPV ? (cnt + kWave - 1) / kWave : cnt;
            const int total = n_light + hseg;
            for (int k = gw; k < total; k += nw) {
                const int it = k < hseg ? n_light + k : k - hseg;  // heavy segments first
                if (it >= n_light) {  // a segment of a heavy frontier vertex
                    const int t = it - n_light;
                    const int h = seg_owner(a.hq.seg, h0, h1, t);
                    const int s = t - a.hq.seg[h];
                    const int v = a.queue[a.hq.pos[h]];
                    const int a0 = rp[v] + s * kSeg, a1 = min(rp[v + 1], a0 + kSeg);
                    if (lane == 0) my_arcs += (unsigned)(a1 - a0);
                    const unsigned long long sv = MODE == 0 ? sig[v] : 0ull;
                    plain_push_arcs<MODE>(a, l, sv, a0, a1, (uint32_t)qe, hqb, my_edges, my_larcs, my_ovf, st, sn);
                } else if (variant == V_PUSH_WPV) {
                    const int v = a.queue[qb + it];
                    const int e0 = rp[v], e1 = rp[v + 1];
                    if (e1 - e0 > kSeg) continue;  // runs as segments
                    if (lane == 0) my_arcs += (unsigned)(e1 - e0);
                    const unsigned long long sv = MODE == 0 ? sig[v] : 0ull;
                    plain_push_arcs<MODE>(a, l, sv, e0, e1, (uint32_t)qe, hqb, my_edges, my_larcs, my_ovf, st, sn);
                } else {  // TPV: 64 frontier vertices per wavefront
                    const int i = it * kWave + lane;
                    const bool valid = i < cnt;
                    const int v = valid ? a.queue[qb + i] : 0;
                    const int e0 = valid ? rp[v] : 0;
                    const int deg = valid ? rp[v + 1] - e0 : 0;
                    const int len = deg <= kLightDeg ? deg : 0;
                    const unsigned long long sv = (MODE == 0 && valid) ? sig[v] : 0ull;
                    my_arcs += (unsigned)(deg <= kSeg ? deg : 0);
                    const int maxlen = wave_max_i(len);
                    for (int t = 0; t < maxlen; ++t) {
                        bool newly = false;
                        int w = 0, dw = 0;
                        if (t < len) {
                            w = col[e0 + t];
                            int dv = d[w];
                            if (dv == -1) {
                                const int old = atomicCAS(&d[w], -1, l + 1);
                                newly = (old == -1);
                                dv = newly ? l + 1 : old;
                            }
                            if (MODE == 0 && dv == l + 1) {
                                const unsigned long long old = atomicAdd(&sig[w], sv);
                                const unsigned long long nv = old + sv;
                                if (nv < old || nv > a.sigma_limit) my_ovf = 1;
                                ++my_larcs;
                            }
                            if (newly) {
                                dw = rp[w + 1] - rp[w];
                                my_edges += (unsigned)dw;
                            }
                        }
                        stage_push(newly, w, dw, st, sn, c, a.queue, (uint32_t)qe, (uint32_t)n, a.hq, hqb, &c->err, GroupArgs{});
                    }
                    // medium-degree vertices: the whole wavefront, one at a time
                    unsigned long long mm = __ballot(deg > kLightDeg && deg <= kSeg);
                    while (mm) {
                        const int j = __ffsll(mm) - 1;
                        mm &= mm - 1;
                        const int m0 = __shfl(e0, j), m1 = m0 + __shfl(deg, j);
                        plain_push_arcs<MODE>(a, l, shfl_u64(sv, j), m0, m1, (uint32_t)qe, hqb, my_edges, my_larcs,
                                              my_ovf, st, sn);
                    }
                }
            }
        } else {  // V_PULL: every unvisited vertex looks for neighbours on level l
            const int n_light = (n + kWave - 1) / kWave;
            const int total = n_light + hseg;
            for (int k = gw; k < total; k += nw) {
                const int it = k < hseg ? n_light + k : k - hseg;  // heavy segments first
                if (it >= n_light) {  // a segment of a heavy vertex
                    const int t = it - n_light;
                    const int h = seg_owner(a.g.hv_seg, h0, h1, t);
                    const int s = t - a.g.hv_seg[h];
                    const int w = a.g.hv_vtx[h];
                    const int dw0 = d[w];
                    // unvisited before this level (another segment may have
                    // claimed it during this step)
                    if (dw0 != -1 && dw0 != l + 1) continue;
                    const int a0 = rp[w] + s * kSeg, a1 = min(rp[w + 1], a0 + kSeg);
                    unsigned long long lo = 0, hi = 0;
                    bool found = false;
                    int scanned = 0;
                    for (int eb = a0; eb < a1; eb += kWave) {
                        const int e = eb + lane;
                        if (e < a1) {
                            const int u = col[e];
                            if (d[u] == l) {
                                found = true;
                                if (MODE == 0) {
                                    const unsigned long long x = sig[u];
                                    lo += x;
                                    hi += (lo < x) ? 1ull : 0ull;
                                    ++my_larcs;
                                }
                            }
                        }
                        scanned += min(kWave, a1 - eb);
                        if (MODE == 1 && __any(found)) break;
                    }
                    if (lane == 0) my_arcs += (unsigned)scanned;
                    const bool any = __any(found);
                    bool newly = false;
                    if (any) {
                        if (MODE == 0) {  // exact 128-bit sum of the segment, one atomic
                            wave_sum_u128(lo, hi);
                            if (lane == 0) {
                                const unsigned long long old = atomicAdd(&sig[w], lo);
                                const unsigned long long nv = old + lo;
                                if (hi != 0 || nv < old || nv > a.sigma_limit) my_ovf = 1;
                            }
                        }
                        if (lane == 0) newly = atomicCAS(&d[w], -1, l + 1) == -1;
                    }
                    const int deg = rp[w + 1] - rp[w];
                    if (newly) my_edges += (unsigned)deg;
                    stage_push(newly, w, deg, st, sn, c, a.queue, (uint32_t)qe, (uint32_t)n, a.hq, hqb, &c->err, GroupArgs{});
                    continue;
                }
                const int w = it * kWave + lane;
                const bool cand = (w < n) && d[w] == -1;
                const int e0 = cand ? rp[w] : 0;
                const int deg = cand ? rp[w + 1] - e0 : 0;
                const int len = deg <= kLightDeg ? deg : 0;
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
                                const unsigned long long x = sig[u];
                                lo += x;
                                hi += (lo < x) ? 1ull : 0ull;
                                ++my_larcs;
                            }
                            found = true;
                        }
                    }
                    if (MODE == 1 && !__any(t + 1 < len && !found)) break;
                }
                // medium-degree candidates: the whole wavefront, one at a time
                unsigned long long mm = __ballot(deg > kLightDeg && deg <= kSeg);
                while (mm) {
                    const int j = __ffsll(mm) - 1;
                    mm &= mm - 1;
                    const int m0 = __shfl(e0, j), m1 = m0 + __shfl(deg, j);
                    unsigned long long ml = 0, mh = 0;
                    bool mf = false;
                    for (int eb = m0; eb < m1; eb += kWave) {
                        const int e = eb + lane;
                        if (e < m1) {
                            const int u = col[e];
                            if (d[u] == l) {
                                mf = true;
                                if (MODE == 0) {
                                    const unsigned long long x = sig[u];
                                    ml += x;
                                    mh += (ml < x) ? 1ull : 0ull;
                                    ++my_larcs;
                                }
                            }
                        }
                        if (lane == 0) scanned += min(kWave, m1 - eb);
                        if (MODE == 1 && __any(mf)) break;
                    }
                    const bool fj = __any(mf);
                    if (MODE == 0) wave_sum_u128(ml, mh);
                    if (lane == j) {
                        found = fj;
                        lo = ml;
                        hi = mh;
                    }
                }
                my_arcs += (unsigned)scanned;
                const bool ok = found && deg <= kSeg;
                if (ok) {
                    d[w] = l + 1;
                    if (MODE == 0) {
                        sig[w] = lo;
                        if (hi != 0 || lo > a.sigma_limit) my_ovf = 1;
                    }
                    my_edges += (unsigned)deg;
                }
                stage_push(ok, w, deg, st, sn, c, a.queue, (uint32_t)qe, (uint32_t)n, a.hq, hqb, &c->err, GroupArgs{});
            }
        }
        stage_flush(st, sn, c, a.queue, (uint32_t)qe, (uint32_t)n, a.hq, hqb, &c->err, GroupArgs{});
    } else if (MODE == 1 && phase == PH_SIG) {
        // FP64 path counts of level l+1, pulled in CSR order
        const int qs = s_qe, cnt = s_qn - s_qe;
        const int sh = s_sh0;
        const int n_light = (cnt + kWave - 1) / kWave;
        const int total = n_light + hseg;
        for (int k = gw; k < total; k += nw) {
            const int it = k < hseg ? n_light + k : k - hseg;  // heavy segments first
            if (it >= n_light) {  // a segment of a heavy new vertex
                const int t = it - n_light;
                const int h = seg_owner(a.hq.seg, h0, h1, t);
                const int s = t - a.hq.seg[h];
                const int w = a.queue[a.hq.pos[h]];
                const int e0 = rp[w], e1 = rp[w + 1];
                const int a0 = e0 + s * kSeg, a1 = min(e1, a0 + kSeg);
                const double p = plain_wave_sum(a, a0, a1, l, false, sh, my_larcs);
                if (lane == 0) {
                    my_arcs += (unsigned)(a1 - a0);
                    part_store(&a.hq.part_lo[a.hq.seg[h] + s], as_u64(p));
                }
                const int ns = n_segments(e1 - e0);
                if (!seg_arrive(&a.hq.cnt[h], ns)) continue;
                if (lane == 0) {
                    double acc = 0.0;
                    for (int k = 0; k < ns; ++k) acc += as_f64(part_load(&a.hq.part_lo[a.hq.seg[h] + k]));
                    sig[w] = as_u64(acc);
                    if (acc > 0.0) {
                        int ex;
                        frexp(acc, &ex);
                        my_maxe = max(my_maxe, ex);
                        my_mine = min(my_mine, ex);
                    }
                    a.hq.cnt[h] = 0;
                }
                continue;
            }
            const int i = it * kWave + lane;
            const bool valid = i < cnt;
            const int w = valid ? a.queue[qs + i] : 0;
            const int e0 = valid ? rp[w] : 0;
            const int deg = valid ? rp[w + 1] - e0 : 0;
            const int len = deg <= kLightDeg ? deg : 0;
            const int maxlen = wave_max_i(len);
            double acc = 0.0;
            for (int t = 0; t < maxlen; ++t) {
                if (t < len) {
                    const int u = col[e0 + t];
                    if (d[u] == l) { acc += ldexp(as_f64(sig[u]), -sh); ++my_larcs; }
                }
            }
            my_arcs += (unsigned)(deg <= kSeg ? deg : 0);
            unsigned long long mm = __ballot(deg > kLightDeg && deg <= kSeg);
            while (mm) {
                const int j = __ffsll(mm) - 1;
                mm &= mm - 1;
                const int m0 = __shfl(e0, j), m1 = m0 + __shfl(deg, j);
                const double p = plain_wave_sum(a, m0, m1, l, false, sh, my_larcs);
                if (lane == j) acc = p;
            }
            if (valid && deg <= kSeg) {
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
        const int n_light = (cnt + kWave - 1) / kWave;
        const int total = n_light + hseg;
        for (int k = gw; k < total; k += nw) {
            const int it = k < hseg ? n_light + k : k - hseg;  // heavy segments first
            if (it >= n_light) {  // a segment of a heavy vertex of level l
                const int t = it - n_light;
                const int h = seg_owner(a.hq.seg, h0, h1, t);
                const int s = t - a.hq.seg[h];
                const int v = a.queue[a.hq.pos[h]];
                const int e0 = rp[v], e1 = rp[v + 1];
                const int a0 = e0 + s * kSeg, a1 = min(e1, a0 + kSeg);
                const double p = plain_wave_sum(a, a0, a1, l + 1, true, 0, my_larcs);
                if (lane == 0) {
                    my_arcs += (unsigned)(a1 - a0);
                    part_store(&a.hq.part_lo[a.hq.seg[h] + s], as_u64(p));
                }
                const int ns = n_segments(e1 - e0);
                if (!seg_arrive(&a.hq.cnt[h], ns)) continue;
                if (lane == 0) {
                    double acc = 0.0;
                    for (int k = 0; k < ns; ++k) acc += as_f64(part_load(&a.hq.part_lo[a.hq.seg[h] + k]));
                    const double sv = norm_sigma<MODE>(a, v, sh);
                    double delta = sv * acc;
                    if (MODE == 1) delta = ldexp(delta, -shn);
                    a.chat[v] = (1.0 + delta) / sv;
                    a.bc[v] += delta;
                    if (dump) a.dump_delta[v] = delta;
                    a.hq.cnt[h] = 0;
                }
                continue;
            }
            const int i = it * kWave + lane;
            const bool valid = i < cnt;
            const int v = valid ? a.queue[qb + i] : 0;
            const int e0 = valid ? rp[v] : 0;
            const int deg = valid ? rp[v + 1] - e0 : 0;
            const int len = deg <= kLightDeg ? deg : 0;
            const int maxlen = wave_max_i(len);
            double acc = 0.0;
            for (int t = 0; t < maxlen; ++t) {
                if (t < len) {
                    const int w = col[e0 + t];
                    if (d[w] == l + 1) { acc += a.chat[w]; ++my_larcs; }
                }
            }
            my_arcs += (unsigned)(deg <= kSeg ? deg : 0);
            unsigned long long mm = __ballot(deg > kLightDeg && deg <= kSeg);
            while (mm) {
                const int j = __ffsll(mm) - 1;
                mm &= mm - 1;
                const int m0 = __shfl(e0, j), m1 = m0 + __shfl(deg, j);
                const double p = plain_wave_sum(a, m0, m1, l + 1, true, 0, my_larcs);
                if (lane == j) acc = p;
            }
            if (valid && deg <= kSeg) {
                const double sv = norm_sigma<MODE>(a, v, sh);
                double delta = sv * acc;
                if (MODE == 1) delta = ldexp(delta, -shn);
                a.chat[v] = (1.0 + delta) / sv;
                a.bc[v] += delta;
                if (dump) a.dump_delta[v] = delta;
            }
        }
    } else if (phase == PH_FIN) {
        const int total = s_qe, next_src = s_sh0;
        for (int i = blockIdx.x * kBlock + tid; i < total; i += (int)nblk * kBlock) {
            const int v = a.queue[i];
            if (v == next_src) continue;
            d[v] = -1;
            sig[v] = 0ull;
        }
    } else if (phase == PH_DUMP_FWD) {
        for (int v = blockIdx.x * kBlock + tid; v < n; v += (int)nblk * kBlock) {
            a.dump_d[v] = d[v];
            a.dump_sig[v] = sig[v];
        }
        if (blockIdx.x == 0)
            for (int i = tid; i < c->n_levels; i += kBlock) a.dump_shift[i] = MODE ? a.shift[i] : 0;
    }

    // ---- per-launch counters into the slots; the last workgroup continues
    Counters cn;
    cn.v[SC_EDGES] = my_edges;
    cn.v[SC_ARCS] = my_arcs;
    cn.v[SC_LARCS] = my_larcs;
    cn.v[SC_OVF] = my_ovf ? 1ull : 0ull;
    if (my_maxe != INT_MIN) cn.exponent(my_maxe);
    if (my_mine != INT_MAX) cn.exponent(my_mine);
    if (!step_epilogue(c, cn, s_red, &s_last, active)) return;
    collect_slots(c, s_tot, s_red);

    // ---- the last workgroup advances the state machine
    int begin_pos = 0;
    int advance = 0;
    uint32_t cnt_next = 0;
    unsigned long long edges_next = 0;
    if (tid == 0) {
        c->st_steps += 1;
        c->st_arcs += s_tot[SC_ARCS];
        c->st_lane_arcs += s_tot[SC_LARCS];
        c->st_parcs[phase] += s_tot[SC_ARCS];
        c->st_plarcs[phase] += s_tot[SC_LARCS];
        c->st_ppairs[phase] += s_tot[SC_PAIRS];
        const unsigned long long now = wall_clock64();
        const unsigned long long dt = c->last_tick ? now - c->last_tick : 0ull;
        c->st_ticks[phase] += dt;
        if (phase == PH_FWD) c->st_vticks[s_variant] += dt;
        c->last_tick = now;
        const int rl = (phase == PH_FWD || phase == PH_BWD) ? l : (phase == PH_SIG ? l + 1 : -1);
        if (rl >= 0) {
            LevelRec &r = level_rec(a.lvl, rl);
            r.arcs += s_tot[SC_ARCS];
            r.ticks += dt;
            if (phase == PH_FWD) {
                r.visits += 1;
                r.var[s_variant] += 1;
            }
        }
        if (phase == PH_FWD) {
            const uint32_t cnt = (uint32_t)ld_agent(&c->next_qc);
            const unsigned long long nh = ld_agent(&c->next_hq);
            const int qe = a.level_off[l + 1];
            a.level_off[l + 2] = qe + (int)cnt;
            a.hq.off[l + 2] = a.hq.off[l + 1] + (int)(uint32_t)nh;
            a.hq.nseg[l + 1] = (int)(nh >> 32);
            c->next_hq = 0;
            c->st_fwd_levels += 1;
            c->st_var[s_variant] += 1;
            c->st_qentries += cnt;
            c->st_lane_entries += cnt;
            level_rec(a.lvl, l + 1).entries += cnt;
            if (MODE == 0 && s_tot[SC_OVF]) {
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
                c->next_edges = s_tot[SC_EDGES];  // kept for the level advance after the path counts
            } else {
                advance = 1;
                cnt_next = cnt;
                edges_next = s_tot[SC_EDGES];
            }
        } else if (phase == PH_SIG) {
            const bool any = s_tot[SC_MAXE] != 0;
            const int mx = (int)s_tot[SC_MAXE] - 4096, mn = 4096 - (int)s_tot[SC_MINE];
            int sh = 0;
            if (any && mx > kExpHigh) sh = mx - kExpTarget;
            if (any && mn - sh < kExpLow) c->err |= ERR_SIGMA_RANGE;
            a.shift[l + 1] = sh;
            advance = 1;
            cnt_next = (uint32_t)ld_agent(&c->next_qc);
            edges_next = c->next_edges;
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
