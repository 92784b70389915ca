// bc_batched.hip -- batched Brandes engine: up to 64 sources traversed
// together, one wavefront lane per source.
//
// The paper's forward phase exploits that BC needs a traversal from many
// sources (Section "Introduction" and "Comparison with Totem": one-time work
// amortised over many sources).  Here that multi-source property becomes the
// batching axis: the frontier of a level is one list of vertices, each with a
// 64-bit lane mask (bit k = the vertex is on this level for source k), so a
// vertex's adjacency is read once per level for all sources that reach it
// there.  Per-source state lives in vertex-major slabs [n][64] (sigma, then
// delta; and c = (1 + delta) / sigma), so the 64 lanes of a wavefront touch
// one contiguous 512-byte row.
//
// Per level l (Algorithm "Betweenness Centrality Algorithm", forward loop):
//   PH_FWD  discover: visited/next words, push (thread or wavefront per
//           frontier vertex, 64-bit atomicOr) or pull (thread per unvisited
//           vertex, early exit once every needed lane is found).
//   PH_SIG  sigma_k(w) = sum over neighbours u of w on level l in lane k of
//           sigma_k(u), in CSR order, one wavefront per new vertex.  uint64
//           with the carry kept (exact overflow test); scaled FP64 in mode 1.
// Backward, per level l = L-1 .. 1 (same figure, backward loop; Eq. 2):
//   PH_BWD  delta_k(v) = sigma_k(v) * sum over w on level l+1 of c_k(w).
//   PH_BC   BC[v] += delta_k(v) for k = 0 .. 63 in order (source-list
//           order), then the visited words are cleared.
// Frontier words carry a level tag so stale entries never need clearing.
#include "bc_common.h"

namespace bcx {

__device__ __forceinline__ unsigned long long shfl_u64(unsigned long long x, int src) {
    const unsigned lo = __shfl((unsigned)x, src), hi = __shfl((unsigned)(x >> 32), src);
    return ((unsigned long long)hi << 32) | lo;
}

template <int MODE>
__device__ void batch_begin(BatchArgs &a, Ctl *c, int64_t b, float *lds, LevelFeatures *sf, int *s_lsrc,
                            int *s_cnt, unsigned long long *s_tmp) {
    const int t = threadIdx.x;
    const int64_t start = a.batch_start[b], end = a.batch_start[b + 1];
    const int lanes = (int)(end - start);
    // Tags of the previous batch end at epoch_b + n_levels; start above them.
    const uint32_t epoch = c->epoch_b + (uint32_t)c->n_levels + 1u;
    __syncthreads();
    if (t == 0) *s_cnt = 0;
    if (t < kLanes) {
        const int s = t < lanes ? a.srcs[start + t] : -1;
        s_lsrc[t] = s;
        a.lane_src[t] = s;
    }
    __syncthreads();
    if (t < lanes) {
        const int s = s_lsrc[t];
        unsigned long long m = 0;
        bool leader = true;
        for (int k = 0; k < lanes; ++k) {
            if (s_lsrc[k] == s) {
                m |= 1ull << k;
                if (k < t) leader = false;
            }
        }
        a.sig[(size_t)s * kLanes + t] = MODE ? as_u64(1.0) : 1ull;
        if (MODE) a.shift[t] = 0;
        if (leader) {
            const int j = atomicAdd(s_cnt, 1);
            a.lq_vtx[j] = s;
            a.lq_mask[j] = m;
            a.vn[s].vis = m;
            Tagged tg;
            tg.mask = m;
            tg.tag = epoch;
            tg.pad = 0;
            a.fw0[s] = tg;
            s_tmp[j] = (unsigned long long)(a.g.row_ptr[s + 1] - a.g.row_ptr[s]);
        }
    } else if (MODE && t < kLanes) {
        a.shift[t] = 0;
    }
    __syncthreads();
    if (t == 0) {
        const int cnt = *s_cnt;
        unsigned long long mf = 0;
        for (int j = 0; j < cnt; ++j) mf += s_tmp[j];
        c->epoch = epoch;
        c->pos = b;
        c->lanes = lanes;
        c->lane_mask = lanes >= 64 ? ~0ull : ((1ull << lanes) - 1ull);
        c->active = c->lane_mask;
        c->dead = 0;
        c->ovf_lanes = 0;
        c->range_lo = a.batch_lo[b];
        c->range_hi = a.batch_hi[b];
        c->range_arcs = (unsigned long long)(a.g.row_ptr[c->range_hi] - a.g.row_ptr[c->range_lo]);
        c->range_nodeg = (unsigned long long)(c->range_hi - c->range_lo);
        c->full_n = 0;
        c->full_m = 0;
        c->level = 0;
        c->n_levels = 0;
        a.level_off[0] = 0;
        a.level_off[1] = cnt;
        c->next_count = 0;
        c->next_edges = 0;
        c->next_active = 0;
        c->prev_variant = V_PUSH_TPV;
        c->phase = PH_FWD;
        c->st_batches += 1;
        const int64_t dp = c->dump_pos;
        c->dump_lane = (dp >= start && dp < end && c->dump_state == 0) ? (int)(dp - start) : -1;
        sf->nf = (float)cnt;
        sf->mf = (float)mf;
        sf->nu = (float)c->range_nodeg;
        sf->mu = (float)c->range_arcs;
        sf->level = 0;
    }
    __syncthreads();
    const int v = choose_variant(a.p, c->policy, V_PUSH_TPV, *sf, (float)(c->range_hi - c->range_lo),
                                 (float)c->range_arcs, lds);
    if (t == 0) c->variant = v;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void batch_step(BatchArgs a) {
    __shared__ int s_phase, s_level, s_variant, s_last, s_qb, s_qe, s_qn, s_L, s_lo, s_hi, s_dlane, s_cnt;
    __shared__ uint32_t s_epoch, s_epoch_b;
    __shared__ unsigned long long s_active, s_dead, s_lmask;
    __shared__ unsigned long long s_red[kWavesPerBlock];
    __shared__ unsigned long long s_tmp[kLanes];
    __shared__ int s_lsrc[kLanes];
    __shared__ float s_lds[2 * kMlpH + 4];
    __shared__ LevelFeatures s_feat;
    Ctl *c = a.ctl;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    if (tid == 0) {
        s_phase = c->phase;
        s_level = c->level;
        s_variant = c->variant;
        s_epoch = c->epoch;
        s_epoch_b = c->epoch_b;
        s_active = c->active & ~c->dead;
        s_dead = c->dead;
        s_lmask = c->lane_mask;
        s_L = c->n_levels;
        s_lo = c->range_lo;
        s_hi = c->range_hi;
        s_dlane = c->dump_lane;
        const int l = s_level;
        if (s_phase == PH_FWD || s_phase == PH_SIG || s_phase == PH_BWD) {
            s_qb = a.level_off[l];
            s_qe = a.level_off[l + 1];
            s_qn = (s_phase == PH_SIG) ? a.level_off[l + 2] : 0;
        } else if (s_phase == PH_DUMP_FWD || s_phase == PH_DUMP_BWD) {
            s_qb = 0;
            s_qe = a.level_off[s_L];
            s_qn = 0;
        } else {
            s_qb = s_qe = s_qn = 0;
        }
    }
    if (tid < kLanes) s_lsrc[tid] = a.lane_src[tid];
    __syncthreads();
    const int phase = s_phase;
    if (phase == PH_DONE || phase == PH_IDLE) return;

    const int gw = blockIdx.x * kWavesPerBlock + wid;
    const int nw = gridDim.x * kWavesPerBlock;
    const int l = s_level;
    const int32_t *__restrict__ rp = a.g.row_ptr;
    const int32_t *__restrict__ col = a.g.col;
    Tagged *fw_cur = (l & 1) ? a.fw1 : a.fw0;
    Tagged *fw_nxt = (l & 1) ? a.fw0 : a.fw1;

    unsigned long long my_edges = 0, my_arcs = 0, my_larcs = 0, my_act = 0, my_ovf = 0;
    unsigned long long my_full_n = 0, my_full_m = 0;
    int my_maxe = INT_MIN, my_mine = INT_MAX;

    if (phase == PH_FWD) {
        const int qb = s_qb, qe = s_qe, cnt = qe - qb;
        const uint32_t T = s_epoch + (uint32_t)l;
        const unsigned long long act = s_active;
        const uint32_t cap = a.lq_cap - (uint32_t)qe;
        int32_t *nq = a.lq_vtx + qe;
        const int variant = s_variant;
        if (variant == V_PUSH_TPV) {
            for (int base = gw * kWave; base < cnt; base += nw * kWave) {
                const int i = base + lane;
                const bool valid = i < cnt;
                const int u = valid ? a.lq_vtx[qb + i] : 0;
                const unsigned long long f = valid ? (a.lq_mask[qb + i] & act) : 0ull;
                const int e0 = f ? rp[u] : 0;
                const int len = f ? rp[u + 1] - e0 : 0;
                my_arcs += (unsigned)len;
                const int maxlen = wave_max_i(len);
                for (int t = 0; t < maxlen; ++t) {
                    bool newly = false;
                    int w = 0;
                    if (t < len) {
                        w = col[e0 + t];
                        const VisNext x = a.vn[w];
                        const unsigned long long add = f & ~x.vis & ~x.nxt;
                        if (add) {
                            const unsigned long long old = atomicOr(&a.vn[w].nxt, add);
                            newly = (old == 0ull);
                        }
                        if (newly) my_edges += (unsigned)(rp[w + 1] - rp[w]);
                    }
                    wave_append(newly, w, &c->next_count, nq, cap, &c->err);
                }
            }
        } else if (variant == V_PUSH_WPV) {
            for (int i = gw; i < cnt; i += nw) {
                const int u = a.lq_vtx[qb + i];
                const unsigned long long f = a.lq_mask[qb + i] & act;
                if (!f) continue;
                const int e0 = rp[u], e1 = rp[u + 1];
                if (lane == 0) my_arcs += (unsigned)(e1 - e0);
                for (int eb = e0; eb < e1; eb += kWave) {
                    const int e = eb + lane;
                    bool newly = false;
                    int w = 0;
                    if (e < e1) {
                        w = col[e];
                        const VisNext x = a.vn[w];
                        const unsigned long long add = f & ~x.vis & ~x.nxt;
                        if (add) {
                            const unsigned long long old = atomicOr(&a.vn[w].nxt, add);
                            newly = (old == 0ull);
                        }
                        if (newly) my_edges += (unsigned)(rp[w + 1] - rp[w]);
                    }
                    wave_append(newly, w, &c->next_count, nq, cap, &c->err);
                }
            }
        } else {  // V_PULL over the batch's vertex range
            const int lo = s_lo, span = s_hi - s_lo;
            for (int base = gw * kWave; base < span; base += nw * kWave) {
                const int w = lo + base + lane;
                const bool valid = base + lane < span;
                const unsigned long long vis = valid ? a.vn[w].vis : ~0ull;
                const unsigned long long need = act & ~vis;
                const int e0 = need ? rp[w] : 0;
                const int len = need ? rp[w + 1] - e0 : 0;
                const int maxlen = wave_max_i(len);
                unsigned long long got = 0;
                int scanned = 0;
                for (int t = 0; t < maxlen; ++t) {
                    if (t < len && got != need) {
                        ++scanned;
                        const int u = col[e0 + t];
                        const Tagged F = fw_cur[u];
                        if (F.tag == T) got |= F.mask & need;
                    }
                    if (!__any(t + 1 < len && got != need)) break;
                }
                my_arcs += (unsigned)scanned;
                if (got) {
                    a.vn[w].nxt = got;
                    my_edges += (unsigned)len;
                }
                wave_append(got != 0ull, w, &c->next_count, nq, cap, &c->err);
            }
        }
    } else if (phase == PH_SIG) {
        // path counts of the new level, one wavefront per vertex, lane = source
        const int qs = s_qe, cnt = s_qn - s_qe;
        const uint32_t T = s_epoch + (uint32_t)l;
        const int sh = MODE ? a.shift[(size_t)l * kLanes + lane] : 0;
        const unsigned long long lmask = s_lmask;
        for (int i = gw; i < cnt; i += nw) {
            const int w = a.lq_vtx[qs + i];
            const VisNext x = a.vn[w];
            const unsigned long long m = x.nxt;
            const int e0 = rp[w], e1 = rp[w + 1];
            unsigned long long lo = 0, hi = 0;
            double accd = 0.0;
            for (int eb = e0; eb < e1; eb += kWave) {
                const int e = eb + lane;
                int uj = 0;
                unsigned long long xj = 0;
                if (e < e1) {
                    uj = col[e];
                    const Tagged F = fw_cur[uj];
                    if (F.tag == T) xj = F.mask & m;
                }
                unsigned long long bal = __ballot(xj != 0ull);
                while (bal) {
                    const int j = __ffsll(bal) - 1;
                    bal &= bal - 1;
                    const int u = __shfl(uj, j);
                    const unsigned long long xm = shfl_u64(xj, j);
                    if ((xm >> lane) & 1ull) {
                        const unsigned long long val = a.sig[(size_t)u * kLanes + lane];
                        if (MODE == 0) {
                            lo += val;
                            hi += (lo < val) ? 1ull : 0ull;
                        } else {
                            accd += ldexp(as_f64(val), -sh);
                        }
                    }
                    if (lane == 0) my_larcs += (unsigned)__popcll(xm);
                }
            }
            if (lane == 0) my_arcs += (unsigned)(e1 - e0);
            const bool mine = (m >> lane) & 1ull;
            if (mine) {
                if (MODE == 0) {
                    a.sig[(size_t)w * kLanes + lane] = lo;
                    if (hi != 0 || lo > a.sigma_limit) my_ovf |= 1ull << lane;
                } else {
                    a.sig[(size_t)w * kLanes + lane] = as_u64(accd);
                    if (accd > 0.0) {
                        int ex;
                        frexp(accd, &ex);
                        my_maxe = max(my_maxe, ex);
                        my_mine = min(my_mine, ex);
                    }
                }
            }
            if (lane == 0) {
                VisNext y;
                y.vis = x.vis | m;
                y.nxt = 0ull;
                a.vn[w] = y;
                Tagged tg;
                tg.mask = m;
                tg.tag = T + 1u;
                tg.pad = 0;
                fw_nxt[w] = tg;
                a.lq_mask[qs + i] = m;
                const unsigned deg = (unsigned)(e1 - e0);
                my_edges += deg;
                my_act |= m;
                if ((y.vis & lmask) == lmask) {
                    my_full_n += 1;
                    my_full_m += deg;
                }
            }
        }
    } else if (phase == PH_BWD) {
        const int qb = s_qb, cnt = s_qe - s_qb;
        const uint32_t TB = s_epoch_b + (uint32_t)l;
        Tagged *fb_cur = fw_cur;  // written with this level's tag
        Tagged *fb_nxt = fw_nxt;  // read: level l+1's tag
        const unsigned long long dead = s_dead;
        const int sh = MODE ? a.shift[(size_t)l * kLanes + lane] : 0;
        const int shn = (MODE && l + 1 < s_L) ? a.shift[(size_t)(l + 1) * kLanes + lane] : 0;
        for (int i = gw; i < cnt; i += nw) {
            const int v = a.lq_vtx[qb + i];
            const unsigned long long M = a.lq_mask[qb + i] & ~dead;
            const int e0 = rp[v], e1 = rp[v + 1];
            double acc = 0.0;
            if (M) {
                for (int eb = e0; eb < e1; eb += kWave) {
                    const int e = eb + lane;
                    int wj = 0;
                    unsigned long long xj = 0;
                    if (e < e1) {
                        wj = col[e];
                        const Tagged F = fb_nxt[wj];
                        if (F.tag == TB + 1u) xj = F.mask & M;
                    }
                    unsigned long long bal = __ballot(xj != 0ull);
                    while (bal) {
                        const int j = __ffsll(bal) - 1;
                        bal &= bal - 1;
                        const int w = __shfl(wj, j);
                        const unsigned long long xm = shfl_u64(xj, j);
                        if ((xm >> lane) & 1ull) acc += a.chat[(size_t)w * kLanes + lane];
                        if (lane == 0) my_larcs += (unsigned)__popcll(xm);
                    }
                }
                if (lane == 0) my_arcs += (unsigned)(e1 - e0);
                if ((M >> lane) & 1ull) {
                    const size_t at = (size_t)v * kLanes + lane;
                    const unsigned long long raw = a.sig[at];
                    const double sv = MODE ? ldexp(as_f64(raw), -sh) : (double)raw;
                    double delta = sv * acc;
                    if (MODE) delta = ldexp(delta, -shn);
                    a.chat[at] = (1.0 + delta) / sv;
                    a.sig[at] = as_u64(delta);
                }
            }
            if (lane == 0) {
                Tagged tg;
                tg.mask = M;
                tg.tag = TB;
                tg.pad = 0;
                fb_cur[v] = tg;
            }
        }
    } else if (phase == PH_BC) {
        // dependencies -> BC in source-list order, then clear the visited words
        const int lo = s_lo, span = s_hi - s_lo;
        const unsigned long long keep = s_lmask & ~s_dead;
        for (int i = blockIdx.x * kBlock + tid; i < span; i += gridDim.x * kBlock) {
            const int w = lo + i;
            const VisNext x = a.vn[w];
            unsigned long long vis = x.vis & keep;
            if (vis) {
                double b = a.bc[w];
                while (vis) {
                    const int k = __ffsll(vis) - 1;
                    vis &= vis - 1;
                    if (s_lsrc[k] != w) b += as_f64(a.sig[(size_t)w * kLanes + k]);
                }
                a.bc[w] = b;
            }
            if (x.vis | x.nxt) {
                VisNext z;
                z.vis = 0ull;
                z.nxt = 0ull;
                a.vn[w] = z;
            }
        }
    } else if (phase == PH_DUMP_FWD || phase == PH_DUMP_BWD) {
        const int k = s_dlane;
        const int L = s_L;
        const int total = s_qe;
        for (int j = blockIdx.x * kBlock + tid; j < total; j += gridDim.x * kBlock) {
            if (!((a.lq_mask[j] >> k) & 1ull)) continue;
            int lo = 0, hi = L;  // level of entry j: level_off[lvl] <= j < level_off[lvl+1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (a.level_off[mid] <= j) lo = mid;
                else hi = mid;
            }
            const int v = a.lq_vtx[j];
            const unsigned long long val = a.sig[(size_t)v * kLanes + k];
            if (phase == PH_DUMP_FWD) {
                a.dump_d[v] = lo;
                a.dump_sig[v] = val;
            } else if (lo >= 1) {
                a.dump_delta[v] = as_f64(val);
            }
        }
        if (phase == PH_DUMP_FWD && blockIdx.x == 0)
            for (int i = tid; i < L; i += kBlock) a.dump_shift[i] = MODE ? a.shift[(size_t)i * kLanes + k] : 0;
    }

    // ---- per-launch statistics and level counters
    {
        const unsigned long long e = block_sum_u64(my_edges, s_red);
        if (tid == 0 && e) atomicAdd(&c->next_edges, e);
        const unsigned long long ar = block_sum_u64(my_arcs, s_red);
        if (tid == 0 && ar) atomicAdd(&c->st_arcs, ar);
        const unsigned long long la = block_sum_u64(my_larcs, s_red);
        if (tid == 0 && la) atomicAdd(&c->st_lane_arcs, la);
        if (phase == PH_SIG) {
            const unsigned long long fn = block_sum_u64(my_full_n, s_red);
            if (tid == 0 && fn) atomicAdd(&c->full_n, fn);
            const unsigned long long fm = block_sum_u64(my_full_m, s_red);
            if (tid == 0 && fm) atomicAdd(&c->full_m, fm);
            const unsigned long long ac = wave_or_u64(my_act);
            if (lane == 0 && ac) atomicOr(&c->next_active, ac);
            if (MODE == 0) {
                const unsigned long long ov = wave_or_u64(my_ovf);
                if (lane == 0 && ov) atomicOr(&c->ovf_lanes, ov);
            } else {
                if (my_maxe != INT_MIN) atomicMax(&a.maxexp[lane], my_maxe);
                if (my_mine != INT_MAX) atomicMin(&a.maxexp[kLanes + lane], my_mine);
            }
        }
    }

    if (!last_block_arrive(&c->blocks_done, &s_last)) return;

    // ---- the last workgroup advances the state machine
    int action = 0;  // 1 = begin batch, 2 = advance level
    if (tid == 0) {
        c->blocks_done = 0;
        c->st_steps += 1;
        if (phase == PH_FWD) {
            const uint32_t cnt = ld_agent(&c->next_count);
            const int qe = a.level_off[l + 1];
            c->st_fwd_levels += 1;
            c->st_var[s_variant] += 1;
            c->st_qentries += cnt;
            if (cnt == 0) {
                const int L = l + 1;
                c->n_levels = L;
                // backward tags epoch_b + 1 .. epoch_b + L lie above every forward tag
                c->epoch_b = c->epoch + (uint32_t)L + 1u;
                if ((unsigned long long)L > c->st_max_levels) c->st_max_levels = L;
                if (c->dump_lane >= 0 && !((c->dead >> c->dump_lane) & 1ull)) c->phase = PH_DUMP_FWD;
                else if (L >= 2) { c->phase = PH_BWD; c->level = L - 1; }
                else c->phase = PH_BC;
            } else if (l + 2 >= a.max_levels) {
                c->err |= ERR_LEVEL_CAP;
                c->phase = PH_DONE;
            } else {
                a.level_off[l + 2] = qe + (int)cnt;
                c->phase = PH_SIG;
            }
        } else if (phase == PH_SIG) {
            action = 2;
        } else if (phase == PH_BWD) {
            if (l - 1 >= 1) {
                c->level = l - 1;
            } else if (c->dump_lane >= 0 && c->dump_state == 1) {
                c->phase = PH_DUMP_BWD;
            } else {
                c->phase = PH_BC;
            }
        } else if (phase == PH_DUMP_FWD) {
            c->dump_state = 1;
            const int L = c->n_levels;
            if (L >= 2) { c->phase = PH_BWD; c->level = L - 1; }
            else c->phase = PH_DUMP_BWD;
        } else if (phase == PH_DUMP_BWD) {
            c->dump_state = 2;
            c->phase = PH_BC;
        } else if (phase == PH_BC) {
            const int64_t next = c->pos + 1;
            c->pos = next;
            if (next < c->n_items) action = 1;
            else c->phase = PH_DONE;
        }
        s_cnt = action;
    }
    __syncthreads();
    action = s_cnt;
    if (action == 1) {
        batch_begin<MODE>(a, c, c->pos, s_lds, &s_feat, s_lsrc, &s_qn, s_tmp);
    } else if (action == 2) {
        // finish level l+1: lane deaths, FP64 shifts, features, policy
        if (tid == 0) {
            const unsigned long long ovf = ld_agent(&c->ovf_lanes) & ~c->dead;
            if (ovf) {
                unsigned long long o = ovf;
                const int64_t start = a.batch_start[c->pos];
                while (o) {
                    const int k = __ffsll(o) - 1;
                    o &= o - 1;
                    const uint32_t q = c->n_ovf;
                    if (q < a.ovf_cap) a.ovf_list[q] = start + k;
                    else c->err |= ERR_OVF_CAP;
                    c->n_ovf = q + 1;
                }
                c->dead |= ovf;
                c->ovf_lanes = 0;
            }
            c->active = ld_agent(&c->next_active) & ~c->dead;
            c->next_active = 0;
        }
        if (MODE && tid < kLanes) {
            const int mx = a.maxexp[tid], mn = a.maxexp[kLanes + tid];
            int sh = 0;
            if (mx != INT_MIN && mx > 960) sh = mx - 900;
            if (mn != INT_MAX && mn - sh < -1000) atomicOr(&c->err, ERR_SIGMA_RANGE);
            a.shift[(size_t)(l + 1) * kLanes + tid] = sh;
            a.maxexp[tid] = INT_MIN;
            a.maxexp[kLanes + tid] = INT_MAX;
        }
        if (tid == 0) {
            const uint32_t cnt = ld_agent(&c->next_count);
            const unsigned long long edges = ld_agent(&c->next_edges);
            c->level = l + 1;
            c->visited_n += cnt;
            c->visited_m += edges;
            const unsigned long long fn = ld_agent(&c->full_n), fm = ld_agent(&c->full_m);
            s_feat.nf = (float)cnt;
            s_feat.mf = (float)edges;
            s_feat.nu = (float)((long long)c->range_nodeg - (long long)fn);
            s_feat.mu = (float)((long long)c->range_arcs - (long long)fm);
            s_feat.level = l + 1;
            c->next_count = 0;
            c->next_edges = 0;
            c->prev_variant = c->variant;
            c->phase = PH_FWD;
        }
        __syncthreads();
        const int v = choose_variant(a.p, c->policy, c->prev_variant, s_feat, (float)(c->range_hi - c->range_lo),
                                     (float)c->range_arcs, s_lds);
        if (tid == 0) c->variant = v;
    }
}

template __global__ void batch_step<0>(BatchArgs);
template __global__ void batch_step<1>(BatchArgs);

}  // namespace bcx
