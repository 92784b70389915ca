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
//
// Load balance: a vertex of degree <= kLightDeg is handled by one thread
// (thread-per-vertex variants), one of degree <= kSeg by one wavefront, and a
// heavier one is split into kSeg-arc segments, one wavefront each.  Segment
// partial sums are combined in segment order by the last segment to finish,
// so every sum has an order fixed by the vertex and the results are bitwise
// reproducible.
#include "bc_common.h"

namespace bcx {

// ------------------------------------------------------------------ pieces

// Push from frontier vertex u (lane mask f) over arcs [a0, a1), one arc per
// lane per chunk.  Appends newly reached vertices to the next level.
__device__ __forceinline__ void push_arcs_wave(const BatchArgs &a, unsigned long long f, int a0, int a1,
                                               const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                                               uint32_t qe, uint32_t hq_base, unsigned long long &my_edges,
                                               Stage &st, int &sn, const GroupArgs &gr) {
    Ctl *c = a.ctl;
    for (int eb = a0; eb < a1; eb += kWave) {
        const int e = eb + lane_id();
        bool newly = false;
        int w = 0, cw = 0;
        if (e < a1) {
            w = col[e];
            const VisNext x = a.vn[w];
            const unsigned long long add = f & ~x.vis & ~x.nxt;
            if (add) newly = atomicOr(&a.vn[w].nxt, add) == 0ull;
            if (newly) {
                const int dw = rp[w + 1] - rp[w];
                my_edges += (unsigned)dw;
                cw = class_deg(a.g, w, dw);
            }
        }
        stage_push(newly, w, cw, st, sn, c, a.lq_vtx, qe, a.lq_cap, a.hq, hq_base, &c->err, gr);
    }
}

#ifndef BC_UNROLL
#define BC_UNROLL 4
#endif
constexpr int kUnroll = BC_UNROLL;  // matched neighbours whose values are loaded together

// Per-source values live in vertex-major slabs [n][64]: path count, c and
// delta of vertex v for lane k at v * 64 + k.  Each (vertex, lane) pair is on
// exactly one level of a batch, so the slot is written once per batch and
// read only through a matching level tag and lane mask; nothing is cleared.
__device__ __forceinline__ unsigned long long readlane_u64(unsigned long long x, int j) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, j);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(x >> 32), j);
    return ((unsigned long long)hi << 32) | lo;
}

// Up to kUnroll matches, popped in ascending lane order: the lanes x that
// take the neighbour's value, the slab row of the neighbour (v * 64) and the
// group entry the match belongs to (all wavefront-uniform).
struct Matches {
    unsigned long long x[kUnroll];
    size_t row[kUnroll];
    int own[kUnroll];
};

__device__ __forceinline__ void pop_matches(unsigned long long &bal, unsigned long long xj, int uj, int ownj,
                                            Matches &mt) {
#pragma unroll
    for (int q = 0; q < kUnroll; ++q) {
        if (bal) {
            const int j = __ffsll(bal) - 1;
            bal &= bal - 1;
            mt.x[q] = readlane_u64(xj, j);
            mt.row[q] = (size_t)__builtin_amdgcn_readlane(uj, j) * kLanes;
            mt.own[q] = __builtin_amdgcn_readlane(ownj, j);
        } else {
            mt.x[q] = 0ull;
            mt.row[q] = 0;
            mt.own[q] = -1;
        }
    }
}

// Path counts: sum over arcs [a0, a1) of w's neighbours u on level l (tag T)
// of sigma_k(u) for the lanes k of m; lane k accumulates its own source, in
// CSR order.  Loads of up to kUnroll neighbours are issued together.
template <int MODE>
__device__ __forceinline__ void sig_arcs(const BatchArgs &a, const Tagged *__restrict__ fw_cur, uint32_t T,
                                         unsigned long long m, int a0, int a1, int sh,
                                         const int32_t *__restrict__ col, unsigned long long &lo,
                                         unsigned long long &hi, double &accd, unsigned long long &my_larcs,
                                         unsigned long long &my_pairs) {
    const int lane = lane_id();
    for (int eb = a0; eb < a1; eb += kWave) {
        const int e = eb + lane;
        unsigned long long xj = 0;
        int uj = 0;
        if (e < a1) {
            uj = col[e];
            const Tagged F = fw_cur[uj];
            if (F.tag == T) xj = F.mask & m;
        }
        unsigned long long bal = __ballot(xj != 0ull);
        while (bal) {
            Matches mt;
            pop_matches(bal, xj, uj, 0, mt);
            unsigned long long val[kUnroll];
#pragma unroll
            for (int q = 0; q < kUnroll; ++q)
                val[q] = ((mt.x[q] >> lane) & 1ull) ? a.sigma[mt.row[q] + lane] : 0ull;
#pragma unroll
            for (int q = 0; q < kUnroll; ++q) {
                if ((mt.x[q] >> lane) & 1ull) {
                    if (MODE == 0) {
                        lo += val[q];
                        hi += (lo < val[q]) ? 1ull : 0ull;
                    } else {
                        accd += ldexp(as_f64(val[q]), -sh);
                    }
                }
                if (lane == 0) {
                    my_larcs += (unsigned)__popcll(mt.x[q]);
                    my_pairs += mt.x[q] ? 1u : 0u;
                }
            }
        }
    }
}

// Dependencies: sum over arcs [a0, a1) of v's neighbours w on level l+1 (tag
// TB1) of c_k(w) for the lanes k of M, in CSR order.
__device__ __forceinline__ double bwd_arcs(const BatchArgs &a, const Tagged *__restrict__ fb_nxt, uint32_t TB1,
                                           unsigned long long M, int a0, int a1, const int32_t *__restrict__ col,
                                           unsigned long long &my_larcs, unsigned long long &my_pairs) {
    const int lane = lane_id();
    double acc = 0.0;
    for (int eb = a0; eb < a1; eb += kWave) {
        const int e = eb + lane;
        unsigned long long xj = 0;
        int uj = 0;
        if (e < a1) {
            uj = col[e];
            const Tagged F = fb_nxt[uj];
            if (F.tag == TB1) xj = F.mask & M;
        }
        unsigned long long bal = __ballot(xj != 0ull);
        while (bal) {
            Matches mt;
            pop_matches(bal, xj, uj, 0, mt);
            double val[kUnroll];
#pragma unroll
            for (int q = 0; q < kUnroll; ++q)
                val[q] = ((mt.x[q] >> lane) & 1ull) ? a.chat[mt.row[q] + lane] : 0.0;
#pragma unroll
            for (int q = 0; q < kUnroll; ++q) {
                if ((mt.x[q] >> lane) & 1ull) acc += val[q];
                if (lane == 0) {
                    my_larcs += (unsigned)__popcll(mt.x[q]);
                    my_pairs += mt.x[q] ? 1u : 0u;
                }
            }
        }
    }
    return acc;
}


// Per-lane counters the path-count finalisation feeds.
struct SigCounters {
    unsigned long long edges = 0, act = 0, ovf = 0, full_n = 0, full_m = 0, larcs = 0, arcs = 0, pairs = 0, lent = 0;
    int maxe = INT_MIN, mine = INT_MAX;
};

// New vertex w (queue position p, visited/next words vis/m, degree deg)
// joins the level-(l+1) frontier; called by one thread per entry.
__device__ __forceinline__ void sig_publish(const BatchArgs &a, Tagged *fw_nxt, uint32_t T1, int p, int w,
                                            unsigned long long vis, unsigned long long m, int deg,
                                            unsigned long long lmask, SigCounters &sc) {
    VisNext y;
    y.vis = vis | m;
    y.nxt = 0ull;
    a.vn[w] = y;
    Tagged tg;
    tg.mask = m;
    tg.tag = T1;
    fw_nxt[w] = tg;
    a.lq_mask[p] = m;
    sc.edges += (unsigned)deg;
    sc.act |= m;
    sc.lent += (unsigned)__popcll(m);
    if ((y.vis & lmask) == lmask) {
        sc.full_n += 1;
        sc.full_m += (unsigned)deg;
    }
}

// Store the path counts of new vertex w (queue position p, visited/next words
// vis/m, degree deg) and publish it as part of the level-(l+1) frontier.
template <int MODE>
__device__ __forceinline__ void sig_finalize(const BatchArgs &a, Tagged *fw_nxt, uint32_t T1, int p, int w,
                                             unsigned long long vis, unsigned long long m, int deg,
                                             unsigned long long lo, unsigned long long hi, double accd,
                                             unsigned long long lmask, SigCounters &sc) {
    const int lane = lane_id();
    if ((m >> lane) & 1ull) {
        const size_t at = (size_t)w * kLanes + lane;
        if (MODE == 0) a.sigma[at] = lo;
        else a.sigma[at] = as_u64(accd);
        if (MODE == 0) {
            if (hi != 0 || lo > a.sigma_limit) sc.ovf |= 1ull << lane;
        } else if (accd > 0.0) {
            int ex;
            frexp(accd, &ex);
            sc.maxe = max(sc.maxe, ex);
            sc.mine = min(sc.mine, ex);
        }
    }
    if (lane == 0) sig_publish(a, fw_nxt, T1, p, w, vis, m, deg, lmask, sc);
}

// Dependencies of vertex v (entry mask Mf, live lanes M) from the sum acc:
// delta into the delta slab (read by PH_BC), c into the c slab.
template <int MODE>
__device__ __forceinline__ void bwd_finalize(const BatchArgs &a, Tagged *fb_cur, uint32_t TB, int v,
                                             unsigned long long Mf, unsigned long long M, double acc, int sh,
                                             int shn) {
    const int lane = lane_id();
    if ((M >> lane) & 1ull) {
        const size_t at = (size_t)v * kLanes + lane;
        const unsigned long long raw = a.sigma[at];
        const double sv = MODE ? ldexp(as_f64(raw), -sh) : (double)raw;
        double delta = sv * acc;
        if (MODE) delta = ldexp(delta, -shn);
        a.chat[at] = (1.0 + delta) / sv;
        a.delta[at] = delta;
    }
    if (lane == 0) {
        Tagged tg;
        tg.mask = Mf;
        tg.tag = TB;
        fb_cur[v] = tg;
    }
}

// Owner of packed arc index ai: the number of entries whose inclusive arc
// prefix is <= ai (all lanes take part; incl[63] > ai is required).
__device__ __forceinline__ int packed_owner(int incl, int ai) {
    int o = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int v = __shfl(incl, o + step - 1);
        if (v <= ai) o += step;
    }
    return o;
}

// Index of the j-th set bit (j counted from 0) of m; m has more than j bits.
__device__ __forceinline__ int nth_set_bit(unsigned long long m, int j) {
    for (; j > 0; --j) m &= m - 1;
    return __ffsll(m) - 1;
}

// Entry-lane items: when the entries of a group carry few sources each, the
// per-source sums run one thread per (entry, source) pair instead of one
// wavefront lane per source.  Each thread then scans its entry's adjacency
// on its own and reads only its source's value of each matched neighbour, so
// the matched neighbours of single-source entries are no longer visited one
// after another by the whole wavefront.  Every sum is still taken over the
// entry's arcs in CSR order with the same operations, so the results are the
// same bits as in the per-lane form.
//   cnt   this lane's entry's item count (0 for entries handled elsewhere)
// Returns the group's items; item it belongs to entry packed_owner(incl, it).
__device__ __forceinline__ int group_items(int cnt, int &incl) {
    incl = wave_incl_scan(cnt);
    return __shfl(incl, 63);
}

#ifndef BC_PACK
#define BC_PACK 64
#endif
constexpr int kPack = BC_PACK;    // entries of degree <= kPack share 64-arc scan chunks

// Path counts for the entries [i0, i1) of level l+1 (one group, at most 64):
// entries of degree <= kPack have their adjacencies packed into dense 64-arc
// chunks; entries of degree <= kSeg follow one at a time; heavier ones run as
// segments elsewhere.  Every entry's sum keeps CSR order.
template <int MODE>
__device__ __forceinline__ void sig_group(const BatchArgs &a, const Tagged *__restrict__ fw_cur, Tagged *fw_nxt,
                                          uint32_t T, int qs, int i0, int i1, int sh, unsigned long long lmask,
                                          SigCounters &sc, int l, int *s_emax, int *s_emin, float il) {
    // predecessors: the in-arcs (the adjacency itself for undirected graphs)
    const int32_t *__restrict__ rp = a.g.in_row_ptr;
    const int32_t *__restrict__ col = a.g.in_col;
    const int lane = lane_id();
    const int i = i0 + lane;
    const int ne = i1 - i0;
    const bool valid = i < i1;
    const int p = qs + i;
    const int w = valid ? a.lq_vtx[p] : 0;
    const int e0 = valid ? rp[w] : 0;
    const int na = valid ? rp[w + 1] - e0 : 0;  // arcs to scan
    const int od = (valid && a.g.directed) ? a.g.row_ptr[w + 1] - a.g.row_ptr[w] : na;  // out-degree
    const int deg = a.g.directed ? (valid ? max(na, od) : 0) : na;  // class degree
    const bool light = valid && deg <= kPack;
    const bool medium = valid && deg > kPack && deg <= kSeg;
    unsigned long long vis = 0, nxt = 0;
    if (light || medium) {
        const VisNext x = a.vn[w];
        vis = x.vis;
        nxt = x.nxt;
    }
    // few sources per light entry: one thread per (entry, source) pair
    int iincl = 0;
    const int n_items = group_items(light ? __popcll(nxt) : 0, iincl);
    const int n_light = __popcll(__ballot(light));
    if (n_light > 0 && (float)n_items <= il * (float)n_light) {
        for (int base = 0; base < n_items; base += kWave) {
            const int it = base + lane;
            const int o = packed_owner(iincl, min(it, n_items - 1));
            const int wo = __shfl(w, o), e0o = __shfl(e0, o), dgo = __shfl(na, o), io = __shfl(iincl, o);
            const unsigned long long mo = shfl_u64(nxt, o);
            if (it < n_items) {
                const int k = nth_set_bit(mo, it - (io - __popcll(mo)));
                const int shk = MODE ? a.shift[(size_t)l * kLanes + k] : 0;
                unsigned long long ilo = 0, ihi = 0;
                double iacc = 0.0;
                unsigned matched = 0;
                for (int e = e0o; e < e0o + dgo; ++e) {
                    const int u = col[e];
                    const Tagged F = fw_cur[u];
                    if (F.tag == T && ((F.mask >> k) & 1ull)) {
                        const unsigned long long v = a.sigma[(size_t)u * kLanes + k];
                        if (MODE == 0) {
                            ilo += v;
                            ihi += (ilo < v) ? 1ull : 0ull;
                        } else {
                            iacc += ldexp(as_f64(v), -shk);
                        }
                        ++matched;
                    }
                }
                sc.larcs += matched;
                sc.pairs += matched;
                sc.arcs += (unsigned)dgo;
                const size_t at = (size_t)wo * kLanes + k;
                if (MODE == 0) {
                    a.sigma[at] = ilo;
                    if (ihi != 0 || ilo > a.sigma_limit) sc.ovf |= 1ull << k;
                } else {
                    a.sigma[at] = as_u64(iacc);
                    if (iacc > 0.0) {
                        int ex;
                        frexp(iacc, &ex);
                        atomicMax(&s_emax[k], ex);
                        atomicMin(&s_emin[k], ex);
                    }
                }
            }
        }
        if (light) sig_publish(a, fw_nxt, T + 1u, p, w, vis, nxt, od, lmask, sc);
    } else {
    const int dl = light ? na : 0;
    const int incl = wave_incl_scan(dl);
    const int off = incl - dl;
    const int total = __shfl(incl, 63);
    unsigned long long lo = 0, hi = 0;
    double accd = 0.0;
    int cur = 0;  // entries below cur are finalised; cur is being summed
    auto finalize_upto = [&](int upto) {  // finalise cur (with the sum) .. upto-1 (empty sums)
        for (int e = cur; e < upto; ++e) {
            if (__builtin_amdgcn_readlane((int)light, e)) {
                sig_finalize<MODE>(a, fw_nxt, T + 1u, __builtin_amdgcn_readlane(p, e),
                                   __builtin_amdgcn_readlane(w, e), readlane_u64(vis, e), readlane_u64(nxt, e),
                                   __builtin_amdgcn_readlane(od, e), lo, hi, accd, lmask, sc);
            }
            lo = hi = 0;
            accd = 0.0;
        }
        cur = upto;
    };
    for (int base = 0; base < total; base += kWave) {
        const int ai = base + lane;
        const int o = packed_owner(incl, min(ai, total - 1));
        const int e0o = __shfl(e0, o), offo = __shfl(off, o);
        const unsigned long long mo = shfl_u64(nxt, o);
        unsigned long long xj = 0;
        int uj = 0;
        if (ai < total) {
            uj = col[e0o + (ai - offo)];
            const Tagged F = fw_cur[uj];
            if (F.tag == T) xj = F.mask & mo;
        }
        if (lane == 0) sc.arcs += (unsigned)min(kWave, total - base);
        unsigned long long bal = __ballot(xj != 0ull);
        while (bal) {
            Matches mt;
            pop_matches(bal, xj, uj, o, mt);
            unsigned long long val[kUnroll];
#pragma unroll
            for (int q = 0; q < kUnroll; ++q)
                val[q] = ((mt.x[q] >> lane) & 1ull) ? a.sigma[mt.row[q] + lane] : 0ull;
#pragma unroll
            for (int q = 0; q < kUnroll; ++q) {
                if (mt.own[q] < 0) continue;
                if (mt.own[q] != cur) finalize_upto(mt.own[q]);
                if ((mt.x[q] >> lane) & 1ull) {
                    if (MODE == 0) {
                        lo += val[q];
                        hi += (lo < val[q]) ? 1ull : 0ull;
                    } else {
                        accd += ldexp(as_f64(val[q]), -sh);
                    }
                }
                if (lane == 0) {
                    sc.larcs += (unsigned)__popcll(mt.x[q]);
                    sc.pairs += mt.x[q] ? 1u : 0u;
                }
            }
        }
    }
    finalize_upto(ne);
    }
    // medium-degree entries: one wavefront-wide scan each
    unsigned long long mm = __ballot(medium);
    while (mm) {
        const int j = __ffsll(mm) - 1;
        mm &= mm - 1;
        const int wj = __builtin_amdgcn_readlane(w, j);
        const int a0 = __builtin_amdgcn_readlane(e0, j), dj = __builtin_amdgcn_readlane(na, j);
        const unsigned long long mj = readlane_u64(nxt, j);
        unsigned long long lo = 0, hi = 0;
        double accd = 0.0;
        sig_arcs<MODE>(a, fw_cur, T, mj, a0, a0 + dj, sh, col, lo, hi, accd, sc.larcs, sc.pairs);
        if (lane == 0) sc.arcs += (unsigned)dj;
        sig_finalize<MODE>(a, fw_nxt, T + 1u, __builtin_amdgcn_readlane(p, j), wj, readlane_u64(vis, j), mj,
                           __builtin_amdgcn_readlane(od, j), lo, hi, accd, lmask, sc);
    }
}

// Dependencies for the entries [i0, i1) of level l (one group), packed like
// sig_group.
template <int MODE>
__device__ __forceinline__ void bwd_group(const BatchArgs &a, const Tagged *__restrict__ fb_nxt, Tagged *fb_cur,
                                          uint32_t TB, int qb, int i0, int i1, unsigned long long dead, int sh,
                                          int shn, unsigned long long &my_larcs, unsigned long long &my_arcs,
                                          unsigned long long &my_pairs, int l, bool has_next, float il) {
    const int32_t *__restrict__ rp = a.g.row_ptr;
    const int32_t *__restrict__ col = a.g.col;
    const int lane = lane_id();
    const int i = i0 + lane;
    const int ne = i1 - i0;
    const bool valid = i < i1;
    const int p = qb + i;
    const int v = valid ? a.lq_vtx[p] : 0;
    const int e0 = valid ? rp[v] : 0;
    const int na = valid ? rp[v + 1] - e0 : 0;  // successors: the out-arcs
    const int deg = valid ? class_deg(a.g, v, na) : 0;
    const bool light = valid && deg <= kPack;
    const bool medium = valid && deg > kPack && deg <= kSeg;
    const unsigned long long Mf = (light || medium) ? a.lq_mask[p] : 0ull;
    const unsigned long long M = Mf & ~dead;
    // few sources per light entry: one thread per (entry, source) pair
    int iincl = 0;
    const int n_items = group_items(light ? __popcll(M) : 0, iincl);
    const int n_light = __popcll(__ballot(light));
    if (n_light > 0 && (float)n_items <= il * (float)n_light) {
        for (int base = 0; base < n_items; base += kWave) {
            const int it = base + lane;
            const int o = packed_owner(iincl, min(it, n_items - 1));
            const int vo = __shfl(v, o), e0o = __shfl(e0, o), dgo = __shfl(na, o), io = __shfl(iincl, o);
            const unsigned long long mo = shfl_u64(M, o);
            if (it < n_items) {
                const int k = nth_set_bit(mo, it - (io - __popcll(mo)));
                double iacc = 0.0;
                unsigned matched = 0;
                for (int e = e0o; e < e0o + dgo; ++e) {
                    const int u = col[e];
                    const Tagged F = fb_nxt[u];
                    if (F.tag == TB + 1u && ((F.mask >> k) & 1ull)) {
                        iacc += a.chat[(size_t)u * kLanes + k];
                        ++matched;
                    }
                }
                my_larcs += matched;
                my_pairs += matched;
                my_arcs += (unsigned)dgo;
                const size_t at = (size_t)vo * kLanes + k;
                const int shk = MODE ? a.shift[(size_t)l * kLanes + k] : 0;
                const int shnk = (MODE && has_next) ? a.shift[(size_t)(l + 1) * kLanes + k] : 0;
                const unsigned long long raw = a.sigma[at];
                const double sv = MODE ? ldexp(as_f64(raw), -shk) : (double)raw;
                double delta = sv * iacc;
                if (MODE) delta = ldexp(delta, -shnk);
                a.chat[at] = (1.0 + delta) / sv;
                a.delta[at] = delta;
            }
        }
        if (light) {
            Tagged tg;
            tg.mask = Mf;
            tg.tag = TB;
            fb_cur[v] = tg;
        }
    } else {
    const int dl = (light && M) ? na : 0;
    const int incl = wave_incl_scan(dl);
    const int off = incl - dl;
    const int total = __shfl(incl, 63);
    double acc = 0.0;
    int cur = 0;
    auto finalize_upto = [&](int upto) {
        for (int e = cur; e < upto; ++e) {
            if (__builtin_amdgcn_readlane((int)light, e))
                bwd_finalize<MODE>(a, fb_cur, TB, __builtin_amdgcn_readlane(v, e), readlane_u64(Mf, e),
                                   readlane_u64(M, e), acc, sh, shn);
            acc = 0.0;
        }
        cur = upto;
    };
    for (int base = 0; base < total; base += kWave) {
        const int ai = base + lane;
        const int o = packed_owner(incl, min(ai, total - 1));
        const int e0o = __shfl(e0, o), offo = __shfl(off, o);
        const unsigned long long mo = shfl_u64(M, o);
        unsigned long long xj = 0;
        int uj = 0;
        if (ai < total) {
            uj = col[e0o + (ai - offo)];
            const Tagged F = fb_nxt[uj];
            if (F.tag == TB + 1u) xj = F.mask & mo;
        }
        if (lane == 0) my_arcs += (unsigned)min(kWave, total - base);
        unsigned long long bal = __ballot(xj != 0ull);
        while (bal) {
            Matches mt;
            pop_matches(bal, xj, uj, o, mt);
            double val[kUnroll];
#pragma unroll
            for (int q = 0; q < kUnroll; ++q)
                val[q] = ((mt.x[q] >> lane) & 1ull) ? a.chat[mt.row[q] + lane] : 0.0;
#pragma unroll
            for (int q = 0; q < kUnroll; ++q) {
                if (mt.own[q] < 0) continue;
                if (mt.own[q] != cur) finalize_upto(mt.own[q]);
                if ((mt.x[q] >> lane) & 1ull) acc += val[q];
                if (lane == 0) {
                    my_larcs += (unsigned)__popcll(mt.x[q]);
                    my_pairs += mt.x[q] ? 1u : 0u;
                }
            }
        }
    }
    finalize_upto(ne);
    }
    unsigned long long mm = __ballot(medium);
    while (mm) {
        const int j = __ffsll(mm) - 1;
        mm &= mm - 1;
        const int vj = __builtin_amdgcn_readlane(v, j);
        const int a0 = __builtin_amdgcn_readlane(e0, j), dj = __builtin_amdgcn_readlane(na, j);
        const unsigned long long Mj = readlane_u64(M, j);
        const double sm = Mj ? bwd_arcs(a, fb_nxt, TB + 1u, Mj, a0, a0 + dj, col, my_larcs, my_pairs) : 0.0;
        if (lane == 0) my_arcs += (unsigned)dj;
        bwd_finalize<MODE>(a, fb_cur, TB, vj, readlane_u64(Mf, j), Mj, sm, sh, shn);
    }
}

// The variant of the next level and the summation options chosen with it
// (lbo, see choose_variant); when collecting timings, every level starts
// with variant 0 and its normalised features are kept for the samples.
__device__ __forceinline__ void set_level_variant(const BatchArgs &a, Ctl *c, int v, int lbo, const LevelFeatures &f,
                                                  float n, float nnz) {
    if (f.level < a.max_levels + 2) a.lbsel[f.level] = lbo;
    if (c->collect) {
        float x[kMlpIn];
        mlp_inputs(f, n, nnz, x);
        for (int i = 0; i < kMlpIn; ++i) c->feat[i] = x[i];
        if (a.col_F && f.level < a.max_levels + 2)
            for (int i = 0; i < kMlpIn; ++i) a.col_F[(size_t)f.level * kMlpIn + i] = x[i];
        c->cvar = 0;
        c->variant = 0;
    } else {
        c->variant = v;
    }
}

template <int MODE>
__device__ __forceinline__ void batch_begin(const BatchArgs &a, Ctl *c, int64_t b, float *lds, LevelFeatures *sf, int *s_lsrc,
                            int *s_cnt, unsigned long long *s_tmp, int *s_lead) {
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
        c->lane_E[t] = 0;
        c->lane_emax[t] = INT_MIN;
    }
    __syncthreads();
    // lanes with the same source share one level-0 entry, led by its lowest lane
    unsigned long long m = 0;
    int lead = t;
    if (t < lanes) {
        const int s = s_lsrc[t];
        for (int k = lanes - 1; k >= 0; --k) {
            if (s_lsrc[k] == s) {
                m |= 1ull << k;
                lead = k;
            }
        }
        s_lead[t] = lead;
    }
    __syncthreads();
    if (t < lanes) {
        const int s = s_lsrc[t];
        a.sigma[(size_t)s * kLanes + t] = MODE ? as_u64(1.0) : 1ull;
        if (lead == t) {
            const int j = atomicAdd(s_cnt, 1);
            a.lq_vtx[j] = s;
            a.lq_mask[j] = m;
            a.vn[s].vis = m;
            Tagged tg;
            tg.mask = m;
            tg.tag = epoch;
            a.fw0[s] = tg;
            const int od = a.g.row_ptr[s + 1] - a.g.row_ptr[s];
            s_tmp[j] = (unsigned long long)(unsigned)od | ((unsigned long long)(unsigned)class_deg(a.g, s, od) << 32);
        }
    }
    if (MODE && t < kLanes) a.shift[t] = 0;
    __syncthreads();
    if (t == 0) {
        const int cnt = *s_cnt;
        unsigned long long mf = 0;
        int nh = 0, segs = 0;
        for (int j = 0; j < cnt; ++j) {
            const int deg = (int)(uint32_t)s_tmp[j], cdeg = (int)(s_tmp[j] >> 32);
            mf += (unsigned long long)deg;
            if (cdeg > kSeg) {  // heavy source: level-0 segments for the push
                a.hq.pos[nh] = j;
                a.hq.seg[nh] = segs;
                a.hq.cnt[nh] = 0;
                segs += n_segments(cdeg);
                ++nh;
            }
        }
        a.hq.off[0] = 0;
        a.hq.off[1] = nh;
        a.hq.nseg[0] = segs;
        c->next_hq = 0;
        a.gstart[0] = 0u;  // level 0 has no groups; level 1 appends from slot 1
        a.gbase[0] = 0u;
        a.gbase[1] = 1u;
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
        c->next_qc = 0ull;
        c->next_edges = 0;
        c->next_active = 0;
        c->prev_variant = V_PUSH_TPV;
        c->phase = PH_FWD;
        c->st_batches += 1;
        c->st_lane_entries += (unsigned long long)lanes;
        if (a.lvl) level_rec(a.lvl, 0).entries += (unsigned long long)cnt;
        const int64_t dp = c->dump_pos;
        c->dump_lane = (dp >= start && dp < end && c->dump_state == 0) ? (int)(dp - start) : -1;
        sf->nf = (float)cnt;
        sf->mf = (float)mf;
        sf->nu = (float)c->range_nodeg;
        sf->mu = (float)c->range_arcs;
        sf->level = 0;
    }
    __syncthreads();
    int lbo;
    const int v = choose_variant(a.p, c->policy, V_PUSH_TPV, *sf, (float)(c->range_hi - c->range_lo),
                                 (float)c->range_arcs, lds, &lbo);
    if (t == 0) set_level_variant(a, c, v, lbo, *sf, (float)(c->range_hi - c->range_lo), (float)c->range_arcs);
}

#ifndef BC_WAVES
#define BC_WAVES 6
#endif
// Register budget of the step kernel: at least BC_WAVES wavefronts per SIMD
// (memory latency is hidden by resident wavefronts).
// One step of the level state machine for workgroup bid of a launch of
// `grid` workgroups: the step kernel below runs it once per launch over the
// whole grid; the block engine runs it in a loop inside one workgroup
// (grid = 1), which then owns the state machine alone.
template <int MODE>
__device__ __forceinline__ void batch_step_body(const BatchArgs &a, const unsigned bid, const unsigned grid) {
    __shared__ int s_phase, s_level, s_variant, s_last, s_qb, s_qe, s_qn, s_L, s_lo, s_hi, s_dlane, s_cnt;
    __shared__ int s_h0, s_h1, s_hseg, s_hqb;
    __shared__ uint32_t s_gb, s_ng;
    __shared__ unsigned s_nblk;
    __shared__ uint32_t s_epoch, s_epoch_b;
    __shared__ unsigned long long s_active, s_dead, s_lmask;
    __shared__ unsigned long long s_red[kSlots * kNCnt];
    __shared__ unsigned long long s_tot[kNCnt];
    __shared__ unsigned long long s_tmp[kLanes];
    __shared__ int s_lsrc[kLanes];
    __shared__ int s_lead[kLanes];
    __shared__ Stage s_stage[kWavesPerBlock];
    __shared__ float s_lds[2 * kMlpH + kMlpOut + 4];
    __shared__ LevelFeatures s_feat;
    __shared__ float s_il;  // sources-per-entry threshold of this path-count / backward step
    __shared__ int s_usig;  // an undo step restores a path-count step (timing collection)
    __shared__ int s_emax[kLanes], s_emin[kLanes];
    __shared__ double s_bct[kWavesPerBlock][kWave * 8];  // score accumulation: 64 rows x 8 lanes per wavefront
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
        s_qb = s_qe = s_qn = 0;
        s_h0 = s_h1 = s_hseg = s_hqb = 0;
        s_gb = s_ng = 0;
        const int l = s_level;
        s_il = a.p.item_lanes;
        if (s_phase == PH_SIG || s_phase == PH_BWD) {
            // the option timed (collection), else the one chosen with level l
            const int sel = (l < a.max_levels + 2) ? a.lbsel[l] : kLbDefault;
            const int opt = c->collect ? c->clb : (s_phase == PH_SIG ? (sel & 3) : ((sel >> 2) & 3));
            s_il = lb_item_lanes(a.p, opt);
        }
        if (s_phase == PH_FWD || s_phase == PH_SIG || s_phase == PH_BWD) {
            s_qb = a.level_off[l];
            s_qe = a.level_off[l + 1];
            if (s_phase == PH_SIG) s_qn = a.level_off[l + 2];
        } else if (s_phase == PH_DUMP_FWD || s_phase == PH_DUMP_BWD) {
            s_qe = a.level_off[s_L];
        } else if (s_phase == PH_UNDO) {
            s_qe = a.level_off[l + 1];
            s_qn = (int)(uint32_t)c->next_qc;
        }
        s_usig = c->undo_sig;
        if (s_phase == PH_FWD) {
            if (s_variant == V_PULL) {  // static heavy vertices of the batch's range
                const int i0 = lower_bound_i32(a.g.hv_vtx, a.g.n_heavy, s_lo);
                const int i1 = lower_bound_i32(a.g.hv_vtx, a.g.n_heavy, s_hi);
                s_h0 = i0;
                s_h1 = i1;
                s_hseg = a.g.hv_seg[i1] - a.g.hv_seg[i0];
            } else {                    // heavy frontier entries of level l
                s_h0 = a.hq.off[l];
                s_h1 = a.hq.off[l + 1];
                s_hseg = a.hq.nseg[l];
            }
            s_hqb = a.hq.off[l + 1];    // heavy entries of level l+1 start here
            s_gb = a.gbase[l + 1];      // groups of level l+1 are appended here
        } else if (s_phase == PH_SIG) {
            s_h0 = a.hq.off[l + 1];
            s_h1 = a.hq.off[l + 2];
            s_hseg = a.hq.nseg[l + 1];
            s_gb = a.gbase[l + 1];
            s_ng = a.gbase[l + 2] - s_gb - 1u;
        } else if (s_phase == PH_BWD) {
            s_h0 = a.hq.off[l];
            s_h1 = a.hq.off[l + 1];
            s_hseg = a.hq.nseg[l];
            s_gb = a.gbase[l];
            s_ng = a.gbase[l + 1] - s_gb - 1u;
        }
        // wavefront work items of this step -> workgroups taking part
        long long items = 1;
        const int cnt = s_qe - s_qb;
        if (s_phase == PH_FWD) {
            if (s_variant == V_PUSH_TPV) items = (cnt + kWave - 1) / kWave + s_hseg;
            else if (s_variant == V_PUSH_WPV) items = cnt + s_hseg;
            else items = (s_hi - s_lo + kWave - 1) / kWave + s_hseg;
        } else if (s_phase == PH_SIG || s_phase == PH_BWD) {
            items = (long long)s_ng + s_hseg;
        } else if (s_phase == PH_BC) {
            items = (s_hi - s_lo + kWave - 1) / kWave;
        } else if (s_phase == PH_DUMP_FWD || s_phase == PH_DUMP_BWD) {
            items = (s_qe + kWave - 1) / kWave;
        } else if (s_phase == PH_UNDO) {
            items = (s_qn + kWave - 1) / kWave;
        }
        s_nblk = active_blocks(items, grid);
    }
    if (tid < kLanes) {
        s_lsrc[tid] = a.lane_src[tid];
        s_emax[tid] = INT_MIN;
        s_emin[tid] = INT_MAX;
    }
    __syncthreads();
    const int phase = s_phase;
    if (phase == PH_DONE || phase == PH_IDLE) return;
    const unsigned nblk = s_nblk;
    const bool active = bid < nblk;  // workgroups beyond nblk only count in

    const int gw = (int)bid * kWavesPerBlock + wid;
    const int nw = (int)nblk * kWavesPerBlock;
    const int l = s_level;
    const int32_t *__restrict__ rp = a.g.row_ptr;
    const int32_t *__restrict__ col = a.g.col;
    Tagged *fw_cur = (l & 1) ? a.fw1 : a.fw0;
    Tagged *fw_nxt = (l & 1) ? a.fw0 : a.fw1;
    const int h0 = s_h0, h1 = s_h1, hseg = s_hseg;

    unsigned long long my_edges = 0, my_arcs = 0, my_larcs = 0, my_act = 0, my_ovf = 0;
    unsigned long long my_full_n = 0, my_full_m = 0, my_pairs = 0, my_lent = 0;
    int my_maxe = INT_MIN, my_mine = INT_MAX;

    if (!active) {
    } else if (phase == PH_FWD) {
        const int qb = s_qb, qe = s_qe, cnt = qe - qb;
        const uint32_t T = s_epoch + (uint32_t)l;
        const unsigned long long act = s_active;
        const uint32_t hqb = (uint32_t)s_hqb;
        const int variant = s_variant;
        Stage &st = s_stage[wid];
        int sn = 0;
        GroupArgs gr;
        gr.gstart = a.gstart;
        gr.gb = s_gb;
        gr.gcap = a.gcap;
        if (variant == V_PUSH_TPV || variant == V_PUSH_WPV) {
            const int n_light = variant == V_PUSH_TPV ? (cnt + kWave - 1) / kWave : cnt;
            const int total = n_light + hseg;
            for (int k = gw; k < total; k += nw) {
                const int it = k < hseg ? n_light + k : k - hseg;  // heavy segments first
                if (it >= n_light) {  // one segment of a heavy frontier vertex
                    const int t = it - n_light;
                    const int h = seg_owner(a.hq.seg, h0, h1, t);
                    const int s = t - a.hq.seg[h];
                    const int p = a.hq.pos[h];
                    const int u = a.lq_vtx[p];
                    const unsigned long long f = a.lq_mask[p] & act;
                    const int a0 = rp[u] + s * kSeg;
                    const int a1 = max(a0, min(rp[u + 1], a0 + kSeg));
                    if (lane == 0) my_arcs += (unsigned)(a1 - a0);
                    if (f) push_arcs_wave(a, f, a0, a1, rp, col, (uint32_t)qe, hqb, my_edges, st, sn, gr);
                } else if (variant == V_PUSH_WPV) {
                    const int u = a.lq_vtx[qb + it];
                    const unsigned long long f = a.lq_mask[qb + it] & act;
                    const int e0 = rp[u], e1 = rp[u + 1];
                    if (!f || class_deg(a.g, u, e1 - e0) > kSeg) continue;  // heavy ones run as segments
                    if (lane == 0) my_arcs += (unsigned)(e1 - e0);
                    push_arcs_wave(a, f, e0, e1, rp, col, (uint32_t)qe, hqb, my_edges, st, sn, gr);
                } else {  // TPV: 64 frontier vertices per wavefront
                    const int i = it * kWave + lane;
                    const bool valid = i < cnt;
                    const int u = valid ? a.lq_vtx[qb + i] : 0;
                    const unsigned long long f = valid ? (a.lq_mask[qb + i] & act) : 0ull;
                    const int e0 = f ? rp[u] : 0;
                    const int od = f ? rp[u + 1] - e0 : 0;  // out-arcs to push over
                    const int deg = f ? class_deg(a.g, u, od) : 0;
                    const int len = deg <= kLightDeg ? od : 0;
                    my_arcs += (unsigned)(deg <= kSeg ? od : 0);
                    const int maxlen = wave_max_i(len);
                    for (int t = 0; t < maxlen; ++t) {
                        bool newly = false;
                        int w = 0, cw = 0;
                        if (t < len) {
                            w = col[e0 + t];
                            const VisNext x = a.vn[w];
                            const unsigned long long add = f & ~x.vis & ~x.nxt;
                            if (add) newly = atomicOr(&a.vn[w].nxt, add) == 0ull;
                            if (newly) {
                                const int dw = rp[w + 1] - rp[w];
                                my_edges += (unsigned)dw;
                                cw = class_deg(a.g, w, dw);
                            }
                        }
                        stage_push(newly, w, cw, st, sn, c, a.lq_vtx, (uint32_t)qe, a.lq_cap, a.hq, hqb, &c->err, gr);
                    }
                    // medium-degree vertices: the whole wavefront, one at a time
                    unsigned long long mm = __ballot(deg > kLightDeg && deg <= kSeg);
                    while (mm) {
                        const int j = __ffsll(mm) - 1;
                        mm &= mm - 1;
                        const int m0 = __shfl(e0, j), m1 = m0 + __shfl(od, j);
                        push_arcs_wave(a, shfl_u64(f, j), m0, m1, rp, col, (uint32_t)qe, hqb, my_edges, st, sn, gr);
                    }
                }
            }
        } else {  // V_PULL over the batch's vertex range, scanning in-arcs (predecessors)
            const int32_t *__restrict__ irp = a.g.in_row_ptr;
            const int32_t *__restrict__ icol = a.g.in_col;
            const int lo = s_lo, span = s_hi - s_lo;
            const int n_light = (span + kWave - 1) / kWave;
            const int total = n_light + hseg;
            const int hs0 = a.g.hv_seg[h0];
            for (int k = gw; k < total; k += nw) {
                const int it = k < hseg ? n_light + k : k - hseg;  // heavy segments first
                if (it >= n_light) {  // one segment of a heavy unvisited vertex
                    const int t = hs0 + (it - n_light);
                    const int h = seg_owner(a.g.hv_seg, h0, h1, t);
                    const int s = t - a.g.hv_seg[h];
                    const int w = a.g.hv_vtx[h];
                    const unsigned long long need = act & ~a.vn[w].vis;
                    unsigned long long got = 0;
                    const int a0 = irp[w] + s * kSeg, a1 = max(a0, min(irp[w + 1], a0 + kSeg));
                    int scanned = 0;
                    if (need) {
                        for (int eb = a0; eb < a1; eb += kWave) {
                            const int e = eb + lane;
                            if (e < a1) {
                                const Tagged F = fw_cur[icol[e]];
                                if (F.tag == T) got |= F.mask & need;
                            }
                            scanned += kWave;
                            got = wave_or_u64(got);
                            if (got == need) break;
                        }
                    }
                    if (lane == 0) my_arcs += (unsigned)min(scanned, a1 - a0);
                    bool newly = false;
                    if (lane == 0 && got) newly = atomicOr(&a.vn[w].nxt, got) == 0ull;
                    const int od = rp[w + 1] - rp[w];
                    if (newly) my_edges += (unsigned)od;
                    stage_push(newly, w, class_deg(a.g, w, od), st, sn, c, a.lq_vtx, (uint32_t)qe, a.lq_cap, a.hq, hqb,
                               &c->err, gr);
                    continue;
                }
                const int w = lo + it * kWave + lane;
                const bool valid = it * kWave + lane < span;
                const unsigned long long vis = valid ? a.vn[w].vis : ~0ull;
                const unsigned long long need = act & ~vis;
                const int e0 = need ? irp[w] : 0;
                const int ni = need ? irp[w + 1] - e0 : 0;  // in-arcs to scan
                const int od = (need && a.g.directed) ? rp[w + 1] - rp[w] : ni;
                const int deg = a.g.directed ? max(ni, od) : ni;  // class degree
                const int len = deg <= kLightDeg ? ni : 0;
                const int maxlen = wave_max_i(len);
                unsigned long long got = 0;
                int scanned = 0;
                for (int t = 0; t < maxlen; ++t) {
                    if (t < len && got != need) {
                        ++scanned;
                        const Tagged F = fw_cur[icol[e0 + t]];
                        if (F.tag == T) got |= F.mask & need;
                    }
                    if (!__any(t + 1 < len && got != need)) break;
                }
                // medium-degree vertices: the whole wavefront, one at a time
                unsigned long long mm = __ballot(deg > kLightDeg && deg <= kSeg);
                while (mm) {
                    const int j = __ffsll(mm) - 1;
                    mm &= mm - 1;
                    const int m0 = __shfl(e0, j), m1 = m0 + __shfl(ni, j);
                    const unsigned long long nj = shfl_u64(need, j);
                    unsigned long long gj = 0;
                    for (int eb = m0; eb < m1; eb += kWave) {
                        const int e = eb + lane;
                        if (e < m1) {
                            const Tagged F = fw_cur[icol[e]];
                            if (F.tag == T) gj |= F.mask & nj;
                        }
                        if (lane == 0) scanned += min(kWave, m1 - eb);
                        gj = wave_or_u64(gj);
                        if (gj == nj) break;
                    }
                    if (lane == j) got = gj;
                }
                my_arcs += (unsigned)scanned;
                const bool found = got != 0ull && deg <= kSeg;
                if (found) {
                    a.vn[w].nxt = got;
                    my_edges += (unsigned)od;
                }
                stage_push(found, w, deg, st, sn, c, a.lq_vtx, (uint32_t)qe, a.lq_cap, a.hq, hqb, &c->err, gr);
            }
        }
        stage_flush(st, sn, c, a.lq_vtx, (uint32_t)qe, a.lq_cap, a.hq, hqb, &c->err, gr);
    } else if (phase == PH_SIG) {
        // path counts of the new level; lane = source
        const int qs = s_qe, cnt = s_qn - s_qe;
        const uint32_t T = s_epoch + (uint32_t)l;
        const int sh = MODE ? a.shift[(size_t)l * kLanes + lane] : 0;
        const unsigned long long lmask = s_lmask;
        const int n_groups = (int)s_ng;
        const uint32_t *gs = a.gstart + s_gb;
        const int total = n_groups + hseg;
        const float il = s_il;
        SigCounters sc;
        for (WorkCursor wc(c, nblk, bid); wc.item() < total; wc.next(total)) {
            const int k = wc.item();
            const int it = k < hseg ? n_groups + k : k - hseg;  // heavy segments first
            if (it < n_groups) {
                const int i0 = (int)gs[it], i1 = min((int)gs[it + 1], cnt);
                if (i1 > i0) sig_group<MODE>(a, fw_cur, fw_nxt, T, qs, i0, i1, sh, lmask, sc, l, s_emax, s_emin, il);
                continue;
            }
            // a segment of a heavy new vertex
            const int t = it - n_groups;
            const int h = seg_owner(a.hq.seg, h0, h1, t);
            const int s = t - a.hq.seg[h];
            const int p = a.hq.pos[h];
            const int w = a.lq_vtx[p];
            const int e0 = a.g.in_row_ptr[w], e1 = a.g.in_row_ptr[w + 1];  // predecessors: in-arcs
            const int od = rp[w + 1] - rp[w];
            const unsigned long long m = a.vn[w].nxt;
            const int a0 = e0 + s * kSeg, a1 = max(a0, min(e1, a0 + kSeg));
            unsigned long long lo = 0, hi = 0;
            double accd = 0.0;
            sig_arcs<MODE>(a, fw_cur, T, m, a0, a1, sh, a.g.in_col, lo, hi, accd, sc.larcs, sc.pairs);
            if (lane == 0) sc.arcs += (unsigned)(a1 - a0);
            const size_t slot = (size_t)(a.hq.seg[h] + s) * kLanes + lane;
            if (MODE == 0) {
                part_store(&a.hq.part_lo[slot], lo);
                part_store(&a.hq.part_hi[slot], hi);
            } else {
                part_store(&a.hq.part_lo[slot], as_u64(accd));
            }
            const int ns = n_segments(class_deg(a.g, w, od));
            if (!seg_arrive(&a.hq.cnt[h], ns)) continue;
            lo = hi = 0;
            accd = 0.0;
            for (int k = 0; k < ns; ++k) {  // combine in segment order
                const size_t sl = (size_t)(a.hq.seg[h] + k) * kLanes + lane;
                if (MODE == 0) {
                    const unsigned long long x = part_load(&a.hq.part_lo[sl]);
                    lo += x;
                    hi += part_load(&a.hq.part_hi[sl]) + ((lo < x) ? 1ull : 0ull);
                } else {
                    accd += as_f64(part_load(&a.hq.part_lo[sl]));
                }
            }
            if (lane == 0) a.hq.cnt[h] = 0;
            const VisNext x = a.vn[w];
            sig_finalize<MODE>(a, fw_nxt, T + 1u, p, w, x.vis, x.nxt, od, lo, hi, accd, lmask, sc);
        }
        my_edges += sc.edges;
        my_act |= sc.act;
        my_ovf |= sc.ovf;
        my_full_n += sc.full_n;
        my_full_m += sc.full_m;
        my_larcs += sc.larcs;
        my_arcs += sc.arcs;
        my_pairs += sc.pairs;
        my_lent += sc.lent;
        my_maxe = max(my_maxe, sc.maxe);
        my_mine = min(my_mine, sc.mine);
    } else if (phase == PH_BWD) {
        const int qb = s_qb, cnt = s_qe - s_qb;
        const uint32_t TB = s_epoch_b + (uint32_t)l;
        Tagged *fb_cur = fw_cur;  // written with this level's tag
        Tagged *fb_nxt = fw_nxt;  // read: level l+1's tag
        const unsigned long long dead = s_dead;
        const int sh = MODE ? a.shift[(size_t)l * kLanes + lane] : 0;
        const int shn = (MODE && l + 1 < s_L) ? a.shift[(size_t)(l + 1) * kLanes + lane] : 0;
        const int n_groups = (int)s_ng;
        const uint32_t *gs = a.gstart + s_gb;
        const int total = n_groups + hseg;
        for (WorkCursor wc(c, nblk, bid); wc.item() < total; wc.next(total)) {
            const int k = wc.item();
            const int it = k < hseg ? n_groups + k : k - hseg;  // heavy segments first
            if (it < n_groups) {
                const int i0 = (int)gs[it], i1 = min((int)gs[it + 1], cnt);
                if (i1 > i0)
                    bwd_group<MODE>(a, fb_nxt, fb_cur, TB, qb, i0, i1, dead, sh, shn, my_larcs, my_arcs, my_pairs, l,
                                    l + 1 < s_L, s_il);
                continue;
            }
            const int t = it - n_groups;
            const int h = seg_owner(a.hq.seg, h0, h1, t);
            const int s = t - a.hq.seg[h];
            const int p = a.hq.pos[h];
            const int v = a.lq_vtx[p];
            const unsigned long long Mf = a.lq_mask[p];
            const unsigned long long M = Mf & ~dead;
            const int e0 = rp[v], e1 = rp[v + 1];  // successors: out-arcs
            const int a0 = e0 + s * kSeg, a1 = max(a0, min(e1, a0 + kSeg));
            double acc = M ? bwd_arcs(a, fb_nxt, TB + 1u, M, a0, a1, col, my_larcs, my_pairs) : 0.0;
            if (lane == 0) my_arcs += (unsigned)(a1 - a0);
            part_store(&a.hq.part_lo[(size_t)(a.hq.seg[h] + s) * kLanes + lane], as_u64(acc));
            const int ns = n_segments(class_deg(a.g, v, e1 - e0));
            if (!seg_arrive(&a.hq.cnt[h], ns)) continue;
            acc = 0.0;
            for (int k = 0; k < ns; ++k) acc += as_f64(part_load(&a.hq.part_lo[(size_t)(a.hq.seg[h] + k) * kLanes + lane]));
            if (lane == 0) a.hq.cnt[h] = 0;
            bwd_finalize<MODE>(a, fb_cur, TB, v, Mf, M, acc, sh, shn);
        }
    } else if (phase == PH_UNDO) {
        const int qs = s_qe, cnt = s_qn;
        if (s_usig) {
            // timing collection: the entries of level l+1 get back the words
            // they had before their path-count step (that step set the lanes
            // of their queue masks visited and cleared their next words)
            for (int i = (int)bid * kBlock + tid; i < cnt; i += (int)nblk * kBlock) {
                const int w = a.lq_vtx[qs + i];
                const unsigned long long m = a.lq_mask[qs + i];
                VisNext x = a.vn[w];
                x.vis &= ~m;
                x.nxt = m;
                a.vn[w] = x;
            }
        } else {
            // timing collection: forget the level just discovered (its
            // entries are the only vertices with next words set)
            for (int i = (int)bid * kBlock + tid; i < cnt; i += (int)nblk * kBlock) a.vn[a.lq_vtx[qs + i]].nxt = 0ull;
        }
    } else if (phase == PH_BC) {
        // dependencies -> BC in lane order (the run's source order), then
        // clear the visited words.  A wavefront takes 64 consecutive
        // vertices; their delta rows are read 8 lanes (64 bytes) at a time,
        // 8 rows per load (coalesced), staged through LDS, and each vertex's
        // own thread adds its lanes in ascending order (a source's own lane
        // and lanes not reached are skipped: they would add +0.0, which
        // leaves the non-negative sum's bits unchanged)
        const int lo = s_lo, span = s_hi - s_lo;
        const unsigned long long keep = s_lmask & ~s_dead;
        const int lane = lane_id(), wv = tid / kWave;
        double *tile = s_bct[wv];
        for (int base = ((int)bid * kWavesPerBlock + wv) * kWave; base < span; base += (int)nblk * kBlock) {
            const int i = base + lane;
            const int w = lo + i;
            VisNext x;
            x.vis = 0ull;
            x.nxt = 0ull;
            if (i < span) x = a.vn[w];
            const unsigned long long vis = x.vis & keep;
            if (__ballot(vis != 0ull)) {
                double b = vis ? a.bc[w] : 0.0;
                for (int c = 0; c < kLanes / 8; ++c) {
                    const unsigned m8 = (unsigned)(vis >> (8 * c)) & 0xFFu;
                    if (!__ballot(m8 != 0u)) continue;
#pragma unroll
                    for (int r = 0; r < 8; ++r) {
                        const int vi = 8 * r + (lane >> 3);  // vertex of the 64 whose row this lane reads
                        const int kk = lane & 7;
                        const unsigned mv = (unsigned)__shfl((int)m8, vi);
                        double d = 0.0;
                        if ((mv >> kk) & 1u) d = a.delta[(size_t)(lo + base + vi) * kLanes + 8 * c + kk];
                        tile[vi * 8 + (kk ^ (vi & 7))] = d;
                    }
                    __builtin_amdgcn_wave_barrier();
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        if (((m8 >> j) & 1u) && s_lsrc[8 * c + j] != w) b += tile[lane * 8 + (j ^ (lane & 7))];
                    }
                    __builtin_amdgcn_wave_barrier();
                }
                if (vis) a.bc[w] = b;
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
        for (int j = (int)bid * kBlock + tid; j < total; j += (int)nblk * kBlock) {
            if (!((a.lq_mask[j] >> k) & 1ull)) continue;
            int lo = 0, hi = L;  // level of entry j: level_off[lvl] <= j < level_off[lvl+1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (a.level_off[mid] <= j) lo = mid;
                else hi = mid;
            }
            const int v = a.lq_vtx[j];
            if (phase == PH_DUMP_FWD) {
                a.dump_d[v] = lo;
                a.dump_sig[v] = a.sigma[(size_t)v * kLanes + k];
            } else if (lo >= 1) {
                a.dump_delta[v] = a.delta[(size_t)v * kLanes + k];
            }
        }
        if (phase == PH_DUMP_FWD && bid == 0)
            for (int i = tid; i < L; i += kBlock) a.dump_shift[i] = MODE ? a.shift[(size_t)i * kLanes + k] : 0;
    }

    // ---- per-launch counters into the slots; the last workgroup continues
    Counters cn;
    cn.v[SC_EDGES] = my_edges;
    cn.v[SC_ARCS] = my_arcs;
    cn.v[SC_LARCS] = my_larcs;
    cn.v[SC_FULLN] = my_full_n;
    cn.v[SC_FULLM] = my_full_m;
    cn.v[SC_ACT] = my_act;
    cn.v[SC_OVF] = my_ovf;
    cn.v[SC_PAIRS] = my_pairs;
    cn.v[SC_LENT] = my_lent;
    if (MODE == 1 && phase == PH_SIG) {
        // per-lane exponent range of the new level: reduced over the
        // workgroup in LDS, then one atomic per lane into the workgroup's slot
        if (active) {
            if (my_maxe != INT_MIN) atomicMax(&s_emax[lane], my_maxe);
            if (my_mine != INT_MAX) atomicMin(&s_emin[lane], my_mine);
        }
        __syncthreads();
        const int slot = (int)(bid % kSlots);
        if (tid < kLanes && s_emax[tid] != INT_MIN) atomicMax(&a.maxexp[slot * kLanes + tid], s_emax[tid]);
        else if (tid >= kLanes && tid < 2 * kLanes && s_emin[tid - kLanes] != INT_MAX)
            atomicMin(&a.maxexp[(kSlots + slot) * kLanes + tid - kLanes], s_emin[tid - kLanes]);
        // completed before this workgroup arrives (the last one reads them)
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
    }
    if (!step_epilogue(c, cn, s_red, &s_last, active, bid, grid)) return;
    collect_slots(c, s_tot, s_red);

    // ---- the last workgroup advances the state machine
    int action = 0;  // 1 = begin batch, 2 = advance level
    if (tid == 0) {
        c->st_steps += 1;
        c->st_arcs += s_tot[SC_ARCS];
        c->st_lane_arcs += s_tot[SC_LARCS];
        c->st_lane_entries += s_tot[SC_LENT];
        c->st_parcs[phase] += s_tot[SC_ARCS];
        c->st_plarcs[phase] += s_tot[SC_LARCS];
        c->st_ppairs[phase] += s_tot[SC_PAIRS];
        const unsigned long long now = wall_clock64();
        const unsigned long long prev_tick = c->last_tick;
        const unsigned long long dt = prev_tick ? now - prev_tick : 0ull;
        c->st_ticks[phase] += dt;
        if (phase == PH_FWD) c->st_vticks[s_variant] += dt;
        c->last_tick = now;
        const int rl = (phase == PH_FWD || phase == PH_BWD) ? l : (phase == PH_SIG ? l + 1 : -1);
        if (rl >= 0 && a.lvl) {
            LevelRec &r = level_rec(a.lvl, rl);
            r.arcs += s_tot[SC_ARCS];
            r.ticks += dt;
            if (phase == PH_FWD) {
                r.visits += 1;
                r.var[s_variant] += 1;
            }
        }
        bool timed_again = false;
        // one training sample: features x, device ticks t[0..2] at outputs k0..k0+2
        auto put_sample = [&](const float *x, const unsigned long long *t, int k0) {
            const uint32_t k = c->n_samples;
            if (k < a.col_cap) {
                for (int i = 0; i < kMlpIn; ++i) a.col_X[(size_t)k * kMlpIn + i] = x[i];
                for (int j = 0; j < kMlpOut; ++j)
                    a.col_Y[(size_t)k * kMlpOut + j] = (j >= k0 && j < k0 + 3) ? (float)t[j - k0] : -1.0f;
            }
            c->n_samples = k + 1;
        };
        if (phase == PH_FWD && c->collect) {
            c->ct[c->cvar] = c->last_tick ? now - prev_tick : 0ull;
            if (c->cvar < 2) {
                timed_again = true;  // undo, then run the level with the next variant
                c->phase = PH_UNDO;
                c->undo_sig = 0;
            } else {
                put_sample(c->feat, c->ct, kOutFwd);
                c->cvar = 0;
            }
        }
        if (phase == PH_SIG && c->collect) {
            // the path counts of level l+1 under each summation option (the
            // features are those of level l, which chose the option)
            c->ct_lb[c->clb] = dt;
            if (c->clb < 2) {
                timed_again = true;  // restore the level's words, then sum again
                c->phase = PH_UNDO;
                c->undo_sig = 1;
            } else {
                if (a.col_F && l < a.max_levels + 2) put_sample(a.col_F + (size_t)l * kMlpIn, c->ct_lb, kOutSig);
                c->clb = 0;
            }
        }
        if (phase == PH_BWD && c->collect) {
            // the backward step overwrites what it writes: run it again as is
            c->ct_lb[c->clb] = dt;
            if (c->clb < 2) {
                timed_again = true;
                c->clb += 1;
            } else {
                if (a.col_F && l < a.max_levels + 2) put_sample(a.col_F + (size_t)l * kMlpIn, c->ct_lb, kOutBwd);
                c->clb = 0;
            }
        }
        if (phase == PH_UNDO && c->undo_sig) {
            c->undo_sig = 0;
            c->clb += 1;
            c->phase = PH_SIG;
        } else if (phase == PH_UNDO) {
            c->next_qc = 0ull;
            c->next_hq = 0;
            c->cvar += 1;
            c->variant = c->cvar;
            c->phase = PH_FWD;
        } else if (timed_again) {
        } else if (phase == PH_FWD) {
            const unsigned long long qc = ld_agent(&c->next_qc);
            const uint32_t cnt = (uint32_t)qc, cost = (uint32_t)(qc >> 32);
            const unsigned long long nh = ld_agent(&c->next_hq);
            const int qe = a.level_off[l + 1];
            c->st_fwd_levels += 1;
            c->st_var[s_variant] += 1;
            c->st_qentries += cnt;
            if (a.lvl) level_rec(a.lvl, l + 1).entries += cnt;
            a.hq.off[l + 2] = a.hq.off[l + 1] + (int)(uint32_t)nh;
            a.hq.nseg[l + 1] = (int)(nh >> 32);
            c->next_hq = 0;
            if (cnt == 0) {
                const int L = l + 1;
                c->n_levels = L;
                if (MODE == 1 && c->f64_check) {
                    // counts below 2^65 might fit in 64 bits: hand the lane back
                    // (no contribution here), a 64-bit pass decides its mode
                    unsigned long long back = 0;
                    for (int k = 0; k < kLanes; ++k)
                        if (c->lane_emax[k] <= 65) back |= 1ull << k;
                    back &= c->lane_mask & ~c->dead;
                    const int64_t start = a.batch_start[c->pos];
                    for (unsigned long long o = back; o; o &= o - 1) {
                        const int k = __ffsll(o) - 1;
                        const uint32_t q = c->n_ovf;
                        if (q < a.ovf_cap) a.ovf_list[q] = start + k;
                        else c->err |= ERR_OVF_CAP;
                        c->n_ovf = q + 1;
                    }
                    c->dead |= back;
                }
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
                // close the groups of level l+1 (every entry costs >= 2 units)
                const uint32_t gb = a.gbase[l + 1];
                const uint32_t ng = (cost - 1u) / (uint32_t)kBudget + 1u;
                if ((unsigned long long)gb + ng + 1u > a.gcap) {
                    c->err |= ERR_QUEUE_CAP;
                    c->phase = PH_DONE;
                } else {
                    a.gstart[gb] = 0u;
                    a.gstart[gb + ng] = cnt;
                    a.gbase[l + 2] = gb + ng + 1u;
                    c->phase = PH_SIG;
                }
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
            // the next batch is set up by the last workgroup of a launch of
            // its own: this launch's workgroups have just cleared visited
            // words that the set-up writes again
            const int64_t next = c->pos + 1;
            c->pos = next;
            c->phase = next < c->n_items ? PH_FIN : PH_DONE;
        } else if (phase == PH_FIN) {
            action = 1;
        }
        s_cnt = action;
    }
    __syncthreads();
    action = s_cnt;
    if (action == 1) {
        batch_begin<MODE>(a, c, c->pos, s_lds, &s_feat, s_lsrc, &s_qn, s_tmp, s_lead);
    } else if (action == 2) {
        // finish level l+1: lane deaths, FP64 shifts, features, policy
        if (tid == 0) {
            const unsigned long long ovf = s_tot[SC_OVF] & ~c->dead;
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
            }
            c->active = s_tot[SC_ACT] & ~c->dead;
        }
        if (MODE && tid < kLanes) {
            int mx = INT_MIN, mn = INT_MAX;
            for (int sl = 0; sl < kSlots; ++sl) {
                mx = max(mx, ld_agent(&a.maxexp[sl * kLanes + tid]));
                mn = min(mn, ld_agent(&a.maxexp[(kSlots + sl) * kLanes + tid]));
                a.maxexp[sl * kLanes + tid] = INT_MIN;
                a.maxexp[(kSlots + sl) * kLanes + tid] = INT_MAX;
            }
            int sh = 0;
            if (mx != INT_MIN && mx > kExpHigh) sh = mx - kExpTarget;
            if (mn != INT_MAX && mn - sh < kExpLow) atomicOr(&c->err, ERR_SIGMA_RANGE);
            a.shift[(size_t)(l + 1) * kLanes + tid] = sh;
            // true counts of level l+1 are the stored ones times 2^lane_E
            if (mx != INT_MIN) c->lane_emax[tid] = max(c->lane_emax[tid], mx + c->lane_E[tid]);
            c->lane_E[tid] += sh;
        }
        if (tid == 0) {
            const uint32_t cnt = (uint32_t)ld_agent(&c->next_qc);
            const unsigned long long edges = s_tot[SC_EDGES];
            c->level = l + 1;
            c->visited_n += cnt;
            c->visited_m += edges;
            c->full_n += s_tot[SC_FULLN];
            c->full_m += s_tot[SC_FULLM];
            const unsigned long long fn = c->full_n, fm = c->full_m;
            s_feat.nf = (float)cnt;
            s_feat.mf = (float)edges;
            s_feat.nu = (float)((long long)c->range_nodeg - (long long)fn);
            s_feat.mu = (float)((long long)c->range_arcs - (long long)fm);
            s_feat.level = l + 1;
            c->next_qc = 0ull;
            c->prev_variant = c->variant;
            c->phase = PH_FWD;
        }
        __syncthreads();
        int lbo;
        const int v = choose_variant(a.p, c->policy, c->prev_variant, s_feat, (float)(c->range_hi - c->range_lo),
                                     (float)c->range_arcs, s_lds, &lbo);
        if (tid == 0)
            set_level_variant(a, c, v, lbo, s_feat, (float)(c->range_hi - c->range_lo), (float)c->range_arcs);
    }
}

template <int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(BC_WAVES))) void batch_step(BatchArgs a) {
    batch_step_body<MODE>(a, blockIdx.x, gridDim.x);
}

template __global__ void batch_step<0>(BatchArgs);
template __global__ void batch_step<1>(BatchArgs);

#ifndef BC_BLOCK_WAVES
#define BC_BLOCK_WAVES 2
#endif
// Block engine: a persistent launch in which every workgroup owns a level
// state machine.  A workgroup takes a chunk (batches [b0, b1) of one graph
// with vertices [lo, hi)), points the per-vertex arrays of its arguments at
// its private scratch shifted by lo (every index the steps use lies in
// [lo, hi): arcs never leave a graph), and runs the steps of the chunk one
// after another with workgroup barriers in between.  Scores of the chunk go
// to its own partial vector.  The control block keeps its tag epochs from
// chunk to chunk, so tags left by an earlier chunk never match.  Exit: the
// work queue runs dry (every workgroup takes chunks until the counter passes
// n_chunks), a step reports an error, or a chunk exceeds max_steps per batch.
template <int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(BC_BLOCK_WAVES))) void block_run(BlockArgs ra) {
    // the workgroup's arguments live in LDS: thread 0 points them at the
    // chunk's state, every thread reads them there
    __shared__ BatchArgs s_a;
    __shared__ int s_go;
    const int tid = threadIdx.x;
    Ctl *c = ra.ctls + blockIdx.x;
    char *base = ra.scratch + (size_t)blockIdx.x * ra.stride;
    const BlockLayout L((size_t)ra.nmax, ra.lq_cap, (size_t)ra.max_levels, ra.gcap, ra.hq_entries, ra.hq_levels,
                        ra.part_cap, ra.ovf_cap);
    if (tid == 0) {
        BatchArgs &a = s_a;
        a = ra.a;
        a.ctl = c;
        a.lvl = nullptr;
        a.lq_vtx = (int32_t *)(base + L.lq_vtx);
        a.lq_mask = (unsigned long long *)(base + L.lq_mask);
        a.lq_cap = ra.lq_cap;
        a.level_off = (int32_t *)(base + L.level_off);
        a.max_levels = ra.max_levels;
        a.gstart = (uint32_t *)(base + L.gstart);
        a.gbase = (uint32_t *)(base + L.gbase);
        a.lbsel = (int32_t *)(a.gbase + ra.max_levels + 2);
        a.gcap = ra.gcap;
        a.shift = (int32_t *)(base + L.shift);
        a.maxexp = (int32_t *)(base + L.maxexp);
        a.lane_src = (int32_t *)(base + L.lane_src);
        a.hq.pos = (int32_t *)(base + L.hq_pos);
        a.hq.seg = (int32_t *)(base + L.hq_seg);
        a.hq.cnt = (int32_t *)(base + L.hq_cnt);
        a.hq.off = (int32_t *)(base + L.hq_off);
        a.hq.nseg = (int32_t *)(base + L.hq_nseg);
        a.hq.cap = ra.hq_entries;
        a.hq.part_lo = (unsigned long long *)(base + L.part_lo);
        a.hq.part_hi = (unsigned long long *)(base + L.part_hi);
        a.hq.part_cap = ra.part_cap;
        a.ovf_list = (int64_t *)(base + L.ovf);
        a.ovf_cap = ra.ovf_cap;
        a.dump_d = nullptr;
        a.dump_sig = nullptr;
        a.dump_delta = nullptr;
        a.dump_shift = nullptr;
        a.col_X = nullptr;
        a.col_Y = nullptr;
        a.col_cap = 0;
    }
    int32_t *mx = (int32_t *)(base + L.maxexp);
    for (int i = tid; i < 2 * kSlots * kLanes; i += kBlock) mx[i] = i < kSlots * kLanes ? INT_MIN : INT_MAX;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            const uint32_t k = atomicAdd(ra.next, 1u);
            const int t = (k < (uint32_t)ra.n_chunks && c->err == 0) ? ra.order[k] : -1;
            s_go = t;
            if (t >= 0) {
                const int b0 = ra.c_b0[t], b1 = ra.c_b1[t];
                const int lo = ra.a.batch_lo[b0], hi = ra.a.batch_hi[b0];
                BatchArgs &a = s_a;
                a.vn = (VisNext *)(base + L.vn) - lo;
                a.fw0 = (Tagged *)(base + L.fw0) - lo;
                a.fw1 = (Tagged *)(base + L.fw1) - lo;
                a.sigma = (unsigned long long *)(base + L.sigma) - (size_t)lo * kLanes;
                a.chat = (double *)(base + L.chat) - (size_t)lo * kLanes;
                a.delta = (double *)(base + L.delta) - (size_t)lo * kLanes;
                a.bc = ra.partials + ra.c_part[t] - lo;
                // the first step (phase BC of an empty batch) clears the
                // visited words of [lo, hi), then the chunk's batches follow
                c->phase = PH_BC;
                c->pos = (int64_t)b0 - 1;
                c->n_items = b1;
                c->range_lo = lo;
                c->range_hi = hi;
                c->lane_mask = 0ull;
                c->dead = 0ull;
                c->active = 0ull;
                c->level = 0;
            }
        }
        __syncthreads();
        const int t = s_go;
        if (t < 0) break;
        const int b0 = ra.c_b0[t], b1 = ra.c_b1[t];
        const int lo = ra.a.batch_lo[b0], hi = ra.a.batch_hi[b0];
        double *part = ra.partials + ra.c_part[t];
        for (int i = tid; i < hi - lo; i += kBlock) part[i] = 0.0;
        const int64_t max_steps = (int64_t)(b1 - b0 + 1) * ra.max_steps;
        for (int64_t step = 0;; ++step) {
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0) {
                int go = (c->phase != PH_DONE && c->err == 0) ? 1 : 0;
                if (go && step >= max_steps) {
                    c->err |= ERR_LEVEL_CAP;
                    go = 0;
                }
                s_go = go;
            }
            __syncthreads();
            if (!s_go) break;
            batch_step_body<MODE>(s_a, 0u, 1u);
        }
    }
}

template __global__ void block_run<0>(BlockArgs);

}  // namespace bcx
