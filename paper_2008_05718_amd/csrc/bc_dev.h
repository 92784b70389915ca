// bc_dev.h -- device-side structures shared by the libbc kernels and the host
// driver.  Internal to libbc (not part of the public C ABI in include/bc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bcx {

constexpr int kBlock = 256;  // threads per workgroup of every step kernel
constexpr int kWave = 64;    // CDNA wavefront width
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kLanes = 64;   // sources per batch = wavefront lanes
constexpr int kLightDeg = 32;  // thread-per-vertex loops handle up to this many arcs
#ifndef BC_SEG
#define BC_SEG 1024
#endif
#ifndef BC_SEG_PLAIN
#define BC_SEG_PLAIN 512
#endif
// heavy vertices (degree > kSeg) are split into kSeg-arc segments; each
// engine has its own size (the plain engine is compiled with BC_PLAIN_TU)
constexpr int kSegBatched = BC_SEG;
constexpr int kSegPlain = BC_SEG_PLAIN;
#ifdef BC_PLAIN_TU
constexpr int kSeg = kSegPlain;
#else
constexpr int kSeg = kSegBatched;
#endif
constexpr int kPhases = 10;
// Scaled FP64 path counts (mode 1): a level whose largest binary exponent
// exceeds kExpHigh is divided by a power of two that brings it to kExpTarget,
// so a sum over fewer than 2^31 predecessors stays below 2^932.  Its
// smallest count must then stay at or above 2^kExpLow: c = (1 + delta) /
// sigma with delta < 2^31 then stays below 2^1021 (a wider spread within
// one level is reported as a range error).
constexpr int kExpHigh = 960, kExpTarget = 900, kExpLow = -990;
constexpr int kSlots = 32;     // per-step counters and arrivals are spread over this many slots

// Counters every step kernel accumulates per workgroup into its slot.
enum : int {
    SC_EDGES = 0,  // arcs of newly appended vertices (sum)
    SC_ARCS,       // adjacency entries scanned (sum)
    SC_LARCS,      // (arc, source) pairs on shortest-path DAGs (sum)
    SC_FULLN,      // vertices newly visited in every lane (sum)
    SC_FULLM,      // their arcs (sum)
    SC_ACT,        // lanes present in the new level (or)
    SC_OVF,        // lanes / sources whose path counts overflowed (or)
    SC_MAXE,       // max binary exponent + 4096 (max)
    SC_MINE,       // 4096 - min binary exponent (max)
    SC_PAIRS,      // matched (vertex, neighbour) pairs whose per-source rows were read (sum)
    SC_LENT,       // (vertex, source) pairs of the entries appended (sum)
    kNCnt
};

// Phases of the device-resident state machine.  One launch of a step kernel
// performs the work of the current phase; the last workgroup to finish moves
// the machine to the next phase.
enum : int32_t {
    PH_IDLE = 0,
    PH_FWD = 1,      // discover level l+1 from the frontier at level l
    PH_SIG = 2,      // path counts of level l+1 (pull, fixed summation order)
    PH_BWD = 3,      // dependencies of level l (pull from level l+1)
    PH_FIN = 4,      // plain: reset the visited set, start the next source; batched: set up the next batch
    PH_BC = 5,       // batched: add dependencies to BC in source order, reset
    PH_DUMP_FWD = 6, // copy one source's d / sigma out (detail runs only)
    PH_DUMP_BWD = 7, // copy one source's delta out (detail runs only)
    PH_DONE = 8,
    PH_UNDO = 9,     // timing collection: clear the level just discovered
};

enum : int32_t { V_PUSH_TPV = 0, V_PUSH_WPV = 1, V_PULL = 2 };
enum : int32_t { POL_HEUR = 1, POL_MLP = 2, POL_FORCE_TPV = 3, POL_FORCE_WPV = 4, POL_FORCE_PULL = 5 };

// Policy network: kMlpIn level features -> 32 -> 32 -> kMlpOut predicted
// log2 times.  Outputs 0-2: the discover variants (V_*); 3-5: the path-count
// step of the entries discovered next, 6-8: the backward step of the
// level's entries, each under the three summation options (LB_*).
constexpr int kMlpIn = 5, kMlpH = 32, kMlpOut = 9;
constexpr int kOutFwd = 0, kOutSig = 3, kOutBwd = 6;
// How path-count and backward groups sum their light entries: one wavefront
// lane per source always (packed), by the run's sources-per-entry rule, or
// one thread per (entry, source) pair always.  Same bits every way.
enum : int32_t { LB_PACKED = 0, LB_RULE = 1, LB_ITEMS = 2 };
constexpr int32_t kLbDefault = LB_RULE | (LB_RULE << 2);  // sig option | bwd option << 2
// default override margin of the learned policy (log2 units, about 11 %):
// learned over heuristic on the damaged grid 0.961 without a margin, 0.970
// at 0.07, 0.983 at 0.15, 0.996 at 0.30; on R-MAT 22 1.011, 1.015, 1.011, 1.006
constexpr float kPolicyMargin = 0.15f;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpOut * kMlpH + kMlpOut;

// Control block in device memory.  Written by the host before a run, then
// only by the last workgroup of each step launch.
struct Ctl {
    // --- polled by the host after every chunk of launches (keep first)
    int32_t phase;
    int32_t err;          // sticky device error bits (capacity, range)
    // --- progress
    int64_t pos;          // plain: index of the current source; batched: current batch
    int64_t n_items;      // plain: number of sources; batched: number of batches
    int32_t level;        // current level l
    int32_t n_levels;     // levels of the finished forward (L)
    int32_t variant;      // discover variant of the current level
    int32_t prev_variant;
    int32_t policy;
    int32_t mode;         // 0 = uint64 path counts, 1 = scaled FP64
    int32_t lanes;        // batched: sources in the current batch
    uint32_t epoch;       // batched: tag base of the current forward
    uint32_t epoch_b;     // batched: tag base of the current backward
    int32_t range_lo;     // batched: vertex range of the current batch's graph
    int32_t range_hi;
    unsigned long long lane_mask;   // valid lanes of the batch
    unsigned long long active;      // lanes with a non-empty frontier at level l
    unsigned long long dead;        // lanes that overflowed in uint64 mode
    // --- level under construction (atomics)
    uint32_t blocks_done;
    unsigned long long next_qc;  // appends to the next level: entries (low 32 bits), cost units (high 32)
    unsigned long long next_edges;
    unsigned long long next_active;
    unsigned long long ovf_lanes;
    int32_t overflow;     // plain: the current source overflowed
    int32_t maxexp;       // plain FP64: max binary exponent of the level built
    int32_t minexp;
    uint32_t total_queued;
    uint32_t n_ovf;       // overflowed sources recorded
    // --- features of the frontier at level l
    unsigned long long f_nf, f_mf, visited_n, visited_m, full_n, full_m;
    unsigned long long range_nodeg, range_arcs;  // non-isolated vertices / arcs of the range
    // --- timing collection (policy training data)
    int32_t collect;      // 1 = run every forward level with each variant, every path-count
                          // and backward step with each summation option
    int32_t cvar;         // variant being timed
    int32_t clb;          // summation option being timed (path-count and backward steps)
    int32_t undo_sig;     // the pending undo step restores a path-count step, not a discover step
    unsigned long long ct[3];
    unsigned long long ct_lb[3];
    float feat[kMlpIn];   // normalised features of the level being timed
    uint32_t n_samples;
    // --- detail dump
    int64_t dump_pos;     // source position to dump (-1 = none)
    int32_t dump_lane;    // batched: lane of the dumped source in its batch
    int32_t dump_state;   // 0 = pending, 1 = forward dumped, 2 = done
    int32_t f64_check;    // batched FP64 pass: hand back lanes whose counts stay below 2^65
    int32_t lane_E[64];   // batched FP64: power of two of the current level's stored counts, per lane
    int32_t lane_emax[64];  // batched FP64: largest binary exponent of a true count so far, per lane
    // --- heavy entries of the level under construction: count | segments << 32
    unsigned long long next_hq;
    // --- per-slot counters and workgroup arrivals of the running step
    unsigned long long slot[kSlots][kNCnt];
    uint32_t arrive[kSlots];
    uint32_t work[kSlots][32];  // per-slot work counters, one 128-byte line each
    // --- statistics
    unsigned long long st_steps, st_fwd_levels, st_var[3], st_arcs, st_lane_arcs, st_qentries,
        st_max_levels, st_batches;
    unsigned long long st_lane_entries;      // (vertex, source) pairs reached, level 0 included
    unsigned long long last_tick;            // wall clock at the end of the previous step
    unsigned long long st_ticks[kPhases];    // wall-clock ticks spent per phase
    unsigned long long st_vticks[3];         // forward (discover) ticks per variant
    unsigned long long st_parcs[kPhases];    // arcs scanned per phase
    unsigned long long st_plarcs[kPhases];   // DAG (arc, source) pairs per phase
    unsigned long long st_ppairs[kPhases];   // matched neighbour rows per phase
};

enum : int32_t { ERR_QUEUE_CAP = 1, ERR_SIGMA_RANGE = 2, ERR_LEVEL_CAP = 4, ERR_OVF_CAP = 8 };

// Per-level record of a run (statistics): index = distance from the source;
// levels at or beyond kLevelRecs - 1 share the last record.  Written only by
// the last workgroup of a step launch.
constexpr int kLevelRecs = 65538;
struct LevelRec {
    unsigned long long visits;   // forward steps at this level (batches or sources that reached it)
    unsigned long long entries;  // level-queue entries of this level
    unsigned long long arcs;     // adjacency entries scanned by this level's steps, all phases
    unsigned long long var[3];   // forward steps of this level per discover variant
    unsigned long long ticks;    // device clock ticks of this level's steps, all phases
    unsigned long long pad;
};
__device__ __forceinline__ LevelRec &level_rec(LevelRec *r, int l) { return r[l < kLevelRecs ? l : kLevelRecs - 1]; }

// Read-only graph description passed to every kernel.
struct GraphArgs {
    int32_t n;
    int32_t nnz_lo;         // nnz fits int32 by construction
    const int32_t *row_ptr; // int32[n+1]
    const int32_t *col;     // int32[nnz]
    int64_t nonisolated;    // vertices with degree >= 1
    // vertices of degree > kSeg in ascending order, and the exclusive prefix
    // sum of their segment counts (hv_seg[n_heavy] = all segments)
    const int32_t *hv_vtx;
    const int32_t *hv_seg;
    int32_t n_heavy;
    // Directed graphs: row_ptr / col hold the out-arcs and these the in-arcs
    // (the transpose).  Undirected graphs point both at the one symmetric
    // adjacency.
    const int32_t *in_row_ptr;
    const int32_t *in_col;
    int32_t directed;
};

// Heavy entries of the level queues (vertices of degree > kSeg), per level:
// entries hq_off[l] .. hq_off[l+1]; hq_seg holds each entry's first segment
// relative to its level, hq_nseg[l] the level's segment count.
struct HeavyQ {
    int32_t *pos;            // queue position of the entry
    int32_t *seg;            // first segment (relative to the level)
    int32_t *cnt;            // arrival counter of the entry's segments
    int32_t *off;            // [max_levels + 2]
    int32_t *nseg;           // [max_levels + 2]
    uint32_t cap;
    unsigned long long *part_lo;  // [segments][lanes] partial sums
    unsigned long long *part_hi;
    uint32_t part_cap;       // segments the partial buffers hold
};

struct PolicyArgs {
    float alpha, beta, wpv_degree;
    float item_lanes;       // path-count / backward groups whose light entries carry at most this many
                            // sources on average run one thread per (entry, source) pair
    float margin;           // learned policy: predicted log2 gain needed to override the rule (0 = none)
    int32_t has_mlp;
    const float *mlp;       // kMlpParams floats (device), or nullptr
};

// Plain engine (one source at a time, whole GPU per level).
struct PlainArgs {
    GraphArgs g;
    PolicyArgs p;
    Ctl *ctl;
    int32_t *d;              // int32[n], -1 = unvisited (kept -1 between sources)
    unsigned long long *sig; // uint64[n] or FP64 bits (mode 1); kept 0 between sources
    double *chat;            // FP64[n] scaled (1 + delta) / sigma
    double *bc;              // FP64[n]
    int32_t *queue;          // int32[n]: all levels of the current source
    int32_t *level_off;      // int32[n + 2]
    int32_t *shift;          // int32[n + 2]: per-level exponent shift (mode 1)
    const int32_t *srcs;     // sources of this run
    int64_t *ovf_list;       // positions of sources that overflowed uint64
    uint32_t ovf_cap;
    unsigned long long sigma_limit;
    // detail dump (host-pinned or device buffers of length n)
    int32_t *dump_d;
    unsigned long long *dump_sig;
    double *dump_delta;
    int32_t *dump_shift;     // per-level shifts of the dumped source
    HeavyQ hq;
    LevelRec *lvl;           // [kLevelRecs]
};

// Tagged frontier word: lanes of vertex v that sit on level (tag - epoch).
struct __attribute__((aligned(16))) Tagged {
    unsigned long long mask;
    uint32_t tag;
    uint32_t pad;
};
// Visited / next lane words of a vertex, one 16-byte load.
struct __attribute__((aligned(16))) VisNext {
    unsigned long long vis;
    unsigned long long nxt;
};

// Batched engine (64 sources per traversal, one wavefront lane per source).
struct BatchArgs {
    GraphArgs g;
    PolicyArgs p;
    Ctl *ctl;
    VisNext *vn;                 // [n]
    Tagged *fw0, *fw1;           // [n] each; level parity selects the buffer
    int32_t *lq_vtx;             // level queues: vertex
    unsigned long long *lq_mask; // level queues: lane mask
    uint32_t lq_cap;
    int32_t *level_off;          // [max_levels + 2]
    int32_t max_levels;
    double *delta;               // [n][64] dependencies (read by PH_BC and dumps)
    unsigned long long *sigma;   // [n][64] path counts (uint64, or FP64 bits in mode 1)
    double *chat;                // [n][64] c = (1 + delta) / sigma
    int32_t *shift;              // [max_levels + 2][64] (mode 1)
    int32_t *maxexp;             // [2][kSlots][64]: per-slot, per-lane max then min exponents (mode 1)
    double *bc;                  // [n]
    const int32_t *srcs;         // source list of this run
    const int64_t *batch_start;  // [n_batches + 1] positions into srcs
    const int32_t *batch_lo;     // [n_batches] vertex range of each batch's graph
    const int32_t *batch_hi;
    int32_t *lane_src;           // [64] sources of the current batch
    int64_t *ovf_list;
    uint32_t ovf_cap;
    unsigned long long sigma_limit;
    int32_t *dump_d;
    unsigned long long *dump_sig;
    double *dump_delta;
    int32_t *dump_shift;         // [max_levels + 2]
    HeavyQ hq;
    float *col_X;                // collected features [cap][kMlpIn]
    float *col_Y;                // collected device ticks [cap][kMlpOut], -1 = not timed
    float *col_F;                // features of every level of the batch [max_levels + 2][kMlpIn]
    uint32_t col_cap;
    uint32_t *gstart;            // group starts of every level of the batch (see GroupArgs)
    uint32_t *gbase;             // [max_levels + 2]: first gstart slot of each level
    int32_t *lbsel;              // [max_levels + 2]: summation options chosen at each level
                                 // (path-count option | backward option << 2)
    uint32_t gcap;
    LevelRec *lvl;               // [kLevelRecs]
};

// ---------------------------------------------------------- block engine
// Unions of small graphs (and single small graphs): every workgroup runs the
// batched state machine on its own (one workgroup per launch in effect, so
// steps are separated by workgroup barriers, not by launches) over chunks of
// consecutive batches of one graph that it takes from a work queue, for the
// whole run in one persistent launch.  Each workgroup owns a private copy of
// the per-vertex state, sized for the largest graph it may hold; a chunk's
// scores go to a partial vector of its own, and the partials of a graph are
// added in chunk order afterwards.
constexpr int kBlockMaxN = 131072;  // largest graph (vertices) the block engine takes

// Byte offsets of one workgroup's state inside its scratch region; the same
// arithmetic on the host (sizing) and on the device (carving).
struct BlockLayout {
    size_t vn, fw0, fw1, lq_vtx, lq_mask, level_off, sigma, chat, delta, gstart, gbase, shift, maxexp, lane_src,
        hq_pos, hq_seg, hq_cnt, hq_off, hq_nseg, part_lo, part_hi, ovf, bytes;
    __host__ __device__ static size_t up(size_t x) { return (x + 255) & ~(size_t)255; }
    __host__ __device__ BlockLayout(size_t nmax, size_t lq_cap, size_t max_levels, size_t gcap, size_t hq_entries,
                                    size_t hq_levels, size_t part_cap, size_t ovf_cap) {
        size_t o = 0;
        auto take = [&](size_t bytes) { const size_t at = o; o = up(o + bytes); return at; };
        vn = take(nmax * sizeof(VisNext));
        fw0 = take(nmax * sizeof(Tagged));
        fw1 = take(nmax * sizeof(Tagged));
        lq_vtx = take(lq_cap * 4);
        lq_mask = take(lq_cap * 8);
        level_off = take((max_levels + 2) * 4);
        sigma = take(nmax * kLanes * 8);
        chat = take(nmax * kLanes * 8);
        delta = take(nmax * kLanes * 8);
        gstart = take(gcap * 4);
        gbase = take((max_levels + 2) * 4 * 2);  // group bases, then the level's summation options
        shift = take((max_levels + 2) * kLanes * 4);
        maxexp = take(2 * kSlots * kLanes * 4);
        lane_src = take(kLanes * 4);
        hq_pos = take(hq_entries * 4);
        hq_seg = take(hq_entries * 4);
        hq_cnt = take(hq_entries * 4);
        hq_off = take(hq_levels * 4);
        hq_nseg = take(hq_levels * 4);
        part_lo = take(part_cap * kLanes * 8);
        part_hi = take(part_cap * kLanes * 8);
        ovf = take(ovf_cap * 8);
        bytes = o;
    }
};

struct BlockArgs {
    BatchArgs a;                 // graph, policy, source list and batch table of the run
    char *scratch;               // per-workgroup state, `stride` bytes each (BlockLayout)
    size_t stride;
    Ctl *ctls;                   // one control block per workgroup
    int32_t nmax;
    uint32_t lq_cap, gcap, hq_entries, hq_levels, part_cap, ovf_cap;
    int32_t max_levels;
    // chunk t: batches [c_b0[t], c_b1[t]) of one graph; its partial scores
    // are partials[c_part[t] + (v - lo)]
    const int32_t *c_b0, *c_b1;
    const int64_t *c_part;
    const int32_t *order;        // chunks in dispatch order (largest graphs first)
    int32_t n_chunks;
    uint32_t *next;              // work-queue counter
    double *partials;
    int64_t max_steps;           // per batch: a bound no valid run reaches
};

// ------------------------------------------------------- weighted engine
// (bc_weighted.hip) One workgroup's state for a graph of n vertices, and the
// arguments of the persistent launch.
struct WeightedLayout {
    size_t dist, sig, chat, dep, cnt, mark, reached, qa, qb, lvl, lvl_off, bytes;
    __host__ __device__ static size_t up(size_t x) { return (x + 255) & ~(size_t)255; }
    __host__ __device__ explicit WeightedLayout(size_t n) {
        size_t o = 0;
        auto take = [&](size_t b) { const size_t at = o; o = up(o + b); return at; };
        dist = take(n * 8);
        sig = take(n * 8);
        chat = take(n * 8);
        dep = take(n * 8);
        cnt = take(n * 4);
        mark = take(n * 4);
        reached = take(n * 4);
        qa = take(n * 4);
        qb = take(n * 4);
        lvl = take(n * 4);
        lvl_off = take((n + 2) * 4);
        bytes = o;
    }
};

struct WeightedArgs {
    GraphArgs g;
    const int32_t *wt;        // weights of the out-arcs (aligned with g.col)
    const int32_t *in_wt;     // weights of the in-arcs (aligned with g.in_col)
    const int32_t *srcs;      // source list of the pass
    const int64_t *pos;       // absolute positions of the pass's sources in the run (for the overflow list)
    const int32_t *c_s0, *c_s1;  // chunk t: pass positions [c_s0[t], c_s1[t])
    const int32_t *order;     // chunks in dispatch order
    int32_t n_chunks;
    uint32_t *next;           // work-queue counter
    double *partials;         // chunk t: partials[t * n .. (t + 1) * n)
    char *scratch;            // per-workgroup state, `stride` bytes each
    size_t stride;
    int32_t *err;             // ERR_* bits
    int64_t *ovf_list;        // positions whose path counts overflowed (MODE 0)
    uint32_t *ovf_count;
    uint32_t ovf_cap;
    unsigned long long sigma_limit;
    int64_t dump_pos;         // pass position whose d / sigma / delta are copied out (-1 = none)
    int64_t *dump_d;
    unsigned long long *dump_sig;
    double *dump_delta;
    unsigned long long *st;   // statistics: [0] relaxation rounds, [1] arcs scanned, [2] DAG rounds,
                              // [3] reached pairs, [4] DAG-pass arcs, [5] relaxation (arc, source)
                              // pairs, [6] DAG-pass (arc, source) pairs, [7..9] clock ticks of the
                              // three phases, [10] longest batch (the last six: lane batches)
};

}  // namespace bcx
