/*
 * bc.h -- C ABI of libbc, exact Brandes betweenness centrality on one
 * AMD Instinct MI355X (gfx950).
 *
 * What is computed (Mishra, Vadhiyar, Nasre, Pingali, "A Fine-Grained Hybrid
 * CPU-GPU Algorithm for Betweenness Centrality Computations", Section
 * "Background"):
 *   Eq. 1   BC[v] = sum over s != v != t of sigma_st(v) / sigma_st,
 *   Eq. 2   delta_s(v) = sum over successors u of v of
 *                        sigma_sv / sigma_su * (1 + delta_s(u)),
 *           BC[v] = sum over sources s != v of delta_s(v),
 * evaluated with the level-synchronous forward phase (distances d and path
 * counts sigma) and the level-by-level backward phase of the algorithm figure
 * "Betweenness Centrality Algorithm".  Input graphs are undirected and
 * unweighted (Section "Experiments and Results" converts every graph to an
 * undirected one), stored as CSR (Section "Space Complexity").
 *
 * Conventions for every entry point:
 *   - Every call returns a bc_status; no exception or abort crosses the ABI.
 *     bc_last_error() returns a thread-local text for the last failure.
 *   - Output buffers are left untouched on error.
 *   - A handle is not re-entrant: calls on one handle must not overlap.
 *     Separate handles are independent.  After BC_ERR_DEVICE the handle must
 *     be destroyed; after argument errors it stays usable.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it and the call returns once that work is complete.
 */
#ifndef BC_H
#define BC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bc_status {
    BC_OK = 0,
    BC_ERR_INVALID_ARG = 1,    /* bad pointer, size, source id or option   */
    BC_ERR_INVALID_GRAPH = 2,  /* CSR fails validation (see bc_graph_create) */
    BC_ERR_OUT_OF_MEMORY = 3,  /* device allocation failed, or over bc_set_device_limit's cap */
    BC_ERR_DEVICE = 4,         /* a HIP call failed; destroy the handle     */
    BC_ERR_SIGMA_RANGE = 5,    /* scaled FP64 path counts left the double range */
    BC_ERR_NOT_SUPPORTED = 6
} bc_status;

typedef struct bc_graph bc_graph;

/* Name of a status code, and the thread-local text of the last failure. */
const char *bc_status_string(bc_status s);
const char *bc_last_error(void);

/* ------------------------------------------------------------------ graph */

/* bc_graph_create flags */
#define BC_INPUT_DEVICE        0x1u  /* row_ptr / col_idx are device pointers   */
#define BC_SKIP_SYMMETRY_CHECK 0x2u  /* caller guarantees symmetric arcs        */
#define BC_KEEP_ORDER          0x4u  /* no internal hub-first relabelling        */
#define BC_DIRECTED            0x8u  /* arcs are directed (see below)            */

/*
 * Build a graph handle from a CSR adjacency (Section "Space Complexity":
 * offsets plus adjacency arrays).
 *   n        number of vertices, 0 <= n < 2^31 - 1.
 *   nnz      number of stored arcs; each undirected edge is stored twice.
 *            nnz <= 2^31 - 1.
 *   row_ptr  int32[n + 1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz.
 *   col_idx  int32[nnz]; the neighbours of v are col_idx[row_ptr[v] ..
 *            row_ptr[v+1]), strictly ascending (no duplicates), in [0, n),
 *            never v itself (no self-loops), and symmetric: w is a neighbour
 *            of v iff v is a neighbour of w.
 *   flags    bits above.
 * Ownership: the arrays are copied into library-owned device memory; the
 * caller may free them on return.  Validation runs on the device.
 * Internally the vertices of each graph are renumbered hub-first (degree at
 * least twice the graph's mean, by decreasing degree; the others keep their
 * order) unless BC_KEEP_ORDER is given, so that the frontier words and
 * rows of the most-read vertices share cache lines.  Such a handle also
 * takes the sources of a run in its own order: by graph, then by hop
 * distance from the graph's vertex of largest degree, then by parent in
 * that vertex's BFS tree, then by decreasing degree (stable), so that the
 * sources of one batch reach most vertices at the same depth.  Every call of this interface takes and returns the
 * caller's vertex ids and source positions; only the order in which
 * floating-point terms of a sum are added can differ.
 * Directed graphs (BC_DIRECTED): the paper converts every input to an
 * undirected graph (Section "Experiments and Results"), but Eq. 1 and Eq. 2
 * are defined for paths that follow arcs, so a directed graph is accepted
 * as well: col_idx[row_ptr[v] .. row_ptr[v+1]) are the heads of the arcs
 * leaving v (strictly ascending, no self-loops, no symmetry required).  The
 * library builds the in-arcs itself; the forward phase pushes over out-arcs
 * and pulls (discovery, path counts) over in-arcs, the backward phase pulls
 * dependencies from successors over out-arcs.  Such a handle keeps the
 * caller's numbering; unless BC_KEEP_ORDER is given it ranks the sources
 * like an undirected handle (hop distance along out-arcs from the vertex of
 * largest out-degree, ...).  It always runs the batched engine (batch = 1
 * means one source per traversal there).
 * Scores are raw sums over ordered pairs, as for undirected graphs.
 * Errors: BC_ERR_INVALID_ARG (NULL pointers, negative sizes),
 * BC_ERR_INVALID_GRAPH (validation failure; bc_last_error names the rule),
 * BC_ERR_OUT_OF_MEMORY, BC_ERR_DEVICE.  *out is set only on success.
 */
bc_status bc_graph_create(int32_t n, int64_t nnz, const int32_t *row_ptr,
                          const int32_t *col_idx, uint32_t flags, bc_graph **out);

/*
 * Weighted graph: as bc_graph_create, plus int32 arc weights aligned with
 * col_idx (host, or device with BC_INPUT_DEVICE like the CSR).  The paper's
 * forward phase is "a BFS traversal or SSSP calculation" (Section
 * "Background") and its layout keeps edge weights (Section "Space
 * Complexity"): shortest paths minimise the sum of weights.  Every weight
 * must be >= 1 (exact integer distances, so equal lengths are recognised
 * exactly); an undirected graph must carry the same weight on both arcs of
 * an edge (else BC_ERR_INVALID_GRAPH).  BC_DIRECTED is accepted (the library
 * builds the in-arcs and their weights).  The handle keeps the caller's
 * numbering; unless BC_KEEP_ORDER is given it still takes the sources of a
 * run in the ranked order described for bc_graph_create (by hop distance
 * from the vertex of largest degree, ...).  It runs the weighted engine: a
 * persistent launch in which every
 * workgroup computes whole batches of 16 sources, or single sources
 * (bc_run_options.weighted_lanes), (distances by relaxation rounds, path
 * counts over the shortest-path DAG in rounds of ready vertices, Eq. 2 over
 * those rounds in reverse); uint64 path counts, redone in FP64 (unscaled; a
 * count beyond the double range gives BC_ERR_SIGMA_RANGE) for sources whose
 * counts overflow.  Run options other than flags, sigma_limit and weighted_lanes
 * are ignored.
 * bc_run_detail reports distances in bc_detail.d64.
 */
bc_status bc_graph_create_weighted(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                   const int32_t *weights, uint32_t flags, bc_graph **out);

/*
 * Block-diagonal union of n_graphs independent graphs, one handle.  Graph g
 * owns vertices [vtx_offsets[g], vtx_offsets[g+1]); vtx_offsets is host
 * int32[n_graphs + 1] with vtx_offsets[0] = 0 and vtx_offsets[n_graphs] = n.
 * No arc may cross a block boundary (BC_ERR_INVALID_GRAPH otherwise).  Since
 * the components are independent, the BC of the union restricted to block g
 * equals the BC of graph g; batches of sources never mix graphs.  Other
 * arguments as in bc_graph_create, except that BC_DIRECTED is refused
 * (BC_ERR_NOT_SUPPORTED) when n_graphs > 1.
 */
bc_status bc_graph_create_multi(int32_t n_graphs, const int32_t *vtx_offsets, int32_t n,
                                int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                                uint32_t flags, bc_graph **out);

/* NULL-safe.  Frees every device and host resource of the handle. */
void bc_destroy(bc_graph *g);

/* Basic facts: n, nnz, number of graphs, bytes of device memory held (the
 * handle and the concurrent replicas or sub-unions it created). */
bc_status bc_graph_info(const bc_graph *g, int32_t *n, int64_t *nnz, int32_t *n_graphs,
                        int64_t *device_bytes);

/*
 * Cap on the device memory the handle may hold: its graph arrays, engine
 * state (allocated at the first run of each engine, then kept), per-run
 * buffers, and the concurrent replicas or sub-unions a run would create.
 * max_device_bytes = 0 removes the cap (the default).  An allocation that
 * would take the handle past the cap fails with BC_ERR_OUT_OF_MEMORY before
 * any device memory is requested (the handle stays usable); concurrent
 * replicas or sub-unions that would not fit are not created, and the run
 * uses one level state machine instead (same results to rounding; see
 * BC_RUN_ONE_QUEUE).  Concurrent parts already created that exceed a new
 * cap are released.  Errors: BC_ERR_INVALID_ARG (NULL g, negative cap).
 */
bc_status bc_set_device_limit(bc_graph *g, int64_t max_device_bytes);

/* -------------------------------------------------------------------- run */

/* Direction / load-balancing variants of one forward level. */
#define BC_VARIANT_PUSH_TPV 0  /* top-down, one thread per frontier vertex   */
#define BC_VARIANT_PUSH_WPV 1  /* top-down, one 64-lane wavefront per vertex */
#define BC_VARIANT_PULL     2  /* bottom-up over unvisited vertices          */

/* Level policies (bc_run_options.policy). */
#define BC_POLICY_AUTO       0 /* MLP when weights are loaded, else heuristic */
#define BC_POLICY_HEURISTIC  1 /* direction-optimising alpha/beta rule        */
#define BC_POLICY_MLP        2 /* learned switch; BC_ERR_INVALID_ARG if no weights */
#define BC_POLICY_FORCE_PUSH_TPV 3
#define BC_POLICY_FORCE_PUSH_WPV 4
#define BC_POLICY_FORCE_PULL     5

/* bc_run_options.flags */
#define BC_RUN_ACCUMULATE  0x1u  /* add to the existing scores instead of resetting */
#define BC_RUN_NO_GRAPHS   0x2u  /* launch level steps one by one, no hipGraph  */
#define BC_RUN_FORCE_F64   0x4u  /* test hook: evaluate every source in FP64 mode */
#define BC_RUN_ONE_QUEUE   0x10u /* a handle over many graphs: run every batch on one
                                    level state machine instead of concurrent parts */
#define BC_RUN_BLOCKS      0x20u /* batched work of graphs of at most 131072 vertices runs on
                                    the block engine (one persistent launch; every workgroup
                                    owns whole batches) even for short source lists       */
#define BC_RUN_NO_BLOCKS   0x40u /* never use the block engine                               */
#define BC_RUN_TUNED       0x8u  /* K, policy, workgroups, chunk and WPV threshold left
                                    automatic (zero) come from bc_autotune's result */

typedef struct bc_run_options {
    uint32_t flags;
    int32_t batch;        /* K: 0 = autotuned, 1 = plain per-source engine,
                             8/16/32/64 = sources traversed together        */
    int32_t policy;       /* BC_POLICY_*                                     */
    float alpha;          /* top-down -> bottom-up when m_f > m_u / alpha (0 = 14) */
    float beta;           /* bottom-up -> top-down when n_f < n / beta   (0 = 24) */
    float wpv_degree;     /* push uses WPV when mean frontier degree > this (0 = 24) */
    int32_t grid_blocks;  /* workgroups per step launch (0 = autotuned)      */
    int32_t chunk_steps;  /* level steps per captured hipGraph (0 = default) */
    int64_t sigma_limit;  /* test hook: treat path counts above this as overflow
                             (0 = none, i.e. 2^64 - 1)                       */
    float lanes_per_entry;/* batched path-count and backward steps: a group of level
                             entries whose entries carry at most this many sources
                             on average is summed one thread per (entry, source)
                             pair instead of one wavefront lane per source
                             (0 = default 4; negative = never).  Same results bit
                             for bit either way; speed only.                */
    float policy_margin;  /* learned policy: a level keeps the rule's choice (the
                             direction-optimising variant, the sources-per-entry
                             summation) unless the network predicts the other
                             choice faster by at least this many log2 units
                             (0 = default 0.15, about 11 %; negative = no margin:
                             the network's argmin).  Speed only.            */
    int32_t replicas;     /* single graphs, batched engine: level state machines run
                             concurrently, each with its own per-vertex state and
                             batches dealt to them in turn (0 = by size: 8 up to
                             2^19 vertices, 4 above; 1 = one; at most 16; autotuned).
                             Scores agree to rounding across values; a given value
                             repeats bit for bit (BC_RUN_ONE_QUEUE: one, whatever
                             this says). */
    int32_t weighted_lanes;/* graphs with arc weights: sources one workgroup runs
                             together (0 = default 16; 1 = one source per
                             workgroup; 16; graphs above 2^27 vertices always
                             run one).  Scores agree to rounding across
                             values; a given value repeats bit for bit.     */
    int32_t reserved[4];
} bc_run_options;

/* Fill *opt with defaults (all zero fields, i.e. autotuned/automatic). */
void bc_run_options_init(bc_run_options *opt);

/*
 * Brandes over a source list (Eq. 2 summed over s).
 *   sources    host int32[n_sources]; NULL means every vertex 0 .. n-1 in order.
 *              Ids outside [0, n) -> BC_ERR_INVALID_ARG.  A source listed
 *              twice is counted twice.
 *   opt        NULL = defaults.
 * Scores are reset to zero first unless opt->flags has BC_RUN_ACCUMULATE.
 * Distances and path counts are exact; a source whose path counts exceed
 * 2^64 - 1 (or opt->sigma_limit) is evaluated again with FP64 path counts
 * scaled by per-level powers of two.  Results do not depend on the policy,
 * the variant chosen at any level, or graph capture.
 */
bc_status bc_run(bc_graph *g, const int32_t *sources, int64_t n_sources,
                 const bc_run_options *opt, void *stream);

/*
 * Autotuner for the launch configuration (the paper fixes one launch shape;
 * here the fastest of a fixed candidate set is measured on the workload).
 * Runs bc_run over the host source list sample[0 .. n_sample) (a few
 * batches' worth of the workload's sources) for every candidate, one
 * dimension at a time starting from base (NULL = defaults): batch K in
 * {64, 32, 16, 8, 1} (K = 1, the per-source engine, is timed on the first
 * 32 sources of the sample and scaled to the whole sample, since it runs
 * sources one after another), policy {heuristic, learned when weights are loaded},
 * workgroups per step {default, 1/2, 1/4}, level steps per captured chunk
 * {8, 16, 32}, push WPV degree threshold {12, 24, 48}, sources per entry
 * below which groups are summed by (entry, source) pairs {never, 2, 4, 12},
 * concurrent replicas of a single graph {half, default, twice}.
 * Each candidate is
 * timed (host clock around a synchronised run, best of two) after one
 * untimed run that builds its captured graphs; a value replaces the current
 * one only when it is at least 2 % faster.  The result goes to *best
 * (non-NULL) and stays in the handle for bc_run with BC_RUN_TUNED (which
 * fills the fields a caller leaves automatic).  Candidates with the same K
 * give the same scores bit for bit; another K may group the additions of
 * concurrent replicas differently (agreement to rounding; see
 * BC_RUN_ONE_QUEUE), so the tuner changes speed only.  Scores are reset
 * afterwards.
 * Tune cache: every result is also kept for the rest of the process under
 * (device architecture and CU count, the graph's fingerprint -- sizes,
 * flags, block offsets and degree sequence --, the sample, the resolved base
 * options).  A later call with the same key returns the kept result without
 * timing anything, unless base->flags has BC_TUNE_FRESH, which tunes again
 * and replaces it.  bc_tune_cache_save / _load keep the results in a JSON
 * file across processes.  Graphs with arc weights have nothing to tune: the
 * resolved base options are returned.
 * Errors: BC_ERR_INVALID_ARG for NULL g / best or an empty or invalid
 * sample, or a cached result of the learned policy on a handle without
 * weights.
 */
bc_status bc_autotune(bc_graph *g, const int32_t *sample, int64_t n_sample, const bc_run_options *base,
                      bc_run_options *best, void *stream);

#define BC_TUNE_FRESH 0x80u /* bc_autotune only: ignore and replace a cached result */

/*
 * The tune cache (see bc_autotune) as a file:
 *   {"format": "bc-autotune-cache", "version": 1, "entries": [
 *     {"device": "gfx950:256", "graph": "<16 hex digits>", "sample": "<16 hex>",
 *      "base": "<16 hex>", "batch": 64, "policy": 2, "grid_blocks": 384,
 *      "chunk_steps": 16, "wpv_degree": 24, "lanes_per_entry": 4,
 *      "policy_margin": 0, "replicas": 4, "flags": 0}, ...]}
 * bc_tune_cache_save writes every entry of this process to path (replacing
 * the file); bc_tune_cache_load adds the file's entries (an entry with the
 * same key replaces the one held).  Neither touches the GPU.
 * Errors: BC_ERR_INVALID_ARG for a NULL path, a file that cannot be opened,
 * read or written, or a file that is not in this format (nothing is added
 * then).  bc_tune_cache_clear drops every entry; bc_tune_cache_size counts
 * them.  Safe to call from several threads.
 */
bc_status bc_tune_cache_save(const char *path);
bc_status bc_tune_cache_load(const char *path);
void bc_tune_cache_clear(void);
int64_t bc_tune_cache_size(void);

/* bc_scores flags */
#define BC_OUT_DEVICE 0x1u

/*
 * Copy the n FP64 scores (raw ordered-pair sums over the sources run so far,
 * i.e. twice the unordered-pair betweenness for all-sources runs) to out
 * (host, or device with BC_OUT_DEVICE).  len < n -> BC_ERR_INVALID_ARG.
 */
bc_status bc_scores(const bc_graph *g, double *out, int64_t len, uint32_t flags, void *stream);

/*
 * Per-source detail, extracted from a real run of the same kernels.
 * Runs sources[0 .. n_sources) exactly like bc_run (scores included) and
 * copies out the lane of sources[dump_index]: host arrays of length n, any
 * may be NULL.
 *   d          int32 distance, -1 = unreached.
 *   sigma_u64  path counts (mode 0); zero in mode 1.
 *   sigma_mant, sigma_exp   path count = sigma_mant * 2^sigma_exp (both modes).
 *   delta      dependency delta_s(v); 0 for unreached vertices and for s.
 *   *mode      0 = uint64 path counts, 1 = FP64 fallback.
 */
typedef struct bc_detail {
    int32_t *d;
    uint64_t *sigma_u64;
    double *sigma_mant;
    int32_t *sigma_exp;
    double *delta;
    int32_t mode;
    int32_t n_levels;   /* number of distinct distances of the source (largest d + 1 unweighted) */
    int64_t *d64;       /* optional: distances as int64 (weighted graphs; d is then clamped to
                           INT32_MAX); unweighted runs leave it untouched */
} bc_detail;

bc_status bc_run_detail(bc_graph *g, const int32_t *sources, int64_t n_sources,
                        const bc_run_options *opt, int64_t dump_index, bc_detail *out,
                        void *stream);

/* Statistics of the last bc_run on this handle. */
typedef struct bc_stats {
    int64_t n_sources;
    int64_t n_batches;
    int32_t batch;             /* K actually used                              */
    int32_t policy;            /* policy actually used                         */
    int32_t grid_blocks;
    int32_t chunk_steps;
    int64_t steps;             /* level steps executed (all phases)            */
    int64_t launches;          /* step-kernel launches issued                  */
    int64_t forward_levels;    /* forward levels over all batches              */
    int64_t max_levels;
    int64_t variant_levels[3]; /* forward levels run with each BC_VARIANT_*   */
    int64_t f64_sources;       /* sources evaluated in FP64 mode              */
    int64_t arcs_scanned;      /* adjacency entries read, all phases          */
    int64_t lane_arcs;         /* (arc, source) pairs on shortest-path DAGs, both phases */
    int64_t queue_entries;     /* level-queue entries written                  */
    double algo_bytes;         /* algorithmic bytes: 16 per scanned arc, 8 per DAG
                                  (arc, source) pair, 32 per level-queue entry,
                                  40 per reached (vertex, source) pair         */
    double ms;                 /* wall time of the run, host clock            */
    double phase_ms[10];       /* device time per phase (index = internal phase id:
                                  1 discover, 2 path counts, 3 backward,
                                  4 reset, 5 BC accumulate, 6-7 detail dumps,
                                  9 undo while collecting timings)              */
    double variant_ms[3];      /* discover time per BC_VARIANT_*              */
    int64_t phase_arcs[10];    /* arcs scanned per phase                      */
    int64_t phase_lane_arcs[10];/* DAG (arc, source) pairs per phase          */
    int64_t phase_pairs[10];   /* matched neighbours whose per-source values were read */
    int64_t mode_launches[2];  /* step-kernel launches of the 64-bit (0) and FP64 (1)
                                  path-count passes                            */
    double mode_ms[2];         /* device time of those passes: HIP events on the run's
                                  stream around each pass's launches           */
    double mode_algo_bytes[2]; /* algorithmic bytes of those passes            */
    int64_t reached_pairs;     /* (vertex, source) pairs reached, sources included */
    double algo_bytes_arcs;    /* algo_bytes without the 40 B per reached pair  */
    /* Graphs with arc weights (bc_graph_create_weighted) fill the fields
       above as follows: forward_levels = relaxation rounds, steps = rounds
       of the shortest-path DAG, arcs_scanned = arcs relaxed, lane_arcs = arcs
       read by the four passes over the reached vertices (DAG in-arc counts,
       path counts, release of successors, dependencies), launches and
       mode_* = the engine's launches; algo_bytes_arcs = algo_bytes without
       64 B per reached (vertex, source) pair.  One source per workgroup
       (weighted_lanes 1): algo_bytes = 16 per arc read + 64 per reached pair.
       Lane batches (weighted_lanes 16; arcs counted once per round entry,
       for all of its sources): phase_lane_arcs[1] and [2] = (arc, source)
       pairs of the relaxation rounds and of the four passes; algo_bytes = 8
       per arc read (far end and weight) + 8 per (arc, source) pair (that
       source's value at the far end) + 64 per reached pair; phase_ms[1],
       [2], [3] = device time of the relaxation rounds, of the DAG rounds
       (in-arc counts included) and of the dependencies (score accumulation
       included), summed over the batches; phase_ms[4] = the longest batch. */
    int64_t block_workgroups;  /* block engine: workgroups of its launch (0 = not used) */
    int64_t block_chunks;      /* block engine: chunks of consecutive batches   */
} bc_stats;

bc_status bc_run_stats(const bc_graph *g, bc_stats *out);

/*
 * Per-level records of the last bc_run / bc_run_detail on this handle, one
 * per distance l from the source (the level loop of the forward and
 * backward phases, Section "Background"), summed over every batch (K > 1)
 * or source (K = 1) of the run and over both path-count modes.  Levels at
 * or beyond 65537 share the last record.
 *   out        host array of cap records (may be NULL when cap == 0).
 *   *n_levels  number of levels the run reached (records available).
 * Copies min(cap, *n_levels) records.  Errors: BC_ERR_INVALID_ARG for NULL
 * g / n_levels, cap < 0, or out == NULL with cap > 0.
 */
typedef struct bc_level_stats {
    int64_t visits;      /* forward steps at this level: batches (or sources) whose traversal reached it */
    int64_t entries;     /* level-queue entries: vertices on this level, each with its lane mask (the frontier size) */
    int64_t arcs;        /* adjacency entries scanned by this level's steps, all phases */
    int64_t variant[3];  /* forward steps of this level run with each BC_VARIANT_* */
    double ms;           /* device time of this level's steps, all phases */
} bc_level_stats;

bc_status bc_run_level_stats(const bc_graph *g, bc_level_stats *out, int64_t cap, int64_t *n_levels);

/* ---------------------------------------------------------- learned policy */

/*
 * Policy network: 5 features -> 32 -> 32 -> 9, ReLU hidden layers, FP32,
 * predicting log2 of step times at a level; each group of three outputs is
 * a choice taken by its argmin:
 *   0-2  the discover variant of the level (BC_VARIANT_*: the direction
 *        switch);
 *   3-5  the path-count step of the entries the level discovers, and
 *   6-8  the backward step of the level's own entries, each under the
 *        summation options (the load-balance switch) BC_LB_PACKED, BC_LB_RULE,
 *        BC_LB_ITEMS.
 * The summation options change speed only, never a sum or its order.
 * Weights are packed row-major as W1[32][5], b1[32], W2[32][32], b2[32],
 * W3[9][32], b3[9]: BC_MLP_PARAMS floats.
 * Features of a level, in order: log2(1+n_f)/log2(1+n), log2(1+m_f)/log2(1+nnz),
 * log2(1+n_u)/log2(1+n), log2(1+m_u)/log2(1+nnz), level/64, where n_f/m_f
 * are the frontier's vertices/arcs and n_u/m_u the unvisited ones.
 */
#define BC_MLP_IN 5
#define BC_MLP_OUT 9
#define BC_MLP_PARAMS (32 * 5 + 32 + 32 * 32 + 32 + 9 * 32 + 9)
/* summation options of path-count and backward groups: one wavefront lane
 * per source; the sources-per-entry rule of bc_run_options.lanes_per_entry;
 * one thread per (entry, source) pair */
#define BC_LB_PACKED 0
#define BC_LB_RULE   1
#define BC_LB_ITEMS  2

/* Load weights (host float[len], len == BC_MLP_PARAMS); weights == NULL
 * unloads them.  A wrong length or non-finite weights -> BC_ERR_INVALID_ARG
 * and the handle keeps its previous policy. */
bc_status bc_load_policy(bc_graph *g, const float *weights, int64_t len);

/*
 * Training support for the policy network (no graph handle needed).
 * Samples: X float[n][BC_MLP_IN] (normalised features as above), Y
 * float[n][BC_MLP_OUT] (log2 of the measured time of each choice,
 * microseconds), mask uint8[n][BC_MLP_OUT] (1 = Y entry measured).
 * Loss L = sum mask * (f(x) - y)^2 / (2 * sum mask).
 * All pointers are host memory; weights are BC_MLP_PARAMS floats.
 *   bc_mlp_loss_grad  L and dL/dweights (float[BC_MLP_PARAMS]) at weights.
 *   bc_mlp_train      `steps` full-batch Adam steps (beta1 0.9, beta2 0.999,
 *                     eps 1e-8) from *weights, updated in place; final loss.
 *   bc_mlp_predict    f(X) into Y float[n][BC_MLP_OUT].
 * Errors: BC_ERR_INVALID_ARG for NULL pointers, n < 1, an all-zero mask or
 * non-finite inputs; weights are left unchanged on any error.
 */
bc_status bc_mlp_loss_grad(const float *weights, const float *X, const float *Y, const uint8_t *mask,
                           int64_t n, float *loss, float *grad, void *stream);
bc_status bc_mlp_train(float *weights, const float *X, const float *Y, const uint8_t *mask, int64_t n,
                       int32_t steps, float lr, float *final_loss, void *stream);

/*
 * Allocation-free variant of bc_mlp_loss_grad, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight training loops,
 * harnesses that forbid hipMalloc.  Same kernels, same result bits.
 *   weights, X, Y, mask   DEVICE pointers, layouts as above; read only.
 *   n                     1 <= n <= 16384 samples, else BC_ERR_INVALID_ARG
 *                         (the intermediates live in a fixed 9.0 MB array of
 *                         the library, one per GPU, kept for the process).
 *   loss, grad            DEVICE pointers to float[1] and float[BC_MLP_PARAMS].
 * The work is enqueued on `stream` and the call returns without waiting:
 * outputs are valid once that stream reaches this point.  Inputs are not
 * checked on the host (that would need a copy): a mask with no measured
 * target gives loss 0 and a zero gradient; non-finite inputs give non-finite
 * outputs.  Every call on one GPU uses the same array, so calls whose work
 * can overlap on one GPU (different streams without ordering) race; calls on
 * one stream are ordered.  Nothing is allocated or freed, on the device or
 * the host.  Errors: BC_ERR_INVALID_ARG (NULL pointer, n out of range),
 * BC_ERR_DEVICE (the array's address could not be obtained, a launch failed).
 */
bc_status bc_mlp_loss_grad_noalloc(const float *weights, const float *X, const float *Y,
                                   const uint8_t *mask, int64_t n, float *loss, float *grad,
                                   void *stream);
bc_status bc_mlp_predict(const float *weights, const float *X, int64_t n, float *Y, void *stream);

/*
 * Training data from real runs: runs the batched engine over the sources
 * like bc_run (scores included) but executes every forward level with each
 * of the three variants in turn from the same state (undoing the first two),
 * every path-count step with each of the three summation options (restoring
 * the level's visited and next words in between) and every backward step
 * with each option (it overwrites what it writes), timing each one on the
 * device clock.  One sample per timed step: X float[cap][BC_MLP_IN] features
 * of the level that takes the choice, Y float[cap][BC_MLP_OUT] log2
 * microseconds at the three outputs of that choice and NaN elsewhere.
 * *count gets the number of samples written (at most cap).
 */
bc_status bc_collect_level_times(bc_graph *g, const int32_t *sources, int64_t n_sources,
                                 const bc_run_options *opt, float *X, float *Y, int64_t cap,
                                 int64_t *count, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* BC_H */
