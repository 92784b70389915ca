// bc_wbatch.h -- layout of the lane-batched weighted engine (bc_wbatch.hip),
// shared with the host driver.  Internal to libbc.
#pragma once

#include "bc_dev.h"

namespace bcx {

// (bc_wbatch.hip) Lane-batched weighted engine: one workgroup runs kWL
// sources at once; the per-source values of vertex v are the row
// [v * kWL, (v + 1) * kWL) of each slab (one 128-byte line of distances).
constexpr int kWL = 16;
#ifndef BC_WB_WAVES
#define BC_WB_WAVES 8
#endif
constexpr int kWBatchBlock = BC_WB_WAVES * kWave;  // threads per workgroup of wbatch_run
struct WBLayout {
    size_t dist, sig, chat, dep, cnt, fm0, fm1, rm, reached, qa, qb, lvl, lvlm, lvl_off, bytes;
    __host__ __device__ static size_t up(size_t x) { return (x + 255) & ~(size_t)255; }
    __host__ __device__ explicit WBLayout(size_t n) {
        size_t o = 0;
        auto take = [&](size_t b) { const size_t at = o; o = up(o + b); return at; };
        dist = take(n * kWL * 8);   // uint64 distances, ~0 = unreached
        sig = take(n * kWL * 8);    // path counts (uint64, or double bits)
        chat = take(n * kWL * 8);   // c = (1 + delta) / sigma
        dep = take(n * kWL * 8);    // delta
        cnt = take(n * kWL * 4);    // DAG in-arcs not yet released
        fm0 = take(n * 4);          // lane masks of the two round queues
        fm1 = take(n * 4);
        rm = take(n * 4);           // lanes that reached the vertex
        reached = take(n * 4);      // vertices reached in any lane
        qa = take(n * 4);
        qb = take(n * 4);
        lvl = take(n * kWL * 4);    // DAG-round entries: vertex ...
        lvlm = take(n * kWL * 4);   // ... and its lanes
        lvl_off = take((n + 2) * 4);
        bytes = o;
    }
};

}  // namespace bcx
