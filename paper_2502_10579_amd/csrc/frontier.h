// Frontier plumbing shared by the bound solver and the multi-snapshot relaxer.
//
// A frontier is a list of work items for the next iteration.  A vertex joins
// it at most once per iteration: a per-vertex stamp holds the iteration it was
// last pushed for (stamps only grow within a query, so the array is cleared
// once per query).  High-degree vertices are split into fixed-size edge chunks
// at push time so that no wave is left with a long row.
#pragma once

#include "evq_internal.h"

namespace evq {

// Device-side counters of one frontier pair (parity 0/1).
struct FrontierCounters {
    uint32_t small[2];  // vertices in the small list
    uint32_t big[2];    // tasks in the big-task list
};

// Append the lanes' vertices with `want` set to `list`, one atomic per wave.
// Must be called by every lane of the wave.
__device__ __forceinline__ void wave_append(bool want, uint32_t v, uint32_t* list, uint32_t* cnt) {
    uint64_t bal = __ballot(want);
    if (bal == 0) return;
    const int leader = __ffsll((unsigned long long)bal) - 1;
    uint32_t base = 0;
    if ((int)lane_id() == leader) base = atomicAdd(cnt, (uint32_t)__popcll(bal));
    base = __shfl(base, leader, 64);
    if (want) list[base + (uint32_t)__popcll(bal & lanemask_lt())] = v;
}

// Append `n` tasks (chunk << 32 | id) for each lane with n > 0, one atomic per wave.
__device__ __forceinline__ void wave_append_tasks(uint32_t n, uint32_t id, uint64_t* list, uint32_t* cnt) {
    uint32_t inc = wave_incl_scan(n);
    uint32_t tot = __shfl(inc, 63, 64);
    if (tot == 0) return;
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(cnt, tot);
    base = __shfl(base, 0, 64);
    uint32_t at = base + inc - n;
    for (uint32_t c = 0; c < n; ++c) list[at + c] = ((uint64_t)c << 32) | id;
}

// True when this lane is the first to push vertex v for iteration `stamp`.
__device__ __forceinline__ bool claim(uint32_t* stamps, uint32_t v, bool want, uint32_t stamp) {
    return want && atomicExch(&stamps[v], stamp) != stamp;
}

}  // namespace evq
