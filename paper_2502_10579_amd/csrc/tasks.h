// Balanced task writing for frontier loops whose vertices expand to several
// tasks each.  A compaction emits one item per vertex: its first task in the
// iteration's task range [0, T) and the vertex; write_tasks then writes task t
// as ((t - first) << 32) | vertex.  The range is cut into equal contiguous
// slices, one per wave, so that a hub's many tasks are written at the rate of
// the whole grid: a wave finds the item of its first task with a 64-ary search
// over the items' offsets, then writes 64 consecutive tasks per step, each lane
// locating its task's item among 64 offsets held in registers.
#pragma once

#include "frontier.h"

namespace evq {

__device__ __forceinline__ void write_tasks(const uint32_t* __restrict__ fo, const uint32_t* __restrict__ fv,
                                            uint32_t n, uint32_t NT, uint64_t* __restrict__ tasks) {
    if (NT == 0) return;
    const uint32_t lane = lane_id();
    const uint64_t gw = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) >> 6;
    const uint64_t nw = (uint64_t)gridDim.x * (blockDim.x / 64);
    uint64_t Rw = (NT + nw - 1) / nw;
    Rw = (Rw + 63) & ~63ull;
    const uint64_t b0 = gw * Rw;
    if (b0 >= NT) return;
    uint32_t base = (uint32_t)b0;
    const uint32_t end = (uint32_t)(b0 + Rw < NT ? b0 + Rw : NT);
    uint32_t cur = wave_search(fo, n, base);
    while (base < end) {
        const uint32_t idx = cur + lane;
        uint32_t off = 0xFFFFFFFFu, iv = 0;
        if (idx < n) {
            off = fo[idx];
            iv = fv[idx];
        }
        const uint32_t t = base + lane;
        int o = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const uint32_t q = __shfl(off, o + step, 64);
            if (q <= t) o += step;
        }
        const uint32_t first = __shfl(off, o, 64), v = __shfl(iv, o, 64);
        if (t < end) tasks[t] = ((uint64_t)(t - first) << 32) | v;
        // the next step starts at the item that owns base + 64
        const uint32_t nb = base + 64;
        const uint32_t have = (uint32_t)__popcll(__ballot(off <= nb));
        uint32_t adv = have - 1;
        if (have == 64 && cur + 64 < n && fo[cur + 64] <= nb) adv = 64;
        cur += adv;
        base = nb;
    }
}

}  // namespace evq
