// Reverse CSR of the edges present in all K snapshots of a versioned graph,
// grouped by destination: the pull step of the full-window intersection
// solve (Section 3, Step 1 on the intersection graph) reads a vertex's
// in-edges in one contiguous run.  Counting sort by destination: in-degrees,
// a scan, then every edge placed at its destination's cursor (the order of a
// destination's in-edges does not matter to a minimum or maximum).
#include <cstdlib>

#include "bounds.h"

namespace evq {

namespace {

constexpr int kBlock = 256;

// One wave per source vertex (grid-stride): its all-present out-edges.
template <bool PLACE>
__global__ void __launch_bounds__(kBlock) k_rv_edges(const uint32_t* __restrict__ row_ptr,
                                                     const uint32_t* __restrict__ row_split,
                                                     const uint32_t* __restrict__ col,
                                                     const uint32_t* __restrict__ wgt, uint32_t V,
                                                     uint32_t* __restrict__ cnt, uint32_t* __restrict__ src,
                                                     uint32_t* __restrict__ w) {
    const uint32_t lane = lane_id();
    const uint64_t nw = (uint64_t)gridDim.x * (kBlock / 64);
    for (uint64_t u = (blockIdx.x * (uint64_t)kBlock + threadIdx.x) >> 6; u < V; u += nw) {
        const uint32_t b = row_ptr[u], e = row_split[u];
        for (uint32_t i = b + lane; i < e; i += 64) {
            const uint32_t v = col[i];
            const uint32_t pos = atomicAdd(&cnt[v], 1u);
            if (PLACE) {
                src[pos] = (uint32_t)u;
                w[pos] = wgt[i];
            }
        }
    }
}

__global__ void k_rv_has(const uint32_t* __restrict__ deg, uint32_t V, uint32_t* __restrict__ has) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v < V) has[v] = deg[v] ? 1u : 0u;
}

__global__ void k_rv_items(const uint32_t* __restrict__ deg, const uint32_t* __restrict__ start,
                           const uint32_t* __restrict__ pos, uint32_t V, uint32_t* __restrict__ io,
                           uint32_t* __restrict__ iv) {
    const uint32_t v = blockIdx.x * kBlock + threadIdx.x;
    if (v < V && deg[v]) {
        io[pos[v]] = start[v];
        iv[pos[v]] = v;
    }
}

__global__ void k_rv_total(const uint32_t* __restrict__ start, uint32_t V, uint32_t* __restrict__ cnt) {
    if (threadIdx.x == 0) cnt[1] = start[V];
}

}  // namespace

uint32_t pull_frac() {
    const char* e = getenv("EVQ_PULL_FRAC");
    double f = 0.5;
    if (e && *e) f = strtod(e, nullptr);
    if (!(f >= 0.0) || f > 1.0) return kNone;
    return (uint32_t)(f * 1024.0 + 0.5);
}

void ensure_reverse(const Graph& g, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g.rv_mu);
    if (g.rv_built) {
        EVQ_HIP(hipStreamWaitEvent(s, g.rv_ready, 0));
        return;
    }
    const uint32_t V = g.V;
    const uint64_t E = g.E ? g.E : 1;
    try {
        g.rv_src = (uint32_t*)stream_alloc(E * 4, s);
        g.rv_w = (uint32_t*)stream_alloc(E * 4, s);
        g.rv_io = (uint32_t*)stream_alloc((uint64_t)V * 4 + 4, s);
        g.rv_iv = (uint32_t*)stream_alloc((uint64_t)V * 4 + 4, s);
        g.rv_cnt = (uint32_t*)stream_alloc(8, s);
        fill_u32(g.rv_cnt, 2, 0u, s);
        if (V && g.E) {
            Arena ar(s);
            uint32_t* deg = ar.alloc<uint32_t>(V);
            uint32_t* start = ar.alloc<uint32_t>((uint64_t)V + 1);
            uint32_t* cur = ar.alloc<uint32_t>(V);
            uint32_t* has = ar.alloc<uint32_t>(V);
            fill_u32(deg, V, 0u, s);
            const uint32_t wblocks = grid_for((uint64_t)V * 64, kBlock, 8192);
            EVQ_LAUNCH("reverse_count", k_rv_edges<false>, wblocks, kBlock, s, g.row_ptr, g.row_split, g.col, g.wgt,
                       V, deg, (uint32_t*)nullptr, (uint32_t*)nullptr);
            scan_exclusive(deg, start, V, start + V, s, ar);
            EVQ_HIP(hipMemcpyAsync(cur, start, (uint64_t)V * 4, hipMemcpyDeviceToDevice, s));
            EVQ_LAUNCH("reverse_place", k_rv_edges<true>, wblocks, kBlock, s, g.row_ptr, g.row_split, g.col, g.wgt,
                       V, cur, g.rv_src, g.rv_w);
            const uint32_t vblocks = grid_for(V, kBlock, 1u << 30);
            EVQ_LAUNCH("reverse_items", k_rv_has, vblocks, kBlock, s, deg, V, has);
            scan_exclusive(has, has, V, g.rv_cnt, s, ar);
            EVQ_LAUNCH("reverse_items", k_rv_items, vblocks, kBlock, s, deg, start, has, V, g.rv_io, g.rv_iv);
            EVQ_LAUNCH("reverse_items", k_rv_total, 1, 64, s, start, V, g.rv_cnt);
        }
    } catch (...) {
        uint32_t** arrays[5] = {&g.rv_src, &g.rv_w, &g.rv_io, &g.rv_iv, &g.rv_cnt};
        for (uint32_t** p : arrays) {
            stream_free(*p, s);
            *p = nullptr;
        }
        throw;
    }
    if (!g.rv_ready) EVQ_HIP(hipEventCreateWithFlags(&g.rv_ready, hipEventDisableTiming));
    EVQ_HIP(hipEventRecord(g.rv_ready, s));
    g.rv_built = true;
}

}  // namespace evq
