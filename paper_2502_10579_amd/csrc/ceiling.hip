// Access-pattern ceiling of the bound solves' expansion (measurement only).
//
// An expansion visit streams the edge's column and weight, gathers the
// destination's value and, for the few visits that improve it, issues an
// atomicMin and a flag store; the walk over the frontier's items adds a
// per-vertex lookup on top.  This kernel keeps the memory operations of a
// visit over the graph's own edges (so the destinations have the graph's
// locality) and drops the rest: the values are all zero and a weight is
// never below zero, so the comparison never succeeds and no update is
// issued.  Its rate bounds what the expansion can reach on this graph.
#include "ceiling.h"

namespace evq {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kBlocks = 2048;  // one wave per SIMD slot of the device, as the expansion

__global__ void __launch_bounds__(kBlock) k_gather_ceiling(const uint32_t* __restrict__ col,
                                                           const uint32_t* __restrict__ wgt, uint32_t* R,
                                                           uint8_t* flags, uint64_t E) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t e = blockIdx.x * (uint64_t)kBlock + threadIdx.x; e < E; e += stride) {
        const uint32_t v = col[e];
        const uint32_t cand = wgt[e];
        if (cand < R[v]) {
            atomicMin(&R[v], cand);
            flags[v] = 1;
        }
    }
}

}  // namespace

double gather_ceiling(const Graph& g, uint32_t launches, hipStream_t s) {
    if (g.E == 0) return 0.0;
    const uint64_t vb = ((uint64_t)g.V * 4 + 255) & ~uint64_t(255);
    char* buf = static_cast<char*>(stream_alloc(vb + g.V, s));
    uint32_t* R = reinterpret_cast<uint32_t*>(buf);
    uint8_t* flags = reinterpret_cast<uint8_t*>(buf + vb);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double rate = 0.0;
    try {
        EVQ_HIP(hipMemsetAsync(buf, 0, vb + g.V, s));
        EVQ_HIP(hipEventCreate(&e0));
        EVQ_HIP(hipEventCreate(&e1));
        EVQ_LAUNCH("gather_ceiling", k_gather_ceiling, kBlocks, kBlock, s, g.col, g.wgt, R, flags, g.E);
        EVQ_HIP(hipEventRecord(e0, s));
        for (uint32_t i = 0; i < launches; ++i)
            EVQ_LAUNCH("gather_ceiling", k_gather_ceiling, kBlocks, kBlock, s, g.col, g.wgt, R, flags, g.E);
        EVQ_HIP(hipEventRecord(e1, s));
        EVQ_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        EVQ_HIP(hipEventElapsedTime(&ms, e0, e1));
        rate = ms > 0.f ? (double)g.E * launches / (ms * 1e-3) : 0.0;
    } catch (...) {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        stream_free(buf, s);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    stream_free(buf, s);
    return rate;
}

}  // namespace evq
