// Choice of the pull step of the full-window intersection solve (Section 3,
// Step 1 on the intersection graph), and the lazy build of the graph's
// reverse CSR (its arrays are filled by build_reverse with one radix sort).
#include "bounds.h"

namespace evq {

uint32_t pull_frac() {
    const double f = tuning().pull_frac;
    if (!(f >= 0.0) || f > 1.0) return kNone;
    return (uint32_t)(f * 1024.0 + 0.5);
}

bool reverse_ready(const Graph& g, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g.rv_mu);
    if (g.rv_built) {
        EVQ_HIP(hipStreamWaitEvent(s, g.rv_ready, 0));
        return true;
    }
    if (noalloc_ctx()) return false;  // a call that must not allocate never builds it
    if (++g.rv_asks < 2) return false;
    const uint64_t E = g.E ? g.E : 1;
    try {
        g.rv_src = (uint32_t*)graph_alloc(g, E * 4, s);
        g.rv_w = (uint32_t*)graph_alloc(g, E * 4, s);
        g.rv_dst = (uint32_t*)graph_alloc(g, E * 4, s);
        g.rv_cnt = (uint32_t*)graph_alloc(g, 8, s);
        build_reverse(g, s);
    } catch (...) {
        uint32_t** arrays[4] = {&g.rv_src, &g.rv_w, &g.rv_dst, &g.rv_cnt};
        for (uint32_t** p : arrays) {
            graph_free(g, *p, s);
            *p = nullptr;
        }
        throw;
    }
    if (!g.rv_ready) EVQ_HIP(hipEventCreateWithFlags(&g.rv_ready, hipEventDisableTiming));
    EVQ_HIP(hipEventRecord(g.rv_ready, s));
    g.rv_built = true;
    return true;
}

}  // namespace evq
