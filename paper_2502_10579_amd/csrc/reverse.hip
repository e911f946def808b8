// Choice of the pull step of the full-window intersection solve (Section 3,
// Step 1 on the intersection graph), and the lazy build of the graph's
// reverse CSR (its arrays are filled by build_reverse with one radix sort).
// Also the bucket width of the SSSP intersection solve and the lazy build of
// the weight-ordered rows it reads.
#include <algorithm>

#include "bounds.h"

namespace evq {

namespace {

// One wave per row: the all-present prefix [b, m) is split 64 edges at a time
// by two ballots, heavy edges (weight above the width) written forward from
// b and light ones backward from m; the rest of the row is copied in place.
__global__ void __launch_bounds__(256) k_weight_order(const uint32_t* __restrict__ row_ptr,
                                                      const uint32_t* __restrict__ row_split,
                                                      const uint32_t* __restrict__ col,
                                                      const uint32_t* __restrict__ wgt, uint32_t V, uint32_t width,
                                                      uint32_t* __restrict__ ocol, uint32_t* __restrict__ ow,
                                                      uint32_t* __restrict__ nheavy) {
    const uint32_t lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const uint64_t nw = (uint64_t)gridDim.x * 4;
    for (uint64_t u = (blockIdx.x * 256ull + threadIdx.x) >> 6; u < V; u += nw) {
        const uint32_t b = row_ptr[u], m = row_split[u], e = row_ptr[u + 1];
        uint32_t nh = 0, nl = 0;
        for (uint32_t i0 = b; i0 < m; i0 += 64) {
            const uint32_t i = i0 + lane;
            const bool in = i < m;
            const uint32_t c = in ? col[i] : 0u, w = in ? wgt[i] : 0u;
            const bool hv = in && w > width;
            const uint64_t hb = __ballot(hv), lb = __ballot(in && !hv);
            if (in) {
                const uint32_t pos = hv ? b + nh + (uint32_t)__popcll(hb & lt)
                                        : m - 1u - (nl + (uint32_t)__popcll(lb & lt));
                ocol[pos] = c;
                ow[pos] = w;
            }
            nh += (uint32_t)__popcll(hb);
            nl += (uint32_t)__popcll(lb);
        }
        for (uint32_t i = m + lane; i < e; i += 64) {
            ocol[i] = col[i];
            ow[i] = wgt[i];
        }
        if (lane == 0) nheavy[u] = nh;
    }
}

// Width = this factor times the largest weight over the mean out-degree
// (union edges per vertex): about the weight at which a vertex has a few light
// out-edges, the choice of the delta-stepping analysis for random weights.
constexpr double kWidthScale = 2.0;

}  // namespace

uint32_t choose_bucket_width(uint32_t algo, const Graph& g) {
    if (algo != EVQ_SSSP) return 0;
    const uint32_t t = tuning().bucket_width;
    if (t != kAutoWidth) return t;
    const double deg = g.V ? (double)g.E / (double)g.V : 1.0;
    const double w = kWidthScale * (double)g.maxw / std::max(deg, 1.0);
    return (uint32_t)std::max(1.0, std::min(w + 0.5, 4294967294.0));
}

const WeightOrder* weight_order_ready(const Graph& g, uint32_t width, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g.wo_mu);
    for (uint32_t i = 0; i < g.n_wo; ++i)
        if (g.wo[i].width == width) {
            EVQ_HIP(hipStreamWaitEvent(s, g.wo[i].ready, 0));
            return &g.wo[i];
        }
    if (noalloc_ctx() || g.n_wo >= kWeightOrders) return nullptr;  // a call that must not allocate never builds it
    WeightOrder& o = g.wo[g.n_wo];
    const uint64_t E = g.E ? g.E : 1;
    try {
        o.col = (uint32_t*)graph_alloc(g, E * 4, s);
        o.w = (uint32_t*)graph_alloc(g, E * 4, s);
        o.nheavy = (uint32_t*)graph_alloc(g, (uint64_t)(g.V ? g.V : 1) * 4, s);
        if (g.V)
            EVQ_LAUNCH("weight_order", k_weight_order, grid_for((uint64_t)g.V * 64, 256, 8192), 256, s, g.row_ptr,
                       g.row_split, g.col, g.wgt, g.V, width, o.col, o.w, o.nheavy);
        if (!o.ready) EVQ_HIP(hipEventCreateWithFlags(&o.ready, hipEventDisableTiming));
        EVQ_HIP(hipEventRecord(o.ready, s));
    } catch (...) {
        uint32_t** arrays[3] = {&o.col, &o.w, &o.nheavy};
        for (uint32_t** p : arrays) {
            graph_free(g, *p, s);
            *p = nullptr;
        }
        throw;
    }
    o.width = width;
    ++g.n_wo;
    return &o;
}

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
