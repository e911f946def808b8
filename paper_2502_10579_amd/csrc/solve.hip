// Bound solver (Section 3, Step 1): single-source relaxation of the query on
// the window's intersection graph (edges present in every snapshot of the
// window) or union graph (edges present in at least one), on the versioned
// graph's CSR with a per-edge mask test.  The union solve starts from the
// intersection result and first relaxes the window-partial edges, i.e. it adds
// the edges missing from the intersection graph (Section 6.2).
//
// One iteration = two kernels:
//   compaction  next-frontier bitmap -> vertex list fv[] with running edge
//               offsets fo[] (vertices without edges are dropped);
//   expansion   the frontier's edges, viewed as one range [0, T), are cut
//               into equal contiguous slices, one per wave; a wave finds its
//               first vertex with a 64-ary search over fo[] and then walks 64
//               edges per step, each lane locating its edge's vertex with a
//               binary search over 64 offsets held in registers.
// Values improve with fire-and-forget uint32 atomicMin/atomicMax after a plain
// read shows the candidate is better; improved vertices set their bit.
#include "bounds.h"

namespace evq {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kExpandBlocks = 2048;

struct SolveArgs {
    const uint32_t* row_ptr;
    const uint32_t* row_split;
    const uint32_t* col;
    const uint32_t* wgt;
    const uint64_t* mask;
    uint32_t* R;
    uint32_t* bitmap;
    uint32_t* fv;  // frontier vertices
    uint32_t* fo;  // their first edge offset in the frontier's edge range
    FrontierCounters* cnt;
    unsigned long long* stats;
    uint32_t V;
};

// MODE: 0 = intersection over all K snapshots (only the all-present prefix of
// each row), 1 = intersection over a sub-window, 2 = union.
template <int MODE, int MW>
__device__ __forceinline__ bool partial_in(const uint64_t* __restrict__ mask, uint32_t e, const Mask<MW>& W) {
    Mask<MW> m = load_mask<MW>(mask, e);
    if (MODE == 2) {
        bool any = false;
#pragma unroll
        for (int j = 0; j < MW; ++j) any |= (m.w[j] & W.w[j]) != 0;
        return any;
    }
    bool all = true;
#pragma unroll
    for (int j = 0; j < MW; ++j) all &= (m.w[j] & W.w[j]) == W.w[j];
    return all;
}

template <int MODE>
__device__ __forceinline__ uint32_t row_end(const SolveArgs& a, uint32_t v) {
    return MODE == 0 ? a.row_split[v] : a.row_ptr[v + 1];
}

template <int A, int MODE, int MW>
__device__ __forceinline__ void relax(const SolveArgs& a, uint32_t e, uint32_t split, uint32_t x, const Mask<MW>& W) {
    if (MODE != 0 && e >= split && !partial_in<MODE, MW>(a.mask, e, W)) return;
    const uint32_t v = a.col[e];
    const uint32_t cand = Alg<A>::extend(x, a.wgt[e]);
    if (!Alg<A>::better(cand, a.R[v])) return;
    Alg<A>::improve_nr(&a.R[v], cand);
    mark(a.bitmap, v);
}

template <bool ST>
__device__ __forceinline__ void count_visits(const SolveArgs& a, uint32_t n) {
    if (!ST) return;
    uint32_t s = wave_sum(n);
    if (lane_id() == 0 && s) atomicAdd(&a.stats[0], (unsigned long long)s);
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bitmap -> (fv, fo) of parity p, clearing the bits it reads.  A wave takes 64
// bitmap words, stages their vertex ids in LDS, then reads the degrees of up
// to 64 vertices at a time.
template <int MODE>
__global__ void __launch_bounds__(kBlock) k_compact_frontier(SolveArgs a, int p, int first) {
    if (!first && a.cnt->packed[p ^ 1] == 0ull) return;  // the previous expansion set no bits
    __shared__ uint32_t buf[kBlock / 64][64 * 32];
    const uint32_t nwords = (a.V + 31) >> 5;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t gw = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * (kBlock / 64);
    for (uint32_t wb = gw * 64; wb < nwords; wb += nw * 64) {
        const uint32_t wi = wb + lane;
        uint32_t word = 0;
        if (wi < nwords) {
            word = a.bitmap[wi];
            if (word) a.bitmap[wi] = 0;
        }
        const uint32_t pc = (uint32_t)__popc(word);
        const uint32_t incl = wave_incl_scan(pc);
        const uint32_t tot = __shfl(incl, 63, 64);
        uint32_t k = incl - pc;
        for (uint32_t m = word; m; m &= m - 1) buf[wave][k++] = wi * 32 + (uint32_t)__builtin_ctz(m);
        wave_lds_sync();
        for (uint32_t s0 = 0; s0 < tot; s0 += 64) {
            const uint32_t j = s0 + lane;
            uint32_t v = 0, deg = 0;
            if (j < tot) {
                v = buf[wave][j];
                deg = row_end<MODE>(a, v) - a.row_ptr[v];
            }
            const uint32_t keep = deg > 0 ? 1u : 0u;
            uint32_t item, edge;
            wave_reserve2(keep, deg, &a.cnt->packed[p], item, edge);
            if (keep) {
                a.fv[item] = v;
                a.fo[item] = edge;
            }
        }
        wave_lds_sync();
    }
}

template <int A, int MODE, int MW, bool ST>
__global__ void __launch_bounds__(kBlock) k_expand(SolveArgs a, Mask<MW> W, int p, uint32_t* slot) {
    const unsigned long long cx = expand_prologue(a.cnt, p, slot);
    const uint32_t n = items_of(cx), T = edges_of(cx);
    if (T == 0) return;
    const uint32_t lane = lane_id();
    const uint64_t gw = (blockIdx.x * (uint64_t)kBlock + threadIdx.x) >> 6;
    const uint64_t nw = (uint64_t)gridDim.x * (kBlock / 64);
    uint64_t Rw = (T + nw - 1) / nw;
    Rw = (Rw + 63) & ~63ull;
    const uint64_t a0 = gw * Rw;
    if (a0 >= T) return;
    const uint32_t a1 = (uint32_t)(a0 + Rw < T ? a0 + Rw : T);
    count_visits<ST>(a, lane == 0 ? a1 - (uint32_t)a0 : 0u);
    uint32_t cur = wave_search(a.fo, n, (uint32_t)a0);
    for (uint32_t base = (uint32_t)a0; base < a1; base += 64) {
        const uint32_t idx = cur + lane;
        const uint32_t off = idx < n ? a.fo[idx] : 0xFFFFFFFFu;
        uint32_t rb = 0, sp = 0, xv = 0;
        if (off <= base + 63) {  // only the vertices this step can touch
            const uint32_t v = a.fv[idx];
            rb = a.row_ptr[v];
            sp = a.row_split[v];
            xv = a.R[v];
        }
        const uint32_t t = base + lane;
        int j = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const uint32_t o = __shfl(off, j + step, 64);
            if (o <= t) j += step;
        }
        const uint32_t e = __shfl(rb, j, 64) + (t - __shfl(off, j, 64));
        const uint32_t spj = __shfl(sp, j, 64);
        const uint32_t xs = __shfl(xv, j, 64);
        if (t < a1) relax<A, MODE, MW>(a, e, spj, xs, W);
        // next step starts at the owner of base + 64: one of cur .. cur + 64,
        // since every listed vertex has at least one edge
        const uint32_t nb = base + 64;
        const uint32_t have = (uint32_t)__popcll(__ballot(off <= nb));
        uint32_t adv = have - 1;
        if (have == 64 && cur + 64 < n && a.fo[cur + 64] <= nb) adv = 64;
        cur += adv;
    }
}

// Start of a solve from one source vertex.
__global__ void k_seed_source(uint32_t* R, uint32_t* bitmap, uint32_t source, uint32_t at_source) {
    if (threadIdx.x == 0) {
        R[source] = at_source;
        bitmap[source >> 5] |= 1u << (source & 31);
    }
}

// Union solve, first step: relax every edge present in some but not all
// snapshots of the window, from the values in R (the intersection result).
template <int A, int MW, bool ST>
__global__ void __launch_bounds__(kBlock) k_seed_partial(SolveArgs a, Mask<MW> W, const uint32_t* __restrict__ p_src,
                                                         const uint32_t* __restrict__ p_eid, uint32_t n_partial) {
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t base = blockIdx.x * kBlock; base < n_partial; base += stride) {
        const uint32_t q = base + threadIdx.x;
        bool act = false;
        if (q < n_partial) {
            const uint32_t e = p_eid[q];
            Mask<MW> m = load_mask<MW>(a.mask, e);
            bool any = false, all = true;
#pragma unroll
            for (int j = 0; j < MW; ++j) {
                any |= (m.w[j] & W.w[j]) != 0;
                all &= (m.w[j] & W.w[j]) == W.w[j];
            }
            act = any && !all;
            if (act) {
                const uint32_t v = a.col[e];
                const uint32_t cand = Alg<A>::extend(a.R[p_src[q]], a.wgt[e]);
                if (Alg<A>::better(cand, a.R[v])) {
                    Alg<A>::improve_nr(&a.R[v], cand);
                    mark(a.bitmap, v);
                }
            }
        }
        count_visits<ST>(a, act ? 1u : 0u);
    }
}

template <int A, int MODE, int MW, bool ST>
uint64_t frontier_loop(SolveArgs a, const Mask<MW>& W, Frontier& f, hipStream_t s, uint64_t max_iters) {
    const uint32_t nwords = (a.V + 31) >> 5;
    const uint32_t cblocks = grid_for((nwords + 63) / 64, kBlock / 64, 4096);
    auto issue = [&](uint64_t, int p, bool first, uint32_t* slot) {
        EVQ_LAUNCH("solve_compact", k_compact_frontier<MODE>, cblocks, kBlock, s, a, p, first ? 1 : 0);
        EVQ_LAUNCH("solve_expand", (k_expand<A, MODE, MW, ST>), kExpandBlocks, kBlock, s, a, W, p, slot);
    };
    return drive_loop(issue, f.p, s, max_iters, "bound solve");
}

template <int MW>
Mask<MW> window_mask(const Window& W) {
    Mask<MW> m;
    for (int j = 0; j < MW; ++j) m.w[j] = W.w[j];
    return m;
}

SolveArgs make_args(const Graph& g, const Frontier& f, uint32_t* R) {
    SolveArgs a;
    a.row_ptr = g.row_ptr;
    a.row_split = g.row_split;
    a.col = g.col;
    a.wgt = g.wgt;
    a.mask = g.mask;
    a.R = R;
    a.bitmap = f.bitmap;
    a.fv = f.fv;
    a.fo = f.fo;
    a.cnt = f.cnt;
    a.stats = f.stats;
    a.V = g.V;
    return a;
}

template <int A, int MW, bool ST>
uint64_t solve_cap_t(const Graph& g, const Window& W, uint32_t source, uint32_t* R, Frontier& f, hipStream_t s) {
    SolveArgs a = make_args(g, f, R);
    fill_u32(R, g.V, Alg<A>::unreached, s);
    EVQ_LAUNCH("solve_seed_source", k_seed_source, 1, 64, s, R, f.bitmap, source, Alg<A>::at_source);
    if (W.full) return frontier_loop<A, 0, MW, ST>(a, window_mask<MW>(W), f, s, (uint64_t)g.V + 2);
    return frontier_loop<A, 1, MW, ST>(a, window_mask<MW>(W), f, s, (uint64_t)g.V + 2);
}

template <int A, int MW, bool ST>
uint64_t solve_cup_t(const Graph& g, const Window& W, uint32_t* R, Frontier& f, hipStream_t s) {
    SolveArgs a = make_args(g, f, R);
    if (g.n_partial)
        EVQ_LAUNCH("solve_seed_partial", (k_seed_partial<A, MW, ST>), grid_for(g.n_partial, kBlock, 16384), kBlock, s,
                   a, window_mask<MW>(W), g.p_src, g.p_eid, (uint32_t)g.n_partial);
    return frontier_loop<A, 2, MW, ST>(a, window_mask<MW>(W), f, s, (uint64_t)g.V + 2);
}

template <int MW, bool ST>
uint64_t dispatch_cap(uint32_t algo, const Graph& g, const Window& W, uint32_t source, uint32_t* R, Frontier& f,
                      hipStream_t s) {
    switch (algo) {
    case EVQ_SSSP: return solve_cap_t<EVQ_SSSP, MW, ST>(g, W, source, R, f, s);
    case EVQ_BFS: return solve_cap_t<EVQ_BFS, MW, ST>(g, W, source, R, f, s);
    case EVQ_SSWP: return solve_cap_t<EVQ_SSWP, MW, ST>(g, W, source, R, f, s);
    default: return solve_cap_t<EVQ_SSNP, MW, ST>(g, W, source, R, f, s);
    }
}

template <int MW, bool ST>
uint64_t dispatch_cup(uint32_t algo, const Graph& g, const Window& W, uint32_t* R, Frontier& f, hipStream_t s) {
    switch (algo) {
    case EVQ_SSSP: return solve_cup_t<EVQ_SSSP, MW, ST>(g, W, R, f, s);
    case EVQ_BFS: return solve_cup_t<EVQ_BFS, MW, ST>(g, W, R, f, s);
    case EVQ_SSWP: return solve_cup_t<EVQ_SSWP, MW, ST>(g, W, R, f, s);
    default: return solve_cup_t<EVQ_SSNP, MW, ST>(g, W, R, f, s);
    }
}

__global__ void k_init_frontier(FrontierCounters* c, unsigned long long* st, int n) {
    if (threadIdx.x == 0) c->packed[0] = c->packed[1] = 0ull;
    if ((int)threadIdx.x < n) st[threadIdx.x] = 0ull;
}

}  // namespace

Frontier make_frontier(const Graph& g, Arena& ar, hipStream_t s) {
    Frontier f;
    const uint64_t nwords = ((uint64_t)g.V + 31) / 32;
    f.bitmap = ar.alloc<uint32_t>(nwords);
    f.fv = ar.alloc<uint32_t>(g.V);
    f.fo = ar.alloc<uint32_t>(g.V);
    f.cnt = ar.alloc<FrontierCounters>(1);
    f.stats = ar.alloc<unsigned long long>(8);
    fill_u32(f.bitmap, nwords, 0u, s);
    EVQ_LAUNCH("query_init", k_init_frontier, 1, 64, s, f.cnt, f.stats, 8);
    f.p = 0;
    return f;
}

uint64_t solve_cap(const Graph& g, uint32_t algo, const Window& W, uint32_t source, uint32_t* R, Frontier& f,
                   hipStream_t s, bool stats) {
    if (g.MW == 1) return stats ? dispatch_cap<1, true>(algo, g, W, source, R, f, s)
                                : dispatch_cap<1, false>(algo, g, W, source, R, f, s);
    return stats ? dispatch_cap<2, true>(algo, g, W, source, R, f, s)
                 : dispatch_cap<2, false>(algo, g, W, source, R, f, s);
}

uint64_t solve_cup(const Graph& g, uint32_t algo, const Window& W, uint32_t* R, Frontier& f, hipStream_t s,
                   bool stats) {
    if (g.MW == 1) return stats ? dispatch_cup<1, true>(algo, g, W, R, f, s) : dispatch_cup<1, false>(algo, g, W, R, f, s);
    return stats ? dispatch_cup<2, true>(algo, g, W, R, f, s) : dispatch_cup<2, false>(algo, g, W, R, f, s);
}

}  // namespace evq
