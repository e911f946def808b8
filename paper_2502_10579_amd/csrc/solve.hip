// Bound solver (Section 3, Step 1): single-source relaxation of the query on
// the window's intersection graph (edges present in every snapshot of the
// window) or union graph (edges present in at least one), on the versioned
// graph's CSR with a per-edge mask test.  The union solve starts from the
// intersection result and first relaxes the window-partial edges, i.e. it adds
// the edges missing from the intersection graph (Section 6.2).
//
// Each iteration expands the current frontier with uint32 atomicMin/atomicMax
// and builds the next one with wave ballots (one counter atomic per wave).
// Work split: a wave takes 64 frontier vertices of degree <= kBig and spreads
// their edges over its lanes through a wave prefix sum; vertices of larger
// degree are split into kChunk-edge tasks when pushed, one wave per task.
#include "bounds.h"

namespace evq {

namespace {

constexpr uint32_t kBig = 256;
constexpr uint32_t kChunk = 256;
constexpr int kBlock = 256;

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

// Push the lanes' improved vertices into the next frontier (all lanes call).
template <int MODE>
__device__ __forceinline__ void push(const SolveArgs& a, uint32_t v, bool want, uint32_t stamp, int np) {
    bool fresh = claim(a.stamps, v, want, stamp);
    uint32_t deg = 0;
    if (fresh) deg = row_end<MODE>(a, v) - a.row_ptr[v];
    bool small = fresh && deg > 0 && deg <= kBig;
    wave_append(small, v, a.list[np], &a.cnt->small[np]);
    uint32_t nch = (fresh && deg > kBig) ? (deg + kChunk - 1) / kChunk : 0u;
    wave_append_tasks(nch, v, a.big[np], &a.cnt->big[np]);
}

template <int A, int MODE, int MW>
__device__ __forceinline__ bool relax(const SolveArgs& a, uint32_t e, uint32_t split, uint32_t x, const Mask<MW>& W,
                                      bool act, uint32_t& v) {
    v = 0;
    if (!act) return false;
    if (MODE != 0 && e >= split && !partial_in<MODE, MW>(a.mask, e, W)) return false;
    v = a.col[e];
    uint32_t cand = Alg<A>::extend(x, a.wgt[e]);
    if (!Alg<A>::better(cand, a.R[v])) return false;
    return Alg<A>::better(cand, Alg<A>::improve(&a.R[v], cand));
}

template <bool ST>
__device__ __forceinline__ void count_visits(const SolveArgs& a, bool act) {
    if (!ST) return;
    uint64_t bal = __ballot(act);
    if (lane_id() == 0 && bal) atomicAdd(&a.stats[0], (unsigned long long)__popcll(bal));
}

template <int A, int MODE, int MW, bool ST>
__global__ void __launch_bounds__(kBlock) k_expand_small(SolveArgs a, Mask<MW> W, int p, uint32_t stamp) {
    const uint32_t n = a.cnt->small[p];
    const uint32_t* __restrict__ cur = a.list[p];
    const int lane = lane_id();
    const uint32_t gw = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * (kBlock / 64);
    for (uint32_t chunk = gw; chunk * 64u < n; chunk += nw) {
        uint32_t idx = chunk * 64u + lane;
        bool valid = idx < n;
        uint32_t u = valid ? cur[idx] : 0u;
        uint32_t beg = 0, split = 0, deg = 0, x = 0;
        if (valid) {
            beg = a.row_ptr[u];
            split = a.row_split[u];
            deg = row_end<MODE>(a, u) - beg;
            x = a.R[u];
        }
        uint32_t incl = wave_incl_scan(deg);
        uint32_t excl = incl - deg;
        uint32_t total = __shfl(incl, 63, 64);
        for (uint32_t base = 0; base < total; base += 64) {
            uint32_t t = base + lane;
            bool act = t < total;
            int j = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                uint32_t o = __shfl(excl, j + step, 64);
                if (o <= t) j += step;
            }
            uint32_t e = __shfl(beg, j, 64) + (t - __shfl(excl, j, 64));
            uint32_t sp = __shfl(split, j, 64);
            uint32_t xs = __shfl(x, j, 64);
            count_visits<ST>(a, act);
            uint32_t v;
            bool want = relax<A, MODE, MW>(a, e, sp, xs, W, act, v);
            push<MODE>(a, v, want, stamp, p ^ 1);
        }
    }
}

template <int A, int MODE, int MW, bool ST>
__global__ void __launch_bounds__(kBlock) k_expand_big(SolveArgs a, Mask<MW> W, int p, uint32_t stamp) {
    const uint32_t n = a.cnt->big[p];
    const uint64_t* __restrict__ tasks = a.big[p];
    const int lane = lane_id();
    const uint32_t gw = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * (kBlock / 64);
    for (uint32_t t = gw; t < n; t += nw) {
        uint64_t tk = tasks[t];
        uint32_t u = (uint32_t)tk, c = (uint32_t)(tk >> 32);
        uint32_t beg = a.row_ptr[u], split = a.row_split[u];
        uint32_t end = row_end<MODE>(a, u);
        uint32_t e0 = beg + c * kChunk;
        uint32_t e1 = e0 + kChunk < end ? e0 + kChunk : end;
        uint32_t x = a.R[u];
        for (uint32_t e = e0; e < e1; e += 64) {
            bool act = e + lane < e1;
            count_visits<ST>(a, act);
            uint32_t v;
            bool want = relax<A, MODE, MW>(a, e + lane, split, x, W, act, v);
            push<MODE>(a, v, want, stamp, p ^ 1);
        }
    }
}

// Start of a solve from one source vertex.
template <int MODE>
__global__ void k_seed_source(SolveArgs a, uint32_t source, uint32_t at_source, uint32_t stamp) {
    if (threadIdx.x >= 64) return;
    bool want = lane_id() == 0;
    if (want) a.R[source] = at_source;
    push<MODE>(a, source, want, stamp, 0);
}

// Union solve, first step: relax every edge present in some but not all
// snapshots of the window, from the values in R (the intersection result).
template <int A, int MW, bool ST>
__global__ void __launch_bounds__(kBlock) k_seed_partial(SolveArgs a, Mask<MW> W, const uint32_t* __restrict__ p_src,
                                                         const uint32_t* __restrict__ p_eid, uint32_t n_partial,
                                                         uint32_t stamp) {
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t base = blockIdx.x * kBlock; base < n_partial; base += stride) {
        uint32_t q = base + threadIdx.x;
        bool act = q < n_partial;
        uint32_t e = 0, u = 0;
        if (act) {
            e = p_eid[q];
            u = p_src[q];
            Mask<MW> m = load_mask<MW>(a.mask, e);
            bool any = false, all = true;
#pragma unroll
            for (int j = 0; j < MW; ++j) {
                any |= (m.w[j] & W.w[j]) != 0;
                all &= (m.w[j] & W.w[j]) == W.w[j];
            }
            act = any && !all;
        }
        count_visits<ST>(a, act);
        uint32_t v = 0;
        bool want = false;
        if (act) {
            v = a.col[e];
            uint32_t cand = Alg<A>::extend(a.R[u], a.wgt[e]);
            want = Alg<A>::better(cand, a.R[v]) && Alg<A>::better(cand, Alg<A>::improve(&a.R[v], cand));
        }
        push<2>(a, v, want, stamp, 0);
    }
}

__global__ void k_reset_counters(FrontierCounters* c, int p) {
    if (threadIdx.x == 0) {
        c->small[p] = 0;
        c->big[p] = 0;
    }
}

__global__ void k_init_query(FrontierCounters* c, unsigned long long* stats, int nstats) {
    if (threadIdx.x == 0) {
        c->small[0] = c->small[1] = 0;
        c->big[0] = c->big[1] = 0;
    }
    if ((int)threadIdx.x < nstats) stats[threadIdx.x] = 0;
}

template <int A, int MODE, int MW, bool ST>
struct Loop {
    static uint64_t run(const SolveArgs& a, const Mask<MW>& W, uint32_t& stamp, Mailbox& mb, hipStream_t s,
                        uint64_t max_iters) {
        int p = 0;
        uint64_t iters = 0;
        for (;;) {
            uint32_t ns = mb.h[0], nb = mb.h[1];
            if (ns + nb == 0) break;
            if (++iters > max_iters) fail(EVQ_ENOCONV, "bound solve exceeded its iteration cap");
            ++stamp;
            if (ns) {
                uint32_t blocks = grid_for(ns, 64 * (kBlock / 64), 16384);
                EVQ_LAUNCH("solve_expand_small", (k_expand_small<A, MODE, MW, ST>), blocks, kBlock, s, a, W, p, stamp);
            }
            if (nb) {
                uint32_t blocks = grid_for(nb, kBlock / 64, 16384);
                EVQ_LAUNCH("solve_expand_big", (k_expand_big<A, MODE, MW, ST>), blocks, kBlock, s, a, W, p, stamp);
            }
            EVQ_LAUNCH("solve_reset", k_reset_counters, 1, 64, s, a.cnt, p);
            p ^= 1;
            EVQ_HIP(hipMemcpyAsync(mb.h, dev_small_cnt(a.cnt, p), 4, hipMemcpyDeviceToHost, s));
            EVQ_HIP(hipMemcpyAsync(mb.h + 1, dev_big_cnt(a.cnt, p), 4, hipMemcpyDeviceToHost, s));
            EVQ_HIP(hipStreamSynchronize(s));
        }
        // the final (empty) list sits at parity p; move it to parity 0 for the next phase
        if (p != 0) EVQ_LAUNCH("solve_reset", k_reset_counters, 1, 64, s, a.cnt, p);
        return iters;
    }
};

template <int A, int MW, bool ST>
uint64_t solve_cap_t(const Graph& g, const Window& W, uint32_t source, SolveArgs a, uint32_t& stamp, Mailbox& mb,
                     hipStream_t s) {
    Mask<MW> Wm;
    for (int j = 0; j < MW; ++j) Wm.w[j] = W.w[j];
    fill_u32(a.R, g.V, Alg<A>::unreached, s);
    ++stamp;
    if (W.full) EVQ_LAUNCH("solve_seed_source", k_seed_source<0>, 1, 64, s, a, source, Alg<A>::at_source, stamp);
    else EVQ_LAUNCH("solve_seed_source", k_seed_source<1>, 1, 64, s, a, source, Alg<A>::at_source, stamp);
    EVQ_HIP(hipMemcpyAsync(mb.h, dev_small_cnt(a.cnt, 0), 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipMemcpyAsync(mb.h + 1, dev_big_cnt(a.cnt, 0), 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipStreamSynchronize(s));
    if (W.full) return Loop<A, 0, MW, ST>::run(a, Wm, stamp, mb, s, (uint64_t)g.V + 2);
    return Loop<A, 1, MW, ST>::run(a, Wm, stamp, mb, s, (uint64_t)g.V + 2);
}

template <int A, int MW, bool ST>
uint64_t solve_cup_t(const Graph& g, const Window& W, SolveArgs a, uint32_t& stamp, Mailbox& mb, hipStream_t s) {
    Mask<MW> Wm;
    for (int j = 0; j < MW; ++j) Wm.w[j] = W.w[j];
    ++stamp;
    if (g.n_partial) {
        uint32_t blocks = grid_for(g.n_partial, kBlock, 16384);
        EVQ_LAUNCH("solve_seed_partial", (k_seed_partial<A, MW, ST>), blocks, kBlock, s, a, Wm, g.p_src, g.p_eid,
                   (uint32_t)g.n_partial, stamp);
    }
    EVQ_HIP(hipMemcpyAsync(mb.h, dev_small_cnt(a.cnt, 0), 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipMemcpyAsync(mb.h + 1, dev_big_cnt(a.cnt, 0), 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipStreamSynchronize(s));
    return Loop<A, 2, MW, ST>::run(a, Wm, stamp, mb, s, (uint64_t)g.V + 2);
}

template <int MW, bool ST>
uint64_t dispatch_cap(uint32_t algo, const Graph& g, const Window& W, uint32_t source, const SolveArgs& a,
                      uint32_t& stamp, Mailbox& mb, hipStream_t s) {
    switch (algo) {
    case EVQ_SSSP: return solve_cap_t<EVQ_SSSP, MW, ST>(g, W, source, a, stamp, mb, s);
    case EVQ_BFS: return solve_cap_t<EVQ_BFS, MW, ST>(g, W, source, a, stamp, mb, s);
    case EVQ_SSWP: return solve_cap_t<EVQ_SSWP, MW, ST>(g, W, source, a, stamp, mb, s);
    default: return solve_cap_t<EVQ_SSNP, MW, ST>(g, W, source, a, stamp, mb, s);
    }
}

template <int MW, bool ST>
uint64_t dispatch_cup(uint32_t algo, const Graph& g, const Window& W, const SolveArgs& a, uint32_t& stamp,
                      Mailbox& mb, hipStream_t s) {
    switch (algo) {
    case EVQ_SSSP: return solve_cup_t<EVQ_SSSP, MW, ST>(g, W, a, stamp, mb, s);
    case EVQ_BFS: return solve_cup_t<EVQ_BFS, MW, ST>(g, W, a, stamp, mb, s);
    case EVQ_SSWP: return solve_cup_t<EVQ_SSWP, MW, ST>(g, W, a, stamp, mb, s);
    default: return solve_cup_t<EVQ_SSNP, MW, ST>(g, W, a, stamp, mb, s);
    }
}

}  // namespace

SolveWorkspace make_solve_workspace(const Graph& g, Arena& ar, hipStream_t s) {
    SolveWorkspace w;
    w.stamps = ar.alloc<uint32_t>(g.V);
    w.list[0] = ar.alloc<uint32_t>(g.V);
    w.list[1] = ar.alloc<uint32_t>(g.V);
    w.cap_big = g.E / kChunk + g.E / (kBig + 1) + 64;
    w.big[0] = ar.alloc<uint64_t>(w.cap_big);
    w.big[1] = ar.alloc<uint64_t>(w.cap_big);
    w.cnt = ar.alloc<FrontierCounters>(1);
    w.stats = ar.alloc<unsigned long long>(8);
    fill_u32(w.stamps, g.V, 0u, s);
    EVQ_LAUNCH("query_init", k_init_query, 1, 64, s, w.cnt, w.stats, 8);
    return w;
}

SolveArgs solve_args(const Graph& g, const SolveWorkspace& w, uint32_t* R) {
    SolveArgs a;
    a.row_ptr = g.row_ptr;
    a.row_split = g.row_split;
    a.col = g.col;
    a.wgt = g.wgt;
    a.mask = g.mask;
    a.R = R;
    a.stamps = w.stamps;
    a.list[0] = w.list[0];
    a.list[1] = w.list[1];
    a.big[0] = w.big[0];
    a.big[1] = w.big[1];
    a.cnt = w.cnt;
    a.stats = w.stats;
    return a;
}

uint64_t solve_cap(const Graph& g, uint32_t algo, const Window& W, uint32_t source, uint32_t* R,
                   const SolveWorkspace& w, uint32_t& stamp, Mailbox& mb, hipStream_t s, bool stats) {
    SolveArgs a = solve_args(g, w, R);
    if (g.MW == 1) return stats ? dispatch_cap<1, true>(algo, g, W, source, a, stamp, mb, s)
                                : dispatch_cap<1, false>(algo, g, W, source, a, stamp, mb, s);
    return stats ? dispatch_cap<2, true>(algo, g, W, source, a, stamp, mb, s)
                 : dispatch_cap<2, false>(algo, g, W, source, a, stamp, mb, s);
}

uint64_t solve_cup(const Graph& g, uint32_t algo, const Window& W, uint32_t* R, const SolveWorkspace& w,
                   uint32_t& stamp, Mailbox& mb, hipStream_t s, bool stats) {
    SolveArgs a = solve_args(g, w, R);
    if (g.MW == 1) return stats ? dispatch_cup<1, true>(algo, g, W, a, stamp, mb, s)
                                : dispatch_cup<1, false>(algo, g, W, a, stamp, mb, s);
    return stats ? dispatch_cup<2, true>(algo, g, W, a, stamp, mb, s)
                 : dispatch_cup<2, false>(algo, g, W, a, stamp, mb, s);
}

}  // namespace evq
