// Versioned-graph builder (Section 4.1): base edge set + K update batches ->
// one CSR over every (src, dst, w) triple present in some snapshot, each edge
// carrying a K-bit presence mask (bit i = snapshot i), the edges present in
// all K snapshots first in each row.
//
// Pipeline (all on the device after one host->device copy of the events):
//   1. encode each event as one sortable key  src | dst | w | t  where
//      t = 0 for the base, 2i+1 for a deletion of batch i, 2i+2 for an
//      addition of batch i (deletions of a batch act before its additions);
//   2. LSD radix sort of the keys, 8-bit digits over the used bits only;
//   3. per run of equal triples, replay its events in t order into the mask
//      (an addition at snapshot s makes the triple present from s until the
//      next event of that triple);
//   4. prefix-sum compaction of the triples whose mask is non-zero;
//   5. row offsets from the sorted sources, then a stable per-row partition
//      (all-present edges first) and the list of partial edges.
#include <algorithm>
#include <chrono>

#include "evq_internal.h"

namespace evq {
namespace {

typedef unsigned __int128 u128;

struct KeyLayout {
    int vb, wb, tb;  // bits of a vertex id, a weight, an event time
    int total() const { return 2 * vb + wb + tb; }
};

__host__ __device__ inline int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b < 1 ? 1 : b;
}

template <typename KT>
__device__ __forceinline__ KT make_key(uint32_t s, uint32_t d, uint32_t w, uint64_t t, KeyLayout L) {
    KT k = (KT)s;
    k = (k << L.vb) | (KT)d;
    k = (k << L.wb) | (KT)w;
    k = (k << L.tb) | (KT)t;
    return k;
}

// Event segments: seg_start[j] = first event index of segment j, j = 0 .. 2K+1
// (segment 0 = base, 2i+1 = deletions of batch i, 2i+2 = additions of batch i);
// seg_start[2K+1] = total.  The segment index is the event time t.
template <typename KT>
__global__ void k_encode(const uint32_t* __restrict__ ev, uint64_t n, const uint64_t* __restrict__ seg_start,
                         int nseg, KeyLayout L, KT* __restrict__ keys) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = nseg - 1;  // largest j with seg_start[j] <= i
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (seg_start[mid] <= i) lo = mid;
            else hi = mid - 1;
        }
        keys[i] = make_key<KT>(ev[3 * i], ev[3 * i + 1], ev[3 * i + 2], (uint32_t)lo, L);
    }
}

// ------------------------------------------------------------------ radix sort

constexpr int kRsBlock = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsBlock * kRsItems;

template <typename KT>
__device__ __forceinline__ uint32_t digit_of(KT k, int shift) {
    return (uint32_t)(k >> shift) & 0xFFu;
}

// Lanes of this wave holding the same 8-bit digit (restricted to `valid` lanes).
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        bool bit = (d >> b) & 1u;
        uint64_t bb = __ballot(bit);
        peers &= bit ? bb : ~bb;
    }
    return peers;
}

template <typename KT>
__global__ void __launch_bounds__(kRsBlock) k_rs_hist(const KT* __restrict__ keys, uint64_t n, int shift,
                                                      uint32_t* __restrict__ hist, uint32_t nb) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
        uint64_t i = base + (uint64_t)r * kRsBlock + threadIdx.x;
        bool valid = i < n;
        uint32_t d = valid ? digit_of(keys[i], shift) : 0u;
        uint64_t peers = match_digit(d, valid);
        if (valid && (peers & lanemask_lt()) == 0) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: keys of a tile keep their order within each digit.
template <typename KT>
__global__ void __launch_bounds__(kRsBlock) k_rs_scatter(const KT* __restrict__ in, KT* __restrict__ out, uint64_t n,
                                                         int shift, const uint32_t* __restrict__ offs, uint32_t nb) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wc[kRsBlock / 64][256];
    const int tid = threadIdx.x, wave = tid >> 6;
    run[tid] = offs[(uint64_t)tid * nb + blockIdx.x];
#pragma unroll
    for (int w = 0; w < kRsBlock / 64; ++w) wc[w][tid] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
        uint64_t i = base + (uint64_t)r * kRsBlock + tid;
        bool valid = i < n;
        KT k = valid ? in[i] : (KT)0;
        uint32_t d = valid ? digit_of(k, shift) : 0u;
        uint64_t peers = match_digit(d, valid);
        uint32_t rank = (uint32_t)__popcll(peers & lanemask_lt());
        if (valid && rank == 0) wc[wave][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t off = run[d];
            for (int w = 0; w < wave; ++w) off += wc[w][d];
            out[off + rank] = k;
        }
        __syncthreads();
        uint32_t tot = 0;
#pragma unroll
        for (int w = 0; w < kRsBlock / 64; ++w) {
            tot += wc[w][tid];
            wc[w][tid] = 0;
        }
        run[tid] += tot;
        __syncthreads();
    }
}

// Sorts keys[0..n) on their low `bits` bits; returns the buffer holding the result.
template <typename KT>
KT* radix_sort(KT* keys, KT* tmp, uint64_t n, int bits, hipStream_t s, Arena& ar, int lo = 0) {
    uint64_t nb64 = (n + kRsTile - 1) / kRsTile;
    uint32_t nb = (uint32_t)nb64;
    uint32_t* hist = ar.alloc<uint32_t>(256ull * nb);
    for (int shift = lo; shift < bits; shift += 8) {
        EVQ_LAUNCH("build_rs_hist", k_rs_hist<KT>, nb, kRsBlock, s, keys, n, shift, hist, nb);
        scan_exclusive(hist, hist, 256ull * nb, nullptr, s, ar);
        EVQ_LAUNCH("build_rs_scatter", k_rs_scatter<KT>, nb, kRsBlock, s, keys, tmp, n, shift, hist, nb);
        KT* t = keys;
        keys = tmp;
        tmp = t;
    }
    ar.release(hist);
    return keys;
}

// ------------------------------------------------------------------ masks

__device__ __forceinline__ int snap_of(uint32_t t) { return t == 0 ? -1 : (int)((t - 1) >> 1); }

template <int MW>
__device__ __forceinline__ void set_range(uint64_t (&m)[MW], int a, int b) {
#pragma unroll
    for (int j = 0; j < MW; ++j) {
        int lo = a - 64 * j, hi = b - 64 * j;
        if (lo < 0) lo = 0;
        if (hi > 64) hi = 64;
        if (hi <= lo) continue;
        uint64_t upto = hi == 64 ? ~0ull : ((1ull << hi) - 1ull);
        uint64_t from = (1ull << lo) - 1ull;
        m[j] |= upto & ~from;
    }
}

template <typename KT, int MW>
__global__ void k_seg_masks(const KT* __restrict__ keys, uint64_t n, KeyLayout L, int K, uint64_t* __restrict__ mtmp,
                            uint32_t* __restrict__ flag) {
    const KT tmask = ((KT)1 << L.tb) - 1;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        KT k = keys[i];
        KT trip = k >> L.tb;
        bool head = (i == 0) || ((keys[i - 1] >> L.tb) != trip);
        uint32_t f = 0;
        if (head) {
            uint64_t m[MW];
#pragma unroll
            for (int j = 0; j < MW; ++j) m[j] = 0;
            uint64_t j = i;
            uint32_t t = (uint32_t)(k & tmask);
            while (true) {
                bool has_next = false;
                uint32_t tn = 0;
                if (j + 1 < n) {
                    KT kn = keys[j + 1];
                    if ((kn >> L.tb) == trip) {
                        has_next = true;
                        tn = (uint32_t)(kn & tmask);
                    }
                }
                bool is_add = (t & 1u) == 0;  // base (0) and additions (even)
                if (is_add) {
                    int a = snap_of(t);
                    if (a < 0) a = 0;
                    set_range<MW>(m, a, has_next ? snap_of(tn) : K);
                }
                if (!has_next) break;
                ++j;
                t = tn;
            }
#pragma unroll
            for (int q = 0; q < MW; ++q) {
                mtmp[i * MW + q] = m[q];
                f |= m[q] != 0;
            }
        }
        flag[i] = f;
    }
}

template <typename KT, int MW>
__global__ void k_compact(const KT* __restrict__ keys, uint64_t n, KeyLayout L, const uint32_t* __restrict__ flag,
                          const uint32_t* __restrict__ pos, const uint64_t* __restrict__ mtmp, Mask<MW> all,
                          uint32_t* __restrict__ c_src, uint32_t* __restrict__ c_dst, uint32_t* __restrict__ c_w,
                          uint64_t* __restrict__ c_mask, uint32_t* __restrict__ c_full) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        if (!flag[i]) continue;
        uint32_t p = pos[i];
        KT k = keys[i] >> L.tb;
        uint32_t w = (uint32_t)(k & (((KT)1 << L.wb) - 1));
        k >>= L.wb;
        uint32_t d = (uint32_t)(k & (((KT)1 << L.vb) - 1));
        k >>= L.vb;
        c_src[p] = (uint32_t)k;
        c_dst[p] = d;
        c_w[p] = w;
        bool full = true;
#pragma unroll
        for (int q = 0; q < MW; ++q) {
            uint64_t m = mtmp[i * MW + q];
            c_mask[(uint64_t)p * MW + q] = m;
            full &= m == all.w[q];
        }
        c_full[p] = full ? 1u : 0u;
    }
}

// row_ptr[v] = first compacted edge with src >= v (sources are sorted), by a
// binary search per vertex, so that long runs of vertices without edges (the
// lowest-degree ids come last) cost no more than any other.
__global__ void k_row_ptr(const uint32_t* __restrict__ c_src, uint64_t E, uint32_t V, uint32_t* __restrict__ row_ptr) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v <= V; v += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t lo = 0, hi = E;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (c_src[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        row_ptr[v] = (uint32_t)lo;
    }
}

template <int MW>
__global__ void k_partition(const uint32_t* __restrict__ c_src, const uint32_t* __restrict__ c_dst,
                            const uint32_t* __restrict__ c_w, const uint64_t* __restrict__ c_mask,
                            const uint32_t* __restrict__ c_full, const uint32_t* __restrict__ fb, uint64_t E,
                            const uint32_t* __restrict__ row_ptr, uint32_t* __restrict__ col,
                            uint32_t* __restrict__ wgt, uint64_t* __restrict__ mask, uint32_t* __restrict__ p_src,
                            uint32_t* __restrict__ p_dst, uint32_t* __restrict__ p_w,
                            uint64_t* __restrict__ p_mask) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < E; i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t u = c_src[i];
        uint32_t c0 = row_ptr[u], c1 = row_ptr[u + 1];
        uint32_t fr = fb[i] - fb[c0];
        uint32_t nf = fb[c1] - fb[c0];
        uint32_t pos;
        if (c_full[i]) {
            pos = c0 + fr;
        } else {
            pos = c0 + nf + ((uint32_t)i - c0 - fr);
            uint32_t p = (uint32_t)i - fb[i];
            p_src[p] = u;
            p_dst[p] = c_dst[i];
            p_w[p] = c_w[i];
#pragma unroll
            for (int q = 0; q < MW; ++q) p_mask[(uint64_t)p * MW + q] = c_mask[i * MW + q];
        }
        col[pos] = c_dst[i];
        wgt[pos] = c_w[i];
#pragma unroll
        for (int q = 0; q < MW; ++q) mask[(uint64_t)pos * MW + q] = c_mask[i * MW + q];
    }
}

__global__ void k_row_split(const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ fb, uint32_t V,
                            uint32_t* __restrict__ row_split) {
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < V; u += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t c0 = row_ptr[u], c1 = row_ptr[u + 1];
        row_split[u] = c0 + (fb[c1] - fb[c0]);
    }
}

// Steps 4-5 from the sorted keys and, at the head of each run of equal
// triples, its mask (mtmp) and whether it is kept (flag).  Releases its inputs.
template <typename KT, int MW>
void finish_build(Graph* g, KT* sorted, uint64_t N, KeyLayout L, uint64_t* mtmp, uint32_t* flag, hipStream_t s,
                  Arena& ar) {
    const uint32_t K = g->K;
    uint32_t* pos = ar.alloc<uint32_t>(N + 1);
    scan_exclusive(flag, pos, N, pos + N, s, ar);
    Mailbox mb(1);
    EVQ_HIP(hipMemcpyAsync(mb.h, pos + N, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipStreamSynchronize(s));
    const uint64_t E = mb.h[0];
    g->E = E;

    Mask<MW> all;
#pragma unroll
    for (int q = 0; q < MW; ++q) {
        int hi = (int)K - 64 * q;
        all.w[q] = hi >= 64 ? ~0ull : (hi <= 0 ? 0ull : ((1ull << hi) - 1ull));
    }

    uint32_t* c_src = ar.alloc<uint32_t>(E + 1);
    uint32_t* c_dst = ar.alloc<uint32_t>(E + 1);
    uint32_t* c_w = ar.alloc<uint32_t>(E + 1);
    uint64_t* c_mask = ar.alloc<uint64_t>((E + 1) * MW);
    uint32_t* c_full = ar.alloc<uint32_t>(E + 1);
    uint32_t* fb = ar.alloc<uint32_t>(E + 1);
    EVQ_LAUNCH("build_compact", (k_compact<KT, MW>), grid_for(N, 256), 256, s, sorted, N, L, flag, pos, mtmp, all,
               c_src, c_dst, c_w, c_mask, c_full);
    ar.release(mtmp);
    ar.release(flag);
    ar.release(pos);
    ar.release(sorted);

    g->row_ptr = (uint32_t*)graph_alloc(*g, ((uint64_t)g->V + 1) * 4, s);
    g->row_split = (uint32_t*)graph_alloc(*g, (uint64_t)g->V * 4, s);
    g->col = (uint32_t*)graph_alloc(*g, E * 4, s);
    g->wgt = (uint32_t*)graph_alloc(*g, E * 4, s);
    g->mask = (uint64_t*)graph_alloc(*g, E * 8 * MW, s);
    g->bytes = ((uint64_t)g->V + 1) * 4 + (uint64_t)g->V * 4 + E * (8 + 8 * MW);

    EVQ_LAUNCH("build_row_ptr", k_row_ptr, grid_for((uint64_t)g->V + 1, 256), 256, s, c_src, E, g->V, g->row_ptr);
    scan_exclusive(c_full, fb, E, fb + E, s, ar);
    EVQ_HIP(hipMemcpyAsync(mb.h, fb + E, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipStreamSynchronize(s));
    const uint64_t n_full = mb.h[0];
    g->n_partial = E - n_full;
    g->p_src = (uint32_t*)graph_alloc(*g, g->n_partial * 4 + 4, s);
    g->p_dst = (uint32_t*)graph_alloc(*g, g->n_partial * 4 + 4, s);
    g->p_w = (uint32_t*)graph_alloc(*g, g->n_partial * 4 + 4, s);
    g->p_mask = (uint64_t*)graph_alloc(*g, g->n_partial * 8 * MW + 16, s);
    g->bytes += g->n_partial * (12 + 8 * MW);
    if (E > 0)
        EVQ_LAUNCH("build_partition", k_partition<MW>, grid_for(E, 256), 256, s, c_src, c_dst, c_w, c_mask, c_full, fb,
                   E, g->row_ptr, g->col, g->wgt, g->mask, g->p_src, g->p_dst, g->p_w, g->p_mask);
    EVQ_LAUNCH("build_row_split", k_row_split, grid_for(g->V, 256), 256, s, g->row_ptr, fb, g->V, g->row_split);
    EVQ_HIP(hipStreamSynchronize(s));
}

template <typename KT, int MW>
void build_impl(Graph* g, const uint32_t* d_ev, uint64_t N, const uint64_t* d_seg, int nseg, KeyLayout L,
                hipStream_t s, Arena& ar) {
    KT* keys = ar.alloc<KT>(N);
    KT* tmp = ar.alloc<KT>(N);
    EVQ_LAUNCH("build_encode", k_encode<KT>, grid_for(N, 256), 256, s, d_ev, N, d_seg, nseg, L, keys);
    KT* sorted = radix_sort<KT>(keys, tmp, N, L.total(), s, ar);
    ar.release(sorted == keys ? tmp : keys);
    uint64_t* mtmp = ar.alloc<uint64_t>(N * MW);
    uint32_t* flag = ar.alloc<uint32_t>(N + 1);
    EVQ_LAUNCH("build_seg_masks", (k_seg_masks<KT, MW>), grid_for(N, 256), 256, s, sorted, N, L, (int)g->K, mtmp,
               flag);
    finish_build<KT, MW>(g, sorted, N, L, mtmp, flag, s, ar);
}

// ------------------------------------------------------------------ ring append

// A[x] = number of rows starting at edge x (x < E); then the source of edge
// e is (rows starting at or before e) - 1.
__global__ void k_row_starts(const uint32_t* __restrict__ row_ptr, uint32_t V, uint64_t E, uint32_t* __restrict__ A) {
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < V; u += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t x = row_ptr[u];
        if (x < E) atomicAdd(&A[x], 1u);
    }
}

// Keys of an append: every edge of the old version (tag 0, its edge index),
// then the batch's deletions (tag 1) and additions (tag 2) with their index.
// The time field of the key is (tag << ib) | index.
template <typename KT>
__global__ void k_encode_append(const uint32_t* __restrict__ A, const uint32_t* __restrict__ S,
                                const uint32_t* __restrict__ col, const uint32_t* __restrict__ wgt, uint64_t E,
                                const uint32_t* __restrict__ ev, uint64_t n_del, uint64_t n_ev, int ib, KeyLayout L,
                                KT* __restrict__ keys) {
    const uint64_t n = E + n_ev;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        if (i < E) {
            keys[i] = make_key<KT>(S[i] + A[i] - 1u, col[i], wgt[i], i, L);
        } else {
            const uint64_t j = i - E;
            const uint64_t tag = j < n_del ? 1u : 2u;
            keys[i] = make_key<KT>(ev[3 * j], ev[3 * j + 1], ev[3 * j + 2], (tag << ib) | j, L);
        }
    }
}

// Per run of equal triples: the old mask (from its tag-0 entry, if any) with
// bit s_new replaced by presence in the new snapshot: present in the old
// newest snapshot (bit s_prev) unless the batch deletes it, or added by the
// batch (deletions act before additions).
template <typename KT, int MW>
__global__ void k_append_masks(const KT* __restrict__ keys, uint64_t n, KeyLayout L, int ib,
                               const uint64_t* __restrict__ old_mask, uint32_t s_prev, uint32_t s_new,
                               uint64_t* __restrict__ mtmp, uint32_t* __restrict__ flag) {
    const KT tmask = ((KT)1 << L.tb) - 1;
    const uint64_t imask = (1ull << ib) - 1ull;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const KT trip = keys[i] >> L.tb;
        const bool head = (i == 0) || ((keys[i - 1] >> L.tb) != trip);
        uint32_t f = 0;
        if (head) {
            uint64_t m[MW];
#pragma unroll
            for (int q = 0; q < MW; ++q) m[q] = 0;
            bool del = false, add = false;
            for (uint64_t j = i; j < n; ++j) {
                const KT k = keys[j];
                if ((k >> L.tb) != trip) break;
                const uint64_t t = (uint64_t)(k & tmask);
                const uint64_t tag = t >> ib, idx = t & imask;
                if (tag == 0) {
#pragma unroll
                    for (int q = 0; q < MW; ++q) m[q] = old_mask[(uint64_t)idx * MW + q];
                } else if (tag == 1) {
                    del = true;
                } else {
                    add = true;
                }
            }
            const bool prev = (m[s_prev >> 6] >> (s_prev & 63)) & 1ull;
            const bool now = add || (prev && !del);
            m[s_new >> 6] &= ~(1ull << (s_new & 63));
            if (now) m[s_new >> 6] |= 1ull << (s_new & 63);
#pragma unroll
            for (int q = 0; q < MW; ++q) {
                mtmp[i * MW + q] = m[q];
                f |= m[q] != 0;
            }
        }
        flag[i] = f;
    }
}

template <typename KT, int MW>
void append_impl(const Graph& old, Graph* g, const uint32_t* d_ev, uint64_t n_del, uint64_t n_ev, KeyLayout L, int ib,
                 hipStream_t s, Arena& ar) {
    const uint64_t E = old.E, N = E + n_ev;
    uint32_t* A = ar.alloc<uint32_t>(E + 1);
    uint32_t* S = ar.alloc<uint32_t>(E + 1);
    if (E) {
        fill_u32(A, E + 1, 0u, s);
        EVQ_LAUNCH("append_rows", k_row_starts, grid_for(old.V, 256), 256, s, old.row_ptr, old.V, E, A);
        scan_exclusive(A, S, E, nullptr, s, ar);
    }
    KT* keys = ar.alloc<KT>(N);
    KT* tmp = ar.alloc<KT>(N);
    EVQ_LAUNCH("append_encode", k_encode_append<KT>, grid_for(N, 256), 256, s, A, S, old.col, old.wgt, E, d_ev, n_del,
               n_ev, ib, L, keys);
    ar.release(A);
    ar.release(S);
    // Only the triple bits are sorted: k_append_masks reads a run's entries in
    // any order (the tag and index in the low bits ride along), and the LSD
    // passes are stable, so the runs come out whole (7 passes instead of 11
    // for the 86-bit keys of the served ring).
    KT* sorted = radix_sort<KT>(keys, tmp, N, L.total(), s, ar, L.tb);
    ar.release(sorted == keys ? tmp : keys);
    uint64_t* mtmp = ar.alloc<uint64_t>(N * MW);
    uint32_t* flag = ar.alloc<uint32_t>(N + 1);
    const uint32_t s_new = (uint32_t)(old.first % old.K);
    const uint32_t s_prev = (uint32_t)((old.first + old.K - 1) % old.K);
    EVQ_LAUNCH("append_masks", (k_append_masks<KT, MW>), grid_for(N, 256), 256, s, sorted, N, L, ib, old.mask, s_prev,
               s_new, mtmp, flag);
    finish_build<KT, MW>(g, sorted, N, L, mtmp, flag, s, ar);
}


// ------------------------------------------------------------------ incremental ring append
//
// An append changes one mask bit of every held edge (the recycled slot takes
// presence in the new snapshot) and adds or drops the few triples its events
// touch, so it need not re-sort the held edges.  It (1) sorts the events and
// merges each triple's run into delete / add flags, (2) looks every distinct
// event triple up in its row (both parts of a row are sorted by (dst, w)),
// (3) recomputes every mask in one streaming pass and classes each edge
// (stays in its part, moves to the other part, or is dropped), (4) sorts the
// movers and the new triples ("inserts") by (row, part, dst, w), and (5)
// places each staying edge at its part's new start + its rank among the
// part's stayers + the inserts before it, and each insert at its rank among
// the part's inserts + the stayers before it.  Every part stays sorted by
// (dst, w), so the arrays equal those of a full rebuild.

enum : uint8_t { kDrop = 0, kStayFull = 1, kToFull = 2, kToPartial = 3, kStayPartial = 4 };

// src_of holds the exclusive scan of A (rows starting at each edge); the
// source of edge e is the number of rows starting at or before e, minus one.
__global__ void k_src_of(const uint32_t* __restrict__ A, uint64_t E, uint32_t* __restrict__ src_of) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < E; e += (uint64_t)gridDim.x * blockDim.x)
        src_of[e] = src_of[e] + A[e] - 1u;
}

template <typename KT>
__global__ void k_ev_keys(const uint32_t* __restrict__ ev, uint64_t n_del, uint64_t n_ev, KeyLayout L,
                          KT* __restrict__ keys) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_ev; i += (uint64_t)gridDim.x * blockDim.x)
        keys[i] = make_key<KT>(ev[3 * i], ev[3 * i + 1], ev[3 * i + 2], i < n_del ? 1u : 2u, L);
}

template <typename KT>
__global__ void k_ev_heads(const KT* __restrict__ keys, uint64_t n, int tb, uint32_t* __restrict__ head) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        head[i] = (i == 0 || (keys[i] >> tb) != (keys[i - 1] >> tb)) ? 1u : 0u;
}

// Distinct event triples (sorted) and their flags: bit 0 deleted, bit 1 added.
template <typename KT>
__global__ void k_ev_unique(const KT* __restrict__ keys, uint64_t n, int tb, const uint32_t* __restrict__ head,
                            const uint32_t* __restrict__ hpos, KT* __restrict__ utrip, uint32_t* __restrict__ ufl) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        if (!head[i]) continue;
        const KT trip = keys[i] >> tb;
        uint32_t fl = 0;
        for (uint64_t j = i; j < n && (keys[j] >> tb) == trip; ++j) fl |= (uint32_t)(keys[j] & 3u);
        utrip[hpos[i]] = trip;
        ufl[hpos[i]] = fl;
    }
}

// First edge of [lo, hi) whose (col, wgt) is not below (d, w) (the range is sorted).
__device__ __forceinline__ uint32_t lower_edge(const uint32_t* __restrict__ col, const uint32_t* __restrict__ wgt,
                                               uint32_t lo, uint32_t hi, uint32_t d, uint32_t w) {
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        const uint32_t c = col[mid];
        if (c < d || (c == d && wgt[mid] < w)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int MW>
__device__ __forceinline__ bool mask_bit(const uint64_t* __restrict__ mask, uint64_t e, uint32_t slot) {
    return (mask[e * MW + (slot >> 6)] >> (slot & 63)) & 1ull;
}

// Each distinct event triple: an edge it names gets its new-snapshot bit
// (added, or present in the newest snapshot and not deleted) in ovr; an added
// triple held in no snapshot is new.
template <typename KT, int MW>
__global__ void k_ev_lookup(const KT* __restrict__ utrip, const uint32_t* __restrict__ ufl, uint32_t nu, KeyLayout L,
                            const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ row_split,
                            const uint32_t* __restrict__ col, const uint32_t* __restrict__ wgt,
                            const uint64_t* __restrict__ mask, uint32_t s_prev, uint8_t* __restrict__ ovr,
                            uint32_t* __restrict__ isnew) {
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < nu; k += (uint64_t)gridDim.x * blockDim.x) {
        const KT t = utrip[k];
        const uint32_t w = (uint32_t)(t & (((KT)1 << L.wb) - 1));
        const uint32_t d = (uint32_t)((t >> L.wb) & (((KT)1 << L.vb) - 1));
        const uint32_t u = (uint32_t)(t >> (L.wb + L.vb));
        const bool del = ufl[k] & 1u, add = (ufl[k] >> 1) & 1u;
        const uint32_t a = row_ptr[u], sp = row_split[u], z = row_ptr[u + 1];
        uint32_t e = lower_edge(col, wgt, a, sp, d, w);
        if (!(e < sp && col[e] == d && wgt[e] == w)) {
            e = lower_edge(col, wgt, sp, z, d, w);
            if (!(e < z && col[e] == d && wgt[e] == w)) e = kNone;
        }
        if (e != kNone) {
            const bool nb = add || (mask_bit<MW>(mask, e, s_prev) && !del);
            ovr[e] = (uint8_t)(2u | (nb ? 1u : 0u));
        }
        isnew[k] = (e == kNone && add) ? 1u : 0u;
    }
}

template <int MW>
__device__ __forceinline__ void new_mask(const uint64_t* __restrict__ mask, const uint8_t* __restrict__ ovr,
                                         uint64_t e, uint32_t s_prev, uint32_t s_new, uint64_t (&m)[MW]) {
#pragma unroll
    for (int q = 0; q < MW; ++q) m[q] = mask[e * MW + q];
    const uint8_t o = ovr[e];
    const bool nb = (o & 2u) ? (o & 1u) : ((m[s_prev >> 6] >> (s_prev & 63)) & 1ull);
    m[s_new >> 6] &= ~(1ull << (s_new & 63));
    if (nb) m[s_new >> 6] |= 1ull << (s_new & 63);
}

template <int MW>
__device__ __forceinline__ bool mask_eq(const uint64_t (&m)[MW], const Mask<MW>& all) {
    bool eq = true;
#pragma unroll
    for (int q = 0; q < MW; ++q) eq &= m[q] == all.w[q];
    return eq;
}

template <int MW>
__device__ __forceinline__ bool mask_any(const uint64_t (&m)[MW]) {
    bool any = false;
#pragma unroll
    for (int q = 0; q < MW; ++q) any |= m[q] != 0;
    return any;
}

template <int MW>
__global__ void k_classify(const uint64_t* __restrict__ mask, const uint8_t* __restrict__ ovr, uint64_t E,
                           uint32_t s_prev, uint32_t s_new, Mask<MW> all, uint8_t* __restrict__ cls,
                           uint32_t* __restrict__ stay, uint32_t* __restrict__ mover) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < E; e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t m0[MW], m[MW];
#pragma unroll
        for (int q = 0; q < MW; ++q) m0[q] = mask[e * MW + q];
        new_mask<MW>(mask, ovr, e, s_prev, s_new, m);
        const bool was = mask_eq<MW>(m0, all), full = mask_eq<MW>(m, all), kept = mask_any<MW>(m);
        uint8_t c = kDrop;
        if (kept) c = was ? (full ? kStayFull : kToPartial) : (full ? kToFull : kStayPartial);
        cls[e] = c;
        stay[e] = (c == kStayFull || c == kStayPartial) ? 1u : 0u;
        mover[e] = (c == kToFull || c == kToPartial) ? 1u : 0u;
    }
}

// Insert keys (u128): u | part | dst | w | payload (32 bits: a mover's edge id,
// or (1 << 31) | the index of a new triple among the distinct event triples).
struct InsLayout {
    int vb, wb;
    __host__ __device__ int total() const { return 2 * vb + wb + 1 + 32; }
};

__device__ __forceinline__ u128 ins_key(uint32_t u, uint32_t part, uint32_t d, uint32_t w, uint32_t payload,
                                        InsLayout L) {
    u128 k = (u128)u;
    k = (k << 1) | (u128)part;
    k = (k << L.vb) | (u128)d;
    k = (k << L.wb) | (u128)w;
    return (k << 32) | (u128)payload;
}

struct InsFields {
    uint32_t u, part, d, w, payload;
};

__device__ __forceinline__ InsFields ins_fields(u128 k, InsLayout L) {
    InsFields f;
    f.payload = (uint32_t)k;
    k >>= 32;
    f.w = (uint32_t)(k & (((u128)1 << L.wb) - 1));
    k >>= L.wb;
    f.d = (uint32_t)(k & (((u128)1 << L.vb) - 1));
    k >>= L.vb;
    f.part = (uint32_t)(k & 1u);
    f.u = (uint32_t)(k >> 1);
    return f;
}

__global__ void k_ins_movers(const uint8_t* __restrict__ cls, const uint32_t* __restrict__ mpos, uint64_t E,
                             const uint32_t* __restrict__ src_of, const uint32_t* __restrict__ col,
                             const uint32_t* __restrict__ wgt, InsLayout L, u128* __restrict__ ikeys) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < E; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint8_t c = cls[e];
        if (c != kToFull && c != kToPartial) continue;
        ikeys[mpos[e]] = ins_key(src_of[e], c == kToFull ? 0u : 1u, col[e], wgt[e], (uint32_t)e, L);
    }
}

template <typename KT, int MW>
__global__ void k_ins_new(const KT* __restrict__ utrip, const uint32_t* __restrict__ isnew,
                          const uint32_t* __restrict__ npos, uint32_t nu, uint32_t nm, KeyLayout EL, InsLayout L,
                          uint32_t s_new, Mask<MW> all, u128* __restrict__ ikeys) {
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < nu; k += (uint64_t)gridDim.x * blockDim.x) {
        if (!isnew[k]) continue;
        const KT t = utrip[k];
        const uint32_t w = (uint32_t)(t & (((KT)1 << EL.wb) - 1));
        const uint32_t d = (uint32_t)((t >> EL.wb) & (((KT)1 << EL.vb) - 1));
        const uint32_t u = (uint32_t)(t >> (EL.wb + EL.vb));
        uint64_t m[MW];
#pragma unroll
        for (int q = 0; q < MW; ++q) m[q] = 0;
        m[s_new >> 6] = 1ull << (s_new & 63);
        const uint32_t part = mask_eq<MW>(m, all) ? 0u : 1u;  // full only when K == 1
        ikeys[nm + npos[k]] = ins_key(u, part, d, w, (1u << 31) | (uint32_t)k, L);
    }
}

// Per (row, part): the inserts' count and first index in the sorted list.
__global__ void k_ins_rows(const u128* __restrict__ ikeys, uint32_t ni, InsLayout L, uint32_t V,
                           uint32_t* __restrict__ icnt, uint32_t* __restrict__ ioff) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < ni; i += (uint64_t)gridDim.x * blockDim.x) {
        const InsFields f = ins_fields(ikeys[i], L);
        const uint64_t slot = (uint64_t)f.part * V + f.u;
        atomicAdd(&icnt[slot], 1u);
        bool head = i == 0;
        if (!head) {
            const InsFields p = ins_fields(ikeys[i - 1], L);
            head = p.u != f.u || p.part != f.part;
        }
        if (head) ioff[slot] = (uint32_t)i;
    }
}

__global__ void k_new_rows(const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ row_split,
                           const uint32_t* __restrict__ cS, const uint32_t* __restrict__ icnt, uint32_t V,
                           uint32_t* __restrict__ len, uint32_t* __restrict__ nf) {
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < V; u += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t a = row_ptr[u], sp = row_split[u], z = row_ptr[u + 1];
        const uint32_t f = cS[sp] - cS[a] + icnt[u];
        nf[u] = f;
        len[u] = f + (cS[z] - cS[sp]) + icnt[(uint64_t)V + u];
    }
}

// The new arrays.
template <int MW>
struct NewCsr {
    uint32_t *rp, *nf, *fx;  // row starts, full edges per row, full edges before each row
    uint32_t *col, *wgt;
    uint64_t* mask;
    uint32_t *p_src, *p_dst, *p_w;
    uint64_t* p_mask;
};

template <int MW>
__device__ __forceinline__ void put_edge(const NewCsr<MW>& o, uint32_t u, uint32_t part, uint32_t pos, uint32_t d,
                                         uint32_t w, const uint64_t (&m)[MW]) {
    o.col[pos] = d;
    o.wgt[pos] = w;
#pragma unroll
    for (int q = 0; q < MW; ++q) o.mask[(uint64_t)pos * MW + q] = m[q];
    if (part) {
        const uint32_t p = pos - (o.fx[u] + o.nf[u]);
        o.p_src[p] = u;
        o.p_dst[p] = d;
        o.p_w[p] = w;
#pragma unroll
        for (int q = 0; q < MW; ++q) o.p_mask[(uint64_t)p * MW + q] = m[q];
    }
}

// Inserts of (u, part) in [i0, i0 + c) whose (dst, w) is below (d, w).
__device__ __forceinline__ uint32_t ins_before(const u128* __restrict__ ikeys, uint32_t i0, uint32_t c, InsLayout L,
                                               uint32_t d, uint32_t w) {
    uint32_t lo = 0, hi = c;
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        const InsFields f = ins_fields(ikeys[i0 + mid], L);
        if (f.d < d || (f.d == d && f.w < w)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int MW>
__global__ void k_place_stayers(uint64_t E, const uint8_t* __restrict__ cls, const uint32_t* __restrict__ src_of,
                                const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ row_split,
                                const uint32_t* __restrict__ col, const uint32_t* __restrict__ wgt,
                                const uint64_t* __restrict__ mask, const uint8_t* __restrict__ ovr, uint32_t s_prev,
                                uint32_t s_new, const uint32_t* __restrict__ cS, const uint32_t* __restrict__ icnt,
                                const uint32_t* __restrict__ ioff, const u128* __restrict__ ikeys, InsLayout L,
                                uint32_t V, NewCsr<MW> o) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < E; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint8_t c = cls[e];
        if (c != kStayFull && c != kStayPartial) continue;
        const uint32_t u = src_of[e], part = c == kStayPartial ? 1u : 0u;
        const uint32_t pstart = part ? row_split[u] : row_ptr[u];
        const uint32_t d = col[e], w = wgt[e];
        uint32_t pos = o.rp[u] + (part ? o.nf[u] : 0u) + (cS[e] - cS[pstart]);
        const uint64_t slot = (uint64_t)part * V + u;
        const uint32_t ic = icnt[slot];
        if (ic) pos += ins_before(ikeys, ioff[slot], ic, L, d, w);
        uint64_t m[MW];
        new_mask<MW>(mask, ovr, e, s_prev, s_new, m);
        put_edge<MW>(o, u, part, pos, d, w, m);
    }
}

template <int MW>
__global__ void k_place_inserts(uint32_t ni, const u128* __restrict__ ikeys, InsLayout L,
                                const uint32_t* __restrict__ row_ptr, const uint32_t* __restrict__ row_split,
                                const uint32_t* __restrict__ col, const uint32_t* __restrict__ wgt,
                                const uint64_t* __restrict__ mask, const uint8_t* __restrict__ ovr, uint32_t s_prev,
                                uint32_t s_new, const uint32_t* __restrict__ cS, const uint32_t* __restrict__ ioff,
                                uint32_t V, NewCsr<MW> o) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < ni; i += (uint64_t)gridDim.x * blockDim.x) {
        const InsFields f = ins_fields(ikeys[i], L);
        const uint32_t a = f.part ? row_split[f.u] : row_ptr[f.u];
        const uint32_t z = f.part ? row_ptr[f.u + 1] : row_split[f.u];
        const uint32_t ps = lower_edge(col, wgt, a, z, f.d, f.w);
        const uint32_t pos = o.rp[f.u] + (f.part ? o.nf[f.u] : 0u) + (uint32_t)(i - ioff[(uint64_t)f.part * V + f.u]) +
                             (cS[ps] - cS[a]);
        uint64_t m[MW];
        if (f.payload >> 31) {
#pragma unroll
            for (int q = 0; q < MW; ++q) m[q] = 0;
            m[s_new >> 6] = 1ull << (s_new & 63);
        } else {
            new_mask<MW>(mask, ovr, f.payload, s_prev, s_new, m);
        }
        put_edge<MW>(o, f.u, f.part, pos, f.d, f.w, m);
    }
}

__global__ void k_new_split(const uint32_t* __restrict__ rp, const uint32_t* __restrict__ nf, uint32_t V,
                            uint32_t* __restrict__ row_split) {
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < V; u += (uint64_t)gridDim.x * blockDim.x)
        row_split[u] = rp[u] + nf[u];
}

template <typename KT, int MW>
void append_incremental(const Graph& old, Graph* g, const uint32_t* d_ev, uint64_t n_del, uint64_t n_ev,
                        hipStream_t s, Arena& ar) {
    const uint32_t V = old.V, K = old.K;
    const uint64_t E = old.E;
    const uint32_t s_new = (uint32_t)(old.first % K), s_prev = (uint32_t)((old.first + K - 1) % K);
    Mask<MW> all;
#pragma unroll
    for (int q = 0; q < MW; ++q) {
        const int hi = (int)K - 64 * q;
        all.w[q] = hi >= 64 ? ~0ull : (hi <= 0 ? 0ull : ((1ull << hi) - 1ull));
    }
    KeyLayout EL;
    EL.vb = bits_for(V - 1);
    EL.wb = bits_for(g->maxw);
    EL.tb = 2;
    InsLayout IL{EL.vb, EL.wb};
    Mailbox mb(4);

    // 1. distinct event triples
    uint32_t nu = 0;
    KT* utrip = ar.alloc<KT>(n_ev + 1);
    uint32_t* ufl = ar.alloc<uint32_t>(n_ev + 1);
    if (n_ev) {
        KT* keys = ar.alloc<KT>(n_ev);
        KT* tmp = ar.alloc<KT>(n_ev);
        EVQ_LAUNCH("append_ev_keys", k_ev_keys<KT>, grid_for(n_ev, 256), 256, s, d_ev, n_del, n_ev, EL, keys);
        KT* sorted = radix_sort<KT>(keys, tmp, n_ev, EL.total(), s, ar, EL.tb);
        uint32_t* head = ar.alloc<uint32_t>(n_ev + 1);
        uint32_t* hpos = ar.alloc<uint32_t>(n_ev + 1);
        EVQ_LAUNCH("append_ev_heads", k_ev_heads<KT>, grid_for(n_ev, 256), 256, s, sorted, n_ev, EL.tb, head);
        scan_exclusive(head, hpos, n_ev, hpos + n_ev, s, ar);
        EVQ_LAUNCH("append_ev_unique", k_ev_unique<KT>, grid_for(n_ev, 256), 256, s, sorted, n_ev, EL.tb, head, hpos,
                   utrip, ufl);
        EVQ_HIP(hipMemcpyAsync(mb.h, hpos + n_ev, 4, hipMemcpyDeviceToHost, s));
        EVQ_HIP(hipStreamSynchronize(s));
        nu = mb.h[0];
    }

    // 2. event triples in the held rows; 3. new masks and classes
    uint8_t* ovr = ar.alloc<uint8_t>(E + 4);
    fill_u32(reinterpret_cast<uint32_t*>(ovr), (E + 4) / 4, 0u, s);
    uint32_t* isnew = ar.alloc<uint32_t>(nu + 1);
    uint32_t* npos = ar.alloc<uint32_t>(nu + 1);
    if (nu) {
        EVQ_LAUNCH("append_ev_lookup", (k_ev_lookup<KT, MW>), grid_for(nu, 256), 256, s, utrip, ufl, nu, EL,
                   old.row_ptr, old.row_split, old.col, old.wgt, old.mask, s_prev, ovr, isnew);
        scan_exclusive(isnew, npos, nu, npos + nu, s, ar);
    } else {
        fill_u32(npos, 1, 0u, s);
    }
    uint8_t* cls = ar.alloc<uint8_t>(E + 1);
    uint32_t* cS = ar.alloc<uint32_t>(E + 1);
    uint32_t* cM = ar.alloc<uint32_t>(E + 1);
    if (E) {
        EVQ_LAUNCH("append_classify", k_classify<MW>, grid_for(E, 256), 256, s, old.mask, ovr, E, s_prev, s_new, all,
                   cls, cS, cM);
        scan_exclusive(cS, cS, E, cS + E, s, ar);
        scan_exclusive(cM, cM, E, cM + E, s, ar);
    } else {
        fill_u32(cS, 1, 0u, s);
        fill_u32(cM, 1, 0u, s);
    }
    EVQ_HIP(hipMemcpyAsync(mb.h, cM + E, 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipMemcpyAsync(mb.h + 1, npos + nu, 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipStreamSynchronize(s));
    const uint32_t nm = mb.h[0], nn = mb.h[1], ni = nm + nn;

    // 4. inserts sorted by (row, part, dst, w), counted per (row, part)
    u128* ikeys = ar.alloc<u128>(ni + 1);
    uint32_t* icnt = ar.alloc<uint32_t>(2ull * V);
    uint32_t* ioff = ar.alloc<uint32_t>(2ull * V);
    fill_u32(icnt, 2ull * V, 0u, s);
    uint32_t* src_of = nullptr;
    if (nm) {
        uint32_t* A = ar.alloc<uint32_t>(E + 1);
        src_of = ar.alloc<uint32_t>(E + 1);
        fill_u32(A, E + 1, 0u, s);
        EVQ_LAUNCH("append_rows", k_row_starts, grid_for(V, 256), 256, s, old.row_ptr, V, E, A);
        scan_exclusive(A, src_of, E, nullptr, s, ar);
        EVQ_LAUNCH("append_src", k_src_of, grid_for(E, 256), 256, s, A, E, src_of);
        ar.release(A);
        EVQ_LAUNCH("append_ins_movers", k_ins_movers, grid_for(E, 256), 256, s, cls, cM, E, src_of, old.col, old.wgt, IL,
                   ikeys);
    }
    if (nn)
        EVQ_LAUNCH("append_ins_new", (k_ins_new<KT, MW>), grid_for(nu, 256), 256, s, utrip, isnew, npos, nu, nm, EL, IL,
                   s_new, all, ikeys);
    if (ni) {
        u128* itmp = ar.alloc<u128>(ni);
        u128* isorted = radix_sort<u128>(ikeys, itmp, ni, IL.total(), s, ar, 32);
        ikeys = isorted;
        EVQ_LAUNCH("append_ins_rows", k_ins_rows, grid_for(ni, 256), 256, s, ikeys, ni, IL, V, icnt, ioff);
    }

    // new row lengths and starts
    NewCsr<MW> o;
    g->row_ptr = o.rp = (uint32_t*)graph_alloc(*g, ((uint64_t)V + 1) * 4, s);
    o.nf = ar.alloc<uint32_t>((uint64_t)V + 1);
    o.fx = ar.alloc<uint32_t>((uint64_t)V + 1);
    uint32_t* len = ar.alloc<uint32_t>((uint64_t)V + 1);
    EVQ_LAUNCH("append_rows_new", k_new_rows, grid_for(V, 256), 256, s, old.row_ptr, old.row_split, cS, icnt, V, len,
               o.nf);
    scan_exclusive(len, o.rp, V, o.rp + V, s, ar);
    scan_exclusive(o.nf, o.fx, V, o.fx + V, s, ar);
    EVQ_HIP(hipMemcpyAsync(mb.h, o.rp + V, 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipMemcpyAsync(mb.h + 1, o.fx + V, 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipStreamSynchronize(s));
    const uint64_t E2 = mb.h[0], NF = mb.h[1];
    g->E = E2;
    g->n_partial = E2 - NF;
    g->row_split = (uint32_t*)graph_alloc(*g, (uint64_t)V * 4, s);
    g->col = o.col = (uint32_t*)graph_alloc(*g, E2 * 4 + 4, s);
    g->wgt = o.wgt = (uint32_t*)graph_alloc(*g, E2 * 4 + 4, s);
    g->mask = o.mask = (uint64_t*)graph_alloc(*g, E2 * 8 * MW + 16, s);
    g->p_src = o.p_src = (uint32_t*)graph_alloc(*g, g->n_partial * 4 + 4, s);
    g->p_dst = o.p_dst = (uint32_t*)graph_alloc(*g, g->n_partial * 4 + 4, s);
    g->p_w = o.p_w = (uint32_t*)graph_alloc(*g, g->n_partial * 4 + 4, s);
    g->p_mask = o.p_mask = (uint64_t*)graph_alloc(*g, g->n_partial * 8 * MW + 16, s);
    g->bytes = ((uint64_t)V + 1) * 4 + (uint64_t)V * 4 + E2 * (8 + 8 * MW) + g->n_partial * (12 + 8 * MW);

    // 5. placement
    if (E) {
        if (!src_of) {
            uint32_t* A = ar.alloc<uint32_t>(E + 1);
            src_of = ar.alloc<uint32_t>(E + 1);
            fill_u32(A, E + 1, 0u, s);
            EVQ_LAUNCH("append_rows", k_row_starts, grid_for(V, 256), 256, s, old.row_ptr, V, E, A);
            scan_exclusive(A, src_of, E, nullptr, s, ar);
            EVQ_LAUNCH("append_src", k_src_of, grid_for(E, 256), 256, s, A, E, src_of);
            ar.release(A);
        }
        EVQ_LAUNCH("append_place", k_place_stayers<MW>, grid_for(E, 256), 256, s, E, cls, src_of, old.row_ptr,
                   old.row_split, old.col, old.wgt, old.mask, ovr, s_prev, s_new, cS, icnt, ioff, ikeys, IL, V, o);
    }
    if (ni)
        EVQ_LAUNCH("append_place_ins", k_place_inserts<MW>, grid_for(ni, 256), 256, s, ni, ikeys, IL, old.row_ptr,
                   old.row_split, old.col, old.wgt, old.mask, ovr, s_prev, s_new, cS, ioff, V, o);
    EVQ_LAUNCH("append_split", k_new_split, grid_for(V, 256), 256, s, o.rp, o.nf, V, g->row_split);
    EVQ_HIP(hipStreamSynchronize(s));
}

// ------------------------------------------------------------------ reverse CSR

// Reverse CSR of the all-present edges (the pull step of the full-window
// intersection solve): one radix sort of packed keys dst | src | w, with the
// edges outside the all-present prefixes given the all-ones key so that they
// sort last.  One wave per source row (grid-stride).
template <typename KT>
__global__ void __launch_bounds__(256) k_rv_keys(const uint32_t* __restrict__ row_ptr,
                                                 const uint32_t* __restrict__ row_split,
                                                 const uint32_t* __restrict__ col, const uint32_t* __restrict__ wgt,
                                                 uint32_t V, int vb, int wb, KT* __restrict__ keys) {
    const uint32_t lane = lane_id();
    const uint64_t nw = (uint64_t)gridDim.x * 4;
    for (uint64_t u = (blockIdx.x * 256ull + threadIdx.x) >> 6; u < V; u += nw) {
        const uint32_t b = row_ptr[u], m = row_split[u], e = row_ptr[u + 1];
        for (uint32_t i = b + lane; i < e; i += 64) {
            KT k = ~(KT)0;
            if (i < m) k = ((((KT)col[i] << vb) | (KT)u) << wb) | (KT)wgt[i];
            keys[i] = k;
        }
    }
}

// Sorted keys -> source, weight and destination per in-edge, and the in-edge
// count (written by the last real key).
template <typename KT>
__global__ void k_rv_decode(const KT* __restrict__ keys, uint64_t E, int vb, int wb, uint32_t* __restrict__ src,
                            uint32_t* __restrict__ w, uint32_t* __restrict__ dst, uint32_t* __restrict__ cnt) {
    const KT none = ~(KT)0;
    const KT vmask = ((KT)1 << vb) - 1, wmask = ((KT)1 << wb) - 1;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < E; i += (uint64_t)gridDim.x * blockDim.x) {
        const KT k = keys[i];
        if (k != none) {
            src[i] = (uint32_t)((k >> wb) & vmask);
            w[i] = (uint32_t)(k & wmask);
            dst[i] = (uint32_t)(k >> (vb + wb));
            if (i + 1 == E || keys[i + 1] == none) cnt[1] = (uint32_t)(i + 1);
        }
    }
}

template <typename KT>
void reverse_sorted(const Graph& g, int vb, int wb, hipStream_t s, Arena& ar) {
    const uint64_t E = g.E;
    KT* keys = ar.alloc<KT>(E);
    KT* tmp = ar.alloc<KT>(E);
    EVQ_LAUNCH("reverse_keys", k_rv_keys<KT>, grid_for((uint64_t)g.V * 64, 256, 8192), 256, s, g.row_ptr,
               g.row_split, g.col, g.wgt, g.V, vb, wb, keys);
    KT* sorted = radix_sort(keys, tmp, E, 2 * vb + wb + 1, s, ar);
    const uint32_t blocks = grid_for(E, 256, 65536);
    EVQ_LAUNCH("reverse_decode", k_rv_decode<KT>, blocks, 256, s, sorted, E, vb, wb, g.rv_src, g.rv_w, g.rv_dst,
               g.rv_cnt);
}

// Vertex numbering by descending degree: every event adds one to the degree
// of both its endpoints (base edges, deletions and additions alike: a rough
// count of how often each vertex's value will be read).  A block first counts
// in an LDS hash table (open addressing, four probes), so that a hub's many
// endpoints cost one device atomic per block rather than one each (the
// same-address device atomics serialise); an endpoint that finds no slot
// goes to the device array directly.
constexpr uint32_t kDegSlots = 2048;
__global__ void __launch_bounds__(256) k_degree(const uint32_t* __restrict__ ev, uint64_t n,
                                                uint32_t* __restrict__ deg) {
    __shared__ uint32_t key[kDegSlots], cnt[kDegSlots];
    for (uint32_t i = threadIdx.x; i < kDegSlots; i += blockDim.x) {
        key[i] = 0xFFFFFFFFu;  // no vertex id (ids are below V <= 2^32 - 1)
        cnt[i] = 0;
    }
    __syncthreads();
    auto add = [&](uint32_t v) {
        const uint32_t h = (v * 2654435761u) >> 21;  // 11 bits: kDegSlots
        for (uint32_t p = 0; p < 4; ++p) {
            const uint32_t slot = (h + p) & (kDegSlots - 1);
            const uint32_t old = atomicCAS(&key[slot], 0xFFFFFFFFu, v);
            if (old == 0xFFFFFFFFu || old == v) {
                atomicAdd(&cnt[slot], 1u);
                return;
            }
        }
        atomicAdd(&deg[v], 1u);
    };
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        add(ev[3 * i]);
        add(ev[3 * i + 1]);
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kDegSlots; i += blockDim.x)
        if (cnt[i]) atomicAdd(&deg[key[i]], cnt[i]);
}

// Sort key of vertex v: the complement of its degree (clamped to db bits)
// above its id, so that ascending keys rank the highest degree first and
// break ties by id.
__global__ void k_order_keys(const uint32_t* __restrict__ deg, uint32_t V, int vb, int db,
                             uint64_t* __restrict__ keys) {
    const uint64_t dmax = (db >= 64 ? ~0ull : (1ull << db) - 1);
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < V; v += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t d = deg[v] < dmax ? deg[v] : dmax;
        keys[v] = ((dmax - d) << vb) | v;
    }
}

// Rank r of the sorted keys is internal id r: iperm[r] = caller id, perm the inverse.
__global__ void k_order_maps(const uint64_t* __restrict__ sorted, uint32_t V, int vb, uint32_t* __restrict__ perm,
                             uint32_t* __restrict__ iperm) {
    const uint64_t vmask = (1ull << vb) - 1;
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < V; r += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)(sorted[r] & vmask);
        iperm[r] = v;
        perm[v] = (uint32_t)r;
    }
}

// Events (src, dst, w) in the caller's ids -> internal ids, in place.
__global__ void k_relabel_events(uint32_t* __restrict__ ev, uint64_t n, const uint32_t* __restrict__ perm) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        ev[3 * i] = perm[ev[3 * i]];
        ev[3 * i + 1] = perm[ev[3 * i + 1]];
    }
}

// Numbers the vertices of a new graph by descending degree over its N events
// (d_ev, device, relabelled in place): g->perm, g->iperm (graph arrays) and
// g->perm_h.  Synchronises s.
void order_vertices(Graph* g, uint32_t* d_ev, uint64_t N, hipStream_t s, Arena& ar) {
    const uint32_t V = g->V;
    uint32_t* deg = ar.alloc<uint32_t>(V);
    uint64_t* keys = ar.alloc<uint64_t>(V);
    uint64_t* tmp = ar.alloc<uint64_t>(V);
    g->perm = (uint32_t*)graph_alloc(*g, (uint64_t)V * 4, s);
    g->iperm = (uint32_t*)graph_alloc(*g, (uint64_t)V * 4, s);
    fill_u32(deg, V, 0u, s);
    EVQ_LAUNCH("order_degree", k_degree, grid_for(N, 256 * 16, 2048), 256, s, d_ev, N, deg);
    const int vb = bits_for(V - 1), db = std::min(32, bits_for(2 * N));
    EVQ_LAUNCH("order_keys", k_order_keys, grid_for(V, 256, 65536), 256, s, deg, V, vb, db, keys);
    uint64_t* sorted = radix_sort<uint64_t>(keys, tmp, V, vb + db, s, ar);
    EVQ_LAUNCH("order_maps", k_order_maps, grid_for(V, 256, 65536), 256, s, sorted, V, vb, g->perm, g->iperm);
    EVQ_LAUNCH("order_relabel", k_relabel_events, grid_for(N, 256, 65536), 256, s, d_ev, N, g->perm);
    auto h = std::make_shared<std::vector<uint32_t>>(V);
    EVQ_HIP(hipMemcpyAsync(h->data(), g->perm, (uint64_t)V * 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipStreamSynchronize(s));
    g->perm_h = std::move(h);
}

}  // namespace

void free_graph(Graph* g, hipStream_t s) {
    if (!g) return;
    std::vector<void*> arrays = {g->row_ptr, g->row_split, g->col,  g->wgt,   g->mask,   g->p_src, g->p_dst,
                                 g->p_w,     g->p_mask,    g->rv_src, g->rv_w, g->rv_dst, g->rv_cnt,
                                 g->perm,    g->iperm};
    for (uint32_t i = 0; i < g->n_wo; ++i) {
        arrays.push_back(g->wo[i].col);
        arrays.push_back(g->wo[i].w);
        arrays.push_back(g->wo[i].nheavy);
    }
    if (g->has_ua) {
        // the caller's allocator frees on the host: the work on s that uses the arrays completes first
        if (s) (void)hipStreamSynchronize(s);
        for (void* p : arrays)
            if (p) g->ua.free(p, g->ua.ctx);
    } else {
        for (void* p : arrays)
            if (p) (void)hipFreeAsync(p, s);
    }
    if (g->rv_ready) (void)hipEventDestroy(g->rv_ready);
    for (uint32_t i = 0; i < kWeightOrders; ++i)
        if (g->wo[i].ready) (void)hipEventDestroy(g->wo[i].ready);
    for (hipEvent_t e : g->uses) (void)hipEventDestroy(e);
    delete g;
}

void build_reverse(const Graph& g, hipStream_t s) {
    fill_u32(g.rv_cnt, 2, 0u, s);
    if (g.V == 0 || g.E == 0) return;
    Arena ar(s, g.has_ua ? &g.ua : nullptr);
    const int vb = bits_for(g.V - 1), wb = bits_for(g.maxw);
    if (2 * vb + wb + 1 <= 64) reverse_sorted<uint64_t>(g, vb, wb, s, ar);
    else reverse_sorted<u128>(g, vb, wb, s, ar);
}

Graph* build_graph(uint32_t V, const evq_edge* base, uint64_t n_base, const evq_batch* batches, uint32_t K,
                   const evq_allocator* ua, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    // ---- validation (host, before any device work)
    uint64_t maxw = 1;
    uint64_t N = n_base;
    auto check = [&](const evq_edge* e, uint64_t n, const char* what) {
        if (n && !e) fail(EVQ_EINVAL, std::string(what) + " is NULL with a non-zero count");
        for (uint64_t i = 0; i < n; ++i) {
            if (e[i].src >= V || e[i].dst >= V)
                fail(EVQ_EINVAL, std::string(what) + ": vertex id out of range at index " + std::to_string(i));
            if (e[i].w == 0) fail(EVQ_EINVAL, std::string(what) + ": zero weight at index " + std::to_string(i));
            if (e[i].w > maxw) maxw = e[i].w;
        }
    };
    check(base, n_base, "base");
    for (uint32_t i = 0; i < K; ++i) {
        check(batches[i].del, batches[i].n_del, "batch deletions");
        check(batches[i].add, batches[i].n_add, "batch additions");
        N += batches[i].n_del + batches[i].n_add;
    }
    if (N >= 0xFFFFFFFEull) fail(EVQ_ERANGE, "more than 2^32 - 2 edge events");

    Graph* g = new Graph();
    g->V = V;
    g->K = K;
    g->MW = K > 64 ? 2 : 1;
    g->maxw = (uint32_t)maxw;
    if (ua) {
        g->ua = *ua;
        g->has_ua = true;
    }
    try {
        Arena ar(s, g->has_ua ? &g->ua : nullptr);
        // A caller's allocator is asked for the event buffer before any device call.
        uint32_t* d_ev = g->has_ua ? ar.alloc<uint32_t>(3 * (N + 1)) : nullptr;
        int dev = 0;
        EVQ_HIP(hipGetDevice(&dev));
        init_mempool(dev);
        g->device = dev;
        // ---- events to the device: [base | del_0 | add_0 | del_1 | add_1 | ...]
        const int nseg = 2 * (int)K + 2;
        std::vector<uint64_t> seg(nseg);
        if (!d_ev) d_ev = ar.alloc<uint32_t>(3 * (N + 1));
        uint64_t at = 0;
        auto put = [&](const evq_edge* e, uint64_t n) {
            if (n) EVQ_HIP(hipMemcpyAsync(d_ev + 3 * at, e, n * sizeof(evq_edge), hipMemcpyHostToDevice, s));
            at += n;
        };
        seg[0] = 0;
        put(base, n_base);
        for (uint32_t i = 0; i < K; ++i) {
            seg[2 * i + 1] = at;
            put(batches[i].del, batches[i].n_del);
            seg[2 * i + 2] = at;
            put(batches[i].add, batches[i].n_add);
        }
        seg[nseg - 1] = at;  // sentinel: never matched for i < N (segments are [seg[j], seg[j+1]))
        uint64_t* d_seg = ar.alloc<uint64_t>(nseg);
        EVQ_HIP(hipMemcpyAsync(d_seg, seg.data(), nseg * sizeof(uint64_t), hipMemcpyHostToDevice, s));

        if (N > 0 && V >= 2 && tuning().vertex_order) order_vertices(g, d_ev, N, s, ar);
        KeyLayout L;
        L.vb = bits_for(V - 1);
        L.wb = bits_for(maxw);
        L.tb = bits_for(2ull * K);
        if (N == 0) {
            g->E = 0;
            g->n_partial = 0;
            g->row_ptr = (uint32_t*)graph_alloc(*g, ((uint64_t)V + 1) * 4, s);
            g->row_split = (uint32_t*)graph_alloc(*g, (uint64_t)V * 4, s);
            fill_u32(g->row_ptr, (uint64_t)V + 1, 0u, s);
            fill_u32(g->row_split, V, 0u, s);
            g->col = (uint32_t*)graph_alloc(*g, 4, s);
            g->wgt = (uint32_t*)graph_alloc(*g, 4, s);
            g->mask = (uint64_t*)graph_alloc(*g, 16, s);
            g->p_src = (uint32_t*)graph_alloc(*g, 4, s);
            g->p_dst = (uint32_t*)graph_alloc(*g, 4, s);
            g->p_w = (uint32_t*)graph_alloc(*g, 4, s);
            g->p_mask = (uint64_t*)graph_alloc(*g, 16, s);
            g->bytes = ((uint64_t)V + 1) * 8;
            EVQ_HIP(hipStreamSynchronize(s));
        } else if (L.total() <= 64) {
            if (g->MW == 1) build_impl<uint64_t, 1>(g, d_ev, N, d_seg, nseg - 1, L, s, ar);
            else build_impl<uint64_t, 2>(g, d_ev, N, d_seg, nseg - 1, L, s, ar);
        } else {
            if (g->MW == 1) build_impl<u128, 1>(g, d_ev, N, d_seg, nseg - 1, L, s, ar);
            else build_impl<u128, 2>(g, d_ev, N, d_seg, nseg - 1, L, s, ar);
        }
        if (g->E >= 0xFFFFFFFEull) fail(EVQ_ERANGE, "more than 2^32 - 2 union edges");
        if (g->perm) g->bytes += (uint64_t)V * 8;
    } catch (...) {
        (void)hipStreamSynchronize(s);
        free_graph(g, s);
        throw;
    }
    EVQ_HIP(hipStreamSynchronize(s));
    g->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return g;
}

// evq_tuning.append_rebuild rebuilds the versioned graph from all held edges
// and the batch (one sort of everything) instead of the incremental append.
bool append_rebuild() { return tuning().append_rebuild != 0; }

Graph* append_graph(const Graph& old, const evq_batch& b, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    const uint32_t V = old.V;
    uint64_t maxw = old.maxw;
    auto check = [&](const evq_edge* e, uint64_t n, const char* what) {
        if (n && !e) fail(EVQ_EINVAL, std::string(what) + " is NULL with a non-zero count");
        for (uint64_t i = 0; i < n; ++i) {
            if (e[i].src >= V || e[i].dst >= V)
                fail(EVQ_EINVAL, std::string(what) + ": vertex id out of range at index " + std::to_string(i));
            if (e[i].w == 0) fail(EVQ_EINVAL, std::string(what) + ": zero weight at index " + std::to_string(i));
            if (e[i].w > maxw) maxw = e[i].w;
        }
    };
    check(b.del, b.n_del, "batch deletions");
    check(b.add, b.n_add, "batch additions");
    const uint64_t n_ev = b.n_del + b.n_add;
    if (old.E + n_ev >= 0xFFFFFFFEull) fail(EVQ_ERANGE, "more than 2^32 - 2 edges and events");

    Graph* g = new Graph();
    g->V = V;
    g->K = old.K;
    g->MW = old.MW;
    g->first = old.first + 1;
    g->maxw = (uint32_t)maxw;
    g->device = old.device;
    g->ua = old.ua;
    g->has_ua = old.has_ua;
    try {
        Arena ar(s, g->has_ua ? &g->ua : nullptr);
        uint32_t* d_ev = ar.alloc<uint32_t>(3 * (n_ev + 1));
        if (b.n_del) EVQ_HIP(hipMemcpyAsync(d_ev, b.del, b.n_del * sizeof(evq_edge), hipMemcpyHostToDevice, s));
        if (b.n_add)
            EVQ_HIP(hipMemcpyAsync(d_ev + 3 * b.n_del, b.add, b.n_add * sizeof(evq_edge), hipMemcpyHostToDevice, s));
        if (old.perm) {  // the new version keeps the old one's numbering
            g->perm = (uint32_t*)graph_alloc(*g, (uint64_t)V * 4, s);
            g->iperm = (uint32_t*)graph_alloc(*g, (uint64_t)V * 4, s);
            g->perm_h = old.perm_h;
            EVQ_HIP(hipMemcpyAsync(g->perm, old.perm, (uint64_t)V * 4, hipMemcpyDeviceToDevice, s));
            EVQ_HIP(hipMemcpyAsync(g->iperm, old.iperm, (uint64_t)V * 4, hipMemcpyDeviceToDevice, s));
            if (n_ev)
                EVQ_LAUNCH("order_relabel", k_relabel_events, grid_for(n_ev, 256, 65536), 256, s, d_ev, n_ev,
                           g->perm);
        }
        KeyLayout L;
        const int ib = bits_for(std::max<uint64_t>(old.E, n_ev));
        L.vb = bits_for(V - 1);
        L.wb = bits_for(maxw);
        L.tb = 2 + ib;
        if (old.E + n_ev == 0) {
            g->E = 0;
            g->n_partial = 0;
            g->row_ptr = (uint32_t*)graph_alloc(*g, ((uint64_t)V + 1) * 4, s);
            g->row_split = (uint32_t*)graph_alloc(*g, (uint64_t)V * 4, s);
            fill_u32(g->row_ptr, (uint64_t)V + 1, 0u, s);
            fill_u32(g->row_split, V, 0u, s);
            g->col = (uint32_t*)graph_alloc(*g, 4, s);
            g->wgt = (uint32_t*)graph_alloc(*g, 4, s);
            g->mask = (uint64_t*)graph_alloc(*g, 16, s);
            g->p_src = (uint32_t*)graph_alloc(*g, 4, s);
            g->p_dst = (uint32_t*)graph_alloc(*g, 4, s);
            g->p_w = (uint32_t*)graph_alloc(*g, 4, s);
            g->p_mask = (uint64_t*)graph_alloc(*g, 16, s);
            g->bytes = ((uint64_t)V + 1) * 8;
        } else if (!append_rebuild()) {
            // incremental: event keys src | dst | w | tag
            if (2 * L.vb + L.wb + 2 <= 64) {
                if (g->MW == 1) append_incremental<uint64_t, 1>(old, g, d_ev, b.n_del, n_ev, s, ar);
                else append_incremental<uint64_t, 2>(old, g, d_ev, b.n_del, n_ev, s, ar);
            } else {
                if (g->MW == 1) append_incremental<u128, 1>(old, g, d_ev, b.n_del, n_ev, s, ar);
                else append_incremental<u128, 2>(old, g, d_ev, b.n_del, n_ev, s, ar);
            }
        } else if (L.total() <= 64) {
            if (g->MW == 1) append_impl<uint64_t, 1>(old, g, d_ev, b.n_del, n_ev, L, ib, s, ar);
            else append_impl<uint64_t, 2>(old, g, d_ev, b.n_del, n_ev, L, ib, s, ar);
        } else if (L.total() <= 128) {
            if (g->MW == 1) append_impl<u128, 1>(old, g, d_ev, b.n_del, n_ev, L, ib, s, ar);
            else append_impl<u128, 2>(old, g, d_ev, b.n_del, n_ev, L, ib, s, ar);
        } else {
            fail(EVQ_ERANGE, "append key does not fit 128 bits");
        }
        if (g->E >= 0xFFFFFFFEull) fail(EVQ_ERANGE, "more than 2^32 - 2 union edges");
        if (g->perm) g->bytes += (uint64_t)V * 8;
    } catch (...) {
        (void)hipStreamSynchronize(s);
        free_graph(g, s);
        throw;
    }
    EVQ_HIP(hipStreamSynchronize(s));
    g->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return g;
}

}  // namespace evq
