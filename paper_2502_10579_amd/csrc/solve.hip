// Bound solver (Section 3, Step 1): single-source relaxation of the query on
// the window's intersection graph (edges present in every snapshot of the
// window) or union graph (edges present in at least one), on the versioned
// graph's CSR with a per-edge mask test.  The union solve starts from the
// intersection result and first relaxes the window-partial edges, i.e. it adds
// the edges missing from the intersection graph (Section 6.2).
//
// One iteration = two kernels:
//   compaction  next-frontier flags -> frontier items in vertex order: the
//               running edge offset and the row position of each vertex with
//               edges, so the expansion reads them contiguously;
//   expansion   the frontier's edges, viewed as one range [0, T), are cut
//               into equal contiguous slices, one per wave; a wave finds its
//               first vertex with a 64-ary search over fo[] and then walks 64
//               edges per step, each lane locating its edge's vertex with a
//               binary search over 64 offsets held in registers.  In the
//               dense iterations of the full-window intersection solve the
//               expansion pulls instead (every vertex over its in-edges); in
//               sparse ones it lists the next frontier itself and the next
//               compaction skips its scan.
// Values improve with fire-and-forget uint32 atomicMin/atomicMax after a plain
// read shows the candidate is better; improved vertices set their bit.
#include "bounds.h"

namespace evq {

namespace {

constexpr int kBlock = 256;
// Tuning knobs (compile-time): blocks of the expansion grid, independent edge
// walks per wave, streaming (non-temporal) loads of the edge arrays.
#ifndef EVQ_EXPAND_BLOCKS
#define EVQ_EXPAND_BLOCKS 2048
#endif
#ifndef EVQ_WALKERS
#define EVQ_WALKERS 1
#endif
#ifndef EVQ_NT_EDGES
#define EVQ_NT_EDGES 0
#endif
constexpr uint32_t kExpandBlocks = EVQ_EXPAND_BLOCKS;
constexpr int kWalkers = EVQ_WALKERS;

template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
#if EVQ_NT_EDGES
    return __builtin_nontemporal_load(p);
#else
    return *p;
#endif
}

struct SolveArgs {
    const uint32_t* row_ptr;
    const uint32_t* row_split;
    const uint32_t* col;
    const uint32_t* wgt;
    const uint64_t* mask;
    uint32_t* R;
    uint8_t* flags;
    // Frontier items, one set per iteration parity (a compaction writes its
    // parity's set, an expansion reads it and, when it appends the next list
    // itself, writes the other):
    uint32_t* fo[2];  // first edge offset in the frontier's edge range
    uint32_t* fd[2];  // row begin minus that offset (edge id = frontier offset + fd)
    uint32_t* fs[2];  // end of the row's all-present prefix
    uint32_t* fv[2];  // the vertex (its value is read when expanded: fresher values save work)
    // Appending expansions: the iteration that last listed each vertex (an
    // iteration's epoch is above every earlier one on this workspace), and the
    // largest frontier edge count at which an expansion appends (0: never).
    uint32_t* stamp;
    uint32_t append_edges;
    uint32_t append_items;  // ... or at most this many frontier vertices (0: never)
    FrontierCounters* cnt;
    unsigned long long* stats;
    uint32_t V;
    // pull step (full-window intersection only): reverse CSR and the share of
    // the all-present edges from which an iteration pulls (kNone: never)
    const uint32_t* rv_src;
    const uint32_t* rv_w;
    const uint32_t* rv_dst;
    const uint32_t* rv_cnt;
    uint32_t pull_frac;
    // bucketed schedule (null: off): heavy edges at the front of each row's
    // all-present prefix in col/wgt (a weight-ordered copy of the rows)
    const uint32_t* nheavy;
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

template <int A>
__host__ __device__ __forceinline__ uint32_t order_key(uint32_t x) {
    return (A == EVQ_SSWP || A == EVQ_VITERBI) ? ~x : x;
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
    mark(a.flags, v);
}

template <bool ST>
__device__ __forceinline__ void count_visits(const SolveArgs& a, uint32_t n) {
    if (!ST) return;
    uint32_t s = wave_sum(n);
    if (lane_id() == 0 && s) atomicAdd(&a.stats[0], (unsigned long long)s);
}

// Flags -> frontier items of parity p, clearing the flags it reads; vertices
// without edges in this solve's graph are dropped.
// With near/far scheduling on (delta > 0), a vertex whose order key (its
// value, complemented where larger is better, so smaller is better) is not
// below the threshold keeps its flag for a later iteration.  With a heavy
// bound, only vertices with at least that many edges are gated: re-expanding
// a vertex costs its whole row, and the rows of the few high-degree vertices
// carry most of the repeated edge visits, while light vertices keep the
// iterations full.
// Bucketed schedule (nheavy set; additive weights): the delta-stepping of
// Meyer and Sanders with the buckets' iterations as frontier iterations.  The
// rows are read from a copy whose all-present prefix holds the heavy edges
// (weight above the bucket width) first and the light ones after.  Flag byte 1
// marks a vertex improved since its last light expansion, 2 one whose light
// edges are done and whose heavy edges wait for the end of its bucket.  A
// bucket ends when the expansion before improved nothing below its bound:
// every value below the bound is then final (a value comes from a flagged
// vertex's edge, so it is at least the smallest flagged value, and a heavy
// edge of the bucket lands above the bound), so the heavy edges of the waiting
// vertices are expanded once, in the same iteration as the light edges of the
// next bucket, which spans the width above the smallest value still flagged.
template <int A, int MODE>
__global__ void __launch_bounds__(kCompactBlock) k_compact_frontier(SolveArgs a, int p, int first) {
    FrontierCounters* const c = a.cnt;
    const bool lh = a.nheavy != nullptr;
    uint32_t bt = 0xFFFFFFFFu;  // bucket bound: light edges of flagged vertices below it are expanded
    bool ended = false;         // the previous bucket ended: its waiting heavy edges are expanded
    if (lh) {
        bt = c->bthr[p ^ 1];
        ended = !first && c->near[p ^ 1] == 0u;
        if (ended) {
            const uint32_t m = umin32(c->nmin[p ^ 1], c->fmin[p ^ 1]);
            if (m != 0xFFFFFFFFu) {
                const uint64_t t = (uint64_t)m + c->bdelta;
                bt = t > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)t;
            }
        }
    }
    const bool skip = compaction_skips(c, p, first);
    if (lh && blockIdx.x == 0 && threadIdx.x == 0) c->bthr[p] = bt;
    if (skip) return;
    const uint32_t thr = c->thr;
    const bool nf = c->delta != 0;
    const uint32_t heavy = nf ? c->heavy : 0u;
    compact_flags(
        a.flags, a.V, &c->packed[p], &c->far[p], &c->fmin[p],
        [&](uint32_t v, uint32_t fl, uint32_t& items, uint32_t& edges, uint32_t& key, uint2& rows) {
            const uint32_t rp = a.row_ptr[v], re = row_end<MODE>(a, v);
            if (MODE != 0) rows.y = a.row_split[v];
            if (lh) {
                const uint32_t nh = a.nheavy[v];
                if (fl == 2u) {
                    if (!ended) return 2u;  // still waiting (no key: not a deferred vertex)
                    rows.x = rp;
                    edges = nh;
                    items = nh ? 1u : 0u;
                    return 0u;
                }
                const uint32_t x = order_key<A>(a.R[v]);
                if (x >= bt) {  // a later bucket
                    key = x;
                    return 1u;
                }
                rows.x = rp + nh;
                edges = re - rows.x;
                items = edges ? 1u : 0u;
                return nh ? 2u : 0u;
            }
            rows.x = rp;
            edges = re - rp;
            items = edges ? 1u : 0u;
            if (!nf || !edges) return 0u;
            key = order_key<A>(a.R[v]);
            if (key < thr || edges < heavy) return 0u;
            items = edges = 0;  // deferred
            return 1u;
        },
        [&](uint32_t v, uint32_t item, uint32_t edge, uint32_t, uint32_t, uint2 rows) {
            a.fo[p][item] = edge;
            a.fd[p][item] = rows.x - edge;
            if (MODE != 0) a.fs[p][item] = rows.y;
            a.fv[p][item] = v;
        },
        heavy ? &c->kall[p] : nullptr);
}

// One 64-edge step of a walker over the frontier's edge range: the lane's
// edge t = base + lane, its source vertex's CSR position and value.
struct Step {
    uint32_t e, split, x, v, cand;
    bool act, want;
};

// Pull step of the full-window intersection solve.  When most of the graph
// is in the frontier, pushing costs one atomic per improving edge; instead
// every vertex takes the best candidate over its all-present in-edges from
// the current values of their sources (a valid Bellman-Ford step: a value
// only ever moves to that of a real path, and only when that is better) and
// writes it once.  The in-edges, sorted by destination, are one range
// [0, n_in) cut into equal slices per wave, walked 64 at a time; each lane
// holds one in-edge and its destination, the lanes of one destination take
// their best by a segmented scan over the wave (DPP row shifts, then the row
// broadcasts), and a destination running on into the next step carries its
// partial best.  A destination whose in-edges all lie in this wave's slice is
// written with a plain store (no other wave writes it); one cut by a slice
// boundary uses the atomic.  Every improved vertex is marked for the next
// frontier, as in the push.

// DPP move of x from another lane (ctrl), rows outside row_mask and lanes
// whose source lane is out of range keep `old`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t old, uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, CTRL, ROW_MASK, 0xF, false);
}

// One round of the segmented scan: take the candidate of the lane CTRL names
// when it holds the same key (destination) and is better.
template <int A, int CTRL, int ROW_MASK>
__device__ __forceinline__ void seg_round(uint32_t key, uint32_t& c) {
    const uint32_t ok = dpp_mov<CTRL, ROW_MASK>(kNone, key);
    const uint32_t oc = dpp_mov<CTRL, ROW_MASK>(Alg<A>::unreached, c);
    if (ok == key && Alg<A>::better(oc, c)) c = oc;
}

// Inclusive segmented best-scan over the wave's 64 lanes, segments = runs of
// equal keys (contiguous): row shifts by 1, 2, 4, 8 within rows of 16 lanes,
// then lane 15 of rows 0 and 2 into rows 1 and 3, then lane 31 into rows 2 and 3.
template <int A>
__device__ __forceinline__ uint32_t seg_scan(uint32_t key, uint32_t c) {
    seg_round<A, 0x111, 0xF>(key, c);  // row_shr:1
    seg_round<A, 0x112, 0xF>(key, c);  // row_shr:2
    seg_round<A, 0x114, 0xF>(key, c);  // row_shr:4
    seg_round<A, 0x118, 0xF>(key, c);  // row_shr:8
    seg_round<A, 0x142, 0xA>(key, c);  // row_bcast:15
    seg_round<A, 0x143, 0xC>(key, c);  // row_bcast:31
    return c;
}

// p[i] of an array below 4 GiB, addressed as its base plus a 32-bit byte
// offset (one 32-bit offset register per load, no 64-bit address pairs).
__device__ __forceinline__ uint32_t load_off32(const uint32_t* __restrict__ p, uint32_t i) {
    return *reinterpret_cast<const uint32_t*>(reinterpret_cast<const char*>(p) + (i << 2));
}

// The reverse CSR and the values are addressed with 32-bit byte offsets
// (the host pulls only with fewer than 2^30 vertices and edges).
template <int A, bool ST>
__device__ __forceinline__ void pull_walk(const SolveArgs& a, uint32_t T) {
    const uint32_t lane = lane_id();
    const uint64_t gw = (blockIdx.x * (uint64_t)kBlock + threadIdx.x) >> 6;
    const uint64_t nw = (uint64_t)gridDim.x * (kBlock / 64);
    uint64_t Rw = (T + nw - 1) / nw;
    Rw = (Rw + 63) & ~63ull;
    const uint64_t b0 = gw * Rw;
    if (b0 >= T) return;
    const uint32_t beg = (uint32_t)b0;
    const uint32_t end = (uint32_t)(b0 + Rw < T ? b0 + Rw : T);
    count_visits<ST>(a, lane == 0 ? end - beg : 0u);
    const uint32_t worst = Alg<A>::unreached;
    // destinations whose in-edges cross this slice's ends (other waves write them too)
    const uint32_t v_lo = a.rv_dst[beg], v_hi = a.rv_dst[end - 1];
    const bool cut_lo = beg > 0 && a.rv_dst[beg - 1] == v_lo;
    const bool cut_hi = end < T && a.rv_dst[end] == v_hi;
    uint32_t carry_v = kNone, carry_c = worst;
    uint32_t nup = 0;
    // in-edges of the step at b0 (the slice's last one for lanes and steps past its end, so that every
    // load is issued unconditionally and in the same order)
    auto edge_at = [&](uint32_t b0, uint32_t& u, uint32_t& w, uint32_t& v) {
        const uint32_t t = b0 + lane < end ? b0 + lane : end - 1;
        u = load_off32(a.rv_src, t);
        w = load_off32(a.rv_w, t);
        v = load_off32(a.rv_dst, t);
    };
    // One step of 64 in-edges: weights w, destinations v, the sources' values
    // x and the destinations' values rv; vn is the next step's destination.
    auto step = [&](uint32_t base, uint32_t w, uint32_t v, uint32_t x, uint32_t rv, uint32_t vn) {
        const bool act = base + lane < end;
        const uint32_t key = act ? v : kNone;  // idle lanes form a segment of their own
        const uint32_t nb = base + 64;
        uint32_t c = act ? Alg<A>::extend(x, w) : worst;
        if (lane == 0 && key == carry_v && Alg<A>::better(carry_c, c)) c = carry_c;
        c = seg_scan<A>(key, c);
        const uint32_t knext = dpp_mov<0x130, 0xF>(kNone, key);  // wave_shl:1: the next lane's key
        const bool seg_end = knext != key;                       // lane 63 keeps kNone: always an end
        // the last segment of this step goes on into the next step of this slice
        const uint32_t first_next = uniform(vn);
        const bool carry = lane == 63 && act && nb < end && key == first_next;
        if (seg_end && act && !carry && Alg<A>::better(c, rv)) {
            const bool shared = (cut_lo && key == v_lo) || (cut_hi && key == v_hi);
            if (!shared) a.R[key] = c;
            else Alg<A>::improve_nr(&a.R[key], c);
            mark(a.flags, key);
            ++nup;
        }
        const uint64_t cm = __ballot(carry);
        carry_v = cm ? lane_value(key, 63) : kNone;
        carry_c = cm ? lane_value(c, 63) : worst;
    };
    // Software pipeline: a step's in-edges are loaded four steps ahead and
    // the values of its sources and destinations two steps ahead.  Each step
    // first runs its own chain, then gathers the values two steps ahead, then
    // loads the in-edges four steps ahead.  Loads complete in issue order, so
    // the wait for a step's values leaves the next step's values and the
    // in-edges of the next two in flight, and the wait for the in-edges to
    // gather from leaves the next step's values in flight.  Four sets of
    // in-edge registers and two of value registers rotate; the loop is
    // unrolled four times by hand so that they are renamed rather than
    // copied (a copy would wait for the load in flight into its source).
    // pipe(): the step at `base` with its in-edges in (u0, w0, v0), the next
    // step's destinations in v1, the in-edges two steps ahead in (u2, v2) and
    // this step's values in (x0, r0); gathers the values two steps ahead into
    // (x0, r0) and loads the in-edges four steps ahead into (u0, w0, v0).
    // False after the slice's last step.
    auto pipe = [&](uint32_t& base, uint32_t& u0, uint32_t& w0, uint32_t& v0, uint32_t v1, uint32_t u2, uint32_t v2,
                    uint32_t& x0, uint32_t& r0) {
        step(base, w0, v0, x0, r0, v1);
        x0 = load_off32(a.R, u2);
        r0 = load_off32(a.R, v2);
        edge_at(base + 256, u0, w0, v0);
        base += 64;
        return base < end;
    };
    uint32_t uA, wA, vA, uB, wB, vB, uC, wC, vC, uD, wD, vD;
    edge_at(beg, uA, wA, vA);
    edge_at(beg + 64, uB, wB, vB);
    edge_at(beg + 128, uC, wC, vC);
    edge_at(beg + 192, uD, wD, vD);
    uint32_t xP = load_off32(a.R, uA), rP = load_off32(a.R, vA), xQ = load_off32(a.R, uB), rQ = load_off32(a.R, vB);
    for (uint32_t base = beg;;) {
        if (!pipe(base, uA, wA, vA, vB, uC, vC, xP, rP)) break;
        if (!pipe(base, uB, wB, vB, vC, uD, vD, xQ, rQ)) break;
        if (!pipe(base, uC, wC, vC, vD, uA, vA, xP, rP)) break;
        if (!pipe(base, uD, wD, vD, vA, uB, vB, xQ, rQ)) break;
    }
    if (ST) {
        const uint32_t su = wave_sum(nup);
        if (lane == 0 && su) atomicAdd(&a.stats[4], (unsigned long long)su);
    }
}

// An appending expansion's improved vertices: the first lane to improve a
// vertex in this iteration (it moves the vertex's stamp to this iteration's
// epoch) lists it for the next iteration, if it has edges in this solve's
// graph.  The wave reserves its items and their edges with one packed atomic
// on the next parity's counter, so the list's running edge offsets ascend
// with the item index as a compaction's do.  Every lane of the wave calls it.
template <int MODE>
__device__ __forceinline__ void append_next(const SolveArgs& a, int p, bool improved, uint32_t v, uint32_t epoch) {
    bool app = false;
    uint32_t rb = 0, deg = 0, sp = 0;
    if (improved && atomicMax(&a.stamp[v], epoch) != epoch) {
        rb = a.row_ptr[v];
        deg = row_end<MODE>(a, v) - rb;
        if (MODE != 0) sp = a.row_split[v];
        app = deg != 0;
    }
    const uint64_t bal = __ballot(app);
    if (!bal) return;
    if (!app) deg = 0;
    const uint32_t incl = wave_incl_scan(deg);
    const uint32_t tot = lane_value(incl, 63);
    unsigned long long base = 0;
    if (lane_id() == 0) base = atomicAdd(&a.cnt->packed[p ^ 1], ((unsigned long long)__popcll(bal) << 32) | tot);
    const uint32_t bi = lane_value((uint32_t)(base >> 32), 0);
    const uint32_t be = lane_value((uint32_t)base, 0);
    if (app) {
        const uint32_t item = bi + (uint32_t)__popcll(bal & lanemask_lt());
        const uint32_t edge = be + incl - deg;
        a.fo[p ^ 1][item] = edge;
        a.fd[p ^ 1][item] = rb - edge;
        if (MODE != 0) a.fs[p ^ 1][item] = sp;
        a.fv[p ^ 1][item] = v;
    }
}

template <int A, int MODE, int MW, bool ST>
__global__ void __launch_bounds__(kBlock) k_expand(SolveArgs a, Mask<MW> W, int p, uint32_t epoch, uint32_t* slot) {
    constexpr int NW = kWalkers;
    const unsigned long long c0 = a.cnt->packed[p];
    bool pull = false;
    if (MODE == 0 && a.pull_frac != kNone) {
        const uint32_t n_in = a.rv_cnt[1];
        pull = n_in && (uint64_t)edges_of(c0) * 1024u >= (uint64_t)n_in * a.pull_frac;
    }
    // a sparse iteration (and no near/far schedule) lists the next frontier itself
    const bool small = (a.append_edges && edges_of(c0) <= a.append_edges) ||
                       (a.append_items && items_of(c0) <= a.append_items);
    const bool lh = a.nheavy != nullptr;
    const bool appends = !pull && small && a.cnt->delta == 0 && !lh;
    const unsigned long long cx = expand_prologue(a.cnt, p, slot, appends);
    const uint32_t n = items_of(cx), T = edges_of(cx);
    if (T == 0) return;
    if (pull) {
        pull_walk<A, ST>(a, a.rv_cnt[1]);
        return;
    }
    const uint32_t* __restrict__ fo = a.fo[p];
    const uint32_t* __restrict__ fd = a.fd[p];
    const uint32_t* __restrict__ fs = a.fs[p];
    const uint32_t* __restrict__ fv = a.fv[p];
    const uint32_t lane = lane_id();
    const uint64_t gw = (blockIdx.x * (uint64_t)kBlock + threadIdx.x) >> 6;
    const uint64_t nw = (uint64_t)gridDim.x * (kBlock / 64);
    // a wave owns NW equal sub-slices of [0, T), each a multiple of 64 edges
    uint64_t Rw = (T + nw * NW - 1) / (nw * NW);
    Rw = (Rw + 63) & ~63ull;
    uint32_t base[NW], end[NW], cur[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) {
        const uint64_t b0 = (gw * NW + j) * Rw;
        base[j] = (uint32_t)(b0 < T ? b0 : T);
        end[j] = (uint32_t)(b0 + Rw < T ? b0 + Rw : T);
    }
    if (base[0] >= end[0]) return;
    count_visits<ST>(a, lane == 0 ? end[NW - 1] - base[0] : 0u);
#pragma unroll
    for (int j = 0; j < NW; ++j) cur[j] = base[j] < end[j] ? wave_search(fo, n, base[j]) : 0u;
    // bucketed schedule: report whether a value below the bucket's bound was
    // written (once per wave) and the smallest one written at or above it
    const uint32_t bt = lh ? a.cnt->bthr[p] : 0u;
    bool near_told = false;
    uint32_t above = 0xFFFFFFFFu;
    while (base[0] < end[0]) {
        Step st[NW];
        uint32_t off[NW];
        // loads of every walker first, so their latencies overlap
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            st[j].act = false;
            st[j].want = false;
            off[j] = 0xFFFFFFFFu;
            if (base[j] >= end[j]) continue;
            const uint32_t idx = cur[j] + lane;
            off[j] = idx < n ? stream_load(fo + idx) : 0xFFFFFFFFu;
            uint32_t dl = 0, sp = 0, xv = 0;
            if (off[j] <= base[j] + 63) {
                dl = stream_load(fd + idx);
                if (MODE != 0) sp = stream_load(fs + idx);
                xv = a.R[stream_load(fv + idx)];
            }
            const uint32_t t = base[j] + lane;
            int o = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const uint32_t q = __shfl(off[j], o + step, 64);
                if (q <= t) o += step;
            }
            st[j].e = t + __shfl(dl, o, 64);
            st[j].split = MODE != 0 ? __shfl(sp, o, 64) : 0u;
            st[j].x = __shfl(xv, o, 64);
            st[j].act = t < end[j];
        }
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            if (!st[j].act) continue;
            if (MODE != 0 && st[j].e >= st[j].split && !partial_in<MODE, MW>(a.mask, st[j].e, W)) continue;
            st[j].v = stream_load(a.col + st[j].e);
            st[j].cand = Alg<A>::extend(st[j].x, stream_load(a.wgt + st[j].e));
            st[j].want = true;
        }
#pragma unroll
        for (int j = 0; j < NW; ++j)
            if (st[j].want) st[j].want = Alg<A>::better(st[j].cand, a.R[st[j].v]);
        // then the updates
        uint32_t nup = 0;
        bool below = false;
        uint32_t amin = 0xFFFFFFFFu;
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            if (st[j].want) {
                Alg<A>::improve_nr(&a.R[st[j].v], st[j].cand);
                if (!appends) mark(a.flags, st[j].v);
                ++nup;
                if (lh) {
                    const uint32_t k = order_key<A>(st[j].cand);
                    if (k < bt) below = true;
                    else amin = k < amin ? k : amin;
                }
            }
            if (appends) append_next<MODE>(a, p, st[j].want, st[j].v, epoch);
        }
        if (lh) {
            if (!near_told && __ballot(below)) {
                if (lane == 0) a.cnt->near[p] = 1u;
                near_told = true;
            }
            const uint32_t m = wave_min(amin);
            above = m < above ? m : above;
        }
        if (ST) {
            const uint32_t su = wave_sum(nup);
            if (lane == 0 && su) atomicAdd(&a.stats[4], (unsigned long long)su);
        }
        // advance: the next step starts at the owner of base + 64
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            if (base[j] >= end[j]) continue;
            const uint32_t nb = base[j] + 64;
            const uint32_t have = (uint32_t)__popcll(__ballot(off[j] <= nb));
            uint32_t adv = have - 1;
            if (have == 64 && cur[j] + 64 < n && fo[cur[j] + 64] <= nb) adv = 64;
            cur[j] += adv;
            base[j] = nb;
        }
    }
    // a plain read first: most waves hold no new minimum and skip the atomic
    if (lh && lane == 0 && above != 0xFFFFFFFFu &&
        above < __hip_atomic_load(&a.cnt->nmin[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
        atomicMin(&a.cnt->nmin[p], above);
}

// Start of a solve: the threshold starts one step above the best key.
// With a bucket width (bdelta > 0), the first bucket spans the width above
// the source's key, and the first compaction reads it as unfinished.
__global__ void k_solve_start(FrontierCounters* c, uint32_t delta, uint32_t heavy, uint32_t* R, uint8_t* flags,
                              uint32_t source, uint32_t at_source, uint32_t bdelta, uint32_t first_bound) {
    if (threadIdx.x == 0) {
        c->delta = delta;
        c->heavy = delta ? heavy : 0u;
        c->thr = delta ? delta : 0xFFFFFFFFu;
        c->far[0] = c->far[1] = 0u;
        c->fmin[0] = c->fmin[1] = 0xFFFFFFFFu;
        c->kall[0] = c->kall[1] = 0xFFFFFFFFu;
        c->bdelta = bdelta;
        c->bthr[0] = c->bthr[1] = bdelta ? first_bound : 0xFFFFFFFFu;
        c->near[0] = c->near[1] = 1u;
        c->nmin[0] = c->nmin[1] = 0xFFFFFFFFu;
        if (R) {
            R[source] = at_source;
            flags[source] = 1;
        }
    }
}

// Union solve, first step: relax every edge present in some but not all
// snapshots of the window, from the values in R (the intersection result).
template <int A, int MW, bool ST>
__global__ void __launch_bounds__(kBlock) k_seed_partial(SolveArgs a, Mask<MW> W, const uint32_t* __restrict__ p_src,
                                                         const uint32_t* __restrict__ p_dst,
                                                         const uint32_t* __restrict__ p_w,
                                                         const uint64_t* __restrict__ p_mask, uint32_t n_partial) {
    const uint32_t stride = gridDim.x * kBlock;
    for (uint32_t base = blockIdx.x * kBlock; base < n_partial; base += stride) {
        const uint32_t q = base + threadIdx.x;
        bool act = false;
        if (q < n_partial) {
            Mask<MW> m = load_mask<MW>(p_mask, q);
            bool any = false, all = true;
#pragma unroll
            for (int j = 0; j < MW; ++j) {
                any |= (m.w[j] & W.w[j]) != 0;
                all &= (m.w[j] & W.w[j]) == W.w[j];
            }
            act = any && !all;
            if (act) {
                const uint32_t v = p_dst[q];
                const uint32_t cand = Alg<A>::extend(a.R[p_src[q]], p_w[q]);
                if (Alg<A>::better(cand, a.R[v])) {
                    Alg<A>::improve_nr(&a.R[v], cand);
                    mark(a.flags, v);
                }
            }
        }
        if (ST) {
            const uint32_t sv = wave_sum(act ? 1u : 0u);
            if (lane_id() == 0 && sv) atomicAdd(&a.stats[5], (unsigned long long)sv);
        }
    }
}

template <int A, int MODE, int MW, bool ST>
uint64_t frontier_loop(SolveArgs a, const Mask<MW>& W, Frontier& f, hipStream_t s, uint64_t max_iters) {
    const uint32_t cblocks = grid_for(a.V, kCompactIds, 4096);
    static const char* names[3] = {"solve_expand_cap_all", "solve_expand_cap", "solve_expand_cup"};
    auto issue = [&](uint64_t, int p, bool first, uint32_t* slot) {
        const uint32_t epoch = ++*f.epoch;
        EVQ_LAUNCH("solve_compact", (k_compact_frontier<A, MODE>), cblocks, kCompactBlock, s, a, p, first ? 1 : 0);
        EVQ_LAUNCH(names[MODE], (k_expand<A, MODE, MW, ST>), kExpandBlocks, kBlock, s, a, W, p, epoch, slot);
    };
    return drive_loop(issue, f.p, s, max_iters, "bound solve", &f.items);
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
    a.flags = f.flags;
    a.fo[0] = f.fo;
    a.fd[0] = f.fd;
    a.fs[0] = f.fs;
    a.fv[0] = f.fv;
    a.fo[1] = f.fo1;
    a.fd[1] = f.fd1;
    a.fs[1] = f.fs1;
    a.fv[1] = f.fv1;
    a.stamp = f.stamp;
    a.append_edges = f.append_edges;
    a.append_items = f.append_items;
    a.cnt = f.cnt;
    a.stats = f.stats;
    a.V = g.V;
    a.rv_src = a.rv_w = a.rv_dst = a.rv_cnt = nullptr;
    a.pull_frac = kNone;
    a.nheavy = nullptr;
    return a;
}

template <int A, int MW, bool ST>
uint64_t solve_cap_t(const Graph& g, const Window& W, uint32_t source, uint32_t* R, Frontier& f, hipStream_t s) {
    SolveArgs a = make_args(g, f, R);
    fill_u32(R, g.V, Alg<A>::unreached, s);
    // the bucketed schedule needs additive weights (SSSP); it replaces near/far and the pull step
    uint32_t bd = 0;
    if (A == EVQ_SSSP && f.bdelta && g.E) {
        if (const WeightOrder* wo = weight_order_ready(g, f.bdelta, s)) {
            a.col = wo->col;
            a.wgt = wo->w;
            a.nheavy = wo->nheavy;
            bd = f.bdelta;
        }
    }
    const uint32_t fd = bd ? 0u : f.delta;
    // a guard against runaway loops: a bucket end takes an iteration of its own at most once per vertex
    const uint64_t cap = bd ? 4ull * g.V + 16 : (uint64_t)g.V + 2;
    EVQ_LAUNCH("solve_start", k_solve_start, 1, 64, s, f.cnt, fd, f.heavy, R, f.flags, source, Alg<A>::at_source,
               bd, bd ? order_key<A>(Alg<A>::at_source) + bd : 0u);
    if (W.full) {
        const uint32_t pf = fd == 0 && !bd && g.E && g.E < (1ull << 30) && g.V < (1u << 30) ? pull_frac() : kNone;
        if (pf != kNone && reverse_ready(g, s)) {
            a.rv_src = g.rv_src;
            a.rv_w = g.rv_w;
            a.rv_dst = g.rv_dst;
            a.rv_cnt = g.rv_cnt;
            a.pull_frac = pf;
        }
        return frontier_loop<A, 0, MW, ST>(a, window_mask<MW>(W), f, s, cap);
    }
    return frontier_loop<A, 1, MW, ST>(a, window_mask<MW>(W), f, s, cap);
}

template <int A, int MW, bool ST>
uint64_t solve_cup_t(const Graph& g, const Window& W, uint32_t* R, Frontier& f, hipStream_t s) {
    SolveArgs a = make_args(g, f, R);
    EVQ_LAUNCH("solve_start", k_solve_start, 1, 64, s, f.cnt, f.delta, f.heavy, (uint32_t*)nullptr, f.flags, 0u,
               0u, 0u, 0u);
    if (g.n_partial)
        EVQ_LAUNCH("solve_seed_partial", (k_seed_partial<A, MW, ST>), grid_for(g.n_partial, kBlock, 16384), kBlock, s,
                   a, window_mask<MW>(W), g.p_src, g.p_dst, g.p_w, g.p_mask, (uint32_t)g.n_partial);
    return frontier_loop<A, 2, MW, ST>(a, window_mask<MW>(W), f, s, (uint64_t)g.V + 2);
}

template <int MW, bool ST>
uint64_t dispatch_cap(uint32_t algo, const Graph& g, const Window& W, uint32_t source, uint32_t* R, Frontier& f,
                      hipStream_t s) {
    switch (algo) {
    case EVQ_SSSP: return solve_cap_t<EVQ_SSSP, MW, ST>(g, W, source, R, f, s);
    case EVQ_BFS: return solve_cap_t<EVQ_BFS, MW, ST>(g, W, source, R, f, s);
    case EVQ_SSWP: return solve_cap_t<EVQ_SSWP, MW, ST>(g, W, source, R, f, s);
    case EVQ_SSNP: return solve_cap_t<EVQ_SSNP, MW, ST>(g, W, source, R, f, s);
    default: return solve_cap_t<EVQ_VITERBI, MW, ST>(g, W, source, R, f, s);
    }
}

template <int MW, bool ST>
uint64_t dispatch_cup(uint32_t algo, const Graph& g, const Window& W, uint32_t* R, Frontier& f, hipStream_t s) {
    switch (algo) {
    case EVQ_SSSP: return solve_cup_t<EVQ_SSSP, MW, ST>(g, W, R, f, s);
    case EVQ_BFS: return solve_cup_t<EVQ_BFS, MW, ST>(g, W, R, f, s);
    case EVQ_SSWP: return solve_cup_t<EVQ_SSWP, MW, ST>(g, W, R, f, s);
    case EVQ_SSNP: return solve_cup_t<EVQ_SSNP, MW, ST>(g, W, R, f, s);
    default: return solve_cup_t<EVQ_VITERBI, MW, ST>(g, W, R, f, s);
    }
}

__global__ void k_init_frontier(FrontierCounters* c, unsigned long long* st, int n) {
    if (threadIdx.x == 0) {
        c->packed[0] = c->packed[1] = 0ull;
        c->status[0] = c->status[1] = 0u;
        c->far[0] = c->far[1] = 0u;
        c->fmin[0] = c->fmin[1] = 0xFFFFFFFFu;
        c->thr = 0xFFFFFFFFu;
        c->delta = 0u;
        c->heavy = 0u;
        c->kall[0] = c->kall[1] = 0xFFFFFFFFu;
    }
    if ((int)threadIdx.x < n) st[threadIdx.x] = 0ull;
}

}  // namespace

Frontier make_frontier(const Graph& g, Workspace& ws, hipStream_t s) {
    Frontier f;
    const uint64_t nflag = flag_bytes(g.V);
    f.flags = ws.buf<uint8_t>(Workspace::kFlags, nflag);
    f.fo = ws.buf<uint32_t>(Workspace::kFo, g.V);
    f.fd = ws.buf<uint32_t>(Workspace::kFd, g.V);
    f.fs = ws.buf<uint32_t>(Workspace::kFs, g.V);
    f.fv = ws.buf<uint32_t>(Workspace::kFv, g.V);
    f.fo1 = ws.buf<uint32_t>(Workspace::kFo1, g.V);
    f.fd1 = ws.buf<uint32_t>(Workspace::kFd1, g.V);
    f.fs1 = ws.buf<uint32_t>(Workspace::kFs1, g.V);
    f.fv1 = ws.buf<uint32_t>(Workspace::kFv1, g.V);
    f.stamp = ws.buf<uint32_t>(Workspace::kStamp, g.V);
    // stamps below every epoch to come: cleared when the buffer is new (or after a no-allocation
    // call, whose scratch another call may have used) and before the epoch counter wraps
    if (f.stamp != ws.stamp_seen || ws.epoch > 0xFFFF0000u) {
        fill_u32(f.stamp, g.V, 0u, s);
        ws.stamp_seen = f.stamp;
        ws.epoch = 0;
    }
    f.epoch = &ws.epoch;
    {
        const evq_tuning tn = tuning();
        f.append_edges = tn.append_edges;
        f.append_items = tn.append_items;
    }
    char* ctl = ws.buf<char>(Workspace::kControl, 512);
    f.cnt = reinterpret_cast<FrontierCounters*>(ctl);
    f.stats = reinterpret_cast<unsigned long long*>(ctl + 128);
    f.aux = reinterpret_cast<unsigned long long*>(ctl + 256);
    // flags are clear after every completed loop; clear them after a failure
    if (ws.fresh_flags || ws.in_use) fill_u32(reinterpret_cast<uint32_t*>(f.flags), nflag / 4, 0u, s);
    ws.fresh_flags = false;
    ws.in_use = true;
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
