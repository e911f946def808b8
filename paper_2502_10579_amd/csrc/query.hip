// One query over a window of snapshots (Algorithm 1 then Algorithm 2):
//   bounds  -> intersection and union solves (solve.hip)
//   K3      -> U = {v : R_cap[v] != R_cup[v]} with compact ids (Step 2,
//              Theorem 2), then the reduced subgraph built from U's rows
//              ("in reverse", Section 6.2): every window edge u -> v with both
//              ends in U, stored as (dst id, w, window lane bits)
//   K4      -> per-snapshot values X[|U|][S] start at R_cap (Step 3); the
//              window-partial edges into U (the reduced addition batches of
//              Step 4) seed them, then one snapshot-oblivious frontier is
//              relaxed until empty, lane i of an edge group testing bit i of
//              the edge's window mask (Section 4.2)
//   K5      -> values[v][i] = R_cap[v] for v outside U, X row of v otherwise
//
// Lane layout: L snapshots of a window map to LG = 8/16/32/64/128 lanes
// (LG >= L, a power of two); a wave holds 64/LG edge groups (one for
// LG >= 64; with LG = 128 each lane serves snapshots i and i + 64).  Rows of
// X are LG uint32 wide, so a group's reads and atomics on one destination row
// are one contiguous, coalesced span.
#include <chrono>

#include "bounds.h"
#include "tasks.h"

namespace evq {

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kRowChunk = 1024;   // union-row edges per compaction task
#ifndef EVQ_RELAX_CHUNK
#define EVQ_RELAX_CHUNK 8
#endif
#ifndef EVQ_RELAX_BLOCKS
#define EVQ_RELAX_BLOCKS 4096
#endif
constexpr uint32_t kRelaxChunk = EVQ_RELAX_CHUNK;  // reduced-subgraph edges per relaxation task
// Largest task count (reduced edges / kRelaxChunk + vertices) whose tasks the
// relax compaction writes itself (evq_tuning.direct_tasks).
uint64_t direct_tasks_limit() { return tuning().direct_tasks; }


template <int NLW>
struct Rec {
    uint32_t dst;
    uint32_t w;
    uint64_t lanes[NLW];
};

template <int LG>
struct Lanes {
    static constexpr int G = LG >= 64 ? 1 : 64 / LG;  // edge groups per wave
    static constexpr int SPL = LG > 64 ? 2 : 1;       // snapshots per lane
    static constexpr int NLW = LG > 64 ? 2 : 1;       // 64-bit lane words per record
    static constexpr uint32_t S = LG;                 // X row stride (uint32)
};

__device__ __forceinline__ uint64_t low_mask(uint32_t n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

// Window lane bits of edge e: bit i = present in the window's snapshot i,
// held in mask bit (b + i) mod K.  The K-bit mask is rotated right by b
// (bits moved past K are cleared by the L-bit lane mask, L <= K).
template <int MW, int NLW>
__device__ __forceinline__ void edge_lanes(const uint64_t* __restrict__ mask, uint32_t e, bool full_edge, uint32_t b,
                                           uint32_t L, uint32_t K, uint64_t (&out)[NLW]) {
    if (full_edge) {
        out[0] = low_mask(L);
        if (NLW == 2) out[NLW - 1] = L > 64 ? low_mask(L - 64) : 0ull;
        return;
    }
    if (MW == 1) {
        uint64_t m = mask[e];
        if (b) m = (m >> b) | (m << (K - b));
        out[0] = m & low_mask(L);
        if (NLW == 2) out[NLW - 1] = 0ull;
        return;
    }
    unsigned __int128 m = ((unsigned __int128)mask[2ull * e + 1] << 64) | mask[2ull * e];
    if (b) m = (m >> b) | (m << (K - b));
    out[0] = (uint64_t)m & low_mask(L);
    if (NLW == 2) out[NLW - 1] = L > 64 ? ((uint64_t)(m >> 64) & low_mask(L - 64)) : 0ull;
}

template <int NLW>
__device__ __forceinline__ bool lanes_partial(const uint64_t (&x)[NLW], uint32_t L) {
    bool any = false, all = true;
#pragma unroll
    for (int j = 0; j < NLW; ++j) {
        any |= x[j] != 0;
        uint32_t n = L > 64u * j ? L - 64u * j : 0u;
        all &= x[j] == low_mask(n > 64 ? 64 : n);
    }
    return any && !all;
}

// ------------------------------------------------------------------ K3: unstable set and reduced subgraph

constexpr int kUBlock = 512;
constexpr int kUPerThread = 8;
constexpr int kUPerBlock = kUBlock * kUPerThread;

// Block-wide exclusive scan of three counters (one value triple per thread).
__device__ __forceinline__ void block_scan3(const uint32_t (&v)[3], uint32_t (&pre)[3], uint32_t (&tot)[3]) {
    __shared__ uint32_t ws[kUBlock / 64][3];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint32_t inc[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        inc[q] = wave_incl_scan(v[q]);
        if (lane == 63) ws[wave][q] = inc[q];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        uint32_t bq = 0, tq = 0;
        for (uint32_t w = 0; w < kUBlock / 64; ++w) {
            if (w < wave) bq += ws[w][q];
            tq += ws[w][q];
        }
        pre[q] = bq + inc[q] - v[q];
        tot[q] = tq;
    }
    __syncthreads();
}

// Counters of the reduction: compact ids, and rows (U vertices with edges)
// packed with their total edge count so rows and edge offsets share an order.
struct UCounters {
    unsigned long long ids;
    unsigned long long rows;  // (rows << 32) | edges
};

// U = {v : R_cap[v] != R_cup[v]} (all vertices when rcap is null).  Every U
// vertex gets a compact id c (ascending within a block), ulist[c] = v and the
// start cuo[c] of its union row in a buffer holding all of U's rows back to
// back; cid_of[v] = kNone for the others, and bit v of ubits says whether v is
// in U.  U vertices with edges are also listed as rows: rv (vertex), rc
// (compact id), ruo (row start).  A thread takes 8 consecutive vertices: two
// 16-byte loads of each bound and two 16-byte stores of their compact ids when
// the bounds are 16-byte aligned and the 8 are in range, one byte of ubits.
__device__ __forceinline__ void load8(const uint32_t* __restrict__ p, uint64_t v0, uint64_t V, bool vec,
                                      uint32_t (&o)[kUPerThread]) {
    if (vec) {
        const uint4 x = reinterpret_cast<const uint4*>(p + v0)[0], y = reinterpret_cast<const uint4*>(p + v0)[1];
        o[0] = x.x, o[1] = x.y, o[2] = x.z, o[3] = x.w, o[4] = y.x, o[5] = y.y, o[6] = y.z, o[7] = y.w;
        return;
    }
#pragma unroll
    for (int k = 0; k < kUPerThread; ++k) o[k] = v0 + k < V ? p[v0 + k] : 0u;
}

__global__ void __launch_bounds__(kUBlock) k_unstable(const uint32_t* __restrict__ rcap,
                                                      const uint32_t* __restrict__ rcup, uint32_t V,
                                                      const uint32_t* __restrict__ row_ptr,
                                                      uint32_t* __restrict__ cid_of, uint32_t* __restrict__ ulist,
                                                      uint32_t* __restrict__ cuo, uint32_t* __restrict__ rv,
                                                      uint32_t* __restrict__ rc, uint32_t* __restrict__ ruo,
                                                      uint8_t* __restrict__ ubits, UCounters* cnt) {
    __shared__ unsigned long long base_id, base_row;
    // 16-byte accesses need aligned bound arrays (the caller's, for evq_query_bounds); cid_of is a workspace buffer
    const bool al = rcap && (((uintptr_t)rcap | (uintptr_t)rcup) % 16 == 0) && (uintptr_t)cid_of % 16 == 0;
    for (uint64_t b0 = (uint64_t)blockIdx.x * kUPerBlock; b0 < V; b0 += (uint64_t)gridDim.x * kUPerBlock) {
        const uint64_t v0 = b0 + (uint64_t)threadIdx.x * kUPerThread;
        const bool vec = al && v0 + kUPerThread <= V;
        uint32_t bits = 0;
        uint32_t deg[kUPerThread];
        uint32_t val[3] = {0, 0, 0};  // ids, rows, edges
        uint32_t cap[kUPerThread], cup[kUPerThread];
        if (rcap) {
            load8(rcap, v0, V, vec, cap);
            load8(rcup, v0, V, vec, cup);
        }
#pragma unroll
        for (int k = 0; k < kUPerThread; ++k) {
            deg[k] = 0;
            const uint64_t v = v0 + k;
            if (v < V && (!rcap || cap[k] != cup[k])) {
                bits |= 1u << k;
                deg[k] = row_ptr[v + 1] - row_ptr[v];
                val[0] += 1;
                val[1] += deg[k] ? 1u : 0u;
                val[2] += deg[k];
            }
        }
        if (v0 < V) ubits[v0 >> 3] = (uint8_t)bits;
        uint32_t pre[3], tot[3];
        block_scan3(val, pre, tot);
        if (threadIdx.x == 0) {
            base_id = tot[0] ? atomicAdd(&cnt->ids, (unsigned long long)tot[0]) : 0ull;
            base_row = tot[1] ? atomicAdd(&cnt->rows, ((unsigned long long)tot[1] << 32) | tot[2]) : 0ull;
        }
        __syncthreads();
        uint32_t id = (uint32_t)base_id + pre[0];
        uint32_t row = (uint32_t)(base_row >> 32) + pre[1];
        uint32_t edge = (uint32_t)base_row + pre[2];
        uint32_t cids[kUPerThread];
#pragma unroll
        for (int k = 0; k < kUPerThread; ++k) {
            cids[k] = kNone;
            const uint64_t v = v0 + k;
            if ((bits >> k) & 1u) {
                cids[k] = id;
                ulist[id] = (uint32_t)v;
                cuo[id] = edge;
                if (deg[k]) {
                    rv[row] = (uint32_t)v;
                    rc[row] = id;
                    ruo[row] = edge;
                    ++row;
                    edge += deg[k];
                }
                ++id;
            }
        }
        if (vec) {
            reinterpret_cast<uint4*>(cid_of + v0)[0] = make_uint4(cids[0], cids[1], cids[2], cids[3]);
            reinterpret_cast<uint4*>(cid_of + v0)[1] = make_uint4(cids[4], cids[5], cids[6], cids[7]);
        } else {
#pragma unroll
            for (int k = 0; k < kUPerThread; ++k)
                if (v0 + k < V) cid_of[v0 + k] = cids[k];
        }
        __syncthreads();
    }
}

struct ReduceArgs {
    const uint32_t* row_ptr;
    const uint32_t* row_split;
    const uint32_t* col;
    const uint32_t* wgt;
    const uint64_t* mask;
    const uint32_t* rv;
    const uint32_t* rc;
    const uint32_t* ruo;
    const uint32_t* cid_of;
    uint32_t* kc;  // kept edges per compact id (must start at zero)
    void* recs;
    uint32_t nR, TU, b, L, K;
};

// The reduced subgraph, built from U's rows (Section 6.2): every edge of a U
// vertex's union row present in some snapshot of the window whose destination
// is also in U, stored as (dst compact id, w, window lane bits) from the
// row's start in a buffer of all U rows.  The rows' edges are walked as one
// range [0, TU) cut into equal slices per wave; each run of lanes in one row
// reserves its slots with one atomic.
template <int MW, int NLW>
__global__ void __launch_bounds__(kBlock) k_reduce(ReduceArgs a) {
    Rec<NLW>* __restrict__ out = static_cast<Rec<NLW>*>(a.recs);
    const uint32_t lane = lane_id();
    const uint64_t gw = (blockIdx.x * (uint64_t)kBlock + threadIdx.x) >> 6;
    const uint64_t nw = (uint64_t)gridDim.x * (kBlock / 64);
    uint64_t Rw = (a.TU + nw - 1) / nw;
    Rw = (Rw + 63) & ~63ull;
    const uint64_t b0 = gw * Rw;
    if (b0 >= a.TU) return;
    const uint32_t end = (uint32_t)(b0 + Rw < a.TU ? b0 + Rw : a.TU);
    uint32_t cur = wave_search(a.ruo, a.nR, (uint32_t)b0);
    for (uint32_t base = (uint32_t)b0; base < end; base += 64) {
        const uint32_t idx = cur + lane;
        const uint32_t off = idx < a.nR ? a.ruo[idx] : 0xFFFFFFFFu;
        uint32_t rb = 0, sp = 0, cc = 0, ro = 0;
        if (off <= base + 63) {
            const uint32_t u = a.rv[idx];
            rb = a.row_ptr[u];
            sp = a.row_split[u];
            cc = a.rc[idx];
            ro = off;
        }
        const uint32_t t = base + lane;
        int o = 0;
#pragma unroll
        for (int step = 32; step >= 1; step >>= 1) {
            const uint32_t q = __shfl(off, o + step, 64);
            if (q <= t) o += step;
        }
        const uint32_t rstart = __shfl(ro, o, 64);
        const uint32_t e = __shfl(rb, o, 64) + (t - rstart);
        const uint32_t split = __shfl(sp, o, 64);
        const uint32_t c = __shfl(cc, o, 64);
        bool keep = false;
        uint32_t cd = 0;
        uint64_t lanes[NLW];
#pragma unroll
        for (int j = 0; j < NLW; ++j) lanes[j] = 0;
        if (t < end) {
            cd = a.cid_of[a.col[e]];
            if (cd != kNone) {
                edge_lanes<MW, NLW>(a.mask, e, e < split, a.b, a.L, a.K, lanes);
                bool any = false;
#pragma unroll
                for (int j = 0; j < NLW; ++j) any |= lanes[j] != 0;
                keep = any;
            }
        }
        // lanes of one row form a contiguous run; its last kept lane reserves
        const uint64_t kmask = __ballot(keep);
        const int prev = __shfl_up(o, 1, 64);  // every lane takes part in the shuffle
        const uint64_t head = __ballot(lane == 0 || prev != o);
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const uint32_t start = 63u - (uint32_t)__clzll((unsigned long long)(head & upto));
        const uint64_t after = head & ~upto;
        const uint32_t stop = after ? (uint32_t)__ffsll((unsigned long long)after) - 2u : 63u;
        const uint64_t run = (stop == 63 ? ~0ull : ((2ull << stop) - 1ull)) & ~((1ull << start) - 1ull);
        const uint64_t rk = kmask & run;
        const uint32_t leader = rk ? 63u - (uint32_t)__clzll((unsigned long long)rk) : 0u;
        uint32_t old = 0;
        if (keep && lane == leader) old = atomicAdd(&a.kc[c], (uint32_t)__popcll(rk));
        old = (uint32_t)__shfl((int)old, (int)leader, 64);
        if (keep) {
            Rec<NLW> r;
            r.dst = cd;
            r.w = a.wgt[e];
#pragma unroll
            for (int j = 0; j < NLW; ++j) r.lanes[j] = lanes[j];
            out[rstart + old + (uint32_t)__popcll(rk & lanemask_lt())] = r;
        }
        // next step starts at the owner of base + 64 (every listed row has edges)
        const uint32_t nb = base + 64;
        const uint32_t have = (uint32_t)__popcll(__ballot(off <= nb));
        uint32_t adv = have - 1;
        if (have == 64 && cur + 64 < a.nR && a.ruo[cur + 64] <= nb) adv = 64;
        cur += adv;
    }
}

// ------------------------------------------------------------------ K4: multi-snapshot relaxation

struct RelaxArgs {
    const uint32_t* cuo;  // row start of each compact id in recs
    const uint32_t* kc;   // its reduced-subgraph edge count
    const void* recs;
    uint32_t* X;
    uint8_t* flags;    // next-frontier flags over compact ids
    // Frontier items written by each compaction, one per improved vertex with
    // edges: its first task in the iteration's task range [0, T) (a task is
    // kRelaxChunk consecutive reduced-subgraph edges of one vertex) and its
    // compact id; then each task as (chunk << 32 | compact id).
    uint32_t* fo;
    uint32_t* fv;
    uint64_t* tasks;
    FrontierCounters* cnt;
    unsigned long long* stats;  // [1] edge visits, [2] lane relaxations, [3] seed edges
    uint32_t nU;
};

template <int LG>
__device__ __forceinline__ bool group_any(bool x) {
    uint64_t bal = __ballot(x);
    if (LG >= 64) return bal != 0;
    const int g = lane_id() / LG;
    return ((bal >> (g * LG)) & low_mask(LG)) != 0;
}

template <bool ST>
__device__ __forceinline__ void add_stat(unsigned long long* p, uint32_t v) {
    if (!ST) return;
    uint32_t s = wave_sum(v);
    if (lane_id() == 0 && s) atomicAdd(p, (unsigned long long)s);
}

// Bitmap of improved compact ids -> frontier items of parity p: per vertex its
// running task offset (the packed reservation counts vertices and tasks) and
// its compact id.  DIRECT: the compaction also writes the tasks itself (through
// a block task list), which saves k_relax_tasks' launch when the reduced
// subgraph is small; with a large one the block that holds a hub would write
// most of an iteration's tasks alone, so k_relax_tasks writes them instead.
template <bool DIRECT>
__global__ void __launch_bounds__(kCompactBlock) k_relax_compact(RelaxArgs r, int p, int first) {
    if (compaction_skips(r.cnt, p, first)) return;
    __shared__ TaskList tl;
    if (DIRECT) task_list_init(tl);
    compact_flags(
        r.flags, r.nU, &r.cnt->packed[p], &r.cnt->far[p], &r.cnt->fmin[p],
        [&](uint32_t c, uint32_t, uint32_t& items, uint32_t& tasks, uint32_t&, uint2&) {
            tasks = (r.kc[c] + kRelaxChunk - 1) / kRelaxChunk;
            items = tasks ? 1u : 0u;
            return 0u;
        },
        [&](uint32_t c, uint32_t item, uint32_t task, uint32_t, uint32_t tasks, uint2) {
            if (!DIRECT) {
                r.fo[item] = task;
                r.fv[item] = c;
            } else if (tasks == 1) {
                r.tasks[task] = c;
            } else {
                task_list_add(tl, r.tasks, c, task, tasks);
            }
        },
        nullptr, [&]() {
            if (DIRECT) task_list_flush(tl, r.tasks);
        });
}

// Frontier items of parity p -> the iteration's tasks (write_tasks).
__global__ void __launch_bounds__(kBlock) k_relax_tasks(RelaxArgs r, int p) {
    const unsigned long long cx = r.cnt->packed[p];
    write_tasks(r.fo, r.fv, items_of(cx), edges_of(cx), r.tasks);
}

// Seeding pass (the parfor over the reduced addition batches in Algorithm 2):
// each window-partial edge u -> v with v in U improves v's lanes from R_cap[u].
// Lanes first test one partial edge each; the wave lists its survivors in LDS
// (compact id, candidate, lane bits), and each lane group then applies them
// eight at a time, issuing the eight destination rows before any update, so
// a survivor costs no chain of dependent loads of its own.
constexpr int kSeedChunk = 8;

template <int A, int MW, int LG, bool ST>
__global__ void __launch_bounds__(kBlock) k_relax_seed(RelaxArgs r, const uint32_t* __restrict__ p_src,
                                                       const uint32_t* __restrict__ p_dst,
                                                       const uint32_t* __restrict__ p_w,
                                                       const uint64_t* __restrict__ p_mask, uint32_t n_partial,
                                                       const uint32_t* __restrict__ cid_of,
                                                       const uint8_t* __restrict__ ubits,
                                                       const uint32_t* __restrict__ rcap, uint32_t b, uint32_t L,
                                                       uint32_t K, uint32_t pb, uint32_t pL) {
    using T = Lanes<LG>;
    __shared__ uint32_t s_cv[kBlock / 64][64], s_cand[kBlock / 64][64];
    __shared__ uint64_t s_lanes[kBlock / 64][64][T::NLW];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const int g = LG >= 64 ? 0 : (int)lane / LG;
    const int i0 = LG >= 64 ? (int)lane : (int)lane % LG;
    const uint32_t gw = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * (kBlock / 64);
    for (uint32_t qb = gw * 64; qb < n_partial; qb += nw * 64) {
        const uint32_t q = qb + lane;
        bool act = q < n_partial;
        uint32_t cv = 0, cand = 0;
        uint64_t lanes[T::NLW];
#pragma unroll
        for (int j = 0; j < T::NLW; ++j) lanes[j] = 0;
        if (act) {
            // the U bitmap (V / 8 bytes, cache-resident) first: most destinations are stable
            const uint32_t d = p_dst[q];
            act = ((ubits[d >> 3] >> (d & 7)) & 1u) != 0u;
            if (act) cv = cid_of[d];
            if (act) {
                // seeded lanes: the relaxed window (b, L); the edge must be
                // partial in the bound window (pb, pL), which contains it
                uint64_t pl[2];
                edge_lanes<MW, 2>(p_mask, q, false, pb, pL, K, pl);
                edge_lanes<MW, T::NLW>(p_mask, q, false, b, L, K, lanes);
                bool any = false;
#pragma unroll
                for (int j = 0; j < T::NLW; ++j) any |= lanes[j] != 0;
                act = any && lanes_partial<2>(pl, pL);
                if (act) cand = Alg<A>::extend(rcap[p_src[q]], p_w[q]);
            }
        }
        const uint64_t bal = __ballot(act);
        add_stat<ST>(&r.stats[3], lane == 0 ? (uint32_t)__popcll(bal) : 0u);
        if (!bal) continue;
        if (act) {
            const uint32_t k = (uint32_t)__popcll(bal & lanemask_lt());
            s_cv[wave][k] = cv;
            s_cand[wave][k] = cand;
#pragma unroll
            for (int j = 0; j < T::NLW; ++j) s_lanes[wave][k][j] = lanes[j];
        }
        wave_lds_sync();
        const uint32_t ns = (uint32_t)__popcll(bal);
        for (uint32_t j0 = 0; j0 < ns; j0 += T::G * kSeedChunk) {
            uint32_t cur[kSeedChunk][T::SPL];
#pragma unroll
            for (int k = 0; k < kSeedChunk; ++k) {
                const uint32_t j = j0 + (uint32_t)g + (uint32_t)(T::G * k);
#pragma unroll
                for (int s = 0; s < T::SPL; ++s) {
                    const int i = i0 + 64 * s;
                    const bool bit = j < ns && ((s_lanes[wave][j < ns ? j : 0][s] >> (i & 63)) & 1ull);
                    cur[k][s] = bit ? r.X[(uint64_t)s_cv[wave][j] * T::S + i] : Alg<A>::unreached;
                }
            }
#pragma unroll
            for (int k = 0; k < kSeedChunk; ++k) {
                const uint32_t j = j0 + (uint32_t)g + (uint32_t)(T::G * k);
                const bool has = j < ns;
                const uint32_t jj = has ? j : 0;
                const uint32_t gcv = s_cv[wave][jj], gcand = s_cand[wave][jj];
                bool imp = false;
#pragma unroll
                for (int s = 0; s < T::SPL; ++s) {
                    const int i = i0 + 64 * s;
                    if (has && ((s_lanes[wave][jj][s] >> (i & 63)) & 1ull) && Alg<A>::better(gcand, cur[k][s])) {
                        Alg<A>::improve_nr(&r.X[(uint64_t)gcv * T::S + i], gcand);
                        imp = true;
                    }
                }
                if (group_any<LG>(imp) && i0 == 0) mark(r.flags, gcv);
            }
        }
        wave_lds_sync();  // the list is read until here
    }
}

// One iteration of Algorithm 2's loop over the snapshot-oblivious frontier.
// Each LG-lane group takes one task (<= kRelaxChunk edges of one vertex);
// the task's edge records and destination rows are loaded before any update.
// The read-only arrays come as their own restrict-qualified arguments: with
// one group per wave (LG >= 64) a task, its row bounds and its edge records
// are wave-uniform, and the compiler may then fetch them with scalar loads,
// since no store of the kernel can reach them.
template <int A, int LG, bool ST>
__global__ void __launch_bounds__(kBlock)
    k_relax(RelaxArgs r, const uint64_t* __restrict__ tasks, const uint32_t* __restrict__ cuo,
            const uint32_t* __restrict__ kc, const void* __restrict__ recs_v, int p, uint32_t* slot) {
    using T = Lanes<LG>;
    const unsigned long long cx = expand_prologue(r.cnt, p, slot);
    const uint32_t n = edges_of(cx);  // tasks (the items are their vertices)
    if (n == 0) return;
    const Rec<T::NLW>* __restrict__ recs = static_cast<const Rec<T::NLW>*>(recs_v);
    const uint32_t lane = lane_id();
    const int g = LG >= 64 ? 0 : (int)lane / LG;
    const int i0 = LG >= 64 ? (int)lane : (int)lane % LG;
    const uint32_t gw = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * (kBlock / 64);
    for (uint32_t tb = gw * T::G; tb < n; tb += nw * T::G) {
        const uint32_t ti = tb + g;
        uint32_t c = 0, e0 = 0, ne = 0;
        if (ti < n) {
            uint64_t tk = tasks[ti];
            if (T::G == 1) tk = ((uint64_t)uniform((uint32_t)(tk >> 32)) << 32) | uniform((uint32_t)tk);
            c = (uint32_t)tk;
            const uint32_t rb = cuo[c], re = rb + kc[c];
            e0 = rb + (uint32_t)(tk >> 32) * kRelaxChunk;
            ne = re - e0 < kRelaxChunk ? re - e0 : kRelaxChunk;
        }
        uint32_t xu[T::SPL];
#pragma unroll
        for (int s = 0; s < T::SPL; ++s) xu[s] = ne ? r.X[(uint64_t)c * T::S + i0 + 64 * s] : Alg<A>::unreached;
        Rec<T::NLW> rec[kRelaxChunk];
        uint32_t cur[kRelaxChunk][T::SPL];
        uint32_t lanes_done = 0;
#pragma unroll
        for (uint32_t k = 0; k < kRelaxChunk; ++k) {
            if (k < ne) {
                rec[k] = recs[e0 + k];
            } else {
                rec[k].dst = 0;
                rec[k].w = 0;
#pragma unroll
                for (int j = 0; j < T::NLW; ++j) rec[k].lanes[j] = 0;
            }
        }
#pragma unroll
        for (uint32_t k = 0; k < kRelaxChunk; ++k)
#pragma unroll
            for (int s = 0; s < T::SPL; ++s) {
                const int i = i0 + 64 * s;
                const bool bit = (rec[k].lanes[s] >> (i & 63)) & 1ull;
                cur[k][s] = bit ? r.X[(uint64_t)rec[k].dst * T::S + i] : Alg<A>::unreached;
            }
#pragma unroll
        for (uint32_t k = 0; k < kRelaxChunk; ++k) {
            bool imp = false;
#pragma unroll
            for (int s = 0; s < T::SPL; ++s) {
                const int i = i0 + 64 * s;
                if ((rec[k].lanes[s] >> (i & 63)) & 1ull) {
                    ++lanes_done;
                    const uint32_t cand = Alg<A>::extend(xu[s], rec[k].w);
                    if (Alg<A>::better(cand, cur[k][s])) {
                        Alg<A>::improve_nr(&r.X[(uint64_t)rec[k].dst * T::S + i], cand);
                        imp = true;
                    }
                }
            }
            if (group_any<LG>(imp) && i0 == 0) mark(r.flags, rec[k].dst);
        }
        if (ST) {
            add_stat<true>(&r.stats[1], i0 == 0 ? ne : 0u);
            add_stat<true>(&r.stats[2], lanes_done);
        }
    }
}

// The same iteration with the block staging its tasks in LDS: each round the
// block takes (waves x lane groups x kStagePerWave) tasks, its threads load
// their headers (task, row start and length) and then all their edge records
// (one load each), and after a barrier every lane group takes kStagePerWave
// (2 or 4) of the staged tasks and issues the source rows and the destination
// rows of all of them before any update.  A task's records then cost one
// coalesced load per thread of the block instead of a chain of dependent
// loads per group, and each group keeps kStagePerWave * (1 + 8) row loads in
// flight (Section 4.2: edge records and hot frontier chunks staged on chip,
// values laid out snapshot-minor).
template <int A, int LG, int kStagePerWave, bool ST>
__global__ void __launch_bounds__(kBlock)
    k_relax_staged(RelaxArgs r, const uint64_t* __restrict__ tasks, const uint32_t* __restrict__ cuo,
                   const uint32_t* __restrict__ kc, const void* __restrict__ recs_v, int p, uint32_t* slot) {
    using T = Lanes<LG>;
    constexpr int kGroups = (kBlock / 64) * T::G;             // lane groups per block
    constexpr int kStageTasks = kGroups * kStagePerWave;      // tasks per round
    constexpr int kStageRecs = kStageTasks * (int)kRelaxChunk;
    __shared__ uint32_t s_c[kStageTasks], s_e0[kStageTasks], s_ne[kStageTasks];
    __shared__ Rec<T::NLW> s_rec[kStageTasks][kRelaxChunk];
    const unsigned long long cx = expand_prologue(r.cnt, p, slot);
    const uint32_t n = edges_of(cx);  // tasks
    if (n == 0) return;
    const Rec<T::NLW>* __restrict__ recs = static_cast<const Rec<T::NLW>*>(recs_v);
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const int g = LG >= 64 ? 0 : (int)lane / LG;
    const int i0 = LG >= 64 ? (int)lane : (int)lane % LG;
    const uint32_t grp = wave * T::G + g;  // this lane group's index in the block
    for (uint32_t t0 = blockIdx.x * (uint32_t)kStageTasks; t0 < n; t0 += gridDim.x * (uint32_t)kStageTasks) {
        for (uint32_t j = threadIdx.x; j < (uint32_t)kStageTasks; j += kBlock) {
            const uint32_t ti = t0 + j;
            uint32_t c = 0, e0 = 0, ne = 0;
            if (ti < n) {
                const uint64_t tk = tasks[ti];
                c = (uint32_t)tk;
                const uint32_t rb = cuo[c], re = rb + kc[c];
                e0 = rb + (uint32_t)(tk >> 32) * kRelaxChunk;
                ne = re - e0 < kRelaxChunk ? re - e0 : kRelaxChunk;
            }
            s_c[j] = c;
            s_e0[j] = e0;
            s_ne[j] = ne;
        }
        __syncthreads();
        for (uint32_t j = threadIdx.x; j < (uint32_t)kStageRecs; j += kBlock) {
            const uint32_t tt = j / kRelaxChunk, k = j % kRelaxChunk;
            Rec<T::NLW> rc;
            rc.dst = 0;
            rc.w = 0;
#pragma unroll
            for (int q = 0; q < T::NLW; ++q) rc.lanes[q] = 0;
            if (k < s_ne[tt]) rc = recs[s_e0[tt] + k];
            s_rec[tt][k] = rc;
        }
        __syncthreads();
        uint32_t xu[kStagePerWave][T::SPL];
        uint32_t cur[kStagePerWave][kRelaxChunk][T::SPL];
#pragma unroll
        for (int q = 0; q < kStagePerWave; ++q) {
            const uint32_t tt = grp * kStagePerWave + q;
            const uint32_t c = s_c[tt], ne = s_ne[tt];
#pragma unroll
            for (int s = 0; s < T::SPL; ++s)
                xu[q][s] = ne ? r.X[(uint64_t)c * T::S + i0 + 64 * s] : Alg<A>::unreached;
#pragma unroll
            for (uint32_t k = 0; k < kRelaxChunk; ++k)
#pragma unroll
                for (int s = 0; s < T::SPL; ++s) {
                    const int i = i0 + 64 * s;
                    const bool bit = (s_rec[tt][k].lanes[s] >> (i & 63)) & 1ull;
                    cur[q][k][s] = bit ? r.X[(uint64_t)s_rec[tt][k].dst * T::S + i] : Alg<A>::unreached;
                }
        }
        uint32_t lanes_done = 0, edges_done = 0;
#pragma unroll
        for (int q = 0; q < kStagePerWave; ++q) {
            const uint32_t tt = grp * kStagePerWave + q;
            edges_done += s_ne[tt];
#pragma unroll
            for (uint32_t k = 0; k < kRelaxChunk; ++k) {
                const Rec<T::NLW> rc = s_rec[tt][k];
                bool imp = false;
#pragma unroll
                for (int s = 0; s < T::SPL; ++s) {
                    const int i = i0 + 64 * s;
                    if ((rc.lanes[s] >> (i & 63)) & 1ull) {
                        ++lanes_done;
                        const uint32_t cand = Alg<A>::extend(xu[q][s], rc.w);
                        if (Alg<A>::better(cand, cur[q][k][s])) {
                            Alg<A>::improve_nr(&r.X[(uint64_t)rc.dst * T::S + i], cand);
                            imp = true;
                        }
                    }
                }
                if (group_any<LG>(imp) && i0 == 0) mark(r.flags, rc.dst);
            }
        }
        if (ST) {
            add_stat<true>(&r.stats[1], i0 == 0 ? edges_done : 0u);
            add_stat<true>(&r.stats[2], lanes_done);
        }
        __syncthreads();  // the staged tasks are read until here
    }
}

// ------------------------------------------------------------------ init / K5

// X[c][i] = R_cap[ulist[c]]: 16-byte stores when a row holds a multiple of 4 lanes.
template <int LG>
__global__ void k_xinit(const uint32_t* __restrict__ ulist, uint32_t nU, const uint32_t* __restrict__ rcap,
                        uint32_t* __restrict__ X) {
    if constexpr (LG % 4 == 0) {
        constexpr uint32_t Q = LG / 4;  // 16-byte words per row
        const uint64_t n = (uint64_t)nU * Q;
        uint4* __restrict__ X4 = reinterpret_cast<uint4*>(X);
        for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n;
             k += (uint64_t)gridDim.x * blockDim.x) {
            const uint32_t b = rcap[ulist[k / Q]];
            X4[k] = make_uint4(b, b, b, b);
        }
    } else {
        const uint64_t n = (uint64_t)nU * LG;
        for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n;
             k += (uint64_t)gridDim.x * blockDim.x)
            X[k] = rcap[ulist[k / LG]];
    }
}

// Plain evaluation: every vertex starts unreached except the source (compact
// ids follow the reduction's order, so the source is found through ulist).
template <int LG>
__global__ void k_xinit_plain(const uint32_t* __restrict__ ulist, uint32_t nU, uint32_t source, uint32_t unreached,
                              uint32_t at_source, uint32_t* __restrict__ X) {
    const uint64_t n = (uint64_t)nU * LG;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x)
        X[k] = ulist[k / LG] == source ? at_source : unreached;
}

__global__ void k_init_frontier_stats(unsigned long long* st) {
    if (threadIdx.x >= 1 && threadIdx.x < 4) st[threadIdx.x] = 0ull;
}

__global__ void k_mark_source(uint8_t* flags, const uint32_t* __restrict__ cid_of, uint32_t source) {
    if (threadIdx.x == 0) flags[cid_of[source]] = 1;
}

// 16-byte store that streams past the caches (the output is written once and
// not read again by the query).
__device__ __forceinline__ void stream_store(uint4 v, uint4* p) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    u32x4 x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(p));
}

// values[v * OS + i], i < L (L % 4 == 0, L <= 256, 16-byte aligned rows of
// stride OS).  A wave takes 64 consecutive vertices: one coalesced load of
// their compact ids (and of R_cap for the stable ones), then their rows as
// lane-contiguous 16-byte streaming stores, 64 / (L / 4) rows per
// instruction, with eight instructions' values gathered before any is
// stored, so that the per-row loads do not serialise the stores.
__global__ void __launch_bounds__(kBlock) k_writeback4(uint32_t V, uint32_t L, uint32_t S, uint32_t OS,
                                                       const uint32_t* __restrict__ perm,
                                                       const uint32_t* __restrict__ cid_of,
                                                       const uint32_t* __restrict__ rcap,
                                                       const uint32_t* __restrict__ X, uint32_t* __restrict__ out) {
    const uint32_t Lq = L >> 2, OSq = OS >> 2, Sq = S >> 2;
    const uint32_t lane = lane_id();
    const uint32_t rpi = 64 / Lq;  // rows per store instruction
    const uint32_t r = lane / Lq, j = lane - r * Lq;
    const bool on = r < rpi;
    const uint32_t steps = (64 + rpi - 1) / rpi;
    const uint64_t nw = (uint64_t)gridDim.x * (kBlock / 64);
    uint4* __restrict__ o4 = reinterpret_cast<uint4*>(out);
    const uint4* __restrict__ x4 = reinterpret_cast<const uint4*>(X);
    for (uint64_t w = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; w * 64 < V; w += nw) {
        const uint64_t v0 = w * 64;
        uint32_t c = kNone, b = 0;
        if (v0 + lane < V) {
            const uint32_t u = perm ? perm[v0 + lane] : (uint32_t)(v0 + lane);
            if (cid_of) c = cid_of[u];
            if (c == kNone) b = rcap[u];
        }
        for (uint32_t s0 = 0; s0 < steps; s0 += 8) {
            uint4 val[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const uint32_t k = (s0 + t) * rpi + r;  // row within the wave's 64
                const uint32_t ck = (uint32_t)__shfl((int)c, (int)(k & 63), 64);
                const uint32_t bk = (uint32_t)__shfl((int)b, (int)(k & 63), 64);
                val[t] = make_uint4(bk, bk, bk, bk);
                if (on && k < 64 && v0 + k < V && ck != kNone) val[t] = x4[(uint64_t)ck * Sq + j];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const uint32_t k = (s0 + t) * rpi + r;
                if (on && k < 64 && v0 + k < V) stream_store(val[t], &o4[(v0 + k) * OSq + j]);
            }
        }
    }
}

// values[v * L + i] with rows stored back to back (4 <= L <= 256): the 64 rows
// of a wave are one contiguous range of 64 L values that starts 256-byte
// aligned, written as lane-contiguous 16-byte streaming stores, one of which
// may straddle two rows.  The rows' compact ids and R_cap values are staged in
// LDS; magic = floor(2^32 / L) + 1 turns the row lookup into a multiply-high,
// exact for offsets below 64 L.
__global__ void __launch_bounds__(kBlock) k_writeback_flat(uint32_t V, uint32_t L, uint32_t S, uint32_t magic,
                                                           const uint32_t* __restrict__ perm,
                                                           const uint32_t* __restrict__ cid_of,
                                                           const uint32_t* __restrict__ rcap,
                                                           const uint32_t* __restrict__ X,
                                                           uint32_t* __restrict__ out) {
    __shared__ uint32_t sc[kBlock / 64][64], sb[kBlock / 64][64];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint64_t nw = (uint64_t)gridDim.x * (kBlock / 64);
    for (uint64_t w = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; w * 64 < V; w += nw) {
        const uint64_t v0 = w * 64;
        const uint32_t rows = V - v0 < 64 ? (uint32_t)(V - v0) : 64u;
        uint32_t c = kNone, b = 0;
        if (lane < rows) {
            const uint32_t u = perm ? perm[v0 + lane] : (uint32_t)(v0 + lane);
            if (cid_of) c = cid_of[u];
            if (c == kNone) b = rcap[u];
        }
        sc[wave][lane] = c;
        sb[wave][lane] = b;
        wave_lds_sync();
        const uint32_t n = rows * L, n4 = n >> 2;
        uint32_t* __restrict__ o = out + v0 * L;
        for (uint32_t q = lane; q < n4; q += 64) {
            uint32_t row = __umulhi(q * 4, magic);
            uint32_t col = q * 4 - row * L;
            uint32_t val[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                if (col >= L) {
                    col -= L;
                    ++row;
                }
                const uint32_t cr = sc[wave][row];
                val[t] = cr == kNone ? sb[wave][row] : X[(uint64_t)cr * S + col];
                ++col;
            }
            stream_store(make_uint4(val[0], val[1], val[2], val[3]), reinterpret_cast<uint4*>(o) + q);
        }
        for (uint32_t e = n4 * 4 + lane; e < n; e += 64) {  // a last partial wave's n % 4 values
            const uint32_t row = __umulhi(e, magic), col = e - row * L;
            const uint32_t cr = sc[wave][row];
            __builtin_nontemporal_store(cr == kNone ? sb[wave][row] : X[(uint64_t)cr * S + col], &o[e]);
        }
        wave_lds_sync();
    }
}

// values[v * L + i] (L % 32 == 0, 128-byte aligned rows back to back) of a
// graph that numbers its vertices itself: a wave takes 64 consecutive
// internal ids, reads their caller ids, compact ids and R_cap values with
// coalesced loads, and writes each row at its caller id with lane-contiguous
// 16-byte streaming stores (a row is whole 128-byte lines, so the scattered
// rows write no partial line).
__global__ void __launch_bounds__(kBlock) k_writeback_scatter(uint32_t V, uint32_t L, uint32_t S,
                                                              const uint32_t* __restrict__ iperm,
                                                              const uint32_t* __restrict__ cid_of,
                                                              const uint32_t* __restrict__ rcap,
                                                              const uint32_t* __restrict__ X,
                                                              uint32_t* __restrict__ out) {
    __shared__ uint32_t sc[kBlock / 64][64], sb[kBlock / 64][64], so[kBlock / 64][64];
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    const uint32_t Lq = L >> 2, Sq = S >> 2;
    const uint64_t nw = (uint64_t)gridDim.x * (kBlock / 64);
    uint4* __restrict__ o4 = reinterpret_cast<uint4*>(out);
    const uint4* __restrict__ x4 = reinterpret_cast<const uint4*>(X);
    for (uint64_t w = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6; w * 64 < V; w += nw) {
        const uint64_t v0 = w * 64;
        const uint32_t rows = V - v0 < 64 ? (uint32_t)(V - v0) : 64u;
        uint32_t c = kNone, b = 0, o = 0;
        if (lane < rows) {
            o = iperm[v0 + lane];
            if (cid_of) c = cid_of[v0 + lane];
            if (c == kNone) b = rcap[v0 + lane];
        }
        sc[wave][lane] = c;
        sb[wave][lane] = b;
        so[wave][lane] = o;
        wave_lds_sync();
        const uint32_t n4 = rows * Lq;
        for (uint32_t q = lane; q < n4; q += 64) {
            const uint32_t row = q / Lq, j = q - row * Lq;
            const uint32_t cr = sc[wave][row], br = sb[wave][row];
            const uint4 val = cr == kNone ? make_uint4(br, br, br, br) : x4[(uint64_t)cr * Sq + j];
            stream_store(val, &o4[(uint64_t)so[wave][row] * Lq + j]);
        }
        wave_lds_sync();
    }
}

// values[v * L + i], one value per lane (any L).
__global__ void __launch_bounds__(kBlock) k_writeback1(uint32_t V, uint32_t L, uint32_t S, uint32_t OS,
                                                       const uint32_t* __restrict__ perm,
                                                       const uint32_t* __restrict__ cid_of,
                                                       const uint32_t* __restrict__ rcap,
                                                       const uint32_t* __restrict__ X, uint32_t* __restrict__ out) {
    const uint64_t n = (uint64_t)V * L;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t v = k / L;
        const uint32_t i = (uint32_t)(k - v * L);
        const uint32_t u = perm ? perm[v] : (uint32_t)v;
        const uint32_t c = cid_of ? cid_of[u] : kNone;
        __builtin_nontemporal_store(c == kNone ? rcap[u] : X[(uint64_t)c * S + i], &out[v * OS + i]);
    }
}

// dst[i] = src[i], i < n (4 values per thread where aligned).
__global__ void k_copy4(const uint32_t* __restrict__ src, uint32_t* __restrict__ dst, uint32_t n) {
    const uint64_t n4 = n / 4;
    const bool al = ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 16 == 0);
    const uint64_t i0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x, st = (uint64_t)gridDim.x * blockDim.x;
    if (al) {
        for (uint64_t i = i0; i < n4; i += st)
            reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
        for (uint64_t i = n4 * 4 + i0; i < n; i += st) dst[i] = src[i];
    } else {
        for (uint64_t i = i0; i < n; i += st) dst[i] = src[i];
    }
}

// Rows of a compact result into values[v * L + i]: four values per thread.
__global__ void k_scatter_rows4(const uint32_t* __restrict__ ulist, uint32_t nU, const uint32_t* __restrict__ X,
                                uint32_t LG, uint32_t L, uint32_t* __restrict__ out) {
    const uint32_t Lq = L / 4;
    const uint64_t n = (uint64_t)nU * Lq;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t c = k / Lq;
        const uint32_t j = (uint32_t)(k - c * Lq);
        reinterpret_cast<uint4*>(out)[(uint64_t)ulist[c] * Lq + j] =
            reinterpret_cast<const uint4*>(X)[c * (LG / 4) + j];
    }
}

__global__ void k_scatter_rows1(const uint32_t* __restrict__ ulist, uint32_t nU, const uint32_t* __restrict__ X,
                                uint32_t LG, uint32_t L, uint32_t* __restrict__ out) {
    const uint64_t n = (uint64_t)nU * L;
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t c = k / L;
        const uint32_t i = (uint32_t)(k - c * L);
        out[(uint64_t)ulist[c] * L + i] = X[c * LG + i];
    }
}

// Column of one snapshot: col[v] = R_cap[v] for stable v, else its relaxed value.
__global__ void k_column(uint32_t V, const uint32_t* __restrict__ perm, const uint32_t* __restrict__ cid_of,
                         const uint32_t* __restrict__ rcap, const uint32_t* __restrict__ X,
                         uint32_t* __restrict__ col) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < V; v += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t u = perm ? perm[v] : (uint32_t)v;
        const uint32_t c = cid_of ? cid_of[u] : kNone;
        col[v] = c == kNone ? rcap[u] : X[c];
    }
}

// out[v] = in[perm[v]]: an array over internal ids in the caller's order.
__global__ void k_to_caller_order(const uint32_t* __restrict__ in, const uint32_t* __restrict__ perm, uint32_t V,
                                  uint32_t* __restrict__ out) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < V; v += (uint64_t)gridDim.x * blockDim.x)
        out[v] = in[perm[v]];
}

// out[i] = iperm[in[i]]: internal vertex ids as the caller's.
__global__ void k_to_caller_ids(const uint32_t* __restrict__ in, const uint32_t* __restrict__ iperm, uint32_t n,
                                uint32_t* __restrict__ out) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        out[i] = iperm[in[i]];
}

// T[i][v] (L columns of V values) -> out[v * L + i], through a 64 x 64 LDS tile.
__global__ void __launch_bounds__(256) k_columns_to_rows(const uint32_t* __restrict__ T, uint32_t L, uint32_t V,
                                                         uint32_t* __restrict__ out) {
    __shared__ uint32_t tile[64][65];
    const uint32_t tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const uint64_t vt = (V + 63) / 64, it = (L + 63) / 64;
    for (uint64_t t = blockIdx.x; t < vt * it; t += gridDim.x) {
        const uint64_t v0 = (t % vt) * 64, i0 = (t / vt) * 64;
#pragma unroll 4
        for (uint32_t k = ty; k < 64; k += 4) {  // rows i0 + k of T, columns v0 + tx
            const uint64_t i = i0 + k, v = v0 + tx;
            tile[k][tx] = (i < L && v < V) ? T[i * V + v] : 0u;
        }
        __syncthreads();
#pragma unroll 4
        for (uint32_t k = ty; k < 64; k += 4) {  // out rows v0 + k, columns i0 + tx
            const uint64_t v = v0 + k, i = i0 + tx;
            if (v < V && i < L) out[v * L + i] = tile[tx][k];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host side

}  // namespace

uint32_t pick_lg(uint32_t L) {
    if (L <= 8) return 8;
    if (L <= 16) return 16;
    if (L <= 32) return 32;
    if (L <= 64) return 64;
    return 128;
}

namespace {

struct Timer {
    bool on;
    hipStream_t s;
    std::vector<hipEvent_t> ev;
    Timer(bool o, hipStream_t st) : on(o), s(st) {}
    void mark() {
        if (!on) return;
        hipEvent_t e;
        EVQ_HIP(hipEventCreate(&e));
        EVQ_HIP(hipEventRecord(e, s));
        ev.push_back(e);
    }
    double ms(size_t a, size_t b) {
        if (!on || b >= ev.size()) return 0.0;
        float m = 0.f;
        EVQ_HIP(hipEventSynchronize(ev[b]));
        EVQ_HIP(hipEventElapsedTime(&m, ev[a], ev[b]));
        return m;
    }
    ~Timer() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

struct Reduced {
    uint32_t nU = 0, nR = 0;
    uint64_t TU = 0;
    uint32_t* cid_of = nullptr;
    uint8_t* ubits = nullptr;  // bit v: v is in U
    uint32_t* ulist = nullptr;
    uint32_t* cuo = nullptr;
    uint32_t* rv = nullptr;   // U rows: vertex, compact id, start in the record buffer
    uint32_t* rc = nullptr;
    uint32_t* ruo = nullptr;
    uint32_t* kc = nullptr;
    void* recs = nullptr;
    bool split = false;  // |U| exceeded the caller's threshold: no subgraph was built
};

void reduce_edges(const Graph& g, Reduced& r, const Window& W, uint32_t NLW, Workspace& ws, hipStream_t s);

// Builds U's compact ids and the reduced subgraph.  all_vertices: U = V.
// One host read-back (|U|, rows, edges) sizes the subgraph buffer.
Reduced reduce_graph(const Graph& g, const uint32_t* rcap, const uint32_t* rcup, bool all_vertices, const Window& W,
                     uint32_t NLW, const Frontier& f, Workspace& ws, Mailbox& mb, hipStream_t s,
                     uint32_t split_above = 0xFFFFFFFFu) {
    Reduced r;
    const uint32_t V = g.V;
    r.cid_of = ws.buf<uint32_t>(Workspace::kCidOf, V);
    r.ubits = ws.buf<uint8_t>(Workspace::kUbits, (uint64_t)V / 8 + 8);
    r.ulist = ws.buf<uint32_t>(Workspace::kUlist, V);
    r.cuo = ws.buf<uint32_t>(Workspace::kCuo, V);
    uint32_t* rv = r.rv = ws.buf<uint32_t>(Workspace::kRv, V);
    uint32_t* rc = r.rc = ws.buf<uint32_t>(Workspace::kRc, V);
    uint32_t* ruo = r.ruo = ws.buf<uint32_t>(Workspace::kRuo, V);
    UCounters* uc = reinterpret_cast<UCounters*>(f.aux);
    fill_u32(reinterpret_cast<uint32_t*>(uc), sizeof(UCounters) / 4, 0u, s);
    EVQ_LAUNCH("compact_unstable", k_unstable, grid_for(V, kUPerBlock, 65535), kUBlock, s,
               all_vertices ? nullptr : rcap, rcup, V, g.row_ptr, r.cid_of, r.ulist, r.cuo, rv, rc, ruo, r.ubits, uc);
    EVQ_HIP(hipMemcpyAsync(mb.h, uc, sizeof(UCounters), hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipStreamSynchronize(s));
    const unsigned long long* hc = reinterpret_cast<const unsigned long long*>(mb.h);
    r.nU = (uint32_t)hc[0];
    r.nR = (uint32_t)(hc[1] >> 32);
    r.TU = (uint32_t)hc[1];
    if (r.nU == 0) return r;
    if (r.nU > split_above) {
        r.split = true;
        return r;
    }
    reduce_edges(g, r, W, NLW, ws, s);
    return r;
}

// The reduced subgraph's records for window W over the unstable set of r
// (rebuilt in place: kc and the records).
void reduce_edges(const Graph& g, Reduced& r, const Window& W, uint32_t NLW, Workspace& ws, hipStream_t s) {
    r.kc = ws.buf<uint32_t>(Workspace::kKc, r.nU);
    fill_u32(r.kc, r.nU, 0u, s);
    r.recs = ws.raw(Workspace::kRecs, (r.TU + 1) * (NLW == 1 ? sizeof(Rec<1>) : sizeof(Rec<2>)));
    if (r.TU) {
        ReduceArgs a;
        a.row_ptr = g.row_ptr;
        a.row_split = g.row_split;
        a.col = g.col;
        a.wgt = g.wgt;
        a.mask = g.mask;
        a.rv = r.rv;
        a.rc = r.rc;
        a.ruo = r.ruo;
        a.cid_of = r.cid_of;
        a.kc = r.kc;
        a.recs = r.recs;
        a.nR = r.nR;
        a.TU = (uint32_t)r.TU;
        a.b = W.b;
        a.L = W.L;
        a.K = g.K;
        const uint32_t blocks = grid_for((r.TU + 63) / 64, kBlock / 64, 2048);
        if (g.MW == 1) EVQ_LAUNCH("compact_reduce", (k_reduce<1, 1>), blocks, kBlock, s, a);
        else if (NLW == 1) EVQ_LAUNCH("compact_reduce", (k_reduce<2, 1>), blocks, kBlock, s, a);
        else EVQ_LAUNCH("compact_reduce", (k_reduce<2, 2>), blocks, kBlock, s, a);
    }
}

uint64_t sum_u32(const uint32_t* d, uint32_t n, hipStream_t s) {
    std::vector<uint32_t> h(n);
    EVQ_HIP(hipMemcpyAsync(h.data(), d, (uint64_t)n * 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipStreamSynchronize(s));
    uint64_t t = 0;
    for (uint32_t x : h) t += x;
    return t;
}

template <int A, int LG, bool ST>
void relax_phase(const Graph& g, const Window& W, const Window& PW, const uint32_t* rcap, const Reduced& red,
                 uint32_t* X, bool plain, uint32_t source, Frontier& f, Workspace& ws, hipStream_t s, QueryOut& qo) {
    using T = Lanes<LG>;
    RelaxArgs ra;
    ra.cuo = red.cuo;
    ra.kc = red.kc;
    ra.recs = red.recs;
    ra.X = X;
    ra.flags = f.flags;
    ra.fo = f.fo;  // V entries each, free once the bound solves are done (nU <= V)
    ra.fv = f.fv;
    ra.tasks = ws.buf<uint64_t>(Workspace::kTasks, (uint64_t)red.nU + red.TU / kRelaxChunk + 64);
    ra.cnt = f.cnt;
    ra.stats = f.stats;
    ra.nU = red.nU;
    if (plain) {
        EVQ_LAUNCH("relax_xinit", k_xinit_plain<LG>, grid_for((uint64_t)red.nU * LG, 256 * 4), 256, s, red.ulist,
                   red.nU, source, Alg<A>::unreached, Alg<A>::at_source, X);
        EVQ_LAUNCH("relax_seed", k_mark_source, 1, 64, s, f.flags, red.cid_of, source);
    } else {
        EVQ_LAUNCH("relax_xinit", k_xinit<LG>, grid_for((uint64_t)red.nU * (LG % 4 == 0 ? LG / 4 : LG), 256 * 4), 256,
                   s, red.ulist, red.nU,
                   rcap, X);
        if (g.n_partial) {
            const uint32_t waves = (uint32_t)((g.n_partial + 63) / 64);
#define EVQ_SEED(MW_)                                                                                             \
    EVQ_LAUNCH("relax_seed", (k_relax_seed<A, MW_, LG, ST>), grid_for(waves, kBlock / 64, 8192), kBlock, s, ra,   \
               g.p_src, g.p_dst, g.p_w, g.p_mask, (uint32_t)g.n_partial, red.cid_of, red.ubits, rcap, W.b, W.L, g.K, \
               PW.b, PW.L)
            if (g.MW == 1) EVQ_SEED(1);
            else EVQ_SEED(2);
#undef EVQ_SEED
        }
    }
    const uint32_t cblocks = grid_for(red.nU, kCompactIds, 4096);
    const bool direct = red.TU / kRelaxChunk + red.nU <= direct_tasks_limit();
    const uint32_t tblocks = grid_for(((uint64_t)red.nU + red.TU / kRelaxChunk + 63) / 64, kBlock / 64, 2048);
    const uint32_t rblocks =
        grid_for(((uint64_t)red.nU + red.TU / kRelaxChunk + T::G - 1) / T::G, kBlock / 64, EVQ_RELAX_BLOCKS);
    // the block stages its tasks in LDS, 2 or 4 per lane group (evq_tuning.relax_staged); the one-lane
    // layout of the sequential ablation keeps the per-group kernel
    const uint32_t staged = LG >= 8 ? tuning().relax_staged : 0u;
    const uint32_t sblocks = grid_for((uint64_t)red.nU + red.TU / kRelaxChunk,
                                      (kBlock / 64) * T::G * (staged ? staged : 1), EVQ_RELAX_BLOCKS);
    auto issue = [&](uint64_t, int p, bool first, uint32_t* slot) {
        if (direct) {
            EVQ_LAUNCH("relax_compact", k_relax_compact<true>, cblocks, kCompactBlock, s, ra, p, first ? 1 : 0);
        } else {
            EVQ_LAUNCH("relax_compact", k_relax_compact<false>, cblocks, kCompactBlock, s, ra, p, first ? 1 : 0);
            EVQ_LAUNCH("relax_tasks", k_relax_tasks, tblocks, kBlock, s, ra, p);
        }
        if (staged == 2)
            EVQ_LAUNCH("relax", (k_relax_staged<A, (LG >= 8 ? LG : 8), 2, ST>), sblocks, kBlock, s, ra, ra.tasks,
                       ra.cuo, ra.kc, ra.recs, p, slot);
        else if (staged == 4)
            EVQ_LAUNCH("relax", (k_relax_staged<A, (LG >= 8 ? LG : 8), 4, ST>), sblocks, kBlock, s, ra, ra.tasks,
                       ra.cuo, ra.kc, ra.recs, p, slot);
        else
            EVQ_LAUNCH("relax", (k_relax<A, LG, ST>), rblocks, kBlock, s, ra, ra.tasks, ra.cuo, ra.kc, ra.recs, p, slot);
    };
    qo.st.iters_relax = drive_loop(issue, f.p, s, (uint64_t)g.V + 2, "snapshot relaxation");
}

template <int A>
void relax_dispatch(uint32_t LG, bool st, const Graph& g, const Window& W, const Window& PW, const uint32_t* rcap,
                    const Reduced& red, uint32_t* X, bool plain, uint32_t source, Frontier& f, Workspace& ws,
                    hipStream_t s, QueryOut& qo) {
#define EVQ_RX(LG_)                                                                               \
    case LG_:                                                                                     \
        if (st) relax_phase<A, LG_, true>(g, W, PW, rcap, red, X, plain, source, f, ws, s, qo);  \
        else relax_phase<A, LG_, false>(g, W, PW, rcap, red, X, plain, source, f, ws, s, qo);    \
        break;
    switch (LG) {
        EVQ_RX(1)
        EVQ_RX(8)
        EVQ_RX(16)
        EVQ_RX(32)
        EVQ_RX(64)
        EVQ_RX(128)
    }
#undef EVQ_RX
}

// PW: the window whose bounds rcap belongs to (seeding edges are partial in
// it); W: the snapshots relaxed (W == PW, or one snapshot of PW).
void relax_algo(uint32_t algo, uint32_t LG, bool st, const Graph& g, const Window& W, const Window& PW,
                const uint32_t* rcap, const Reduced& red, uint32_t* X, bool plain, uint32_t source, Frontier& f,
                Workspace& ws, hipStream_t s, QueryOut& qo) {
    switch (algo) {
    case EVQ_SSSP: relax_dispatch<EVQ_SSSP>(LG, st, g, W, PW, rcap, red, X, plain, source, f, ws, s, qo); break;
    case EVQ_BFS: relax_dispatch<EVQ_BFS>(LG, st, g, W, PW, rcap, red, X, plain, source, f, ws, s, qo); break;
    case EVQ_SSWP: relax_dispatch<EVQ_SSWP>(LG, st, g, W, PW, rcap, red, X, plain, source, f, ws, s, qo); break;
    case EVQ_SSNP: relax_dispatch<EVQ_SSNP>(LG, st, g, W, PW, rcap, red, X, plain, source, f, ws, s, qo); break;
    default: relax_dispatch<EVQ_VITERBI>(LG, st, g, W, PW, rcap, red, X, plain, source, f, ws, s, qo); break;
    }
}

// values[v * OS + i], i < L (OS: the output's row stride, >= L).
// Row v of out (the caller's id) is internal vertex perm[v] (perm null: v;
// iperm, the inverse, given with it).
void writeback(uint32_t LG, uint32_t V, uint32_t L, const uint32_t* perm, const uint32_t* iperm, const uint32_t* cid_of,
               const uint32_t* rcap, const uint32_t* X, uint32_t* out, hipStream_t s, uint32_t OS = 0) {
    if (OS == 0) OS = L;
    // rows of whole 128-byte lines are scattered to their caller ids; other
    // lengths keep the output contiguous and gather the rows' inputs
    if (perm && OS == L && L % 32 == 0 && L <= 256 && (uintptr_t)out % 128 == 0 && (X == nullptr || LG % 4 == 0)) {
        EVQ_LAUNCH("writeback", k_writeback_scatter, grid_for(V, kBlock, 65535), kBlock, s, V, L, LG, iperm, cid_of,
                   rcap, X, out);
        return;
    }
    if (OS == L && L >= 4 && L <= 256 && (uintptr_t)out % 16 == 0) {
        const uint32_t magic = (uint32_t)((1ull << 32) / L + 1);
        EVQ_LAUNCH("writeback", k_writeback_flat, grid_for(V, kBlock, 65535), kBlock, s, V, L, LG, magic, perm,
                   cid_of, rcap, X, out);
        return;
    }
    const bool vec = (L % 4 == 0) && (L <= 256) && (OS % 4 == 0) && ((uintptr_t)out % 16 == 0) &&
                     (X == nullptr || LG % 4 == 0);
    if (vec) {
        EVQ_LAUNCH("writeback", k_writeback4, grid_for(V, kBlock, 65535), kBlock, s, V, L, LG, OS, perm, cid_of,
                   rcap, X, out);
    } else {
        EVQ_LAUNCH("writeback", k_writeback1, grid_for((uint64_t)V * L, kBlock * 4, 65535), kBlock, s, V, L, LG, OS,
                   perm, cid_of, rcap, X, out);
    }
}

}  // namespace

uint32_t choose_delta(uint32_t algo) { return tuning().delta[algo <= EVQ_VITERBI ? algo : 0]; }

uint32_t choose_heavy(uint32_t algo) { return tuning().heavy[algo <= EVQ_VITERBI ? algo : 0]; }

namespace {

uint64_t read_stat(const unsigned long long* d, int i, hipStream_t s) {
    unsigned long long h = 0;
    EVQ_HIP(hipMemcpyAsync(&h, d + i, sizeof(h), hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipStreamSynchronize(s));
    return h;
}

}  // namespace

namespace {

// Step 1: both bounds (the union solve starts from the intersection values).
void bounds_impl(const Graph& g, uint32_t algo, uint32_t source, const Window& W, uint32_t* rcap, uint32_t* rcup,
                 Frontier& f, QueryOut& qo, hipStream_t s, Timer& tm) {
    const bool st = qo.want_stats;
    qo.st.iters_cap = solve_cap(g, algo, W, source, rcap, f, s, st);
    tm.mark();
    EVQ_LAUNCH("copy_bound", k_copy4, grid_for((g.V + 3) / 4, 256 * 4, 8192), 256, s, rcap, rcup, g.V);
    if (st) {
        qo.st.edges_cap = read_stat(f.stats, 0, s);
        qo.st.updates_cap = read_stat(f.stats, 4, s);
    }
    qo.st.items_cap = f.items;
    qo.st.iters_cup = solve_cup(g, algo, W, rcup, f, s, st);
    tm.mark();
    qo.st.items_cup = f.items - qo.st.items_cap;
    if (st) {
        qo.st.edges_cup = read_stat(f.stats, 0, s) - qo.st.edges_cap;
        qo.st.updates_cup = read_stat(f.stats, 4, s) - qo.st.updates_cap;
        qo.st.seed_visits_cup = read_stat(f.stats, 5, s);
    }
}

// Steps 2-3 and Algorithm 2: reduction, then the multi-snapshot relaxation
// into X (the workspace, or a compact result's rows), then the writeback of
// values[V][L] when d_values is given.
bool tail_impl(const Graph& g, uint32_t algo, uint32_t source, const Window& W, const uint32_t* rcap,
               const uint32_t* rcup, Frontier& f, Workspace& ws, uint32_t* d_values, Compact* c, QueryOut& qo,
               hipStream_t s, Timer& tm, uint32_t OS = 0, uint32_t split_above = 0xFFFFFFFFu) {
    const bool st = qo.want_stats;
    Mailbox& mb = Mailbox::get();
    const uint32_t LG = pick_lg(W.L);
    const uint32_t NLW = LG > 64 ? 2 : 1;
    Reduced red = reduce_graph(g, rcap, rcup, false, W, NLW, f, ws, mb, s, split_above);
    if (red.split) return false;
    tm.mark();
    uint32_t* X = nullptr;
    if (c) {
        c->nU = red.nU;
        c->LG = LG;
        c->ulist = c->X = nullptr;
        if (red.nU) {
            const uint64_t ub = ((uint64_t)red.nU * 4 + 255) & ~uint64_t(255);
            char* p = static_cast<char*>(stream_alloc(ub + (uint64_t)red.nU * LG * 4, s));
            c->ulist = reinterpret_cast<uint32_t*>(p);
            c->X = reinterpret_cast<uint32_t*>(p + ub);
            if (g.iperm)
                EVQ_LAUNCH("result_ids", k_to_caller_ids, grid_for(red.nU, 256 * 4, 8192), 256, s, red.ulist,
                           g.iperm, red.nU, c->ulist);
            else
                EVQ_LAUNCH("result_copy", k_copy4, grid_for((red.nU + 3) / 4, 256 * 4, 8192), 256, s, red.ulist,
                           c->ulist, red.nU);
            X = c->X;
        }
    } else if (red.nU) {
        X = ws.buf<uint32_t>(Workspace::kX, (uint64_t)red.nU * LG);
    }
    if (red.nU) relax_algo(algo, LG, st, g, W, W, rcap, red, X, false, source, f, ws, s, qo);
    tm.mark();
    if (d_values) writeback(LG, g.V, W.L, g.perm, g.iperm, red.cid_of, rcap, X, d_values, s, OS);
    if (c && g.perm) {  // the compact result's bound in the caller's order (its ids are mapped above)
        uint32_t* t = ws.buf<uint32_t>(Workspace::kOrder, g.V);
        EVQ_LAUNCH("result_order", k_copy4, grid_for((g.V + 3) / 4, 256 * 4, 8192), 256, s, c->rcap, t, g.V);
        EVQ_LAUNCH("result_order", k_to_caller_order, grid_for(g.V, 256 * 4, 8192), 256, s, t, g.perm, g.V,
                   c->rcap);
    }
    tm.mark();
    qo.st.n_unstable += red.nU;
    qo.st.subwindows += 1;
    if (st) {
        qo.st.n_relax_edges += red.nU ? sum_u32(red.kc, red.nU, s) : 0;
        // cumulative over the sub-windows of a split query
        qo.st.edge_visits_relax = read_stat(f.stats, 1, s);
        qo.st.lane_relaxations = read_stat(f.stats, 2, s);
        qo.st.n_seed_edges = read_stat(f.stats, 3, s);
    }
    return true;
}

// Sub-window splitting (off unless EVQ_SPLIT_FRAC > 0): a window whose
// unstable set holds more than EVQ_SPLIT_FRAC of the vertices is answered as
// two halves of at least EVQ_SPLIT_MIN snapshots each (default 8), each with
// its own bound solves (the intersection grows and the union shrinks as the
// window narrows, so fewer vertices stay unstable), to depth 4.  Under churn
// spread evenly over the window the halves stay about as unstable and the
// extra bound solves cost more than they save, hence off by default.
struct SplitRule {
    double frac = 0.0;
    uint32_t min_len = 8;
    static SplitRule get() {
        const evq_tuning t = tuning();
        SplitRule r;
        r.frac = t.split_frac;
        r.min_len = t.split_min < 1 ? 1 : t.split_min;
        return r;
    }
};

Window sub_window(const Graph& g, const Window& W, uint32_t off, uint32_t len) {
    Window S;
    S.b = (W.b + off) % g.K;
    S.L = len;
    S.K = g.K;
    for (uint32_t i = 0; i < len; ++i) {
        const uint32_t t = (S.b + i) % g.K;
        S.w[t >> 6] |= 1ull << (t & 63);
    }
    S.full = len == g.K;
    return S;
}

// The tail of window W (whose bounds are in rcap / rcup) into out, row stride OS.
void answer(const Graph& g, uint32_t algo, uint32_t source, const Window& W, uint32_t* rcap, uint32_t* rcup,
            Frontier& f, Workspace& ws, uint32_t* out, uint32_t OS, QueryOut& qo, hipStream_t s, Timer& tm,
            uint32_t depth, const SplitRule& sr) {
    const bool can = sr.frac > 0.0 && W.L >= 2 * sr.min_len && depth < 4;
    const uint32_t above = can ? (uint32_t)(sr.frac * (double)g.V) : 0xFFFFFFFFu;
    if (tail_impl(g, algo, source, W, rcap, rcup, f, ws, out, nullptr, qo, s, tm, OS, above)) return;
    const uint32_t L1 = W.L / 2;
    for (int h = 0; h < 2; ++h) {
        const uint32_t off = h ? L1 : 0, len = h ? W.L - L1 : L1;
        const Window S = sub_window(g, W, off, len);
        QueryOut qs;
        qs.want_stats = false;
        Timer quiet(false, s);
        bounds_impl(g, algo, source, S, rcap, rcup, f, qs, s, quiet);
        answer(g, algo, source, S, rcap, rcup, f, ws, out + off, OS, qo, s, quiet, depth + 1, sr);
    }
}

}  // namespace

void run_query(const Graph& g, uint32_t algo, uint32_t source, const Window& W, uint32_t* d_values,
               uint32_t* d_rcap_out, uint32_t* d_rcup_out, bool bounds_only, QueryOut& qo, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    if (!noalloc_ctx()) init_mempool(g.device);
    Workspace& ws = Workspace::get(s);
    const bool st = qo.want_stats;
    Timer tm(st, s);
    tm.mark();
    Frontier f = make_frontier(g, ws, s);
    f.delta = choose_delta(algo);
    f.heavy = choose_heavy(algo);
    f.bdelta = choose_bucket_width(algo, g);
    // the bounds go straight to the caller's arrays unless the graph numbers its vertices itself
    uint32_t* rcap = d_rcap_out && !g.perm ? d_rcap_out : ws.buf<uint32_t>(Workspace::kRcap, g.V);
    uint32_t* rcup = d_rcup_out && !g.perm ? d_rcup_out : ws.buf<uint32_t>(Workspace::kRcup, g.V);
    bounds_impl(g, algo, source, W, rcap, rcup, f, qo, s, tm);
    if (bounds_only) {
        if (g.perm && d_rcap_out)
            EVQ_LAUNCH("bounds_order", k_to_caller_order, grid_for(g.V, 256 * 4, 8192), 256, s, rcap, g.perm, g.V,
                       d_rcap_out);
        if (g.perm && d_rcup_out)
            EVQ_LAUNCH("bounds_order", k_to_caller_order, grid_for(g.V, 256 * 4, 8192), 256, s, rcup, g.perm, g.V,
                       d_rcup_out);
        EVQ_HIP(hipStreamSynchronize(s));
        ws.in_use = false;
        return;
    }
    answer(g, algo, source, W, rcap, rcup, f, ws, d_values, W.L, qo, s, tm, 0,
           noalloc_ctx() ? SplitRule{} : SplitRule::get());
    ws.in_use = false;
    if (st) {
        qo.st.ms_cap = tm.ms(0, 1);
        qo.st.ms_cup = tm.ms(1, 2);
        qo.st.ms_compact = tm.ms(2, 3);
        qo.st.ms_relax = tm.ms(3, 4);
        qo.st.ms_writeback = tm.ms(4, 5);
        EVQ_HIP(hipStreamSynchronize(s));
        qo.st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
}

void run_query_compact(const Graph& g, uint32_t algo, uint32_t source, const Window& W, Compact& c, QueryOut& qo,
                       hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    if (!noalloc_ctx()) init_mempool(g.device);
    Workspace& ws = Workspace::get(s);
    const bool st = qo.want_stats;
    Timer tm(st, s);
    tm.mark();
    Frontier f = make_frontier(g, ws, s);
    f.delta = choose_delta(algo);
    f.heavy = choose_heavy(algo);
    f.bdelta = choose_bucket_width(algo, g);
    uint32_t* rcup = ws.buf<uint32_t>(Workspace::kRcup, g.V);
    bounds_impl(g, algo, source, W, c.rcap, rcup, f, qo, s, tm);
    qo.bounds_done = std::chrono::steady_clock::now();
    tail_impl(g, algo, source, W, c.rcap, rcup, f, ws, nullptr, &c, qo, s, tm);
    ws.in_use = false;
    if (st) {
        qo.st.ms_cap = tm.ms(0, 1);
        qo.st.ms_cup = tm.ms(1, 2);
        qo.st.ms_compact = tm.ms(2, 3);
        qo.st.ms_relax = tm.ms(3, 4);
        EVQ_HIP(hipStreamSynchronize(s));
        qo.st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
}

void run_tail_compact(const Graph& g, uint32_t algo, uint32_t source, const Window& W, const uint32_t* rcup,
                      Compact& c, QueryOut& qo, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    if (!noalloc_ctx()) init_mempool(g.device);
    Workspace& ws = Workspace::get(s);
    const bool st = qo.want_stats;
    Timer tm(st, s);
    tm.mark();
    Frontier f = make_frontier(g, ws, s);
    tail_impl(g, algo, source, W, c.rcap, rcup, f, ws, nullptr, &c, qo, s, tm);
    ws.in_use = false;
    if (st) {
        qo.st.ms_compact = tm.ms(0, 1);
        qo.st.ms_relax = tm.ms(1, 2);
        EVQ_HIP(hipStreamSynchronize(s));
        qo.st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
}

void expand_compact(uint32_t V, uint32_t L, const uint32_t* rcap, const uint32_t* ulist, const uint32_t* X,
                    uint32_t nU, uint32_t LG, uint32_t* d_values, hipStream_t s) {
    writeback(LG, V, L, nullptr, nullptr, nullptr, rcap, nullptr, d_values, s);
    if (!nU) return;
    if (L % 4 == 0 && (uintptr_t)d_values % 16 == 0) {
        EVQ_LAUNCH("expand_rows", k_scatter_rows4, grid_for((uint64_t)nU * (L / 4), 256 * 4, 65535), 256, s, ulist,
                   nU, X, LG, L, d_values);
    } else {
        EVQ_LAUNCH("expand_rows", k_scatter_rows1, grid_for((uint64_t)nU * L, 256 * 4, 65535), 256, s, ulist, nU, X,
                   LG, L, d_values);
    }
}

// Ablation: the snapshots of the window one after another on the window's
// reduced subgraph (Algorithm 1's per-snapshot evaluation), each as a
// one-lane relaxation (one edge per lane), instead of all of them at once.
void run_sequential(const Graph& g, uint32_t algo, uint32_t source, const Window& W, uint32_t* d_values,
                    QueryOut& qo, hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    init_mempool(g.device);
    Workspace& ws = Workspace::get(s);
    Mailbox& mb = Mailbox::get();
    const bool st = qo.want_stats;
    Timer tm(st, s);
    tm.mark();
    Frontier f = make_frontier(g, ws, s);
    f.delta = choose_delta(algo);
    f.heavy = choose_heavy(algo);
    f.bdelta = choose_bucket_width(algo, g);
    uint32_t* rcap = ws.buf<uint32_t>(Workspace::kRcap, g.V);
    uint32_t* rcup = ws.buf<uint32_t>(Workspace::kRcup, g.V);
    bounds_impl(g, algo, source, W, rcap, rcup, f, qo, s, tm);
    uint32_t* T = ws.buf<uint32_t>(Workspace::kBatchCap, (uint64_t)W.L * g.V);
    Reduced red;
    uint64_t iters = 0, visits = 0, lanes = 0, seeds = 0;
    for (uint32_t i = 0; i < W.L; ++i) {
        Window Wi;
        Wi.b = (W.b + i) % g.K;
        Wi.L = 1;
        Wi.K = g.K;
        Wi.w[Wi.b >> 6] = 1ull << (Wi.b & 63);
        Wi.full = g.K == 1;
        if (i == 0) red = reduce_graph(g, rcap, rcup, false, Wi, 1, f, ws, mb, s);
        else if (red.nU) reduce_edges(g, red, Wi, 1, ws, s);
        uint32_t* X = nullptr;
        if (red.nU) {
            X = ws.buf<uint32_t>(Workspace::kX, red.nU);
            relax_algo(algo, 1, st, g, Wi, W, rcap, red, X, false, source, f, ws, s, qo);
            iters += qo.st.iters_relax;
            if (st) {
                visits += read_stat(f.stats, 1, s);
                lanes += read_stat(f.stats, 2, s);
                seeds += read_stat(f.stats, 3, s);
                EVQ_LAUNCH("query_init", k_init_frontier_stats, 1, 64, s, f.stats);
            }
        }
        EVQ_LAUNCH("writeback", k_column, grid_for(g.V, 256 * 4, 65535), 256, s, g.V, g.perm,
                   red.nU ? red.cid_of : nullptr, rcap, X, T + (uint64_t)i * g.V);
    }
    tm.mark();
    const uint64_t tiles = ((g.V + 63) / 64) * (((uint64_t)W.L + 63) / 64);
    EVQ_LAUNCH("writeback", k_columns_to_rows, grid_for(tiles, 1, 65535), 256, s, T, W.L, g.V, d_values);
    tm.mark();
    ws.in_use = false;
    qo.st.iters_relax = iters;
    if (st) {
        qo.st.ms_cap = tm.ms(0, 1);
        qo.st.ms_cup = tm.ms(1, 2);
        qo.st.ms_relax = tm.ms(2, 3);
        qo.st.ms_writeback = tm.ms(3, 4);
        qo.st.n_unstable = red.nU;
        qo.st.edge_visits_relax = visits;
        qo.st.lane_relaxations = lanes;
        qo.st.n_seed_edges = seeds;
        EVQ_HIP(hipStreamSynchronize(s));
        qo.st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
}

void run_plain(const Graph& g, uint32_t algo, uint32_t source, const Window& W, uint32_t* d_values, QueryOut& qo,
               hipStream_t s) {
    auto t0 = std::chrono::steady_clock::now();
    init_mempool(g.device);
    Workspace& ws = Workspace::get(s);
    Mailbox& mb = Mailbox::get();
    const bool st = qo.want_stats;
    Timer tm(st, s);
    tm.mark();
    Frontier f = make_frontier(g, ws, s);
    const uint32_t LG = pick_lg(W.L);
    const uint32_t NLW = LG > 64 ? 2 : 1;
    Reduced red = reduce_graph(g, nullptr, nullptr, true, W, NLW, f, ws, mb, s);
    tm.mark();
    uint32_t* X = ws.buf<uint32_t>(Workspace::kX, (uint64_t)g.V * LG);
    relax_algo(algo, LG, st, g, W, W, nullptr, red, X, true, source, f, ws, s, qo);
    tm.mark();
    writeback(LG, g.V, W.L, g.perm, g.iperm, red.cid_of, nullptr, X, d_values, s);
    tm.mark();
    ws.in_use = false;
    if (st) {
        qo.st.ms_compact = tm.ms(0, 1);
        qo.st.ms_relax = tm.ms(1, 2);
        qo.st.ms_writeback = tm.ms(2, 3);
        qo.st.n_unstable = red.nU;
        qo.st.n_relax_edges = red.nU ? sum_u32(red.kc, red.nU, s) : 0;
        qo.st.edge_visits_relax = read_stat(f.stats, 1, s);
        qo.st.lane_relaxations = read_stat(f.stats, 2, s);
        EVQ_HIP(hipStreamSynchronize(s));
        qo.st.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
}

}  // namespace evq
