// Frontier plumbing shared by the bound solver and the multi-snapshot relaxer.
//
// An iteration's improvements only set a byte flag per vertex of the next
// frontier (an idempotent plain store), so no vertex is listed twice and no
// counter is hit per improvement.  A compaction kernel turns the flags into
// the next work list in vertex order, clearing the flags it reads, with one
// packed 64-bit counter reservation per block (items in the high word, edges
// in the low word) so that the list and the running edge offsets stay in the
// same order.
//
// Counters are double-buffered by iteration parity p: the compaction of
// iteration i zeroes the item counter of parity p ^ 1 (the previous
// iteration's, whose readers have finished) and adds into parity p, whose
// deferral counters the expansion before it has reset; the expansion of
// iteration i reads cnt[p],
// tells the next compaction whether it produced work, and publishes its item
// count to a host-mapped slot, so the host never has to synchronise the
// stream to learn when a loop has drained.  A compaction that finds the
// previous expansion empty returns at once, so iterations issued past the end
// cost one launch.  In a sparse iteration the bound solves' expansion may
// instead append its improved vertices to the next work list itself (into
// cnt[p ^ 1], zeroed by the compaction before it); the next compaction then
// skips its scan.
#pragma once

#include "evq_internal.h"

namespace evq {

struct FrontierCounters {
    unsigned long long packed[2];  // (items << 32) | edges, by parity
    uint32_t far[2];               // ids left flagged (for a later threshold or bucket), by parity
    uint32_t fmin[2];              // smallest order key among the ids left for a later threshold, by parity
    uint32_t thr;                  // near/far threshold of the bound solves (order keys below it are near)
    uint32_t delta;                // threshold step (0: every id is near)
    uint32_t heavy;                // with delta > 0: only ids with at least this many edges are gated (0: all)
    uint32_t kall[2];              // smallest order key over the compacted ids with edges, by parity (heavy > 0)
    uint32_t status[2];            // for the compaction of parity q: bit 0 the expansion before it had work
                                   // or deferred ids, bit 1 it appended the next list itself
    // Bucketed schedule with light and heavy edges (bound solves of SSSP):
    uint32_t bdelta;               // bucket width (0: off)
    uint32_t bthr[2];              // the bucket's upper key bound set by the compaction of parity q
    uint32_t near[2];              // the expansion of parity q improved a vertex below bthr[q]
    uint32_t nmin[2];              // smallest value it wrote at or above bthr[q]
};
static_assert(sizeof(FrontierCounters) <= 128, "frontier counters share a 128-byte control slot");

__device__ __forceinline__ uint32_t items_of(unsigned long long x) { return (uint32_t)(x >> 32); }
__device__ __forceinline__ uint32_t edges_of(unsigned long long x) { return (uint32_t)x; }

// Next-frontier membership is one byte per id: marking is an idempotent plain
// byte store, so an improvement costs no second atomic.
__device__ __forceinline__ void mark(uint8_t* __restrict__ flags, uint32_t v) { flags[v] = 1; }

// Bytes of the flag array for n ids (a multiple of the 8 ids a lane reads).
inline uint64_t flag_bytes(uint64_t n) { return (n + 7) & ~uint64_t(7); }

// Expansion prologue: read this iteration's counts, tell the next compaction
// whether there was work and whether this expansion appends the next list
// itself (`appends`, the same on every block), publish the item count to the
// host slot.
// When nothing was near but ids were deferred, the threshold moves to the
// smallest deferred order key plus delta, so the next compaction releases the
// best of them.  When only heavy ids are gated, the threshold also follows the
// frontier: it rises to the smallest key of this iteration's ids plus delta,
// so a heavy id is expanded once its value is within delta of the best one
// still moving (and, with positive steps, close to final).
__device__ __forceinline__ unsigned long long expand_prologue(FrontierCounters* c, int p, uint32_t* slot,
                                                              bool appends = false) {
    const unsigned long long x = c->packed[p];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint32_t f = c->far[p];
        uint64_t t = c->thr;
        if (items_of(x) == 0 && f) t = (uint64_t)c->fmin[p] + c->delta;
        if (c->heavy && c->kall[p] != 0xFFFFFFFFu) {
            const uint64_t u = (uint64_t)c->kall[p] + c->delta;
            t = u > t ? u : t;
        }
        c->thr = t > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)t;
        c->status[p ^ 1] = (x != 0ull || f ? 1u : 0u) | (appends ? 2u : 0u);
        // the other parity's deferral counters, last read by the compaction
        // before this expansion, start afresh for the next compaction
        c->far[p ^ 1] = 0u;
        c->fmin[p ^ 1] = 0xFFFFFFFFu;
        c->kall[p ^ 1] = 0xFFFFFFFFu;
        __hip_atomic_store(slot, items_of(x) + f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    return x;
}

// Compaction prologue: zero the other parity's item counters (the previous
// iteration's, read only by kernels that have finished) for the next
// iteration, clear this parity's bucket reports for the expansion that
// follows, and say whether the scan can be skipped: the previous expansion
// had no work and deferred nothing (no flag can be set), or it appended the
// next list itself.  The first compaction of a loop always scans.
__device__ __forceinline__ bool compaction_skips(FrontierCounters* c, int p, int first) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->packed[p ^ 1] = 0ull;
        c->near[p] = 0u;
        c->nmin[p] = 0xFFFFFFFFu;
    }
    return !first && c->status[p] != 1u;
}

// Largest i in [0, n) with off[i] <= x (off ascending, off[0] == 0), found by
// the whole wave with a 64-ary search.  Every lane must call it.
__device__ __forceinline__ uint32_t wave_search(const uint32_t* __restrict__ off, uint32_t n, uint32_t x) {
    uint32_t lo = 0, hi = n;  // answer in [lo, hi)
    const uint32_t lane = lane_id();
    while (hi - lo > 64) {
        const uint32_t step = (hi - lo + 63) / 64;
        const uint32_t idx = lo + lane * step;
        const bool ok = idx < hi && off[idx] <= x;
        const uint64_t b = __ballot(ok);
        const uint32_t last = 63u - (uint32_t)__clzll((unsigned long long)b);  // lane 0 is always ok
        const uint32_t nlo = lo + last * step;
        const uint32_t nhi = nlo + step < hi ? nlo + step : hi;
        lo = nlo;
        hi = nhi;
    }
    const uint32_t idx = lo + lane;
    const bool ok = idx < hi && off[idx] <= x;
    const uint64_t b = __ballot(ok);
    return lo + 63u - (uint32_t)__clzll((unsigned long long)b);
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Flag compaction shared by the frontier loops.  A block of kCompactBlock
// threads takes kCompactIds consecutive ids (8 flag bytes per lane), stages
// the flagged ids and their flag bytes in LDS, reads every id's work size with
// all loads in flight at once, rewrites the flag bytes, and reserves (items,
// edges) for the whole block with one packed atomic.
// size_of(id, flag, items, edges, key, aux) gives an id's work (items and
// edges, zero for none), may keep two words of what it read in aux for emit,
// and returns the flag byte the id keeps: 0 clears it; an id left flagged is
// counted in *far and, unless size_of leaves key at 0xFFFFFFFF, its order key
// enters the minimum *fmin.  emit(id, item, edge, items, edges, aux) writes an
// id's work.  Ids appear in ascending order within a block.  With kall
// non-null, size_of gives every id with edges its order key and the smallest
// of them enters the minimum *kall.  post() runs on every thread of the block
// after each group of ids has been emitted (and the block synchronised),
// before the next group is compacted.
struct NoPost {
    __device__ void operator()() const {}
};
constexpr int kCompactBlock = 512;
constexpr int kCompactWaves = kCompactBlock / 64;
constexpr int kIdsPerWave = 512;
constexpr int kCompactIds = kCompactWaves * kIdsPerWave;
constexpr int kIdSteps = kIdsPerWave / 64;

template <typename SizeFn, typename EmitFn, typename PostFn = NoPost>
__device__ __forceinline__ void compact_flags(uint8_t* __restrict__ flags, uint32_t n, unsigned long long* cnt,
                                              uint32_t* far, uint32_t* fmin, SizeFn size_of, EmitFn emit,
                                              uint32_t* kall = nullptr, PostFn post = PostFn()) {
    __shared__ uint32_t ids[kCompactWaves][kIdsPerWave];
    __shared__ uint8_t fbyte[kCompactWaves][kIdsPerWave];  // flag byte of each listed id
    __shared__ uint2 nflag[kCompactWaves][64];             // the wave's new flag bytes, in id order
    __shared__ uint32_t wtot[kCompactWaves][5];
    __shared__ unsigned long long bbase;
    const uint32_t lane = lane_id(), wave = threadIdx.x >> 6;
    uint2* __restrict__ f8 = reinterpret_cast<uint2*>(flags);
    uint8_t* const nf8 = reinterpret_cast<uint8_t*>(nflag[wave]);
    for (uint64_t b0 = (uint64_t)blockIdx.x * kCompactIds; b0 < n; b0 += (uint64_t)gridDim.x * kCompactIds) {
        const uint32_t w0 = (uint32_t)b0 + wave * kIdsPerWave;  // first id of this wave
        const uint32_t g0 = w0 + lane * 8;                       // first id of this lane
        uint2 fl = make_uint2(0u, 0u);
        if (g0 < n) fl = f8[g0 >> 3];
        uint32_t word = 0;  // bit k: id g0 + k is flagged
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            word |= ((fl.x >> (8 * k)) & 0xFFu) ? (1u << k) : 0u;
            word |= ((fl.y >> (8 * k)) & 0xFFu) ? (1u << (k + 4)) : 0u;
        }
        const uint32_t pc = (uint32_t)__popc(word);
        const uint32_t incl = wave_incl_scan(pc);
        const uint32_t tot = lane_value(incl, 63);
        uint32_t id[kIdSteps], ni[kIdSteps], ne[kIdSteps], pi[kIdSteps], pe[kIdSteps];
        uint2 aux[kIdSteps];
#pragma unroll
        for (int s = 0; s < kIdSteps; ++s) {
            id[s] = ni[s] = ne[s] = pi[s] = pe[s] = 0;
            aux[s] = make_uint2(0u, 0u);
        }
        uint32_t ti = 0, te = 0, tf = 0, tk = 0xFFFFFFFFu, ta = 0xFFFFFFFFu;
        if (tot) {
            nflag[wave][lane] = make_uint2(0u, 0u);
            uint32_t k = incl - pc;
            for (uint32_t m = word; m; m &= m - 1) {
                const uint32_t b = (uint32_t)__builtin_ctz(m);
                ids[wave][k] = g0 + b;
                fbyte[wave][k] = (uint8_t)(((b < 4 ? fl.x : fl.y) >> (8 * (b & 3))) & 0xFFu);
                ++k;
            }
            wave_lds_sync();
            uint32_t nf = 0, kmin = 0xFFFFFFFFu, amin = 0xFFFFFFFFu;
            // the steps past the wave's count (tot, wave-uniform) are skipped
#pragma unroll
            for (int s = 0; s < kIdSteps; ++s) {
                if (s * 64u >= tot) break;
                const uint32_t j = s * 64 + lane;
                if (j < tot) {
                    id[s] = ids[wave][j];
                    uint32_t key = 0xFFFFFFFFu;
                    const uint32_t kept = size_of(id[s], (uint32_t)fbyte[wave][j], ni[s], ne[s], key, aux[s]);
                    amin = key < amin ? key : amin;
                    if (kept) {  // its flag stays set
                        ++nf;
                        kmin = key < kmin ? key : kmin;
                        nf8[id[s] - w0] = (uint8_t)kept;
                    }
                }
            }
#pragma unroll
            for (int s = 0; s < kIdSteps; ++s) {
                if (s * 64u >= tot) break;
                const uint32_t a = wave_incl_scan(ni[s]), b = wave_incl_scan(ne[s]);
                pi[s] = ti + a - ni[s];
                pe[s] = te + b - ne[s];
                ti += lane_value(a, 63);
                te += lane_value(b, 63);
            }
            tf = wave_sum(nf);
            tk = wave_min(kmin);
            if (kall) ta = wave_min(amin);
            wave_lds_sync();
            if (word) f8[g0 >> 3] = nflag[wave][lane];
        }
        if (lane == 0) {
            wtot[wave][0] = ti;
            wtot[wave][1] = te;
            wtot[wave][2] = tf;
            wtot[wave][3] = tk;
            wtot[wave][4] = ta;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long sum = 0;
            uint32_t fsum = 0, kmin = 0xFFFFFFFFu, amin = 0xFFFFFFFFu;
            for (int w = 0; w < kCompactWaves; ++w) {
                sum += ((unsigned long long)wtot[w][0] << 32) | wtot[w][1];
                fsum += wtot[w][2];
                kmin = wtot[w][3] < kmin ? wtot[w][3] : kmin;
                amin = wtot[w][4] < amin ? wtot[w][4] : amin;
            }
            bbase = sum ? atomicAdd(cnt, sum) : 0ull;
            if (fsum) {
                atomicAdd(far, fsum);
                atomicMin(fmin, kmin);
            }
            // a plain read first: most blocks hold no new minimum and skip the atomic
            if (kall && amin < __hip_atomic_load(kall, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(kall, amin);
        }
        __syncthreads();
        if (ti) {
            uint32_t bi = (uint32_t)(bbase >> 32), be = (uint32_t)bbase;
            for (uint32_t w = 0; w < wave; ++w) {
                bi += wtot[w][0];
                be += wtot[w][1];
            }
#pragma unroll
            for (int s = 0; s < kIdSteps; ++s)
                if (ni[s]) emit(id[s], bi + pi[s], be + pe[s], ni[s], ne[s], aux[s]);
        }
        __syncthreads();
        post();
    }
}

// Task lists of a compaction whose ids expand to several tasks each (task q
// of id c is the 64-bit word (q << 32) | c).  An id with one task has it
// written by the lane that holds it; an id with more is listed in LDS, and
// after each group of ids (post() of compact_flags) the whole block writes the
// listed tasks, each thread finding the id of its task by a binary search over
// the list's running task counts, so a hub's 10^5 tasks and many small ids
// are written at the same rate.  A full list falls back to the holding lane.
constexpr uint32_t kTaskListCap = 2048;
struct TaskList {
    uint32_t n;
    uint32_t id[kTaskListCap], first[kTaskListCap], cnt[kTaskListCap], pre[kTaskListCap];
    uint32_t wsum[kCompactWaves];
};

__device__ __forceinline__ void task_list_init(TaskList& tl) {
    if (threadIdx.x == 0) tl.n = 0;
    __syncthreads();
}

__device__ __forceinline__ void task_list_add(TaskList& tl, uint64_t* __restrict__ tasks, uint32_t c, uint32_t first,
                                              uint32_t items) {
    uint32_t k = kTaskListCap;
    if (items > 1) k = atomicAdd(&tl.n, 1u);
    if (k < kTaskListCap) {
        tl.id[k] = c;
        tl.first[k] = first;
        tl.cnt[k] = items;
    } else {
        for (uint32_t q = 0; q < items; ++q) tasks[first + q] = ((uint64_t)q << 32) | c;
    }
}

// Every thread of the block (kCompactBlock of them) calls it.
__device__ __forceinline__ void task_list_flush(TaskList& tl, uint64_t* __restrict__ tasks) {
    constexpr uint32_t kPer = kTaskListCap / kCompactBlock;
    const uint32_t nb = tl.n < kTaskListCap ? tl.n : kTaskListCap;
    if (nb) {
        const uint32_t lane = lane_id(), wave = threadIdx.x >> 6, k0 = threadIdx.x * kPer;
        uint32_t s = 0;
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j) s += k0 + j < nb ? tl.cnt[k0 + j] : 0u;
        const uint32_t incl = wave_incl_scan(s);
        if (lane == 63) tl.wsum[wave] = incl;
        __syncthreads();
        uint32_t off = incl - s, tot = 0;
        for (uint32_t w = 0; w < kCompactWaves; ++w) {
            off += w < wave ? tl.wsum[w] : 0u;
            tot += tl.wsum[w];
        }
#pragma unroll
        for (uint32_t j = 0; j < kPer; ++j)
            if (k0 + j < nb) {
                tl.pre[k0 + j] = off;
                off += tl.cnt[k0 + j];
            }
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < tot; t += kCompactBlock) {
            uint32_t lo = 0, hi = nb;  // largest k with pre[k] <= t
            while (hi - lo > 1) {
                const uint32_t mid = (lo + hi) >> 1;
                if (tl.pre[mid] <= t) lo = mid;
                else hi = mid;
            }
            const uint32_t q = t - tl.pre[lo];
            tasks[tl.first[lo] + q] = ((uint64_t)q << 32) | tl.id[lo];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) tl.n = 0;
}

// Host side: launch-ahead driver of a frontier loop.
class HostSlots {
  public:
    static constexpr uint32_t kSlots = 256;
    static constexpr uint32_t kEmpty = 0xFFFFFFFFu;
    static HostSlots& get();  // one per host thread
    uint32_t* host() const { return h_; }
    uint32_t* dev() const { return d_; }
    // Slot numbering runs on across loops, so that the iterations a finished
    // loop issued past its end (still queued) never write a slot that the
    // next loop has just reset.
    uint64_t next = 0;

  private:
    HostSlots();
    uint32_t* h_ = nullptr;
    uint32_t* d_ = nullptr;
};

// Issues iterations (issue(it, parity, first)) `depth` ahead of the one whose
// published count it waits for; stops at the first iteration with count 0.
// Returns the number of non-empty iterations and adds the published counts
// (items processed) to *items; f_parity is advanced past every issued
// iteration.
template <typename IssueFn>
uint64_t drive_loop(IssueFn issue, int& f_parity, hipStream_t s, uint64_t max_iters, const char* what,
                    uint64_t* items = nullptr);

void wait_slot(volatile uint32_t* slot, hipStream_t s, const char* what);

// Iterations kept in flight by drive_loop: EVQ_LAUNCH_DEPTH (1..32), default 3.
uint64_t launch_depth();
// EVQ_TRACE_LOOPS=1: drive_loop prints each iteration's published count to stderr.
bool trace_loops();

// Inside a no-allocation call: the published counts go to the first words of
// the scratch array; each batch of launch_depth() + 1 iterations is followed
// by one copy of its counts to host memory and a stream synchronisation.
template <typename IssueFn>
uint64_t drive_loop_sync(IssueFn issue, int& f_parity, hipStream_t s, uint64_t max_iters, const char* what,
                         uint64_t* items, NoAlloc& na) {
    static_assert(kNoAllocSlotBytes >= 33 * 4, "slots of one batch");
    uint32_t* dslots = reinterpret_cast<uint32_t*>(na.base);
    const uint64_t batch = launch_depth() + 1;
    uint32_t h[33];
    uint64_t issued = 0, consumed = 0;
    for (;;) {
        for (uint64_t j = 0; j < batch; ++j, ++issued) {
            issue(issued, f_parity, issued == 0, dslots + j);
            f_parity ^= 1;
        }
        EVQ_HIP(hipMemcpyAsync(h, dslots, batch * 4, hipMemcpyDeviceToHost, s));
        EVQ_HIP(hipStreamSynchronize(s));
        for (uint64_t j = 0; j < batch; ++j) {
            if (trace_loops()) fprintf(stderr, "[evq] %s iteration %llu: %u\n", what, (unsigned long long)consumed, h[j]);
            if (h[j] == 0) return consumed;
            if (items) *items += h[j];
            if (++consumed > max_iters) fail(EVQ_ENOCONV, std::string(what) + " exceeded its iteration cap");
        }
    }
}

template <typename IssueFn>
uint64_t drive_loop(IssueFn issue, int& f_parity, hipStream_t s, uint64_t max_iters, const char* what,
                    uint64_t* items) {
    if (NoAlloc* na = noalloc_ctx()) return drive_loop_sync(issue, f_parity, s, max_iters, what, items, *na);
    const uint64_t kDepth = launch_depth();
    HostSlots& hs = HostSlots::get();
    uint64_t issued = 0, consumed = 0;
    const uint64_t base = hs.next;
    struct Advance {
        HostSlots& hs;
        const uint64_t& end;
        ~Advance() { hs.next = end; }
    };
    uint64_t end = base;
    Advance adv{hs, end};
    for (;;) {
        while (issued < consumed + kDepth) {
            const uint32_t k = (uint32_t)((base + issued) % HostSlots::kSlots);
            __atomic_store_n(&hs.host()[k], HostSlots::kEmpty, __ATOMIC_RELEASE);
            issue(issued, f_parity, issued == 0, hs.dev() + k);
            f_parity ^= 1;
            ++issued;
            end = base + issued;
        }
        volatile uint32_t* slot = hs.host() + ((base + consumed) % HostSlots::kSlots);
        wait_slot(slot, s, what);
        if (trace_loops()) fprintf(stderr, "[evq] %s iteration %llu: %u\n", what, (unsigned long long)consumed, *slot);
        if (*slot == 0) break;
        if (items) *items += *slot;
        if (++consumed > max_iters) fail(EVQ_ENOCONV, std::string(what) + " exceeded its iteration cap");
    }
    return consumed;
}

}  // namespace evq
