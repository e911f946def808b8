// Frontier plumbing shared by the bound solver and the multi-snapshot relaxer.
//
// An iteration's improvements only set bits in a bitmap of the next frontier
// (fire-and-forget atomicOr, after a plain read shows the bit clear), so no
// vertex is listed twice and no counter is hit per improvement.  A compaction
// kernel turns the bitmap into the next work list in vertex order, clearing
// the bits it reads, with one packed 64-bit counter reservation per wave
// (items in the high word, edges in the low word) so that the list and the
// running edge offsets stay in the same order.
//
// Counters are double-buffered by iteration parity p: the compaction of
// iteration i adds into cnt[p]; the expansion of iteration i reads cnt[p],
// zeroes cnt[p ^ 1] for the next compaction and publishes its item count to a
// host-mapped slot, so the host never has to synchronise the stream to learn
// when a loop has drained.  A compaction that finds the previous expansion
// empty returns at once, so iterations issued past the end cost one launch.
#pragma once

#include "evq_internal.h"

namespace evq {

struct FrontierCounters {
    unsigned long long packed[2];  // (items << 32) | edges, by parity
};

__device__ __forceinline__ uint32_t items_of(unsigned long long x) { return (uint32_t)(x >> 32); }
__device__ __forceinline__ uint32_t edges_of(unsigned long long x) { return (uint32_t)x; }

__device__ __forceinline__ void mark(uint32_t* __restrict__ bitmap, uint32_t v) {
    uint32_t* w = bitmap + (v >> 5);
    const uint32_t bit = 1u << (v & 31);
    if (!(*w & bit)) __hip_atomic_fetch_or(w, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wave-wide reservation of (items, edges) on a packed counter: returns this
// lane's first item slot and first edge offset.  Every lane must call it.
__device__ __forceinline__ void wave_reserve2(uint32_t n, uint32_t ne, unsigned long long* cnt, uint32_t& item,
                                              uint32_t& edge) {
    const uint32_t in = wave_incl_scan(n), ie = wave_incl_scan(ne);
    const uint32_t tn = __shfl(in, 63, 64), te = __shfl(ie, 63, 64);
    unsigned long long base = 0;
    if (lane_id() == 63 && (tn | te)) base = atomicAdd(cnt, ((unsigned long long)tn << 32) | te);
    const uint32_t bi = (uint32_t)(__shfl((int)(base >> 32), 63, 64));
    const uint32_t be = (uint32_t)(__shfl((int)(uint32_t)base, 63, 64));
    item = bi + in - n;
    edge = be + ie - ne;
}

// Expansion prologue: read this iteration's counts, clear the other parity,
// publish the item count to the host slot.
__device__ __forceinline__ unsigned long long expand_prologue(FrontierCounters* c, int p, uint32_t* slot) {
    const unsigned long long x = c->packed[p];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->packed[p ^ 1] = 0ull;
        __hip_atomic_store(slot, items_of(x), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    return x;
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

// Host side: launch-ahead driver of a frontier loop.
class HostSlots {
  public:
    static constexpr uint32_t kSlots = 256;
    static constexpr uint32_t kEmpty = 0xFFFFFFFFu;
    static HostSlots& get();  // one per host thread
    uint32_t* host() const { return h_; }
    uint32_t* dev() const { return d_; }

  private:
    HostSlots();
    uint32_t* h_ = nullptr;
    uint32_t* d_ = nullptr;
};

// Issues iterations (issue(it, parity, first)) `depth` ahead of the one whose
// published count it waits for; stops at the first iteration with count 0.
// Returns the number of non-empty iterations; f_parity is advanced past every
// issued iteration.
template <typename IssueFn>
uint64_t drive_loop(IssueFn issue, int& f_parity, hipStream_t s, uint64_t max_iters, const char* what);

void wait_slot(volatile uint32_t* slot, hipStream_t s, const char* what);

template <typename IssueFn>
uint64_t drive_loop(IssueFn issue, int& f_parity, hipStream_t s, uint64_t max_iters, const char* what) {
    constexpr uint64_t kDepth = 3;
    HostSlots& hs = HostSlots::get();
    uint64_t issued = 0, consumed = 0;
    for (;;) {
        while (issued < consumed + kDepth) {
            const uint32_t k = (uint32_t)(issued % HostSlots::kSlots);
            __atomic_store_n(&hs.host()[k], HostSlots::kEmpty, __ATOMIC_RELEASE);
            issue(issued, f_parity, issued == 0, hs.dev() + k);
            f_parity ^= 1;
            ++issued;
        }
        volatile uint32_t* slot = hs.host() + (consumed % HostSlots::kSlots);
        wait_slot(slot, s, what);
        if (*slot == 0) break;
        if (++consumed > max_iters) fail(EVQ_ENOCONV, std::string(what) + " exceeded its iteration cap");
    }
    return consumed;
}

}  // namespace evq
