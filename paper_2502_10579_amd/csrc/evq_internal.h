// Internal declarations shared by the library's HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "evq.h"

namespace evq {

// ------------------------------------------------------------------ errors

struct Error {
    evq_status code;
    std::string msg;
};

[[noreturn]] void fail(evq_status code, const std::string& msg);
extern thread_local std::string g_last_error;  // message of the last failing C ABI call on this thread
void hip_check(hipError_t e, const char* what);

#define EVQ_HIP(expr) ::evq::hip_check((expr), #expr)

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr uint32_t kSat = 0xFFFFFFFEu;

// ------------------------------------------------------------------ graph

// A graph's rows with each all-present prefix reordered for a bucket width:
// the edges heavier than the width first (nheavy of them), the lighter ones
// after; the other edges keep their places (so masks still index them).
struct WeightOrder {
    uint32_t width = 0;
    uint32_t* col = nullptr;     // E
    uint32_t* w = nullptr;       // E
    uint32_t* nheavy = nullptr;  // V
    hipEvent_t ready = nullptr;  // recorded after the copy was written
};
constexpr uint32_t kWeightOrders = 4;  // widths kept per graph version

// Snapshot t (a global id, counted from the first snapshot ever built) is
// held in mask bit (t mod K); the graph holds snapshots first .. first+K-1.
struct Graph {
    uint32_t V = 0, K = 0, MW = 1;
    uint64_t first = 0;             // global id of the oldest snapshot held
    uint32_t maxw = 1;              // largest weight ever seen (key layout of appends)
    uint64_t E = 0, n_partial = 0;
    uint32_t* row_ptr = nullptr;    // V + 1
    uint32_t* row_split = nullptr;  // V: end of the edges present in all K snapshots
    uint32_t* col = nullptr;        // E
    uint32_t* wgt = nullptr;        // E
    uint64_t* mask = nullptr;       // E * MW, bit i of the 128/64-bit word group = snapshot i
    // Edges present in some but not all K snapshots, in edge-id order, as a
    // table of their own so that the passes over them stream it:
    uint32_t* p_src = nullptr;      // n_partial: source
    uint32_t* p_dst = nullptr;      // n_partial: destination
    uint32_t* p_w = nullptr;        // n_partial: weight
    uint64_t* p_mask = nullptr;     // n_partial * MW: presence mask
    // Vertex numbering: every array above is indexed by internal ids, the
    // vertices ranked by descending degree when the graph was first built
    // (the values of the hubs then share cache lines); null: the caller's ids.
    uint32_t* perm = nullptr;   // V: caller id -> internal id
    uint32_t* iperm = nullptr;  // V: internal id -> caller id
    std::shared_ptr<const std::vector<uint32_t>> perm_h;  // host copy of perm, shared by later versions
    int device = 0;
    uint64_t bytes = 0;
    double build_ms = 0.0;
    // The caller's allocator (evq_build): every array of every version, the
    // reverse CSR and the temporaries of builds and appends come from it.
    evq_allocator ua{};
    bool has_ua = false;
    // Events recorded on the streams of calls that read this version; its
    // arrays are released (stream-ordered, after all of them) when it retires.
    mutable std::mutex use_mu;
    mutable std::vector<hipEvent_t> uses;
    // Reverse CSR of the edges present in all K snapshots, grouped by
    // destination (the pull step of the full-window intersection solve).  It
    // is built by the second query that asks for it (a ring version that
    // lives for one query or none never pays for it); later users on other
    // streams wait for rv_ready.
    mutable std::mutex rv_mu;
    mutable uint32_t rv_asks = 0;
    mutable bool rv_built = false;
    mutable hipEvent_t rv_ready = nullptr;
    mutable uint32_t* rv_src = nullptr;  // source of each in-edge (capacity E), grouped by destination
    mutable uint32_t* rv_w = nullptr;    // its weight (capacity E)
    mutable uint32_t* rv_dst = nullptr;  // its destination (capacity E), ascending
    mutable uint32_t* rv_cnt = nullptr;  // [1] in-edges (device)
    // Weight-ordered copies of the rows for the bucketed SSSP intersection
    // solve, one per width in use, built by the first query that asks.
    mutable std::mutex wo_mu;
    mutable WeightOrder wo[kWeightOrders];
    mutable uint32_t n_wo = 0;
};

// Internal id of the caller's vertex v.
inline uint32_t internal_id(const Graph& g, uint32_t v) { return g.perm_h ? (*g.perm_h)[v] : v; }

// Records that work reading g was queued on s (call after the last launch).
void note_use(const Graph& g, hipStream_t s);
struct UseGuard {
    const Graph& g;
    hipStream_t s;
    ~UseGuard() {
        try {
            note_use(g, s);
        } catch (...) {
        }
    }
};

// ------------------------------------------------------------------ memory

// Per-call device temporaries, stream-ordered (hipMallocAsync / hipFreeAsync).
// With a caller's allocator, buffers come from it and are returned to it
// once the work queued on the stream has completed.
class Arena {
  public:
    explicit Arena(hipStream_t s, const evq_allocator* ua = nullptr) : s_(s), ua_(ua) {}
    ~Arena();
    Arena(const Arena&) = delete;
    Arena& operator=(const Arena&) = delete;
    template <typename T>
    T* alloc(uint64_t n) {
        return static_cast<T*>(raw(n * sizeof(T)));
    }
    void* raw(uint64_t bytes);
    void release(void* p);
    uint64_t bytes() const { return bytes_; }

  private:
    hipStream_t s_;
    const evq_allocator* ua_;
    std::vector<void*> ptrs_;
    uint64_t bytes_ = 0;
};

// Device memory of a graph version: from the graph's caller allocator when it
// has one (throws EVQ_ENOMEM when that returns NULL), else from the device's
// stream-ordered pool.  graph_free returns one such array.
void* graph_alloc(const Graph& g, uint64_t bytes, hipStream_t s);
void graph_free(const Graph& g, void* p, hipStream_t s);

// A call that must not allocate (evq_query_noalloc).  While it is set on a
// thread, the query path takes its device buffers from `base` by bump
// allocation (the first kNoAllocSlotBytes hold the frontier loops' published
// counts, which the host reads back with a copy), reads counters into plain
// host memory, launches untimed and never builds the pull step's reverse CSR.
struct NoAlloc {
    char* base = nullptr;
    uint64_t cap = 0, used = 0;
};
constexpr uint64_t kNoAllocSlotBytes = 256;
NoAlloc*& noalloc_ctx();  // thread-local; null outside such a call
// Device address of this device's scratch array (looked up once per device)
// and its size; throws EVQ_EDEVICE if the lookup fails.
char* noalloc_scratch(int device, uint64_t* bytes);

// Query workspace: device buffers kept between queries on one host thread
// and stream, grown on demand (growth waits for the stream).  Queries on one
// stream are ordered, so reuse is safe.  Inside a no-allocation call the
// thread's arena workspace is used instead (reset by arena()).
class Workspace {
  public:
    enum Slot {
        kFlags, kFo, kFd, kFs, kFv, kFo1, kFd1, kFs1, kFv1, kStamp, kControl, kRcap, kRcup, kCidOf, kUlist, kCuo,
        kRv, kRc, kRuo, kKc, kRecs, kTasks, kX, kBatchCap, kBatchCup, kBatchTable, kUbits, kOrder, kSlots
    };
    static Workspace& get(hipStream_t s);
    static Workspace& arena(hipStream_t s, NoAlloc& na);
    void* raw(Slot slot, uint64_t bytes);
    template <typename T>
    T* buf(Slot slot, uint64_t n) {
        return static_cast<T*>(raw(slot, n * sizeof(T)));
    }
    bool fresh_flags = true;  // flags must be cleared before use
    bool in_use = false;      // a query is running on it (a failed one leaves flags unknown)
    uint32_t epoch = 0;               // last epoch handed to an expansion (appending iterations)
    const void* stamp_seen = nullptr; // stamp buffer those epochs refer to (cleared when it changes)

  private:
    explicit Workspace(hipStream_t s) : s_(s) {}
    hipStream_t s_;
    NoAlloc* na_ = nullptr;
    void* p_[kSlots] = {};
    uint64_t cap_[kSlots] = {};
};

void* stream_alloc(uint64_t bytes, hipStream_t s);  // hipMallocAsync from the device pool; throws EVQ_ENOMEM
void stream_free(void* p, hipStream_t s);          // hipFreeAsync (NULL allowed)
void init_mempool(int device);

// Small pinned host mailbox used to read counters back (one per host thread;
// plain host memory inside a no-allocation call).
struct Mailbox {
    uint32_t* h = nullptr;
    bool pinned = true;
    explicit Mailbox(size_t n);
    explicit Mailbox(uint32_t* plain) : h(plain), pinned(false) {}
    ~Mailbox();
    static Mailbox& get();
};

// ------------------------------------------------------------------ tuning

// Scheduling knobs: read from the environment once per process, replaced by
// evq_tuning_set; each call takes a copy.
evq_tuning tuning();
void set_tuning(const evq_tuning& t);
constexpr uint32_t kAutoWidth = 0xFFFFFFFFu;  // evq_tuning::bucket_width: derived from the graph

// ------------------------------------------------------------------ launches

bool timing_on();
struct TimingScope {
    TimingScope(const char* name, hipStream_t s);
    ~TimingScope();
    const char* name;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
};
void post_launch(const char* name);

#define EVQ_LAUNCH(NAME, KERNEL, GRID, BLOCK, STREAM, ...)          \
    do {                                                            \
        ::evq::TimingScope _evq_ts((NAME), (STREAM));               \
        KERNEL<<<(GRID), (BLOCK), 0, (STREAM)>>>(__VA_ARGS__);      \
        ::evq::post_launch(NAME);                                   \
    } while (0)

inline uint32_t grid_for(uint64_t work, uint32_t per_block, uint32_t cap = 65536u) {
    uint64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

// ------------------------------------------------------------------ host entry points of each part

// Device-wide exclusive scan of n uint32 (in may equal out).  If d_total is
// non-null it receives the sum.  n < 2^32.
void scan_exclusive(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* d_total, hipStream_t s, Arena& ar);

void fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);

Graph* build_graph(uint32_t V, const evq_edge* base, uint64_t n_base, const evq_batch* batches, uint32_t K,
                   const evq_allocator* ua, hipStream_t s);
// The next version of a graph: snapshot first+K (old newest with batch b
// applied) replaces snapshot `first` in its mask bit.  `old` is not changed.
Graph* append_graph(const Graph& old, const evq_batch& b, hipStream_t s);
// Fills g's reverse CSR arrays (allocated by the caller: rv_src, rv_w and
// rv_dst with E entries, rv_cnt with 2) on s.
void build_reverse(const Graph& g, hipStream_t s);
// Releases g's device arrays, ordered on s, and deletes g.
void free_graph(Graph* g, hipStream_t s);
// A retired version: its arrays are released on a private stream once every
// recorded use has completed; no device-wide synchronisation.
void retire_graph(Graph* g);

// A window of L consecutive snapshots; lane i is snapshot (first of the
// window) + i, held in mask bit (b + i) mod K.
struct Window {
    uint32_t b = 0, L = 0, K = 0;
    uint64_t w[2] = {0, 0};  // the window's mask bits
    bool full = false;       // the window is all K snapshots
};

struct QueryOut {
    evq_query_stats st{};
    bool want_stats = false;
    std::chrono::steady_clock::time_point bounds_done{};  // host time the bound solves drained
};

void run_query(const Graph& g, uint32_t algo, uint32_t source, const Window& W, uint32_t* d_values,
               uint32_t* d_rcap_out, uint32_t* d_rcup_out, bool bounds_only, QueryOut& qo, hipStream_t s);
void run_plain(const Graph& g, uint32_t algo, uint32_t source, const Window& W, uint32_t* d_values, QueryOut& qo,
               hipStream_t s);
void run_sequential(const Graph& g, uint32_t algo, uint32_t source, const Window& W, uint32_t* d_values,
                    QueryOut& qo, hipStream_t s);

// Compact result of one query: rcap (V values, allocated by the caller) and,
// after the tail, the unstable vertices and their relaxed rows in one
// allocation (ulist first, rows of LG values from X).
struct Compact {
    uint32_t* rcap = nullptr;
    uint32_t* ulist = nullptr;
    uint32_t* X = nullptr;
    uint32_t nU = 0, LG = 0;
};

// Whole query with a compact result (bound solves into c.rcap).
void run_query_compact(const Graph& g, uint32_t algo, uint32_t source, const Window& W, Compact& c, QueryOut& qo,
                       hipStream_t s);
// Steps after the bound solves, given both bounds: reduction and relaxation
// into a compact result (c.rcap holds the intersection bound).
void run_tail_compact(const Graph& g, uint32_t algo, uint32_t source, const Window& W, const uint32_t* rcup,
                      Compact& c, QueryOut& qo, hipStream_t s);
// values[v * L + i] from a compact result.
void expand_compact(uint32_t V, uint32_t L, const uint32_t* rcap, const uint32_t* ulist, const uint32_t* X,
                    uint32_t nU, uint32_t LG, uint32_t* d_values, hipStream_t s);
uint32_t pick_lg(uint32_t L);

}  // namespace evq

// ------------------------------------------------------------------ device helpers

namespace evq {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t lanemask_lt() { return (1ull << lane_id()) - 1ull; }

template <typename T>
__device__ __forceinline__ T uniform(T x) {
    return (T)__builtin_amdgcn_readfirstlane((int)x);
}

// Wave-wide inclusive prefix sum (64 lanes) with DPP moves, no LDS permutes:
// row shifts by 1, 2, 4 and 8 sum within each row of 16 lanes (a lane whose
// source is outside its row adds 0), then lane 15 of rows 0 and 2 is added
// into rows 1 and 3, then lane 31 into rows 2 and 3.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_or_zero(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xF, false);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += dpp_or_zero<0x111, 0xF>(v);  // row_shr:1
    v += dpp_or_zero<0x112, 0xF>(v);  // row_shr:2
    v += dpp_or_zero<0x114, 0xF>(v);  // row_shr:4
    v += dpp_or_zero<0x118, 0xF>(v);  // row_shr:8
    v += dpp_or_zero<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
    v += dpp_or_zero<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
    return v;
}

// Lane l's value of v (l a constant or wave-uniform), read into a scalar register.
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// Wave-wide sum and minimum, wave-uniform results: the row shifts leave each
// row's total in its lane 15, and the four row totals are combined in scalar
// registers.
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    v += dpp_or_zero<0x111, 0xF>(v);
    v += dpp_or_zero<0x112, 0xF>(v);
    v += dpp_or_zero<0x114, 0xF>(v);
    v += dpp_or_zero<0x118, 0xF>(v);
    return lane_value(v, 15) + lane_value(v, 31) + lane_value(v, 47) + lane_value(v, 63);
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_or_max(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)0xFFFFFFFFu, (int)v, CTRL, 0xF, 0xF, false);
}

__device__ __forceinline__ uint32_t umin32(uint32_t a, uint32_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint32_t wave_min(uint32_t v) {
    v = umin32(v, dpp_or_max<0x111>(v));
    v = umin32(v, dpp_or_max<0x112>(v));
    v = umin32(v, dpp_or_max<0x114>(v));
    v = umin32(v, dpp_or_max<0x118>(v));
    return umin32(umin32(lane_value(v, 15), lane_value(v, 31)), umin32(lane_value(v, 47), lane_value(v, 63)));
}

// Query value algebra (Table 2).  `better(a, b)`: a strictly improves on b.
template <int A>
struct Alg;

template <>
struct Alg<EVQ_SSSP> {
    static constexpr uint32_t unreached = kInf, at_source = 0u;
    __device__ static __forceinline__ uint32_t extend(uint32_t x, uint32_t w) {
        if (x == kInf) return kInf;
        uint64_t s = (uint64_t)x + w;
        return s > kSat ? kSat : (uint32_t)s;
    }
    __device__ static __forceinline__ bool better(uint32_t a, uint32_t b) { return a < b; }
    __device__ static __forceinline__ uint32_t improve(uint32_t* p, uint32_t v) { return atomicMin(p, v); }
    __device__ static __forceinline__ void improve_nr(uint32_t* p, uint32_t v) {
        __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

template <>
struct Alg<EVQ_BFS> {
    static constexpr uint32_t unreached = kInf, at_source = 0u;
    __device__ static __forceinline__ uint32_t extend(uint32_t x, uint32_t) {
        return x == kInf ? kInf : (x >= kSat ? kSat : x + 1u);
    }
    __device__ static __forceinline__ bool better(uint32_t a, uint32_t b) { return a < b; }
    __device__ static __forceinline__ uint32_t improve(uint32_t* p, uint32_t v) { return atomicMin(p, v); }
    __device__ static __forceinline__ void improve_nr(uint32_t* p, uint32_t v) {
        __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

template <>
struct Alg<EVQ_SSWP> {
    static constexpr uint32_t unreached = 0u, at_source = kInf;
    __device__ static __forceinline__ uint32_t extend(uint32_t x, uint32_t w) { return x < w ? x : w; }
    __device__ static __forceinline__ bool better(uint32_t a, uint32_t b) { return a > b; }
    __device__ static __forceinline__ uint32_t improve(uint32_t* p, uint32_t v) { return atomicMax(p, v); }
    __device__ static __forceinline__ void improve_nr(uint32_t* p, uint32_t v) {
        __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

template <>
struct Alg<EVQ_SSNP> {
    static constexpr uint32_t unreached = kInf, at_source = 0u;
    __device__ static __forceinline__ uint32_t extend(uint32_t x, uint32_t w) {
        return x == kInf ? kInf : (x > w ? x : w);
    }
    __device__ static __forceinline__ bool better(uint32_t a, uint32_t b) { return a < b; }
    __device__ static __forceinline__ uint32_t improve(uint32_t* p, uint32_t v) { return atomicMin(p, v); }
    __device__ static __forceinline__ void improve_nr(uint32_t* p, uint32_t v) {
        __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

// Viterbi (Table 2: the best of Val(u) / w): IEEE single values held as
// their bit patterns (non-negative, so the integer order is the float
// order); a step divides in double precision and rounds to single, and a
// quotient below the smallest normal single is unreachable (0).
template <>
struct Alg<EVQ_VITERBI> {
    static constexpr uint32_t unreached = 0u, at_source = 0x3F800000u;  // 0.0f, 1.0f
    __device__ static __forceinline__ uint32_t extend(uint32_t x, uint32_t w) {
        if (x == 0u) return 0u;
        const double q = (double)__uint_as_float(x) / (double)w;
        if (q < 1.1754943508222875e-38) return 0u;  // FLT_MIN
        return __float_as_uint((float)q);
    }
    __device__ static __forceinline__ bool better(uint32_t a, uint32_t b) { return a > b; }
    __device__ static __forceinline__ uint32_t improve(uint32_t* p, uint32_t v) { return atomicMax(p, v); }
    __device__ static __forceinline__ void improve_nr(uint32_t* p, uint32_t v) {
        __hip_atomic_fetch_max(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

inline bool max_type(uint32_t algo) { return algo == EVQ_SSWP || algo == EVQ_VITERBI; }
inline uint32_t host_unreached(uint32_t algo) { return max_type(algo) ? 0u : kInf; }
inline uint32_t host_at_source(uint32_t algo) {
    return algo == EVQ_SSWP ? kInf : (algo == EVQ_VITERBI ? 0x3F800000u : 0u);
}

// Snapshot-mask helpers: MW 64-bit words per edge.
template <int MW>
struct Mask {
    uint64_t w[MW];
};

template <int MW>
__device__ __forceinline__ Mask<MW> load_mask(const uint64_t* m, uint64_t e) {
    Mask<MW> r;
#pragma unroll
    for (int j = 0; j < MW; ++j) r.w[j] = m[e * MW + j];
    return r;
}

// Bits [b, b+L) of a mask, moved down to bit 0 (L <= 64 -> one word, else two).
__device__ __forceinline__ uint64_t window_bits64(const uint64_t* w, int MW, uint32_t b) {
    // MW == 1: b < 64
    if (MW == 1) return w[0] >> b;
    if (b == 0) return w[0];
    if (b < 64) return (w[0] >> b) | (w[1] << (64 - b));
    return w[1] >> (b - 64);
}

}  // namespace evq
