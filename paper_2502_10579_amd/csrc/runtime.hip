// Host runtime pieces shared by every entry point: errors, device memory,
// pinned mailboxes, optional per-kernel timing, a fill kernel and a
// device-wide exclusive scan.
#include <algorithm>
#include <map>
#include <mutex>

#include <chrono>

#include "frontier.h"

namespace evq {

// ------------------------------------------------------------------ errors

[[noreturn]] void fail(evq_status code, const std::string& msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return;
    evq_status c = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? EVQ_ENOMEM : EVQ_EDEVICE;
    fail(c, std::string(what) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------------ memory

void note_use(const Graph& g, hipStream_t s) {
    hipEvent_t e = nullptr;
    EVQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipError_t r = hipEventRecord(e, s);
    if (r != hipSuccess) {
        (void)hipEventDestroy(e);
        hip_check(r, "hipEventRecord");
    }
    std::lock_guard<std::mutex> lk(g.use_mu);
    if (g.uses.size() >= 64) {  // drop the uses that have completed
        std::vector<hipEvent_t> keep;
        for (hipEvent_t x : g.uses) {
            if (hipEventQuery(x) == hipSuccess) (void)hipEventDestroy(x);
            else keep.push_back(x);
        }
        g.uses.swap(keep);
    }
    g.uses.push_back(e);
}

void retire_graph(Graph* g) {
    static std::mutex mu;
    static std::vector<std::pair<int, hipStream_t>> reapers;
    hipStream_t r = nullptr;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto& kv : reapers)
            if (kv.first == g->device) r = kv.second;
        if (!r) {
            int prev = 0;
            (void)hipGetDevice(&prev);
            (void)hipSetDevice(g->device);
            if (hipStreamCreateWithFlags(&r, hipStreamNonBlocking) != hipSuccess) r = nullptr;
            (void)hipSetDevice(prev);
            if (r) reapers.push_back({g->device, r});
        }
    }
    std::vector<hipEvent_t> uses;
    {
        std::lock_guard<std::mutex> lk(g->use_mu);
        uses.swap(g->uses);
    }
    if (g->has_ua) {  // the caller's allocator frees on the host: wait for every use first
        for (hipEvent_t e : uses) {
            (void)hipEventSynchronize(e);
            (void)hipEventDestroy(e);
        }
        try {
            free_graph(g, nullptr);
        } catch (...) {
        }
        return;
    }
    if (!r) {  // no stream for ordered release: wait for everything instead
        (void)hipDeviceSynchronize();
        for (hipEvent_t e : uses) (void)hipEventDestroy(e);
        try {
            free_graph(g, nullptr);
        } catch (...) {
        }
        return;
    }
    for (hipEvent_t e : uses) {
        (void)hipStreamWaitEvent(r, e, 0);
        (void)hipEventDestroy(e);
    }
    try {
        free_graph(g, r);
    } catch (...) {
    }
}

void* stream_alloc(uint64_t bytes, hipStream_t s) {
    void* p = nullptr;
    const uint64_t n = bytes ? (bytes + 255) & ~uint64_t(255) : 256;
    hipError_t e = hipMallocAsync(&p, n, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        fail(EVQ_ENOMEM, "hipMallocAsync of " + std::to_string(bytes) + " bytes failed");
    }
    return p;
}

void stream_free(void* p, hipStream_t s) {
    if (p) EVQ_HIP(hipFreeAsync(p, s));
}

namespace {

void* user_alloc(const evq_allocator& ua, uint64_t bytes) {
    const uint64_t n = bytes ? (bytes + 255) & ~uint64_t(255) : 256;
    void* p = ua.alloc((size_t)n, ua.ctx);
    if (!p) fail(EVQ_ENOMEM, "the caller's allocator returned NULL for " + std::to_string(n) + " bytes");
    return p;
}

}  // namespace

void* graph_alloc(const Graph& g, uint64_t bytes, hipStream_t s) {
    return g.has_ua ? user_alloc(g.ua, bytes) : stream_alloc(bytes, s);
}

void graph_free(const Graph& g, void* p, hipStream_t s) {
    if (!p) return;
    if (g.has_ua) {
        (void)hipStreamSynchronize(s);
        g.ua.free(p, g.ua.ctx);
    } else {
        stream_free(p, s);
    }
}

void init_mempool(int device) {
    static std::mutex mu;
    static std::vector<int> done;
    std::lock_guard<std::mutex> lk(mu);
    if (std::find(done.begin(), done.end(), device) != done.end()) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
        uint64_t thr = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    (void)hipGetLastError();
    done.push_back(device);
}

namespace {
thread_local Workspace* t_arena = nullptr;
}  // namespace

NoAlloc*& noalloc_ctx() {
    thread_local NoAlloc* p = nullptr;
    return p;
}

Workspace& Workspace::arena(hipStream_t s, NoAlloc& na) {
    if (!t_arena) t_arena = new Workspace(s);  // host object only, once per thread
    Workspace& w = *t_arena;
    w.s_ = s;
    w.na_ = &na;
    for (int i = 0; i < kSlots; ++i) {
        w.p_[i] = nullptr;
        w.cap_[i] = 0;
    }
    w.fresh_flags = true;  // the scratch holds whatever the last call left
    w.in_use = false;
    w.stamp_seen = nullptr;
    w.epoch = 0;
    return w;
}

Workspace& Workspace::get(hipStream_t s) {
    if (noalloc_ctx() && t_arena) return *t_arena;
    thread_local std::vector<std::pair<std::pair<int, hipStream_t>, Workspace*>> all;  // per thread
    int dev = 0;
    EVQ_HIP(hipGetDevice(&dev));
    for (auto& kv : all)
        if (kv.first.first == dev && kv.first.second == s) return *kv.second;
    all.push_back({{dev, s}, new Workspace(s)});
    return *all.back().second;
}

// Buffers come from the device's stream-ordered pool on the workspace's own
// stream (every use is on that stream), so growing one needs no
// synchronisation.
void* Workspace::raw(Slot slot, uint64_t bytes) {
    if (bytes == 0) bytes = 16;
    if (cap_[slot] >= bytes) return p_[slot];
    if (na_) {  // bump allocation in the caller-less scratch array
        const uint64_t want = (bytes + 255) & ~uint64_t(255);
        if (na_->used + want > na_->cap)
            fail(EVQ_ERANGE, "the query needs more than the " + std::to_string(na_->cap >> 20) +
                                 " MiB scratch of evq_query_noalloc (" + std::to_string((na_->used + want) >> 20) +
                                 " MiB asked for so far); use evq_query");
        p_[slot] = na_->base + na_->used;
        cap_[slot] = want;
        na_->used += want;
        if (slot == kFlags) fresh_flags = true;
        if (slot == kStamp) stamp_seen = nullptr;  // new memory: its stamps are unknown
        return p_[slot];
    }
    if (p_[slot]) {
        stream_free(p_[slot], s_);
        p_[slot] = nullptr;
        cap_[slot] = 0;
    }
    const uint64_t want = ((bytes + bytes / 4) + 4095) & ~uint64_t(4095);
    p_[slot] = stream_alloc(want, s_);
    cap_[slot] = want;
    if (slot == kFlags) fresh_flags = true;
    // a larger buffer may start at the old one's address: its stamps are unknown all the same
    if (slot == kStamp) stamp_seen = nullptr;
    return p_[slot];
}

void* Arena::raw(uint64_t bytes) {
    void* p = nullptr;
    uint64_t n = (bytes + 255) & ~uint64_t(255);
    if (n == 0) n = 256;
    ptrs_.reserve(ptrs_.size() + 1);  // so that recording p below cannot throw
    if (ua_) {
        p = user_alloc(*ua_, n);
    } else {
        hipError_t e = hipMallocAsync(&p, n, s_);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            fail(EVQ_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        }
    }
    ptrs_.push_back(p);
    bytes_ += n;
    return p;
}

void Arena::release(void* p) {
    auto it = std::find(ptrs_.begin(), ptrs_.end(), p);
    if (it == ptrs_.end()) return;
    if (ua_) {
        (void)hipStreamSynchronize(s_);
        ua_->free(p, ua_->ctx);
    } else {
        (void)hipFreeAsync(p, s_);
    }
    ptrs_.erase(it);
}

Arena::~Arena() {
    if (ua_) {
        if (!ptrs_.empty()) (void)hipStreamSynchronize(s_);
        for (void* p : ptrs_) ua_->free(p, ua_->ctx);
        return;
    }
    for (void* p : ptrs_) (void)hipFreeAsync(p, s_);
}

Mailbox::Mailbox(size_t n) {
    void* p = nullptr;
    EVQ_HIP(hipHostMalloc(&p, n * sizeof(uint32_t), hipHostMallocDefault));
    h = static_cast<uint32_t*>(p);
    std::memset(h, 0, n * sizeof(uint32_t));
}

Mailbox::~Mailbox() {
    if (h && pinned) (void)hipHostFree(h);
}

Mailbox& Mailbox::get() {
    if (noalloc_ctx()) {
        thread_local uint32_t plain[16];
        thread_local Mailbox pmb(plain);
        return pmb;
    }
    thread_local Mailbox* mb = new Mailbox(16);  // lives as long as the thread
    return *mb;
}

// ------------------------------------------------------------------ host slots

HostSlots::HostSlots() {
    void* p = nullptr;
    EVQ_HIP(hipHostMalloc(&p, kSlots * sizeof(uint32_t),
                          hipHostMallocMapped | hipHostMallocCoherent | hipHostMallocPortable));
    h_ = static_cast<uint32_t*>(p);
    for (uint32_t i = 0; i < kSlots; ++i) h_[i] = kEmpty;
    void* d = nullptr;
    EVQ_HIP(hipHostGetDevicePointer(&d, p, 0));
    d_ = static_cast<uint32_t*>(d);
}

HostSlots& HostSlots::get() {
    thread_local HostSlots* hs = new HostSlots();  // lives as long as the thread
    return *hs;
}

// ------------------------------------------------------------------ tuning

namespace {

std::mutex g_tuning_mu;
bool g_tuning_init = false;
evq_tuning g_tuning;

double env_f64(const char* name, double dflt) {
    const char* e = getenv(name);
    if (!e || !*e) return dflt;
    char* endp = nullptr;
    const double v = strtod(e, &endp);
    return endp != e ? v : dflt;  // an unreadable value keeps the default
}

uint32_t env_u32(const char* name, uint32_t dflt) {
    const char* e = getenv(name);
    if (!e || !*e) return dflt;
    char* endp = nullptr;
    const unsigned long long v = strtoull(e, &endp, 10);
    if (endp == e) return dflt;
    return v > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)v;
}

evq_tuning tuning_from_env() {
    evq_tuning t;
    std::memset(&t, 0, sizeof(t));
    t.pull_frac = env_f64("EVQ_PULL_FRAC", 0.5);
    t.split_frac = env_f64("EVQ_SPLIT_FRAC", 0.0);
    t.split_min = std::max<uint32_t>(1u, env_u32("EVQ_SPLIT_MIN", 8u));
    t.launch_depth = std::min<uint32_t>(32u, std::max<uint32_t>(1u, env_u32("EVQ_LAUNCH_DEPTH", 3u)));
    t.direct_tasks = env_u32("EVQ_DIRECT_TASKS", 1u << 18);
    t.append_rebuild = env_u32("EVQ_APPEND_REBUILD", 0u) != 0;
    t.trace_loops = env_u32("EVQ_TRACE_LOOPS", 0u) != 0;
    t.append_edges = env_u32("EVQ_APPEND_EDGES", 1u << 17);
    t.append_items = env_u32("EVQ_APPEND_ITEMS", 0u);
    t.relax_staged = env_u32("EVQ_RELAX_STAGED", 2u);
    t.bucket_width = env_u32("EVQ_BUCKET_WIDTH", 0u);
    t.vertex_order = env_u32("EVQ_VERTEX_ORDER", 1u) != 0;
    static const char* delta_names[5] = {"EVQ_DELTA_SSSP", "EVQ_DELTA_BFS", "EVQ_DELTA_SSWP", "EVQ_DELTA_SSNP",
                                         "EVQ_DELTA_VITERBI"};
    static const char* heavy_names[5] = {"EVQ_HEAVY_SSSP", "EVQ_HEAVY_BFS", "EVQ_HEAVY_SSWP", "EVQ_HEAVY_SSNP",
                                         "EVQ_HEAVY_VITERBI"};
    const uint32_t delta_all = env_u32("EVQ_DELTA", 0u), heavy_all = env_u32("EVQ_HEAVY", 0u);
    for (int a = 0; a < 5; ++a) {
        t.delta[a] = env_u32(delta_names[a], delta_all);
        t.heavy[a] = env_u32(heavy_names[a], heavy_all);
    }
    return t;
}

}  // namespace

evq_tuning tuning() {
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    if (!g_tuning_init) {
        g_tuning = tuning_from_env();
        g_tuning_init = true;
    }
    return g_tuning;
}

void set_tuning(const evq_tuning& t) {
    if (t.launch_depth < 1 || t.launch_depth > 32) fail(EVQ_EINVAL, "tuning: launch_depth must be in [1, 32]");
    if (t.split_min < 1) fail(EVQ_EINVAL, "tuning: split_min must be >= 1");
    if (t.relax_staged != 0 && t.relax_staged != 2 && t.relax_staged != 4)
        fail(EVQ_EINVAL, "tuning: relax_staged must be 0, 2 or 4");
    std::lock_guard<std::mutex> lk(g_tuning_mu);
    g_tuning = t;
    g_tuning_init = true;
}

uint64_t launch_depth() { return tuning().launch_depth; }

bool trace_loops() { return tuning().trace_loops != 0; }

void wait_slot(volatile uint32_t* slot, hipStream_t s, const char* what) {
    if (__atomic_load_n(slot, __ATOMIC_ACQUIRE) != HostSlots::kEmpty) return;
    const auto t0 = std::chrono::steady_clock::now();
    auto next_check = t0 + std::chrono::microseconds(200);
    for (;;) {
        if (__atomic_load_n(slot, __ATOMIC_ACQUIRE) != HostSlots::kEmpty) return;
        const auto now = std::chrono::steady_clock::now();
        if (now < next_check) continue;
        next_check = now + std::chrono::microseconds(200);
        const hipError_t e = hipStreamQuery(s);
        if (e == hipSuccess) {
            EVQ_HIP(hipStreamSynchronize(s));
            if (__atomic_load_n(slot, __ATOMIC_ACQUIRE) != HostSlots::kEmpty) return;
            fail(EVQ_EDEVICE, std::string(what) + ": the stream drained without publishing a frontier size");
        }
        if (e != hipErrorNotReady) fail(EVQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(300))
            fail(EVQ_EDEVICE, std::string(what) + ": no progress for 300 s");
    }
}

// ------------------------------------------------------------------ timing

namespace {
struct TimingState {
    std::mutex mu;
    bool on = false;
    struct Rec {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::map<std::string, std::pair<uint64_t, double>> acc;
};
TimingState& ts() {
    static TimingState t;
    return t;
}
void drain_locked(TimingState& t) {
    for (auto& r : t.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto& x = t.acc[r.name];
            x.first += 1;
            x.second += ms;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    t.pending.clear();
    (void)hipGetLastError();
}
}  // namespace

bool timing_on() { return ts().on; }

TimingScope::TimingScope(const char* n, hipStream_t st) : name(n), s(st) {
    if (!ts().on || noalloc_ctx()) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        a = b = nullptr;
        return;
    }
    (void)hipEventRecord(a, s);
}

TimingScope::~TimingScope() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    TimingState& t = ts();
    std::lock_guard<std::mutex> lk(t.mu);
    t.pending.push_back({name, a, b});
    if (t.pending.size() > 4096) drain_locked(t);
}

void post_launch(const char* name) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(EVQ_EDEVICE, std::string("launch of ") + name + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------------ fill

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
    if (n == 0) return;
    EVQ_LAUNCH("fill_u32", k_fill_u32, grid_for(n, 256 * 8, 8192), 256, s, p, n, v);
}

// ------------------------------------------------------------------ scan

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

// Block-wide exclusive scan of one value per thread; returns the block total in *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wsum[kScanBlock / 64];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kScanBlock / 64; ++w) {
        uint32_t x = wsum[w];
        if (w < wave) before += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

__global__ void k_scan_reduce(const uint32_t* __restrict__ in, uint64_t n, uint32_t* __restrict__ sums) {
    uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint32_t acc = 0;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        uint64_t i = base + (uint64_t)r * kScanBlock + threadIdx.x;
        if (i < n) acc += in[i];
    }
    uint32_t tot;
    (void)block_excl_scan(acc, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_scan_apply(const uint32_t* in, uint32_t* out, uint64_t n, const uint32_t* __restrict__ offs,
                             uint32_t* total) {
    __shared__ uint32_t tile[kScanTile];
    uint64_t base = (uint64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        uint64_t i = base + (uint64_t)r * kScanBlock + threadIdx.x;
        tile[r * kScanBlock + threadIdx.x] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t v[kScanItems];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = acc;
        acc += tile[threadIdx.x * kScanItems + k];
    }
    uint32_t tot;
    uint32_t pre = block_excl_scan(acc, &tot);
    uint32_t off = offs ? offs[blockIdx.x] : 0u;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) tile[threadIdx.x * kScanItems + k] = v[k] + pre + off;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kScanItems; ++r) {
        uint64_t i = base + (uint64_t)r * kScanBlock + threadIdx.x;
        if (i < n) out[i] = tile[r * kScanBlock + threadIdx.x];
    }
    if (total && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = off + tot;
}

void scan_exclusive(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* d_total, hipStream_t s, Arena& ar) {
    if (n == 0) {
        if (d_total) fill_u32(d_total, 1, 0u, s);
        return;
    }
    uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb > 0x7FFFFFFFull) fail(EVQ_ERANGE, "scan too large");
    if (nb == 1) {
        EVQ_LAUNCH("scan_apply", k_scan_apply, 1, kScanBlock, s, in, out, n, (const uint32_t*)nullptr, d_total);
        return;
    }
    uint32_t* sums = ar.alloc<uint32_t>(nb);
    EVQ_LAUNCH("scan_reduce", k_scan_reduce, (uint32_t)nb, kScanBlock, s, in, n, sums);
    scan_exclusive(sums, sums, nb, nullptr, s, ar);
    EVQ_LAUNCH("scan_apply", k_scan_apply, (uint32_t)nb, kScanBlock, s, in, out, n, (const uint32_t*)sums, d_total);
    ar.release(sums);
}

}  // namespace evq

// ------------------------------------------------------------------ timing ABI

extern "C" void evq_timing_enable(int on) {
    auto& t = evq::ts();
    std::lock_guard<std::mutex> lk(t.mu);
    t.on = on != 0;
}

extern "C" void evq_timing_reset(void) {
    auto& t = evq::ts();
    std::lock_guard<std::mutex> lk(t.mu);
    evq::drain_locked(t);
    t.acc.clear();
}

extern "C" int evq_timing_report(evq_kernel_time* out, int cap) {
    auto& t = evq::ts();
    std::lock_guard<std::mutex> lk(t.mu);
    evq::drain_locked(t);
    int i = 0;
    for (auto& kv : t.acc) {
        if (out && i < cap) {
            std::memset(out[i].name, 0, sizeof(out[i].name));
            std::strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
            out[i].launches = kv.second.first;
            out[i].total_ms = kv.second.second;
        }
        ++i;
    }
    return i;
}
