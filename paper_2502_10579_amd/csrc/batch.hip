// Batched queries.  Queries of one algorithm are solved up to 64 at a time
// with one query per lane: the intersection and union bound solves of all of
// them run as one multi-lane relaxation over the shared versioned graph, lane
// q testing the edge's presence mask against query q's own window.  Values
// are laid out [vertex][LQ], LQ = the group size rounded up to a power of
// two, so that a lane group of LQ lanes reads and updates one destination row
// as one contiguous span; a wave holds 64 / LQ such groups, each on its own
// task.  The frontier is the union of the queries' frontiers (query-
// oblivious, as the snapshot-oblivious frontier of Section 4.2).  The bounds
// are then transposed into one column per query, and each query's reduction
// and multi-snapshot relaxation run on worker streams, concurrently,
// producing a compact result (R_cap, compact ids, relaxed rows) that is
// expanded to values[V][L] on demand.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>

#include "batch.h"
#include "tasks.h"

namespace evq {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxLanes = 64;

struct BatchArgs {
    const uint32_t* row_ptr;
    const uint32_t* row_split;
    const uint32_t* col;
    const uint32_t* wgt;
    const uint64_t* mask;
    uint32_t* X;          // [V][LQ] values of this solve
    const uint64_t* win;  // [LQ][2] window bits per lane (0 for an unused lane)
    uint8_t* flags;
    uint64_t* tasks;      // (chunk << 32 | vertex)
    uint32_t* fo;         // frontier items: first task of each vertex in the iteration's task range
    uint32_t* fv;         //   and the vertex
    FrontierCounters* cnt;
    uint32_t V;
    uint32_t chunk;       // edges per task
    uint32_t LQ;          // lanes per row: 1, 2, 4, ..., 64
};

// Lane layout of a wave: 64 / LQ groups of LQ lanes.
struct LaneGroup {
    uint32_t q, g, G;
    uint64_t gmask;  // this group's lanes in a ballot
    __device__ explicit LaneGroup(uint32_t LQ) {
        const uint32_t l = lane_id();
        q = l & (LQ - 1);
        g = l / LQ;
        G = 64 / LQ;
        gmask = (LQ >= 64 ? ~0ull : ((1ull << LQ) - 1ull)) << (g * LQ);
    }
    __device__ bool any(bool x) const { return (__ballot(x) & gmask) != 0; }
};

// Frontier vertices -> items (first task, vertex), a task being `chunk` edges
// of a union row; the packed reservation counts vertices and tasks.  Union
// rows of hubs have 10^4-10^5 tasks, so k_btasks writes them (write_tasks).
__global__ void __launch_bounds__(kCompactBlock) k_bcompact(BatchArgs a, int p, int first) {
    if (compaction_skips(a.cnt, p, first)) return;
    compact_flags(
        a.flags, a.V, &a.cnt->packed[p], &a.cnt->far[p], &a.cnt->fmin[p],
        [&](uint32_t v, uint32_t, uint32_t& items, uint32_t& tasks, uint32_t&, uint2&) {
            tasks = (a.row_ptr[v + 1] - a.row_ptr[v] + a.chunk - 1) / a.chunk;
            items = tasks ? 1u : 0u;
            return 0u;
        },
        [&](uint32_t v, uint32_t item, uint32_t task, uint32_t, uint32_t, uint2) {
            a.fo[item] = task;
            a.fv[item] = v;
        });
}

__global__ void __launch_bounds__(256) k_btasks(BatchArgs a, int p) {
    const unsigned long long cx = a.cnt->packed[p];
    write_tasks(a.fo, a.fv, items_of(cx), edges_of(cx), a.tasks);
}

template <int MW>
__device__ __forceinline__ bool lane_has(const uint64_t* __restrict__ mask, uint32_t e, bool full,
                                         const uint64_t (&w)[MW], bool cup) {
    if (full) return true;
    bool any = false, all = true;
#pragma unroll
    for (int j = 0; j < MW; ++j) {
        const uint64_t m = mask[(uint64_t)e * MW + j] & w[j];
        any |= m != 0;
        all &= m == w[j];
    }
    return cup ? any : all;
}

// One iteration of the batched bound solve: each lane group takes one task
// (up to CH edges of one vertex); lane q relaxes query q over the edges
// present in its window's intersection (CUP = false) or union (CUP = true).
template <int A, bool CUP, int MW, int CH>
__global__ void __launch_bounds__(kBlock) k_bexpand(BatchArgs a, int p, uint32_t* slot) {
    const unsigned long long cx = expand_prologue(a.cnt, p, slot);
    const uint32_t n = edges_of(cx);  // tasks (the items are their vertices)
    if (n == 0) return;
    const uint32_t LQ = a.LQ;
    const LaneGroup lg(LQ);
    const uint32_t q = lg.q;
    uint64_t w[MW];
    bool used = false;
#pragma unroll
    for (int j = 0; j < MW; ++j) {
        w[j] = a.win[q * 2 + j];
        used |= w[j] != 0;
    }
    const uint32_t gw = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * (kBlock / 64);
    for (uint32_t tb = gw * lg.G; tb < n; tb += nw * lg.G) {
        const uint32_t t = tb + lg.g;
        uint32_t u = 0, ne = 0, e0 = 0, split = 0;
        if (t < n) {
            const uint64_t tk = a.tasks[t];
            u = (uint32_t)tk;
            const uint32_t ch = (uint32_t)(tk >> 32);
            const uint32_t rb = a.row_ptr[u], re = a.row_ptr[u + 1];
            split = a.row_split[u];
            e0 = rb + ch * CH;
            ne = re - e0 < (uint32_t)CH ? re - e0 : (uint32_t)CH;
        }
        const uint32_t xu = ne ? a.X[(uint64_t)u * LQ + q] : 0u;
        uint32_t dst[CH], wt[CH], cur[CH];
        bool in[CH];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            in[k] = false;
            dst[k] = 0;
            wt[k] = 0;
            if ((uint32_t)k < ne) {
                const uint32_t e = e0 + k;
                dst[k] = a.col[e];
                wt[k] = a.wgt[e];
                in[k] = used && lane_has<MW>(a.mask, e, e < split, w, CUP);
            }
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) cur[k] = in[k] ? a.X[(uint64_t)dst[k] * LQ + q] : 0u;
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            bool imp = false;
            if (in[k]) {
                const uint32_t cand = Alg<A>::extend(xu, wt[k]);
                if (Alg<A>::better(cand, cur[k])) {
                    Alg<A>::improve_nr(&a.X[(uint64_t)dst[k] * LQ + q], cand);
                    imp = true;
                }
            }
            if (lg.any(imp) && q == 0) mark(a.flags, dst[k]);
        }
    }
}

// Every value unreached, then each used lane's source at its start value.
__global__ void k_binit(uint32_t* X, uint64_t n, uint32_t unreached) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        X[i] = unreached;
}

__global__ void k_bsources(uint32_t* X, uint8_t* flags, const uint32_t* __restrict__ src, uint32_t nq, uint32_t LQ,
                           uint32_t at_source) {
    const uint32_t q = threadIdx.x;
    if (q < nq) {
        X[(uint64_t)src[q] * LQ + q] = at_source;
        flags[src[q]] = 1;
    }
}

// Union solve, first step: every edge partial in some lane's window relaxes
// that lane from the intersection values (one partial edge per lane group).
template <int A, int MW>
__global__ void __launch_bounds__(kBlock) k_bseed(BatchArgs a, const uint32_t* __restrict__ p_src,
                                                  const uint32_t* __restrict__ p_dst, const uint32_t* __restrict__ p_w,
                                                  const uint64_t* __restrict__ p_mask, uint32_t n_partial) {
    const uint32_t LQ = a.LQ;
    const LaneGroup lg(LQ);
    const uint32_t q = lg.q;
    uint64_t w[MW];
    bool used = false;
#pragma unroll
    for (int j = 0; j < MW; ++j) {
        w[j] = a.win[q * 2 + j];
        used |= w[j] != 0;
    }
    const uint32_t gw = (blockIdx.x * kBlock + threadIdx.x) >> 6;
    const uint32_t nw = gridDim.x * (kBlock / 64);
    for (uint32_t ib = gw * lg.G; ib < n_partial; ib += nw * lg.G) {
        const uint32_t i = ib + lg.g;
        bool act = false;
        uint32_t u = 0;
        if (i < n_partial) {
            u = p_src[i];
            bool any = false, all = true;
#pragma unroll
            for (int j = 0; j < MW; ++j) {
                const uint64_t m = p_mask[(uint64_t)i * MW + j] & w[j];
                any |= m != 0;
                all &= m == w[j];
            }
            act = used && any && !all;
        }
        if (!__ballot(act)) continue;
        bool imp = false;
        uint32_t v = 0;
        if (act) {
            v = p_dst[i];
            const uint32_t cand = Alg<A>::extend(a.X[(uint64_t)u * LQ + q], p_w[i]);
            uint32_t* px = &a.X[(uint64_t)v * LQ + q];
            if (Alg<A>::better(cand, *px)) {
                Alg<A>::improve_nr(px, cand);
                imp = true;
            }
        }
        // the group's lanes share the partial edge and so v; any improving lane marks it
        const uint64_t bal = __ballot(imp) & lg.gmask;
        if (bal && lane_id() == (uint32_t)__ffsll((unsigned long long)bal) - 1) mark(a.flags, v);
    }
}

// [V][LQ] -> column q of each used lane (cols[q][v]), through a 64-vertex LDS tile.
__global__ void __launch_bounds__(256) k_transpose(const uint32_t* __restrict__ X, uint32_t V, uint32_t LQ,
                                                   uint32_t* const* __restrict__ cols, uint32_t nq) {
    __shared__ uint32_t tile[64][65];
    for (uint64_t v0 = (uint64_t)blockIdx.x * 64; v0 < V; v0 += (uint64_t)gridDim.x * 64) {
        const uint32_t nv = V - v0 < 64 ? (uint32_t)(V - v0) : 64u;
        for (uint32_t k = threadIdx.x; k < 64 * LQ; k += 256) {
            const uint32_t r = k / LQ, c = k - r * LQ;
            tile[r][c] = r < nv ? X[(v0 + r) * LQ + c] : 0u;
        }
        __syncthreads();
        for (uint32_t k = threadIdx.x; k < 64 * nq; k += 256) {
            const uint32_t q = k / 64, r = k - q * 64;
            if (r < nv) cols[q][v0 + r] = tile[r][q];
        }
        __syncthreads();
    }
}

__global__ void k_copy_u32x4(const uint4* __restrict__ a, uint4* __restrict__ b, uint64_t n4) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n4; i += (uint64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

template <int A, bool CUP, int MW>
void batch_loop(BatchArgs a, uint32_t chunk, uint32_t blocks, Frontier& f, hipStream_t s, uint64_t max_iters,
                uint64_t* iters) {
    const uint32_t cblocks = grid_for(a.V, kCompactIds, 4096);
    const uint32_t tblocks = 2048;
    a.chunk = chunk;
    auto issue = [&](uint64_t, int p, bool first, uint32_t* slot) {
        EVQ_LAUNCH("batch_compact", k_bcompact, cblocks, kCompactBlock, s, a, p, first ? 1 : 0);
        EVQ_LAUNCH("batch_tasks", k_btasks, tblocks, 256, s, a, p);
        switch (chunk) {
        case 4: EVQ_LAUNCH("batch_expand", (k_bexpand<A, CUP, MW, 4>), blocks, kBlock, s, a, p, slot); break;
        case 16: EVQ_LAUNCH("batch_expand", (k_bexpand<A, CUP, MW, 16>), blocks, kBlock, s, a, p, slot); break;
        default: EVQ_LAUNCH("batch_expand", (k_bexpand<A, CUP, MW, 8>), blocks, kBlock, s, a, p, slot); break;
        }
    };
    *iters += drive_loop(issue, f.p, s, max_iters, "batched bound solve");
}

template <int A, int MW>
void batch_bounds_t(const Graph& g, BatchArgs a, uint32_t* Xcap, uint32_t* Xcup, const uint32_t* d_src, uint32_t nq,
                    const BatchTuning& tu, Frontier& f, hipStream_t s, BatchTimes& bt) {
    const uint64_t n = (uint64_t)g.V * a.LQ;
    EVQ_LAUNCH("batch_init", k_binit, grid_for(n, 256 * 8, 16384), 256, s, Xcap, n, Alg<A>::unreached);
    EVQ_LAUNCH("batch_init", k_bsources, 1, 64, s, Xcap, f.flags, d_src, nq, a.LQ, Alg<A>::at_source);
    a.X = Xcap;
    batch_loop<A, false, MW>(a, tu.chunk, tu.blocks, f, s, (uint64_t)g.V + 2, &bt.iters_cap);
    EVQ_LAUNCH("batch_copy", k_copy_u32x4, grid_for((n + 3) / 4, 256 * 4, 16384), 256, s,
               reinterpret_cast<const uint4*>(Xcap), reinterpret_cast<uint4*>(Xcup), (n + 3) / 4);
    a.X = Xcup;
    if (g.n_partial)
        EVQ_LAUNCH("batch_seed", (k_bseed<A, MW>), grid_for((g.n_partial + 63) / 64 * a.LQ, kBlock / 64, 16384), kBlock,
                   s, a, g.p_src, g.p_dst, g.p_w, g.p_mask, (uint32_t)g.n_partial);
    batch_loop<A, true, MW>(a, tu.chunk, tu.blocks, f, s, (uint64_t)g.V + 2, &bt.iters_cup);
}

template <int MW>
void batch_bounds_mw(uint32_t algo, const Graph& g, BatchArgs a, uint32_t* Xcap, uint32_t* Xcup,
                     const uint32_t* d_src, uint32_t nq, const BatchTuning& tu, Frontier& f, hipStream_t s,
                     BatchTimes& bt) {
    switch (algo) {
    case EVQ_SSSP: batch_bounds_t<EVQ_SSSP, MW>(g, a, Xcap, Xcup, d_src, nq, tu, f, s, bt); break;
    case EVQ_BFS: batch_bounds_t<EVQ_BFS, MW>(g, a, Xcap, Xcup, d_src, nq, tu, f, s, bt); break;
    case EVQ_SSWP: batch_bounds_t<EVQ_SSWP, MW>(g, a, Xcap, Xcup, d_src, nq, tu, f, s, bt); break;
    case EVQ_SSNP: batch_bounds_t<EVQ_SSNP, MW>(g, a, Xcap, Xcup, d_src, nq, tu, f, s, bt); break;
    default: batch_bounds_t<EVQ_VITERBI, MW>(g, a, Xcap, Xcup, d_src, nq, tu, f, s, bt); break;
    }
}

}  // namespace

// Bound solves of up to 64 queries of one algorithm; writes query i's R_cap
// and R_cup to rcap_cols[i], rcup_cols[i] (device arrays of V values).
void batch_bounds(const Graph& g, uint32_t algo, const Window* wins, const uint32_t* sources, uint32_t nq,
                  uint32_t* const* rcap_cols, uint32_t* const* rcup_cols, const BatchTuning& tu, hipStream_t s,
                  BatchTimes& bt) {
    if (nq == 0 || nq > (uint32_t)kMaxLanes) fail(EVQ_EINVAL, "a batch holds 1..64 queries");
    uint32_t LQ = 1;
    while (LQ < nq) LQ <<= 1;
    Workspace& ws = Workspace::get(s);
    Frontier f = make_frontier(g, ws, s);
    const uint64_t n = (uint64_t)g.V * LQ;
    uint32_t* Xcap = ws.buf<uint32_t>(Workspace::kBatchCap, n + 4);
    uint32_t* Xcup = ws.buf<uint32_t>(Workspace::kBatchCup, n + 4);
    // per-lane table: windows (2 words), sources, column pointers
    std::vector<uint64_t> hwin(kMaxLanes * 2, 0ull);
    std::vector<uint32_t> hsrc(kMaxLanes, 0u);
    std::vector<uint32_t*> hcols(2 * kMaxLanes, nullptr);
    for (uint32_t i = 0; i < nq; ++i) {
        hwin[2 * i] = wins[i].w[0];
        hwin[2 * i + 1] = wins[i].w[1];
        hsrc[i] = sources[i];
        hcols[i] = rcap_cols[i];
        hcols[kMaxLanes + i] = rcup_cols[i];
    }
    char* tab = ws.buf<char>(Workspace::kBatchTable, 4096);
    uint64_t* d_win = reinterpret_cast<uint64_t*>(tab);
    uint32_t* d_src = reinterpret_cast<uint32_t*>(tab + 1024);
    uint32_t** d_cols = reinterpret_cast<uint32_t**>(tab + 2048);
    EVQ_HIP(hipMemcpyAsync(d_win, hwin.data(), hwin.size() * 8, hipMemcpyHostToDevice, s));
    EVQ_HIP(hipMemcpyAsync(d_src, hsrc.data(), hsrc.size() * 4, hipMemcpyHostToDevice, s));
    EVQ_HIP(hipMemcpyAsync(d_cols, hcols.data(), hcols.size() * sizeof(uint32_t*), hipMemcpyHostToDevice, s));
    BatchArgs a;
    a.row_ptr = g.row_ptr;
    a.row_split = g.row_split;
    a.col = g.col;
    a.wgt = g.wgt;
    a.mask = g.mask;
    a.X = Xcap;
    a.win = d_win;
    a.flags = f.flags;
    a.tasks = ws.buf<uint64_t>(Workspace::kTasks, (uint64_t)g.V + g.E / 4 + 64);
    a.fo = f.fo;
    a.fv = f.fv;
    a.cnt = f.cnt;
    a.V = g.V;
    a.chunk = tu.chunk;
    a.LQ = LQ;
    if (g.MW == 1) batch_bounds_mw<1>(algo, g, a, Xcap, Xcup, d_src, nq, tu, f, s, bt);
    else batch_bounds_mw<2>(algo, g, a, Xcap, Xcup, d_src, nq, tu, f, s, bt);
    const uint32_t tb = grid_for(g.V, 64, 16384);
    EVQ_LAUNCH("batch_transpose", k_transpose, tb, 256, s, Xcap, g.V, LQ, d_cols, nq);
    EVQ_LAUNCH("batch_transpose", k_transpose, tb, 256, s, Xcup, g.V, LQ, d_cols + kMaxLanes, nq);
    ws.in_use = false;
}

// ------------------------------------------------------------------ tuning

namespace {

std::mutex g_tune_mu;
bool g_tune_init = false;
BatchTuning g_tune;

uint32_t env_u32(const char* name, uint32_t dflt) {
    const char* e = getenv(name);
    return e ? (uint32_t)strtoul(e, nullptr, 10) : dflt;
}

BatchTuning checked(BatchTuning t) {
    if (t.lanes != 1 && t.lanes != 2) fail(EVQ_EINVAL, "batch config: lanes must be 1 or 2");
    if (t.chunk != 4 && t.chunk != 8 && t.chunk != 16) fail(EVQ_EINVAL, "batch config: chunk must be 4, 8 or 16");
    if (t.blocks < 64 || t.blocks > 16384) fail(EVQ_EINVAL, "batch config: blocks must be in [64, 16384]");
    if (t.group < 1 || t.group > 64) fail(EVQ_EINVAL, "batch config: group must be in [1, 64]");
    return t;
}

}  // namespace

BatchTuning batch_tuning() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_init) {
        BatchTuning t;
        t.lanes = env_u32("EVQ_BATCH_LANES", t.lanes);
        t.chunk = env_u32("EVQ_BATCH_CHUNK", t.chunk);
        t.blocks = env_u32("EVQ_BATCH_BLOCKS", t.blocks);
        t.group = env_u32("EVQ_BATCH_GROUP", t.group);
        g_tune = checked(t);
        g_tune_init = true;
    }
    return g_tune;
}

void set_batch_tuning(const BatchTuning& t) {
    BatchTuning c = checked(t);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune = c;
    g_tune_init = true;
}

// ------------------------------------------------------------------ worker pool

namespace {

// Completion count and first error of one batch.
struct BatchState {
    std::mutex mu;
    std::condition_variable cv;
    uint64_t pending = 0;
    bool failed = false;
    Error err{EVQ_OK, ""};

    void add(uint64_t k) {
        std::lock_guard<std::mutex> lk(mu);
        pending += k;
    }
    void done() {
        std::lock_guard<std::mutex> lk(mu);
        if (--pending == 0) cv.notify_all();
    }
    bool ok() {
        std::lock_guard<std::mutex> lk(mu);
        return !failed;
    }
    void record_current() {  // inside a catch block
        Error e{EVQ_EDEVICE, "unknown failure"};
        try {
            throw;
        } catch (const Error& x) {
            e = x;
        } catch (const std::bad_alloc&) {
            e = Error{EVQ_ENOMEM, "host allocation failed"};
        } catch (const std::exception& x) {
            e = Error{EVQ_EDEVICE, x.what()};
        } catch (...) {
        }
        std::lock_guard<std::mutex> lk(mu);
        if (!failed) {
            failed = true;
            err = e;
        }
    }
    void wait() {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait(lk, [this] { return pending == 0; });
    }
};

hipEvent_t new_event() {
    hipEvent_t e = nullptr;
    EVQ_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return e;
}

}  // namespace

// ------------------------------------------------------------------ worker pool

Pool& Pool::get(int device) {
    static std::mutex mu;
    static std::vector<std::pair<int, Pool*>> all;
    std::lock_guard<std::mutex> lk(mu);
    for (auto& kv : all)
        if (kv.first == device) return *kv.second;
    Pool* p = new Pool(device, std::max(1u, std::min(16u, env_u32("EVQ_BATCH_WORKERS", 4))));
    all.push_back({device, p});
    return *p;
}

Pool::Pool(int device, uint32_t n) : device_(device), st_(n, nullptr) {
    int prev = 0;
    EVQ_HIP(hipGetDevice(&prev));
    EVQ_HIP(hipSetDevice(device));
    for (uint32_t i = 0; i < n; ++i) EVQ_HIP(hipStreamCreateWithFlags(&st_[i], hipStreamNonBlocking));
    EVQ_HIP(hipSetDevice(prev));
    for (uint32_t i = 0; i < n; ++i) std::thread([this, i] { loop(i); }).detach();
}

void Pool::submit(Job j) {
    {
        std::lock_guard<std::mutex> lk(mu_);
        q_.push_back(std::move(j));
    }
    cv_.notify_one();
}

void Pool::loop(uint32_t i) {
    (void)hipSetDevice(device_);
    for (;;) {
        Job j;
        {
            std::unique_lock<std::mutex> lk(mu_);
            cv_.wait(lk, [this] { return !q_.empty(); });
            j = std::move(q_.front());
            q_.pop_front();
        }
        j(st_[i]);
    }
}

// ------------------------------------------------------------------ batch executor

void run_batch(const Graph& g, const BatchQuery* q, uint32_t n, Compact* out, evq_query_stats* stats,
               hipStream_t s) {
    init_mempool(g.device);
    Pool& pool = Pool::get(g.device);
    const BatchTuning tu = batch_tuning();
    auto st = std::make_shared<BatchState>();
    std::vector<QueryOut> qo(n);
    for (uint32_t i = 0; i < n; ++i) {
        out[i] = Compact{};
        qo[i].want_stats = stats != nullptr;
    }
    std::vector<hipEvent_t> events;
    hipEvent_t e0 = new_event();
    events.push_back(e0);
    EVQ_HIP(hipEventRecord(e0, s));
    const uint64_t vbytes = (uint64_t)g.V * 4;

    // groups of one algorithm, up to 64 queries each
    std::vector<std::vector<uint32_t>> groups;
    if (tu.lanes == 1) {
        for (uint32_t a = 0; a <= EVQ_VITERBI; ++a) {
            std::vector<uint32_t> ids;
            for (uint32_t i = 0; i < n; ++i)
                if (q[i].algo == a) ids.push_back(i);
            // equal groups of at most tu.group queries
            const size_t ng = (ids.size() + tu.group - 1) / tu.group;
            for (size_t k = 0; k < ng; ++k)
                groups.emplace_back(ids.begin() + ids.size() * k / ng, ids.begin() + ids.size() * (k + 1) / ng);
        }
    }
    std::vector<BatchTimes> times(groups.size());
    std::vector<hipEvent_t> gev(groups.size(), nullptr);
    for (auto& e : gev) {
        e = new_event();
        events.push_back(e);
    }

    // add + submit; a job that cannot be queued counts as done and failed
    auto spawn = [&pool](const std::shared_ptr<BatchState>& bs, Pool::Job j) {
        bs->add(1);
        try {
            pool.submit(std::move(j));
        } catch (...) {
            bs->record_current();
            bs->done();
        }
    };
    if (tu.lanes == 2) {
        for (uint32_t i = 0; i < n; ++i) {
            spawn(st, [&, i, st](hipStream_t ws) {
                try {
                    EVQ_HIP(hipStreamWaitEvent(ws, e0, 0));
                    if (st->ok()) {
                        out[i].rcap = static_cast<uint32_t*>(stream_alloc(vbytes, ws));
                        run_query_compact(g, q[i].algo, q[i].source, q[i].W, out[i], qo[i], ws);
                    }
                } catch (...) {
                    st->record_current();
                }
                st->done();
            });
        }
    } else {
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            spawn(st, [&, gi, st](hipStream_t ws) {
                const std::vector<uint32_t>& ids = groups[gi];
                const uint32_t nq = (uint32_t)ids.size();
                std::vector<uint32_t*> rcup(nq, nullptr);
                bool spawned = false;
                try {
                    EVQ_HIP(hipStreamWaitEvent(ws, e0, 0));
                    if (st->ok()) {
                        std::vector<uint32_t*> rcap(nq);
                        std::vector<Window> wins(nq);
                        std::vector<uint32_t> srcs(nq);
                        for (uint32_t k = 0; k < nq; ++k) {
                            const uint32_t i = ids[k];
                            out[i].rcap = rcap[k] = static_cast<uint32_t*>(stream_alloc(vbytes, ws));
                            rcup[k] = static_cast<uint32_t*>(stream_alloc(vbytes, ws));
                            wins[k] = q[i].W;
                            srcs[k] = q[i].source;
                        }
                        batch_bounds(g, q[ids[0]].algo, wins.data(), srcs.data(), nq, rcap.data(), rcup.data(), tu,
                                     ws, times[gi]);
                        EVQ_HIP(hipEventRecord(gev[gi], ws));
                        spawned = true;
                        for (uint32_t k = 0; k < nq; ++k) {
                            const uint32_t i = ids[k];
                            uint32_t* ru = rcup[k];
                            spawn(st, [&, i, ru, gi, st](hipStream_t ts) {
                                try {
                                    EVQ_HIP(hipStreamWaitEvent(ts, gev[gi], 0));
                                    if (st->ok())
                                        run_tail_compact(g, q[i].algo, q[i].source, q[i].W, ru, out[i], qo[i], ts);
                                } catch (...) {
                                    st->record_current();
                                }
                                try {
                                    stream_free(ru, ts);
                                } catch (...) {
                                    st->record_current();
                                }
                                st->done();
                            });
                        }
                    }
                } catch (...) {
                    st->record_current();
                }
                if (!spawned) {
                    for (uint32_t* p : rcup) {
                        try {
                            stream_free(p, ws);
                        } catch (...) {
                        }
                    }
                }
                st->done();
            });
        }
    }
    st->wait();

    // the caller's stream waits for every worker stream
    for (hipStream_t w : pool.streams()) {
        hipEvent_t e = new_event();
        events.push_back(e);
        EVQ_HIP(hipEventRecord(e, w));
        EVQ_HIP(hipStreamWaitEvent(s, e, 0));
    }
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    if (!st->ok()) {
        for (uint32_t i = 0; i < n; ++i) {
            try {
                stream_free(out[i].rcap, s);
                stream_free(out[i].ulist, s);
            } catch (...) {
            }
            out[i] = Compact{};
        }
        throw st->err;
    }
    if (stats) {
        for (uint32_t i = 0; i < n; ++i) stats[i] = qo[i].st;
        for (size_t gi = 0; gi < groups.size(); ++gi)
            for (uint32_t i : groups[gi]) {
                stats[i].iters_cap = times[gi].iters_cap;
                stats[i].iters_cup = times[gi].iters_cup;
            }
    }
}

// Times run_batch on the caller's queries under each candidate (lanes,
// chunk, blocks), after one warm-up run, and installs the fastest.
BatchTuning autotune_batch(const Graph& g, const BatchQuery* q, uint32_t n, hipStream_t s, double* best_ms) {
    std::vector<BatchTuning> cand;
    for (uint32_t group : {16u, 32u, 64u})
        for (uint32_t chunk : {4u, 8u, 16u}) {
            BatchTuning t;
            t.lanes = 1;
            t.chunk = chunk;
            t.blocks = 2048;
            t.group = group;
            cand.push_back(t);
        }
    BatchTuning one;
    one.lanes = 2;
    cand.push_back(one);
    const BatchTuning before = batch_tuning();
    std::vector<Compact> out(n);
    auto run = [&]() {
        run_batch(g, q, n, out.data(), nullptr, s);
        EVQ_HIP(hipStreamSynchronize(s));
        for (Compact& c : out) {
            stream_free(c.rcap, s);
            stream_free(c.ulist, s);
            c = Compact{};
        }
        EVQ_HIP(hipStreamSynchronize(s));
    };
    BatchTuning best = before;
    double best_t = 1e300;
    try {
        set_batch_tuning(before);
        run();  // warm-up: workspaces, first launches
        for (const BatchTuning& t : cand) {
            set_batch_tuning(t);
            const auto t0 = std::chrono::steady_clock::now();
            run();
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (ms < best_t) {
                best_t = ms;
                best = t;
            }
        }
    } catch (...) {
        set_batch_tuning(before);
        throw;
    }
    set_batch_tuning(best);
    if (best_ms) *best_ms = best_t;
    return best;
}

}  // namespace evq
