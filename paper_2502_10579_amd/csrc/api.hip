// C ABI of the library: argument validation, error capture and dispatch.
// Nothing throws across this boundary; every failure becomes an evq_status
// with a thread-local message.
#include <algorithm>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.h"
#include "ceiling.h"
#include "evq_internal.h"
#include "handle.h"

namespace evq {
thread_local std::string g_last_error;
}  // namespace evq

using evq::g_last_error;

namespace {

evq_status guard_exc() {
    try {
        throw;
    } catch (const evq::Error& e) {
        g_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return EVQ_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return EVQ_EDEVICE;
    } catch (...) {
        g_last_error = "unknown failure";
        return EVQ_EDEVICE;
    }
}

evq_status bad(evq_status c, const char* msg) {
    g_last_error = msg;
    return c;
}

// Validates a query and forms the mask of the window of snapshots
// [b, b + L) (global ids; the graph holds first .. first + K - 1).
evq_status make_window(const evq::Graph& g, uint32_t algo, uint32_t source, uint64_t b, uint32_t L,
                       evq::Window& W) {
    if (algo > EVQ_VITERBI) return bad(EVQ_EINVAL, "unknown algorithm");
    if (source >= g.V) return bad(EVQ_ERANGE, "source vertex out of range");
    if (L == 0 || L > g.K || b < g.first || b - g.first > g.K - L) return bad(EVQ_ERANGE, "window out of range");
    W.b = (uint32_t)(b % g.K);
    W.L = L;
    W.K = g.K;
    W.w[0] = W.w[1] = 0;
    for (uint32_t i = 0; i < L; ++i) {
        const uint32_t t = (W.b + i) % g.K;
        W.w[t >> 6] |= 1ull << (t & 63);
    }
    W.full = L == g.K;
    return EVQ_OK;
}

}  // namespace

extern "C" {

evq_status evq_build(uint32_t num_vertices, const evq_edge* base, uint64_t n_base, const evq_batch* batches,
                     uint32_t K, const evq_allocator* alloc, void* stream, evq_graph** out) {
    g_last_error.clear();
    if (!out) return bad(EVQ_EINVAL, "out is NULL");
    *out = nullptr;
    if (num_vertices == 0) return bad(EVQ_EINVAL, "num_vertices must be >= 1");
    if (K == 0 || K > EVQ_MAX_SNAPSHOTS) return bad(EVQ_EINVAL, "K must be in [1, 128]");
    if (!batches) return bad(EVQ_EINVAL, "batches is NULL");
    if (n_base && !base) return bad(EVQ_EINVAL, "base is NULL with n_base > 0");
    if (alloc && (!alloc->alloc || !alloc->free)) return bad(EVQ_EINVAL, "allocator without alloc or free");
    try {
        evq::Graph* g = evq::build_graph(num_vertices, base, n_base, batches, K, alloc, (hipStream_t)stream);
        std::shared_ptr<const evq::Graph> sp;
        try {
            sp = std::shared_ptr<const evq::Graph>(g, evq::release_graph);
        } catch (...) {
            evq::free_graph(g, (hipStream_t)stream);
            throw;
        }
        evq_graph* h = new evq_graph();
        h->cur = std::move(sp);
        *out = h;
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_graph_info_get(const evq_graph* h, evq_graph_info* info) {
    g_last_error.clear();
    if (!h || !info) return bad(EVQ_EINVAL, "NULL argument");
    auto gp = h->get();
    const evq::Graph& g = *gp;
    std::memset(info, 0, sizeof(*info));
    info->num_vertices = g.V;
    info->num_snapshots = g.K;
    info->mask_words = g.MW;
    info->num_edges = g.E;
    info->num_partial = g.n_partial;
    info->device_bytes = g.bytes;
    {
        std::lock_guard<std::mutex> lk(g.rv_mu);  // reverse CSR of the pull step, once built
        if (g.rv_built) info->device_bytes += (g.E ? g.E : 1) * 12 + 8;
    }
    {
        std::lock_guard<std::mutex> lk(g.wo_mu);  // weight-ordered rows of the bucketed solve
        info->device_bytes += (uint64_t)g.n_wo * ((g.E ? g.E : 1) * 8 + (uint64_t)(g.V ? g.V : 1) * 4);
    }
    info->build_ms = g.build_ms;
    info->first_snapshot = g.first;
    return EVQ_OK;
}

namespace {

// Export of a graph that numbers its vertices itself: its arrays come to the
// host and are rewritten in the caller's numbering, row by row, each row's
// all-present edges and then its partial ones ordered by (destination,
// weight), as a graph built in the caller's numbering holds them.  Rows are
// rewritten by up to 16 host threads.
void export_caller_order(const evq::Graph& g, uint32_t* row_ptr, uint32_t* row_split, uint32_t* col, uint32_t* w,
                         uint64_t* mask, hipStream_t s) {
    const uint32_t V = g.V, MW = g.MW;
    const uint64_t E = g.E;
    std::vector<uint32_t> rp((uint64_t)V + 1), rs(V), iperm(V), c(E), ww(E);
    std::vector<uint64_t> m(E * MW);
    EVQ_HIP(hipMemcpyAsync(rp.data(), g.row_ptr, ((uint64_t)V + 1) * 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipMemcpyAsync(rs.data(), g.row_split, (uint64_t)V * 4, hipMemcpyDeviceToHost, s));
    EVQ_HIP(hipMemcpyAsync(iperm.data(), g.iperm, (uint64_t)V * 4, hipMemcpyDeviceToHost, s));
    if (E) {
        EVQ_HIP(hipMemcpyAsync(c.data(), g.col, E * 4, hipMemcpyDeviceToHost, s));
        EVQ_HIP(hipMemcpyAsync(ww.data(), g.wgt, E * 4, hipMemcpyDeviceToHost, s));
        EVQ_HIP(hipMemcpyAsync(m.data(), g.mask, E * 8 * MW, hipMemcpyDeviceToHost, s));
    }
    EVQ_HIP(hipStreamSynchronize(s));
    const std::vector<uint32_t>& perm = *g.perm_h;
    std::vector<uint32_t> nrp((uint64_t)V + 1);
    nrp[0] = 0;
    for (uint32_t v = 0; v < V; ++v) nrp[v + 1] = nrp[v] + (rp[perm[v] + 1] - rp[perm[v]]);
    if (row_ptr) std::memcpy(row_ptr, nrp.data(), ((uint64_t)V + 1) * 4);
    auto rows = [&](uint32_t v0, uint32_t v1) {
        std::vector<uint32_t> idx;
        for (uint32_t v = v0; v < v1; ++v) {
            const uint32_t i = perm[v], b = rp[i], e = rp[i + 1], sp = rs[i];
            if (row_split) row_split[v] = nrp[v] + (sp - b);
            idx.resize(e - b);
            for (uint32_t j = b; j < e; ++j) idx[j - b] = j;
            auto by_dst_w = [&](uint32_t x, uint32_t y) {
                const uint32_t dx = iperm[c[x]], dy = iperm[c[y]];
                return dx != dy ? dx < dy : ww[x] < ww[y];
            };
            std::sort(idx.begin(), idx.begin() + (sp - b), by_dst_w);
            std::sort(idx.begin() + (sp - b), idx.end(), by_dst_w);
            for (uint32_t k = 0; k < e - b; ++k) {
                const uint64_t o = (uint64_t)nrp[v] + k, j = idx[k];
                if (col) col[o] = iperm[c[j]];
                if (w) w[o] = ww[j];
                if (mask)
                    for (uint32_t q = 0; q < MW; ++q) mask[o * MW + q] = m[j * MW + q];
            }
        }
    };
    const uint32_t nt = std::max(1u, std::min(16u, std::min(std::thread::hardware_concurrency(), V / 4096 + 1)));
    std::vector<std::thread> th;
    for (uint32_t t = 0; t < nt; ++t)
        th.emplace_back(rows, (uint32_t)((uint64_t)V * t / nt), (uint32_t)((uint64_t)V * (t + 1) / nt));
    for (std::thread& t : th) t.join();
}

}  // namespace

evq_status evq_graph_export(const evq_graph* h, uint32_t* row_ptr, uint32_t* row_split, uint32_t* col, uint32_t* w,
                            uint64_t* mask, void* stream) {
    g_last_error.clear();
    if (!h) return bad(EVQ_EINVAL, "graph handle is NULL");
    try {
        auto gp = h->get();
        const evq::Graph& g = *gp;
        hipStream_t s = (hipStream_t)stream;
        evq::UseGuard ug{g, s};
        if (g.perm_h) {
            export_caller_order(g, row_ptr, row_split, col, w, mask, s);
            return EVQ_OK;
        }
        if (row_ptr) EVQ_HIP(hipMemcpyAsync(row_ptr, g.row_ptr, ((uint64_t)g.V + 1) * 4, hipMemcpyDeviceToHost, s));
        if (row_split) EVQ_HIP(hipMemcpyAsync(row_split, g.row_split, (uint64_t)g.V * 4, hipMemcpyDeviceToHost, s));
        if (g.E) {
            if (col) EVQ_HIP(hipMemcpyAsync(col, g.col, g.E * 4, hipMemcpyDeviceToHost, s));
            if (w) EVQ_HIP(hipMemcpyAsync(w, g.wgt, g.E * 4, hipMemcpyDeviceToHost, s));
            if (mask) EVQ_HIP(hipMemcpyAsync(mask, g.mask, g.E * 8 * g.MW, hipMemcpyDeviceToHost, s));
        }
        EVQ_HIP(hipStreamSynchronize(s));
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_gather_ceiling(const evq_graph* h, uint32_t launches, double* edges_per_s, void* stream) {
    g_last_error.clear();
    if (!h || !edges_per_s) return bad(EVQ_EINVAL, "NULL argument");
    if (launches == 0) return bad(EVQ_EINVAL, "launches must be positive");
    try {
        auto gp = h->get();
        const evq::Graph& g = *gp;
        hipStream_t s = (hipStream_t)stream;
        evq::UseGuard ug{g, s};
        *edges_per_s = evq::gather_ceiling(g, launches, s);
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_query(const evq_graph* h, uint32_t algo, uint32_t source, uint32_t win_begin, uint32_t win_len,
                     uint32_t* d_values, evq_query_stats* stats, void* stream) {
    g_last_error.clear();
    if (!h) return bad(EVQ_EINVAL, "graph handle is NULL");
    auto gp = h->get();
    evq::Window W;
    evq_status rc = make_window(*gp, algo, source, win_begin, win_len, W);
    if (rc != EVQ_OK) return rc;
    if (!d_values) return bad(EVQ_EINVAL, "d_values is NULL");
    try {
        evq::QueryOut qo;
        qo.want_stats = stats != nullptr;
        evq::UseGuard ug{*gp, (hipStream_t)stream};
        evq::run_query(*gp, algo, evq::internal_id(*gp, source), W, d_values, nullptr, nullptr, false, qo,
                       (hipStream_t)stream);
        if (stats) *stats = qo.st;
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_query_noalloc(const evq_graph* h, uint32_t algo, uint32_t source, uint32_t win_begin,
                             uint32_t win_len, uint32_t* d_values, void* stream) {
    g_last_error.clear();
    if (!h) return bad(EVQ_EINVAL, "graph handle is NULL");
    auto gp = h->get();
    evq::Window W;
    evq_status rc = make_window(*gp, algo, source, win_begin, win_len, W);
    if (rc != EVQ_OK) return rc;
    if (!d_values) return bad(EVQ_EINVAL, "d_values is NULL");
    try {
        int dev = 0;
        EVQ_HIP(hipGetDevice(&dev));
        if (dev != gp->device) return bad(EVQ_EINVAL, "the graph is on another device than the current one");
        uint64_t cap = 0;
        char* base = evq::noalloc_scratch(dev, &cap);
        static std::mutex busy_mu[64];  // one no-allocation call per device at a time
        std::unique_lock<std::mutex> busy(busy_mu[dev & 63], std::try_to_lock);
        if (!busy.owns_lock()) return bad(EVQ_EBUSY, "another evq_query_noalloc call is running on this device");
        evq::NoAlloc na;
        na.base = base;
        na.cap = cap;
        na.used = evq::kNoAllocSlotBytes;
        struct Scope {
            explicit Scope(evq::NoAlloc* p) { evq::noalloc_ctx() = p; }
            ~Scope() { evq::noalloc_ctx() = nullptr; }
        } scope(&na);
        hipStream_t s = (hipStream_t)stream;
        evq::Workspace::arena(s, na);
        evq::QueryOut qo;
        try {
            evq::run_query(*gp, algo, evq::internal_id(*gp, source), W, d_values, nullptr, nullptr, false, qo, s);
        } catch (...) {
            (void)hipStreamSynchronize(s);  // nothing queued may still use the scratch or this version
            throw;
        }
        EVQ_HIP(hipStreamSynchronize(s));
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_query_bounds(const evq_graph* h, uint32_t algo, uint32_t source, uint32_t win_begin, uint32_t win_len,
                            uint32_t* d_rcap, uint32_t* d_rcup, void* stream) {
    g_last_error.clear();
    if (!h) return bad(EVQ_EINVAL, "graph handle is NULL");
    auto gp = h->get();
    evq::Window W;
    evq_status rc = make_window(*gp, algo, source, win_begin, win_len, W);
    if (rc != EVQ_OK) return rc;
    try {
        evq::QueryOut qo;
        evq::UseGuard ug{*gp, (hipStream_t)stream};
        evq::run_query(*gp, algo, evq::internal_id(*gp, source), W, nullptr, d_rcap, d_rcup, true, qo,
                       (hipStream_t)stream);
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_query_plain(const evq_graph* h, uint32_t algo, uint32_t source, uint32_t win_begin, uint32_t win_len,
                           uint32_t* d_values, evq_query_stats* stats, void* stream) {
    g_last_error.clear();
    if (!h) return bad(EVQ_EINVAL, "graph handle is NULL");
    auto gp = h->get();
    evq::Window W;
    evq_status rc = make_window(*gp, algo, source, win_begin, win_len, W);
    if (rc != EVQ_OK) return rc;
    if (!d_values) return bad(EVQ_EINVAL, "d_values is NULL");
    try {
        evq::QueryOut qo;
        qo.want_stats = stats != nullptr;
        evq::UseGuard ug{*gp, (hipStream_t)stream};
        evq::run_plain(*gp, algo, evq::internal_id(*gp, source), W, d_values, qo, (hipStream_t)stream);
        if (stats) *stats = qo.st;
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_query_sequential(const evq_graph* h, uint32_t algo, uint32_t source, uint32_t win_begin,
                                uint32_t win_len, uint32_t* d_values, evq_query_stats* stats, void* stream) {
    g_last_error.clear();
    if (!h) return bad(EVQ_EINVAL, "graph handle is NULL");
    auto gp = h->get();
    evq::Window W;
    evq_status rc = make_window(*gp, algo, source, win_begin, win_len, W);
    if (rc != EVQ_OK) return rc;
    if (!d_values) return bad(EVQ_EINVAL, "d_values is NULL");
    try {
        evq::QueryOut qo;
        qo.want_stats = stats != nullptr;
        evq::UseGuard ug{*gp, (hipStream_t)stream};
        evq::run_sequential(*gp, algo, evq::internal_id(*gp, source), W, d_values, qo, (hipStream_t)stream);
        if (stats) *stats = qo.st;
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_query_batch(const evq_graph* h, const evq_query_desc* q, uint32_t n, evq_result* results,
                           evq_query_stats* stats, void* stream) {
    g_last_error.clear();
    if (!h) return bad(EVQ_EINVAL, "graph handle is NULL");
    if (!q || !results) return bad(EVQ_EINVAL, "NULL query or result array");
    if (n == 0 || n > 65536) return bad(EVQ_ERANGE, "a batch holds 1..65536 queries");
    std::memset(results, 0, sizeof(evq_result) * n);
    try {
        auto gp = h->get();
        std::vector<evq::BatchQuery> bq(n);
        for (uint32_t i = 0; i < n; ++i) {
            evq_status rc = make_window(*gp, q[i].algo, q[i].source, q[i].win_begin, q[i].win_len, bq[i].W);
            if (rc != EVQ_OK) {
                g_last_error = "query " + std::to_string(i) + ": " + g_last_error;
                return rc;
            }
            bq[i].algo = q[i].algo;
            bq[i].source = evq::internal_id(*gp, q[i].source);
        }
        std::vector<evq::Compact> c(n);
        evq::UseGuard ug{*gp, (hipStream_t)stream};  // the stream waits for every worker stream
        evq::run_batch(*gp, bq.data(), n, c.data(), stats, (hipStream_t)stream);
        for (uint32_t i = 0; i < n; ++i) {
            evq_result& r = results[i];
            r.algo = q[i].algo;
            r.source = q[i].source;
            r.win_begin = q[i].win_begin;
            r.win_len = q[i].win_len;
            r.num_vertices = gp->V;
            r.n_unstable = c[i].nU;
            r.row_stride = c[i].LG;
            r.d_rcap = c[i].rcap;
            r.d_unstable = c[i].ulist;
            r.d_x = c[i].X;
        }
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_result_expand(const evq_result* r, uint32_t* d_values, void* stream) {
    g_last_error.clear();
    if (!r || !d_values) return bad(EVQ_EINVAL, "NULL argument");
    if (!r->d_rcap || r->win_len == 0 || r->num_vertices == 0) return bad(EVQ_EINVAL, "empty result");
    if (r->n_unstable && (!r->d_unstable || !r->d_x || r->row_stride < r->win_len))
        return bad(EVQ_EINVAL, "malformed result");
    try {
        evq::expand_compact(r->num_vertices, r->win_len, r->d_rcap, r->d_unstable, r->d_x, r->n_unstable,
                            r->row_stride, d_values, (hipStream_t)stream);
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_tuning_get(evq_tuning* t) {
    g_last_error.clear();
    if (!t) return bad(EVQ_EINVAL, "NULL argument");
    *t = evq::tuning();
    return EVQ_OK;
}

evq_status evq_tuning_set(const evq_tuning* t) {
    g_last_error.clear();
    if (!t) return bad(EVQ_EINVAL, "NULL argument");
    try {
        evq::set_tuning(*t);
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_expand(const evq_result* r, uint32_t* d_values, void* stream) {
    return evq_result_expand(r, d_values, stream);
}

evq_status evq_result_free(evq_result* r, void* stream) {
    g_last_error.clear();
    if (!r) return bad(EVQ_EINVAL, "result is NULL");
    try {
        evq::stream_free(const_cast<uint32_t*>(r->d_rcap), (hipStream_t)stream);
        evq::stream_free(const_cast<uint32_t*>(r->d_unstable), (hipStream_t)stream);
        std::memset(r, 0, sizeof(*r));
        return EVQ_OK;
    } catch (...) {
        std::memset(r, 0, sizeof(*r));
        return guard_exc();
    }
}

evq_status evq_batch_config_get(evq_batch_config* c) {
    g_last_error.clear();
    if (!c) return bad(EVQ_EINVAL, "config is NULL");
    try {
        const evq::BatchTuning t = evq::batch_tuning();
        std::memset(c, 0, sizeof(*c));
        c->lanes = t.lanes;
        c->chunk = t.chunk;
        c->blocks = t.blocks;
        c->group = t.group;
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_batch_config_set(const evq_batch_config* c) {
    g_last_error.clear();
    if (!c) return bad(EVQ_EINVAL, "config is NULL");
    try {
        evq::BatchTuning t = evq::batch_tuning();
        if (c->lanes) t.lanes = c->lanes;
        if (c->chunk) t.chunk = c->chunk;
        if (c->blocks) t.blocks = c->blocks;
        if (c->group) t.group = c->group;
        evq::set_batch_tuning(t);
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_append(evq_graph* h, const evq_batch* b, void* stream) {
    g_last_error.clear();
    if (!h || !b) return bad(EVQ_EINVAL, "NULL argument");
    try {
        std::lock_guard<std::mutex> lk(h->append_mu);
        auto old = h->get();
        evq::Graph* g = nullptr;
        {
            evq::UseGuard ug{*old, (hipStream_t)stream};
            g = evq::append_graph(*old, *b, (hipStream_t)stream);
        }
        std::shared_ptr<const evq::Graph> sp;
        try {
            sp = std::shared_ptr<const evq::Graph>(g, evq::release_graph);
        } catch (...) {
            evq::free_graph(g, (hipStream_t)stream);
            throw;
        }
        {
            std::lock_guard<std::mutex> lk2(h->mu);
            h->cur = std::move(sp);
        }
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

evq_status evq_batch_autotune(const evq_graph* h, const evq_query_desc* q, uint32_t n, evq_batch_config* chosen,
                              double* best_ms, void* stream) {
    g_last_error.clear();
    if (!h || !q) return bad(EVQ_EINVAL, "NULL argument");
    if (n == 0 || n > 65536) return bad(EVQ_ERANGE, "a batch holds 1..65536 queries");
    try {
        auto gp = h->get();
        std::vector<evq::BatchQuery> bq(n);
        for (uint32_t i = 0; i < n; ++i) {
            evq_status rc = make_window(*gp, q[i].algo, q[i].source, q[i].win_begin, q[i].win_len, bq[i].W);
            if (rc != EVQ_OK) {
                g_last_error = "query " + std::to_string(i) + ": " + g_last_error;
                return rc;
            }
            bq[i].algo = q[i].algo;
            bq[i].source = evq::internal_id(*gp, q[i].source);
        }
        evq::UseGuard ug{*gp, (hipStream_t)stream};
        const evq::BatchTuning t = evq::autotune_batch(*gp, bq.data(), n, (hipStream_t)stream, best_ms);
        if (chosen) {
            std::memset(chosen, 0, sizeof(*chosen));
            chosen->lanes = t.lanes;
            chosen->chunk = t.chunk;
            chosen->blocks = t.blocks;
            chosen->group = t.group;
        }
        return EVQ_OK;
    } catch (...) {
        return guard_exc();
    }
}

void evq_free(evq_graph* h) {
    if (!h) return;
    {
        std::lock_guard<std::mutex> lk(h->mu);
        h->cur.reset();
    }
    delete h;
}

const char* evq_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
