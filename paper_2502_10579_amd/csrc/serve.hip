// Query server over a resident versioned graph (a systems layer: the paper
// evaluates a fixed set of snapshots known up front).  Queries arrive at any
// time and name only (algorithm, source, window length); at admission the
// window becomes the newest `len` snapshots of the current graph version.
//
// Continuous batching: a dispatcher thread admits queued queries while the
// estimated device footprint of everything in flight stays under a budget,
// and forms groups of up to max_batch queued queries of one algorithm (the
// oldest waiting query picks the algorithm).  A group's bound solves run
// together, one query per lane; each query's reduction and relaxation then
// run on the worker pool and complete independently, so new groups start
// while older queries are still relaxing.  At most max_groups bound solves
// run at once, so that under load queries queue up and later groups fill.
//
// Plain mode runs one query at a time in arrival order (the per-query method
// alone), the baseline the latencies are compared with.
#include <atomic>
#include <chrono>
#include <thread>

#include "batch.h"
#include "handle.h"

namespace evq {
namespace {

struct SQuery {
    uint64_t ticket = 0;
    uint32_t algo = 0, source = 0, len = 0;
    double t_arrival = 0, t_admit = 0, t_bounds = 0, t_done = 0;
    uint32_t group = 1;
    uint64_t win_begin = 0;
    uint32_t win_len = 0, V = 0;
    uint64_t footprint = 0;
    Compact c;
    QueryOut qo;
    evq_status status = EVQ_OK;
    uint32_t* rcup = nullptr;
};

Error current_error() {  // inside a catch block
    try {
        throw;
    } catch (const Error& e) {
        return e;
    } catch (const std::bad_alloc&) {
        return Error{EVQ_ENOMEM, "host allocation failed"};
    } catch (const std::exception& e) {
        return Error{EVQ_EDEVICE, e.what()};
    } catch (...) {
        return Error{EVQ_EDEVICE, "unknown failure"};
    }
}

}  // namespace
}  // namespace evq

struct evq_server {
    evq_graph* h = nullptr;
    evq_server_config cfg{};
    int device = 0;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv;       // dispatcher wake-ups
    std::condition_variable cv_done;  // poll and shutdown
    std::deque<evq::SQuery*> queue;   // arrived, not admitted
    std::deque<evq::SQuery*> done;    // completed, not yet collected
    uint64_t next_ticket = 1;
    uint64_t inflight_bytes = 0;
    uint32_t inflight = 0, groups = 0;
    double est_unstable[5] = {0, 0, 0, 0, 0};  // running estimate of |U| / V per algorithm
    bool stop = false;
    std::thread dispatcher;

    double now() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace evq {
namespace {

uint64_t estimate(const evq_server* sv, const Graph& g, uint32_t algo, uint32_t L) {
    const uint64_t V = g.V;
    const uint64_t LG = pick_lg(L);
    const double fu = sv->est_unstable[algo] > 0 ? sv->est_unstable[algo] : 0.0625;
    return 8 * V + (uint64_t)(fu * (double)V) * (LG * 4 + 4);
}

// Called with sv->mu held.
void finish(evq_server* sv, SQuery* q) {
    q->t_done = sv->now();
    sv->inflight_bytes -= q->footprint;
    sv->inflight -= 1;
    sv->done.push_back(q);
    sv->cv_done.notify_all();
    sv->cv.notify_all();
}

void complete(evq_server* sv, SQuery* q, const Graph& g, hipStream_t s) {
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess && q->status == EVQ_OK) q->status = EVQ_EDEVICE;
    std::lock_guard<std::mutex> lk(sv->mu);
    if (q->status == EVQ_OK) {
        double& est = sv->est_unstable[q->algo];
        const double f = (double)q->c.nU / (double)g.V;
        est = est > 0 ? 0.875 * est + 0.125 * f : f;
    }
    finish(sv, q);
}

void fail_query(SQuery* q, const Error& err, hipStream_t s) {
    q->status = err.code;
    try {
        stream_free(q->c.rcap, s);
        stream_free(q->c.ulist, s);
    } catch (...) {
    }
    q->c = Compact{};
}

// Resolves the window of an admitted query on version g (the newest `len`
// snapshots held, len clamped to K).
void admit(evq_server* sv, SQuery* q, const Graph& g) {
    q->win_len = std::min<uint32_t>(q->len, g.K);
    q->V = g.V;
    q->win_begin = g.first + g.K - q->win_len;
    q->t_admit = sv->now();
}

Window window_of(const Graph& g, const SQuery* q) {
    Window W;
    W.b = (uint32_t)(q->win_begin % g.K);
    W.L = q->win_len;
    W.K = g.K;
    for (uint32_t i = 0; i < W.L; ++i) {
        const uint32_t t = (W.b + i) % g.K;
        W.w[t >> 6] |= 1ull << (t & 63);
    }
    W.full = W.L == g.K;
    return W;
}

// One query alone: bound solves and tail in one call (the per-query method),
// its bounds-done time taken when the bound solves drain.
void run_single(evq_server* sv, const Graph& g, SQuery* q, hipStream_t ws) {
    try {
        q->c.rcap = static_cast<uint32_t*>(stream_alloc((uint64_t)g.V * 4, ws));
        run_query_compact(g, q->algo, internal_id(g, q->source), window_of(g, q), q->c, q->qo, ws);
        q->t_bounds = std::chrono::duration<double, std::milli>(q->qo.bounds_done - sv->t0).count();
    } catch (...) {
        fail_query(q, current_error(), ws);
        q->t_bounds = sv->now();
    }
}

void launch_group(evq_server* sv, std::shared_ptr<const Graph> gp, std::vector<SQuery*> grp) {
    Pool& pool = Pool::get(sv->device);
    if (grp.size() == 1) {
        // one query: the single-query path, as the plain server runs it
        SQuery* q = grp[0];
        pool.submit([sv, gp, q](hipStream_t ws) {
            const Graph& g = *gp;
            UseGuard ug{g, ws};
            run_single(sv, g, q, ws);
            {
                std::lock_guard<std::mutex> lk(sv->mu);
                sv->groups -= 1;
            }
            sv->cv.notify_all();
            complete(sv, q, g, ws);
        });
        return;
    }
    pool.submit([sv, gp, grp](hipStream_t ws) {
        const Graph& g = *gp;
        UseGuard ug{g, ws};
        Pool& pool = Pool::get(sv->device);
        const uint32_t nq = (uint32_t)grp.size();
        const BatchTuning tu = batch_tuning();
        hipEvent_t ev = nullptr;
        bool ok = true;
        Error err{EVQ_OK, ""};
        try {
            std::vector<uint32_t*> rcap(nq), rcup(nq);
            std::vector<Window> wins(nq);
            std::vector<uint32_t> srcs(nq);
            for (uint32_t k = 0; k < nq; ++k) {
                grp[k]->c.rcap = rcap[k] = static_cast<uint32_t*>(stream_alloc((uint64_t)g.V * 4, ws));
                grp[k]->rcup = rcup[k] = static_cast<uint32_t*>(stream_alloc((uint64_t)g.V * 4, ws));
                wins[k] = window_of(g, grp[k]);
                srcs[k] = internal_id(g, grp[k]->source);
            }
            BatchTimes bt;
            batch_bounds(g, grp[0]->algo, wins.data(), srcs.data(), nq, rcap.data(), rcup.data(), tu, ws, bt);
            EVQ_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            EVQ_HIP(hipEventRecord(ev, ws));
            const double tb = sv->now();
            for (SQuery* q : grp) {
                q->qo.st.iters_cap = bt.iters_cap;
                q->qo.st.iters_cup = bt.iters_cup;
                q->t_bounds = tb;
                q->group = nq;
            }
        } catch (...) {
            ok = false;
            err = current_error();
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->groups -= 1;
        }
        sv->cv.notify_all();
        if (!ok) {
            for (SQuery* q : grp) {
                try {
                    stream_free(q->rcup, ws);
                } catch (...) {
                }
                fail_query(q, err, ws);
                complete(sv, q, g, ws);
            }
            if (ev) (void)hipEventDestroy(ev);
            return;
        }
        auto evp = std::shared_ptr<void>(ev, [](void* e) { (void)hipEventDestroy((hipEvent_t)e); });
        for (SQuery* q : grp) {
            pool.submit([sv, gp, q, evp](hipStream_t ts) {
                const Graph& g = *gp;
                UseGuard ug{g, ts};
                try {
                    EVQ_HIP(hipStreamWaitEvent(ts, (hipEvent_t)evp.get(), 0));
                    run_tail_compact(g, q->algo, internal_id(g, q->source), window_of(g, q), q->rcup, q->c, q->qo, ts);
                } catch (...) {
                    fail_query(q, current_error(), ts);
                }
                try {
                    stream_free(q->rcup, ts);
                } catch (...) {
                }
                q->rcup = nullptr;
                complete(sv, q, g, ts);
            });
        }
    });
}

void dispatch_loop(evq_server* sv) {
    (void)hipSetDevice(sv->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        // continuous batching starts a group beside running queries only once a queue has formed
        sv->cv.wait(lk, [sv] {
            return sv->stop || (!sv->queue.empty() && sv->groups < sv->cfg.max_groups &&
                                sv->inflight < sv->cfg.max_inflight &&
                                (sv->cfg.mode == 1 || sv->inflight == 0 || sv->queue.size() >= sv->cfg.queue_hi));
        });
        if (sv->stop) return;
        std::shared_ptr<const Graph> gp = sv->h->get();
        const Graph& g = *gp;
        if (sv->cfg.mode == 1) {
            // plain: one query at a time, in arrival order, on one worker
            SQuery* q = sv->queue.front();
            sv->queue.pop_front();
            admit(sv, q, g);
            q->footprint = 0;
            sv->inflight += 1;
            lk.unlock();
            Pool::get(sv->device).submit([sv, gp, q](hipStream_t ws) {
                const Graph& g = *gp;
                UseGuard ug{g, ws};
                run_single(sv, g, q, ws);
                complete(sv, q, g, ws);
            });
            lk.lock();
            sv->cv.wait(lk, [sv] { return sv->inflight == 0; });
            continue;
        }
        // continuous batching: the oldest query picks the algorithm; others of
        // that algorithm join in arrival order while the footprint fits
        const uint32_t algo = sv->queue.front()->algo;
        std::vector<SQuery*> grp;
        for (auto it = sv->queue.begin(); it != sv->queue.end() && grp.size() < sv->cfg.max_batch;) {
            SQuery* q = *it;
            if (q->algo != algo) {
                ++it;
                continue;
            }
            const uint64_t f = estimate(sv, g, q->algo, std::min<uint32_t>(q->len, g.K));
            const bool fits = sv->inflight_bytes + f <= sv->cfg.mem_budget;
            if (!fits && !(grp.empty() && sv->inflight == 0)) break;
            if (sv->inflight + 1 > sv->cfg.max_inflight) break;
            admit(sv, q, g);
            q->footprint = f;
            sv->inflight_bytes += f;
            sv->inflight += 1;
            grp.push_back(q);
            it = sv->queue.erase(it);
        }
        if (grp.empty()) {
            // the oldest query does not fit yet: wait for a completion
            const uint32_t before = sv->inflight;
            sv->cv.wait(lk, [sv, before] { return sv->stop || sv->inflight < before; });
            continue;
        }
        sv->groups += 1;
        lk.unlock();
        launch_group(sv, gp, std::move(grp));
        lk.lock();
    }
}

}  // namespace
}  // namespace evq

namespace {
evq_status sbad(evq_status c, const char* m) {
    evq::g_last_error = m;
    return c;
}
}  // namespace

extern "C" {

evq_status evq_server_create(evq_graph* h, const evq_server_config* c, evq_server** out) {
    evq::g_last_error.clear();
    if (!h || !out) return sbad(EVQ_EINVAL, "NULL argument");
    *out = nullptr;
    try {
        auto gp = h->get();
        evq::init_mempool(gp->device);
        evq_server_config cfg{};
        if (c) cfg = *c;
        if (cfg.mode > 1) return sbad(EVQ_EINVAL, "mode must be 0 (continuous batching) or 1 (plain)");
        if (cfg.max_batch == 0) cfg.max_batch = 16;  // measured best per-query cost at scale 24
        if (cfg.max_batch > 64) return sbad(EVQ_EINVAL, "max_batch must be <= 64");
        if (cfg.max_inflight == 0) cfg.max_inflight = 256;
        if (cfg.max_groups == 0) cfg.max_groups = 2;
        if (cfg.max_queued == 0) cfg.max_queued = 65536;
        if (cfg.queue_hi == 0) cfg.queue_hi = 4;
        if (cfg.mem_budget == 0) {
            size_t fr = 0, tot = 0;
            EVQ_HIP(hipMemGetInfo(&fr, &tot));
            cfg.mem_budget = fr / 4;
        }
        evq_server* sv = new evq_server();
        sv->h = h;
        sv->cfg = cfg;
        sv->device = gp->device;
        sv->t0 = std::chrono::steady_clock::now();
        sv->dispatcher = std::thread([sv] { evq::dispatch_loop(sv); });
        *out = sv;
        return EVQ_OK;
    } catch (const evq::Error& e) {
        evq::g_last_error = e.msg;
        return e.code;
    } catch (...) {
        return sbad(EVQ_EDEVICE, "server creation failed");
    }
}

evq_status evq_server_submit(evq_server* sv, uint32_t algo, uint32_t source, uint32_t win_len, uint64_t* ticket) {
    evq::g_last_error.clear();
    if (!sv || !ticket) return sbad(EVQ_EINVAL, "NULL argument");
    if (algo > EVQ_VITERBI) return sbad(EVQ_EINVAL, "unknown algorithm");
    auto gp = sv->h->get();
    if (source >= gp->V) return sbad(EVQ_ERANGE, "source vertex out of range");
    if (win_len == 0) return sbad(EVQ_ERANGE, "window length must be >= 1");
    evq::SQuery* q = new (std::nothrow) evq::SQuery();
    if (!q) return sbad(EVQ_ENOMEM, "host allocation failed");
    q->algo = algo;
    q->source = source;
    q->len = win_len;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->stop) {
            delete q;
            return sbad(EVQ_EINVAL, "server is shutting down");
        }
        if (sv->queue.size() >= sv->cfg.max_queued) {
            delete q;
            return sbad(EVQ_EBUSY, "the server's queue is full; submit again after polling");
        }
        q->ticket = sv->next_ticket++;
        q->t_arrival = sv->now();
        sv->queue.push_back(q);
        *ticket = q->ticket;
    }
    sv->cv.notify_all();
    return EVQ_OK;
}

int evq_server_poll(evq_server* sv, evq_completion* out, int cap, int wait_ms) {
    if (!sv || !out || cap <= 0) return 0;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (sv->done.empty() && wait_ms > 0)
        sv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [sv] { return !sv->done.empty(); });
    int n = 0;
    while (n < cap && !sv->done.empty()) {
        evq::SQuery* q = sv->done.front();
        sv->done.pop_front();
        evq_completion& c = out[n++];
        std::memset(&c, 0, sizeof(c));
        c.ticket = q->ticket;
        c.status = q->status;
        c.t_arrival_ms = q->t_arrival;
        c.t_admit_ms = q->t_admit;
        c.t_bounds_ms = q->t_bounds;
        c.t_done_ms = q->t_done;
        c.group_size = q->group;
        evq_result& r = c.result;
        r.algo = q->algo;
        r.source = q->source;
        r.win_begin = (uint32_t)q->win_begin;
        r.win_len = q->win_len;
        if (q->status == EVQ_OK) {
            r.num_vertices = q->V;
            r.n_unstable = q->c.nU;
            r.row_stride = q->c.LG;
            r.d_rcap = q->c.rcap;
            r.d_unstable = q->c.ulist;
            r.d_x = q->c.X;
        }
        c.n_unstable = q->c.nU;
        c.iters_relax = q->qo.st.iters_relax;
        delete q;
    }
    return n;
}

evq_status evq_server_pending(evq_server* sv, uint32_t* queued, uint32_t* inflight) {
    if (!sv) return sbad(EVQ_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (queued) *queued = (uint32_t)sv->queue.size();
    if (inflight) *inflight = sv->inflight;
    return EVQ_OK;
}

evq_status evq_server_destroy(evq_server* sv) {
    if (!sv) return EVQ_OK;
    std::vector<evq::SQuery*> dropped;
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->stop = true;
        for (auto* q : sv->queue) dropped.push_back(q);
        sv->queue.clear();
        sv->cv.notify_all();
    }
    if (sv->dispatcher.joinable()) sv->dispatcher.join();
    {
        std::unique_lock<std::mutex> lk(sv->mu);
        sv->cv_done.wait(lk, [sv] { return sv->inflight == 0; });
        for (auto* q : sv->done) dropped.push_back(q);
        sv->done.clear();
    }
    (void)hipDeviceSynchronize();
    for (auto* q : dropped) {
        try {
            evq::stream_free(q->c.rcap, nullptr);
            evq::stream_free(q->c.ulist, nullptr);
        } catch (...) {
        }
        delete q;
    }
    (void)hipDeviceSynchronize();
    delete sv;
    return EVQ_OK;
}

}  // extern "C"
