// Batched queries: shared bound solves (one query per lane) and the worker
// pool that runs every query's reduction and relaxation concurrently.
#pragma once

#include <condition_variable>
#include <deque>
#include <functional>
#include <mutex>

#include "bounds.h"

namespace evq {

struct BatchTuning {
    uint32_t lanes = 1;     // 1: shared bound solves; 2: one bound solve per query
    uint32_t chunk = 8;     // edges per wave task of the shared solves
    uint32_t blocks = 2048; // workgroups per expansion launch
    uint32_t group = 64;    // queries per shared solve
};

struct BatchTimes {
    uint64_t iters_cap = 0, iters_cup = 0;
};

BatchTuning batch_tuning();
void set_batch_tuning(const BatchTuning& t);

// Bound solves of 1..64 queries of one algorithm together; writes query i's
// intersection bound to rcap_cols[i] and union bound to rcup_cols[i].
void batch_bounds(const Graph& g, uint32_t algo, const Window* wins, const uint32_t* sources, uint32_t nq,
                  uint32_t* const* rcap_cols, uint32_t* const* rcup_cols, const BatchTuning& tu, hipStream_t s,
                  BatchTimes& bt);

// Host threads, each driving its own non-blocking stream (default priority)
// on one device; EVQ_BATCH_WORKERS of them (default 4).  Jobs may submit
// further jobs.  The pool lives as long as the process; each worker keeps its
// own query workspace and host slots.
class Pool {
  public:
    using Job = std::function<void(hipStream_t)>;
    static Pool& get(int device);
    void submit(Job j);
    const std::vector<hipStream_t>& streams() const { return st_; }

  private:
    Pool(int device, uint32_t n);
    void loop(uint32_t i);
    int device_;
    std::vector<hipStream_t> st_;
    std::mutex mu_;
    std::condition_variable cv_;
    std::deque<Job> q_;
};

struct BatchQuery {
    uint32_t algo, source;
    Window W;
};

// n queries into n compact results (caller arrays); stats: nullptr or n
// entries.  The caller's stream s waits for all of the work.  On failure
// every result allocated so far is released and the error rethrown.
void run_batch(const Graph& g, const BatchQuery* q, uint32_t n, Compact* out, evq_query_stats* stats,
               hipStream_t s);

// Tries the execution choices on the given queries and installs the fastest.
BatchTuning autotune_batch(const Graph& g, const BatchQuery* q, uint32_t n, hipStream_t s, double* best_ms);

}  // namespace evq
