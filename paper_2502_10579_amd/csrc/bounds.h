// Bound solver interface (intersection and union solves of one window) and
// the frontier buffers a query's loops share.
#pragma once

#include <cstddef>

#include "frontier.h"

namespace evq {

// Device buffers of one query's frontier loops.
struct Frontier {
    uint8_t* flags = nullptr;    // next-frontier flags over V vertices (all clear between phases)
    uint32_t* fo = nullptr;      // frontier items (V entries each): running edge offset,
    uint32_t* fd = nullptr;      //   row begin minus that offset,
    uint32_t* fs = nullptr;      //   end of the row's all-present prefix,
    uint32_t* fv = nullptr;      //   the vertex
    uint32_t* fo1 = nullptr;     // the same four arrays for odd iterations (bound solves, appending expansions)
    uint32_t* fd1 = nullptr;
    uint32_t* fs1 = nullptr;
    uint32_t* fv1 = nullptr;
    uint32_t* stamp = nullptr;   // per vertex: epoch of the iteration that last appended it
    uint32_t* epoch = nullptr;   // host: the workspace's epoch counter (one per issued iteration)
    uint32_t append_edges = 0;   // appending expansions up to this many frontier edges (0: never)
    uint32_t append_items = 0;   // ... or up to this many frontier vertices (0: never)
    FrontierCounters* cnt = nullptr;
    unsigned long long* stats = nullptr;  // [0] bound-solve edge visits, [1..] relaxer counters
    unsigned long long* aux = nullptr;    // 128 bytes of scratch counters for the reduction
    int p = 0;                            // parity of the next compaction (continues across phases)
    uint32_t delta = 0;                   // near/far step of the bound solves (0: off)
    uint32_t heavy = 0;                   // with delta: gate only vertices with this many edges (0: all)
    uint32_t bdelta = 0;                  // bucket width of the SSSP intersection solve (0: off)
    uint64_t items = 0;                   // frontier items processed so far (published counts)
};

// Near/far step for a query: EVQ_DELTA overrides, else a per-algorithm default.
uint32_t choose_delta(uint32_t algo);
// Edge count from which vertices are gated: EVQ_HEAVY overrides, else a
// per-algorithm default (0: every vertex is gated).
uint32_t choose_heavy(uint32_t algo);


// Bucket width of the intersection solve of a query of algo on g (0: off).
uint32_t choose_bucket_width(uint32_t algo, const Graph& g);
// g's rows ordered for the bucket width, built on s on first use (later users
// on other streams wait for it); null when it cannot be had (a call that must
// not allocate, or all kWeightOrders slots hold other widths).
const WeightOrder* weight_order_ready(const Graph& g, uint32_t width, hipStream_t s);

Frontier make_frontier(const Graph& g, Workspace& ws, hipStream_t s);

// Pull step of the full-window intersection solve: an expansion whose
// frontier holds at least this share of the all-present edges (fixed point,
// 1024 = all of them) takes every vertex's best candidate over its
// all-present in-edges instead.  EVQ_PULL_FRAC (a fraction; above 1 turns the
// pull step off) overrides the default.  Returns kNone when it is off.
uint32_t pull_frac();
// The graph's reverse CSR if it is there or this is the second call asking
// for it (then built on s); later callers' streams wait for it.  False: not
// built yet, push only.
bool reverse_ready(const Graph& g, hipStream_t s);

// R := values on the window's intersection graph.  Returns the iteration count.
uint64_t solve_cap(const Graph& g, uint32_t algo, const Window& W, uint32_t source, uint32_t* R, Frontier& f,
                   hipStream_t s, bool stats);

// R (holding the intersection values) := values on the window's union graph.
uint64_t solve_cup(const Graph& g, uint32_t algo, const Window& W, uint32_t* R, Frontier& f, hipStream_t s,
                   bool stats);

}  // namespace evq
