// Bound solver interface (intersection and union solves of one window) and
// the frontier buffers a query's loops share.
#pragma once

#include <cstddef>

#include "frontier.h"

namespace evq {

// Device buffers of one query's frontier loops.
struct Frontier {
    uint32_t* bitmap = nullptr;  // next-frontier bits over V vertices (all clear between phases)
    uint32_t* fv = nullptr;      // frontier vertices (V entries)
    uint32_t* fo = nullptr;      // their running edge offsets (V entries)
    FrontierCounters* cnt = nullptr;
    unsigned long long* stats = nullptr;  // [0] bound-solve edge visits, [1..] relaxer counters
    int p = 0;                            // parity of the next compaction (continues across phases)
};


Frontier make_frontier(const Graph& g, Arena& ar, hipStream_t s);

// R := values on the window's intersection graph.  Returns the iteration count.
uint64_t solve_cap(const Graph& g, uint32_t algo, const Window& W, uint32_t source, uint32_t* R, Frontier& f,
                   hipStream_t s, bool stats);

// R (holding the intersection values) := values on the window's union graph.
uint64_t solve_cup(const Graph& g, uint32_t algo, const Window& W, uint32_t* R, Frontier& f, hipStream_t s,
                   bool stats);

}  // namespace evq
