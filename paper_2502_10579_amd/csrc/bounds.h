// Bound solver interface (intersection and union solves of one window).
#pragma once

#include <cstddef>

#include "frontier.h"

namespace evq {

struct SolveArgs {
    const uint32_t* row_ptr;
    const uint32_t* row_split;
    const uint32_t* col;
    const uint32_t* wgt;
    const uint64_t* mask;
    uint32_t* R;
    uint32_t* stamps;
    uint32_t* list[2];
    uint64_t* big[2];
    FrontierCounters* cnt;
    unsigned long long* stats;
};

// Device buffers of one query's frontier loops; stamps are cleared once.
struct SolveWorkspace {
    uint32_t* stamps = nullptr;
    uint32_t* list[2] = {nullptr, nullptr};
    uint64_t* big[2] = {nullptr, nullptr};
    uint64_t cap_big = 0;
    FrontierCounters* cnt = nullptr;
    unsigned long long* stats = nullptr;  // [0] bound-solve edge visits, [1..] relaxer counters
};

inline uint32_t* dev_small_cnt(FrontierCounters* c, int p) {
    return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(c) + offsetof(FrontierCounters, small)) + p;
}
inline uint32_t* dev_big_cnt(FrontierCounters* c, int p) {
    return reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(c) + offsetof(FrontierCounters, big)) + p;
}

SolveWorkspace make_solve_workspace(const Graph& g, Arena& ar, hipStream_t s);

// R := values on the window's intersection graph.  Returns the iteration count.
uint64_t solve_cap(const Graph& g, uint32_t algo, const Window& W, uint32_t source, uint32_t* R,
                   const SolveWorkspace& w, uint32_t& stamp, Mailbox& mb, hipStream_t s, bool stats);

// R (holding the intersection values) := values on the window's union graph.
uint64_t solve_cup(const Graph& g, uint32_t algo, const Window& W, uint32_t* R, const SolveWorkspace& w,
                   uint32_t& stamp, Mailbox& mb, hipStream_t s, bool stats);

}  // namespace evq
