// The graph handle behind the C ABI.  It holds the current version of the
// versioned graph; every call takes a reference to the version it starts on,
// so an append never waits for running queries; a version is released once
// its last user has returned, ordered after the work its users queued.
#pragma once

#include <memory>
#include <mutex>

#include "evq_internal.h"

namespace evq {

inline void release_graph(Graph* g) { retire_graph(g); }

}  // namespace evq

struct evq_graph {
    mutable std::mutex mu;
    std::shared_ptr<const evq::Graph> cur;
    std::mutex append_mu;  // one append at a time
    std::shared_ptr<const evq::Graph> get() const {
        std::lock_guard<std::mutex> lk(mu);
        return cur;
    }
};
