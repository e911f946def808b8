// Access-pattern ceiling of the bound solves' expansion (measurement only).
#pragma once

#include "evq_internal.h"

namespace evq {

// Edges per second of `launches` timed passes (after one untimed pass) of a
// kernel that streams every edge's column and weight in CSR order and gathers
// its destination's 4-byte value, with the expansion's conditional atomicMin
// and flag store behind a comparison that never succeeds.
double gather_ceiling(const Graph& g, uint32_t launches, hipStream_t s);

}  // namespace evq
