// Maximum preflow of a large network on the device (gflow.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace lds {

// The network in CSR order (arcs of a node contiguous, rev[e] the paired
// arc), residual capacities in cap; ex holds every node's excess with the
// source arcs already saturated (ex[s] = 0, ex[t] = the flow already at t).
// On return cap holds the residual capacities of a maximum preflow (so the
// minimum cuts follow from it as after any maximum flow) and the result is
// the flow into t.  Synchronises the stream.
int64_t maxflow_device(int64_t N, const std::vector<int64_t>& first, const std::vector<int32_t>& to,
                       std::vector<int64_t>& cap, const std::vector<int64_t>& rev, int64_t s, int64_t t,
                       const std::vector<int64_t>& ex, hipStream_t stream);

}  // namespace lds
