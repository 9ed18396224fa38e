// Minimum cuts of large vertex networks on the device (gflow.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace lds {

// The edge case of IsDensest entirely on the device: Goldberg's vertex network
// over k nodes (source -> v with capacity q (deg v + 2 loops v), scaled by D
// and warm-started from the split when warm, v -> sink 2p, each pair an
// undirected arc of capacity q) is built from the pairs, the flow runs, and
// inX receives the maximal source side of a minimum cut.  Returns the maximum
// of q (|E(X)| + loops(X)) - p |X| (as the host version does).
int64_t edge_mincut_device(int64_t k, const std::vector<int32_t>& pairs, const std::vector<int64_t>& loops, int64_t p,
                           int64_t q, bool warm, int64_t D, const std::vector<uint32_t>* split, std::vector<char>& inX,
                           hipStream_t stream);

}  // namespace lds
