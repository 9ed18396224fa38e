// Batched Frank-Wolfe runs over many graphs (batch.hip) and the autotuner
// that picks their launch shape (tune.cpp).
#pragma once
#include <string>
#include <vector>

#include "graph.hpp"

namespace lds {

// Launch shape of the batched kernel.
struct BatchTune {
    int threads = 1024;              // workgroup size: 256, 512 or 1024
    int wg_per_cu = 1;               // persistent workgroups per compute unit
    int lds_vertices = 8192;         // graphs with at most this many vertices keep their keys in LDS
    int64_t max_kernel_cost = 1ll << 27;  // (slots + vertices) * iters above which a graph runs on its own
    int longest_first = 1;           // order the work queue by cost, largest first
};

struct Batch {
    std::vector<Graph*> gs;
    std::vector<int> modes, iters;
    std::vector<float*> r_out;       // per graph, device, by caller id (may be empty)
    bool want_gap = false;
    bool capture = true;             // replay a captured hipGraph (else launch directly)
    BatchTune tune;
    std::vector<int> kernel_items;   // indices into gs, in queue order
    std::vector<int> plain_items;    // graphs run one by one
    std::vector<int64_t> sum_off;    // per kernel item: offset of its gap sums
    DBuf<uint8_t> items;             // device item table
    DBuf<int32_t> queue;             // work-queue counter
    DBuf<uint64_t> sums;             // exact gap sums of the kernel items
    int32_t kmax = 0;
    unsigned grid = 0;
    size_t lds_bytes = 0;
    hipStream_t cap = nullptr;       // private stream used for capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};  // around the graph launch of the last run
    int64_t runs = 0;
    ~Batch();
};

int64_t batch_cost(const Graph& g, int mode, int iters);
void batch_build(Batch& b, hipStream_t s);  // sizes buffers, builds the item table, captures the hipGraph
void batch_run(Batch& b, hipStream_t s);    // per-graph runs of large graphs, then the captured launch

}  // namespace lds
