// Host side of the top-k LDS / LTDS driver (Alg. 5 and its triangle version).
#pragma once
#include <memory>
#include <utility>
#include <vector>

#include "graph.hpp"

namespace lds {

// Host copy of the adjacency (internal ids) and, for triangles, the triangle
// list with per-vertex incidence lists.
// Allocator whose value-initialisation leaves memory untouched, for host
// copies of large device arrays: their pages are faulted in once, by several
// threads, instead of being zero-filled and then overwritten.
template <class T>
struct NoInit : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInit<U>;
    };
    NoInit() = default;
    template <class U>
    NoInit(const NoInit<U>&) noexcept {}
    template <class U>
    void construct(U* p) noexcept {
        ::new ((void*)p) U;
    }
    template <class U, class... A>
    void construct(U* p, A&&... a) {
        ::new ((void*)p) U(std::forward<A>(a)...);
    }
};
template <class T>
using host_vec = std::vector<T, NoInit<T>>;

struct HostGraph {
    int64_t n = 0;
    std::vector<int64_t> rp;    // n + 1
    host_vec<int32_t> col;      // 2m neighbours
    std::vector<int32_t> orig;  // internal -> caller id
    host_vec<int32_t> tri;      // 3T (triangles only)
    std::vector<int64_t> trp;   // n + 1 offsets into tinc
    host_vec<int32_t> tinc;     // triangle indices incident to each vertex (ascending)
    void load(const Graph& g, int mode, hipStream_t s);
};

// Per-graph host data that does not depend on a query: the adjacency (and
// triangles once a triangle query has run) and the core / tr-core numbers of
// the whole graph.  Built by the first top-k call and kept with the graph.
struct HostCache {
    HostGraph h;
    bool tri_loaded = false;
    std::vector<int32_t> core[2];  // [0] core numbers, [1] tr-core numbers (empty until computed)
};

struct TopkSet {
    int64_t num = 0, den = 1;        // reduced exact density
    std::vector<int32_t> vertices;   // caller ids, ascending
};

struct TopkStats {
    int64_t popped = 0;       // candidates taken from the queue
    int64_t refinements = 0;  // FW + ExtractSG runs on induced subgraphs
    int64_t refine_rounds = 0;  // batched FW launches that carried them
    int64_t flow_splits = 0;  // candidates split by the min cut instead
    int64_t maxflows = 0;     // min-cut computations (IsDensest + IsLDS)
    int64_t pruned = 0;       // vertices removed by the two pruning rules
    // wall-clock ms: host copy of the graph, core numbers, first FW +
    // ExtractSG, pruning, candidate search (verification and refinement)
    double ms_copy = 0, ms_core = 0, ms_fw = 0, ms_prune = 0, ms_search = 0;
};

// Min cuts of large networks use extra host threads (a shared budget).  A
// thread that calls topk_single_thread(true) runs its searches on itself only
// (the serving workers do: their peers use the other cores).
void topk_single_thread(bool on);
bool topk_threads_single();

// reuse_fw: the graph already holds a completed run of `iters` iterations
// for this mode (e.g. from a batched launch); it is used instead of a new run
// prune_out (host, n, by caller id): stop after Pruning (Alg. 3) and write
// the rule that removed each vertex (1 or 2; 0 for the survivors)
void topk_run(Graph& g, int mode, int k, int iters, hipStream_t s, std::vector<TopkSet>& out, TopkStats& st,
              bool reuse_fw = false, int8_t* prune_out = nullptr);
// device bytes a top-k query adds to a resident graph (FW state for `iters`
// iterations, stable-group buffers and their temporaries), an upper estimate
size_t topk_footprint(const Graph& g, int mode, int iters);

}  // namespace lds
