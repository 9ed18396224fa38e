// Definitions behind the opaque handles of the C ABI.
#pragma once
#include <mutex>

#include "lds.h"
#include "graph.hpp"

struct lds_graph_s {
    lds::Graph g;
    std::mutex mu;  // serialises calls on one graph (the server's threads and the caller's)
};
