// Device scoping of IsLDS / IsLTDS (islds.hip), used by the top-k driver.
#pragma once
#include <vector>

#include "graph.hpp"

namespace lds {

// device state of one top-k run: the bounds of every vertex and the
// per-vertex / per-triangle scratch of the search (cleared after each call)
struct BandScope {
    int mode = 2;
    int64_t n = 0, T = 0;
    DBuf<int64_t> lon, lod, hin, hid;  // lower / upper bound numerator and denominator, internal order
    DBuf<uint8_t> flag;                // above / band / below rho
    DBuf<int32_t> inU, loops, loc;     // region membership, self-loops, local index (-1 outside)
    DBuf<int32_t> U, front, next, S, ctr;
    DBuf<uint32_t> tvis;               // triangles: visited
    DBuf<int32_t> tlist, plist;        // triangles visited / kept as patterns
};

struct ScopeOut {
    bool need_flow = false;      // a vertex above the band touches the region
    std::vector<int32_t> U;      // region (internal ids), S first; filled when need_flow
    std::vector<int32_t> pat;    // edges: pairs of local ids (i < j); triangles: triples, -1 for members above
    std::vector<int64_t> loops;  // edges: self-loops per local id
};

void scope_init(Graph& g, int mode, const int64_t* lon, const int64_t* lod, const int64_t* hin, const int64_t* hid,
                BandScope& b, hipStream_t s);
// false: S is rejected at once (a vertex of S outside the band, or a
// neighbour above it); true: o describes the region searched from S
bool scope_band(Graph& g, BandScope& b, const std::vector<int32_t>& S, int64_t rn, int64_t rd, ScopeOut& o,
                hipStream_t s);

// Pruning (Alg. 3) with the bounds of b (internal order): rule 1 once, then
// rule 2 with the core (tr-core) numbers of the residual graph until nothing
// changes, all on the device.  alive[u] = 0 for pruned vertices; rule[u] = the
// rule that removed u (1 or 2), 0 for the survivors.
void prune_device(Graph& g, int mode, const BandScope& b, uint8_t* alive, uint8_t* rule, hipStream_t s);

}  // namespace lds
