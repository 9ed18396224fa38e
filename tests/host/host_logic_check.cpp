// Host-only checks of the top-k driver's exact building blocks, compiled from
// the library's own source with its device entry points stubbed out (nothing
// here touches a GPU).  Each block is compared with a plain definition on
// small random inputs:
//   * minimum cuts (edge network, pattern network, both warm-started from
//     arbitrary splits): the maximum of q*|P(X)| - p*|X| and the union of all
//     maximisers, by enumeration of every X;
//   * connectivity of induced subgraphs (union-find over host threads) by a
//     breadth-first search.
// (Core and tr-core numbers run on the device; their parity is a GPU test.)
// The battery runs twice: with the sequential push-relabel and with every
// vertex network through the parallel one (pflow.hpp; pattern networks always
// take the sequential one); larger random networks then compare the two
// directly.
// Prints "ok" and exits 0 when every case agrees.
#include "../../paper_2504_10937_amd/csrc/topk.cpp"

#include <cstdio>
#include <cstdlib>
#include <random>

namespace lds {
void* dev_alloc(size_t, hipStream_t) { return nullptr; }
void dev_free(void*) {}
Graph::~Graph() {}
void build_graph(Graph&, int64_t, int64_t, const int32_t*, const int32_t*, bool, bool, hipStream_t) {}
void list_triangles(Graph&, hipStream_t) {}
void vertex_triangle_lists(const Graph&, int64_t*, int32_t*, hipStream_t) {}
int64_t edge_mincut_device(int64_t, const std::vector<int32_t>&, const std::vector<int64_t>&, int64_t, int64_t, bool,
                           int64_t, const std::vector<uint32_t>*, std::vector<char>&, hipStream_t) {
    std::abort();  // main() keeps every network on the host
}
void sg_stable_groups(Graph&, int, hipStream_t) {}
void gather_split(const Graph&, int, const int64_t*, int64_t, uint32_t*, hipStream_t) {
    std::abort();  // the checks here pass splits to the min cuts directly
}
void fw_run(Graph&, int, int, bool, hipStream_t) {}
void core_numbers_gpu(Graph&, int, const uint8_t*, int32_t*, hipStream_t) {}
Batch::~Batch() {}
void batch_build(Batch&, hipStream_t) {}
void batch_run(Batch&, hipStream_t) {}
void scope_init(Graph&, int, const int64_t*, const int64_t*, const int64_t*, const int64_t*, BandScope&, hipStream_t) {}
void prune_device(Graph&, int, const BandScope&, uint8_t*, uint8_t*, hipStream_t) {}
bool scope_band(Graph&, BandScope&, const std::vector<int32_t>&, int64_t, int64_t, ScopeOut&, hipStream_t) {
    return false;
}
}  // namespace lds

using namespace lds;

// value and union of maximisers of q * (#patterns inside X + loops(X)) - p * |X|
static int64_t enumerate(int64_t k, int h, const std::vector<int32_t>& pat, const std::vector<int64_t>& loops,
                         int64_t p, int64_t q, std::vector<char>& X) {
    auto value = [&](uint32_t m) {
        int64_t cnt = 0;
        for (size_t i = 0; i < pat.size() / h; ++i) {
            bool in = true;
            for (int j = 0; j < h; ++j) {
                const int32_t v = pat[h * i + j];
                if (v >= 0 && !((m >> v) & 1)) in = false;
            }
            cnt += in;
        }
        if (!loops.empty())
            for (int64_t v = 0; v < k; ++v)
                if ((m >> v) & 1) cnt += loops[v];
        return q * cnt - p * (int64_t)__builtin_popcount(m);
    };
    int64_t best = INT64_MIN;
    for (uint32_t m = 0; m < (1u << k); ++m) best = std::max(best, value(m));
    uint32_t un = 0;
    for (uint32_t m = 0; m < (1u << k); ++m)
        if (value(m) == best) un |= m;
    X.assign(k, 0);
    for (int64_t v = 0; v < k; ++v) X[v] = (un >> v) & 1;
    return best;
}

// every case of the battery, with the current choice of sequential / parallel min cut
static int battery(int& cases) {
    std::mt19937_64 rng(12345);
    int bad = 0;
    for (int it = 0; it < 1500; ++it) {
        const int k = 2 + (int)(rng() % 10);
        const double pe = 0.2 + (double)(rng() % 70) / 100.0;
        std::vector<int32_t> pairs, tris;
        std::vector<int64_t> loops(k, 0);
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b)
                if ((double)(rng() % 1000) < pe * 1000) {
                    pairs.push_back(a);
                    pairs.push_back(b);
                }
        for (int a = 0; a < k; ++a) loops[a] = (rng() % 3 == 0) ? (int64_t)(rng() % 3) : 0;
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b)
                for (int c = b + 1; c < k; ++c)
                    if ((double)(rng() % 1000) < pe * 400) {
                        tris.push_back(a);
                        tris.push_back(b);
                        tris.push_back((rng() % 4) ? c : -1);  // some truncated patterns
                    }
        const int64_t p = 1 + (int64_t)(rng() % 20), q = 1 + (int64_t)(rng() % 10);
        std::vector<char> X, Y;
        // edge network, with and without self-loops
        for (int withl = 0; withl < 2; ++withl) {
            const std::vector<int64_t> L = withl ? loops : std::vector<int64_t>{};
            ++cases;
            if (max_excess_edges(k, pairs, L, p, q, X) != enumerate(k, 2, pairs, L, p, q, Y) || X != Y) ++bad;
        }
        // edge network warm-started from an arbitrary split
        {
            const int64_t D = 2 + (int64_t)(rng() % 50);
            std::vector<uint32_t> sp(pairs.size() / 2);
            for (auto& a : sp) a = (uint32_t)(rng() % (uint64_t)(D + 1));
            ++cases;
            if (max_excess_edges(k, pairs, {}, p, q, X, &sp, D) != enumerate(k, 2, pairs, {}, p, q, Y) || X != Y)
                ++bad;
        }
        // pattern network (truncated patterns allowed), cold
        ++cases;
        if (max_excess(k, 3, tris, p, q, X) != enumerate(k, 3, tris, {}, p, q, Y) || X != Y) ++bad;
        // pattern network warm-started from arbitrary shares (full patterns)
        {
            std::vector<int32_t> full;
            for (size_t i = 0; i + 2 < tris.size(); i += 3)
                if (tris[i + 2] >= 0) full.insert(full.end(), tris.begin() + i, tris.begin() + i + 3);
            const int64_t D = 3 + (int64_t)(rng() % 40);
            std::vector<uint32_t> sp;
            for (size_t i = 0; i < full.size(); i += 3) {
                const int64_t a = (int64_t)(rng() % (uint64_t)(D + 1)), b = (int64_t)(rng() % (uint64_t)(D - a + 1));
                sp.push_back((uint32_t)a);
                sp.push_back((uint32_t)b);
                sp.push_back((uint32_t)(D - a - b));
            }
            ++cases;
            if (max_excess(k, 3, full, p, q, X, &sp, D) != enumerate(k, 3, full, {}, p, q, Y) || X != Y) ++bad;
        }
    }
    return bad;
}

// larger random networks: the parallel push-relabel against the sequential
// one (value and maximal maximiser), cold and warm-started
static int parallel_vs_sequential(int& cases) {
    std::mt19937_64 rng(777);
    int bad = 0;
    for (int it = 0; it < 40; ++it) {
        const int64_t k = 200 + (int64_t)(rng() % 3000);
        const int64_t m = k * (2 + (int64_t)(rng() % 6));
        std::vector<int32_t> pairs;
        for (int64_t e = 0; e < m; ++e) {
            const int32_t a = (int32_t)(rng() % k), b = (int32_t)(rng() % k);
            if (a == b) continue;
            pairs.push_back(std::min(a, b));
            pairs.push_back(std::max(a, b));
        }
        const int64_t ne = (int64_t)pairs.size() / 2;
        // density-like parameters around the graph's own density
        const int64_t q = k, p = ne + (int64_t)(rng() % 7) - 3;
        const int64_t D = 6 + (int64_t)(rng() % 100);
        std::vector<uint32_t> sp(ne);
        for (auto& x : sp) x = (uint32_t)(rng() % (uint64_t)(D + 1));
        for (int warm = 0; warm < 2; ++warm) {
            std::vector<char> X, Y;
            g_flow_parallel_min = 1 << 30;
            const int64_t a = max_excess_edges(k, pairs, {}, p, q, X, warm ? &sp : nullptr, D);
            g_flow_parallel_min = 0;
            const int64_t b = max_excess_edges(k, pairs, {}, p, q, Y, warm ? &sp : nullptr, D);
            ++cases;
            if (a != b || X != Y) ++bad;
        }
    }
    return bad;
}

// connectivity of induced subgraphs over host threads against a plain BFS,
// on random sparse graphs (some split into many pieces) and random subsets
static int connectivity(int& cases) {
    std::mt19937_64 rng(4242);
    int bad = 0;
    for (int it = 0; it < 60; ++it) {
        const int64_t n = 5000 + (int64_t)(rng() % 30000);
        const int64_t m = n * (1 + (int64_t)(rng() % 3)) / 2 + (int64_t)(rng() % 8) * n / 8;
        std::vector<std::vector<int32_t>> adj(n);
        std::vector<int32_t> vs;
        const int keep = (it % 3 == 0) ? 100 : 60 + (int)(rng() % 40);  // percent of the vertices
        for (int32_t v = 0; v < n; ++v)
            if ((int)(rng() % 100) < keep) vs.push_back(v);
        for (int64_t e = 0; e < m; ++e) {
            const int32_t a = (int32_t)(rng() % n), b = (int32_t)(rng() % n);
            if (a == b) continue;
            adj[a].push_back(b);
            adj[b].push_back(a);
        }
        if (it % 2 == 0)  // a random spanning tree of G[vs]: connected
            for (size_t i = 1; i < vs.size(); ++i) {
                const int32_t a = vs[i], b = vs[rng() % i];
                adj[a].push_back(b);
                adj[b].push_back(a);
            }
        HostGraph h;
        h.n = n;
        h.rp.assign(n + 1, 0);
        for (int64_t v = 0; v < n; ++v) h.rp[v + 1] = h.rp[v] + (int64_t)adj[v].size();
        h.col.resize(h.rp[n]);
        for (int64_t v = 0; v < n; ++v) std::copy(adj[v].begin(), adj[v].end(), h.col.begin() + h.rp[v]);
        std::vector<int32_t> loc(n, -1);
        // BFS over G[vs]
        std::vector<char> in(n, 0), seen(n, 0);
        for (int32_t v : vs) in[v] = 1;
        std::vector<int32_t> q{vs.empty() ? 0 : vs[0]};
        if (!vs.empty()) seen[vs[0]] = 1;
        for (size_t i = 0; i < q.size() && !vs.empty(); ++i)
            for (int32_t w : adj[q[i]])
                if (in[w] && !seen[w]) {
                    seen[w] = 1;
                    q.push_back(w);
                }
        const bool want = vs.empty() || q.size() == vs.size();
        if (want != (it % 2 == 0)) ++bad;  // planted trees connect, the sparse rest does not
        ++cases;
        if (induced_connected(h, loc, vs) != want) ++bad;
        for (int32_t x : loc)
            if (x != -1) {
                ++bad;
                break;
            }
    }
    return bad;
}

int main() {
    setenv("LDS_FLOW_GPU_MIN", "9223372036854775807", 1);  // no device here: host min cuts only
    int cases = 0, bad = 0;
    g_flow_threads = 4;
    g_flow_parallel_min = 1 << 30;  // sequential push-relabel
    bad += battery(cases);
    g_flow_parallel_min = 0;  // every vertex network through the parallel one
    bad += battery(cases);
    bad += parallel_vs_sequential(cases);
    bad += connectivity(cases);
    std::printf("%s: %d of %d cases disagree\n", bad ? "FAIL" : "ok", bad, cases);
    return bad ? 1 : 0;
}
