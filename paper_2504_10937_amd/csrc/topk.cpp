// Top-k LDS (Problem LDS, Section 3) and LTDS (Problem LTDS, Section 6): the
// LDScvx driver (Alg. 5) and its triangle version, around the device
// Frank-Wolfe (Alg. 1 / Alg. 6) and stable-group passes (Alg. 2), with every
// decision taken on the host in exact integer arithmetic.
//
//  * Bounds on compact numbers: core(u)/2 <= phi(u) <= core(u) for edges and
//    tr-core(u)/3 <= phi(u) <= tr-core(u) for triangles (Section 4.3 and its
//    triangle counterpart), tightened by the stable groups of one FW +
//    ExtractSG run on the WHOLE graph (Lemma phi-bounds / tr-phi-bounds), so
//    that they bound phi_G of every vertex; they are the only bounds that the
//    verification uses.
//  * Pruning (Alg. 3): rule 1 (Cor. uv-prune) once, then rule 2 (Lemma
//    uu-prune) with core / tr-core numbers of the residual graph until
//    nothing changes.  Core numbers come from level-synchronous peeling on
//    the device (cores.hip).
//  * Candidates are taken in non-increasing order of an upper bound on the
//    density of any LDS inside them (a vertex of an LDS S has phi = density
//    of S).  A disconnected candidate is split into its components.
//  * IsDensest: one min cut at lambda = density(G[S]) on G[S].
//  * IsLDS (Alg. 4) / IsLTDS (Alg. 7 with ExtMaximal, Alg. 8) on G.
//  * A candidate that is not self-densest is refined by FW + ExtractSG on
//    G[S] (Alg. 5 replaces G' by G[S]); if that does not split it, the
//    maximal maximiser of the min cut (the vertices with phi_{G[S]} at least
//    density(G[S])) splits it.  An LDS of G inside S is an LDS of G[S], and
//    both splits keep vertices of equal phi_{G[S]} together, so every LDS
//    stays whole inside one candidate; a self-densest connected candidate
//    that contains an LDS is that LDS.
//  * The search ends when the best remaining upper bound is below the k-th
//    density found; results are sorted by (density desc, smallest caller id).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <queue>

#include "batch.hpp"
#include "gflow.hpp"
#include "pflow.hpp"
#include "islds.hpp"
#include "topk.hpp"

#include <mutex>

namespace lds {

namespace {

typedef __int128 i128;

struct Frac {
    int64_t n = 0, d = 1;  // n / d with d > 0
};
inline bool lt(const Frac& a, const Frac& b) { return (i128)a.n * b.d < (i128)b.n * a.d; }
inline int64_t gcd64(int64_t a, int64_t b) {
    while (b) {
        const int64_t t = a % b;
        a = b;
        b = t;
    }
    return a < 0 ? -a : a;
}
inline Frac reduce(int64_t n, int64_t d) {
    const int64_t g = gcd64(n, d);
    return g ? Frac{n / g, d / g} : Frac{0, 1};
}

// ------------------------------------------------------------ max flow
// Networks with at least this many nodes (2^19: below it the sequential one is
// fast enough, and serving runs several searches at once) use the parallel push-relabel
// (pflow.hpp) on up to 16 host threads; LDS_FLOW_THREADS overrides the
// thread count (1: always sequential) and LDS_FLOW_PARALLEL_MIN the size.
int g_flow_threads = 0;            // 0: not read yet
int64_t g_flow_parallel_min = -1;  // -1: not read yet
int flow_threads() {
    if (g_flow_threads == 0) {
        const char* e = std::getenv("LDS_FLOW_THREADS");
        const unsigned hc = std::thread::hardware_concurrency();
        g_flow_threads = (e && *e) ? std::max(1, std::atoi(e)) : (int)std::min(16u, std::max(1u, hc));
    }
    return g_flow_threads;
}
int64_t flow_parallel_min_nodes() {
    if (g_flow_parallel_min < 0) {
        const char* e = std::getenv("LDS_FLOW_PARALLEL_MIN");
        g_flow_parallel_min = (e && *e) ? (int64_t)std::atoll(e) : (int64_t)1 << 19;
    }
    return g_flow_parallel_min;
}
// Vertex networks with at least this many nodes (2^17) are built and cut on
// the device (gflow.hip) instead; LDS_FLOW_GPU_MIN overrides it, read at
// every call.  The stream is the one of the search that needs the cut.
int64_t flow_gpu_min_nodes() {
    const char* e = std::getenv("LDS_FLOW_GPU_MIN");
    return (e && *e) ? (int64_t)std::atoll(e) : (int64_t)1 << 17;
}
thread_local hipStream_t g_flow_stream = nullptr;

// Host threads for the large min cuts are shared by every top-k search in the
// process (the serving workers run several at once): a search takes what is
// free of the flow_threads() budget and runs sequentially when fewer than two
// threads are free, so the threads in use never exceed the budget.
std::atomic<int> g_threads_busy{0};
struct ThreadGrant {
    int n = 1;
    explicit ThreadGrant(int want) {
        if (topk_threads_single()) return;  // a serving worker: its peers use the other cores
        const int cap = flow_threads();
        int cur = g_threads_busy.load();
        for (;;) {
            const int take = std::min(want, cap - cur);
            if (take < 2) return;  // n = 1: sequential
            if (g_threads_busy.compare_exchange_weak(cur, cur + take)) {
                n = take;
                return;
            }
        }
    }
    ~ThreadGrant() {
        if (n > 1) g_threads_busy.fetch_sub(n);
    }
};

// f(i0, i1) over [0, n) split into one contiguous range per granted thread
template <class F>
void par_for(int64_t n, F f) {
    ThreadGrant grant(flow_threads());
    const int T = grant.n;
    if (T <= 1 || n < 4096) {
        f((int64_t)0, n);
        return;
    }
    std::vector<std::thread> pool;
    for (int k = 1; k < T; ++k) pool.emplace_back([&, k] { f(n * k / T, n * (k + 1) / T); });
    f((int64_t)0, n / T);
    for (auto& th : pool) th.join();
}

// f(u0, u1) over the rows [0, n) of a CSR with offsets rp, one contiguous
// range of about equal slot count per granted thread (rows are in degree
// order, so equal row counts would give the first thread every hub)
template <class F>
void par_for_rows(const std::vector<int64_t>& rp, int64_t n, F f) {
    ThreadGrant grant(flow_threads());
    const int T = grant.n;
    if (T <= 1 || n < 4096) {
        f((int64_t)0, n);
        return;
    }
    std::vector<int64_t> cut(T + 1, n);
    cut[0] = 0;
    for (int k = 1; k < T; ++k) {
        const int64_t want = rp[n] / T * k;
        cut[k] = std::max(cut[k - 1], (int64_t)(std::lower_bound(rp.begin(), rp.begin() + n + 1, want) - rp.begin()));
        cut[k] = std::min(cut[k], n);
    }
    std::vector<std::thread> pool;
    for (int k = 1; k < T; ++k) pool.emplace_back([&, k] { f(cut[k], cut[k + 1]); });
    f(cut[0], cut[1]);
    for (auto& th : pool) th.join();
}

// Network with arcs in CSR order (arcs of a node are contiguous, each with
// the index of its reverse arc).  Arcs are collected with arc() and laid out
// by finalize().
struct Flow {
    int64_t N;
    // the synchronous parallel push-relabel (pflow.hpp) is used for large
    // vertex networks built on the host; on pattern networks, whose
    // pattern-to-member arcs are unbounded, it ran several times slower than
    // the sequential one
    bool allow_parallel = true;
    std::vector<int64_t> pa, pb, pc, pd;  // pending arcs: tail, head, capacity, reverse capacity
    std::vector<int64_t> first, cap, rev;
    std::vector<int32_t> to;
    explicit Flow(int64_t nodes) : N(nodes) {}
    void reserve(size_t arcs) {
        pa.reserve(arcs);
        pb.reserve(arcs);
        pc.reserve(arcs);
        pd.reserve(arcs);
    }
    // arc a -> b of capacity c, paired with b -> a of capacity c_back
    void arc(int64_t a, int64_t b, int64_t c, int64_t c_back = 0) {
        pa.push_back(a);
        pb.push_back(b);
        pc.push_back(c);
        pd.push_back(c_back);
    }
    // Direct construction (no pending list): arcs[v] = the number of arc
    // ends at node v (each arc pair counts once at both of its nodes); then
    // add() places every pair.
    std::vector<int64_t> fillp;
    bool direct = false;
    void begin(const std::vector<int64_t>& arcs) {
        direct = true;
        first.assign(N + 1, 0);
        for (int64_t v = 0; v < N; ++v) first[v + 1] = first[v] + arcs[v];
        fillp.assign(first.begin(), first.end() - 1);
        to.resize(first[N]);
        cap.resize(first[N]);
        rev.resize(first[N]);
    }
    void add(int64_t a, int64_t b, int64_t c, int64_t c_back = 0) {
        const int64_t x = fillp[a]++, y = fillp[b]++;
        to[x] = (int32_t)b;
        cap[x] = c;
        rev[x] = y;
        to[y] = (int32_t)a;
        cap[y] = c_back;
        rev[y] = x;
    }
    // add() from several threads at once: arc positions by atomic increments
    // (the order of a node's arcs then varies; the flow value and the minimum
    // cuts do not depend on it)
    void add_atomic(int64_t a, int64_t b, int64_t c, int64_t c_back) {
        const int64_t x = __atomic_fetch_add(&fillp[a], 1, __ATOMIC_RELAXED);
        const int64_t y = __atomic_fetch_add(&fillp[b], 1, __ATOMIC_RELAXED);
        to[x] = (int32_t)b;
        cap[x] = c;
        rev[x] = y;
        to[y] = (int32_t)a;
        cap[y] = c_back;
        rev[y] = x;
    }
    void finalize() {
        if (direct) {
            std::vector<int64_t>().swap(fillp);
            return;
        }
        const size_t m = pa.size();
        first.assign(N + 1, 0);
        for (size_t i = 0; i < m; ++i) {
            first[pa[i] + 1]++;
            first[pb[i] + 1]++;
        }
        for (int64_t v = 0; v < N; ++v) first[v + 1] += first[v];
        std::vector<int64_t> fill(first.begin(), first.end() - 1);
        to.resize(2 * m);
        cap.resize(2 * m);
        rev.resize(2 * m);
        for (size_t i = 0; i < m; ++i) {
            const int64_t x = fill[pa[i]]++, y = fill[pb[i]]++;
            to[x] = (int32_t)pb[i];
            cap[x] = pc[i];
            rev[x] = y;
            to[y] = (int32_t)pa[i];
            cap[y] = pd[i];
            rev[y] = x;
        }
        std::vector<int64_t>().swap(pa);
        std::vector<int64_t>().swap(pb);
        std::vector<int64_t>().swap(pc);
        std::vector<int64_t>().swap(pd);
    }
    // Maximum preflow by push-relabel (Goldberg and Tarjan), first phase
    // only, highest-label selection, exact distance labels recomputed by a
    // backward BFS from t at the start and after every N relabels.  Returns
    // the flow into t; the minimum cut follows from the residual graph
    // exactly as after a maximum flow (maximal_source_side).
    // init_ex: a preflow already encoded in the arcs' residual capacities
    // (source arcs saturated): the excess of every node and the flow that
    // already reached t; nullptr = start from zero flow
    int64_t maxflow(int64_t s, int64_t t, const std::vector<int64_t>* init_ex = nullptr, int64_t init_t = 0) {
        finalize();
        ThreadGrant grant(allow_parallel && N >= flow_parallel_min_nodes() ? flow_threads() : 1);
        const int threads = grant.n;
        if (threads > 1) {
            std::vector<int64_t> ex(N, 0);
            if (init_ex) {
                for (int64_t v = 0; v < N && v < (int64_t)init_ex->size(); ++v) ex[v] = (*init_ex)[v];
                ex[t] = init_t;
            }
            for (int64_t e = first[s]; e < first[s + 1]; ++e)
                if (cap[e] > 0) {
                    const int64_t d = cap[e];
                    cap[e] = 0;
                    cap[rev[e]] += d;
                    ex[to[e]] += d;
                }
            ex[s] = 0;
            return maxflow_parallel(N, first, to, cap, rev, s, t, ex, threads);
        }
        std::vector<int64_t> h(N, 0), ex(N, 0), it(first.begin(), first.end() - 1);
        if (init_ex) {
            for (int64_t v = 0; v < N && v < (int64_t)init_ex->size(); ++v) ex[v] = (*init_ex)[v];
            ex[t] = init_t;
        }
        std::vector<std::vector<int64_t>> bucket(N);
        int64_t top = -1;
        std::vector<int64_t> q;
        q.reserve(N);
        auto global_relabel = [&]() {
            std::fill(h.begin(), h.end(), N);
            h[t] = 0;
            q.clear();
            q.push_back(t);
            for (size_t qi = 0; qi < q.size(); ++qi) {
                const int64_t y = q[qi];
                for (int64_t e = first[y]; e < first[y + 1]; ++e) {
                    const int64_t x = to[e];
                    if (h[x] == N && x != s && cap[rev[e]] > 0) {
                        h[x] = h[y] + 1;
                        q.push_back(x);
                    }
                }
            }
            for (auto& b : bucket) b.clear();
            top = -1;
            for (int64_t v = 0; v < N; ++v)
                if (v != s && v != t && ex[v] > 0 && h[v] < N) {
                    bucket[h[v]].push_back(v);
                    top = std::max(top, h[v]);
                }
            std::copy(first.begin(), first.end() - 1, it.begin());
        };
        h[s] = N;
        for (int64_t e = first[s]; e < first[s + 1]; ++e)
            if (cap[e] > 0) {
                const int64_t d = cap[e];
                cap[e] = 0;
                cap[rev[e]] += d;
                ex[to[e]] += d;
            }
        ex[s] = 0;
        global_relabel();
        int64_t relabels = 0;
        for (;;) {
            while (top >= 0 && bucket[top].empty()) --top;
            if (top < 0) break;
            const int64_t v = bucket[top].back();
            bucket[top].pop_back();
            if (h[v] != top || ex[v] == 0) continue;
            // discharge v
            const int64_t end = first[v + 1];
            while (ex[v] > 0) {
                int64_t& e = it[v];
                for (; e < end; ++e) {
                    const int64_t w = to[e];
                    if (cap[e] > 0 && h[v] == h[w] + 1) {
                        const int64_t d = std::min(ex[v], cap[e]);
                        cap[e] -= d;
                        cap[rev[e]] += d;
                        ex[v] -= d;
                        if (ex[w] == 0 && w != t) {
                            bucket[h[w]].push_back(w);  // v may have been relabelled above top
                            top = std::max(top, h[w]);
                        }
                        ex[w] += d;
                        if (ex[v] == 0) break;
                    }
                }
                if (ex[v] == 0) break;
                int64_t mh = 2 * N;
                for (int64_t e2 = first[v]; e2 < end; ++e2)
                    if (cap[e2] > 0) mh = std::min(mh, h[to[e2]]);
                h[v] = mh + 1;
                it[v] = first[v];
                ++relabels;
                if (h[v] >= N) break;  // cannot reach t any more
            }
            if (ex[v] > 0 && h[v] < N) {
                bucket[h[v]].push_back(v);
                top = std::max(top, h[v]);
            }
            if (relabels >= N) {
                global_relabel();
                relabels = 0;
            }
        }
        return ex[t];
    }
    // after maxflow: 1 for nodes on the source side of the minimum cut with
    // the largest source side (nodes that cannot reach t in the residual)
    std::vector<char> maximal_source_side(int64_t t) const {
        std::vector<char> src(N, 1);
        std::vector<int64_t> q{t};
        src[t] = 0;
        for (size_t qi = 0; qi < q.size(); ++qi) {
            const int64_t y = q[qi];
            for (int64_t e = first[y]; e < first[y + 1]; ++e) {
                const int64_t x = to[e];
                if (src[x] && cap[rev[e]] > 0) {  // residual arc x -> y
                    src[x] = 0;
                    q.push_back(x);
                }
            }
        }
        return src;
    }
};

// Edges: maximal X ⊆ {0..k-1} maximising q * (|E(X)| + loops(X)) - p * |X|
// on Goldberg's network: source -> v (capacity q * (deg v + 2 loops v)),
// v -> sink (2p), each edge an undirected arc of capacity q.  The cut of X
// is q * sum_v (deg v + 2 loops v) - 2 * (the objective), so the maximal
// source side of a minimum cut is the maximal maximiser.  pairs: 2 local ids
// per edge; loops[v]: self-loops at v.  Returns the maximum value.
//
// split / D (optional, no self-loops): a fractional split of every edge,
// split[i] / D the share of the pair's first vertex (e.g. the FW numerators
// over D_N).  The network is then scaled by D and the flow starts from the
// preflow the split defines: every source arc saturated, q (D - 2 a) on the
// edge from its first vertex, each vertex sending to the sink what its load
// allows (2 q A_v up to 2 p D) and keeping the rest, 2 q (A_v - rho D), as
// excess.  Close to the optimum (a converged FW split) only those excesses
// remain to be pushed, so the search is short; the cut and value are those of
// the unscaled network.
int64_t max_excess_edges(int64_t k, const std::vector<int32_t>& pairs, const std::vector<int64_t>& loops, int64_t p,
                         int64_t q, std::vector<char>& inX, const std::vector<uint32_t>* split = nullptr,
                         int64_t D = 1) {
    const int64_t ne = (int64_t)pairs.size() / 2;
    if (k >= 1 && k + 2 >= flow_gpu_min_nodes()) {  // built, cut and read on the device
        int64_t wsum = 2 * ne;
        for (const int64_t l : loops) wsum += 2 * l;
        const bool warm = split && loops.empty() && D > 0 &&
                          (i128)q * D * (wsum + 1) + (i128)2 * p * D * (k + 1) < ((i128)1 << 61);
        return edge_mincut_device(k, pairs, loops, p, q, warm, D, split, inX, g_flow_stream);
    }
    // large networks are built by several threads (atomic counts and arc slots)
    const bool par = k + 2 >= flow_parallel_min_nodes() && flow_threads() > 1;
    std::vector<int64_t> w(k, 0), deg(k, 0);
    if (par) {
        par_for(2 * ne, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) __atomic_fetch_add(&deg[pairs[i]], 1, __ATOMIC_RELAXED);
        });
        for (int64_t v = 0; v < k; ++v) w[v] = (loops.empty() ? 0 : 2 * loops[v]) + deg[v];
    } else {
        for (int64_t v = 0; v < k; ++v) w[v] = loops.empty() ? 0 : 2 * loops[v];
        for (int64_t i = 0; i < 2 * ne; ++i) {
            w[pairs[i]]++;
            deg[pairs[i]]++;
        }
    }
    int64_t wsum = 0;
    for (int64_t v = 0; v < k; ++v) wsum += w[v];
    // the scaled network must stay well inside int64
    const bool warm = split && loops.empty() && D > 0 &&
                      (i128)q * D * (wsum + 1) + (i128)2 * p * D * (k + 1) < ((i128)1 << 61);
    const int64_t sc = warm ? D : 1;  // capacity scale
    const int64_t S = k, T = k + 1;
    Flow f(k + 2);
    {
        std::vector<int64_t> arcs(k + 2, 0);
        for (int64_t v = 0; v < k; ++v) {
            arcs[v] = deg[v] + 1 + (w[v] > 0 ? 1 : 0);
            arcs[S] += w[v] > 0 ? 1 : 0;
        }
        arcs[T] = k;
        f.begin(arcs);
    }
    std::vector<int64_t> A(warm ? k : 0, 0), ex;
    if (warm && par) {
        par_for(ne, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                const int64_t a = (*split)[i];
                __atomic_fetch_add(&A[pairs[2 * i]], a, __ATOMIC_RELAXED);
                __atomic_fetch_add(&A[pairs[2 * i + 1]], D - a, __ATOMIC_RELAXED);
            }
        });
    } else if (warm) {
        for (int64_t i = 0; i < ne; ++i) {
            const int64_t a = (*split)[i];
            A[pairs[2 * i]] += a;
            A[pairs[2 * i + 1]] += D - a;
        }
    }
    int64_t total = 0, to_t = 0;
    if (warm) ex.assign(k + 2, 0);
    for (int64_t v = 0; v < k; ++v) {
        if (w[v] > 0) {
            if (warm)
                f.add(S, v, 0, q * w[v] * sc);  // saturated
            else
                f.add(S, v, q * w[v]);
        }
        if (warm) {
            const int64_t tv = std::min(2 * q * A[v], 2 * p * D);
            f.add(v, T, 2 * p * D - tv, tv);
            ex[v] = 2 * q * A[v] - tv;
            to_t += tv;
        } else {
            f.add(v, T, 2 * p);
        }
        total += q * w[v] * sc;
    }
    auto edge_arcs = [&](int64_t i0, int64_t i1, bool atomic) {
        for (int64_t i = i0; i < i1; ++i) {
            int64_t c = q, cb = q;
            if (warm) {
                const int64_t fl = q * (D - 2 * (int64_t)(*split)[i]);  // net flow first -> second
                c = q * D - fl;
                cb = q * D + fl;
            }
            if (atomic)
                f.add_atomic(pairs[2 * i], pairs[2 * i + 1], c, cb);
            else
                f.add(pairs[2 * i], pairs[2 * i + 1], c, cb);
        }
    };
    if (par)
        par_for(ne, [&](int64_t i0, int64_t i1) { edge_arcs(i0, i1, true); });
    else
        edge_arcs(0, ne, false);
    const int64_t flow = warm ? f.maxflow(S, T, &ex, to_t) : f.maxflow(S, T);
    const std::vector<char> side = f.maximal_source_side(T);
    inX.assign(k, 0);
    for (int64_t v = 0; v < k; ++v) inX[v] = side[v];
    return (total - flow) / (2 * sc);
}

// Triangles: maximal X ⊆ {0..k-1} maximising q * #patterns inside X - p * |X| (a pattern
// is inside X when all its members are; -1 pads patterns with fewer than h
// members, a one-member pattern is a self-loop).  Network: source -> pattern
// (capacity q), pattern -> member (unbounded), vertex -> sink (p).  Returns
// the maximum value; inX marks the maximal maximiser.
// split / D (optional, full patterns only): per pattern member the share of
// the pattern (summing to D per pattern).  The network is then scaled by D
// and starts from the preflow of the split: source arcs saturated, q a_j from
// a pattern to its member j, every vertex sending min(q A_v, p D) to the sink
// and keeping the rest as excess.
int64_t max_excess(int64_t k, int h, const std::vector<int32_t>& pat, int64_t p, int64_t q, std::vector<char>& inX,
                   const std::vector<uint32_t>* split = nullptr, int64_t D = 1) {
    const int64_t np = (int64_t)pat.size() / h;
    const int64_t S = np + k, T = S + 1;
    Flow f(T + 1);
    f.allow_parallel = false;
    const int64_t INF = INT64_MAX / 4;
    const bool warm = split && D > 0 && (int64_t)split->size() == h * np &&
                      (i128)q * D * (np + 1) + (i128)p * D * (k + 1) < ((i128)1 << 61);
    {
        std::vector<int64_t> arcs(T + 1, 0);
        for (int64_t i = 0; i < np; ++i) {
            arcs[i] = 1;
            for (int j = 0; j < h; ++j)
                if (pat[h * i + j] >= 0) {
                    arcs[i]++;
                    arcs[np + pat[h * i + j]]++;
                }
        }
        for (int64_t v = 0; v < k; ++v) arcs[np + v]++;
        arcs[S] = np;
        arcs[T] = k;
        f.begin(arcs);
    }
    if (warm) {
        std::vector<int64_t> A(k, 0), ex(T + 1, 0);
        for (int64_t i = 0; i < np; ++i) {
            f.add(S, i, 0, q * D);  // saturated
            for (int j = 0; j < h; ++j) {
                const int64_t a = (*split)[h * i + j];
                f.add(i, np + pat[h * i + j], INF - q * a, q * a);
                A[pat[h * i + j]] += a;
            }
        }
        int64_t to_t = 0;
        for (int64_t v = 0; v < k; ++v) {
            const int64_t tv = std::min(q * A[v], p * D);
            f.add(np + v, T, p * D - tv, tv);
            ex[np + v] = q * A[v] - tv;
            to_t += tv;
        }
        const int64_t flow = f.maxflow(S, T, &ex, to_t);
        const std::vector<char> side = f.maximal_source_side(T);
        inX.assign(k, 0);
        for (int64_t v = 0; v < k; ++v) inX[v] = side[np + v];
        return (q * np * D - flow) / D;
    }
    for (int64_t i = 0; i < np; ++i) {
        f.add(S, i, q);
        for (int j = 0; j < h; ++j)
            if (pat[h * i + j] >= 0) f.add(i, np + pat[h * i + j], INF);
    }
    for (int64_t v = 0; v < k; ++v) f.add(np + v, T, p);
    const int64_t flow = f.maxflow(S, T);
    const std::vector<char> side = f.maximal_source_side(T);
    inX.assign(k, 0);
    for (int64_t v = 0; v < k; ++v) inX[v] = side[np + v];
    return q * np - flow;
}

}  // namespace

namespace {
thread_local bool g_single = false;
}
void topk_single_thread(bool on) { g_single = on; }
bool topk_threads_single() { return g_single; }

// ----------------------------------------------------------- host graph
namespace {
// v resized to count elements, left uninitialised, its pages faulted in by
// the granted host threads (one write per page), ready for one device copy;
// a copy into untouched pages faults them in one by one on one thread
template <class V>
void host_prefault(V& v, size_t count) {
    v.resize(count);
    if (count == 0) return;
    char* p = (char*)v.data();
    const size_t bytes = count * sizeof(v[0]);
    par_for((int64_t)((bytes + 4095) / 4096), [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) p[(size_t)i * 4096] = 0;
    });
}
// device -> host copy of count elements into v
template <class V>
void d2h_fill(V& v, const void* dev, size_t count, hipStream_t s) {
    host_prefault(v, count);
    if (count) LDS_HIP(hipMemcpyAsync(v.data(), dev, count * sizeof(v[0]), hipMemcpyDeviceToHost, s));
}
}  // namespace

void HostGraph::load(const Graph& g, int mode, hipStream_t s) {
    n = g.n;
    rp.assign(n + 1, 0);
    orig.assign(n, 0);
    if (n > 0) {
        LDS_HIP(hipMemcpyAsync(rp.data(), g.rowptr.p, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipMemcpyAsync(orig.data(), g.orig_of.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    d2h_fill(col, g.col.p, (size_t)(2 * g.m), s);
    tri.clear();
    if (mode == 3 && g.T > 0) d2h_fill(tri, g.tri.p, (size_t)(3 * g.T), s);
    LDS_HIP(hipStreamSynchronize(s));
    trp.clear();
    tinc.clear();
    if (mode == 3) {  // each vertex's triangles, listed on the device
        trp.resize(n + 1);
        host_prefault(tinc, tri.size());
        vertex_triangle_lists(g, trp.data(), tinc.data(), s);
    }
}


namespace {

// core (mode 2) / tr-core (mode 3) numbers of the subgraph induced by the
// alive vertices (all when alive is null), by peeling on the device;
// internal order, -2 for vertices outside
std::vector<int32_t> device_cores(Graph& g, int mode, const std::vector<char>* alive, hipStream_t s) {
    const int64_t n = g.n;
    std::vector<int32_t> out((size_t)n, 0);
    if (n == 0) return out;
    DBuf<uint8_t> al;
    if (alive) {
        al.alloc(n, s);
        LDS_HIP(hipMemcpyAsync(al.p, alive->data(), n, hipMemcpyHostToDevice, s));
    }
    DBuf<int32_t> c;
    c.alloc(n, s);
    core_numbers_gpu(g, mode, al.p, c.p, s);
    LDS_HIP(hipMemcpyAsync(out.data(), c.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    return out;
}

struct Cand {
    std::vector<int32_t> vs;  // internal ids
    Frac ub;                  // upper bound on the density of an LDS inside
    int64_t seq = 0;          // insertion order: later first among equal bounds
};
struct CandLess {
    bool operator()(const Cand& a, const Cand& b) const {
        if (lt(a.ub, b.ub)) return true;
        if (lt(b.ub, a.ub)) return false;
        return a.seq < b.seq;
    }
};

struct Ctx {
    explicit Ctx(const HostGraph& hg) : h(hg) {}
    Graph* g = nullptr;
    int mode = 2;
    int iters = 0;
    hipStream_t s = nullptr;
    const HostGraph& h;
    std::vector<Frac> lo, hi;     // bounds on phi_G, valid for every vertex
    std::vector<int32_t> loc;     // scratch: internal id -> local index, -1 outside
    std::vector<int32_t> mark;    // scratch, -1 outside
    bool warm = false;            // the graph's FW split (over splitD) is on the device for warm starts
    int64_t splitD = 1;
    TopkStats* st = nullptr;
    int64_t seq = 0;
    BandScope* scope = nullptr;   // device state of the IsLDS / IsLTDS search
};

// patterns of G[vs] by local index (edges: pairs, triangles: triples)
// split (optional): the graph's FW split numerators of the patterns (edges:
// the pair's first vertex's share, triangles: the three members' shares),
// gathered on the device from the indices collected here
void induced_patterns(Ctx& c, const std::vector<int32_t>& vs, std::vector<int32_t>& pat,
                      std::vector<uint32_t>* split = nullptr) {
    const HostGraph& h = c.h;
    pat.clear();
    if (split) split->clear();
    std::vector<int64_t> sidx;  // split indices, in pattern order
    for (size_t i = 0; i < vs.size(); ++i) c.loc[vs[i]] = (int32_t)i;
    // the patterns whose first (edges) / smallest (triangles) local index is in [i0, i1)
    auto range = [&](int64_t i0, int64_t i1, std::vector<int32_t>& P, std::vector<int64_t>* Sp) {
        if (c.mode == 2) {
            for (int64_t i = i0; i < i1; ++i)
                for (int64_t s = h.rp[vs[i]]; s < h.rp[vs[i] + 1]; ++s) {
                    const int32_t j = c.loc[h.col[s]];
                    if (j > (int32_t)i) {
                        P.push_back((int32_t)i);
                        P.push_back(j);
                        if (Sp) Sp->push_back(s);
                    }
                }
        } else {
            for (int64_t i = i0; i < i1; ++i)
                for (int64_t q = h.trp[vs[i]]; q < h.trp[vs[i] + 1]; ++q) {
                    const int32_t* x = &h.tri[3 * h.tinc[q]];
                    const int32_t a = c.loc[x[0]], b = c.loc[x[1]], d = c.loc[x[2]];
                    if (a < 0 || b < 0 || d < 0) continue;
                    if (std::min(a, std::min(b, d)) != (int32_t)i) continue;  // count each triangle once
                    P.push_back(a);
                    P.push_back(b);
                    P.push_back(d);
                    if (Sp) {
                        const int64_t t = h.tinc[q];
                        Sp->push_back(3 * t);
                        Sp->push_back(3 * t + 1);
                        Sp->push_back(3 * t + 2);
                    }
                }
        }
    };
    const int64_t k = (int64_t)vs.size();
    ThreadGrant grant(k >= flow_parallel_min_nodes() ? flow_threads() : 1);
    const int T = grant.n;
    if (T <= 1) {
        range(0, k, pat, split ? &sidx : nullptr);
    } else {
        // contiguous ranges per thread, concatenated in order: the same list
        std::vector<std::vector<int32_t>> P(T);
        std::vector<std::vector<int64_t>> Sp(T);
        std::vector<std::thread> pool;
        for (int t = 0; t < T; ++t)
            pool.emplace_back([&, t] { range(k * t / T, k * (t + 1) / T, P[t], split ? &Sp[t] : nullptr); });
        for (auto& th : pool) th.join();
        size_t np = 0, ns = 0;
        for (int t = 0; t < T; ++t) {
            np += P[t].size();
            ns += Sp[t].size();
        }
        pat.reserve(np);
        if (split) sidx.reserve(ns);
        for (int t = 0; t < T; ++t) {
            pat.insert(pat.end(), P[t].begin(), P[t].end());
            if (split) sidx.insert(sidx.end(), Sp[t].begin(), Sp[t].end());
        }
    }
    for (int32_t v : vs) c.loc[v] = -1;
    if (split && !sidx.empty()) {
        split->resize(sidx.size());
        gather_split(*c.g, c.mode, sidx.data(), (int64_t)sidx.size(), split->data(), c.s);
    }
}

// Is G[vs] connected?  A union-find over host threads: a root is linked
// below a smaller index by compare-and-swap and finds halve their paths, so
// every parent index is at most its own and no cycle can form; a link that
// loses a race is retried from the new roots.  The answer does not depend on
// the thread count or interleaving.  loc is -1 at every vertex on entry and
// on return.
bool induced_connected(const HostGraph& h, std::vector<int32_t>& loc, const std::vector<int32_t>& vs) {
    const int64_t k = (int64_t)vs.size();
    if (k <= 1) return true;
    for (int64_t i = 0; i < k; ++i) loc[vs[i]] = (int32_t)i;
    std::unique_ptr<std::atomic<int32_t>[]> par(new std::atomic<int32_t>[k]);
    for (int64_t i = 0; i < k; ++i) par[i].store((int32_t)i, std::memory_order_relaxed);
    auto find = [&](int32_t x) {
        for (;;) {
            int32_t p = par[x].load(std::memory_order_relaxed);
            if (p == x) return x;
            const int32_t g = par[p].load(std::memory_order_relaxed);
            if (g != p) par[x].compare_exchange_weak(p, g, std::memory_order_relaxed);
            x = g;
        }
    };
    auto unite = [&](int32_t a, int32_t b) {
        for (;;) {
            a = find(a);
            b = find(b);
            if (a == b) return;
            if (a < b) std::swap(a, b);
            int32_t want = a;
            if (par[a].compare_exchange_strong(want, b, std::memory_order_relaxed)) return;
        }
    };
    // chunks of vs taken from a shared counter (a candidate in degree order
    // puts every hub in the first range)
    std::atomic<int64_t> next{0};
    par_for(k, [&](int64_t, int64_t) {
        for (;;) {
            const int64_t c0 = next.fetch_add(4096), c1 = std::min(k, c0 + 4096);
            if (c0 >= k) break;
            for (int64_t i = c0; i < c1; ++i)
                for (int64_t s = h.rp[vs[i]]; s < h.rp[vs[i] + 1]; ++s) {
                    const int32_t j = loc[h.col[s]];
                    if (j > (int32_t)i) unite((int32_t)i, j);
                }
        }
    });
    const int32_t r = find(0);
    bool ok = true;
    for (int64_t i = 1; i < k && ok; ++i) ok = find((int32_t)i) == r;
    for (int32_t v : vs) loc[v] = -1;
    return ok;
}

// connected components (by edges) of G[vs]; a large connected G[vs] (the
// usual case, e.g. a whole graph) is recognised over host threads first
std::vector<std::vector<int32_t>> components(Ctx& c, const std::vector<int32_t>& vs) {
    if ((int64_t)vs.size() >= (1 << 16) && induced_connected(c.h, c.loc, vs)) return {vs};
    for (int32_t v : vs) c.mark[v] = 0;
    std::vector<std::vector<int32_t>> out;
    for (int32_t v0 : vs) {
        if (c.mark[v0] != 0) continue;
        std::vector<int32_t> comp{v0};
        c.mark[v0] = 1;
        for (size_t i = 0; i < comp.size(); ++i)
            for (int64_t s = c.h.rp[comp[i]]; s < c.h.rp[comp[i] + 1]; ++s) {
                const int32_t w = c.h.col[s];
                if (c.mark[w] == 0) {
                    c.mark[w] = 1;
                    comp.push_back(w);
                }
            }
        out.push_back(std::move(comp));
    }
    for (int32_t v : vs) c.mark[v] = -1;
    return out;
}

// IsDensest: is G[vs] its own densest subgraph?  rho = density(G[vs]);
// otherwise `denser` receives the maximal maximiser at lambda = rho, the
// vertices whose compact number in G[vs] is above rho.
bool is_densest(Ctx& c, const std::vector<int32_t>& vs, Frac* rho, std::vector<int32_t>* denser) {
    std::vector<int32_t> pat;
    std::vector<uint32_t> split;
    const bool warm = c.warm;
    induced_patterns(c, vs, pat, warm ? &split : nullptr);
    const int64_t np = (int64_t)pat.size() / c.mode;
    *rho = reduce(np, (int64_t)vs.size());
    if (np == 0) return true;
    std::vector<char> inX;
    c.st->maxflows++;
    // edges: the min cut starts from the FW split of the whole graph
    // restricted to G[S] (exact for S = V, a valid preflow for any S)
    const int64_t val = (c.mode == 2) ? max_excess_edges((int64_t)vs.size(), pat, {}, rho->n, rho->d, inX,
                                                         warm ? &split : nullptr, c.splitD)
                                      : max_excess((int64_t)vs.size(), 3, pat, rho->n, rho->d, inX,
                                                   warm ? &split : nullptr, c.splitD);
    if (val <= 0) return true;
    denser->clear();
    for (size_t i = 0; i < vs.size(); ++i)
        if (inX[i]) denser->push_back(vs[i]);
    return false;
}

// IsLDS (Alg. 4) for edges, IsLTDS (Alg. 7, ExtMaximal Alg. 8) for
// triangles: is the connected, self-densest G[vs] of density rho a maximal
// rho-compact connected subgraph of G?
bool is_lds(Ctx& c, const std::vector<int32_t>& vs, const Frac& rho) {
    const HostGraph& h = c.h;
    // Every vertex of an LDS has compact number rho, and none of its
    // neighbours has a larger one (Lemma lds-out-phi; Thm. cnltds for
    // triangles).  A neighbour whose lower bound exceeds rho is in the
    // maximal rho-compact region, so S would not be maximal: in Alg. 4 that
    // is a self-loop inside S's component, which the proof of Thm. isLDS
    // rules out; the flow network leaves such vertices out, so the device
    // search rejects S at once.  Otherwise it grows the region U over the
    // band lower <= rho <= upper, with one self-loop per edge to a vertex
    // above (edges) or the triangle truncated to its members in the band
    // (triangles), and returns the network when one is needed.
    ScopeOut o;
    if (!scope_band(*c.g, *c.scope, vs, rho.n, rho.d, o, c.s)) return false;
    if (!o.need_flow) return true;
    const std::vector<int32_t>& U = o.U;
    for (size_t i = 0; i < U.size(); ++i) {
        c.loc[U[i]] = (int32_t)i;
        c.mark[U[i]] = 1;  // 1: in U
    }
    std::vector<char> inX;
    c.st->maxflows++;
    if (c.mode == 2)
        max_excess_edges((int64_t)U.size(), o.pat, o.loops, rho.n, rho.d, inX);
    else
        max_excess((int64_t)U.size(), 3, o.pat, rho.n, rho.d, inX);
    // G[S] must be a connected component of G[X] (no vertex of S has a
    // self-loop: rejected above)
    bool ok = true;
    for (int32_t v : vs)
        if (!inX[c.loc[v]]) ok = false;
    if (ok) {
        for (int32_t v : vs) c.mark[v] = 2;
        for (int32_t v : vs)
            for (int64_t s = h.rp[v]; s < h.rp[v + 1] && ok; ++s) {
                const int32_t w = h.col[s];
                if (c.mark[w] == 1 && inX[c.loc[w]]) ok = false;
            }
    }
    for (int32_t v : U) {
        c.loc[v] = -1;
        c.mark[v] = -1;
    }
    return ok;
}

// largest upper bound on phi_G over vs, capped by `cap`
Frac bound_of(const Ctx& c, const std::vector<int32_t>& vs, const Frac* cap) {
    Frac b{0, 1};
    for (int32_t v : vs)
        if (lt(b, c.hi[v])) b = c.hi[v];
    if (cap && lt(*cap, b)) b = *cap;
    return b;
}

// stable groups of the last FW run on graph `gg` as candidate vertex sets;
// map(j) turns gg's internal id into an internal id of the input graph
template <class Map>
void collect_groups(Graph& gg, int mode, int iters, hipStream_t s, Map map, std::vector<std::vector<int32_t>>& sets,
                    std::vector<Frac>& his, std::vector<Frac>* los_per_set) {
    const SgState& q = gg.sg[mode == 2 ? 0 : 1];
    const int64_t k = gg.n;
    std::vector<int32_t> order(k);
    std::vector<int64_t> lo(k), hi(k);
    if (k > 0) {
        LDS_HIP(hipMemcpyAsync(order.data(), q.order.p, k * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipMemcpyAsync(lo.data(), q.lo.p, k * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipMemcpyAsync(hi.data(), q.hi.p, k * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
    }
    const int64_t D = (int64_t)fw_denom(mode, iters);
    int64_t covered = 0;
    for (size_t gi = 0; gi < q.gstart.size(); ++gi) {
        std::vector<int32_t> vs;
        for (int64_t j = q.gstart[gi]; j < q.gend[gi]; ++j) vs.push_back(map(order[j]));
        const int32_t first = order[q.gstart[gi]];
        his.push_back(reduce(hi[first], D));
        if (los_per_set) los_per_set->push_back(reduce(lo[first], D));
        sets.push_back(std::move(vs));
        covered = q.gend[gi];
    }
    if (covered < k) {  // never-accepted remainder: no bounds
        std::vector<int32_t> vs;
        for (int64_t j = covered; j < k; ++j) vs.push_back(map(order[j]));
        his.push_back(Frac{-1, 1});
        if (los_per_set) los_per_set->push_back(Frac{-1, 1});
        sets.push_back(std::move(vs));
    }
}

// FW + ExtractSG on G[vs]: the stable groups of the induced subgraph
// Alg. 5 re-runs FW + ExtractSG on G[S] for a popped candidate S that is not
// self-densest.  The candidates of one round go through the batched FW
// kernel together (one launch for all of their induced subgraphs, bit for
// bit the state of per-graph runs), then ExtractSG per subgraph.  Local ids
// follow caller-id order, so FW breaks ties as on the whole graph.
void refine_batch(Ctx& c, const std::vector<const std::vector<int32_t>*>& cands,
                  std::vector<std::vector<std::vector<int32_t>>>& sets, std::vector<std::vector<Frac>>& his) {
    const size_t nb = cands.size();
    std::vector<std::unique_ptr<Graph>> subs(nb);
    std::vector<std::vector<int32_t>> svs(nb);
    for (size_t b = 0; b < nb; ++b) {
        std::vector<int32_t>& sv = svs[b];
        sv = *cands[b];
        std::sort(sv.begin(), sv.end(), [&](int32_t x, int32_t y) { return c.h.orig[x] < c.h.orig[y]; });
        std::vector<int32_t> src, dst;
        for (size_t i = 0; i < sv.size(); ++i) c.loc[sv[i]] = (int32_t)i;
        for (size_t i = 0; i < sv.size(); ++i)
            for (int64_t q = c.h.rp[sv[i]]; q < c.h.rp[sv[i] + 1]; ++q) {
                const int32_t j = c.loc[c.h.col[q]];
                if (j > (int32_t)i) {
                    src.push_back((int32_t)i);
                    dst.push_back(j);
                }
            }
        for (int32_t v : sv) c.loc[v] = -1;
        subs[b] = std::make_unique<Graph>();
        build_graph(*subs[b], (int64_t)sv.size(), (int64_t)src.size(), src.data(), dst.data(), false, false, c.s);
    }
    {
        Batch bt;
        for (size_t b = 0; b < nb; ++b) {
            bt.gs.push_back(subs[b].get());
            bt.modes.push_back(c.mode);
            bt.iters.push_back(c.iters);
        }
        bt.capture = false;
        batch_build(bt, c.s);
        batch_run(bt, c.s);
        LDS_HIP(hipStreamSynchronize(c.s));
        c.st->refine_rounds++;
    }
    sets.assign(nb, {});
    his.assign(nb, {});
    for (size_t b = 0; b < nb; ++b) {
        Graph& sub = *subs[b];
        sg_stable_groups(sub, c.mode, c.s);
        std::vector<int32_t> orig(sub.n);
        if (sub.n > 0) {
            LDS_HIP(hipMemcpyAsync(orig.data(), sub.orig_of.p, sub.n * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
            LDS_HIP(hipStreamSynchronize(c.s));
        }
        const std::vector<int32_t>& sv = svs[b];
        collect_groups(sub, c.mode, c.iters, c.s, [&](int32_t j) { return sv[orig[j]]; }, sets[b], his[b], nullptr);
        c.st->refinements++;
    }
}

}  // namespace

size_t topk_footprint(const Graph& g, int mode, int iters) {
    const SweepPlan& p = (mode == 2) ? g.edge_plan : g.tri_plan;
    const size_t n = (size_t)g.n, slots = (size_t)p.nslots;
    const size_t T = mode == 3 && g.T > 0 ? (size_t)g.T : 0;
    const size_t fw = 2 * 8 * n + 2 * 2 * n + (size_t)iters * (size_t)p.total_words * 8 + (size_t)iters * 4 * 8 * 1024 +
                      (size_t)((p.n_push + 1) / 2) * 4 * 1024;  // the hub push's per-workgroup counters
    const size_t sg = 4 * n + 8 * n + 8 * n + n + 4 * slots + 12 * T + 16 * n;  // order pos E inI a_slot a_tri lo hi
    // sort keys / values, R T F V, counts, and the slot records (own position,
    // other positions and splits; record offsets by position)
    const size_t rec = slots * (mode == 2 ? 12 : 24) + 8 * (n + 1);
    const size_t tmp = 24 * n + 32 * n + 8 * n + rec;
    return fw + sg + tmp;
}

void topk_run(Graph& g, int mode, int k, int iters, hipStream_t s, std::vector<TopkSet>& out, TopkStats& st,
              bool reuse_fw, int8_t* prune_out) {
    // the device min cuts of this search run on its stream
    struct StreamScope {
        hipStream_t prev;
        explicit StreamScope(hipStream_t s) : prev(g_flow_stream) { g_flow_stream = s; }
        ~StreamScope() { g_flow_stream = prev; }
    } stream_scope(s);
    LDS_CHECK(mode == 2 || mode == 3, ST_INVALID, "mode must be LDS_EDGE or LDS_TRIANGLE");
    LDS_CHECK(k >= 1, ST_INVALID, "k must be >= 1");
    LDS_CHECK(iters >= 0, ST_INVALID, "iters must be >= 0");
    check_split_width(mode, iters);
    out.clear();
    st = TopkStats{};
    auto t0 = std::chrono::steady_clock::now();
    auto lap = [&t0](double* acc) {
        const auto t1 = std::chrono::steady_clock::now();
        *acc += std::chrono::duration<double, std::milli>(t1 - t0).count();
        t0 = t1;
    };
    const int64_t n = g.n;
    if (n == 0) return;
    if (mode == 3 && g.T < 0) list_triangles(g, s);
    // host data of the graph (built once, kept with the resident graph; a
    // per-query view shares its graph's): the adjacency, the triangles and
    // the core numbers of this mode are set up under one lock, and only read
    // afterwards, so that queries on one graph may run at once
    std::shared_ptr<HostCache> hcp;
    {
        static std::mutex setup;
        std::lock_guard<std::mutex> lk(setup);
        Graph& hg = g.origin ? *g.origin : g;
        if (!hg.host) {
            auto hc = std::make_shared<HostCache>();
            hc->h.load(g, mode, s);
            hc->tri_loaded = (mode == 3);
            hg.host = hc;
        } else if (mode == 3 && !hg.host->tri_loaded) {
            hg.host->h.load(g, 3, s);
            hg.host->tri_loaded = true;
        }
        lap(&st.ms_copy);
        std::vector<int32_t>& core = hg.host->core[mode == 2 ? 0 : 1];
        if (core.empty()) core = device_cores(g, mode, nullptr, s);
        hcp = hg.host;
        lap(&st.ms_core);
    }
    HostCache& hc = *hcp;
    Ctx c(hc.h);
    c.g = &g;
    c.mode = mode;
    c.iters = iters;
    c.s = s;
    c.st = &st;
    c.loc.assign(n, -1);
    c.mark.assign(n, -1);
    std::vector<char> alive(n, 1);
    // bounds from core (tr-core) numbers
    {
        const std::vector<int32_t>& core = hc.core[mode == 2 ? 0 : 1];
        c.lo.resize(n);
        c.hi.resize(n);
        for (int64_t u = 0; u < n; ++u) {
            c.lo[u] = reduce(core[u], mode);
            c.hi[u] = Frac{core[u], 1};
        }
    }
    lap(&st.ms_core);
    // FW + ExtractSG on the whole graph; group bounds tighten the core bounds
    const FwState& fs = g.fw[mode == 2 ? 0 : 1];
    if (!(reuse_fw && fs.ran && fs.iters == iters)) fw_run(g, mode, iters, false, s);
    sg_stable_groups(g, mode, s);
    std::vector<std::vector<int32_t>> sets;
    std::vector<Frac> his, los;
    collect_groups(g, mode, iters, s, [](int32_t j) { return j; }, sets, his, &los);
    // the FW split (every CSR slot for edges, every triangle's three shares
    // for triangles) stays on the device; warm-started min cuts gather the
    // shares of their candidate's patterns
    if ((mode == 2 && g.m > 0) || (mode == 3 && g.T > 0)) {
        c.warm = true;
        c.splitD = (int64_t)fw_denom(mode, iters);
    }
    for (size_t i = 0; i < sets.size(); ++i) {
        if (his[i].n < 0) continue;  // remainder without bounds
        for (int32_t u : sets[i]) {
            if (lt(c.lo[u], los[i])) c.lo[u] = los[i];
            if (lt(his[i], c.hi[u])) c.hi[u] = his[i];
        }
    }
    BandScope scope;
    {
        std::vector<int64_t> lon(n), lod(n), hin(n), hid(n);
        for (int64_t u = 0; u < n; ++u) {
            lon[u] = c.lo[u].n;
            lod[u] = c.lo[u].d;
            hin[u] = c.hi[u].n;
            hid[u] = c.hi[u].d;
        }
        scope_init(g, mode, lon.data(), lod.data(), hin.data(), hid.data(), scope, s);
        c.scope = &scope;
    }
    lap(&st.ms_fw);
    // Pruning (Alg. 3) on the device with the bounds just staged there: rule
    // 1, then rule 2 on the residual graph until nothing changes
    {
        DBuf<uint8_t> al, rl;
        al.alloc(n, s);
        rl.alloc(n, s);
        prune_device(g, mode, scope, al.p, rl.p, s);
        LDS_HIP(hipMemcpyAsync(alive.data(), al.p, n, hipMemcpyDeviceToHost, s));
        if (prune_out) {
            std::vector<int8_t> rule((size_t)n);
            LDS_HIP(hipMemcpyAsync(rule.data(), rl.p, n, hipMemcpyDeviceToHost, s));
            LDS_HIP(hipStreamSynchronize(s));
            for (int64_t u = 0; u < n; ++u) prune_out[hc.h.orig[u]] = rule[u];
        }
        LDS_HIP(hipStreamSynchronize(s));
    }
    for (int64_t u = 0; u < n; ++u) st.pruned += alive[u] ? 0 : 1;
    lap(&st.ms_prune);
    if (prune_out) return;
    std::priority_queue<Cand, std::vector<Cand>, CandLess> pq;
    auto push = [&](std::vector<int32_t>&& vs, const Frac* cap) {
        if (vs.empty()) return;
        Cand cd;
        cd.ub = bound_of(c, vs, cap);
        cd.vs = std::move(vs);
        cd.seq = c.seq++;
        pq.push(std::move(cd));
    };
    for (size_t i = 0; i < sets.size(); ++i) {
        std::vector<int32_t> vs;
        for (int32_t u : sets[i])
            if (alive[u]) vs.push_back(u);
        push(std::move(vs), his[i].n >= 0 ? &his[i] : nullptr);
    }
    std::vector<std::pair<Frac, std::vector<int32_t>>> found;
    std::vector<Frac> dens;  // densities found, for the k-th largest
    // LDS_TOPK_TRACE=1 prints one line per candidate to stderr
    const char* tr_env = std::getenv("LDS_TOPK_TRACE");
    const bool trace = tr_env && tr_env[0] == '1';
    auto tick = std::chrono::steady_clock::now();
    auto note = [&](const char* what, size_t size, const Frac& r) {
        if (!trace) return;
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[topk] %-10s |S|=%zu rho=%lld/%lld %.1f ms\n", what, size, (long long)r.n,
                     (long long)r.d, std::chrono::duration<double, std::milli>(now - tick).count());
        tick = now;
    };
    // Candidates that fail IsDensest wait in `pend` and are refined together
    // (one batched FW launch).  The round is closed before a candidate with a
    // smaller bound is examined, before stopping, and when it is full, so
    // candidates are still examined in non-increasing order of their bound.
    struct Pend {
        Cand cd;
        Frac rho;
        std::vector<int32_t> denser;
    };
    std::vector<Pend> pend;
    constexpr size_t kRound = 64;
    auto flush = [&]() {
        if (pend.empty()) return;
        std::vector<const std::vector<int32_t>*> cs;
        for (const Pend& x : pend) cs.push_back(&x.cd.vs);
        std::vector<std::vector<std::vector<int32_t>>> parts;
        std::vector<std::vector<Frac>> phis;
        refine_batch(c, cs, parts, phis);
        for (size_t i = 0; i < pend.size(); ++i) {
            Pend& x = pend[i];
            note("refined", parts[i].size(), x.rho);
            if (parts[i].size() >= 2) {
                for (size_t j = 0; j < parts[i].size(); ++j) {
                    Frac cap = x.cd.ub;
                    if (phis[i][j].n >= 0 && lt(phis[i][j], cap)) cap = phis[i][j];
                    push(std::move(parts[i][j]), &cap);
                }
                continue;
            }
            // FW did not split G[S]: split by the min cut's denser vertex set
            st.flow_splits++;
            std::sort(x.denser.begin(), x.denser.end());
            std::vector<int32_t> top, rest;
            for (int32_t v : x.cd.vs)
                (std::binary_search(x.denser.begin(), x.denser.end(), v) ? top : rest).push_back(v);
            push(std::move(rest), &x.cd.ub);
            push(std::move(top), &x.cd.ub);
        }
        pend.clear();
    };
    for (;;) {
        if (pq.empty()) {
            if (pend.empty()) break;
            flush();
            continue;
        }
        // a candidate with a smaller bound than the waiting ones: refine those first
        if (!pend.empty() && lt(pq.top().ub, pend.front().cd.ub)) {
            flush();
            continue;
        }
        bool stop = pq.top().ub.n <= 0;  // an LDS has positive density
        if (!stop && (int)dens.size() >= k) {
            std::nth_element(dens.begin(), dens.begin() + (k - 1), dens.end(),
                             [](const Frac& a, const Frac& b) { return lt(b, a); });
            stop = lt(pq.top().ub, dens[k - 1]);  // no remaining candidate reaches the k-th density
        }
        if (stop) {
            if (pend.empty()) break;
            flush();
            continue;
        }
        Cand cd = std::move(const_cast<Cand&>(pq.top()));
        pq.pop();
        st.popped++;
        note("pop", cd.vs.size(), cd.ub);
        std::vector<std::vector<int32_t>> comps = components(c, cd.vs);
        if (comps.size() > 1) {
            note("components", comps.size(), cd.ub);
            for (auto& cc : comps) push(std::move(cc), &cd.ub);
            continue;
        }
        Frac rho;
        std::vector<int32_t> denser;
        const bool densest = is_densest(c, cd.vs, &rho, &denser);
        note(densest ? "densest" : "not-dense", denser.size(), rho);
        if (densest) {
            const bool ok = rho.n > 0 && is_lds(c, cd.vs, rho);
            note(ok ? "LDS" : "not-LDS", cd.vs.size(), rho);
            if (ok) {
                found.push_back({rho, cd.vs});
                dens.push_back(rho);
            }
            continue;
        }
        pend.push_back(Pend{std::move(cd), rho, std::move(denser)});
        if (pend.size() >= kRound) flush();
    }
    lap(&st.ms_search);
    for (auto& f : found) {
        TopkSet t;
        t.num = f.first.n;
        t.den = f.first.d;
        for (int32_t v : f.second) t.vertices.push_back(c.h.orig[v]);
        std::sort(t.vertices.begin(), t.vertices.end());
        out.push_back(std::move(t));
    }
    std::sort(out.begin(), out.end(), [](const TopkSet& a, const TopkSet& b) {
        const i128 l = (i128)a.num * b.den, r = (i128)b.num * a.den;
        if (l != r) return l > r;
        return a.vertices.front() < b.vertices.front();
    });
    if ((int64_t)out.size() > k) out.resize(k);
}

}  // namespace lds
