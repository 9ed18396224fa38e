// Maximum preflow by synchronous parallel push-relabel on host threads, for
// the large minimum cuts of IsDensest (a whole-graph candidate of a sparse
// graph is a tight transportation problem: every sink arc must be filled).
//
// The network is the CSR residual graph of the top-k driver's Flow (arcs of
// a node contiguous, rev[e] the paired arc).  Each pulse has phases separated
// by barriers, all labels fixed within a phase:
//   push     every active node v pushes its excess along admissible arcs
//            (h[w] == h[v] - 1).  Two nodes never push along the two arcs of
//            one pair in the same phase (that would need h[v] == h[w] - 1 and
//            h[w] == h[v] - 1), so each arc pair changes in one direction and
//            only excess needs atomic adds;
//   relabel  a node with excess left and no admissible arc takes 1 + the
//            smallest label over its residual arcs, computed from the old
//            labels (labels only grow, so the new labelling stays valid);
//   collect  nodes that received excess or were relabelled below N form the
//            next active set (per-thread lists).
// Exact distance labels come from a level-synchronous backward search from t
// (all threads, nodes claimed by compare-and-swap) at the start and after
// every N relabels.  The result is a maximum preflow, so the residual graph
// gives the same minimum cuts as any maximum flow.
#pragma once
#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <mutex>
#include <thread>
#include <vector>

namespace lds {

// Barrier of the pulse threads: a short spin, then a blocking wait, so that a
// thread preempted by other work in the process does not stall the others.
class PulseBarrier {
public:
    explicit PulseBarrier(int n) : n_(n) {}
    void wait() {
        const int gen = gen_.load(std::memory_order_acquire);
        if (count_.fetch_add(1, std::memory_order_acq_rel) == n_ - 1) {
            count_.store(0, std::memory_order_relaxed);
            {
                std::lock_guard<std::mutex> lk(mu_);
                gen_.fetch_add(1, std::memory_order_acq_rel);
            }
            cv_.notify_all();
            return;
        }
        for (int i = 0; i < 2000; ++i) {
            if (gen_.load(std::memory_order_acquire) != gen) return;
            if (i >= 64) std::this_thread::yield();
        }
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return gen_.load(std::memory_order_acquire) != gen; });
    }

private:
    const int n_;
    std::atomic<int> count_{0}, gen_{0};
    std::mutex mu_;
    std::condition_variable cv_;
};

// ex: excess per node on entry (source arcs already saturated, ex[s] = 0,
// ex[t] = flow already at t); on return the flow into t is ex[t].
inline int64_t maxflow_parallel(int64_t N, const std::vector<int64_t>& first, const std::vector<int32_t>& to,
                                std::vector<int64_t>& cap, const std::vector<int64_t>& rev, int64_t s, int64_t t,
                                std::vector<int64_t>& ex, int nthreads) {
    auto ald = [](const int64_t* p) { return __atomic_load_n(p, __ATOMIC_RELAXED); };
    auto ast = [](int64_t* p, int64_t v) { __atomic_store_n(p, v, __ATOMIC_RELAXED); };
    const int T = std::max(1, nthreads);
    const int32_t HN = (int32_t)N;
    std::vector<int32_t> h(N, 0), hn(N, 0);
    std::vector<uint8_t> queued(N, 0);
    // per-thread lists; a "set" is the concatenation of the T lists of one kind
    std::vector<std::vector<int32_t>> act(T), act2(T), nxt(T), rel(T);
    std::vector<int64_t> off(T + 1, 0);
    PulseBarrier bar(T);
    std::atomic<int64_t> cursor{0}, relabels{0};
    bool done = false, regl = false, level_empty = false;
    constexpr int64_t kGrain = 64;
    auto offsets = [&](std::vector<std::vector<int32_t>>& L) {
        off[0] = 0;
        for (int k = 0; k < T; ++k) off[k + 1] = off[k] + (int64_t)L[k].size();
    };
    // calls f(v) for every element of the set L (offsets in `off`), chunks taken from `cursor`
    auto for_set = [&](std::vector<std::vector<int32_t>>& L, auto&& f) {
        const int64_t total = off[T];
        for (;;) {
            const int64_t i0 = cursor.fetch_add(kGrain, std::memory_order_relaxed);
            if (i0 >= total) break;
            int k = 0;
            while (off[k + 1] <= i0) ++k;
            for (int64_t i = i0; i < std::min(total, i0 + kGrain); ++i) {
                while (off[k + 1] <= i) ++k;
                f((int64_t)L[k][i - off[k]]);
            }
        }
    };
    // collective: exact distance labels, then the active set
    auto global_relabel = [&](int id) {
        const int64_t lo = N * id / T, hi = N * (id + 1) / T;
        for (int64_t v = lo; v < hi; ++v) h[v] = HN;
        act[id].clear();
        act2[id].clear();
        bar.wait();
        if (id == 0) {
            h[t] = 0;
            act[0].push_back((int32_t)t);
            offsets(act);
            cursor.store(0);
        }
        bar.wait();
        for (int32_t lvl = 1;; ++lvl) {
            for_set(act, [&](int64_t y) {
                for (int64_t e = first[y]; e < first[y + 1]; ++e) {
                    const int64_t x = to[e];
                    if (x == s || ald(&cap[rev[e]]) <= 0) continue;
                    int32_t want = HN;
                    if (__atomic_load_n(&h[x], __ATOMIC_RELAXED) == HN &&
                        __atomic_compare_exchange_n(&h[x], &want, lvl, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED))
                        act2[id].push_back((int32_t)x);
                }
            });
            bar.wait();
            act[id].swap(act2[id]);
            act2[id].clear();
            bar.wait();
            if (id == 0) {
                offsets(act);
                cursor.store(0);
                level_empty = off[T] == 0;
            }
            bar.wait();
            if (level_empty) break;
        }
        for (int64_t v = lo; v < hi; ++v)
            if (v != s && v != t && h[v] < HN && ex[v] > 0) act[id].push_back((int32_t)v);
        bar.wait();
        if (id == 0) {
            h[s] = HN;
            offsets(act);
            cursor.store(0);
            done = off[T] == 0;
        }
        bar.wait();
    };
    auto worker = [&](int id) {
        global_relabel(id);
        while (!done) {
            // push phase
            for_set(act, [&](int64_t v) {
                const int32_t hv = h[v];
                if (hv >= HN) return;
                const int64_t ev = ald(&ex[v]);
                if (ev <= 0) return;
                int64_t rem = ev;
                for (int64_t e = first[v]; e < first[v + 1] && rem > 0; ++e) {
                    const int64_t c = ald(&cap[e]);
                    if (c <= 0) continue;
                    const int64_t w = to[e];
                    if (h[w] != hv - 1) continue;
                    const int64_t d = std::min(rem, c);
                    ast(&cap[e], c - d);
                    ast(&cap[rev[e]], ald(&cap[rev[e]]) + d);
                    __atomic_fetch_add(&ex[w], d, __ATOMIC_RELAXED);
                    rem -= d;
                    if (w != t && w != s && __atomic_exchange_n(&queued[w], (uint8_t)1, __ATOMIC_RELAXED) == 0)
                        nxt[id].push_back((int32_t)w);
                }
                if (rem != ev) __atomic_fetch_sub(&ex[v], ev - rem, __ATOMIC_RELAXED);
                if (rem > 0) rel[id].push_back((int32_t)v);
            });
            bar.wait();
            // relabel phase, from the old labels
            for (int32_t v : rel[id]) {
                int32_t mh = 2 * HN;
                for (int64_t e = first[v]; e < first[v + 1]; ++e)
                    if (ald(&cap[e]) > 0) mh = std::min(mh, h[to[e]]);
                hn[v] = std::min<int32_t>(HN, mh + 1);
            }
            bar.wait();
            for (int32_t v : rel[id]) {
                h[v] = hn[v];
                if (h[v] < HN && __atomic_exchange_n(&queued[v], (uint8_t)1, __ATOMIC_RELAXED) == 0)
                    nxt[id].push_back(v);
            }
            relabels.fetch_add((int64_t)rel[id].size(), std::memory_order_relaxed);
            rel[id].clear();
            bar.wait();
            // collect: each thread filters its own candidates
            act[id].clear();
            for (int32_t v : nxt[id]) {
                queued[v] = 0;
                if (h[v] < HN && ex[v] > 0) act[id].push_back(v);
            }
            nxt[id].clear();
            bar.wait();
            if (id == 0) {
                offsets(act);
                cursor.store(0);
                done = off[T] == 0;
                regl = !done && relabels.load() >= N;
                if (regl) relabels.store(0);
            }
            bar.wait();
            if (regl) global_relabel(id);
        }
    };
    std::vector<std::thread> pool;
    for (int i = 1; i < T; ++i) pool.emplace_back(worker, i);
    worker(0);
    for (auto& th : pool) th.join();
    return ex[t];
}

}  // namespace lds
