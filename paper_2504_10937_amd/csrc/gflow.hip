// Maximum preflow on the device for the large vertex networks of IsDensest
// (a whole-graph candidate of a sparse graph is a tight transportation
// problem: every sink arc must be filled), by the synchronous push-relabel of
// the host threads' version (pflow.hpp) laid out for the GPU.
//
// One cooperative launch; the workgroups meet at grid barriers between the
// two phases of a pulse:
//   push     every active node v pushes its excess along admissible arcs
//            (h[w] == h[v] - 1, residual capacity) in arc order: a node
//            with few arcs on one lane, a large one on a wave whose lanes
//            take rows of 64 arcs and split the excess by a prefix sum;
//            two nodes never push along the two arcs of
//            one pair in the same phase (that would need h[v] == h[w] - 1
//            and h[w] == h[v] - 1), so only the excess needs atomics;
//            receivers join the next active list;
//   relabel  a node with excess left (every arc it could push along is
//            saturated, so each residual arc leads to a label >= its own)
//            takes 1 + the smallest label over its residual arcs, written
//            in place, and joins the next active list.  A label read while
//            its node is relabelled is the old or the new one; both are at
//            most the new one, so the labelling stays valid, and the new
//            label still exceeds the old.
// A node joins a list at most once per pulse: it swaps the pulse's tag into
// its mark, and only the swap that changes the mark appends it.  Entries
// whose excess is gone by the next pulse are skipped there.
// Exact distance labels come from a level-synchronous backward search from t
// (nodes claimed by compare-and-swap; its first level, t's arcs, spread over
// the whole grid) at the start and after every N relabels.  The result is a
// maximum preflow, so the residual graph gives the same minimum cuts as any
// maximum flow.
//
// List counters live in two rings of four words indexed by the phase number:
// phase ph counts into slot ph & 3, which workgroup 0 zeroed during phase
// ph - 1 (the relabel phase appends to its push phase's slot).  A slot is
// read right after the barrier that ends its last writer and zeroed again
// in phase ph + 3, behind a barrier that every workgroup reaches only after
// that read.  Every decision is taken from values read after a
// barrier, so control flow is uniform.  Waits and loops are bounded; past a
// bound the kernel raises an error flag and ends.
#include <algorithm>
#include <climits>
#include <cstdlib>

#include "gflow.hpp"
#include "graph.hpp"
#include "gridsync.hpp"

namespace lds {

namespace {

constexpr int kFT = 512;
constexpr int64_t kFlowMaxWG = 64;
enum : int { F_RING1 = 0, F_RING2 = 4, F_ERR = 8 };

struct FlowArgs {
    const int64_t* first;
    const int32_t* to;
    int64_t* cap;
    const int64_t* rev;
    int64_t* ex;
    int32_t* h;
    uint32_t* queued;  // the tag of the last pulse whose next list holds the node
    int32_t* act;
    int32_t* act2;
    int32_t* nxt;
    int32_t* rel;
    int32_t* r3;
    int32_t* ctr;   // F_* words (16)
    unsigned* bar;  // grid barrier counter
    int64_t N, s, t;
    int final_search;  // after the flow: labels < N exactly at the nodes that reach t
};

__device__ inline void push_list(int32_t* list, int32_t* count, int32_t v) { list[atomicAdd(count, 1)] = v; }

__device__ inline int64_t shfl_up_i64(int64_t v, int d) {
    const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)(uint64_t)v, (unsigned)d, 64);
    const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)((uint64_t)v >> 32), (unsigned)d, 64);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ inline int64_t readlane_i64(int64_t v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Calls small(v) on the thread of each node v of list[0, count) with at most
// kSmallDeg arcs, and big(v) on a whole wave for each larger one: most nodes
// of these networks have a handful of arcs, so a lane per node keeps 64 of
// them in flight per wave, while the few hubs get a wave's 64 lanes.  The
// workgroups take the list in blocks of kFT; a block's large nodes go through
// a list in LDS.  Every thread of the workgroup must call it.
#ifndef LDS_FLOW_SMALL_DEG
#define LDS_FLOW_SMALL_DEG 64
#endif
constexpr int kSmallDeg = LDS_FLOW_SMALL_DEG;
constexpr int kLU = 8;  // arcs of a lane's node loaded together
constexpr int kWU = 4;  // rows of 64 arcs of a wave's node loaded together

template <class SmallF, class BigF>
__device__ inline void node_pass(const FlowArgs& a, const int32_t* list, int64_t count, int32_t* sbig, int* sbn,
                                 SmallF small, BigF big) {
    const int w = threadIdx.x >> 6;
    for (int64_t b = (int64_t)blockIdx.x * kFT; b < count; b += (int64_t)gridDim.x * kFT) {
        if (threadIdx.x == 0) *sbn = 0;
        __syncthreads();
        const int64_t i = b + threadIdx.x;
        if (i < count) {
            const int32_t v = list[i];
            if (a.first[v + 1] - a.first[v] <= kSmallDeg)
                small(v);
            else
                sbig[atomicAdd(sbn, 1)] = v;
        }
        __syncthreads();
        const int nb = *sbn;
        for (int j = w; j < nb; j += kFT / 64) big(sbig[j]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(kFT) void k_maxflow(FlowArgs a) {
    __shared__ int64_t s_err;
    __shared__ int32_t sbig[kFT];
    __shared__ int sbn;
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();
    const unsigned nwg = gridDim.x;
    const int64_t gt = (int64_t)blockIdx.x * kFT + threadIdx.x, nthr = (int64_t)nwg * kFT;
    const int lane = threadIdx.x & 63;
    const int64_t N = a.N;
    const int32_t HN = (int32_t)N;
    int32_t* ring1 = a.ctr + F_RING1;
    int32_t* ring2 = a.ctr + F_RING2;
    unsigned ph = 0;
    bool bad = false;
    auto end_phase = [&]() {
        if (gt == 0) {
            ring1[(ph + 1) & 3] = 0;
            ring2[(ph + 1) & 3] = 0;
        }
        grid_sync(a.bar, nwg, &s_err);
    };
    int32_t* act = a.act;
    int32_t* act2 = a.act2;
    int32_t na = 0;
    // exact distance labels by a backward search from t
    auto search_labels = [&]() {
        for (int64_t v = gt; v < N; v += nthr) a.h[v] = HN;
        end_phase();
        ++ph;
        int32_t* F = a.nxt;
        int32_t* G = a.r3;
        // x (the tail of arc rev[e], a residual arc into the frontier) takes
        // label lvl and joins list L, once
        auto claim = [&](int32_t x, int32_t lvl, int32_t* L, int32_t* slot) {
            if (a.h[x] != HN) return;
            int32_t want = HN;
            if (__hip_atomic_compare_exchange_strong(&a.h[x], &want, lvl, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT))
                push_list(L, slot, x);
        };
        // level 1: t has an arc from nearly every node, so its arcs are
        // spread over the whole grid
        int32_t* slot = ring1 + (ph & 3);
        if (gt == 0) a.h[a.t] = 0;
        for (int64_t e = a.first[a.t] + gt; e < a.first[a.t + 1]; e += nthr) {
            const int32_t x = a.to[e];
            if (x != a.s && a.cap[a.rev[e]] > 0) claim(x, 1, F, slot);
        }
        end_phase();
        if (s_err) {  // a barrier gave up: the count may be partial
            bad = true;
            return;
        }
        int32_t fc = *slot;
        ++ph;
        for (int32_t lvl = 2; fc > 0; ++lvl) {
            if (s_err || lvl > HN) {
                bad = true;
                return;
            }
            slot = ring1 + (ph & 3);
            node_pass(
                a, F, fc, sbig, &sbn,
                [&](int32_t y) {  // one lane: the arcs eight at a time
                    const int64_t e1 = a.first[y + 1];
                    for (int64_t e0 = a.first[y]; e0 < e1; e0 += kLU) {
                        int32_t x[kLU];
                        bool ok[kLU];
#pragma unroll
                        for (int u = 0; u < kLU; ++u) {
                            const int64_t e = e0 + u;
                            ok[u] = e < e1;
                            x[u] = ok[u] ? a.to[e] : 0;
                            ok[u] = ok[u] && x[u] != a.s && a.cap[a.rev[e]] > 0;
                        }
#pragma unroll
                        for (int u = 0; u < kLU; ++u)
                            if (ok[u]) claim(x[u], lvl, G, slot);
                    }
                },
                [&](int32_t y) {  // one wave: rows of 64 arcs, kWU rows at a time
                    const int64_t e1 = a.first[y + 1];
                    for (int64_t eb = a.first[y] + lane; eb < e1; eb += 64 * kWU) {
                        int32_t x[kWU];
                        bool ok[kWU];
#pragma unroll
                        for (int u = 0; u < kWU; ++u) {
                            const int64_t e = eb + 64 * u;
                            ok[u] = e < e1;
                            x[u] = ok[u] ? a.to[e] : 0;
                            ok[u] = ok[u] && x[u] != a.s && a.cap[a.rev[e]] > 0;
                        }
#pragma unroll
                        for (int u = 0; u < kWU; ++u)
                            if (ok[u]) claim(x[u], lvl, G, slot);
                    }
                });
            end_phase();
            if (s_err) {
                bad = true;
                return;
            }
            fc = *slot;
            ++ph;
            int32_t* tmp = F;
            F = G;
            G = tmp;
        }
    };
    // ... then the active list
    auto global_relabel = [&]() {
        search_labels();
        if (bad) return;
        int32_t* slot = ring1 + (ph & 3);
        for (int64_t v = gt; v < N; v += nthr)
            if (v != a.s && v != a.t && a.h[v] < HN && a.ex[v] > 0) push_list(act, slot, (int32_t)v);
        end_phase();
        if (s_err) {
            bad = true;
            return;
        }
        na = *slot;
        ++ph;
    };
    global_relabel();
    int64_t relabels = 0;
    // far above what a run needs (a bound, not a budget); it also keeps the
    // pulse tags distinct
    const int64_t max_pulses = min(4 * N + 100000, (int64_t)0x7ffffff0);
    for (int64_t pulse = 0; na > 0 && !bad; ++pulse) {
        if (s_err || pulse > max_pulses) {
            bad = true;
            break;
        }
        const uint32_t tag = (uint32_t)pulse + 1u;
        // push; s1 counts the next list over both phases of the pulse
        int32_t* s1 = ring1 + (ph & 3);
        int32_t* s2 = ring2 + (ph & 3);
        auto join_next = [&](int32_t v) {
            if (atomicExch(&a.queued[v], tag) != tag) push_list(act2, s1, v);
        };
        // pushes d along arc e (v -> w)
        auto push_arc = [&](int64_t e, int32_t w, int64_t c, int64_t d) {
            a.cap[e] = c - d;
            a.cap[a.rev[e]] += d;
            atomicAdd((unsigned long long*)&a.ex[w], (unsigned long long)d);
            if (w != a.t && w != a.s) join_next(w);
        };
        node_pass(
            a, act, na, sbig, &sbn,
            [&](int32_t v) {  // one lane: the arcs in order
                const int32_t hv = a.h[v];
                if (hv >= HN) return;
                const int64_t ev = __hip_atomic_load(&a.ex[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (ev <= 0) return;
                int64_t rem = ev;
                const int64_t e1 = a.first[v + 1];
                for (int64_t e0 = a.first[v]; e0 < e1 && rem > 0; e0 += kLU) {
                    int64_t c[kLU];
                    int32_t w[kLU];
#pragma unroll
                    for (int u = 0; u < kLU; ++u) {
                        const bool in = e0 + u < e1;
                        c[u] = in ? a.cap[e0 + u] : 0;
                        w[u] = in ? a.to[e0 + u] : 0;
                    }
                    bool adm[kLU];
#pragma unroll
                    for (int u = 0; u < kLU; ++u) adm[u] = c[u] > 0 && a.h[w[u]] == hv - 1;
#pragma unroll
                    for (int u = 0; u < kLU; ++u)
                        if (adm[u] && rem > 0) {
                            const int64_t d = min(rem, c[u]);
                            push_arc(e0 + u, w[u], c[u], d);
                            rem -= d;
                        }
                }
                if (rem != ev) atomicAdd((unsigned long long*)&a.ex[v], (unsigned long long)(rem - ev));
                if (rem > 0) push_list(a.rel, s2, v);
            },
            [&](int32_t v) {  // one wave: rows of 64 arcs, the excess split in arc order by a prefix sum
                const int32_t hv = a.h[v];
                if (hv >= HN) return;
                const int64_t ev =
                    readlane_i64(__hip_atomic_load(&a.ex[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT), 0);
                if (ev <= 0) return;
                int64_t rem = ev;
                const int64_t e1 = a.first[v + 1];
                for (int64_t eb = a.first[v]; eb < e1 && rem > 0; eb += 64 * kWU) {
                    int64_t c[kWU];
                    int32_t w[kWU];
#pragma unroll
                    for (int u = 0; u < kWU; ++u) {
                        const int64_t e = eb + 64 * u + lane;
                        c[u] = e < e1 ? a.cap[e] : 0;
                        w[u] = e < e1 ? a.to[e] : 0;
                    }
                    bool adm[kWU];
#pragma unroll
                    for (int u = 0; u < kWU; ++u) adm[u] = c[u] > 0 && a.h[w[u]] == hv - 1;
#pragma unroll
                    for (int u = 0; u < kWU; ++u) {
                        if (rem <= 0) break;
                        const int64_t avail = adm[u] ? c[u] : 0;
                        int64_t incl = avail;
                        for (int off = 1; off < 64; off <<= 1) {
                            const int64_t o = shfl_up_i64(incl, off);
                            if (lane >= off) incl += o;
                        }
                        const int64_t excl = incl - avail;
                        const int64_t d = adm[u] ? min(avail, max((int64_t)0, rem - excl)) : 0;
                        if (d > 0) push_arc(eb + 64 * u + lane, w[u], c[u], d);
                        rem -= min(rem, readlane_i64(incl, 63));
                    }
                }
                if (lane == 0) {
                    if (rem != ev) atomicAdd((unsigned long long*)&a.ex[v], (unsigned long long)(rem - ev));
                    if (rem > 0) push_list(a.rel, s2, v);
                }
            });
        end_phase();
        if (s_err) {  // the relabel list may be partial: leave before reading it
            bad = true;
            break;
        }
        const int32_t nR = *s2;
        ++ph;
        // relabel in place, then join the next list
        auto relabel_to = [&](int32_t v, int32_t mh) {
            const int32_t nh = (mh >= HN) ? HN : mh + 1;
            a.h[v] = nh;
            if (nh < HN) join_next(v);
        };
        node_pass(
            a, a.rel, nR, sbig, &sbn,
            [&](int32_t v) {
                int32_t mh = INT32_MAX;
                const int64_t e1 = a.first[v + 1];
                for (int64_t e0 = a.first[v]; e0 < e1; e0 += kLU) {
                    int32_t w[kLU];
#pragma unroll
                    for (int u = 0; u < kLU; ++u) w[u] = (e0 + u < e1 && a.cap[e0 + u] > 0) ? a.to[e0 + u] : -1;
#pragma unroll
                    for (int u = 0; u < kLU; ++u)
                        if (w[u] >= 0) mh = min(mh, a.h[w[u]]);
                }
                relabel_to(v, mh);
            },
            [&](int32_t v) {
                int32_t mh = INT32_MAX;
                const int64_t e1 = a.first[v + 1];
                for (int64_t eb = a.first[v] + lane; eb < e1; eb += 64 * kWU) {
                    int32_t w[kWU];
#pragma unroll
                    for (int u = 0; u < kWU; ++u) {
                        const int64_t e = eb + 64 * u;
                        w[u] = (e < e1 && a.cap[e] > 0) ? a.to[e] : -1;
                    }
#pragma unroll
                    for (int u = 0; u < kWU; ++u)
                        if (w[u] >= 0) mh = min(mh, a.h[w[u]]);
                }
                for (int o = 32; o > 0; o >>= 1) mh = min(mh, __shfl_xor(mh, o, 64));
                if (lane == 0) relabel_to(v, mh);
            });
        end_phase();
        if (s_err) {
            bad = true;
            break;
        }
        na = *s1;
        ++ph;
        relabels += nR;
        int32_t* tmp = act;
        act = act2;
        act2 = tmp;
        if (na > 0 && relabels >= N) {
            relabels = 0;
            global_relabel();
        }
    }
    if (a.final_search && !bad && !s_err) search_labels();
    if (threadIdx.x == 0 && (bad || s_err)) a.ctr[F_ERR] = 1;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---- Goldberg's vertex network built on the device (nodes 0..k-1, source
// S = k, sink T = k + 1): each node's arcs are its edge arcs (slots taken by
// an atomic cursor, so their order varies; the flow value and the maximal
// minimum cut do not), then the arc to T, then the reverse of the arc from S.
// The source arcs are saturated from the start.
__global__ void k_net_deg(const int32_t* pairs, int64_t ne, int32_t* deg) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= ne) return;
    atomicAdd(&deg[pairs[2 * i]], 1);
    atomicAdd(&deg[pairs[2 * i + 1]], 1);
}

__global__ void k_net_shares(const int32_t* pairs, const uint32_t* split, int64_t ne, int64_t D, int64_t* A) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= ne) return;
    const int64_t a = split[i];
    atomicAdd((unsigned long long*)&A[pairs[2 * i]], (unsigned long long)a);
    atomicAdd((unsigned long long*)&A[pairs[2 * i + 1]], (unsigned long long)(D - a));
}

__global__ void k_net_counts(int64_t k, const int32_t* deg, const int64_t* loops, int64_t* w, uint64_t* cnt) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= k) return;
    const int64_t wv = (loops ? 2 * loops[v] : 0) + deg[v];
    w[v] = wv;
    cnt[v] = (uint64_t)deg[v] + 1 + (wv > 0 ? 1 : 0);
    if (wv > 0) atomicAdd((unsigned long long*)&cnt[k], 1ull);
}

__global__ void k_net_edges(const int32_t* pairs, const uint32_t* split, int64_t ne, int warm, int64_t q, int64_t D,
                            const int64_t* first, int32_t* cur, int32_t* to, int64_t* cap, int64_t* rev) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= ne) return;
    const int32_t a = pairs[2 * i], b = pairs[2 * i + 1];
    int64_t c = q, cb = q;
    if (warm) {
        const int64_t fl = q * (D - 2 * (int64_t)split[i]);  // net flow a -> b
        c = q * D - fl;
        cb = q * D + fl;
    }
    const int64_t pa = first[a] + atomicAdd(&cur[a], 1), pb = first[b] + atomicAdd(&cur[b], 1);
    to[pa] = b;
    to[pb] = a;
    cap[pa] = c;
    cap[pb] = cb;
    rev[pa] = pb;
    rev[pb] = pa;
}

__global__ void k_net_nodes(int64_t k, const int32_t* deg, const int64_t* w, const int64_t* A, int warm, int64_t p,
                            int64_t q, int64_t D, int64_t sc, const int64_t* first, int32_t* curS, int32_t* to,
                            int64_t* cap, int64_t* rev, int64_t* ex, unsigned long long* to_t) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= k) return;
    const int64_t S = k, T = k + 1;
    const int64_t e = first[v] + deg[v], eT = first[T] + v;  // v -> T and its reverse
    to[e] = (int32_t)T;
    to[eT] = (int32_t)v;
    rev[e] = eT;
    rev[eT] = e;
    int64_t exv = 0;
    if (warm) {
        const int64_t tv = min(2 * q * A[v], 2 * p * D);
        cap[e] = 2 * p * D - tv;
        cap[eT] = tv;
        exv = 2 * q * A[v] - tv;
        atomicAdd(to_t, (unsigned long long)tv);
    } else {
        cap[e] = 2 * p;
        cap[eT] = 0;
    }
    if (w[v] > 0) {  // S -> v, saturated
        const int64_t es = first[S] + atomicAdd(curS, 1), ev = e + 1;
        to[es] = (int32_t)v;
        to[ev] = (int32_t)S;
        rev[es] = ev;
        rev[ev] = es;
        cap[es] = 0;
        cap[ev] = q * w[v] * sc;
        if (!warm) exv += q * w[v];
    }
    ex[v] = exv;
}

__global__ void k_net_ends(int64_t k, const unsigned long long* to_t, int64_t* ex) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ex[k] = 0;
        ex[k + 1] = (int64_t)*to_t;
    }
}

// the scratch of a device flow over N nodes
struct FlowScratch {
    DBuf<int64_t> ex;
    DBuf<int32_t> h, act, act2, nxt, rel, r3, ctr;
    DBuf<uint32_t> queued;
    DBuf<unsigned> bar;
    void alloc(int64_t N, hipStream_t st) {
        ex.alloc(N, st);
        h.alloc(N, st);
        queued.alloc(N, st);
        act.alloc(N, st);
        act2.alloc(N, st);
        nxt.alloc(N, st);
        rel.alloc(N, st);
        r3.alloc(N, st);
        ctr.alloc(16, st);
        bar.alloc(2, st);
        k_fill_u32<<<grid_for(N, 256), 256, 0, st>>>(queued.p, N, 0u);
        k_fill_u32<<<1, 256, 0, st>>>((uint32_t*)ctr.p, 16, 0u);
        k_fill_u32<<<1, 256, 0, st>>>(bar.p, 2, 0u);
        LDS_HIP(hipGetLastError());
    }
};

// launches the flow over the network in fa (first / to / cap / rev / ex set)
void run_flow(FlowArgs& fa, FlowScratch& sc, hipStream_t st) {
    const int64_t N = fa.N;
    fa.h = sc.h.p;
    fa.queued = sc.queued.p;
    fa.act = sc.act.p;
    fa.act2 = sc.act2.p;
    fa.nxt = sc.nxt.p;
    fa.rel = sc.rel.p;
    fa.r3 = sc.r3.p;
    fa.ctr = sc.ctr.p;
    fa.bar = sc.bar.p;
    static int cus = 0, per = 0;
    if (!cus) {
        int dev = 0;
        LDS_HIP(hipGetDevice(&dev));
        LDS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        LDS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_maxflow, kFT, 0));
    }
    const int64_t resident = (int64_t)cus * std::max(1, per);
    // at most kFlowMaxWG workgroups, one per 8192 nodes; LDS_FLOW_GPU_WG
    // overrides both (e.g. to run the grid protocol wide on small networks)
    const char* ev = std::getenv("LDS_FLOW_GPU_WG");
    const int64_t forced = (ev && *ev) ? std::max<int64_t>(1, std::atoll(ev)) : 0;
    const int64_t grid = std::max<int64_t>(
        1, std::min<int64_t>({resident, forced ? forced : kFlowMaxWG, forced ? resident : (N + 8191) / 8192}));
    if (grid == 1) {  // one workgroup needs no co-residency guarantee
        k_maxflow<<<1, kFT, 0, st>>>(fa);
        LDS_HIP(hipGetLastError());
    } else {
        void* kargs[] = {&fa};
        LDS_HIP(hipLaunchCooperativeKernel((const void*)k_maxflow, dim3((unsigned)grid), dim3(kFT), kargs, 0, st));
    }
}

int32_t flow_error(const FlowScratch& sc, hipStream_t st) {
    int32_t err = 0;
    LDS_HIP(hipMemcpyAsync(&err, sc.ctr.p + F_ERR, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LDS_HIP(hipStreamSynchronize(st));
    return err;
}

}  // namespace

int64_t edge_mincut_device(int64_t k, const std::vector<int32_t>& pairs, const std::vector<int64_t>& loops, int64_t p,
                           int64_t q, bool warm, int64_t D, const std::vector<uint32_t>* split, std::vector<char>& inX,
                           hipStream_t st) {
    const int64_t ne = (int64_t)pairs.size() / 2, N = k + 2, S = k, T = k + 1;
    LDS_CHECK(k >= 1 && N < INT32_MAX, ST_INVALID, "device min cut: node count out of range");
    LDS_CHECK(!warm || (split && (int64_t)split->size() == ne && loops.empty()), ST_INVALID,
              "device min cut: a warm start needs one split per pair and no loops");
    const int64_t sc = warm ? D : 1;
    DBuf<int32_t> dpairs, deg, cur, dto;
    DBuf<uint32_t> dsplit;
    DBuf<int64_t> dloops, w, A, first, dcap, drev;
    DBuf<unsigned long long> to_t;
    dpairs.alloc(std::max<int64_t>(2 * ne, 1), st);
    deg.alloc(N, st);
    cur.alloc(N, st);
    w.alloc(k, st);
    first.alloc(N + 1, st);
    to_t.alloc(1, st);
    k_fill_u32<<<grid_for(N, 256), 256, 0, st>>>((uint32_t*)deg.p, N, 0u);
    k_fill_u32<<<grid_for(N, 256), 256, 0, st>>>((uint32_t*)cur.p, N, 0u);
    k_fill_u32<<<grid_for(2 * (N + 1), 256), 256, 0, st>>>((uint32_t*)first.p, 2 * (N + 1), 0u);
    k_fill_u32<<<1, 256, 0, st>>>((uint32_t*)to_t.p, 2, 0u);
    if (ne > 0)
        LDS_HIP(hipMemcpyAsync(dpairs.p, pairs.data(), 2 * ne * sizeof(int32_t), hipMemcpyHostToDevice, st));
    if (!loops.empty()) {
        dloops.alloc(k, st);
        LDS_HIP(hipMemcpyAsync(dloops.p, loops.data(), k * sizeof(int64_t), hipMemcpyHostToDevice, st));
    }
    if (warm) {
        dsplit.alloc(std::max<int64_t>(ne, 1), st);
        A.alloc(k, st);
        k_fill_u32<<<grid_for(2 * k, 256), 256, 0, st>>>((uint32_t*)A.p, 2 * k, 0u);
        if (ne > 0) LDS_HIP(hipMemcpyAsync(dsplit.p, split->data(), ne * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    }
    if (ne > 0) {
        k_net_deg<<<grid_for(ne, 256), 256, 0, st>>>(dpairs.p, ne, deg.p);
        if (warm) k_net_shares<<<grid_for(ne, 256), 256, 0, st>>>(dpairs.p, dsplit.p, ne, D, A.p);
    }
    // arc counts per node (S's counted by atomics, T's = k), offsets by a scan
    k_net_counts<<<grid_for(k, 256), 256, 0, st>>>(k, deg.p, dloops.p, w.p, (uint64_t*)first.p);
    LDS_HIP(hipMemcpyAsync(first.p + T, &k, sizeof(int64_t), hipMemcpyHostToDevice, st));
    exclusive_scan_u64((const uint64_t*)first.p, (uint64_t*)first.p, N, (uint64_t*)first.p + N, st);
    int64_t M = 0;
    LDS_HIP(hipMemcpyAsync(&M, first.p + N, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    LDS_HIP(hipStreamSynchronize(st));
    dto.alloc(std::max<int64_t>(M, 1), st);
    dcap.alloc(std::max<int64_t>(M, 1), st);
    drev.alloc(std::max<int64_t>(M, 1), st);
    FlowScratch fs;
    fs.alloc(N, st);
    if (ne > 0)
        k_net_edges<<<grid_for(ne, 256), 256, 0, st>>>(dpairs.p, dsplit.p, ne, warm ? 1 : 0, q, D, first.p, cur.p,
                                                       dto.p, dcap.p, drev.p);
    k_net_nodes<<<grid_for(k, 256), 256, 0, st>>>(k, deg.p, w.p, A.p, warm ? 1 : 0, p, q, D, sc, first.p,
                                                  cur.p + S, dto.p, dcap.p, drev.p, fs.ex.p, to_t.p);
    k_net_ends<<<1, 64, 0, st>>>(k, to_t.p, fs.ex.p);
    LDS_HIP(hipGetLastError());
    FlowArgs fa{};
    fa.first = first.p;
    fa.to = dto.p;
    fa.cap = dcap.p;
    fa.rev = drev.p;
    fa.ex = fs.ex.p;
    fa.N = N;
    fa.s = S;
    fa.t = T;
    fa.final_search = 1;
    run_flow(fa, fs, st);
    int64_t flow = 0;
    std::vector<int32_t> h(k);
    LDS_HIP(hipMemcpyAsync(&flow, fs.ex.p + T, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    LDS_HIP(hipMemcpyAsync(h.data(), fs.h.p, k * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    LDS_CHECK(flow_error(fs, st) == 0, ST_DEVICE, "device min cut: no progress or a grid barrier did not complete");
    // the maximal source side: the nodes that cannot reach T in the residual graph
    inX.assign(k, 0);
    for (int64_t v = 0; v < k; ++v) inX[v] = h[v] >= (int32_t)N ? 1 : 0;
    int64_t wsum = 0;
    for (int64_t v = 0; v < k; ++v) wsum += loops.empty() ? 0 : 2 * loops[v];
    wsum += 2 * ne;
    return (q * wsum * sc - flow) / (2 * sc);
}

}  // namespace lds
