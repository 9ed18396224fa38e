// Core numbers (edges) and tr-core numbers (triangles) on the device, for the
// initial bounds of the compact numbers and for Pruning (Alg. 3, rule 2 needs
// the core numbers of the residual graph).
//
// Level-synchronous peeling.  cnt[v] = number of patterns (edges or alive
// triangles) at v among the vertices not yet peeled.  At level k every
// remaining vertex with cnt <= k gets core k and is peeled; peeling v lowers
// its neighbours' counts (for triangles: kills each alive triangle of v once,
// lowering its two other vertices), and a vertex whose count drops to exactly
// k joins the next frontier of the same level (the decrement from k+1 to k
// happens once, so it joins once).  When a level's cascade ends, k jumps to
// the smallest remaining count.  Remaining vertices are kept in a compacted
// list, so each level costs in proportion to what is left.  The result is
// unique, so it does not depend on the order of atomics.
#include <algorithm>
#include <climits>
#include <cstdlib>

#include "graph.hpp"
#include "gridsync.hpp"

namespace lds {

namespace {

constexpr int kT = 256;
constexpr int32_t kUnset = -1, kOutside = -2;

__device__ inline void push(int32_t* list, int32_t* count, int32_t v) { list[atomicAdd(count, 1)] = v; }

__global__ void k_init_edges(const int64_t* rowptr, const int32_t* col, int64_t n, const uint8_t* alive,
                             int32_t* cnt, int32_t* core, int32_t* active, int32_t* na) {
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    if (alive && !alive[v]) {
        cnt[v] = 0;
        core[v] = kOutside;
        return;
    }
    int32_t c = 0;
    for (int64_t s = rowptr[v]; s < rowptr[v + 1]; ++s) c += (!alive || alive[col[s]]) ? 1 : 0;
    cnt[v] = c;
    core[v] = kUnset;
    push(active, na, (int32_t)v);
}

__global__ void k_init_vertices(int64_t n, const uint8_t* alive, int32_t* cnt, int32_t* core, int32_t* active,
                                int32_t* na) {
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    cnt[v] = 0;
    if (alive && !alive[v]) {
        core[v] = kOutside;
        return;
    }
    core[v] = kUnset;
    push(active, na, (int32_t)v);
}

__global__ void k_init_triangles(const int32_t* tri, int64_t T, const uint8_t* alive, int32_t* cnt,
                                 uint32_t* talive) {
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= T) return;
    const int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
    const bool in = !alive || (alive[a] && alive[b] && alive[c]);
    talive[t] = in ? 1u : 0u;
    if (in) {
        atomicAdd(&cnt[a], 1);
        atomicAdd(&cnt[b], 1);
        atomicAdd(&cnt[c], 1);
    }
}

enum : int { C_NA = 0, C_K = 3 };

__global__ void k_set(int32_t* p, int32_t v) { *p = v; }
__global__ void k_fill8(int32_t* p) { p[threadIdx.x] = 0; }
__global__ void k_fill16(int32_t* p, int32_t v) { p[threadIdx.x] = v; }
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) p[i] = v;
}

// The rest of the peeling in one workgroup once few vertices remain (small
// graphs from the start, the dense cores of large ones, the residual graphs of
// Pruning rule 2): the same levels, frontiers and cascades, separated by
// workgroup barriers.  The remaining vertices get local ids (their index in
// the remaining list; loc maps a vertex to it, -1 for every other vertex), and
// their counts, peeled flags, remaining lists and frontiers live in LDS, so a
// level touches global memory only to walk the frontier's adjacency (and, for
// triangles, to kill each triangle once).  Every level assigns a vertex or
// jumps to a larger count, so the loops are bounded by the number of
// remaining vertices; a bound that is ever reached raises err.
constexpr int kTailT = 1024;
constexpr int32_t kTailMax = 1 << 13;
constexpr int kTailU = 4;  // slots per lane in flight in the adjacency walks

template <bool TRI>
__global__ __launch_bounds__(kTailT) void k_peel_tail(const int32_t* act, int32_t na, int32_t k, int32_t* loc,
                                                      const int64_t* rowptr, const int32_t* col,
                                                      const int32_t* row_of, const int64_t* rp, const int32_t* py,
                                                      const int32_t* tos, uint32_t* talive, const int32_t* cnt,
                                                      int32_t* core, int32_t* err) {
    __shared__ int32_t lcnt[kTailMax];
    __shared__ uint8_t gone[kTailMax];
    __shared__ uint16_t lrem[2][kTailMax];  // remaining local ids, double-buffered
    __shared__ uint16_t lfr[2][kTailMax];   // frontier of a cascade round / the next one
    __shared__ int32_t sc[4];               // [0] frontier, [1] next, [2] minimum, [3] remaining
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int32_t i = tid; i < na; i += kTailT) {
        const int32_t v = act[i];
        loc[v] = i;
        lcnt[i] = cnt[v];
        gone[i] = 0;
        lrem[0][i] = (uint16_t)i;
    }
    __syncthreads();
    // a remaining neighbour w of a peeled vertex loses one pattern; the
    // decrement from k + 1 to k happens once and puts w into the next frontier
    auto lower_local = [&](int32_t lw, uint16_t* nx) {
        if (lw < 0 || gone[lw]) return;
        if (atomicSub(&lcnt[lw], 1) == k + 1) {
            gone[lw] = 1;
            core[act[lw]] = k;
            nx[atomicAdd(&sc[1], 1)] = (uint16_t)lw;
        }
    };
    int cur = 0;
    const int64_t bound = 2 * (int64_t)na + 2;
    for (int64_t it = 0; na > 0; ++it) {
        if (it > bound) {
            if (tid == 0) *err = 1;
            return;
        }
        if (tid == 0) sc[0] = 0;
        __syncthreads();
        for (int32_t i = tid; i < na; i += kTailT) {
            const int32_t l = lrem[cur][i];
            if (!gone[l] && lcnt[l] <= k) {
                gone[l] = 1;
                core[act[l]] = k;
                lfr[0][atomicAdd(&sc[0], 1)] = (uint16_t)l;
            }
        }
        __syncthreads();
        int32_t fc = sc[0];
        if (fc == 0) {  // jump to the smallest remaining count
            if (tid == 0) sc[2] = INT32_MAX;
            __syncthreads();
            for (int32_t i = tid; i < na; i += kTailT) {
                const int32_t l = lrem[cur][i];
                if (!gone[l]) atomicMin(&sc[2], lcnt[l]);
            }
            __syncthreads();
            const int32_t m = sc[2];
            __syncthreads();
            if (m == INT32_MAX || m <= k) {
                if (tid == 0) *err = 1;
                return;
            }
            k = m;
            continue;
        }
        int f = 0;
        for (int64_t round = 0; fc > 0; ++round) {
            if (round > na) {
                if (tid == 0) *err = 1;
                return;
            }
            if (tid == 0) sc[1] = 0;
            __syncthreads();
            uint16_t* nx = lfr[f ^ 1];
            for (int32_t i = wv; i < fc; i += kTailT / 64) {
                const int32_t v = act[lfr[f][i]];
                int64_t q0, q1;
                if (!TRI) {
                    q0 = rowptr[v];
                    q1 = rowptr[v + 1];
                } else {
                    const int32_t r = row_of[v];
                    if (r < 0) continue;
                    q0 = rp[r];
                    q1 = rp[r + 1];
                }
                for (int64_t qb = q0 + lane; qb < q1; qb += 64 * kTailU) {
                    if (!TRI) {
                        int32_t lw[kTailU];
#pragma unroll
                        for (int u = 0; u < kTailU; ++u) {
                            const int64_t q = qb + 64 * u;
                            lw[u] = q < q1 ? loc[col[q]] : -1;
                        }
#pragma unroll
                        for (int u = 0; u < kTailU; ++u) lower_local(lw[u], nx);
                    } else {
                        bool live[kTailU];
#pragma unroll
                        for (int u = 0; u < kTailU; ++u) {
                            const int64_t q = qb + 64 * u;
                            live[u] = q < q1 && atomicExch(&talive[tos[q]], 0u) != 0u;  // killed once
                        }
                        int32_t lw[kTailU][2];
#pragma unroll
                        for (int u = 0; u < kTailU; ++u) {
                            const int64_t q = qb + 64 * u;
                            lw[u][0] = live[u] ? loc[py[2 * q]] : -1;
                            lw[u][1] = live[u] ? loc[py[2 * q + 1]] : -1;
                        }
#pragma unroll
                        for (int u = 0; u < kTailU; ++u) {
                            lower_local(lw[u][0], nx);
                            lower_local(lw[u][1], nx);
                        }
                    }
                }
            }
            __syncthreads();
            fc = sc[1];
            f ^= 1;
            __syncthreads();
        }
        if (tid == 0) sc[3] = 0;
        __syncthreads();
        for (int32_t i = tid; i < na; i += kTailT) {
            const int32_t l = lrem[cur][i];
            if (!gone[l]) lrem[cur ^ 1][atomicAdd(&sc[3], 1)] = (uint16_t)l;
        }
        __syncthreads();
        na = sc[3];
        cur ^= 1;
        ++k;
        __syncthreads();
    }
}

// The levels of the peeling in one cooperative launch while many vertices
// remain: every workgroup works through each phase of a level and the
// workgroups meet at a grid barrier between phases, instead of one host
// round trip per level and per four cascade rounds.  A level is its cascade
// rounds (peeling the frontier lowers its neighbours; a count that falls to
// exactly k joins the next frontier) and one closing phase that compacts the
// remaining vertices, takes the smallest remaining count and already pushes
// the next level's frontier: after the cascade every remaining count is at
// least k + 1, and exactly the vertices at k + 1 open level k + 1.  Only
// when there are none does the level jump to the smallest count, with one
// more phase for that frontier.  List counters live in a ring of four
// indexed by the phase number: a phase pushes into slot ph & 3, which
// workgroup 0 zeroed during phase ph - 1 (its previous value was read right
// after barrier ph - 3, which every workgroup has passed by then).  Every
// decision is taken from values read after a barrier, so control flow is
// uniform.  It stops once at most tail_max vertices remain and leaves
// (remaining count, level, which list is current) in ctr for the
// one-workgroup tail.
constexpr int kPT = 512;
constexpr int64_t kPeelMaxWG = 64;
// ctr words: results, the ring, and per level parity the smallest remaining
// count (G_MIN) and the next frontier's counter (G_NF), written by a closing
// phase and reset by the closing phase after next
enum : int { G_NA = 1, G_K = 2, G_SWAP = 3, G_ERR = 4, G_RING = 8, G_MIN = 12, G_NF = 14 };

struct PeelArgs {
    const int64_t* rowptr;
    const int32_t* col;
    const int32_t* row_of;
    const int64_t* rp;
    const int32_t* py;
    const int32_t* tos;
    uint32_t* talive;
    int32_t* cnt;
    int32_t* core;
    int32_t* act;
    int32_t* act2;
    int32_t* front;
    int32_t* next;
    int32_t* ctr;   // G_* words (16)
    unsigned* bar;  // grid barrier counter
    int64_t n;
    int32_t na, k, tail_max;
};

__device__ inline void lower(int32_t* cnt, int32_t* core, int32_t w, int32_t k, int32_t* next, int32_t* nc) {
    if (core[w] != kUnset) return;
    const int32_t old = atomicSub(&cnt[w], 1);
    if (old == k + 1) {  // the decrement from k + 1 to k happens once
        core[w] = k;
        push(next, nc, w);
    }
}

template <bool TRI>
__global__ __launch_bounds__(kPT) void k_peel_grid(PeelArgs a) {
    __shared__ int64_t s_err;
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();
    const unsigned nwg = gridDim.x;
    const int64_t t = (int64_t)blockIdx.x * kPT + threadIdx.x, nthr = (int64_t)nwg * kPT;
    const int64_t gw = t >> 6, nwave = nthr >> 6;
    const int lane = threadIdx.x & 63;
    int32_t* ring = a.ctr + G_RING;
    int32_t *act = a.act, *act2 = a.act2;
    int32_t *f = a.front, *nx = a.next;
    int32_t na = a.na, k = a.k, fc = 0;
    unsigned ph = 0;
    bool bad = false, need_front = true;
    auto zero_next = [&]() {
        if (t == 0) ring[(ph + 1) & 3] = 0;
    };
    for (int64_t level = 0; na > a.tail_max && !bad; ++level) {
        if (level > a.n) {
            bad = true;
            break;
        }
        if (need_front) {
            // the smallest remaining count (first level: a phase of its own)
            if (level == 0) {
                int32_t m = INT32_MAX;
                for (int64_t i = t; i < na; i += nthr) m = min(m, a.cnt[act[i]]);
                for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o, 64));
                if (lane == 0 && m != INT32_MAX) atomicMin(&a.ctr[G_MIN], m);
                zero_next();
                grid_sync(a.bar, nwg, &s_err);
                ++ph;
            }
            const int32_t m = a.ctr[G_MIN + (level & 1)];
            if (s_err || m == INT32_MAX) {
                bad = true;
                break;
            }
            if (m > k) k = m;
            // phase: remaining vertices with cnt <= k get core k, into the frontier
            int32_t* slot = ring + (ph & 3);
            for (int64_t i = t; i < na; i += nthr) {
                const int32_t v = act[i];
                if (a.core[v] == kUnset && a.cnt[v] <= k) {
                    a.core[v] = k;
                    push(f, slot, v);
                }
            }
            zero_next();
            grid_sync(a.bar, nwg, &s_err);
            fc = *slot;
            ++ph;
        }
        for (int64_t round = 0; fc > 0 && !bad; ++round) {
            if (s_err || round > na) {
                bad = true;
                break;
            }
            int32_t* slot = ring + (ph & 3);
            for (int64_t i = gw; i < fc; i += nwave) {
                const int32_t v = f[i];
                if (!TRI) {
                    for (int64_t q = a.rowptr[v] + lane; q < a.rowptr[v + 1]; q += 64)
                        lower(a.cnt, a.core, a.col[q], k, nx, slot);
                } else {
                    const int32_t r = a.row_of[v];
                    if (r < 0) continue;
                    for (int64_t q = a.rp[r] + lane; q < a.rp[r + 1]; q += 64) {
                        if (atomicExch(&a.talive[a.tos[q]], 0u) == 0u) continue;  // killed before
                        lower(a.cnt, a.core, a.py[2 * q], k, nx, slot);
                        lower(a.cnt, a.core, a.py[2 * q + 1], k, nx, slot);
                    }
                }
            }
            zero_next();
            grid_sync(a.bar, nwg, &s_err);
            fc = *slot;
            ++ph;
            int32_t* tmp = f;
            f = nx;
            nx = tmp;
        }
        if (bad) break;
        // closing phase: compaction, the smallest remaining count, and the
        // next level's frontier (remaining vertices at exactly k + 1), into
        // the words of the next level's parity; the words of this level's
        // parity were read two phases ago at the latest, so they are reset
        // here for the level after next
        int32_t* slot = ring + (ph & 3);
        const int nl = (int)((level + 1) & 1);
        if (t == 0) {
            a.ctr[G_MIN + (nl ^ 1)] = INT32_MAX;
            a.ctr[G_NF + (nl ^ 1)] = 0;
        }
        {
            int32_t m = INT32_MAX;
            for (int64_t i = t; i < na; i += nthr) {
                const int32_t v = act[i];
                if (a.core[v] != kUnset) continue;
                push(act2, slot, v);
                const int32_t c = a.cnt[v];
                m = min(m, c);
                if (c == k + 1) {
                    a.core[v] = k + 1;
                    push(f, &a.ctr[G_NF + nl], v);
                }
            }
            for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o, 64));
            if (lane == 0 && m != INT32_MAX) atomicMin(&a.ctr[G_MIN + nl], m);
        }
        zero_next();
        grid_sync(a.bar, nwg, &s_err);
        na = *slot;
        fc = a.ctr[G_NF + nl];
        ++ph;
        int32_t* tmp = act;
        act = act2;
        act2 = tmp;
        ++k;
        need_front = fc == 0;
        if (s_err) bad = true;
    }
    if (t == 0) {
        a.ctr[G_NA] = na;
        a.ctr[G_K] = k;
        a.ctr[G_SWAP] = (act == a.act) ? 0 : 1;
    }
    if (threadIdx.x == 0 && (bad || s_err)) a.ctr[G_ERR] = 1;
}

__global__ void k_alive_internal(const uint8_t* by_caller, const int32_t* orig_of, int64_t n, uint8_t* by_internal) {
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v < n) by_internal[v] = by_caller[orig_of[v]] ? 1 : 0;
}

__global__ void k_core_caller(const int32_t* core, const int32_t* orig_of, int64_t n, int64_t* by_caller) {
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v < n) by_caller[orig_of[v]] = core[v] == kOutside ? -1 : core[v];
}

int32_t d2h_i32(const int32_t* p, hipStream_t s) {
    int32_t v = 0;
    LDS_HIP(hipMemcpyAsync(&v, p, sizeof(v), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    return v;
}

}  // namespace

void core_numbers_gpu(Graph& g, int mode, const uint8_t* alive, int32_t* core, hipStream_t s) {
    const int64_t n = g.n;
    if (n == 0) return;
    LDS_CHECK(n < INT32_MAX, ST_INVALID, "too many vertices");
    if (mode == 3 && g.T < 0) list_triangles(g, s);
    DBuf<int32_t> cnt, act, act2, front, next, ctr;
    DBuf<uint32_t> talive;
    cnt.alloc(n, s);
    act.alloc(n, s);
    act2.alloc(n, s);
    front.alloc(n, s);
    next.alloc(n, s);
    ctr.alloc(8, s);  // C_* counters; [7] error flag of the one-workgroup tail
    k_fill8<<<1, 8, 0, s>>>(ctr.p);
    if (mode == 2) {
        k_init_edges<<<grid_for(n, kT), kT, 0, s>>>(g.rowptr.p, g.col.p, n, alive, cnt.p, core, act.p, ctr.p);
    } else {
        k_init_vertices<<<grid_for(n, kT), kT, 0, s>>>(n, alive, cnt.p, core, act.p, ctr.p);
        if (g.T > 0) {
            talive.alloc(g.T, s);
            k_init_triangles<<<grid_for(g.T, kT), kT, 0, s>>>(g.tri.p, g.T, alive, cnt.p, talive.p);
        }
    }
    LDS_HIP(hipGetLastError());
    const SweepPlan& tp = g.tri_plan;
    int32_t h[8];
    LDS_HIP(hipMemcpyAsync(h, ctr.p, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    int32_t na = h[C_NA], k = 0;
    if (na > kTailMax) {  // the levels with many vertices: one cooperative launch
        static int cus = 0, per[2] = {0, 0};
        if (!cus) {
            int dev = 0;
            LDS_HIP(hipGetDevice(&dev));
            LDS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            LDS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per[0], k_peel_grid<false>, kPT, 0));
            LDS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per[1], k_peel_grid<true>, kPT, 0));
        }
        // at most kPeelMaxWG workgroups, one per 16384 vertices; LDS_PEEL_WG
        // overrides both (e.g. to run the grid protocol wide on small graphs)
        const char* ev = std::getenv("LDS_PEEL_WG");
        const int64_t forced = (ev && *ev) ? std::max<int64_t>(2, std::atoll(ev)) : 0;
        const int64_t resident = (int64_t)cus * std::max(1, per[mode == 2 ? 0 : 1]);
        const int64_t grid = std::max<int64_t>(
            2, std::min<int64_t>({resident, forced ? forced : kPeelMaxWG, forced ? resident : (na + 16383) / 16384}));
        LDS_CHECK(resident >= 2, ST_DEVICE, "core peeling: the device cannot hold a cooperative grid");
        DBuf<int32_t> gc;
        DBuf<unsigned> bar;
        gc.alloc(16, s);
        bar.alloc(2, s);
        k_fill16<<<1, 16, 0, s>>>(gc.p, 0);
        k_set<<<1, 1, 0, s>>>(gc.p + G_MIN, INT32_MAX);
        k_set<<<1, 1, 0, s>>>(gc.p + G_MIN + 1, INT32_MAX);
        k_fill16<<<1, 2, 0, s>>>((int32_t*)bar.p, 0);
        LDS_HIP(hipGetLastError());
        PeelArgs pa{};
        pa.rowptr = g.rowptr.p;
        pa.col = g.col.p;
        pa.row_of = tp.own_row_of.p;
        pa.rp = tp.rp;
        pa.py = tp.py;
        pa.tos = tp.own_tos.p;
        pa.talive = talive.p;
        pa.cnt = cnt.p;
        pa.core = core;
        pa.act = act.p;
        pa.act2 = act2.p;
        pa.front = front.p;
        pa.next = next.p;
        pa.ctr = gc.p;
        pa.bar = bar.p;
        pa.n = n;
        pa.na = na;
        pa.k = 0;
        pa.tail_max = kTailMax;
        void* kargs[] = {&pa};
        LDS_HIP(hipLaunchCooperativeKernel(mode == 2 ? (const void*)k_peel_grid<false> : (const void*)k_peel_grid<true>,
                                           dim3((unsigned)grid), dim3(kPT), kargs, 0, s));
        int32_t hg[16];
        LDS_HIP(hipMemcpyAsync(hg, gc.p, sizeof(hg), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
        LDS_CHECK(hg[G_ERR] == 0, ST_DEVICE, "core peeling: no progress or a grid barrier did not complete");
        na = hg[G_NA];
        k = hg[G_K];
        if (hg[G_SWAP]) std::swap(act.p, act2.p);
    }
    if (na > 0) {  // the rest in one workgroup
        LDS_CHECK(na <= kTailMax, ST_DEVICE, "core peeling: too many vertices left for the one-workgroup tail");
        DBuf<int32_t> loc;
        loc.alloc(n, s);
        k_fill_i32<<<grid_for(n, kT), kT, 0, s>>>(loc.p, n, -1);
        k_set<<<1, 1, 0, s>>>(ctr.p + 7, 0);
        if (mode == 2)
            k_peel_tail<false><<<1, kTailT, 0, s>>>(act.p, na, k, loc.p, g.rowptr.p, g.col.p, nullptr, nullptr,
                                                    nullptr, nullptr, nullptr, cnt.p, core, ctr.p + 7);
        else
            k_peel_tail<true><<<1, kTailT, 0, s>>>(act.p, na, k, loc.p, nullptr, nullptr, tp.own_row_of.p, tp.rp,
                                                   tp.py, tp.own_tos.p, talive.p, cnt.p, core, ctr.p + 7);
        LDS_HIP(hipGetLastError());
        LDS_CHECK(d2h_i32(ctr.p + 7, s) == 0, ST_DEVICE, "core peeling: no progress");
    }
}

void core_numbers_caller(Graph& g, int mode, const uint8_t* alive_host, int64_t* core_host, hipStream_t s) {
    const int64_t n = g.n;
    if (mode == 3 && g.T < 0) list_triangles(g, s);
    if (n == 0) return;
    DBuf<uint8_t> al, ai;
    if (alive_host) {
        al.alloc(n, s);
        ai.alloc(n, s);
        LDS_HIP(hipMemcpyAsync(al.p, alive_host, n, hipMemcpyHostToDevice, s));
        k_alive_internal<<<grid_for(n, kT), kT, 0, s>>>(al.p, g.orig_of.p, n, ai.p);
        LDS_HIP(hipGetLastError());
    }
    DBuf<int32_t> core;
    DBuf<int64_t> out;
    core.alloc(n, s);
    out.alloc(n, s);
    core_numbers_gpu(g, mode, ai.p, core.p, s);
    k_core_caller<<<grid_for(n, kT), kT, 0, s>>>(core.p, g.orig_of.p, n, out.p);
    LDS_HIP(hipGetLastError());
    LDS_HIP(hipMemcpyAsync(core_host, out.p, n * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
}

}  // namespace lds
