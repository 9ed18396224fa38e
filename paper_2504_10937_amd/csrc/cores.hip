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
#include <climits>

#include "graph.hpp"

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

// Device-side counters of the level loop, read by the kernels themselves so
// that a level's kernels are queued without host round trips (grid-stride
// loops over counts held in memory).
enum : int { C_NA = 0, C_F0 = 1, C_F1 = 2, C_K = 3, C_MIN = 4, C_NA2 = 5 };

__global__ void k_level_begin(int32_t* ctr) {
    ctr[C_MIN] = INT32_MAX;
    ctr[C_F0] = 0;
    ctr[C_NA2] = 0;
}

// smallest count among the remaining vertices
__global__ void k_min_remaining(const int32_t* active, int32_t* ctr, const int32_t* cnt) {
    const int32_t na = ctr[C_NA];
    int32_t m = INT32_MAX;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < na; i += (int64_t)gridDim.x * kT)
        m = min(m, cnt[active[i]]);
    for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0 && m != INT32_MAX) atomicMin(&ctr[C_MIN], m);
}

// the level: k, or the smallest remaining count when no vertex is at or below k
__global__ void k_set_level(int32_t* ctr) {
    const int32_t m = ctr[C_MIN];
    if (m != INT32_MAX && m > ctr[C_K]) ctr[C_K] = m;
}

// remaining vertices with cnt <= k: core k, into the frontier
__global__ void k_frontier(const int32_t* active, int32_t* ctr, const int32_t* cnt, int32_t* core, int32_t* front) {
    const int32_t na = ctr[C_NA], k = ctr[C_K];
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < na; i += (int64_t)gridDim.x * kT) {
        const int32_t v = active[i];
        if (core[v] == kUnset && cnt[v] <= k) {
            core[v] = k;
            push(front, &ctr[C_F0], v);
        }
    }
}

__device__ inline void lower(int32_t* cnt, int32_t* core, int32_t w, int32_t k, int32_t* next, int32_t* nc) {
    if (core[w] != kUnset) return;
    const int32_t old = atomicSub(&cnt[w], 1);
    if (old == k + 1) {
        core[w] = k;
        push(next, nc, w);
    }
}

// one wave per frontier vertex; fc / nc are counters in memory
__global__ void k_peel_edges(const int32_t* front, const int32_t* fcp, const int64_t* rowptr, const int32_t* col,
                             int32_t* cnt, int32_t* core, const int32_t* ctr, int32_t* next, int32_t* ncp) {
    const int lane = threadIdx.x & 63;
    const int32_t fc = *fcp, k = ctr[C_K];
    for (int64_t i = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6); i < fc; i += (int64_t)gridDim.x * (kT / 64)) {
        const int32_t v = front[i];
        for (int64_t s = rowptr[v] + lane; s < rowptr[v + 1]; s += 64) lower(cnt, core, col[s], k, next, ncp);
    }
}

__global__ void k_peel_triangles(const int32_t* front, const int32_t* fcp, const int32_t* row_of, const int64_t* rp,
                                 const int32_t* py, const int32_t* tos, uint32_t* talive, int32_t* cnt,
                                 int32_t* core, const int32_t* ctr, int32_t* next, int32_t* ncp) {
    const int lane = threadIdx.x & 63;
    const int32_t fc = *fcp, k = ctr[C_K];
    for (int64_t i = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6); i < fc; i += (int64_t)gridDim.x * (kT / 64)) {
        const int32_t r = row_of[front[i]];
        if (r < 0) continue;
        for (int64_t s = rp[r] + lane; s < rp[r + 1]; s += 64) {
            if (atomicExch(&talive[tos[s]], 0u) == 0u) continue;  // killed before
            lower(cnt, core, py[2 * s], k, next, ncp);
            lower(cnt, core, py[2 * s + 1], k, next, ncp);
        }
    }
}

__global__ void k_compact(const int32_t* active, int32_t* ctr, const int32_t* core, int32_t* out) {
    const int32_t na = ctr[C_NA];
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < na; i += (int64_t)gridDim.x * kT) {
        const int32_t v = active[i];
        if (core[v] == kUnset) push(out, &ctr[C_NA2], v);
    }
}

__global__ void k_level_end(int32_t* ctr) {
    ctr[C_NA] = ctr[C_NA2];
    ctr[C_K] += 1;
}

__global__ void k_set(int32_t* p, int32_t v) { *p = v; }
__global__ void k_fill8(int32_t* p) { p[threadIdx.x] = 0; }

// The rest of the peeling in one workgroup once few vertices remain (small
// graphs from the start, the dense cores of large ones, the residual graphs of
// Pruning rule 2): the same levels, frontiers and cascades, separated by
// workgroup barriers instead of host round trips.  Every level assigns a
// vertex or jumps to a larger count, so the loops are bounded by the number
// of remaining vertices; a bound that is ever reached raises err.
constexpr int kTailT = 1024;
constexpr int32_t kTailMax = 1 << 13;

template <bool TRI>
__global__ __launch_bounds__(kTailT) void k_peel_tail(int32_t* act, int32_t* act2, int32_t na, int32_t k,
                                                      int32_t* front, int32_t* next, const int64_t* rowptr,
                                                      const int32_t* col, const int32_t* row_of, const int64_t* rp,
                                                      const int32_t* py, const int32_t* tos, uint32_t* talive,
                                                      int32_t* cnt, int32_t* core, int32_t* err) {
    __shared__ int32_t sc[4];  // [0] frontier, [1] next, [2] minimum, [3] remaining
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int64_t bound = 2 * (int64_t)na + 2;
    for (int64_t it = 0; na > 0; ++it) {
        if (it > bound) {
            if (tid == 0) *err = 1;
            return;
        }
        if (tid == 0) sc[0] = 0;
        __syncthreads();
        for (int32_t i = tid; i < na; i += kTailT) {
            const int32_t v = act[i];
            if (core[v] == kUnset && cnt[v] <= k) {
                core[v] = k;
                front[atomicAdd(&sc[0], 1)] = v;
            }
        }
        __syncthreads();
        int32_t fc = sc[0];
        if (fc == 0) {  // jump to the smallest remaining count
            if (tid == 0) sc[2] = INT32_MAX;
            __syncthreads();
            for (int32_t i = tid; i < na; i += kTailT) {
                const int32_t v = act[i];
                if (core[v] == kUnset) atomicMin(&sc[2], cnt[v]);
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
        int32_t* f = front;
        int32_t* nx = next;
        for (int64_t round = 0; fc > 0; ++round) {
            if (round > na) {
                if (tid == 0) *err = 1;
                return;
            }
            if (tid == 0) sc[1] = 0;
            __syncthreads();
            for (int32_t i = wv; i < fc; i += kTailT / 64) {
                const int32_t v = f[i];
                if (!TRI) {
                    for (int64_t q = rowptr[v] + lane; q < rowptr[v + 1]; q += 64) {
                        const int32_t w = col[q];
                        if (core[w] != kUnset) continue;
                        if (atomicSub(&cnt[w], 1) == k + 1) {
                            core[w] = k;
                            nx[atomicAdd(&sc[1], 1)] = w;
                        }
                    }
                } else {
                    const int32_t r = row_of[v];
                    if (r < 0) continue;
                    for (int64_t q = rp[r] + lane; q < rp[r + 1]; q += 64) {
                        if (atomicExch(&talive[tos[q]], 0u) == 0u) continue;
                        for (int j = 0; j < 2; ++j) {
                            const int32_t w = py[2 * q + j];
                            if (core[w] != kUnset) continue;
                            if (atomicSub(&cnt[w], 1) == k + 1) {
                                core[w] = k;
                                nx[atomicAdd(&sc[1], 1)] = w;
                            }
                        }
                    }
                }
            }
            __syncthreads();
            fc = sc[1];
            int32_t* tmp = f;
            f = nx;
            nx = tmp;
            __syncthreads();
        }
        if (tid == 0) sc[3] = 0;
        __syncthreads();
        for (int32_t i = tid; i < na; i += kTailT) {
            const int32_t v = act[i];
            if (core[v] == kUnset) act2[atomicAdd(&sc[3], 1)] = v;
        }
        __syncthreads();
        na = sc[3];
        int32_t* tmp = act;
        act = act2;
        act2 = tmp;
        ++k;
        __syncthreads();
    }
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
    // levels: one host read at the start of a level and one per four cascade
    // rounds; the rest of a level is queued without waiting
    const unsigned ge = std::min<unsigned>(grid_for(n, kT), 2048u);       // element loops
    const unsigned gw = std::min<unsigned>(grid_for(n, kT / 64), 4096u);  // one wave per vertex
    int32_t* fr[2] = {front.p, next.p};
    int32_t h[8];
    auto read_ctr = [&]() {
        LDS_HIP(hipMemcpyAsync(h, ctr.p, 8 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
    };
    for (int64_t level = 0;; ++level) {
        read_ctr();
        const int32_t na = h[C_NA], k = h[C_K];
        if (na == 0) break;
        LDS_CHECK(level <= n, ST_DEVICE, "core peeling: no progress");
        if (na <= kTailMax) {  // the rest in one workgroup, no host round trips
            k_set<<<1, 1, 0, s>>>(ctr.p + 7, 0);
            if (mode == 2)
                k_peel_tail<false><<<1, kTailT, 0, s>>>(act.p, act2.p, na, k, front.p, next.p, g.rowptr.p, g.col.p,
                                                        nullptr, nullptr, nullptr, nullptr, nullptr, cnt.p, core,
                                                        ctr.p + 7);
            else
                k_peel_tail<true><<<1, kTailT, 0, s>>>(act.p, act2.p, na, k, front.p, next.p, nullptr, nullptr,
                                                       tp.own_row_of.p, tp.rp, tp.py, tp.own_tos.p, talive.p, cnt.p,
                                                       core, ctr.p + 7);
            LDS_HIP(hipGetLastError());
            LDS_CHECK(d2h_i32(ctr.p + 7, s) == 0, ST_DEVICE, "core peeling: no progress");
            break;
        }
        k_level_begin<<<1, 1, 0, s>>>(ctr.p);
        k_min_remaining<<<ge, kT, 0, s>>>(act.p, ctr.p, cnt.p);
        k_set_level<<<1, 1, 0, s>>>(ctr.p);
        k_frontier<<<ge, kT, 0, s>>>(act.p, ctr.p, cnt.p, core, fr[0]);
        LDS_HIP(hipGetLastError());
        for (int64_t r = 0;;) {
            for (int j = 0; j < 4; ++j, ++r) {
                const int cur = (int)(r & 1), nx = cur ^ 1;
                k_set<<<1, 1, 0, s>>>(ctr.p + C_F0 + nx, 0);
                if (mode == 2)
                    k_peel_edges<<<gw, kT, 0, s>>>(fr[cur], ctr.p + C_F0 + cur, g.rowptr.p, g.col.p, cnt.p, core,
                                                   ctr.p, fr[nx], ctr.p + C_F0 + nx);
                else
                    k_peel_triangles<<<gw, kT, 0, s>>>(fr[cur], ctr.p + C_F0 + cur, tp.own_row_of.p, tp.rp, tp.py,
                                                       tp.own_tos.p, talive.p, cnt.p, core, ctr.p, fr[nx],
                                                       ctr.p + C_F0 + nx);
                LDS_HIP(hipGetLastError());
            }
            read_ctr();
            if (h[C_F0 + (int)(r & 1)] == 0) break;  // the frontier the next round would take
            LDS_CHECK(r <= (int64_t)na + 8, ST_DEVICE, "core peeling: no progress");
        }
        k_compact<<<ge, kT, 0, s>>>(act.p, ctr.p, core, act2.p);
        k_level_end<<<1, 1, 0, s>>>(ctr.p);
        LDS_HIP(hipGetLastError());
        std::swap(act.p, act2.p);
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
