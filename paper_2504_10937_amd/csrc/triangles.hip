// Triangle listing for the triangle-density program (Eq. trcp, Alg. 6 use
// the triangle set T; the paper does not say how T is obtained), and
// 4-clique listing for the h-clique program that Eq. trcp generalises.
//
// Orientation: internal ids are sorted by degree (descending), so orienting
// every edge towards the smaller internal id points it at the endpoint of
// larger degree; out-lists N+(x) = {y in N(x) : y < x} are the prefixes of
// the ascending CSR rows and have length O(sqrt(m)).  A triangle with
// internal ids a > b > c is found exactly once, from the oriented edge
// (a -> b), as the element c of N+(a) ∩ N+(b).
//
// Per oriented edge, one thread probes the shorter out-list against the
// longer one by binary search.  A count pass, an exclusive scan and a write
// pass give a deterministic order (oriented edges in CSR order, c ascending).
// The incidence CSR for the Frank-Wolfe pull sweep then holds, for every
// vertex with t_u > 0 (rows ordered by t_u descending), the other two
// vertices of each of its triangles, in triangle order.
#include "graph.hpp"

namespace lds {

namespace {

constexpr int kT = 256;

__device__ inline int64_t lower_bound_i32(const int32_t* a, int64_t lo, int64_t hi, int32_t x) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// out-degree of every vertex: number of neighbours with a smaller internal id
__global__ void k_outdeg(const int64_t* rp, const int32_t* col, int64_t n, int32_t* outdeg) {
    const int64_t u = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (u >= n) return;
    outdeg[u] = (int32_t)(lower_bound_i32(col, rp[u], rp[u + 1], (int32_t)u) - rp[u]);
}

// slot s of row u is an oriented edge u -> v iff v < u; emit / count the
// common out-neighbours of u and v (all are < v since N+(v) < v)
template <bool WRITE>
__global__ void k_tri_edges(const int64_t* rp, const int32_t* col, const int32_t* outdeg, int64_t n, int64_t ns,
                            uint32_t* cnt, const uint64_t* off, int32_t* tri) {
    const int64_t s = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (s >= ns) return;
    // row of slot s
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= s) lo = mid; else hi = mid - 1;
    }
    const int32_t u = (int32_t)lo;
    const int32_t v = col[s];
    uint32_t c = 0;
    if (v < u) {
        const int64_t ua = rp[u], ub = rp[u] + outdeg[u];
        const int64_t va = rp[v], vb = rp[v] + outdeg[v];
        // probe the shorter list against the longer
        const bool ushort = (ub - ua) <= (vb - va);
        const int64_t pa = ushort ? ua : va, pb = ushort ? ub : vb;
        const int64_t qa = ushort ? va : ua, qb = ushort ? vb : ub;
        uint64_t o = WRITE ? off[s] : 0;
        int64_t q = qa;
        for (int64_t i = pa; i < pb; ++i) {
            const int32_t w = col[i];
            if (w >= v) break;  // lists ascending; common elements are < v
            q = lower_bound_i32(col, q, qb, w);
            if (q < qb && col[q] == w) {
                if (WRITE) {
                    tri[3 * o + 0] = u;
                    tri[3 * o + 1] = v;
                    tri[3 * o + 2] = w;
                    ++o;
                }
                ++c;
            }
        }
    }
    if (!WRITE) cnt[s] = c;
}

__global__ void k_tcount(const int32_t* tri, int64_t T, int32_t* tc) {
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= T) return;
    atomicAdd(&tc[tri[3 * t]], 1);
    atomicAdd(&tc[tri[3 * t + 1]], 1);
    atomicAdd(&tc[tri[3 * t + 2]], 1);
}

__global__ void k_tmax(const int32_t* tc, int64_t n, int* out, unsigned long long* nz) {
    // grid-stride (the launch is capped at kReduceWG workgroups): one atomic
    // per wave on each of the two counters; with a wave per 64 entries the
    // waves of a 4M-entry array queued ~125k atomics on two addresses (0.75 ms)
    int d = 0;
    unsigned c = 0;  // entries > 0 (fewer than 2^32)
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        const int x = tc[i];
        d = max(d, x);
        c += x > 0 ? 1 : 0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        d = max(d, __shfl_xor(d, off, 64));
        c += (unsigned)__shfl_xor((int)c, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(out, d);
        if (c) atomicAdd(nz, (unsigned long long)c);
    }
}

// rows: vertices with t > 0 ordered by t descending, internal id ascending
__global__ void k_row_keys(const int32_t* tc, int64_t n, int vb, int32_t tmax, uint64_t* keys) {
    const int64_t u = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (u >= n) return;
    // vertices without triangles sort last (key above every t > 0 key)
    const uint64_t t = (uint64_t)tc[u];
    keys[u] = ((t > 0 ? (uint64_t)(tmax - (int32_t)t) : (uint64_t)tmax) << vb) | (uint64_t)u;
}

__global__ void k_row_apply(const uint64_t* keys, int64_t nrows, int vb, const int32_t* tc, int32_t* rid,
                            int32_t* row_of, uint32_t* rcount) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= nrows) return;
    const int32_t u = (int32_t)(keys[r] & ((1ull << vb) - 1));
    rid[r] = u;
    row_of[u] = (int32_t)r;
    rcount[r] = (uint32_t)tc[u];
}

template <int H>
__global__ void k_inc_keys(const int32_t* pat, int64_t np, const int32_t* row_of, int tb, uint64_t* keys) {
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= np) return;
    for (int j = 0; j < H; ++j) keys[H * t + j] = ((uint64_t)row_of[pat[H * t + j]] << tb) | (uint64_t)t;
}

// slot s: the other H-1 members of its pattern, in pattern order
template <int H>
__global__ void k_inc_pay(const uint64_t* keys, int64_t ns, int tb, const int32_t* pat, const int32_t* rid,
                          int32_t* pay, int32_t* tos) {
    const int64_t s = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (s >= ns) return;
    const uint64_t k = keys[s];
    const int64_t t = (int64_t)(k & ((1ull << tb) - 1));
    const int32_t x = rid[k >> tb];
    int o = 0;
    for (int j = 0; j < H; ++j) {
        const int32_t y = pat[H * t + j];
        if (y != x) pay[(H - 1) * s + o++] = y;
    }
    tos[s] = (int32_t)t;
}

__global__ void k_set_last(int64_t* rowptr, int64_t idx, const uint64_t* total) { rowptr[idx] = (int64_t)*total; }

// 4-cliques: a clique with internal ids a > b > c > d is found exactly once,
// from its triangle (a, b, c), as the element d of N+(a) ∩ N+(b) ∩ N+(c)
// (all of N+(c) lies below c).  One thread per triangle walks the shortest
// of the three out-lists cut at c and probes the other two by binary search
// with advancing lower bounds; a count pass, a scan and a write pass give
// the order (triangle order, d ascending).
template <bool WRITE>
__global__ void k_clique_tris(const int64_t* rp, const int32_t* col, const int32_t* tri, int64_t T, uint32_t* cnt,
                              const uint64_t* off, int32_t* q4) {
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= T) return;
    const int32_t x[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};  // a > b > c
    const int32_t c = x[2];
    int64_t lo[3], hi[3];
    for (int j = 0; j < 3; ++j) {
        lo[j] = rp[x[j]];
        hi[j] = lower_bound_i32(col, rp[x[j]], rp[x[j] + 1], c);  // neighbours below c
    }
    int sh = 0;
    for (int j = 1; j < 3; ++j)
        if (hi[j] - lo[j] < hi[sh] - lo[sh]) sh = j;
    const int o1 = sh == 0 ? 1 : 0, o2 = sh == 2 ? 1 : 2;
    int64_t q1 = lo[o1], q2 = lo[o2];
    uint64_t o = WRITE ? off[t] : 0;
    uint32_t k = 0;
    for (int64_t i = lo[sh]; i < hi[sh]; ++i) {
        const int32_t d = col[i];
        q1 = lower_bound_i32(col, q1, hi[o1], d);
        if (q1 >= hi[o1]) break;
        if (col[q1] != d) continue;
        q2 = lower_bound_i32(col, q2, hi[o2], d);
        if (q2 >= hi[o2]) break;
        if (col[q2] != d) continue;
        if (WRITE) {
            q4[4 * o + 0] = x[0];
            q4[4 * o + 1] = x[1];
            q4[4 * o + 2] = x[2];
            q4[4 * o + 3] = d;
            ++o;
        }
        ++k;
    }
    if (!WRITE) cnt[t] = k;
}

// per-vertex 4-clique counts.  Internal ids are ordered by degree, so the
// vertices in most cliques have the smallest ids: their counts are kept in
// an LDS histogram per workgroup (one global atomic per workgroup and hub at
// the end) instead of millions of atomics on a few addresses.
constexpr int kHubIds = 8192;
__global__ __launch_bounds__(kT) void k_qcount(const int32_t* q4, int64_t Q, int32_t* qc) {
    __shared__ int32_t hist[kHubIds];
    for (int i = threadIdx.x; i < kHubIds; i += kT) hist[i] = 0;
    __syncthreads();
    for (int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x; t < Q; t += (int64_t)gridDim.x * kT)
        for (int j = 0; j < 4; ++j) {
            const int32_t v = q4[4 * t + j];
            if (v < kHubIds)
                atomicAdd(&hist[v], 1);
            else
                atomicAdd(&qc[v], 1);
        }
    __syncthreads();
    for (int i = threadIdx.x; i < kHubIds; i += kT)
        if (hist[i]) atomicAdd(&qc[i], hist[i]);
}

template <class T>
T d2h(const T* p, hipStream_t s) {
    T v;
    LDS_HIP(hipMemcpyAsync(&v, p, sizeof(T), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    return v;
}

// Incidence CSR of a pattern list (H vertices per pattern) for the pull
// sweep: rows are the vertices with count > 0 ordered by count descending
// (internal id ascending), each row holding, for every pattern at the
// vertex, the other H-1 members (in pattern order), patterns in list order.
template <int H>
void build_incidence_plan(Graph& g, const int32_t* pat, int64_t np, const int32_t* count, SweepPlan& p,
                          int64_t& cmax, hipStream_t s) {
    const int64_t n = g.n;
    LDS_CHECK(np < (int64_t)INT32_MAX, ST_OVERFLOW, "too many patterns for 32-bit pattern indices");
    p.h = H;
    DBuf<int> tmax;
    DBuf<unsigned long long> nz;
    tmax.alloc(1, s);
    nz.alloc(1, s);
    LDS_HIP(hipMemsetAsync(tmax.p, 0, sizeof(int), s));
    LDS_HIP(hipMemsetAsync(nz.p, 0, sizeof(unsigned long long), s));
    if (n > 0) {
        k_tmax<<<std::min(grid_for(n, kT), kReduceWG), kT, 0, s>>>(count, n, tmax.p, nz.p);
        LDS_HIP(hipGetLastError());
    }
    cmax = d2h(tmax.p, s);
    const int64_t nrows = (int64_t)d2h(nz.p, s);
    p.nrows = nrows;
    p.nslots = H * np;
    p.own_rid.alloc(nrows, s);
    p.own_rp.alloc(nrows + 1, s);
    p.own_py.alloc((H - 1) * H * np, s);
    DBuf<int32_t>& row_of = p.own_row_of;
    row_of.alloc(n, s);
    if (n) LDS_HIP(hipMemsetAsync(row_of.p, 0xff, n * sizeof(int32_t), s));  // -1: no pattern
    DBuf<uint32_t> rcount;
    rcount.alloc(nrows, s);
    if (nrows > 0) {
        const int vb = g.vbits;
        DBuf<uint64_t> rk, rt;
        rk.alloc(n, s);
        rt.alloc(n, s);
        k_row_keys<<<grid_for(n, kT), kT, 0, s>>>(count, n, vb, (int32_t)cmax, rk.p);
        LDS_HIP(hipGetLastError());
        radix_sort_u64(rk.p, nullptr, n, vb + bits_for((uint64_t)cmax), rt.p, nullptr, s);
        k_row_apply<<<grid_for(nrows, kT), kT, 0, s>>>(rk.p, nrows, vb, count, p.own_rid.p, row_of.p, rcount.p);
        LDS_HIP(hipGetLastError());
    }
    DBuf<uint64_t> tot;
    tot.alloc(1, s);
    exclusive_scan_u32_to_u64(rcount.p, (uint64_t*)p.own_rp.p, nrows, tot.p, s);
    k_set_last<<<1, 1, 0, s>>>(p.own_rp.p, nrows, tot.p);
    LDS_HIP(hipGetLastError());
    if (np > 0) {
        const int tb = bits_for((uint64_t)(np - 1)) > 0 ? bits_for((uint64_t)(np - 1)) : 1;
        const int rb = bits_for((uint64_t)nrows);
        LDS_CHECK(tb + rb <= 64, ST_OVERFLOW, "pattern incidence key exceeds 64 bits");
        DBuf<uint64_t> ik, it;
        ik.alloc(H * np, s);
        it.alloc(H * np, s);
        k_inc_keys<H><<<grid_for(np, kT), kT, 0, s>>>(pat, np, row_of.p, tb, ik.p);
        LDS_HIP(hipGetLastError());
        radix_sort_u64(ik.p, nullptr, H * np, tb + rb, it.p, nullptr, s);
        p.own_tos.alloc(H * np, s);
        k_inc_pay<H><<<grid_for(H * np, kT), kT, 0, s>>>(ik.p, H * np, tb, pat, p.own_rid.p, p.own_py.p,
                                                       p.own_tos.p);
        LDS_HIP(hipGetLastError());
    }
    p.rid = p.own_rid.p;
    p.rp = p.own_rp.p;
    p.py = p.own_py.p;
    build_sweep_plan(p, s);
}

}  // namespace

namespace {
// triangles at each vertex, from the incidence rows (a row's slots are in
// ascending triangle order, so each list is too)
__global__ void k_vtx_tcount(const int32_t* row_of, const int64_t* rp, int64_t n, uint64_t* cnt) {
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    const int32_t r = row_of[v];
    cnt[v] = r < 0 ? 0 : (uint64_t)(rp[r + 1] - rp[r]);
}

__global__ void k_vtx_tfill(const int32_t* rid, const int64_t* rp, int64_t nrows, const int32_t* tos,
                            const uint64_t* off, int32_t* tinc) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (r >= nrows) return;
    const int64_t base = (int64_t)off[rid[r]] - rp[r];
    for (int64_t q = rp[r] + lane; q < rp[r + 1]; q += 64) tinc[base + q] = tos[q];
}
}  // namespace

void vertex_triangle_lists(const Graph& g, int64_t* trp_host, int32_t* tinc_host, hipStream_t s) {
    const int64_t n = g.n;
    LDS_CHECK(g.T >= 0, ST_INVALID, "triangles are not listed");
    if (n == 0) return;
    const SweepPlan& p = g.tri_plan;
    DBuf<uint64_t> off;
    off.alloc(n + 1, s);
    k_vtx_tcount<<<grid_for(n, kT), kT, 0, s>>>(p.own_row_of.p, p.rp, n, off.p);
    LDS_HIP(hipGetLastError());
    exclusive_scan_u64(off.p, off.p, n, off.p + n, s);
    DBuf<int32_t> tinc;
    tinc.alloc(3 * g.T, s);
    if (g.T > 0 && p.nrows > 0) {
        k_vtx_tfill<<<grid_for(p.nrows, kT / 64), kT, 0, s>>>(p.rid, p.rp, p.nrows, p.own_tos.p, off.p, tinc.p);
        LDS_HIP(hipGetLastError());
    }
    LDS_HIP(hipMemcpyAsync(trp_host, off.p, (n + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (g.T > 0) LDS_HIP(hipMemcpyAsync(tinc_host, tinc.p, 3 * g.T * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
}

void list_triangles(Graph& g, hipStream_t s) {
    const int64_t n = g.n, ns = 2 * g.m;
    sort_rows(g, s);
    g.tcount.alloc(n, s);
    if (n) LDS_HIP(hipMemsetAsync(g.tcount.p, 0, n * sizeof(int32_t), s));
    int64_t T = 0;
    if (ns > 0) {
        DBuf<int32_t> outdeg;
        outdeg.alloc(n, s);
        k_outdeg<<<grid_for(n, kT), kT, 0, s>>>(g.rowptr.p, g.col.p, n, outdeg.p);
        LDS_HIP(hipGetLastError());
        DBuf<uint32_t> cnt;
        DBuf<uint64_t> off, tot;
        cnt.alloc(ns, s);
        off.alloc(ns, s);
        tot.alloc(1, s);
        k_tri_edges<false><<<grid_for(ns, kT), kT, 0, s>>>(g.rowptr.p, g.col.p, outdeg.p, n, ns, cnt.p, nullptr,
                                                         nullptr);
        LDS_HIP(hipGetLastError());
        exclusive_scan_u32_to_u64(cnt.p, off.p, ns, tot.p, s);
        T = (int64_t)d2h(tot.p, s);
        cnt.release();
        g.tri.alloc(3 * T, s);
        if (T > 0) {
            k_tri_edges<true><<<grid_for(ns, kT), kT, 0, s>>>(g.rowptr.p, g.col.p, outdeg.p, n, ns, nullptr, off.p,
                                                            g.tri.p);
            LDS_HIP(hipGetLastError());
            k_tcount<<<grid_for(T, kT), kT, 0, s>>>(g.tri.p, T, g.tcount.p);
            LDS_HIP(hipGetLastError());
        }
    }
    g.T = T;
    build_incidence_plan<3>(g, g.tri.p, T, g.tcount.p, g.tri_plan, g.t_max, s);
}

void list_cliques4(Graph& g, hipStream_t s) {
    if (g.T < 0) list_triangles(g, s);  // also sorts the rows
    const int64_t n = g.n, T = g.T;
    g.qcount.alloc(n, s);
    if (n) LDS_HIP(hipMemsetAsync(g.qcount.p, 0, n * sizeof(int32_t), s));
    int64_t Q = 0;
    if (T > 0) {
        DBuf<uint32_t> cnt;
        DBuf<uint64_t> off, tot;
        cnt.alloc(T, s);
        off.alloc(T, s);
        tot.alloc(1, s);
        k_clique_tris<false><<<grid_for(T, kT), kT, 0, s>>>(g.rowptr.p, g.col.p, g.tri.p, T, cnt.p, nullptr, nullptr);
        LDS_HIP(hipGetLastError());
        exclusive_scan_u32_to_u64(cnt.p, off.p, T, tot.p, s);
        Q = (int64_t)d2h(tot.p, s);
        cnt.release();
        g.q4.alloc(4 * Q, s);
        if (Q > 0) {
            k_clique_tris<true><<<grid_for(T, kT), kT, 0, s>>>(g.rowptr.p, g.col.p, g.tri.p, T, nullptr, off.p, g.q4.p);
            LDS_HIP(hipGetLastError());
            k_qcount<<<std::min<unsigned>(grid_for(Q, kT), 2048u), kT, 0, s>>>(g.q4.p, Q, g.qcount.p);
            LDS_HIP(hipGetLastError());
        }
    }
    g.Q4 = Q;
    build_incidence_plan<4>(g, g.q4.p, Q, g.qcount.p, g.clique_plan, g.q_max, s);
}

}  // namespace lds
