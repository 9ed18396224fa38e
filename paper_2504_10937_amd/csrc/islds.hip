// Device scoping of IsLDS (Alg. 4) and IsLTDS (Alg. 7 with ExtMaximal,
// Alg. 8): the search from the candidate S over the band of vertices whose
// bounds bracket rho = density(G[S]), the self-loops (edges) or truncated
// patterns (triangles) that stand for the vertices above the band, and the
// flow network of the region; only the min cut itself runs on the host.
//
// Per call: a flag per vertex (above: lower bound > rho; band: lower <= rho
// <= upper; below: upper < rho) from the exact bounds (128-bit cross
// products); the early rejection of S (a vertex of S outside the band or a
// neighbour above it); then a level-synchronous search, one wave per
// frontier vertex, that claims band vertices with an atomic compare-and-swap
// and counts the edges to vertices above (one self-loop each, edges) or
// collects each triangle once (an atomic exchange on its visit flag) whose
// members are all at or above the band.  The per-vertex scratch is cleared
// over the touched vertices only, so a call costs what it visits.
#include "islds.hpp"

namespace lds {

namespace {

constexpr int kT = 256;
constexpr uint8_t kAbove = 0, kBand = 1, kBelow = 2;

__device__ inline void push(int32_t* list, int32_t* count, int32_t v) { list[atomicAdd(count, 1)] = v; }

__global__ void k_flags(int64_t n, const int64_t* lon, const int64_t* lod, const int64_t* hin, const int64_t* hid,
                        int64_t rn, int64_t rd, uint8_t* flag) {
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    const __int128 r_lo = (__int128)rn * lod[v], lo_r = (__int128)lon[v] * rd;
    const __int128 r_hi = (__int128)rn * hid[v], hi_r = (__int128)hin[v] * rd;
    flag[v] = lo_r > r_lo ? kAbove : (hi_r < r_hi ? kBelow : kBand);
}

// a vertex of S outside the band, or a neighbour of S above it: not an LDS
__global__ void k_reject(const int32_t* S, int32_t ns, const int64_t* rowptr, const int32_t* col, const uint8_t* flag,
                         int32_t* bad) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (i >= ns) return;
    const int32_t v = S[i];
    bool b = flag[v] != kBand;
    for (int64_t s = rowptr[v] + lane; s < rowptr[v + 1] && !b; s += 64) b = flag[col[s]] == kAbove;
    if (__ballot(b) && lane == 0) *bad = 1;
}

__global__ void k_claim(const int32_t* S, int32_t ns, int32_t* inU, int32_t* U) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= ns) return;
    inU[S[i]] = 1;
    U[i] = S[i];
}

struct Level {
    const int32_t* front;
    int32_t nf;
    const int64_t* rowptr;
    const int32_t* col;
    const uint8_t* flag;
    int32_t* inU;
    int32_t* loops;    // edges: self-loops per vertex (edges to vertices above the band)
    int32_t* next;
    int32_t* U;
    int32_t* ctr;      // [0] |U|, [1] next frontier, [2] need flow, [3] visited triangles, [4] patterns
    // triangles
    const int32_t* row_of;
    const int64_t* trp;
    const int32_t* tos;
    const int32_t* tri;
    uint32_t* tvis;
    int32_t* tlist;    // every visited triangle (to clear tvis)
    int32_t* plist;    // visited triangles without a member below the band
};

__device__ inline void claim(const Level& a, int32_t w) {
    if (atomicCAS(&a.inU[w], 0, 1) == 0) {
        push(a.next, a.ctr + 1, w);
        push(a.U, a.ctr, w);
    }
}

template <bool TRI>
__global__ void k_level(Level a) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (i >= a.nf) return;
    const int32_t v = a.front[i];
    int32_t above = 0;
    for (int64_t s = a.rowptr[v] + lane; s < a.rowptr[v + 1]; s += 64) {
        const int32_t w = a.col[s];
        const uint8_t f = a.flag[w];
        if (f == kAbove)
            ++above;
        else if (f == kBand && a.inU[w] == 0)
            claim(a, w);
    }
    if (TRI) {
        const int32_t r = a.row_of[v];
        if (r >= 0)
            for (int64_t s = a.trp[r] + lane; s < a.trp[r + 1]; s += 64) {
                const int32_t t = a.tos[s];
                if (atomicExch(&a.tvis[t], 1u) != 0u) continue;
                push(a.tlist, a.ctr + 3, t);
                const int32_t x[3] = {a.tri[3 * t], a.tri[3 * t + 1], a.tri[3 * t + 2]};
                if (a.flag[x[0]] == kBelow || a.flag[x[1]] == kBelow || a.flag[x[2]] == kBelow) continue;
                push(a.plist, a.ctr + 4, t);
                for (int j = 0; j < 3; ++j) {
                    if (a.flag[x[j]] == kAbove)
                        a.ctr[2] = 1;
                    else if (a.inU[x[j]] == 0)
                        claim(a, x[j]);
                }
            }
    }
    for (int o = 32; o > 0; o >>= 1) above += __shfl_xor(above, o, 64);
    if (lane == 0 && above > 0) {
        a.ctr[2] = 1;
        if (!TRI) a.loops[v] = above;  // v is expanded once
    }
}

__global__ void k_loc(const int32_t* U, int32_t nu, int32_t* loc) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < nu) loc[U[i]] = (int32_t)i;
}

// edges of G[U] by local index (i < j), counted then written per U vertex
template <bool WRITE>
__global__ void k_pairs(const int32_t* U, int32_t nu, const int64_t* rowptr, const int32_t* col, const int32_t* loc,
                        uint32_t* cnt, const uint64_t* off, int32_t* pairs) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= nu) return;
    const int32_t v = U[i];
    uint64_t o = WRITE ? off[i] : 0;
    uint32_t c = 0;
    for (int64_t s = rowptr[v]; s < rowptr[v + 1]; ++s) {
        const int32_t j = loc[col[s]];
        if (j > (int32_t)i) {
            if (WRITE) {
                pairs[2 * o] = (int32_t)i;
                pairs[2 * o + 1] = j;
                ++o;
            }
            ++c;
        }
    }
    if (!WRITE) cnt[i] = c;
}

// triangle patterns by local index, -1 for members above the band
__global__ void k_tri_pat(const int32_t* plist, int32_t np, const int32_t* tri, const int32_t* loc, int32_t* pat) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= np) return;
    const int32_t t = plist[i];
    for (int j = 0; j < 3; ++j) pat[3 * i + j] = loc[tri[3 * t + j]];
}

__global__ void k_loops_of(const int32_t* U, int32_t nu, const int32_t* loops, int64_t* out) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < nu) out[i] = loops[U[i]];
}

__global__ void k_clear_u(const int32_t* U, int32_t nu, int32_t* inU, int32_t* loops, int32_t* loc) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= nu) return;
    const int32_t v = U[i];
    inU[v] = 0;
    loops[v] = 0;
    loc[v] = -1;
}

__global__ void k_clear_t(const int32_t* tl, int32_t nt, uint32_t* tvis) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < nt) tvis[tl[i]] = 0u;
}

__global__ void k_fill(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) p[i] = v;
}

// Pruning rule 1 (Alg. 3; Cor. uv-prune): u lies in no LDS when one of its
// neighbours has a lower bound above u's upper bound (then phi of that
// neighbour exceeds phi(u)).  One wave per vertex, bounds compared exactly.
__global__ void k_prune_rule1(const int64_t* rp, const int32_t* col, int64_t n, const int64_t* lon, const int64_t* lod,
                              const int64_t* hin, const int64_t* hid, uint8_t* alive, uint8_t* rule) {
    const int lane = threadIdx.x & 63;
    const int64_t u = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 6;
    if (u >= n) return;
    const __int128 hn = hin[u], hd = hid[u];
    bool hit = false;
    for (int64_t e = rp[u] + lane; e < rp[u + 1] && !hit; e += 64) {
        const int32_t w = col[e];
        hit = (__int128)lon[w] * hd > hn * (__int128)lod[w];
    }
    if (__ballot(hit) != 0ull && lane == 0) {
        alive[u] = 0;
        rule[u] = 1;
    }
}

// Pruning rule 2 (Alg. 3; Lemma uu-prune): u lies in no LDS when its core
// (tr-core) number in the residual graph is below its lower bound
__global__ void k_prune_rule2(const int32_t* core, int64_t n, const int64_t* lon, const int64_t* lod, uint8_t* alive,
                              uint8_t* rule, unsigned* changed) {
    const int64_t u = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (u >= n || !alive[u]) return;
    if ((__int128)core[u] * lod[u] < (__int128)lon[u]) {
        alive[u] = 0;
        rule[u] = 2;
        atomicAdd(changed, 1u);
    }
}

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u32(uint32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) p[i] = 0u;
}

template <class T>
void d2h(T* dst, const T* src, size_t count, hipStream_t s) {
    if (count) LDS_HIP(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyDeviceToHost, s));
}

}  // namespace

void scope_init(Graph& g, int mode, const int64_t* lon, const int64_t* lod, const int64_t* hin, const int64_t* hid,
                BandScope& b, hipStream_t s) {
    const int64_t n = g.n;
    LDS_CHECK(n < INT32_MAX, ST_INVALID, "too many vertices");
    b.mode = mode;
    b.n = n;
    b.T = (mode == 3 && g.T > 0) ? g.T : 0;
    if (n == 0) return;
    b.lon.alloc(n, s);
    b.lod.alloc(n, s);
    b.hin.alloc(n, s);
    b.hid.alloc(n, s);
    LDS_HIP(hipMemcpyAsync(b.lon.p, lon, n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    LDS_HIP(hipMemcpyAsync(b.lod.p, lod, n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    LDS_HIP(hipMemcpyAsync(b.hin.p, hin, n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    LDS_HIP(hipMemcpyAsync(b.hid.p, hid, n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    b.flag.alloc(n, s);
    b.inU.alloc(n, s);
    b.loops.alloc(n, s);
    b.loc.alloc(n, s);
    b.U.alloc(n, s);
    b.front.alloc(n, s);
    b.next.alloc(n, s);
    b.S.alloc(n, s);
    b.ctr.alloc(8, s);
    k_fill<<<grid_for(n, kT), kT, 0, s>>>(b.inU.p, n, 0);
    k_fill<<<grid_for(n, kT), kT, 0, s>>>(b.loops.p, n, 0);
    k_fill<<<grid_for(n, kT), kT, 0, s>>>(b.loc.p, n, -1);
    if (b.T > 0) {
        b.tvis.alloc(b.T, s);
        b.tlist.alloc(b.T, s);
        b.plist.alloc(b.T, s);
        k_fill_u32<<<grid_for(b.T, kT), kT, 0, s>>>(b.tvis.p, b.T);
    }
    LDS_HIP(hipGetLastError());
}

bool scope_band(Graph& g, BandScope& b, const std::vector<int32_t>& S, int64_t rn, int64_t rd, ScopeOut& o,
                hipStream_t s) {
    const int64_t n = b.n;
    const int32_t ns = (int32_t)S.size();
    o.need_flow = false;
    o.U.clear();
    o.loops.clear();
    o.pat.clear();
    if (ns == 0 || n == 0) return true;
    int32_t* ctr = b.ctr.p;
    k_fill<<<1, 8, 0, s>>>(ctr, 8, 0);
    k_flags<<<grid_for(n, kT), kT, 0, s>>>(n, b.lon.p, b.lod.p, b.hin.p, b.hid.p, rn, rd, b.flag.p);
    LDS_HIP(hipMemcpyAsync(b.S.p, S.data(), ns * sizeof(int32_t), hipMemcpyHostToDevice, s));
    k_reject<<<grid_for(ns, kT / 64), kT, 0, s>>>(b.S.p, ns, g.rowptr.p, g.col.p, b.flag.p, ctr + 5);
    LDS_HIP(hipGetLastError());
    int32_t h[8];
    d2h(h, ctr, 8, s);
    LDS_HIP(hipStreamSynchronize(s));
    if (h[5]) return false;
    k_claim<<<grid_for(ns, kT), kT, 0, s>>>(b.S.p, ns, b.inU.p, b.U.p);
    k_fill<<<1, 1, 0, s>>>(ctr, 1, ns);
    LDS_HIP(hipGetLastError());
    const SweepPlan& tp = g.tri_plan;
    Level a{};
    a.rowptr = g.rowptr.p;
    a.col = g.col.p;
    a.flag = b.flag.p;
    a.inU = b.inU.p;
    a.loops = b.loops.p;
    a.U = b.U.p;
    a.ctr = ctr;
    const bool tri = b.mode == 3 && b.T > 0;
    if (tri) {
        a.row_of = tp.own_row_of.p;
        a.trp = tp.rp;
        a.tos = tp.own_tos.p;
        a.tri = g.tri.p;
        a.tvis = b.tvis.p;
        a.tlist = b.tlist.p;
        a.plist = b.plist.p;
    }
    int32_t* cur = b.S.p;
    int32_t nf = ns;
    int32_t* nxt = b.next.p;
    int32_t* spare = b.front.p;
    while (nf > 0) {
        k_fill<<<1, 1, 0, s>>>(ctr + 1, 1, 0);
        a.front = cur;
        a.nf = nf;
        a.next = nxt;
        if (tri)
            k_level<true><<<grid_for(nf, kT / 64), kT, 0, s>>>(a);
        else
            k_level<false><<<grid_for(nf, kT / 64), kT, 0, s>>>(a);
        LDS_HIP(hipGetLastError());
        d2h(h, ctr, 8, s);
        LDS_HIP(hipStreamSynchronize(s));
        nf = h[1];
        cur = nxt;
        std::swap(nxt, spare);
    }
    const int32_t nu = h[0], nt = h[3], np = h[4];
    o.need_flow = h[2] != 0;
    if (o.need_flow) {
        o.U.resize(nu);
        d2h(o.U.data(), b.U.p, nu, s);
        k_loc<<<grid_for(nu, kT), kT, 0, s>>>(b.U.p, nu, b.loc.p);
        LDS_HIP(hipGetLastError());
        if (b.mode == 2) {
            DBuf<uint32_t> cnt;
            DBuf<uint64_t> off, tot;
            DBuf<int64_t> lp;
            cnt.alloc(nu, s);
            off.alloc(nu, s);
            tot.alloc(1, s);
            lp.alloc(nu, s);
            k_pairs<false><<<grid_for(nu, kT), kT, 0, s>>>(b.U.p, nu, g.rowptr.p, g.col.p, b.loc.p, cnt.p, nullptr,
                                                          nullptr);
            LDS_HIP(hipGetLastError());
            exclusive_scan_u32_to_u64(cnt.p, off.p, nu, tot.p, s);
            uint64_t m = 0;
            d2h(&m, tot.p, 1, s);
            LDS_HIP(hipStreamSynchronize(s));
            DBuf<int32_t> pairs;
            pairs.alloc(2 * m, s);
            if (m > 0) {
                k_pairs<true><<<grid_for(nu, kT), kT, 0, s>>>(b.U.p, nu, g.rowptr.p, g.col.p, b.loc.p, nullptr, off.p,
                                                             pairs.p);
                LDS_HIP(hipGetLastError());
            }
            k_loops_of<<<grid_for(nu, kT), kT, 0, s>>>(b.U.p, nu, b.loops.p, lp.p);
            LDS_HIP(hipGetLastError());
            o.pat.resize(2 * m);
            o.loops.resize(nu);
            d2h(o.pat.data(), pairs.p, 2 * m, s);
            d2h(o.loops.data(), lp.p, nu, s);
            LDS_HIP(hipStreamSynchronize(s));
        } else if (np > 0) {
            DBuf<int32_t> pat;
            pat.alloc(3 * (size_t)np, s);
            k_tri_pat<<<grid_for(np, kT), kT, 0, s>>>(b.plist.p, np, g.tri.p, b.loc.p, pat.p);
            LDS_HIP(hipGetLastError());
            o.pat.resize(3 * (size_t)np);
            d2h(o.pat.data(), pat.p, 3 * (size_t)np, s);
            LDS_HIP(hipStreamSynchronize(s));
        }
    }
    // clear the touched scratch for the next call
    k_clear_u<<<grid_for(nu, kT), kT, 0, s>>>(b.U.p, nu, b.inU.p, b.loops.p, b.loc.p);
    if (nt > 0) k_clear_t<<<grid_for(nt, kT), kT, 0, s>>>(b.tlist.p, nt, b.tvis.p);
    LDS_HIP(hipGetLastError());
    return true;
}

void prune_device(Graph& g, int mode, const BandScope& b, uint8_t* alive, uint8_t* rule, hipStream_t s) {
    const int64_t n = g.n;
    if (n == 0) return;
    k_fill_u8<<<grid_for(n, kT), kT, 0, s>>>(alive, n, 1);
    k_fill_u8<<<grid_for(n, kT), kT, 0, s>>>(rule, n, 0);
    k_prune_rule1<<<grid_for(n * 64, kT), kT, 0, s>>>(g.rowptr.p, g.col.p, n, b.lon.p, b.lod.p, b.hin.p, b.hid.p,
                                                      alive, rule);
    LDS_HIP(hipGetLastError());
    DBuf<int32_t> core;
    core.alloc(n, s);
    DBuf<unsigned> changed;
    changed.alloc(1, s);
    for (;;) {
        core_numbers_gpu(g, mode, alive, core.p, s);
        LDS_HIP(hipMemsetAsync(changed.p, 0, sizeof(unsigned), s));
        k_prune_rule2<<<grid_for(n, kT), kT, 0, s>>>(core.p, n, b.lon.p, b.lod.p, alive, rule, changed.p);
        LDS_HIP(hipGetLastError());
        unsigned ch = 0;
        LDS_HIP(hipMemcpyAsync(&ch, changed.p, sizeof(unsigned), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
        if (ch == 0) break;
    }
}

}  // namespace lds
