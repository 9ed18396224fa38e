// Frank-Wolfe iterations of Alg. 1 (edges, Eq. cp) and Alg. 6 (triangles,
// Eq. trcp) on gfx950, in exact integer form.
//
// State.  With gamma_i = 2/(i+2) every load is r_u^(i) = A_u / D_i with the
// common denominator D_i = (i+1)(i+2) (edges) or 3(i+1)(i+2) (triangles), and
// the update r <- (1-gamma) r + gamma b becomes A_u += inc_i * b_u with
// inc_i = D_i - D_{i-1} = 2(i+1) (edges) or 6(i+1) (triangles), b_u = units
// won in iteration i.  Each vertex carries one packed 64-bit key
//     K_u = (A_u << B) | (2^B - 1 - orig_id(u)),
// so "smallest load, ties to the larger original id" is a single unsigned
// compare, and adding (inc * b) << B updates A without touching the id bits.
//
// Sweep (one launch per iteration, keys ping-pong between two buffers so that
// every decision reads r^(i-1)).  Pull over incidence slots: a vertex wins a
// slot's pattern iff its key is below the keys of the other h-1 vertices.
//   * chunk waves: a wave64 streams one row-aligned chunk in 64-slot words;
//     the wave ballot of wins is the iteration's decision word for those
//     slots (stored once, coalesced); row-start flags turn the ballot into
//     per-row win counts with popcounts (segmented count, no atomics), and
//     the lane holding a row's last slot writes the row's new key.
//   * hub workgroups: one 256-thread workgroup per row with more slots than
//     a chunk; per-wave ballots, LDS reduction, one key write.
// The duality-gap terms sum_u A_u^2 and sum_u A_u b_u (= sum over patterns of
// the winning numerator, i.e. the minimum) are accumulated exactly in 128-bit
// integers per workgroup and reduced once after the last iteration.
#include "graph.hpp"

namespace lds {

namespace {

typedef unsigned __int128 u128;

struct SweepArgs {
    const int32_t* rid;
    const int64_t* rp;
    const int32_t* py;
    int64_t n_hub;
    const int64_t* hwo;
    int64_t n_chunks;
    const int64_t* chunk_row;
    const int64_t* cwo;
    const uint64_t* head;
    int64_t chunk_words;
    const uint64_t* Kin;
    uint64_t* Kout;
    uint64_t* bits;      // this iteration's decision words
    uint64_t inc;
    int B;
    uint64_t* partial;   // 4 words per workgroup (or nullptr)
};

__device__ inline uint64_t readlane64(uint64_t v, int lane) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t shfl_xor64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline u128 wave_sum128(u128 x) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        const uint64_t lo = shfl_xor64((uint64_t)x, m), hi = shfl_xor64((uint64_t)(x >> 64), m);
        x += ((u128)hi << 64) | lo;
    }
    return x;
}

// does the row vertex (key Ku) win the pattern stored at slot s?
template <int H>
__device__ inline bool slot_wins(const uint64_t* __restrict__ K, uint64_t Ku, const int32_t* __restrict__ py,
                                 int64_t s);
template <>
__device__ inline bool slot_wins<2>(const uint64_t* __restrict__ K, uint64_t Ku, const int32_t* __restrict__ py,
                                    int64_t s) {
    return Ku < K[py[s]];
}
template <>
__device__ inline bool slot_wins<3>(const uint64_t* __restrict__ K, uint64_t Ku, const int32_t* __restrict__ py,
                                    int64_t s) {
    const int2 p = reinterpret_cast<const int2*>(py)[s];
    return Ku < K[p.x] && Ku < K[p.y];
}

template <int H, bool IDENT, bool GAP>
__global__ __launch_bounds__(256) void k_fw_sweep(SweepArgs a) {
    __shared__ uint64_t red[4][4];
    __shared__ uint32_t hcnt[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    u128 sq = 0, mn = 0;
    if ((int64_t)blockIdx.x < a.n_hub) {
        // ---- hub row: one workgroup
        const int64_t r = blockIdx.x;
        const int32_t u = IDENT ? (int32_t)r : a.rid[r];
        const int64_t s0 = a.rp[r], s1 = a.rp[r + 1];
        const uint64_t Ku = a.Kin[u];
        uint64_t* bw = a.bits + a.chunk_words + a.hwo[r];
        uint32_t cnt = 0;
        for (int64_t base = s0; base < s1; base += 256) {
            const int64_t s = base + threadIdx.x;
            const bool win = (s < s1) && slot_wins<H>(a.Kin, Ku, a.py, s);
            const uint64_t W = __ballot(win);
            if (lane == 0 && base + 64 * w < s1) bw[(base - s0) / 64 + w] = W;
            cnt += (uint32_t)__popcll(W);
        }
        if (lane == 0) hcnt[w] = cnt;
        __syncthreads();
        if (threadIdx.x == 0) {
            const uint64_t tot = (uint64_t)hcnt[0] + hcnt[1] + hcnt[2] + hcnt[3];
            a.Kout[u] = Ku + ((tot * a.inc) << a.B);
            if (GAP) {
                const uint64_t A = Ku >> a.B;
                sq = (u128)A * A;
                mn = (u128)A * tot;
            }
        }
    } else {
        // ---- chunk: one wave64
        const int64_t c = ((int64_t)blockIdx.x - a.n_hub) * 4 + w;
        if (c < a.n_chunks) {
            const int64_t r0 = a.chunk_row[c], r1 = a.chunk_row[c + 1];
            if (r0 < r1) {
                const int64_t s0 = a.rp[r0], s1 = a.rp[r1];
                const int64_t w0 = a.cwo[c];
                const int nw = (int)(a.cwo[c + 1] - w0);
                const uint64_t hreg = (lane < nw) ? a.head[w0 + lane] : 0ull;
                const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
                int64_t rowbase = r0 - 1;  // row of the slot just before this word
                uint32_t carry = 0;        // wins of the still-open row from earlier words
                uint64_t mybits = 0;
                for (int t = 0; t < nw; ++t) {
                    const uint64_t Hd = readlane64(hreg, t);
                    const uint64_t Hn = (t + 1 < nw) ? readlane64(hreg, t + 1) : 1ull;
                    const int64_t s = s0 + (int64_t)t * 64 + lane;
                    const bool valid = s < s1;
                    const int64_t row = rowbase + __popcll(Hd & le);
                    bool win = false;
                    uint64_t Ku = 0;
                    int32_t u = 0;
                    if (valid) {
                        u = IDENT ? (int32_t)row : a.rid[row];
                        Ku = a.Kin[u];
                        win = slot_wins<H>(a.Kin, Ku, a.py, s);
                    }
                    const uint64_t W = __ballot(win);
                    if (lane == t) mybits = W;
                    // lanes whose slot is the last of its row
                    const int64_t rem = s1 - (s0 + (int64_t)t * 64);
                    uint64_t E = (Hd >> 1) | (Hn << 63);
                    if (rem < 64) E |= 1ull << (rem - 1);
                    if (valid && ((E >> lane) & 1ull)) {
                        const uint64_t hb = Hd & le;
                        const int st = hb ? 63 - __clzll(hb) : 0;
                        const uint64_t seg = le & (~0ull << st);
                        const uint32_t cnt = (uint32_t)__popcll(W & seg) + (hb ? 0u : carry);
                        a.Kout[u] = Ku + (((uint64_t)cnt * a.inc) << a.B);
                        if (GAP) {
                            const uint64_t A = Ku >> a.B;
                            sq += (u128)A * A;
                            mn += (u128)A * cnt;
                        }
                    }
                    if (t + 1 < nw && !(Hn & 1ull)) {
                        const int lh = Hd ? 63 - __clzll(Hd) : -1;
                        carry = (lh < 0) ? carry + (uint32_t)__popcll(W) : (uint32_t)__popcll(W & (~0ull << lh));
                    } else {
                        carry = 0;
                    }
                    rowbase += __popcll(Hd);
                }
                if (lane < nw) a.bits[w0 + lane] = mybits;
            }
        }
    }
    if (GAP) {
        sq = wave_sum128(sq);
        mn = wave_sum128(mn);
        if (lane == 0) {
            red[w][0] = (uint64_t)sq;
            red[w][1] = (uint64_t)(sq >> 64);
            red[w][2] = (uint64_t)mn;
            red[w][3] = (uint64_t)(mn >> 64);
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            u128 S = 0, M = 0;
            for (int q = 0; q < 4; ++q) {
                S += ((u128)red[q][1] << 64) | red[q][0];
                M += ((u128)red[q][3] << 64) | red[q][2];
            }
            uint64_t* o = a.partial + (int64_t)blockIdx.x * 4;
            o[0] = (uint64_t)S;
            o[1] = (uint64_t)(S >> 64);
            o[2] = (uint64_t)M;
            o[3] = (uint64_t)(M >> 64);
        }
    }
}

// per iteration: sum the per-workgroup partials exactly
__global__ __launch_bounds__(256) void k_gap_reduce(const uint64_t* partial, int64_t nblocks, uint64_t* out) {
    __shared__ uint64_t red[4][4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t* p = partial + (int64_t)blockIdx.x * nblocks * 4;
    u128 S = 0, M = 0;
    for (int64_t b = threadIdx.x; b < nblocks; b += 256) {
        S += ((u128)p[4 * b + 1] << 64) | p[4 * b];
        M += ((u128)p[4 * b + 3] << 64) | p[4 * b + 2];
    }
    S = wave_sum128(S);
    M = wave_sum128(M);
    if (lane == 0) {
        red[w][0] = (uint64_t)S;
        red[w][1] = (uint64_t)(S >> 64);
        red[w][2] = (uint64_t)M;
        red[w][3] = (uint64_t)(M >> 64);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        S = 0;
        M = 0;
        for (int q = 0; q < 4; ++q) {
            S += ((u128)red[q][1] << 64) | red[q][0];
            M += ((u128)red[q][3] << 64) | red[q][2];
        }
        out[4 * blockIdx.x + 0] = (uint64_t)S;
        out[4 * blockIdx.x + 1] = (uint64_t)(S >> 64);
        out[4 * blockIdx.x + 2] = (uint64_t)M;
        out[4 * blockIdx.x + 3] = (uint64_t)(M >> 64);
    }
}

// initial keys: A0 = deg (edges, r0 = deg/2 with D0 = 2) or 2 t_u (triangles,
// r0 = t_u/3 with D0 = 6), packed with the original-id code
__global__ void k_init_keys(const int32_t* count, int mult, const int32_t* orig_of, int64_t n, int B,
                            uint64_t* K0, uint64_t* K1) {
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (u >= n) return;
    const uint64_t idm = (1ull << B) - 1ull;
    const uint64_t k = ((uint64_t)count[u] * (uint64_t)mult << B) | (idm - (uint64_t)orig_of[u]);
    K0[u] = k;
    K1[u] = k;
}

__global__ void k_loads(const uint64_t* K, const int32_t* orig_of, int64_t n, int B, double D, float* r32,
                        uint64_t* A_out) {
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (u >= n) return;
    const uint64_t A = K[u] >> B;
    const int32_t o = orig_of[u];
    if (r32) r32[o] = (float)((double)A / D);
    if (A_out) A_out[o] = A;
}

// exact split numerator of every incidence slot from the stored decision
// words: a = a0 + sum_i inc_i [slot won in iteration i]
template <int H>
__global__ void k_splits(const int64_t* rp, const int32_t* rid, const int32_t* py, const int64_t* bitbase,
                         int64_t nrows, int64_t nslots, const uint64_t* bits, int64_t total_words, int iters,
                         int tri, const int32_t* orig_of, int32_t* verts, uint64_t* num) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= nslots) return;
    // row of slot s: last r with rp[r] <= s
    int64_t lo = 0, hi = nrows - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (rp[mid] <= s) lo = mid; else hi = mid - 1;
    }
    const int64_t r = lo;
    const int64_t pos = bitbase[r] + (s - rp[r]);
    uint64_t a = tri ? 2 : 1;
    for (int i = 1; i <= iters; ++i) {
        const uint64_t wd = bits[(int64_t)(i - 1) * total_words + pos / 64];
        if ((wd >> (pos % 64)) & 1ull) a += (uint64_t)(tri ? 6 : 2) * (uint64_t)(i + 1);
    }
    const int32_t x = rid ? rid[r] : (int32_t)r;
    verts[H * s] = orig_of[x];
    for (int j = 0; j < H - 1; ++j) verts[H * s + 1 + j] = orig_of[py[(H - 1) * s + j]];
    num[s] = a;
}

uint64_t denom(int mode, int64_t i) { return (uint64_t)(mode == 3 ? 3 : 1) * (uint64_t)(i + 1) * (uint64_t)(i + 2); }

template <int H, bool IDENT>
void launch_sweep(const SweepArgs& a, unsigned blocks, bool gap, hipStream_t s) {
    if (gap)
        k_fw_sweep<H, IDENT, true><<<blocks, 256, 0, s>>>(a);
    else
        k_fw_sweep<H, IDENT, false><<<blocks, 256, 0, s>>>(a);
}

}  // namespace

unsigned __int128 fw_max_numerator(const Graph& g, int mode, int iters) {
    // a vertex that wins every incident pattern in every iteration:
    // deg (1 + sum_i 2(i+1)) or t (2 + sum_i 6(i+1))
    const unsigned __int128 N = (unsigned)iters;
    if (mode == 2) return (unsigned __int128)(uint64_t)g.max_deg * (N * N + 3 * N + 1);
    return (unsigned __int128)(uint64_t)g.t_max * (2 + 3 * N * (N + 3));
}

void fw_run(Graph& g, int mode, int iters, bool want_gap, hipStream_t s) {
    LDS_CHECK(mode == 2 || mode == 3, ST_INVALID, "mode must be LDS_EDGE or LDS_TRIANGLE");
    LDS_CHECK(iters >= 0, ST_INVALID, "iters must be >= 0");
    if (mode == 3 && g.T < 0) list_triangles(g, s);
    SweepPlan& p = (mode == 2) ? g.edge_plan : g.tri_plan;
    FwState& f = g.fw[mode == 2 ? 0 : 1];
    const int B = g.idbits;
    // overflow: the largest numerator must leave B bits for the id code
    const u128 amax = fw_max_numerator(g, mode, iters);
    LDS_CHECK(B < 64 && (amax >> (64 - B)) == 0, ST_OVERFLOW, "exact load numerator would overflow the 64-bit key");
    const int64_t n = g.n;
    if (f.K[0].n != (size_t)n) {
        f.K[0].alloc(n, s);
        f.K[1].alloc(n, s);
    }
    if (n > 0) {
        const int32_t* cnt = (mode == 2) ? g.deg.p : g.tcount.p;
        k_init_keys<<<grid_for(n, 256), 256, 0, s>>>(cnt, mode == 2 ? 1 : 2, g.orig_of.p, n, B, f.K[0].p, f.K[1].p);
        LDS_HIP(hipGetLastError());
    }
    f.cur = 0;
    const size_t nbits = (size_t)iters * (size_t)p.total_words;
    if (f.bits.n < nbits) f.bits.alloc(nbits, s);
    const unsigned blocks = p.blocks();
    const size_t npart = want_gap ? (size_t)iters * blocks * 4 : 0;
    if (f.partial.n < npart) f.partial.alloc(npart, s);
    SweepArgs a{};
    a.rid = p.rid;
    a.rp = p.rp;
    a.py = p.py;
    a.n_hub = p.n_hub;
    a.hwo = p.hwo.p;
    a.n_chunks = p.n_chunks;
    a.chunk_row = p.chunk_row.p;
    a.cwo = p.cwo.p;
    a.head = p.head.p;
    a.chunk_words = p.chunk_words;
    a.B = B;
    for (int i = 1; i <= iters && blocks > 0 && p.nrows > 0; ++i) {
        a.Kin = f.K[f.cur].p;
        a.Kout = f.K[f.cur ^ 1].p;
        a.bits = f.bits.p + (size_t)(i - 1) * p.total_words;
        a.inc = denom(mode, i) - denom(mode, i - 1);
        a.partial = want_gap ? f.partial.p + (size_t)(i - 1) * blocks * 4 : nullptr;
        if (mode == 2)
            launch_sweep<2, true>(a, blocks, want_gap, s);
        else
            launch_sweep<3, false>(a, blocks, want_gap, s);
        LDS_HIP(hipGetLastError());
        f.cur ^= 1;
    }
    f.iters = iters;
    f.gap.assign(want_gap ? iters : 0, 0.0);
    f.lb.assign(want_gap ? iters : 0, 0.0);
    if (want_gap && iters > 0) {
        std::vector<uint64_t> sums((size_t)iters * 4, 0);
        if (blocks > 0 && p.nrows > 0) {
            DBuf<uint64_t> out;
            out.alloc((size_t)iters * 4, s);
            k_gap_reduce<<<iters, 256, 0, s>>>(f.partial.p, blocks, out.p);
            LDS_HIP(hipGetLastError());
            LDS_HIP(hipMemcpyAsync(sums.data(), out.p, out.bytes(), hipMemcpyDeviceToHost, s));
            LDS_HIP(hipStreamSynchronize(s));
        }
        for (int i = 1; i <= iters; ++i) {
            const u128 S = ((u128)sums[4 * (i - 1) + 1] << 64) | sums[4 * (i - 1)];
            const u128 M = ((u128)sums[4 * (i - 1) + 3] << 64) | sums[4 * (i - 1) + 2];
            const uint64_t D = denom(mode, i - 1);
            // (D^2/2) gap = sum A^2 - D * sum_patterns min A  (exact)
            const u128 num = S - (u128)D * M;
            const long double LD = (long double)D;
            const long double gap = 2.0L * (long double)num / (LD * LD);
            f.gap[i - 1] = (double)gap;
            f.lb[i - 1] = (double)((long double)S / (LD * LD) - gap);
        }
    }
}

void fw_loads(const Graph& g, int mode, float* r32_dev, double* r64_host, uint64_t* A_host, hipStream_t s) {
    const FwState& f = g.fw[mode == 2 ? 0 : 1];
    const int64_t n = g.n;
    if (n == 0) return;
    LDS_CHECK(f.K[0].n == (size_t)n, ST_INVALID, "no Frank-Wolfe state: call lds_frank_wolfe first");
    const double D = (double)denom(mode, f.iters);
    DBuf<uint64_t> A;
    if (r64_host || A_host) A.alloc(n, s);
    k_loads<<<grid_for(n, 256), 256, 0, s>>>(f.K[f.cur].p, g.orig_of.p, n, g.idbits, D, r32_dev, A.p);
    LDS_HIP(hipGetLastError());
    if (A.p) {
        std::vector<uint64_t> h(n);
        LDS_HIP(hipMemcpyAsync(h.data(), A.p, n * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < n; ++i) {
            if (A_host) A_host[i] = h[i];
            if (r64_host) r64_host[i] = (double)h[i] / D;
        }
    }
}

void fw_splits(const Graph& g, int mode, int32_t* verts_host, uint64_t* num_host, hipStream_t s) {
    const FwState& f = g.fw[mode == 2 ? 0 : 1];
    const SweepPlan& p = (mode == 2) ? g.edge_plan : g.tri_plan;
    const int64_t ns = p.nslots;
    if (ns == 0) return;
    LDS_CHECK(f.K[0].n == (size_t)g.n, ST_INVALID, "no Frank-Wolfe state: call lds_frank_wolfe first");
    const int H = mode;
    DBuf<int32_t> v;
    DBuf<uint64_t> a;
    v.alloc((size_t)ns * H, s);
    a.alloc(ns, s);
    if (mode == 2)
        k_splits<2><<<grid_for(ns, 256), 256, 0, s>>>(p.rp, p.rid, p.py, p.bitbase.p, p.nrows, ns, f.bits.p,
                                                      p.total_words, f.iters, 0, g.orig_of.p, v.p, a.p);
    else
        k_splits<3><<<grid_for(ns, 256), 256, 0, s>>>(p.rp, p.rid, p.py, p.bitbase.p, p.nrows, ns, f.bits.p,
                                                      p.total_words, f.iters, 1, g.orig_of.p, v.p, a.p);
    LDS_HIP(hipGetLastError());
    LDS_HIP(hipMemcpyAsync(verts_host, v.p, v.bytes(), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipMemcpyAsync(num_host, a.p, a.bytes(), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
}

}  // namespace lds
