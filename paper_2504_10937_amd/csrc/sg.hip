// Alg. 2 (ExtractSG) on the device: sort of the converged loads, prefix
// pattern counts, the candidate index set I, and the stable-group scan with
// Def. 5 (edges) / Def. trsg (triangles).
//
// a7  Sort: vertices by r descending, ties by caller id ascending.  The
//     packed keys K = (A << B) | (2^B - 1 - id) are distinct and ordered like
//     (r asc, id desc), so one ascending radix sort of K read backwards gives
//     the order.
// a8  Prefix: c_j = patterns whose latest vertex (largest position) is at
//     position j, counted on the per-slot records, which are stored in
//     position order (built once here and read again by the scan); E =
//     inclusive scan;
//     j+1 (1-based) is in I iff E_j/(j+1) is strictly above every later
//     E_k/(k+1) (argmax with ties to the larger index).
// a9  Stable groups.  Candidates are the runs ending at I.  A pending group
//     S = [S0, b) is tested with the restriction: every pattern touching S or
//     the vertices below gives weight only to its vertices in the lowest group
//     it touches (accepted groups above < S < everything below), and the
//     shares freed from higher vertices go to the lowest-r vertex of that
//     group.  S is accepted iff max_S r' < min r' of the last accepted group
//     and max_{below} r' < min_S r'.  Restricted loads below S depend only on
//     b, and for a fixed S0 the tests at different b are independent, so the
//     scan runs in rounds (one per accepted group): find, in order, the
//     boundaries b that pass two necessary conditions
//        (1) T_x < minH for every x in [S0, b), where T_x is x's restricted
//            load when S ends right after x (max_S r' >= max T_x, and the
//            restricted loads of S only grow with b, so the first violation
//            ends the whole scan);
//        (2) R of the first vertex below < T of the last vertex of S, where R_w
//            is w's restricted load when everything before w is above it
//            (max_below >= R_first, min_S <= T_last);
//     and verify each exactly, accepting the first that passes: restricted
//     loads of S from S's own patterns; the restricted loads of the vertices
//     below b are kept current as b advances (verification boundaries only
//     increase) with block maxima for the suffix maximum.
//     T is kept current by adding, after each acceptance, the change of the
//     accepted group's patterns.  All quantities are integer numerators over
//     D_N.  The whole scan (search, verification, acceptance, over every
//     round) is one cooperative kernel whose workgroups meet at grid barriers
//     between phases; the host only reads the group list at the end.
#include <algorithm>
#include <cstdlib>
#include <climits>
#include <type_traits>

#include "graph.hpp"
#include "gridsync.hpp"
#include "push.hpp"
#include "wave.hpp"

namespace lds {

namespace {

constexpr int kT = 256;


// ---------------------------------------------------------------- a7 sort
__global__ void k_sort_init(const uint64_t* K, int64_t n, uint64_t* keys, uint32_t* vals) {
    const int64_t u = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (u >= n) return;
    keys[u] = K[u];
    vals[u] = (uint32_t)u;
}

__global__ void k_order(const uint32_t* vals, int64_t n, int32_t* order, int64_t* pos) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const int64_t j = n - 1 - i;  // ascending keys read backwards: r descending
    order[j] = (int32_t)vals[i];
    pos[vals[i]] = j;
}

// --------------------------------------------------- split numerators per slot
// a = a0 + sum_i inc_i [slot won in iteration i], walking the sweep plan so
// that the bit position of a slot is known without a row search.  A block
// takes one hub-row piece or one chunk (at most kPiece slots either way, so
// the largest rows do not serialise in one block) in spans of kSpanW
// decision words (64 slots each).  The span's words of two batches of
// kIterB = 64 iterations at a time are staged in LDS by coalesced loads,
// all issued before the first is waited for.  A wave then
// takes a word column (64 slots x 64 iterations, lane l holding iteration
// l's word), transposes that bit matrix across its lanes (six exchange
// steps), so that lane s holds slot s's 64 decisions, and sums the
// increments c (j + 1) of the iterations j = i0 + i + 1 it won (bit i of
// its mask m) with popcounts:
//   sum over won i of (i0 + i + 2) = (i0 + 2) popc(m) + sum_k 2^k popc(m & M_k),
// M_k the batch rows whose index i has bit k set.
constexpr int kSpanW = 16;
constexpr int kIterB = 64;

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
    return ((uint64_t)hi << 32) | lo;
}

// 64 x 64 bit transpose across a wave: on entry lane l holds row l, on exit
// lane s holds column s (bit l = bit s of row l).  Step j swaps the
// off-diagonal j x j blocks of every 2j x 2j block.  All 64 lanes active.
__device__ inline uint64_t wave_transpose64(uint64_t x) {
    const int lane = threadIdx.x & 63;
    const uint64_t masks[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                               0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int j = 32 >> k;
        const uint64_t m = masks[k];
        const uint64_t p = shfl_xor_u64(x, j);
        x = (lane & j) ? ((x & ~m) | ((p >> j) & m)) : ((x & m) | ((p & m) << j));
    }
    return x;
}

__global__ __launch_bounds__(kT) void k_slot_splits(const int64_t* rp, int64_t n_pieces, const int32_t* hp_row,
                                                    const int32_t* hp_off, const int64_t* hwo, int64_t n_chunks,
                                                    const int64_t* chunk_row, const int64_t* cwo, int64_t chunk_words,
                                                    const uint64_t* bits, int64_t total_words, int iters, int tri,
                                                    int64_t heavy_positions, int64_t heavy_word0,
                                                    const uint32_t* heavy_csr, uint32_t* a_slot) {
    // one padding word per iteration row: the lanes of a wave read one
    // column, 17 words apart, so their reads spread over the banks
    __shared__ uint64_t sw[2][kIterB][kSpanW + 1];
    const int64_t b = blockIdx.x;
    int64_t s0, s1, word0;
    bool heavy = false;  // positions of the 2D part: the slot of position x is heavy_csr[x]
    if (b < n_pieces) {  // a hub row's piece (word-aligned, at most kPiece slots)
        const int64_t r = hp_row[b];
        s0 = rp[r] + hp_off[b];
        s1 = min(rp[r + 1], s0 + (int64_t)kPiece);
        word0 = chunk_words + hwo[r] + hp_off[b] / 64;
    } else if (b < n_pieces + n_chunks) {
        const int64_t c = b - n_pieces;
        s0 = rp[chunk_row[c]];
        s1 = rp[chunk_row[c + 1]];
        word0 = cwo[c];
    } else {
        const int64_t h = b - n_pieces - n_chunks;
        s0 = h * (int64_t)kPiece;
        if (s0 >= heavy_positions) return;
        s1 = min(heavy_positions, s0 + (int64_t)kPiece);
        word0 = heavy_word0 + s0 / 64;
        heavy = true;
    }
    constexpr int kWaves = kT / 64;
    constexpr int kCols = kSpanW / kWaves;  // word columns per wave and span
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    // split numerators are at most D, which the 32-bit per-slot array holds
    const uint32_t a0 = tri ? 2u : 1u, c2 = tri ? 6u : 2u;
    for (int64_t base = s0; base < s1; base += 64 * kSpanW) {
        const int64_t w0 = word0 + (base - s0) / 64;
        const int64_t nw = min<int64_t>(kSpanW, (s1 - base + 63) / 64);
        uint32_t acc[kCols];
#pragma unroll
        for (int q = 0; q < kCols; ++q) acc[q] = a0;
        for (int i2 = 0; i2 < iters; i2 += 2 * kIterB) {
            constexpr int kLoads = 2 * kIterB * kSpanW / kT;  // words per thread
            static_assert(2 * kIterB * kSpanW % kT == 0, "whole loads per thread");
            uint64_t v[kLoads];
#pragma unroll
            for (int l = 0; l < kLoads; ++l) {
                const int e = t + l * kT, it = i2 + e / kSpanW, ww = e % kSpanW;
                v[l] = (it < iters && ww < nw) ? bits[(int64_t)it * total_words + w0 + ww] : 0ull;
            }
            __syncthreads();  // the previous batches have been read
#pragma unroll
            for (int l = 0; l < kLoads; ++l) {
                const int e = t + l * kT, ii = e / kSpanW;
                sw[ii / kIterB][ii % kIterB][e % kSpanW] = v[l];
            }
            __syncthreads();
            for (int bb = 0; bb < 2 && i2 + bb * kIterB < iters; ++bb) {
                const int i0 = i2 + bb * kIterB;
#pragma unroll
                for (int q = 0; q < kCols; ++q) {
                    const int c = w + kWaves * q;
                    const uint64_t m = wave_transpose64(sw[bb][lane][c]);  // lane: its slot's 64 iterations
                    uint32_t sum = (uint32_t)(i0 + 2) * (uint32_t)__popcll(m);
#pragma unroll
                    for (int k = 0; k < 6; ++k) {
                        const uint64_t mk = ~0ull / ((1ull << (1 << k)) + 1ull) << (1 << k);  // bit k of the index set
                        sum += (uint32_t)__popcll(m & mk) << k;
                    }
                    acc[q] += c2 * sum;
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kCols; ++q) {
            const int64_t s = base + 64 * (w + kWaves * q) + lane;
            if (s < s1) {
                if (!heavy) {
                    a_slot[s] = acc[q];
                } else {
                    const uint32_t x = heavy_csr[s];
                    if (x != 0xffffffffu) a_slot[x] = acc[q];
                }
            }
        }
    }
}

// Hub push, stable-group splits: the split of hub row h's slot against a
// non-hub vertex v is D minus v's split of the same edge.  A non-hub row
// lists its hub neighbours first (rows are sorted by neighbour id), and rows
// come in id order, so the pairs (h, v's split) taken row by row and then
// sorted stably by h come out, for each h, in ascending v: the order of h's
// slots past its hub prefix.  One sort of those pairs replaces a search per
// slot (k_push_mirror: 3.2 ms on lds_large).
__global__ void k_hub_nb_count(const int64_t* rp, const int32_t* py, int64_t r0, int64_t r1, int32_t Hp,
                               uint32_t* cnt) {
    const int64_t r = r0 + (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= r1) return;
    int64_t lo = rp[r], hi = rp[r + 1];
    const int64_t s0 = lo;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (py[mid] < Hp)
            lo = mid + 1;
        else
            hi = mid;
    }
    cnt[r - r0] = (uint32_t)(lo - s0);
}

__global__ void k_hub_nb_pairs(const int64_t* rp, const int32_t* py, int64_t r0, int64_t r1, const uint32_t* cnt,
                               const uint64_t* off, const uint32_t* a_slot, uint64_t* keys, uint32_t* vals) {
    const int64_t r = r0 + (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= r1) return;
    const int64_t s0 = rp[r], o = (int64_t)off[r - r0];
    const uint32_t c = cnt[r - r0];
    for (uint32_t k0 = 0; k0 < c; k0 += 8) {  // eight loads in flight before the stores
        int32_t v[8];
        uint32_t x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            v[u] = k0 + u < c ? py[s0 + k0 + u] : 0;
            x[u] = k0 + u < c ? a_slot[s0 + k0 + u] : 0u;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (k0 + u < c) {
                keys[o + k0 + u] = (uint64_t)(uint32_t)v[u];
                vals[o + k0 + u] = x[u];
            }
    }
}

__global__ void k_hub_sfx_len(const int64_t* rp, const int32_t* hub_pre, int64_t Hp, uint32_t* len) {
    const int64_t h = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (h < Hp) len[h] = (uint32_t)(rp[h + 1] - rp[h] - hub_pre[h]);
}

__global__ void k_hub_scatter(const uint64_t* keys, const uint32_t* vals, int64_t np, const uint64_t* first,
                              const int64_t* rp, const int32_t* hub_pre, uint32_t D, uint32_t* a_slot) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= np) return;
    const int64_t h = (int64_t)keys[i];
    a_slot[rp[h] + hub_pre[h] + (i - (int64_t)first[h])] = D - vals[i];
}

// triangles: index of the slot's row vertex within tri[t] (the slot holds the
// other two in triangle order)
__device__ inline int tri_index(const int32_t* tri, int64_t t, int32_t v, int32_t w) {
    return (tri[3 * t] != v) ? 0 : ((tri[3 * t + 1] != w) ? 1 : 2);
}

__global__ void k_tri_splits(const int32_t* py, const int32_t* tos, const int32_t* tri, const uint32_t* a_slot,
                             int64_t ns, uint32_t* a_tri) {
    const int64_t s = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (s >= ns) return;
    const int64_t t = tos[s];
    a_tri[3 * t + tri_index(tri, t, py[2 * s], py[2 * s + 1])] = a_slot[s];
}

// ----------------------------------------------------- row passes (a8, a9)

struct PassArgs {
    const int32_t* rid;
    const int64_t* rp;
    const int32_t* py;
    const int32_t* tos;
    const int32_t* tri;
    const uint32_t* a_slot;
    const uint32_t* a_tri;
    const int64_t* pos;
    const int32_t* row_of;  // triangles: internal vertex -> row (edges: identity below nrows)
    int64_t nrows, n_big;
    uint64_t D;
};

__device__ inline int grp(int64_t p, int64_t t1, int64_t t2) { return p < t1 ? 0 : (p < t2 ? 1 : 2); }

__global__ void k_inclusive(const uint64_t* excl, const int64_t* c, int64_t n, int64_t* E) {
    const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (j < n) E[j] = (int64_t)excl[j] + c[j];
}

// ---------------------------------------------- strict suffix maxima of E/j
// fraction (num, den), den = 0 means "minus infinity"
__device__ inline bool frac_gt(int64_t an, int64_t ad, int64_t bn, int64_t bd) {
    if (bd == 0) return ad != 0;
    if (ad == 0) return false;
    return (__int128)an * bd > (__int128)bn * ad;
}

constexpr int kTile = 4096;

__global__ __launch_bounds__(kT) void k_tile_fmax(const int64_t* E, int64_t n, int64_t* tn, int64_t* td) {
    __shared__ int64_t sn[kT], sd[kT];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int64_t bn = 0, bd = 0;
    for (int k = 0; k < kTile / kT; ++k) {
        const int64_t j = base + (int64_t)k * kT + threadIdx.x;
        if (j < n && frac_gt(E[j], j + 1, bn, bd)) { bn = E[j]; bd = j + 1; }
    }
    sn[threadIdx.x] = bn;
    sd[threadIdx.x] = bd;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kT; ++i)
            if (frac_gt(sn[i], sd[i], bn, bd)) { bn = sn[i]; bd = sd[i]; }
        tn[blockIdx.x] = bn;
        td[blockIdx.x] = bd;
    }
}

// carry (cn, cd) = max over all later tiles; each thread owns 16 consecutive
// positions, walked backwards after a block-level suffix max of thread maxima
__global__ __launch_bounds__(kT) void k_tile_inI(const int64_t* E, int64_t n, const int64_t* cn_, const int64_t* cd_,
                                               uint8_t* inI) {
    __shared__ int64_t sn[kT], sd[kT];
    const int per = kTile / kT;
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * per;
    int64_t bn = 0, bd = 0;
    for (int k = 0; k < per; ++k) {
        const int64_t j = base + k;
        if (j < n && frac_gt(E[j], j + 1, bn, bd)) { bn = E[j]; bd = j + 1; }
    }
    sn[threadIdx.x] = bn;
    sd[threadIdx.x] = bd;
    __syncthreads();
    if (threadIdx.x == 0) {
        // exclusive suffix max over threads, seeded with the later tiles' max
        int64_t rn = cn_[blockIdx.x], rd = cd_[blockIdx.x];
        for (int i = kT - 1; i >= 0; --i) {
            const int64_t xn = sn[i], xd = sd[i];
            sn[i] = rn;
            sd[i] = rd;
            if (frac_gt(xn, xd, rn, rd)) { rn = xn; rd = xd; }
        }
    }
    __syncthreads();
    int64_t rn = sn[threadIdx.x], rd = sd[threadIdx.x];
    for (int k = per - 1; k >= 0; --k) {
        const int64_t j = base + k;
        if (j >= n) continue;
        const bool in = frac_gt(E[j], j + 1, rn, rd);
        inI[j] = in ? 1 : 0;
        if (in) { rn = E[j]; rd = j + 1; }
    }
}

// exclusive suffix maximum of the tile maxima, one workgroup: thread i owns
// a contiguous block of tiles (its maximum, then an exclusive suffix maximum
// over the threads' maxima in LDS, then its block walked backwards)
__global__ __launch_bounds__(kT) void k_tile_carry(const int64_t* tn, const int64_t* td, int64_t tiles, int64_t* cn,
                                                 int64_t* cd) {
    __shared__ int64_t sn[kT], sd[kT];
    const int64_t per = (tiles + kT - 1) / kT;
    const int64_t t0 = (int64_t)threadIdx.x * per, t1 = min(tiles, t0 + per);
    int64_t bn = 0, bd = 0;  // den 0: minus infinity
    for (int64_t t = t0; t < t1; ++t)
        if (frac_gt(tn[t], td[t], bn, bd)) { bn = tn[t]; bd = td[t]; }
    sn[threadIdx.x] = bn;
    sd[threadIdx.x] = bd;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t rn = 0, rd = 0;
        for (int i = kT - 1; i >= 0; --i) {
            const int64_t xn = sn[i], xd = sd[i];
            sn[i] = rn;
            sd[i] = rd;
            if (frac_gt(xn, xd, rn, rd)) { rn = xn; rd = xd; }
        }
    }
    __syncthreads();
    int64_t rn = sn[threadIdx.x], rd = sd[threadIdx.x];
    for (int64_t t = t1 - 1; t >= t0; --t) {
        cn[t] = rn;
        cd[t] = rd;
        if (frac_gt(tn[t], td[t], rn, rd)) { rn = tn[t]; rd = td[t]; }
    }
}

// ------------------------------------------------------ a9 round helpers
__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---- incremental maintenance of T and restricted verification passes
// group of position p under thresholds: 0 above (< t1), 1 tested ([t1, t2)), 2 below
// contribution of pattern vertex k (of h) given positions and split numerators
template <int H>
__device__ inline int64_t pat_contrib(int k, const int64_t* p, const int64_t* al, uint64_t D, int64_t t1, int64_t t2) {
    int g[H];
    int gl = 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        g[i] = grp(p[i], t1, t2);
        gl = max(gl, g[i]);
    }
    if (g[k] < gl) return 0;
    int64_t freed = 0;
    bool recv = true;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        if (g[i] < gl) freed += al[i];
        else if (i != k && p[i] > p[k]) recv = false;
    }
    (void)D;
    return al[k] + (recv ? freed : 0);
}

// positions, numerators and internal ids of the pattern at slot s of row x
template <int H>
__device__ inline void load_pattern(const PassArgs& a, int64_t s, int32_t x, int64_t* p, int64_t* al, int32_t* id);
template <>
__device__ inline void load_pattern<2>(const PassArgs& a, int64_t s, int32_t x, int64_t* p, int64_t* al, int32_t* id) {
    id[0] = x;
    id[1] = a.py[s];
    p[0] = a.pos[x];
    p[1] = a.pos[id[1]];
    al[0] = a.a_slot[s];
    al[1] = (int64_t)a.D - al[0];
}
template <>
__device__ inline void load_pattern<3>(const PassArgs& a, int64_t s, int32_t x, int64_t* p, int64_t* al, int32_t* id) {
    const int32_t v = a.py[2 * s], w = a.py[2 * s + 1];
    const int64_t t = a.tos[s];
    const int jx = tri_index(a.tri, t, v, w);
    const int jv = (jx == 0) ? 1 : 0, jw = (jx == 2) ? 1 : 2;
    id[0] = x;
    id[1] = v;
    id[2] = w;
    p[0] = a.pos[x];
    p[1] = a.pos[v];
    p[2] = a.pos[w];
    al[0] = a.a_tri[3 * t + jx];
    al[1] = a.a_tri[3 * t + jv];
    al[2] = a.a_tri[3 * t + jw];
}

// The restricted load F_w(b) of a vertex below the boundary b (everything
// before b is above it) only grows with b.  Verification boundaries increase
// over the whole scan, so F is advanced incrementally: when positions
// [p0, p1) move above, each of their patterns (handled once, from its latest
// moving vertex) adds (after - before) to the vertices still below; block
// maxima over 1024 positions, and maxima of 64 blocks (superblocks), stay
// valid under these increases, so the largest load below b is read from at
// most 1024 + 64 + n / 65536 values.
constexpr int kFB = 1024;
constexpr int kSB = 64;  // blocks per superblock

// F at b = 0 (nothing above): the plain load numerators, by position
__global__ void k_f_init(const uint64_t* K, const int32_t* order, int64_t n, int B, int64_t* F) {
    const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (j < n) F[j] = (int64_t)(K[order[j]] >> B);
}

__global__ __launch_bounds__(kT) void k_bmax_init(const int64_t* F, int64_t n, long long* bmax) {
    const int64_t base = (int64_t)blockIdx.x * kFB;
    long long mx = LLONG_MIN;
    for (int64_t j = base + threadIdx.x; j < base + kFB && j < n; j += kT) mx = max(mx, (long long)F[j]);
    mx = wave::max_all(mx);
    __shared__ long long sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) bmax[blockIdx.x] = max(max(sh[0], sh[1]), max(sh[2], sh[3]));
}

// superblock maxima from the block maxima (one wave per superblock)
__global__ __launch_bounds__(64) void k_bmax2_init(const long long* bmax, int64_t nblk, long long* bmax2) {
    const int64_t blk = (int64_t)blockIdx.x * kSB + threadIdx.x;
    const long long mx = wave::max_all(blk < nblk ? bmax[blk] : LLONG_MIN);
    if (threadIdx.x == 0) bmax2[blockIdx.x] = mx;
}

// ------------------------------------------- the whole scan on the device
// One launch runs every round of the scan.  Workgroup 0 (the leader) holds
// the control: it searches, verifies and accepts.  A phase with little work
// (a search window, a walk over few records, the minimum and maximum over a
// short pending group) runs in the leader alone, and its phases are
// separated by workgroup barriers only: no device-scope fences, so the
// leader's caches stay warm and a verification costs a few dependent
// accesses.  A phase with much work is posted to the whole grid (a
// cooperative launch, so every workgroup is resident): the leader writes the
// phase descriptor, releases its writes at device scope and bumps the post
// counter; the other workgroups (helpers) wait for the post, run their share
// and meet the leader at a grid barrier, where every workgroup releases and
// acquires at device scope.  Cross-workgroup reductions go through
// per-workgroup partial records, double-buffered by phase parity.  Every
// wait is bounded: past the spin limit a workgroup raises the error flag and
// leaves the wait, so the kernel always ends and the host reports the error.
// A helper's wait for a post restarts its count whenever the leader's
// heartbeat moves, so a long run of leader-only phases is not an error.
constexpr int kRT = 512;                 // threads per workgroup of the scan
constexpr int kRW = kRT / 64;
constexpr int64_t kSearchWin = 1 << 20;  // largest window of positions searched in one phase
constexpr unsigned kSpinLimit = kGridSpinLimit;
// defaults of the launch shape: one workgroup up to 16384 vertices, else up
// to kScanMaxWG (as many as are resident); a posted phase goes to one
// workgroup per kPartWork records or positions of its work (at least 8, in
// multiples of 8), so that only the large walks spread over a wide grid; and
// the largest walk (records) and search window / min-max / bounds range
// (positions) that the leader runs alone (a few trips of its 512 threads).
// The environment variables LDS_SCAN_WG, LDS_SCAN_PART_WORK,
// LDS_SCAN_LEAD_RECS and LDS_SCAN_LEAD_POS override them (LDS_SCAN_WG also
// on graphs of at most 16384 vertices), e.g. to run the grid phases on small
// graphs.
constexpr int kScanMaxWG = 128;
constexpr int64_t kPartWork = 1024;
constexpr int64_t kLeadRecs = 2048;
constexpr int64_t kLeadPos = 8192;

enum : long long { PH_EXIT = 0, PH_SEARCH = 1, PH_UPDATE = 2, PH_MINMAX = 3, PH_ACCEPT = 4, PH_UNDO = 5 };
// a posted phase: kind, parity, up to six arguments, then its workgroups
// (the first `parts` of the grid) and its barrier target
constexpr int kDesc = 10;

struct ScanArgs {
    PassArgs a;
    const int32_t* order;
    const uint8_t* inI;
    const int64_t* R;
    int64_t* T;
    int64_t* F;
    int64_t* V;            // restricted loads of the pending group, by position
    long long* bmax;
    long long* bmax2;      // maxima of kSB consecutive blocks
    int64_t nsb;
    int64_t nblk;
    int64_t n;
    int64_t* lo;           // bounds by internal vertex
    int64_t* hi;
    int64_t* groups;       // (start, end) per accepted group
    int64_t* info;         // [0] groups, [1] rounds, [2] verifications, [3] error flag
    long long* part;       // 2 * gridDim * 4 partial records
    unsigned* bar;         // [0] barrier arrivals, [2] posts, [3] leader heartbeat
    long long* desc;       // the posted phase: kind, parity, up to six arguments
    int64_t part_work;     // records or positions per workgroup of a posted phase
    int64_t lead_recs;     // largest walk the leader runs alone
    int64_t lead_pos;      // largest position range the leader runs alone
    // compact records built once per scan (k_slot_records), one per
    // incidence slot, stored in position order: the records of the vertex at
    // position j are [P[j], P[j+1]), so the patterns of a range of positions
    // are one contiguous range of records, streamed instead of chased
    // through order -> row -> slot -> neighbour -> position
    const int64_t* P;      // n + 1 record offsets by position
    const int32_t* own;    // position of the record's own vertex
    const int2* rec2;      // edges: (position of the other end, a_x)
    const int4* rec3;      // triangles: (position v, position w, a_x, a_v)
    const uint32_t* rec3w; // triangles: a_w
};

// the pattern of record k, from the records
template <int H>
__device__ inline void rec_pattern(const ScanArgs& g, int64_t k, int64_t* p, int64_t* al);
template <>
__device__ inline void rec_pattern<2>(const ScanArgs& g, int64_t k, int64_t* p, int64_t* al) {
    const int2 r = g.rec2[k];
    p[0] = g.own[k];
    p[1] = r.x;
    al[0] = (uint32_t)r.y;
    al[1] = (int64_t)g.a.D - al[0];
}
template <>
__device__ inline void rec_pattern<3>(const ScanArgs& g, int64_t k, int64_t* p, int64_t* al) {
    const int4 r = g.rec3[k];
    p[0] = g.own[k];
    p[1] = r.x;
    p[2] = r.y;
    al[0] = (uint32_t)r.z;
    al[1] = (uint32_t)r.w;
    al[2] = g.rec3w[k];
}

// Record walks.  A wave takes kRecRows(H) rows of 64 consecutive records per
// trip (lane l reads record 64 r + l of row r, so every load is coalesced)
// and keeps the loads, the atomics and the reads that depend on them of all
// its rows in flight together: the walks are bound by the latency of these
// dependent accesses, not by bandwidth, and a long row no longer runs as one
// wave's serial loop.  Rows go round-robin over the walk's waves (row r to
// wave r mod nwave), so a walk shorter than one full trip spreads over every
// workgroup of its phase: a compute unit issues its scattered atomics and
// reads about one address per cycle, and a walk that filled the first
// workgroups' waves alone queued them on a few compute units.
template <int H>
constexpr int kRecRows = (H == 2) ? 8 : 4;


// Adds, per position, the values of one row of 64 records into V.  The
// positions of a row's valid lanes do not decrease from lane to lane and its
// unused lanes (key -1) come last, so equal keys are contiguous: a segmented
// prefix sum leaves each position's total in its last lane, which makes the
// one atomic (V starts at zero and a position's own sum is added once).
// Called by all 64 lanes.
__device__ inline void add_by_position(int64_t* V, int32_t key, int64_t val) {
    val = wave::seg_prefix_sum(key, val);
    if (wave::run_tail(key) && key >= 0 && val != 0) atomicAdd((unsigned long long*)&V[key], (unsigned long long)val);
}

// Positions [f0, b) move from below the boundary into the pending group
// S = [S0, b).  One walk over their patterns gives their own restricted
// loads (into V), advances the loads F of the vertices that stay below b
// (with the block maxima), and changes the loads of S's earlier members
// through the patterns they share with the joining vertices.  Each pattern
// is handled once, from its latest joining vertex.
// spec (only when f0 == S0, the first boundary of a round): the joining
// vertices are all of S, so the walk also applies, ahead of the decision,
// the change of T that accepting S would make (accept_walk's); a rejected
// boundary takes it back with accept_walk's negation.
// Records [k0, k1) = [P[f0], P[b]); wave gw of nwave.
template <int H>
__device__ inline void update_walk(const ScanArgs& g, int64_t S0, int64_t f0, int64_t b, int64_t k0, int64_t k1,
                                   int64_t gw, int64_t nwave, bool spec) {
    constexpr int U = kRecRows<H>;
    const int lane = threadIdx.x & 63;
    const uint64_t D = g.a.D;
    for (int64_t r0 = gw; k0 + 64 * r0 < k1; r0 += nwave * U) {  // this trip: rows r0 + nwave u
        int64_t p[U][H], al[U][H];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = k0 + 64 * (r0 + nwave * u) + lane;
            if (k < k1) rec_pattern<H>(g, k, p[u], al[u]);
            else p[u][0] = -1;
        }
        int64_t own[U], fd[U][H - 1], fo[U][H - 1];
        long long bm[U][H - 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            own[u] = 0;
#pragma unroll
            for (int i = 0; i < H - 1; ++i) fd[u][i] = 0;
            if (p[u][0] < 0) continue;
            own[u] = pat_contrib<H>(0, p[u], al[u], D, S0, b);
            bool latest = true;
#pragma unroll
            for (int i = 1; i < H; ++i)
                if (p[u][i] >= f0 && p[u][i] < b && p[u][i] > p[u][0]) latest = false;
            if (!latest) continue;
#pragma unroll
            for (int i = 1; i < H; ++i) {
                if (p[u][i] >= b) {  // stays below
                    if (spec) {
                        const int64_t dt = pat_contrib<H>(i, p[u], al[u], D, b, p[u][i] + 1) -
                                           pat_contrib<H>(i, p[u], al[u], D, S0, p[u][i] + 1);
                        if (dt != 0) atomicAdd((unsigned long long*)&g.T[p[u][i]], (unsigned long long)dt);
                    }
                    const int64_t d = pat_contrib<H>(i, p[u], al[u], D, b, b) - pat_contrib<H>(i, p[u], al[u], D, f0, f0);
                    if (d != 0) {
                        fd[u][i - 1] = d;
                        fo[u][i - 1] = (int64_t)atomicAdd((unsigned long long*)&g.F[p[u][i]], (unsigned long long)d);
                        bm[u][i - 1] = g.bmax[p[u][i] / kFB];
                    }
                } else if (p[u][i] >= S0 && p[u][i] < f0) {  // earlier member of S
                    const int64_t d =
                        pat_contrib<H>(i, p[u], al[u], D, S0, b) - pat_contrib<H>(i, p[u], al[u], D, S0, f0);
                    if (d != 0) atomicAdd((unsigned long long*)&g.V[p[u][i]], (unsigned long long)d);
                }
            }
        }
        // the joining vertices' own loads first: their segmented sums need
        // no value the returning atomics above bring back, so they run while
        // those are in flight
#pragma unroll
        for (int u = 0; u < U; ++u) add_by_position(g.V, (int32_t)p[u][0], own[u]);
        // block maxima only grow (F only grows, bmax only by atomicMax): a
        // read that is at least the new value, even a stale one or one made
        // before the add, makes the atomic redundant
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < H - 1; ++i)
                if (fd[u][i] != 0) {
                    const long long nv = (long long)(fo[u][i] + fd[u][i]);
                    if (nv > bm[u][i]) {  // the superblock maximum is raised with its block's
                        atomicMax(&g.bmax[p[u][i + 1] / kFB], nv);
                        atomicMax(&g.bmax2[p[u][i + 1] / ((int64_t)kFB * kSB)], nv);
                    }
                }
    }
}

// After S = [S0, b) is accepted: the change of T_x (S ending after x) for
// the vertices below b, from the patterns of S (each handled once, from its
// latest vertex in S); sgn = -1 takes back a change applied ahead of a
// decision that rejected b.
// Records [k0, k1) = [P[S0], P[b]); wave gw of nwave.
template <int H>
__device__ inline void accept_walk(const ScanArgs& g, int64_t S0, int64_t b, int64_t k0, int64_t k1, int64_t gw,
                                   int64_t nwave, int64_t sgn) {
    constexpr int U = kRecRows<H>;
    const int lane = threadIdx.x & 63;
    const uint64_t D = g.a.D;
    for (int64_t r0 = gw; k0 + 64 * r0 < k1; r0 += nwave * U) {  // this trip: rows r0 + nwave u
        int64_t p[U][H], al[U][H];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t k = k0 + 64 * (r0 + nwave * u) + lane;
            if (k < k1) rec_pattern<H>(g, k, p[u], al[u]);
            else p[u][0] = -1;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (p[u][0] < 0) continue;
            bool latest = true;
#pragma unroll
            for (int i = 1; i < H; ++i)
                if (p[u][i] >= S0 && p[u][i] < b && p[u][i] > p[u][0]) latest = false;
            if (!latest) continue;
#pragma unroll
            for (int i = 1; i < H; ++i) {
                if (p[u][i] < b) continue;
                const int64_t d = pat_contrib<H>(i, p[u], al[u], D, b, p[u][i] + 1) -
                                  pat_contrib<H>(i, p[u], al[u], D, S0, p[u][i] + 1);
                if (d != 0) atomicAdd((unsigned long long*)&g.T[p[u][i]], (unsigned long long)(sgn * d));
            }
        }
    }
}

// slots per position (rows are vertices with slots; the rest stay 0)
__global__ void k_pos_slots(PassArgs a, uint64_t* cnt) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= a.nrows) return;
    const int32_t x = a.rid ? a.rid[r] : (int32_t)r;
    cnt[a.pos[x]] = (uint64_t)(a.rp[r + 1] - a.rp[r]);
}

// Records of every slot of row r, written in position order: slot s of the
// row at position px goes to P[px] + (s - rp[r]).  The same pass sums three
// values over the row's patterns, by position: c_px (a8: the patterns whose
// latest vertex is px's; optional), R_px (its share when every earlier
// vertex is above it) and T_px (its share when S = [0, px]; the scan keeps T
// current from there).  A vertex has one row, so the row's group of lanes
// stores its vertex's sums; positions without slots keep the zero they were
// filled with.  G lanes per row, 64 / G rows per wave: rows [r0, r1) of one
// length class, so that short rows do not leave most of a wave idle, and a
// row of at most 64 slots takes one trip of dependent loads (every lane
// loops over its row with stride G, so any row length is handled).
template <int H, int G>
__global__ __launch_bounds__(kT) void k_slot_records(PassArgs a, int64_t r0, int64_t r1, const int64_t* P,
                                                     int32_t* own, int2* rec2, int4* rec3, uint32_t* rec3w,
                                                     int64_t* c, int64_t* R, int64_t* T) {
    static_assert(G == 8 || G == 16 || G == 32 || G == 64, "lanes per row: 8, 16, 32 or 64");
    const int lane = threadIdx.x & 63;
    const int64_t rw = r0 + ((int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6)) * (64 / G);
    if (rw >= r1) return;  // uniform over the wave
    const int64_t r = rw + lane / G;
    const bool live = r < r1;
    int64_t cs = 0, rs = 0, ts = 0, px = 0;
    if (live) {
        const int32_t x = a.rid ? a.rid[r] : (int32_t)r;
        px = a.pos[x];
        const int64_t shift = P[px] - a.rp[r];
        const uint64_t D = a.D;
        // an edge row per wave: U slots per lane and trip, all loaded before
        // any is used, so that a long row's trips overlap their gathers
        // (lds_large 1.82 against 1.88 ms; triangle rows, with three times
        // the loads per slot, were slower so: 1.87 against 1.65 ms)
        constexpr int U = (G == 64 && H == 2) ? 4 : 1;
        const int64_t e = a.rp[r + 1];
        for (int64_t s0 = a.rp[r] + lane % G; s0 < e; s0 += (int64_t)G * U) {
            int64_t p[U][H], al[U][H];
            int32_t id[U][H];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (s0 + (int64_t)u * G < e) load_pattern<H>(a, s0 + (int64_t)u * G, x, p[u], al[u], id[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t s = s0 + (int64_t)u * G;
                if (s >= e) break;
                own[shift + s] = (int32_t)px;
                if (H == 2) {
                    rec2[shift + s] = make_int2((int)p[u][1], (int)(uint32_t)al[u][0]);
                } else {
                    rec3[shift + s] =
                        make_int4((int)p[u][1], (int)p[u][2], (int)(uint32_t)al[u][0], (int)(uint32_t)al[u][1]);
                    rec3w[shift + s] = (uint32_t)al[u][2];
                }
                bool latest = true;
#pragma unroll
                for (int i = 1; i < H; ++i) latest = latest && p[u][i] < p[u][0];
                cs += latest ? 1 : 0;
                rs += pat_contrib<H>(0, p[u], al[u], D, p[u][0], p[u][0]);
                ts += pat_contrib<H>(0, p[u], al[u], D, 0, p[u][0] + 1);
            }
        }
    }
    // every lane of the wave takes part in the sums
    if (G == 64) {
        auto plus = [](int64_t u, int64_t v) { return u + v; };
        cs = wave::lane63(wave::scan(cs, 0, plus));
        rs = wave::lane63(wave::scan(rs, 0, plus));
        ts = wave::lane63(wave::scan(ts, 0, plus));
    } else {
        // the row's last lane ends with the row's totals
        cs = wave::seg_prefix_sum(lane / G, cs);
        rs = wave::seg_prefix_sum(lane / G, rs);
        ts = wave::seg_prefix_sum(lane / G, ts);
    }
    if (live && lane % G == (G == 64 ? 0 : G - 1)) {
        if (c) c[px] = cs;
        R[px] = rs;
        T[px] = ts;
    }
}

// first row with at most 32, 16 and 8 slots: the class limits of
// k_slot_records (rows are ordered by slot count, longest first)
__global__ void k_record_classes(const int64_t* rp, int64_t nrows, int64_t* out) {
    const int i = threadIdx.x;
    if (i >= 3) return;
    const int64_t t = (int64_t)32 >> i;
    int64_t lo = 0, hi = nrows;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (rp[mid + 1] - rp[mid] > t) lo = mid + 1;
        else hi = mid;
    }
    out[i] = lo;
}

// Barrier of the workgroups of one posted phase: the first P workgroups
// (P = parts of the phase), the leader among them.  The arrival counter only
// grows; the leader keeps the total of the arrivals that every phase so far
// has asked for and posts it as the phase's target, so each participant
// adds one and waits until the counter reaches the target.  Otherwise as
// grid_sync: one device-scope release / acquire per workgroup (thread 0),
// a bounded wait that raises *err.
__device__ inline void phase_barrier(const ScanArgs& g, unsigned target, int64_t* err) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(g.bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while ((int)(__hip_atomic_load(g.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > kGridSpinLimit) {
                *err = 1;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// reduce the partial records of phase `ph` (4 values per workgroup: min,
// max, max, min) of its `parts` workgroups into sh[0..3]
__device__ inline void gather_partials(const ScanArgs& g, int ph, unsigned parts, long long* sh) {
    if (threadIdx.x < 64) {
        long long v0 = LLONG_MAX, v1 = LLONG_MIN, v2 = LLONG_MIN, v3 = LLONG_MAX;
        const long long* P = g.part + (int64_t)(ph & 1) * gridDim.x * 4;
        for (unsigned w = threadIdx.x; w < parts; w += 64) {
            v0 = min(v0, P[4 * w]);
            v1 = max(v1, P[4 * w + 1]);
            v2 = max(v2, P[4 * w + 2]);
            v3 = min(v3, P[4 * w + 3]);
        }
        v0 = wave::min_all(v0);
        v1 = wave::max_all(v1);
        v2 = wave::max_all(v2);
        v3 = wave::min_all(v3);
        if (threadIdx.x == 0) {
            sh[0] = v0;
            sh[1] = v1;
            sh[2] = v2;
            sh[3] = v3;
        }
    }
    __syncthreads();
}

// this workgroup's partial record of phase `ph` from per-thread values
__device__ inline void put_partial(const ScanArgs& g, int ph, long long v0, long long v1, long long v2, long long v3,
                                   long long (*sred)[4]) {
    v0 = wave::min_all(v0);
    v1 = wave::max_all(v1);
    v2 = wave::max_all(v2);
    v3 = wave::min_all(v3);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sred[w][0] = v0;
        sred[w][1] = v1;
        sred[w][2] = v2;
        sred[w][3] = v3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kRW; ++q) {
            v0 = min(v0, sred[q][0]);
            v1 = max(v1, sred[q][1]);
            v2 = max(v2, sred[q][2]);
            v3 = min(v3, sred[q][3]);
        }
        v0 = min(v0, sred[0][0]);
        v1 = max(v1, sred[0][1]);
        v2 = max(v2, sred[0][2]);
        v3 = min(v3, sred[0][3]);
        long long* P = g.part + ((int64_t)(ph & 1) * gridDim.x + blockIdx.x) * 4;
        P[0] = v0;
        P[1] = v1;
        P[2] = v2;
        P[3] = v3;
    }
    __syncthreads();
}

// WG-level reduction of per-thread values into sh[0..3] (min, max, max, min)
__device__ inline void reduce_local(long long v0, long long v1, long long v2, long long v3, long long (*sred)[4],
                                    long long* sh) {
    v0 = wave::min_all(v0);
    v1 = wave::max_all(v1);
    v2 = wave::max_all(v2);
    v3 = wave::min_all(v3);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        sred[w][0] = v0;
        sred[w][1] = v1;
        sred[w][2] = v2;
        sred[w][3] = v3;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int q = 1; q < kRW; ++q) {
            v0 = min(v0, sred[q][0]);
            v1 = max(v1, sred[q][1]);
            v2 = max(v2, sred[q][2]);
            v3 = min(v3, sred[q][3]);
        }
        sh[0] = v0;
        sh[1] = v1;
        sh[2] = v2;
        sh[3] = v3;
    }
    __syncthreads();
}

// First event in [lo, hi) among this thread's positions lo + t + i * nthr:
// a stop position (T >= minH) or a candidate boundary (in I, and R of the
// next position below T), as 2 j + 1 for a stop and 2 j for a candidate, so
// that the smallest code is the first event.  LLONG_MAX: none.
__device__ inline long long search_part(const ScanArgs& g, int64_t lo, int64_t hi, bool hasH, long long minH,
                                        int64_t t, int64_t nthr) {
    for (int64_t j0 = lo + t; j0 < hi; j0 += 4 * nthr) {
        // every load of the trip at once (R of the next position whether or
        // not j is in I): the search is bound by their latency
        int64_t Tv[4], Rn[4];
        uint8_t in[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = j0 + u * nthr;
            Tv[u] = j < hi ? g.T[j] : 0;
            in[u] = j < hi ? g.inI[j] : 0;
            Rn[u] = (j < hi && j + 1 < g.n) ? g.R[j + 1] : LLONG_MIN;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = j0 + u * nthr;
            if (j >= hi) break;
            if (hasH && Tv[u] >= minH) return 2 * j + 1;
            if (in[u] && Rn[u] < Tv[u]) return 2 * j;
        }
    }
    return LLONG_MAX;
}

// min and max of the restricted loads of S = [S0, b), and the largest
// restricted load below b, over this thread's share
__device__ inline void minmax_part(const ScanArgs& g, int64_t S0, int64_t b, int64_t t, int64_t nthr, long long& vmn,
                                   long long& vmx, long long& fmx) {
    vmn = LLONG_MAX;
    vmx = LLONG_MIN;
    fmx = LLONG_MIN;
    for (int64_t j = S0 + t; j < b; j += nthr) {
        const long long v = (long long)g.V[j];
        vmn = min(vmn, v);
        vmx = max(vmx, v);
    }
    if (b < g.n) {
        const int64_t bend = min(g.n, (b / kFB + 1) * kFB);
        const int64_t sb = b / ((int64_t)kFB * kSB), blk_end = min(g.nblk, (sb + 1) * kSB);
        for (int64_t j = b + t; j < bend; j += nthr) fmx = max(fmx, (long long)g.F[j]);
        for (int64_t blk = b / kFB + 1 + t; blk < blk_end; blk += nthr) fmx = max(fmx, g.bmax[blk]);
        for (int64_t q = sb + 1 + t; q < g.nsb; q += nthr) fmx = max(fmx, g.bmax2[q]);
    }
}

// bounds of the accepted group S = [S0, b) and the change of T below it
// (records [k0, k1); an empty range when the change was applied ahead)
template <int H>
__device__ inline void accept_part(const ScanArgs& g, int64_t S0, int64_t b, int64_t k0, int64_t k1, long long mnS,
                                   long long mxS, int64_t t, int64_t nthr, int64_t gw, int64_t nwave) {
    for (int64_t j = S0 + t; j < b; j += nthr) {
        const int32_t x = g.order[j];
        g.lo[x] = mnS;
        g.hi[x] = mxS;
    }
    accept_walk<H>(g, S0, b, k0, k1, gw, nwave, 1);
}

// this workgroup's share of a posted phase (thread and wave indices over the
// phase's d[8] workgroups)
template <int H>
__device__ inline void run_posted(const ScanArgs& g, const long long* d, long long (*sred)[4]) {
    const int64_t t = (int64_t)blockIdx.x * kRT + threadIdx.x, nthr = d[8] * kRT;
    const int64_t gw = t >> 6, nwave = nthr >> 6;
    const int ph = (int)d[1];
    if (d[0] == PH_SEARCH) {
        const long long first = search_part(g, d[2], d[3], d[4] != 0, d[5], t, nthr);
        put_partial(g, ph, first, LLONG_MIN, LLONG_MIN, LLONG_MAX, sred);
    } else if (d[0] == PH_UPDATE) {
        update_walk<H>(g, d[2], d[3], d[4], d[5], d[6], gw, nwave, d[7] != 0);
    } else if (d[0] == PH_MINMAX) {
        long long vmn, vmx, fmx;
        minmax_part(g, d[2], d[3], t, nthr, vmn, vmx, fmx);
        put_partial(g, ph, vmn, vmx, fmx, LLONG_MAX, sred);
    } else if (d[0] == PH_ACCEPT) {
        accept_part<H>(g, d[2], d[3], d[4], d[5], d[6], d[7], t, nthr, gw, nwave);
    } else if (d[0] == PH_UNDO) {
        accept_walk<H>(g, d[2], d[3], d[4], d[5], gw, nwave, -1);
    }
}

// leader: publish phase descriptor d (uniform over the workgroup) to the
// helpers.  The post word carries the phase's sequence number and its
// workgroup count, (seq << 9) | (parts - 1), so that a helper outside the
// phase learns it from one load, without reading the descriptor (which the
// leader may already be rewriting for the next phase) or invalidating its
// caches; a helper inside it reads the descriptor, which cannot change
// before the helper arrives at the phase's barrier.
__device__ inline void post_phase(const ScanArgs& g, unsigned& posted, const long long* d) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    ++posted;
    if (threadIdx.x == 0) {
        for (int i = 0; i < kDesc; ++i) g.desc[i] = d[i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(g.bar + 2, (posted << 9) | (unsigned)(d[8] - 1), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ inline void heartbeat(const ScanArgs& g, unsigned& beat) {
    ++beat;
    if (threadIdx.x == 0) __hip_atomic_store(g.bar + 3, beat, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int H>
__device__ void scan_helper(const ScanArgs& g, long long (*sred)[4], int64_t* s_err) {
    __shared__ long long sd[kDesc];
    __shared__ unsigned s_seq, s_in;
    for (unsigned want = 1;;) {
        if (threadIdx.x == 0) {
            unsigned beat = __hip_atomic_load(g.bar + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned spins = 0, word = 0;
            bool ok = true;
            // a phase this workgroup is part of ends at a barrier it joins, so
            // the posts run ahead of it only by phases it is not part of (or
            // by the final exit after an error)
            for (;;) {
                word = __hip_atomic_load(g.bar + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((int)((word >> 9) - want) >= 0) break;
                __builtin_amdgcn_s_sleep(2);
                if ((++spins & 63) == 0) {  // the heartbeat is read now and then
                    const unsigned nb = __hip_atomic_load(g.bar + 3, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (nb != beat) {
                        beat = nb;
                        spins = 0;
                    }
                }
                if (spins > kSpinLimit) {
                    ok = false;
                    break;
                }
            }
            s_seq = word >> 9;
            s_in = ok ? (blockIdx.x <= (word & 511u) ? 1u : 0u) : 1u;
            if (!ok) {
                *s_err = 1;
                sd[0] = PH_EXIT;
            } else if (s_in) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                for (int i = 0; i < kDesc; ++i) sd[i] = g.desc[i];
            }
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const unsigned seq = s_seq, in = s_in;
        __syncthreads();  // read by every thread before thread 0 rewrites them
        want = seq + 1;
        if (!in) continue;  // not one of this phase's workgroups
        long long d[kDesc];
        for (int i = 0; i < kDesc; ++i) d[i] = sd[i];
        if (d[0] == PH_EXIT) break;
        run_posted<H>(g, d, sred);
        phase_barrier(g, (unsigned)d[9], s_err);
        if (*s_err) break;
    }
}

// The leader keeps the events of its last search window in LDS, one bit
// per position (bit i of word w: position lo + 64 w + i) for candidates and
// for stop positions.  Within a round nothing they depend on changes (T
// changes only when a group is accepted: a change applied ahead by an
// update walk is taken back before the next search; minH, R and I are
// fixed), so the search that follows a rejected boundary inside the window
// reads the bitmaps instead of memory.
constexpr int kEvWords = 128;  // windows of at most 8192 positions are kept

// first event at or after position `from` in the kept window [lo, hi) as a
// search code (2 j + 1 stop, 2 j candidate; LLONG_MAX none), in sh[0] and
// returned to every thread
__device__ inline long long first_kept(int64_t lo, int64_t hi, int64_t from, const uint64_t* evb,
                                       const uint64_t* stb, long long* sh) {
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        const int64_t w0 = (from - lo) / 64, w1 = (hi - lo + 63) / 64;
        long long code = LLONG_MAX;
        for (int64_t wb = w0; wb < w1 && code == LLONG_MAX; wb += 64) {
            const int64_t wi = wb + lane;
            uint64_t e = 0, st = 0;
            if (wi < w1) {
                e = evb[wi];
                st = stb[wi];
                const int64_t p0 = lo + 64 * wi;  // position of bit 0
                uint64_t keep = ~0ull;
                if (p0 < from) keep &= ~0ull << (from - p0);
                if (p0 + 64 > hi) keep &= (hi - p0 >= 64) ? ~0ull : ((1ull << (hi - p0)) - 1);
                e &= keep;
                st &= keep;
            }
            const uint64_t any = __ballot((e | st) != 0);
            if (any) {
                const int src = __ffsll((long long)any) - 1;  // first word with an event
                const uint64_t be = (uint64_t)__shfl((unsigned long long)e, src, 64);
                const uint64_t bs = (uint64_t)__shfl((unsigned long long)st, src, 64);
                const int bit = __ffsll((long long)(be | bs)) - 1;
                const int64_t j = lo + 64 * (wb + src) + bit;
                code = ((bs >> bit) & 1) ? 2 * j + 1 : 2 * j;
            }
        }
        if (lane == 0) sh[0] = code;
    }
    __syncthreads();
    return sh[0];
}

// leader: the events of [lo, hi) (hi - lo <= 64 kEvWords) into the bitmaps,
// then the first one; the loads of up to 4 kRT positions are in flight at once
__device__ inline long long search_kept(const ScanArgs& g, int64_t lo, int64_t hi, bool hasH, long long minH,
                                        uint64_t* evb, uint64_t* stb, long long* sh) {
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    for (int64_t base = 0; base < hi - lo; base += 4 * kRT) {
        int64_t Tv[4], Rn[4];
        uint8_t in[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = lo + base + u * kRT + t;
            Tv[u] = j < hi ? g.T[j] : 0;
            in[u] = j < hi ? g.inI[j] : 0;
            Rn[u] = (j < hi && j + 1 < g.n) ? g.R[j + 1] : LLONG_MIN;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t j = lo + base + u * kRT + t;
            const bool st = j < hi && hasH && Tv[u] >= minH;
            const bool ev = j < hi && !st && in[u] && Rn[u] < Tv[u];
            const uint64_t be = __ballot(ev), bs = __ballot(st);
            const int64_t wi = (base + u * kRT) / 64 + w;
            if (lane == 0 && wi < kEvWords) {
                evb[wi] = be;
                stb[wi] = bs;
            }
        }
    }
    __syncthreads();
    return first_kept(lo, hi, lo, evb, stb, sh);
}

template <int H>
__device__ void scan_leader(const ScanArgs& g, long long (*sred)[4], long long* sh, int64_t* s_err) {
    const unsigned nwg = gridDim.x;
    const bool grid = nwg > 1;
    const int64_t t = threadIdx.x, w = threadIdx.x >> 6;
    const int64_t n = g.n;
    int ph = 0;
    unsigned posted = 0, beat = 0;
    int64_t S0 = 0, fb = 0, kS0 = 0, kfb = 0, ng = 0, rounds = 0, verifs = 0;
    // phase profile: grid-wide phases and wall-clock ticks per kind (search,
    // update walk, min / max, acceptance), positions searched, records walked
    int64_t gridc[4] = {0, 0, 0, 0}, searched = 0, walked = 0;
    long long ticks[4] = {0, 0, 0, 0};
    long long minH = 0;
    bool hasH = false, failed = false;
    bool spec = false;  // the last update walk applied the change of T of accepting S ahead
    // a posted phase goes to the first parts_for(work) workgroups: one per
    // part_work records or positions, in multiples of 8, at least 8, so
    // that only the large walks occupy a wide grid
    unsigned arrivals = 0;  // barrier arrivals that every phase posted so far asks for
    auto parts_for = [&](int64_t work) -> long long {
        int64_t p = (work + g.part_work - 1) / g.part_work;
        p = max<int64_t>(8, (p + 7) / 8 * 8);
        return (long long)min<int64_t>((int64_t)nwg, p);
    };
    auto grid_phase = [&](long long* d, bool gather) {
        arrivals += (unsigned)d[8];
        d[9] = (long long)arrivals;
        post_phase(g, posted, d);
        run_posted<H>(g, d, sred);
        phase_barrier(g, arrivals, s_err);
        if (gather) gather_partials(g, (int)d[1], (unsigned)d[8], sh);
        if (posted >= (1u << 23) - 2) *s_err = 1;  // the post word holds 23 bits of sequence
    };
    __shared__ uint64_t evb[kEvWords], stb[kEvWords];  // the kept search window's events
    while (S0 < n && !failed) {
        ++rounds;
        bool accepted = false, stop = false;
        int64_t from = S0, accb = -1;
        long long mnS = 0, mxS = 0;
        int64_t win = 4 * kRT;  // grows while windows come back empty
        int64_t kept_lo = 0, kept_hi = 0;  // kept window (a round's windows only)
        while (!accepted && !stop && from < n && !failed) {
            heartbeat(g, beat);
            // first event in [from, hi): from the kept window when it holds
            // `from`, else by a new search
            const bool inkept = from >= kept_lo && from < kept_hi;
            const int64_t hi = inkept ? kept_hi : min(n, from + win);
            long long t0 = (long long)wall_clock64();
            if (inkept) {
                first_kept(kept_lo, kept_hi, from, evb, stb, sh);
            } else if (grid && hi - from > g.lead_pos) {
                kept_lo = kept_hi = 0;
                searched += hi - from;
                ++gridc[0];
                long long d[kDesc] = {PH_SEARCH, ph, from, hi, hasH ? 1 : 0, minH, 0, 0, parts_for(hi - from), 0};
                grid_phase(d, true);
            } else if (hi - from <= 64 * kEvWords) {
                searched += hi - from;
                search_kept(g, from, hi, hasH, minH, evb, stb, sh);
                kept_lo = from;
                kept_hi = hi;
            } else {
                searched += hi - from;
                kept_lo = kept_hi = 0;
                const long long first = search_part(g, from, hi, hasH, minH, t, kRT);
                reduce_local(first, LLONG_MIN, LLONG_MIN, LLONG_MAX, sred, sh);
            }
            ticks[0] += (long long)wall_clock64() - t0;
            ++ph;
            failed = *s_err != 0;
            const long long code = sh[0];
            if (failed) break;
            if (code == LLONG_MAX) {
                from = hi;
                if (!inkept) win = min<int64_t>(2 * win, kSearchWin);
                continue;
            }
            const long long e = code >> 1;
            if (code & 1) {
                stop = true;  // no boundary at or after e can pass
                break;
            }
            const int64_t b = e + 1;
            ++verifs;
            // positions [fb, b) join the pending group S = [S0, b); the
            // frontier of the loads below and the end of S always coincide:
            // both start at the accepted boundary and move to every verified b
            const int64_t k1 = g.P[b];
            t0 = (long long)wall_clock64();
            walked += k1 - kfb;
            // ahead only where the separate acceptance walk would be a grid
            // phase: a walk the leader runs alone costs less than the extra
            // atomics of applying it ahead
            spec = fb == S0 && grid && k1 - kfb > g.lead_recs;
            if (grid && k1 - kfb > g.lead_recs) {
                ++gridc[1];
                long long d[kDesc] = {PH_UPDATE, ph, S0, fb, b, kfb, k1, spec ? 1 : 0, parts_for(k1 - kfb), 0};
                grid_phase(d, false);
            } else {
                update_walk<H>(g, S0, fb, b, kfb, k1, w, kRW, spec);
                __syncthreads();
            }
            ticks[1] += (long long)wall_clock64() - t0;
            fb = b;
            kfb = k1;
            failed = *s_err != 0;
            if (failed) break;
            // min and max of the restricted loads of S, largest load below b
            const int64_t mm = (b - S0) + (b < n ? kFB + kSB + g.nsb - b / ((int64_t)kFB * kSB) : 0);
            t0 = (long long)wall_clock64();
            if (grid && mm > g.lead_pos) {
                ++gridc[2];
                long long d[kDesc] = {PH_MINMAX, ph, S0, b, 0, 0, 0, 0, parts_for(mm), 0};
                grid_phase(d, true);
            } else {
                long long vmn, vmx, fmx;
                minmax_part(g, S0, b, t, kRT, vmn, vmx, fmx);
                reduce_local(vmn, vmx, fmx, LLONG_MAX, sred, sh);
            }
            ticks[2] += (long long)wall_clock64() - t0;
            ++ph;
            failed = *s_err != 0;
            if (failed) break;
            mnS = sh[0];
            mxS = sh[1];
            const long long below = sh[2];
            bool ok = !(hasH && !(mxS < minH));
            ok = ok && (b == n || below < mnS);
            if (ok) {
                accepted = true;
                accb = b;
            } else {
                from = b;  // resume after the boundary examined
                if (spec) {  // take back the change of T applied ahead
                    t0 = (long long)wall_clock64();
                    walked += kfb - kS0;
                    if (grid && kfb - kS0 > g.lead_recs) {
                        ++gridc[3];
                        long long d[kDesc] = {PH_UNDO, ph, S0, b, kS0, kfb, 0, 0, parts_for(kfb - kS0), 0};
                        grid_phase(d, false);
                    } else {
                        accept_walk<H>(g, S0, b, kS0, kfb, w, kRW, -1);
                        __syncthreads();
                    }
                    ticks[3] += (long long)wall_clock64() - t0;
                    spec = false;
                    failed = *s_err != 0;
                }
            }
        }
        if (!accepted || failed) break;  // the rest is never accepted: no bounds
        const int64_t b = accb;  // == fb, so P[b] == kfb
        const long long t0 = (long long)wall_clock64();
        // the change of T is still to make unless the boundary's update walk
        // applied it ahead
        const int64_t k0 = spec ? kfb : kS0;
        walked += kfb - k0;
        if (grid && (b - S0 > g.lead_pos || kfb - k0 > g.lead_recs)) {
            ++gridc[3];
            long long d[kDesc] = {PH_ACCEPT, ph, S0, b, k0, kfb, mnS, mxS, parts_for(max(b - S0, kfb - k0)), 0};
            grid_phase(d, false);
        } else {
            accept_part<H>(g, S0, b, k0, kfb, mnS, mxS, t, kRT, w, kRW);
            __syncthreads();
        }
        ticks[3] += (long long)wall_clock64() - t0;
        if (threadIdx.x == 0) {
            g.groups[2 * ng] = S0;
            g.groups[2 * ng + 1] = b;
        }
        ++ng;
        failed = *s_err != 0;
        minH = mnS;
        hasH = true;
        S0 = b;
        kS0 = kfb;
    }
    if (grid) {
        const long long d[kDesc] = {PH_EXIT, 0, 0, 0, 0, 0, 0, 0, (long long)nwg, 0};  // every helper leaves
        post_phase(g, posted, d);
    }
    if (threadIdx.x == 0) {
        g.info[0] = ng;
        g.info[1] = rounds;
        g.info[2] = verifs;
        for (int k = 0; k < 4; ++k) {
            g.info[4 + k] = gridc[k];
            g.info[8 + k] = ticks[k];
        }
        g.info[12] = searched;
        g.info[13] = walked;
    }
}

template <int H>
__global__ __launch_bounds__(kRT) void k_sg_scan(ScanArgs g) {
    __shared__ long long sred[kRW][4];
    __shared__ long long sh[4];
    __shared__ int64_t s_err;
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();
    if (blockIdx.x == 0)
        scan_leader<H>(g, sred, sh, &s_err);
    else
        scan_helper<H>(g, sred, &s_err);
    __syncthreads();
    if (threadIdx.x == 0 && s_err) g.info[3] = 1;
}

// the records of every slot in position order (needs the order and the
// split numerators), with R and T by position (q.R, q.T) and, when c is
// given, the a8 counts c_j (c: n entries, filled with zero by the caller)
void build_records(Graph& g, int mode, const PassArgs& a, hipStream_t s, int64_t* c) {
    SgState& q = g.sg[mode == 2 ? 0 : 1];
    const SweepPlan& pl = (mode == 2) ? g.edge_plan : g.tri_plan;
    const int64_t n = g.n;
    q.rec_P.alloc(n + 1, s);
    k_fill_i64<<<grid_for(n + 1, kT), kT, 0, s>>>(q.rec_P.p, n + 1, 0);
    q.R.alloc(n, s);
    q.T.alloc(n, s);
    if (n > 0) {
        k_fill_i64<<<grid_for(n, kT), kT, 0, s>>>(q.R.p, n, 0);
        k_fill_i64<<<grid_for(n, kT), kT, 0, s>>>(q.T.p, n, 0);
    }
    LDS_HIP(hipGetLastError());
    q.rec_own.alloc(pl.nslots, s);
    if (mode == 2) {
        q.rec2.alloc(pl.nslots, s);
        q.rec3.release();
        q.rec3w.release();
    } else {
        q.rec2.release();
        q.rec3.alloc(pl.nslots, s);
        q.rec3w.alloc(pl.nslots, s);
    }
    if (pl.nrows == 0) return;
    k_pos_slots<<<grid_for(pl.nrows, kT), kT, 0, s>>>(a, (uint64_t*)q.rec_P.p);
    exclusive_scan_u64((const uint64_t*)q.rec_P.p, (uint64_t*)q.rec_P.p, n, (uint64_t*)q.rec_P.p + n, s);
    // length classes: more than 32 slots (a wave per row), 17-32 (32 lanes),
    // 9-16 (16 lanes), at most 8 (8 lanes)
    int64_t cls[3] = {0, 0, 0};
    {
        DBuf<int64_t> d;
        d.alloc(3, s);
        k_record_classes<<<1, 64, 0, s>>>(pl.rp, pl.nrows, d.p);
        LDS_HIP(hipGetLastError());
        LDS_HIP(hipMemcpyAsync(cls, d.p, sizeof(cls), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
    }
    const int64_t b1 = cls[0], b2 = std::max(b1, cls[1]), b3 = std::max(b2, cls[2]), b4 = pl.nrows;
    const int wpb = kT / 64;  // waves per workgroup
    auto launch = [&](auto h, int64_t lo, int64_t hi, auto gl) {
        constexpr int H = decltype(h)::value, G = decltype(gl)::value;
        if (hi <= lo) return;
        const int64_t waves = (hi - lo + 64 / G - 1) / (64 / G);
        k_slot_records<H, G><<<grid_for(waves, wpb), kT, 0, s>>>(a, lo, hi, q.rec_P.p, q.rec_own.p, q.rec2.p,
                                                                 q.rec3.p, q.rec3w.p, c, q.R.p, q.T.p);
        LDS_HIP(hipGetLastError());
    };
    // (triangle rows stay one per wave: their slots gather the pattern's
    // vertices, split numerators and positions, and the shared waves were
    // slower there: 1.86 against 1.66 ms on ltds_hk; edges: 2.5 against 3.3 ms
    // on lds_large)
    if (mode == 2) {
        using H2 = std::integral_constant<int, 2>;
        launch(H2{}, 0, b1, std::integral_constant<int, 64>{});
        launch(H2{}, b1, b2, std::integral_constant<int, 32>{});
        launch(H2{}, b2, b3, std::integral_constant<int, 16>{});
        launch(H2{}, b3, b4, std::integral_constant<int, 8>{});
    } else {
        launch(std::integral_constant<int, 3>{}, 0, b4, std::integral_constant<int, 64>{});
    }
}

// the hub rows' slots past their hub prefixes, from the non-hub rows' splits
// (see k_hub_nb_count); every other slot of a_slot is already set
void hub_suffix_splits(const SweepPlan& p, uint32_t D, uint32_t* a_slot, hipStream_t s) {
    const int64_t Hp = p.n_push, r0 = Hp, r1 = p.nrows, nr = r1 - r0;
    if (Hp <= 0 || nr <= 0) return;
    DBuf<uint32_t> cnt, len;
    DBuf<uint64_t> off, first, tot;
    cnt.alloc(nr, s);
    off.alloc(nr, s);
    tot.alloc(1, s);
    k_hub_nb_count<<<grid_for(nr, kT), kT, 0, s>>>(p.rp, p.py, r0, r1, (int32_t)Hp, cnt.p);
    LDS_HIP(hipGetLastError());
    exclusive_scan_u32_to_u64(cnt.p, off.p, nr, tot.p, s);
    uint64_t np = 0;
    LDS_HIP(hipMemcpyAsync(&np, tot.p, sizeof(np), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    if (np == 0) return;
    DBuf<uint64_t> keys, tkeys;
    DBuf<uint32_t> vals, tvals;
    keys.alloc(np, s);
    tkeys.alloc(np, s);
    vals.alloc(np, s);
    tvals.alloc(np, s);
    k_hub_nb_pairs<<<grid_for(nr, kT), kT, 0, s>>>(p.rp, p.py, r0, r1, cnt.p, off.p, a_slot, keys.p, vals.p);
    LDS_HIP(hipGetLastError());
    radix_sort_u64(keys.p, vals.p, (int64_t)np, std::max(1, bits_for((uint64_t)(Hp - 1))), tkeys.p, tvals.p, s);
    len.alloc(Hp, s);
    first.alloc(Hp, s);
    k_hub_sfx_len<<<grid_for(Hp, kT), kT, 0, s>>>(p.rp, p.hub_pre.p, Hp, len.p);
    LDS_HIP(hipGetLastError());
    exclusive_scan_u32_to_u64(len.p, first.p, Hp, tot.p, s);
    k_hub_scatter<<<grid_for((int64_t)np, kT), kT, 0, s>>>(keys.p, vals.p, (int64_t)np, first.p, p.rp, p.hub_pre.p,
                                                          D, a_slot);
    LDS_HIP(hipGetLastError());
}

ScanArgs record_args(const SgState& q, const PassArgs& a) {
    ScanArgs r{};
    r.a = a;
    r.P = q.rec_P.p;
    r.own = q.rec_own.p;
    r.rec2 = q.rec2.p;
    r.rec3 = q.rec3.p;
    r.rec3w = q.rec3w.p;
    return r;
}

PassArgs plan_args(const Graph& g, int mode, PassArgs a) {
    const SweepPlan& p = (mode == 2) ? g.edge_plan : g.tri_plan;
    a.rid = p.rid;
    a.rp = p.rp;
    a.py = p.py;
    a.tos = p.own_tos.p;
    a.tri = g.tri.p;
    a.row_of = p.own_row_of.p;
    a.nrows = p.nrows;
    a.n_big = p.n_big;
    return a;
}

}  // namespace

void sg_sort_prefix(Graph& g, int mode, hipStream_t s) {
    FwState& f = g.fw[mode == 2 ? 0 : 1];
    SgState& q = g.sg[mode == 2 ? 0 : 1];
    LDS_CHECK(f.ran && f.K[0].n == (size_t)g.n, ST_INVALID,
              "no Frank-Wolfe state: call lds_frank_wolfe first");
    check_split_width(mode, f.iters);
    const SweepPlan& p = (mode == 2) ? g.edge_plan : g.tri_plan;
    const int64_t n = g.n;
    q.valid = false;
    q.iters = f.iters;
    q.order.alloc(n, s);
    q.pos.alloc(n, s);
    q.E.alloc(n, s);
    q.inI.alloc(n, s);
    if (n == 0) {
        q.valid = true;
        return;
    }
    // a7: sort
    {
        DBuf<uint64_t> k, kt;
        DBuf<uint32_t> v, vt;
        k.alloc(n, s);
        kt.alloc(n, s);
        v.alloc(n, s);
        vt.alloc(n, s);
        k_sort_init<<<grid_for(n, kT), kT, 0, s>>>(f.K[f.cur].p, n, k.p, v.p);
        LDS_HIP(hipGetLastError());
        const int kb = g.idbits + bits_for((uint64_t)fw_max_numerator(g, mode, f.iters));
        radix_sort_u64(k.p, v.p, n, std::min(kb, 64), kt.p, vt.p, s);
        k_order<<<grid_for(n, kT), kT, 0, s>>>(v.p, n, q.order.p, q.pos.p);
        LDS_HIP(hipGetLastError());
    }
    // per-slot split numerators (and per triangle)
    q.a_slot.alloc(p.nslots, s);
    if (p.nslots > 0 && f.iters >= 0) {
        const HeavyPlan& hv = p.heavy;
        // with the hub push only the pieces of the hub prefixes carry decision
        // bits; the rest of the hub rows comes from the mirror slots below
        const bool push = p.n_push > 0;
        const int64_t npc = push ? p.n_ppieces : p.n_pieces;
        const int64_t blocks = npc + p.n_chunks + (hv.positions + kPiece - 1) / kPiece;
        k_slot_splits<<<grid_for(blocks, 1), kT, 0, s>>>(p.rp, npc, push ? p.pp_row.p : p.hp_row.p,
                                                         push ? p.pp_off.p : p.hp_off.p, p.hwo.p, p.n_chunks,
                                                         p.chunk_row.p, p.cwo.p, p.chunk_words, f.bits.p,
                                                         p.total_words, f.iters, mode == 3, hv.positions, hv.word0,
                                                         hv.csr.p, q.a_slot.p);
        LDS_HIP(hipGetLastError());
        if (p.n_push > 0) hub_suffix_splits(p, (uint32_t)fw_denom(mode, f.iters), q.a_slot.p, s);
    }
    if (mode == 3) {
        q.a_tri.alloc(3 * g.T, s);
        if (g.T > 0) {
            k_tri_splits<<<grid_for(p.nslots, kT), kT, 0, s>>>(p.py, p.own_tos.p, g.tri.p, q.a_slot.p, p.nslots,
                                                              q.a_tri.p);
            LDS_HIP(hipGetLastError());
        }
    }
    // the records of every slot in position order, then a8: counts by
    // position from them, prefix, suffix maxima
    PassArgs a{};
    a.a_slot = q.a_slot.p;
    a.a_tri = q.a_tri.p;
    a.pos = q.pos.p;
    a.D = fw_denom(mode, f.iters);
    a = plan_args(g, mode, a);
    DBuf<int64_t> c;
    c.alloc(n, s);
    if (n > 0) k_fill_i64<<<grid_for(n, kT), kT, 0, s>>>(c.p, n, 0);
    LDS_HIP(hipGetLastError());
    build_records(g, mode, a, s, c.p);
    {
        DBuf<uint64_t> ex;
        ex.alloc(n, s);
        exclusive_scan_u64((const uint64_t*)c.p, ex.p, n, nullptr, s);
        k_inclusive<<<grid_for(n, kT), kT, 0, s>>>(ex.p, c.p, n, q.E.p);
        LDS_HIP(hipGetLastError());
    }
    const int64_t tiles = (n + kTile - 1) / kTile;
    DBuf<int64_t> tn, td;
    tn.alloc(tiles, s);
    td.alloc(tiles, s);
    k_tile_fmax<<<grid_for(tiles, 1), kT, 0, s>>>(q.E.p, n, tn.p, td.p);
    LDS_HIP(hipGetLastError());
    DBuf<int64_t> cn, cd;
    cn.alloc(tiles, s);
    cd.alloc(tiles, s);
    k_tile_carry<<<1, kT, 0, s>>>(tn.p, td.p, tiles, cn.p, cd.p);
    LDS_HIP(hipGetLastError());
    k_tile_inI<<<grid_for(tiles, 1), kT, 0, s>>>(q.E.p, n, cn.p, cd.p, q.inI.p);
    LDS_HIP(hipGetLastError());
    q.valid = true;
    q.gstart.clear();
    q.gend.clear();
}

void sg_stable_groups(Graph& g, int mode, hipStream_t s) {
    SgState& q = g.sg[mode == 2 ? 0 : 1];
    const FwState& f = g.fw[mode == 2 ? 0 : 1];
    if (!q.valid || q.iters != f.iters) sg_sort_prefix(g, mode, s);
    const int64_t n = g.n;
    q.gstart.clear();
    q.gend.clear();
    q.lo.alloc(n, s);
    q.hi.alloc(n, s);
    q.rounds = q.verifications = 0;
    if (n == 0) return;
    k_fill_i64<<<grid_for(n, kT), kT, 0, s>>>(q.lo.p, n, -1);
    k_fill_i64<<<grid_for(n, kT), kT, 0, s>>>(q.hi.p, n, -1);
    PassArgs a{};
    a.a_slot = q.a_slot.p;
    a.a_tri = q.a_tri.p;
    a.pos = q.pos.p;
    a.D = fw_denom(mode, f.iters);
    a = plan_args(g, mode, a);

    // the slot records with R_w (w's restricted load when every earlier
    // vertex is above it) and T_x for S0 = 0 (kept from the sort / prefix
    // pass unless a scan since released them); the scan keeps T current
    if (q.rec_P.n != (size_t)n + 1) build_records(g, mode, a, s, nullptr);
    const ScanArgs rv = record_args(q, a);

    // the round loop: one cooperative launch
    const int64_t nblk = (n + kFB - 1) / kFB;
    DBuf<int64_t> F, Vb, groups, info;
    DBuf<long long> bmax, part;
    DBuf<unsigned> bar;
    F.alloc(n, s);
    Vb.alloc(n, s);
    k_fill_i64<<<grid_for(n, kT), kT, 0, s>>>(Vb.p, n, 0);  // each position's own load is added once
    bmax.alloc(nblk, s);
    k_f_init<<<grid_for(n, kT), kT, 0, s>>>(f.K[f.cur].p, q.order.p, n, g.idbits, F.p);
    k_bmax_init<<<grid_for(nblk, 1), kT, 0, s>>>(F.p, n, bmax.p);
    const int64_t nsb = (nblk + kSB - 1) / kSB;
    DBuf<long long> bmax2;
    bmax2.alloc(nsb, s);
    k_bmax2_init<<<grid_for(nsb, 1), 64, 0, s>>>(bmax.p, nblk, bmax2.p);
    LDS_HIP(hipGetLastError());
    static int cus = 0, per[2] = {0, 0};
    if (!cus) {
        int dev = 0;
        LDS_HIP(hipGetDevice(&dev));
        LDS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        LDS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per[0], k_sg_scan<2>, kRT, 0));
        LDS_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per[1], k_sg_scan<3>, kRT, 0));
    }
    const int64_t resident = (int64_t)cus * std::max(1, per[mode == 2 ? 0 : 1]);
    // the helpers only join the large phases, and each phase only as many of
    // them as its work needs
    auto env_i64 = [](const char* name, int64_t def) {
        const char* v = std::getenv(name);
        return (v && *v) ? std::max<int64_t>(0, std::atoll(v)) : def;
    };
    const int64_t wg_env = env_i64("LDS_SCAN_WG", 0);
    // (at most 512: the post word holds a phase's workgroup count in 9 bits)
    const int64_t grid = std::min<int64_t>(
        512, std::max<int64_t>(1, wg_env ? std::min<int64_t>(resident, wg_env)
                                         : (n <= 16384 ? 1 : std::min<int64_t>(resident, (int64_t)kScanMaxWG))));
    groups.alloc(2 * n, s);
    info.alloc(16, s);
    part.alloc((size_t)2 * grid * 4, s);
    bar.alloc(4, s);
    DBuf<long long> desc;
    desc.alloc(kDesc, s);
    k_fill_i64<<<1, kT, 0, s>>>(info.p, 16, 0);
    k_fill_i64<<<1, kT, 0, s>>>((int64_t*)bar.p, 2, 0);
    k_fill_i64<<<1, kT, 0, s>>>((int64_t*)desc.p, kDesc, 0);
    LDS_HIP(hipGetLastError());
    ScanArgs sa{};
    sa.a = a;
    sa.order = q.order.p;
    sa.inI = q.inI.p;
    sa.R = q.R.p;
    sa.T = q.T.p;
    sa.F = F.p;
    sa.V = Vb.p;
    sa.bmax = bmax.p;
    sa.bmax2 = bmax2.p;
    sa.nsb = nsb;
    sa.nblk = nblk;
    sa.n = n;
    sa.lo = q.lo.p;
    sa.hi = q.hi.p;
    sa.groups = groups.p;
    sa.info = info.p;
    sa.part = part.p;
    sa.bar = bar.p;
    sa.desc = desc.p;
    sa.lead_recs = env_i64("LDS_SCAN_LEAD_RECS", kLeadRecs);
    sa.part_work = std::max<int64_t>(1, env_i64("LDS_SCAN_PART_WORK", kPartWork));
    sa.lead_pos = env_i64("LDS_SCAN_LEAD_POS", kLeadPos);
    sa.P = rv.P;
    sa.own = rv.own;
    sa.rec2 = rv.rec2;
    sa.rec3 = rv.rec3;
    sa.rec3w = rv.rec3w;
    if (grid == 1) {  // one workgroup needs no co-residency guarantee
        if (mode == 2)
            k_sg_scan<2><<<1, kRT, 0, s>>>(sa);
        else
            k_sg_scan<3><<<1, kRT, 0, s>>>(sa);
        LDS_HIP(hipGetLastError());
    } else {
        void* kargs[] = {&sa};
        LDS_HIP(hipLaunchCooperativeKernel(mode == 2 ? (const void*)k_sg_scan<2> : (const void*)k_sg_scan<3>,
                                           dim3((unsigned)grid), dim3(kRT), kargs, 0, s));
    }
    int64_t hinfo[16];
    LDS_HIP(hipMemcpyAsync(hinfo, info.p, sizeof(hinfo), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    LDS_CHECK(hinfo[3] == 0, ST_DEVICE, "stable-group scan: a grid barrier did not complete");
    const int64_t ng = hinfo[0];
    q.rounds = hinfo[1];
    q.verifications = hinfo[2];
    static int rate_khz = 0;  // wall clock of the device
    if (!rate_khz) {
        int dev = 0;
        LDS_HIP(hipGetDevice(&dev));
        LDS_HIP(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    }
    for (int k = 0; k < 10; ++k) q.scan_profile[k] = hinfo[4 + k];
    for (int k = 4; k < 8; ++k) q.scan_profile[k] = q.scan_profile[k] * 1000 / std::max(rate_khz, 1);
    q.scan_wg = grid;
    // the records are only read by the scan (the stream has finished it)
    q.rec_P.release();
    q.rec_own.release();
    q.rec2.release();
    q.rec3.release();
    q.rec3w.release();
    q.R.release();
    q.T.release();  // changed by the scan
    std::vector<int64_t> hg((size_t)2 * ng);
    if (ng > 0) {
        LDS_HIP(hipMemcpyAsync(hg.data(), groups.p, hg.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
    }
    for (int64_t i = 0; i < ng; ++i) {
        q.gstart.push_back(hg[2 * i]);
        q.gend.push_back(hg[2 * i + 1]);
    }
}

namespace {
__global__ void k_by_orig(const int64_t* lo, const int64_t* hi, const int32_t* orig_of, int64_t n, int64_t* out) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const int64_t o = orig_of[i];
    out[o] = lo[i];
    out[n + o] = hi[i];
}
}  // namespace

namespace {
// out[i] = src[idx[i]]; an index outside [0, n_src) raises *err and gives 0
__global__ void k_gather_u32(const uint32_t* src, int64_t n_src, const int64_t* idx, int64_t n, uint32_t* out,
                             int32_t* err) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const int64_t j = idx[i];
    if (j < 0 || j >= n_src) {
        *err = 1;
        out[i] = 0;
        return;
    }
    out[i] = src[j];
}
}  // namespace

void gather_split(const Graph& g, int mode, const int64_t* idx, int64_t n, uint32_t* out, hipStream_t s) {
    if (n <= 0) return;
    const SgState& q = g.sg[mode == 2 ? 0 : 1];
    const uint32_t* src = mode == 2 ? q.a_slot.p : q.a_tri.p;
    const int64_t n_src = mode == 2 ? 2 * g.m : 3 * g.T;
    LDS_CHECK(src != nullptr && n_src > 0, ST_INVALID, "split gather: no split numerators for this mode");
    DBuf<int64_t> di;
    DBuf<uint32_t> dout;
    DBuf<int32_t> err;
    di.alloc(n, s);
    dout.alloc(n, s);
    err.alloc(1, s);
    LDS_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
    LDS_HIP(hipMemcpyAsync(di.p, idx, n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    k_gather_u32<<<grid_for(n, kT), kT, 0, s>>>(src, n_src, di.p, n, dout.p, err.p);
    LDS_HIP(hipGetLastError());
    int32_t bad = 0;
    LDS_HIP(hipMemcpyAsync(out, dout.p, n * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipMemcpyAsync(&bad, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    LDS_CHECK(bad == 0, ST_INVALID, "split gather: index out of range");
}

void sg_copy_bounds(const Graph& g, int mode, int64_t* lo_out, int64_t* hi_out, hipStream_t s) {
    const SgState& q = g.sg[mode == 2 ? 0 : 1];
    const int64_t n = g.n;
    if (n == 0 || (!lo_out && !hi_out)) return;
    DBuf<int64_t> out;
    out.alloc((size_t)2 * n, s);
    k_by_orig<<<grid_for(n, kT), kT, 0, s>>>(q.lo.p, q.hi.p, g.orig_of.p, n, out.p);
    LDS_HIP(hipGetLastError());
    if (lo_out) LDS_HIP(hipMemcpyAsync(lo_out, out.p, n * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (hi_out) LDS_HIP(hipMemcpyAsync(hi_out, out.p + n, n * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
}

}  // namespace lds
