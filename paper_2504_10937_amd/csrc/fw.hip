// Frank-Wolfe iterations of Alg. 1 (edges, Eq. cp) and Alg. 6 (triangles,
// Eq. trcp) on gfx950, in exact integer form, and the same iteration over
// 4-cliques (the h-clique program that Eq. trcp generalises, h = 4).
//
// State.  With gamma_i = 2/(i+2) every load is r_u^(i) = A_u / D_i with the
// common denominator D_i = (i+1)(i+2) (edges), 3(i+1)(i+2) (triangles) or
// 2(i+1)(i+2) (4-cliques), and the update r <- (1-gamma) r + gamma b becomes
// A_u += inc_i * b_u with inc_i = D_i - D_{i-1} = 2(i+1), 6(i+1) or 4(i+1),
// b_u = units won in iteration i.  Each vertex carries one packed 64-bit key
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
//   * hub pieces: a row with more slots than a chunk is cut into word-aligned
//     pieces of at most kPiece slots, one wave each, scheduled before the
//     chunks over all waves; a piece adds its wins to the row's counter and
//     the wave that completes the row's last piece writes the row's key.
// The duality-gap terms sum_u A_u^2 and sum_u A_u b_u (= sum over patterns of
// the winning numerator, i.e. the minimum) are accumulated exactly in 128-bit
// integers per workgroup and reduced once after the last iteration.
#include "graph.hpp"
#include "push.hpp"

#include <mutex>

// Scratch of lds_frank_wolfe_noalloc, for callers that cannot allocate device
// memory: the per-workgroup gap partial sums of every iteration, their
// per-iteration totals and the gap values.  One copy per device (4 MiB),
// held until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device.
static constexpr size_t kScratchWords = (size_t)1 << 19;
static __device__ __align__(256) uint64_t scratch[kScratchWords];

namespace lds {

namespace {

typedef unsigned __int128 u128;

struct SweepArgs {
    const int32_t* rid;
    const int64_t* rp;
    const int32_t* py;
    int64_t n_hub;
    const int64_t* hwo;
    int64_t n_pieces;
    const int32_t* hp_row;
    const int32_t* hp_off;
    unsigned long long* hub_ctr;  // per hub row: (pieces done << 40) | wins so far
    int64_t n_chunks;
    const int64_t* chunk_row;
    const int64_t* cwo;
    const uint64_t* head;
    int64_t chunk_words;
    const uint64_t* Kin;
    uint64_t* Kout;
    const uint16_t* Qin;  // 16-bit codes of the loads (see qcode)
    uint16_t* Qout;
    uint64_t* bits;      // this iteration's decision words
    uint64_t inc;
    int B;
    uint64_t* partial;   // 4 words per workgroup (or nullptr)
    int ncache;          // codes staged in LDS: min(n, kCacheQ)
    // 2D part (edge plans of large graphs; n_parts = 0 otherwise)
    int64_t n_parts;
    const int32_t* part_blk;
    const int32_t* part_j0;
    const int32_t* part_j1;
    const int64_t* part_lo;
    const int64_t* part_hi;
    const int64_t* hseg;
    const int64_t* hblk_row;
    const uint32_t* hpay;
    uint32_t* part_cnt;
    int64_t hP;
    int hR, hC;
    int64_t n_heavy;
    int64_t hword0;
    int64_t nv;          // vertices (slabs are clipped to it)
    // hub push (n_push > 0; edge plans only): the pieces above are those of
    // the hub prefixes, hub_pre[r] slots of hub row r; every workgroup stores
    // its hub counters (pstride words, two 16-bit counts each) at
    // push_part + blockIdx * pstride
    int64_t n_push;
    const int32_t* hub_pre;
    uint32_t* push_part;
    int64_t pstride;
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

// 16-bit monotone code of a load numerator: a pseudo-float with the 6-bit
// position of the leading one and the next 10 bits (0 for A = 0).  A < A'
// implies qcode(A) <= qcode(A'), so different codes decide a comparison of
// packed keys exactly and equal codes fall back to the 64-bit keys.  The code
// array is a quarter of the key array, so the gathered working set stays in
// the L2 caches far more often.
__device__ inline uint16_t qcode(uint64_t A) {
    if (A == 0) return 0;
    const int e = 63 - __clzll(A);
    const uint64_t mant = (e >= 10) ? (A >> (e - 10)) : (A << (10 - e));
    return (uint16_t)(((uint32_t)e << 10) | (uint32_t)(mant & 0x3FFu));
}

// does the row vertex (key ku, code qu) beat the vertex with code qv, whose
// 64-bit key is gathered only when the codes tie?
__device__ inline bool beats(uint64_t ku, uint16_t qu, uint16_t qv, const uint64_t* __restrict__ K, int32_t v) {
    if (qu != qv) return qu < qv;
    return ku < K[v];
}

// the h-1 other vertices of the pattern stored at a slot; the slot arrays
// are streamed once per iteration, so they are read non-temporally to keep
// the caches for the gathered keys
template <int H>
struct Slot {
    int32_t v[H - 1];
};

template <int H>
__device__ inline Slot<H> load_slot(const int32_t* __restrict__ py, int64_t s);
template <>
__device__ inline Slot<2> load_slot<2>(const int32_t* __restrict__ py, int64_t s) {
    Slot<2> r;
    r.v[0] = __builtin_nontemporal_load(py + s);
    return r;
}
template <>
__device__ inline Slot<3> load_slot<3>(const int32_t* __restrict__ py, int64_t s) {
    const long long x = __builtin_nontemporal_load(reinterpret_cast<const long long*>(py) + s);
    Slot<3> r;
    r.v[0] = (int32_t)(uint32_t)(unsigned long long)x;
    r.v[1] = (int32_t)(uint32_t)((unsigned long long)x >> 32);
    return r;
}
template <>
__device__ inline Slot<4> load_slot<4>(const int32_t* __restrict__ py, int64_t s) {
    Slot<4> r;
    r.v[0] = __builtin_nontemporal_load(py + 3 * s);
    r.v[1] = __builtin_nontemporal_load(py + 3 * s + 1);
    r.v[2] = __builtin_nontemporal_load(py + 3 * s + 2);
    return r;
}

#ifndef LDS_SWEEP_WORDS
#define LDS_SWEEP_WORDS 8
#endif
#ifndef LDS_SWEEP_THREADS
#define LDS_SWEEP_THREADS 1024
#endif
#ifndef LDS_SWEEP_CACHE
#define LDS_SWEEP_CACHE 77824
#endif
#ifndef LDS_SWEEP_WG_PER_CU
#define LDS_SWEEP_WG_PER_CU 1
#endif
constexpr int kG = LDS_SWEEP_WORDS;         // 64-slot words of a chunk in flight per wave
constexpr int kPT = LDS_SWEEP_THREADS;      // threads of a persistent workgroup
constexpr int kWaves = kPT / 64;
constexpr int kCacheQ = LDS_SWEEP_CACHE;    // codes of the first (highest-degree) vertices staged in LDS
constexpr int kWgPerCU = LDS_SWEEP_WG_PER_CU;

// code of vertex v: from the LDS copy for the hot prefix, else from memory
__device__ inline uint16_t qload(const uint16_t* __restrict__ qc, int nc, const uint16_t* __restrict__ Q,
                                 uint32_t v) {
    uint16_t q;
    if (v < (uint32_t)nc)
        q = qc[v];
    else
        q = Q[v];
    return q;
}

// LDS bytes of the 2D part: block codes (u16) and win counts (u32), two slabs
constexpr size_t kHeavyLds = (size_t)kHeavyRows * 2 + (size_t)kHeavyRows * 4 + (size_t)2 * kHeavySlab * 2;
constexpr int kSlabChunks = (kHeavySlab / 8 + kPT - 1) / kPT;  // 16-byte chunks of a slab per thread

// slab j's codes, 16 bytes (8 codes) per chunk, clipped to the vertex count
__device__ inline void slab_load(const uint16_t* __restrict__ Q, int64_t nv, int64_t first, int C, uint4 (&st)[kSlabChunks]) {
#pragma unroll
    for (int q = 0; q < kSlabChunks; ++q) {
        const int c = (int)threadIdx.x + kPT * q;
        const int64_t v = first + 8 * (int64_t)c;
        uint4 x = make_uint4(0, 0, 0, 0);
        if (8 * c < C) {
            if (v + 8 <= nv) {
                x = *reinterpret_cast<const uint4*>(Q + v);
            } else {
                uint16_t e[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) e[k] = (v + k < nv) ? Q[v + k] : (uint16_t)0;
                x.x = e[0] | ((uint32_t)e[1] << 16);
                x.y = e[2] | ((uint32_t)e[3] << 16);
                x.z = e[4] | ((uint32_t)e[5] << 16);
                x.w = e[6] | ((uint32_t)e[7] << 16);
            }
        }
        st[q] = x;
    }
}

__device__ inline void slab_store(uint16_t* __restrict__ slab, int C, const uint4 (&st)[kSlabChunks]) {
#pragma unroll
    for (int q = 0; q < kSlabChunks; ++q) {
        const int c = (int)threadIdx.x + kPT * q;
        if (8 * c < C) reinterpret_cast<uint4*>(slab)[c] = st[q];
    }
}

// The 2D part of an edge sweep (heavy rows; see HeavyPlan).  A workgroup
// takes whole parts.  It stages the block's codes and zeroed win counts in
// LDS, then walks the part's slabs: slab j's codes sit in one LDS buffer
// while the next slab's are loaded into registers and stored into the other
// buffer; the segment's words are decided with both codes from LDS (64-bit
// keys only on equal codes), each word's ballot is its decision word, and
// the wins of each run of one row within a word are added to the row's LDS
// count once.  The part's counts go to part_cnt; k_heavy_finish sums the
// parts of each row after the sweep.
template <bool ENABLE>
__device__ inline void heavy_parts(const SweepArgs& a, uint8_t* dyn, int64_t* sgc) {
    if constexpr (ENABLE) {
        const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
        const int R = a.hR, C = a.hC;
        uint16_t* rq = reinterpret_cast<uint16_t*>(dyn);
        uint32_t* rc = reinterpret_cast<uint32_t*>(dyn + (size_t)kHeavyRows * 2);
        uint16_t* slabs = reinterpret_cast<uint16_t*>(dyn + (size_t)kHeavyRows * 6);
        const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
        for (int64_t pt = blockIdx.x; pt < a.n_parts; pt += gridDim.x) {
            const int64_t b = a.part_blk[pt];
            const int64_t j0 = a.part_j0[pt], j1 = a.part_j1[pt];
            const int64_t lo = a.part_lo[pt], hi = a.part_hi[pt];
            const int64_t row0 = a.hblk_row[b];
            const int nr = (int)(a.hblk_row[b + 1] - row0);
            // the part's segment bounds, clipped to its positions, staged in
            // LDS when they fit (a few hundred slabs)
            const int64_t* sgg = a.hseg + b * a.hP;
            const bool cached = j1 - j0 + 1 <= kWaves * 32;
            for (int64_t k = threadIdx.x; cached && k <= j1 - j0; k += kPT) sgc[k] = min(max(sgg[j0 + k], lo), hi);
            for (int i = threadIdx.x; i < nr; i += kPT) {
                rq[i] = a.Qin[row0 + i];
                rc[i] = 0u;
            }
            __syncthreads();
            auto bound = [&](int64_t j) { return cached ? sgc[j - j0] : min(max(sgg[j], lo), hi); };
            auto next_j = [&](int64_t j) {
                while (j < j1 && bound(j + 1) <= bound(j)) ++j;
                return j;
            };
            int64_t j = next_j(j0);
            uint4 st[kSlabChunks];
            if (j < j1) {
                slab_load(a.Qin, a.nv, j * C, C, st);
                slab_store(slabs, C, st);
            }
            __syncthreads();
            int cur = 0;
            while (j < j1) {
                const int64_t jn = next_j(j + 1);
                if (jn < j1) slab_load(a.Qin, a.nv, jn * C, C, st);
                const uint16_t* sl = slabs + (size_t)cur * kHeavySlab;
                const int64_t q0 = bound(j), q1 = bound(j + 1);
                const uint64_t* __restrict__ Kin = a.Kin;
                constexpr int U = 8;
                for (int64_t base = q0 + (int64_t)64 * U * w; base < q1; base += (int64_t)64 * U * kWaves) {
                    uint32_t x[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int64_t pos = base + 64 * u + lane;
                        x[u] = pos < q1 ? __builtin_nontemporal_load(a.hpay + pos) : 0xffffffffu;
                    }
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const bool valid = x[u] != 0xffffffffu;
                        const uint32_t rl = (x[u] >> 16) & 0x7fffu, nl = x[u] & 0xffffu;
                        bool win = false;
                        if (valid) {
                            const uint16_t qu = rq[rl], qv = sl[nl];
                            win = (qu != qv) ? (qu < qv) : (Kin[row0 + rl] < Kin[j * C + nl]);
                        }
                        const uint64_t W = __ballot(win);
                        const int64_t wpos = base + 64 * u;
                        if (lane == 0 && wpos < q1) __builtin_nontemporal_store(W, a.bits + a.hword0 + wpos / 64);
                        // runs of one row within the word (run heads are marked
                        // in the payload): one LDS add per run
                        const uint64_t V = __ballot(valid);
                        const uint64_t Hm = __ballot(valid && (x[u] >> 31));
                        const uint64_t nv1 = (V >> lane) >> 1, nh1 = (Hm >> lane) >> 1;  // next lane's bits (0 past 63)
                        const bool last = valid && (!(nv1 & 1ull) || (nh1 & 1ull));
                        if (last) {
                            const uint64_t hm = Hm & le;
                            const uint64_t from = hm ? (~0ull << (63 - __clzll(hm))) : ~0ull;
                            const uint32_t c = (uint32_t)__popcll(W & le & from);
                            if (c) atomicAdd(&rc[rl], c);
                        }
                    }
                }
                if (jn < j1) slab_store(slabs + (size_t)(cur ^ 1) * kHeavySlab, C, st);
                __syncthreads();
                cur ^= 1;
                j = jn;
            }
            for (int i = threadIdx.x; i < nr; i += kPT) a.part_cnt[pt * R + i] = rc[i];
            __syncthreads();
        }
    }
}

// Persistent sweep: one workgroup per CU.  The workgroup first copies the
// codes of the kCacheQ highest-degree vertices (internal ids [0, kCacheQ))
// into LDS; those vertices take most of the gathers of a power-law graph.
// It then processes hub rows (whole workgroup each) and chunks (one wave
// each), both strided over the grid.
template <int H, bool IDENT, bool GAP>
__global__ __launch_bounds__(kPT) void k_fw_sweep(SweepArgs a) {
    extern __shared__ uint16_t qc[];
    __shared__ uint64_t red[kWaves][4];
    __shared__ uint64_t words[kWaves][32];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nc = a.ncache;
    // the 2D part first (its LDS layout), then the hot codes for the rest
    heavy_parts<H == 2 && IDENT>(a, reinterpret_cast<uint8_t*>(qc), reinterpret_cast<int64_t*>(&words[0][0]));
    for (int i = threadIdx.x; i < nc; i += kPT) qc[i] = a.Qin[i];
    // hub push: the hub rows' win counters of this workgroup, after the codes
    const int Hp = (H == 2 && IDENT) ? (int)a.n_push : 0;
    uint32_t* hcnt = reinterpret_cast<uint32_t*>(qc + ((nc + 1) & ~1));
    for (int i = threadIdx.x; i < (Hp + 1) / 2; i += kPT) hcnt[i] = 0u;
    __syncthreads();
    u128 sq = 0, mn = 0;
    // ---- hub rows: cut into word-aligned pieces of <= kPiece slots, one wave
    //      each.  A piece stores its decision words and adds (1 << 40) + its
    //      wins to the row's counter with one atomic, so the wave whose add
    //      completes the row's last piece reads the row's total from the value
    //      returned, with no fence; it writes the row's key and clears the
    //      counter for the next sweep.  With the hub push a piece covers only
    //      the row's hub prefix and adds its wins alone: k_push_finish adds
    //      the pushed wins and writes the key.
    for (int64_t pc = (int64_t)blockIdx.x * kWaves + w; pc < a.n_pieces; pc += (int64_t)gridDim.x * kWaves) {
        const int64_t r = a.hp_row[pc];
        const uint32_t u = IDENT ? (uint32_t)r : (uint32_t)a.rid[r];
        const int64_t rs = a.rp[r], re = a.rp[r + 1];
        const int64_t s0 = rs + a.hp_off[pc];
        const int64_t s1 = min(Hp > 0 ? rs + a.hub_pre[r] : re, s0 + (int64_t)kPiece);
        const uint64_t Ku = a.Kin[u];
        const uint16_t Qu = qcode(Ku >> a.B);
        uint64_t* bw = a.bits + a.chunk_words + a.hwo[r] + (s0 - rs) / 64;
        uint32_t cnt = 0;
        for (int64_t base = s0; base < s1; base += 64 * kG) {
            Slot<H> sl[kG];
            bool in[kG];
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                const int64_t s = base + 64 * j + lane;
                in[j] = s < s1;
                if (in[j]) sl[j] = load_slot<H>(a.py, s);
            }
            uint16_t qv[kG][H - 1];
#pragma unroll
            for (int j = 0; j < kG; ++j)
#pragma unroll
                for (int q = 0; q < H - 1; ++q)
                    qv[j][q] = in[j] ? qload(qc, nc, a.Qin, (uint32_t)sl[j].v[q]) : (uint16_t)0;
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                bool win = in[j];
#pragma unroll
                for (int q = 0; q < H - 1; ++q) win = win && beats(Ku, Qu, qv[j][q], a.Kin, sl[j].v[q]);
                const uint64_t W = __ballot(win);
                const int64_t wb = base + 64 * j;  // first slot of this word
                if (lane == 0 && wb < s1) __builtin_nontemporal_store(W, bw + (wb - s0) / 64);
                cnt += (uint32_t)__popcll(W);
            }
        }
        if (lane == 0 && Hp > 0) {
            atomicAdd(a.hub_ctr + r, (unsigned long long)cnt);
        } else if (lane == 0) {
            const unsigned long long npc = (unsigned long long)((re - rs + kPiece - 1) / kPiece);
            const unsigned long long old = atomicAdd(a.hub_ctr + r, (1ull << 40) | (unsigned long long)cnt);
            if ((old >> 40) == npc - 1) {
                const uint64_t tot = (old & ((1ull << 40) - 1)) + cnt;
                const uint64_t Kn = Ku + ((tot * a.inc) << a.B);
                a.Kout[u] = Kn;
                a.Qout[u] = qcode(Kn >> a.B);
                if (GAP) {
                    const uint64_t A = Ku >> a.B;
                    sq += (u128)A * A;
                    mn += (u128)A * tot;
                }
                atomicExch(a.hub_ctr + r, 0ull);
            }
        }
    }
    // ---- chunks: one wave each
    //   A. decision words: kG words per batch, slot payloads then codes in
    //      flight; each word's ballot is kept by lane t
    //   B. one lane per row: popcount of the row's slot range in the chunk's
    //      decision words (staged in LDS), key and code update
    for (int64_t c = (int64_t)blockIdx.x * kWaves + w; c < a.n_chunks; c += (int64_t)gridDim.x * kWaves) {
        const int64_t r0 = a.chunk_row[c], r1 = a.chunk_row[c + 1];
        if (r0 >= r1) continue;
        const int64_t s0 = a.rp[r0], s1 = a.rp[r1];
        const int64_t w0 = a.cwo[c];
        const int nw = (int)(a.cwo[c + 1] - w0);  // <= 32: a chunk spans < 2048 slots
        const int nsl = (int)(s1 - s0);
        const int32_t* __restrict__ pyc = a.py + s0 * (H - 1);
        const uint64_t hreg = (lane < nw) ? __builtin_nontemporal_load(a.head + w0 + lane) : 0ull;
        const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
        int32_t rowrel = -1;  // chunk-relative row of the slot before the current word
        uint64_t mybits = 0;
        for (int t0 = 0; t0 < nw; t0 += kG) {
            uint64_t Hw[kG];
#pragma unroll
            for (int j = 0; j < kG; ++j) Hw[j] = readlane64(hreg, t0 + j);  // t0 + j < 40
            Slot<H> sl[kG];
            uint32_t uu[kG];
            bool val[kG];
            int32_t rb = rowrel;
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                const int off = (t0 + j) * 64 + lane;
                val[j] = off < nsl;
                const int32_t row = rb + (int32_t)__popcll(Hw[j] & le);
                rb += (int32_t)__popcll(Hw[j]);
                uu[j] = 0;
                if (val[j]) {
                    sl[j] = load_slot<H>(pyc, off);
                    uu[j] = IDENT ? (uint32_t)(r0 + row) : (uint32_t)a.rid[r0 + row];
                }
            }
            rowrel = rb;
            uint16_t qu[kG], qv[kG][H - 1];
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                qu[j] = val[j] ? qload(qc, nc, a.Qin, uu[j]) : (uint16_t)0;
#pragma unroll
                for (int q = 0; q < H - 1; ++q)
                    qv[j][q] = val[j] ? qload(qc, nc, a.Qin, (uint32_t)sl[j].v[q]) : (uint16_t)0;
            }
#pragma unroll
            for (int j = 0; j < kG; ++j) {
                if (t0 + j < nw) {
                    bool win = val[j];
#pragma unroll
                    for (int q = 0; q < H - 1; ++q) {
                        if (qu[j] != qv[j][q]) {
                            win = win && (qu[j] < qv[j][q]);
                        } else if (win) {
                            win = a.Kin[uu[j]] < a.Kin[(uint32_t)sl[j].v[q]];
                        }
                    }
                    if (H == 2 && Hp > 0 && val[j] && !win) {  // a hub's win, pushed to its counter
                        const uint32_t v = (uint32_t)sl[j].v[0];
                        if (v < (uint32_t)Hp) atomicAdd(&hcnt[v >> 1], 1u << ((v & 1u) * 16));
                    }
                    const uint64_t W = __ballot(win);
                    if (lane == t0 + j) mybits = W;
                }
            }
        }
        if (lane < nw) {
            __builtin_nontemporal_store(mybits, a.bits + w0 + lane);
            words[w][lane] = mybits;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int64_t rbase = r0; rbase < r1; rbase += 64) {
            const int64_t r = rbase + lane;
            if (r < r1) {
                const int sa = (int)(a.rp[r] - s0), sb = (int)(a.rp[r + 1] - s0);  // sb > sa
                uint32_t cnt = 0;
                for (int wd = sa >> 6; wd <= ((sb - 1) >> 6); ++wd) {
                    const int lo = max(sa - wd * 64, 0), hi = min(sb - wd * 64, 64);
                    const uint64_t mk = ((hi >= 64) ? ~0ull : ((1ull << hi) - 1ull)) & (~0ull << lo);
                    cnt += (uint32_t)__popcll(words[w][wd] & mk);
                }
                const uint32_t u = IDENT ? (uint32_t)r : (uint32_t)a.rid[r];
                const uint64_t Ku = a.Kin[u];
                const uint64_t Kn = Ku + (((uint64_t)cnt * a.inc) << a.B);
                a.Kout[u] = Kn;
                a.Qout[u] = qcode(Kn >> a.B);
                if (GAP) {
                    const uint64_t A = Ku >> a.B;
                    sq += (u128)A * A;
                    mn += (u128)A * cnt;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();  // words[w] is rewritten by the next chunk
    }
    if (Hp > 0) {  // this workgroup's hub counters (uniform branch)
        __syncthreads();
        uint32_t* o = a.push_part + (int64_t)blockIdx.x * a.pstride;
        for (int i = threadIdx.x; i < (Hp + 1) / 2; i += kPT) o[i] = hcnt[i];
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
            for (int q = 0; q < kWaves; ++q) {
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

// After a sweep with the hub push: hub row r's wins are its prefix's wins
// (hub_ctr, cleared here for the next sweep) plus the counts every sweep
// workgroup pushed (the r & 1 half of word r >> 1 of its slice); then the
// row's new key and code, and its gap terms (per workgroup, written after
// the sweep's own partial sums of the iteration).  A workgroup takes 64 hub
// rows, one per lane; its four waves each sum every fourth sweep
// workgroup's counts (16 loads in flight per lane), and wave 0 finishes.
template <bool GAP>
__global__ __launch_bounds__(256) void k_push_finish(unsigned long long* hub_ctr, const uint32_t* push_part,
                                                     int64_t pstride, int nblocks, int64_t n_push,
                                                     const uint64_t* Kin, uint64_t* Kout, uint16_t* Qout,
                                                     uint64_t inc, int B, uint64_t* partial) {
    __shared__ uint64_t ps[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * 64 + lane;
    uint64_t part = 0;
    if (r < n_push) {
        const uint32_t* col = push_part + (r >> 1);
        const int sh = (int)(r & 1) * 16;
#pragma unroll 16
        for (int b = w; b < nblocks; b += 4) part += (col[(int64_t)b * pstride] >> sh) & 0xffffu;
    }
    ps[w][lane] = part;
    __syncthreads();
    if (w != 0) return;
    u128 sq = 0, mn = 0;
    if (r < n_push) {
        const uint64_t tot = hub_ctr[r] + ps[0][lane] + ps[1][lane] + ps[2][lane] + ps[3][lane];
        hub_ctr[r] = 0ull;
        const uint64_t Ku = Kin[r];
        const uint64_t Kn = Ku + ((tot * inc) << B);
        Kout[r] = Kn;
        Qout[r] = qcode(Kn >> B);
        if (GAP) {
            const uint64_t A = Ku >> B;
            sq = (u128)A * A;
            mn = (u128)A * tot;
        }
    }
    if (GAP) {  // wave 0 alone: all 64 lanes active
        sq = wave_sum128(sq);
        mn = wave_sum128(mn);
        if (lane == 0) {
            uint64_t* o = partial + (int64_t)blockIdx.x * 4;
            o[0] = (uint64_t)sq;
            o[1] = (uint64_t)(sq >> 64);
            o[2] = (uint64_t)mn;
            o[3] = (uint64_t)(mn >> 64);
        }
    }
}

// After a sweep with a 2D part: every heavy row's wins summed over the parts
// of its block, its new key and code, and the gap terms of those rows (per
// workgroup, written after the sweep's own partial sums of the iteration).
template <bool GAP>
__global__ __launch_bounds__(256) void k_heavy_finish(const uint32_t* part_cnt, const int32_t* blk_part,
                                                      const int32_t* row_blk, const int64_t* blk_row, int R,
                                                      int64_t n_heavy, const uint64_t* Kin, uint64_t* Kout,
                                                      uint16_t* Qout, uint64_t inc, int B, uint64_t* partial) {
    __shared__ uint64_t red[4][4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    u128 sq = 0, mn = 0;
    for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n_heavy; r += (int64_t)gridDim.x * 256) {
        const int64_t b = row_blk[r], rl = r - blk_row[b];
        const int p0 = blk_part[b], p1 = blk_part[b + 1];
        uint64_t tot = 0;
        int p = p0;
        for (; p + 8 <= p1; p += 8) {
            uint32_t c[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) c[k] = part_cnt[(int64_t)(p + k) * R + rl];
#pragma unroll
            for (int k = 0; k < 8; ++k) tot += c[k];
        }
        for (; p < p1; ++p) tot += part_cnt[(int64_t)p * R + rl];
        const uint64_t Ku = Kin[r];
        const uint64_t Kn = Ku + ((tot * inc) << B);
        Kout[r] = Kn;
        Qout[r] = qcode(Kn >> B);
        if (GAP) {
            const uint64_t A = Ku >> B;
            sq += (u128)A * A;
            mn += (u128)A * tot;
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
            uint64_t* o = partial + (int64_t)blockIdx.x * 4;
            o[0] = (uint64_t)S;
            o[1] = (uint64_t)(S >> 64);
            o[2] = (uint64_t)M;
            o[3] = (uint64_t)(M >> 64);
        }
    }
}

// initial keys: A0 = deg (edges, r0 = deg/2 with D0 = 2), 2 t_u (triangles,
// r0 = t_u/3 with D0 = 6) or q_u (4-cliques, r0 = q_u/4 with D0 = 4), packed
// with the original-id code
__global__ void k_init_keys(const int32_t* count, int mult, const int32_t* orig_of, int64_t n, int B,
                            uint64_t* K0, uint64_t* K1, uint16_t* Q0, uint16_t* Q1) {
    const int64_t u = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (u >= n) return;
    const uint64_t idm = (1ull << B) - 1ull;
    const uint64_t A = (uint64_t)count[u] * (uint64_t)mult;
    const uint64_t k = (A << B) | (idm - (uint64_t)orig_of[u]);
    K0[u] = k;
    K1[u] = k;
    Q0[u] = Q1[u] = qcode(A);
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
// words: a = a0 + sum_i inc_i [slot won in iteration i], inc_i = incm (i+1)
template <int H>
__global__ void k_splits(const int64_t* rp, const int32_t* rid, const int32_t* py, const int64_t* bitbase,
                         int64_t nrows, int64_t nslots, const uint64_t* bits, int64_t total_words, int iters,
                         uint64_t a0, uint64_t incm, const int32_t* orig_of, int32_t* verts, uint64_t* num) {
    const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (s >= nslots) return;
    // row of slot s: last r with rp[r] <= s
    int64_t lo = 0, hi = nrows - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (rp[mid] <= s) lo = mid; else hi = mid - 1;
    }
    const int64_t r = lo;
    if (bitbase[r] < 0) return;  // a heavy row: k_splits_heavy
    const int64_t pos = bitbase[r] + (s - rp[r]);
    uint64_t a = a0;
    for (int i = 1; i <= iters; ++i) {
        const uint64_t wd = bits[(int64_t)(i - 1) * total_words + pos / 64];
        if ((wd >> (pos % 64)) & 1ull) a += incm * (uint64_t)(i + 1);
    }
    const int32_t x = rid ? rid[r] : (int32_t)r;
    verts[H * s] = orig_of[x];
    for (int j = 0; j < H - 1; ++j) verts[H * s + 1 + j] = orig_of[py[(H - 1) * s + j]];
    num[s] = a;
}

// the same for the slots of heavy rows (edges), position by position of the
// 2D part: the slot is csr[pos], its decision bits follow from word0
__global__ void k_splits_heavy(const uint32_t* csr, const uint32_t* pay, int64_t positions, int64_t word0,
                               const int64_t* rp, int64_t nrows, const int32_t* py, const uint64_t* bits,
                               int64_t total_words, int iters, uint64_t a0, uint64_t incm, const int32_t* orig_of,
                               int32_t* verts, uint64_t* num) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= positions || pay[k] == 0xffffffffu) return;
    const int64_t s = csr[k];
    int64_t lo = 0, hi = nrows - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (rp[mid] <= s) lo = mid; else hi = mid - 1;
    }
    uint64_t a = a0;
    const int64_t pos = word0 * 64 + k;
    for (int i = 1; i <= iters; ++i) {
        const uint64_t wd = bits[(int64_t)(i - 1) * total_words + pos / 64];
        if ((wd >> (pos % 64)) & 1ull) a += incm * (uint64_t)(i + 1);
    }
    verts[2 * s] = orig_of[lo];
    verts[2 * s + 1] = orig_of[py[s]];
    num[s] = a;
}

uint64_t denom(int mode, int64_t i) { return fw_denom(mode, i); }

template <int H, bool IDENT>
void launch_sweep(const SweepArgs& a, unsigned blocks, bool gap, hipStream_t s) {
    const bool heavy = H == 2 && IDENT && a.n_parts > 0;
    const size_t push_lds = a.n_push > 0 ? (size_t)((a.ncache + 1) & ~1) * 2 + (size_t)a.pstride * 4 : 0;
    const size_t lds = std::max(std::max((size_t)a.ncache * sizeof(uint16_t), push_lds), heavy ? kHeavyLds : (size_t)0);
    const int max_lds = (int)std::max((size_t)kCacheQ * 2 + 16, (H == 2 && IDENT) ? kHeavyLds : (size_t)0);
    if (gap) {
        static bool attr = false;
        if (!attr) {
            LDS_HIP(hipFuncSetAttribute((const void*)k_fw_sweep<H, IDENT, true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, max_lds));
            attr = true;
        }
        k_fw_sweep<H, IDENT, true><<<blocks, kPT, lds, s>>>(a);
    } else {
        static bool attr = false;
        if (!attr) {
            LDS_HIP(hipFuncSetAttribute((const void*)k_fw_sweep<H, IDENT, false>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, max_lds));
            attr = true;
        }
        k_fw_sweep<H, IDENT, false><<<blocks, kPT, lds, s>>>(a);
    }
}

// one persistent workgroup per compute unit
unsigned sweep_grid() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        LDS_HIP(hipGetDevice(&dev));
        LDS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        if (cus <= 0) cus = 1;
    }
    return (unsigned)(cus * kWgPerCU);
}

// workgroups of the heavy rows' finishing kernel (0 without a 2D part); its
// gap partial sums follow the sweep's in each iteration's slice
unsigned finish_grid(const SweepPlan& p) { return p.heavy.n_parts > 0 ? sweep_grid() : 0u; }

// workgroups of the hub push's finishing kernel (64 hub rows each); its gap
// partial sums follow the sweep's likewise (a plan has a 2D part or the push,
// never both)
unsigned push_grid(const SweepPlan& p) { return (unsigned)((p.n_push + 63) / 64); }

// switch the sweep arguments to the hub push of plan p (sweep workgroups
// `blocks`; push_part sized here)
void use_push(const SweepPlan& p, FwState& f, unsigned blocks, SweepArgs& a, hipStream_t s) {
    a.n_push = p.n_push;
    a.hub_pre = p.hub_pre.p;
    a.n_pieces = p.n_ppieces;
    a.hp_row = p.pp_row.p;
    a.hp_off = p.pp_off.p;
    a.ncache = (int)p.push_nc;
    a.pstride = (p.n_push + 1) / 2;
    const size_t words = (size_t)blocks * (size_t)a.pstride;
    if (f.push_part.n < words) f.push_part.alloc(words, s);
    a.push_part = f.push_part.p;
}

void fill_sweep_args(const Graph& g, const SweepPlan& p, SweepArgs& a) {
    a = SweepArgs{};
    a.rid = p.rid;
    a.rp = p.rp;
    a.py = p.py;
    a.n_hub = p.n_hub;
    a.hwo = p.hwo.p;
    a.n_pieces = p.n_pieces;
    a.hp_row = p.hp_row.p;
    a.hp_off = p.hp_off.p;
    a.hub_ctr = p.hub_ctr.p;
    a.n_chunks = p.n_chunks;
    a.chunk_row = p.chunk_row.p;
    a.cwo = p.cwo.p;
    a.head = p.head.p;
    a.chunk_words = p.chunk_words;
    a.B = g.idbits;
    a.ncache = (int)std::min<int64_t>(g.n, kCacheQ);
    const HeavyPlan& h = p.heavy;
    a.n_parts = h.n_parts;
    a.part_blk = h.part_blk.p;
    a.part_j0 = h.part_j0.p;
    a.part_j1 = h.part_j1.p;
    a.part_lo = h.part_lo.p;
    a.part_hi = h.part_hi.p;
    a.hseg = h.seg.p;
    a.hblk_row = h.blk_row.p;
    a.hpay = h.pay.p;
    a.part_cnt = h.part_cnt.p;
    a.hP = h.P;
    a.hR = h.R;
    a.hC = h.C;
    a.n_heavy = h.n_heavy;
    a.hword0 = h.word0;
    a.nv = g.n;
}

// iteration i: the sweep, then the heavy rows' keys; partial = this
// iteration's gap slice (sweep workgroups, then finishing workgroups) or null
void sweep_iteration(FwState& f, const SweepPlan& p, SweepArgs& a, int mode, int i, unsigned blocks,
                     uint64_t* partial, hipStream_t s) {
    const bool gap = partial != nullptr;
    a.Kin = f.K[f.cur].p;
    a.Kout = f.K[f.cur ^ 1].p;
    a.Qin = f.Q[f.cur].p;
    a.Qout = f.Q[f.cur ^ 1].p;
    a.bits = f.bits.p + (size_t)(i - 1) * p.total_words;
    a.inc = denom(mode, i) - denom(mode, i - 1);
    a.partial = partial;
    if (mode == 2)
        launch_sweep<2, true>(a, blocks, gap, s);
    else if (mode == 3)
        launch_sweep<3, false>(a, blocks, gap, s);
    else
        launch_sweep<4, false>(a, blocks, gap, s);
    LDS_HIP(hipGetLastError());
    if (a.n_push > 0) {
        const unsigned pg = push_grid(p);
        if (gap)
            k_push_finish<true><<<pg, 256, 0, s>>>(a.hub_ctr, a.push_part, a.pstride, (int)blocks, a.n_push, a.Kin,
                                                   a.Kout, a.Qout, a.inc, a.B, partial + (size_t)blocks * 4);
        else
            k_push_finish<false><<<pg, 256, 0, s>>>(a.hub_ctr, a.push_part, a.pstride, (int)blocks, a.n_push,
                                                    a.Kin, a.Kout, a.Qout, a.inc, a.B, nullptr);
        LDS_HIP(hipGetLastError());
    }
    const unsigned fb = finish_grid(p);
    if (fb > 0) {
        const HeavyPlan& h = p.heavy;
        uint64_t* fp = gap ? partial + (size_t)blocks * 4 : nullptr;
        if (gap)
            k_heavy_finish<true><<<fb, 256, 0, s>>>(h.part_cnt.p, h.blk_part.p, h.row_blk.p, h.blk_row.p, h.R,
                                                    h.n_heavy, a.Kin, a.Kout, a.Qout, a.inc, a.B, fp);
        else
            k_heavy_finish<false><<<fb, 256, 0, s>>>(h.part_cnt.p, h.blk_part.p, h.row_blk.p, h.blk_row.p, h.R,
                                                     h.n_heavy, a.Kin, a.Kout, a.Qout, a.inc, a.B, fp);
        LDS_HIP(hipGetLastError());
    }
    f.cur ^= 1;
}

}  // namespace

unsigned __int128 fw_max_numerator(const Graph& g, int mode, int iters) {
    // a vertex that wins every incident pattern in every iteration:
    // deg (1 + sum_i 2(i+1)), t (2 + sum_i 6(i+1)) or q (1 + sum_i 4(i+1))
    const unsigned __int128 N = (unsigned)iters;
    if (mode == 2) return (unsigned __int128)(uint64_t)g.max_deg * (N * N + 3 * N + 1);
    if (mode == 3) return (unsigned __int128)(uint64_t)g.t_max * (2 + 3 * N * (N + 3));
    return (unsigned __int128)(uint64_t)g.q_max * (1 + 2 * N * (N + 3));
}

void fw_prepare(Graph& g, int mode, int iters, hipStream_t s) {
    LDS_CHECK(mode >= 2 && mode <= 4, ST_INVALID, "mode must be LDS_EDGE, LDS_TRIANGLE or LDS_CLIQUE4");
    LDS_CHECK(iters >= 0, ST_INVALID, "iters must be >= 0");
    if (mode == 3 && g.T < 0) list_triangles(g, s);
    if (mode == 4 && g.Q4 < 0) list_cliques4(g, s);
    const SweepPlan& p = plan_of(g, mode);
    FwState& f = g.fw[mode_slot(mode)];
    const int B = g.idbits;
    // overflow: the largest numerator must leave B bits for the id code
    const u128 amax = fw_max_numerator(g, mode, iters);
    LDS_CHECK(B < 64 && (amax >> (64 - B)) == 0, ST_OVERFLOW, "exact load numerator would overflow the 64-bit key");
    const int64_t n = g.n;
    if (f.K[0].n != (size_t)n) {
        f.K[0].alloc(n, s);
        f.K[1].alloc(n, s);
        f.Q[0].alloc(n, s);
        f.Q[1].alloc(n, s);
    }
    const size_t nbits = (size_t)iters * (size_t)p.total_words;
    if (f.bits.n < nbits) f.bits.alloc(nbits, s);
}

void fw_gap_from_sums(FwState& f, int mode, int iters, const uint64_t* sums) {
    f.gap.assign(iters, 0.0);
    f.lb.assign(iters, 0.0);
    f.fval.assign(iters, 0.0);
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
        f.fval[i - 1] = (double)((long double)S / (LD * LD));
    }
}

void fw_run(Graph& g, int mode, int iters, bool want_gap, hipStream_t s) {
    fw_prepare(g, mode, iters, s);
    SweepPlan& p = plan_of(g, mode);
    FwState& f = g.fw[mode_slot(mode)];
    const int B = g.idbits;
    const int64_t n = g.n;
    if (n > 0) {
        const int32_t* cnt = (mode == 2) ? g.deg.p : (mode == 3 ? g.tcount.p : g.qcount.p);
        k_init_keys<<<grid_for(n, 256), 256, 0, s>>>(cnt, mode == 3 ? 2 : 1, g.orig_of.p, n, B, f.K[0].p, f.K[1].p,
                                                    f.Q[0].p, f.Q[1].p);
        LDS_HIP(hipGetLastError());
    }
    f.cur = 0;
    g.sg[mode_slot(mode)].valid = false;
    const unsigned blocks = sweep_grid();
    const unsigned gblocks = blocks + finish_grid(p) + push_grid(p);  // gap partial sums per iteration
    const size_t npart = want_gap ? (size_t)iters * gblocks * 4 : 0;
    if (f.partial.n < npart) f.partial.alloc(npart, s);
    SweepArgs a;
    fill_sweep_args(g, p, a);
    if (p.n_push > 0) use_push(p, f, blocks, a, s);
    if (!f.ev[0]) {
        LDS_HIP(hipEventCreate(&f.ev[0]));
        LDS_HIP(hipEventCreate(&f.ev[1]));
    }
    LDS_HIP(hipEventRecord(f.ev[0], s));
    f.launches = 0;
    for (int i = 1; i <= iters && blocks > 0 && p.nrows > 0; ++i) {
        sweep_iteration(f, p, a, mode, i, blocks, want_gap ? f.partial.p + (size_t)(i - 1) * gblocks * 4 : nullptr,
                        s);
        ++f.launches;
    }
    LDS_HIP(hipEventRecord(f.ev[1], s));
    f.iters = iters;
    f.ran = true;
    f.timed = true;
    f.gap.clear();
    f.lb.clear();
    f.fval.clear();
    if (want_gap && iters > 0) {
        std::vector<uint64_t> sums((size_t)iters * 4, 0);
        if (blocks > 0 && p.nrows > 0) {
            DBuf<uint64_t> out;
            out.alloc((size_t)iters * 4, s);
            k_gap_reduce<<<iters, 256, 0, s>>>(f.partial.p, gblocks, out.p);
            LDS_HIP(hipGetLastError());
            LDS_HIP(hipMemcpyAsync(sums.data(), out.p, out.bytes(), hipMemcpyDeviceToHost, s));
            LDS_HIP(hipStreamSynchronize(s));
        }
        fw_gap_from_sums(f, mode, iters, sums.data());
    }
}

namespace {

// gap of iteration j + 1 at r^(j) from the exact sums (sum A^2, sum of the
// patterns' minimum A), over D_j = c (j+1)(j+2):
// gap = 2 (sum A^2 - D_j sum min A) / D_j^2, rounded to FP64 on the device
__global__ void k_gap_values(const uint64_t* sums, int iters, uint64_t c, double* gap) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= iters) return;
    const u128 S = ((u128)sums[4 * j + 1] << 64) | sums[4 * j];
    const u128 M = ((u128)sums[4 * j + 3] << 64) | sums[4 * j + 2];
    const uint64_t D = c * (uint64_t)(j + 1) * (uint64_t)(j + 2);
    const u128 num = S - (u128)D * M;
    const double nd = (double)(uint64_t)(num >> 64) * 18446744073709551616.0 + (double)(uint64_t)num;
    const double Dd = (double)D;
    gap[j] = 2.0 * nd / (Dd * Dd);
}

// this device's copy of the scratch array, looked up once per device with
// that device current
uint64_t* scratch_on_current_device() {
    constexpr int kMaxDev = 64;
    static std::mutex mu;
    static uint64_t* ptr[kMaxDev] = {};
    int dev = 0;
    LDS_HIP(hipGetDevice(&dev));
    LDS_CHECK(dev >= 0 && dev < kMaxDev, ST_DEVICE, "device index out of range for the scratch table");
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        LDS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        LDS_CHECK(p != nullptr, ST_DEVICE, "hipGetSymbolAddress returned no address for the scratch array");
        ptr[dev] = (uint64_t*)p;
    }
    return ptr[dev];
}

}  // namespace


void fw_run_noalloc(Graph& g, int mode, int iters, float* r32_dev, double* gap_host, hipStream_t s) {
    LDS_CHECK(mode >= 2 && mode <= 4, ST_INVALID, "mode must be LDS_EDGE, LDS_TRIANGLE or LDS_CLIQUE4");
    LDS_CHECK(iters >= 0, ST_INVALID, "iters must be >= 0");
    LDS_CHECK(mode != 3 || g.T >= 0, ST_INVALID, "triangles are not listed: run lds_frank_wolfe (or lds_triangles) first");
    LDS_CHECK(mode != 4 || g.Q4 >= 0, ST_INVALID, "4-cliques are not listed: run lds_frank_wolfe (or lds_cliques4) first");
    const SweepPlan& p = plan_of(g, mode);
    FwState& f = g.fw[mode_slot(mode)];
    const int B = g.idbits;
    const u128 amax = fw_max_numerator(g, mode, iters);
    LDS_CHECK(B < 64 && (amax >> (64 - B)) == 0, ST_OVERFLOW, "exact load numerator would overflow the 64-bit key");
    const int64_t n = g.n;
    LDS_CHECK(f.K[0].n == (size_t)n && f.K[1].n == (size_t)n && f.Q[0].n == (size_t)n && f.Q[1].n == (size_t)n &&
                  f.bits.n >= (size_t)iters * (size_t)p.total_words,
              ST_INVALID,
              "Frank-Wolfe state is not sized for this many iterations: run lds_frank_wolfe with at least iters "
              "iterations on this graph and mode first");
    const unsigned blocks = sweep_grid();
    const unsigned gblocks = blocks + finish_grid(p);
    const bool gap = gap_host != nullptr && iters > 0;
    const size_t words = gap ? (size_t)iters * ((size_t)gblocks * 4 + 5) : 0;
    LDS_CHECK(words <= kScratchWords, ST_INVALID,
              "iters exceeds the no-allocation limit with the gap (" +
                  std::to_string(kScratchWords / ((size_t)gblocks * 4 + 5)) + " iterations for this graph)");
    uint64_t* sc = scratch_on_current_device();
    uint64_t* partial = sc;
    uint64_t* sums = sc + (size_t)iters * gblocks * 4;
    double* gapv = reinterpret_cast<double*>(sums + (size_t)iters * 4);
    if (n > 0) {
        const int32_t* cnt = (mode == 2) ? g.deg.p : (mode == 3 ? g.tcount.p : g.qcount.p);
        k_init_keys<<<grid_for(n, 256), 256, 0, s>>>(cnt, mode == 3 ? 2 : 1, g.orig_of.p, n, B, f.K[0].p, f.K[1].p,
                                                    f.Q[0].p, f.Q[1].p);
        LDS_HIP(hipGetLastError());
    }
    f.cur = 0;
    g.sg[mode_slot(mode)].valid = false;
    SweepArgs a;
    fill_sweep_args(g, p, a);
    const bool any = blocks > 0 && p.nrows > 0;
    for (int i = 1; i <= iters && any; ++i)
        sweep_iteration(f, p, a, mode, i, blocks, gap ? partial + (size_t)(i - 1) * gblocks * 4 : nullptr, s);
    f.iters = iters;
    f.ran = true;
    f.timed = false;
    f.launches = any ? iters : 0;
    f.gap.clear();
    f.lb.clear();
    f.fval.clear();
    if (n > 0 && r32_dev) {
        k_loads<<<grid_for(n, 256), 256, 0, s>>>(f.K[f.cur].p, g.orig_of.p, n, B, (double)denom(mode, iters), r32_dev,
                                                 nullptr);
        LDS_HIP(hipGetLastError());
    }
    if (gap) {
        if (any) {
            k_gap_reduce<<<iters, 256, 0, s>>>(partial, gblocks, sums);
            LDS_HIP(hipGetLastError());
            k_gap_values<<<grid_for(iters, 256), 256, 0, s>>>(sums, iters, denom(mode, 0) / 2, gapv);
            LDS_HIP(hipGetLastError());
            LDS_HIP(hipMemcpyAsync(gap_host, gapv, (size_t)iters * sizeof(double), hipMemcpyDeviceToHost, s));
            LDS_HIP(hipStreamSynchronize(s));
        } else {
            for (int i = 0; i < iters; ++i) gap_host[i] = 0.0;
        }
    }
}

void fw_loads(const Graph& g, int mode, float* r32_dev, double* r64_host, uint64_t* A_host, hipStream_t s) {
    const FwState& f = g.fw[mode_slot(mode)];
    const int64_t n = g.n;
    if (n == 0) return;
    LDS_CHECK(f.ran && f.K[0].n == (size_t)n, ST_INVALID, "no Frank-Wolfe state: call lds_frank_wolfe first");
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
    const FwState& f = g.fw[mode_slot(mode)];
    const SweepPlan& p = plan_of(g, mode);
    const int64_t ns = p.nslots;
    if (ns == 0) return;
    LDS_CHECK(f.ran && f.K[0].n == (size_t)g.n, ST_INVALID, "no Frank-Wolfe state: call lds_frank_wolfe first");
    const int H = mode;
    DBuf<int32_t> v;
    DBuf<uint64_t> a;
    v.alloc((size_t)ns * H, s);
    a.alloc(ns, s);
    // a0 = D_0 / h; inc_i = D_i - D_{i-1} = incm (i+1) with incm = inc_1 / 2
    const uint64_t a0 = denom(mode, 0) / (uint64_t)H, incm = (denom(mode, 1) - denom(mode, 0)) / 2;
    if (mode == 2) {
        k_splits<2><<<grid_for(ns, 256), 256, 0, s>>>(p.rp, p.rid, p.py, p.bitbase.p, p.nrows, ns, f.bits.p,
                                                      p.total_words, f.iters, a0, incm, g.orig_of.p, v.p, a.p);
        const HeavyPlan& h = p.heavy;
        if (h.positions > 0)
            k_splits_heavy<<<grid_for(h.positions, 256), 256, 0, s>>>(h.csr.p, h.pay.p, h.positions, h.word0, p.rp,
                                                                      p.nrows, p.py, f.bits.p, p.total_words,
                                                                      f.iters, a0, incm, g.orig_of.p, v.p, a.p);
        if (p.n_push > 0)  // the hub rows' slots against non-hub vertices, from their mirror slots
            k_push_mirror<uint64_t><<<(unsigned)std::min<int64_t>(p.n_push, 4096), 256, 0, s>>>(
                p.rp, p.py, p.hub_pre.p, p.n_push, denom(mode, f.iters), a.p);
    }
    else if (mode == 3)
        k_splits<3><<<grid_for(ns, 256), 256, 0, s>>>(p.rp, p.rid, p.py, p.bitbase.p, p.nrows, ns, f.bits.p,
                                                      p.total_words, f.iters, a0, incm, g.orig_of.p, v.p, a.p);
    else
        k_splits<4><<<grid_for(ns, 256), 256, 0, s>>>(p.rp, p.rid, p.py, p.bitbase.p, p.nrows, ns, f.bits.p,
                                                      p.total_words, f.iters, a0, incm, g.orig_of.p, v.p, a.p);
    LDS_HIP(hipGetLastError());
    LDS_HIP(hipMemcpyAsync(verts_host, v.p, v.bytes(), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipMemcpyAsync(num_host, a.p, a.bytes(), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
}

}  // namespace lds
