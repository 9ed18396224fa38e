// Graph ingest on the device: canonical simple graph (Section 3 assumes an
// undirected simple graph), degree renumbering, symmetric CSR and the sweep
// plan (hub rows, row-aligned chunks, word offsets and row-start flags) that
// the Frank-Wolfe kernels stream over.

#include "graph.hpp"

#include <algorithm>
#include <cstdlib>
#include <type_traits>
#include <vector>

namespace lds {

namespace {

constexpr int kT = 256;

// every pair becomes two keys (a,b) and (b,a): sorting them gives the
// symmetric CSR in original ids, with duplicates adjacent
__global__ void k_canon(const int32_t* src, const int32_t* dst, int64_t np, int64_t n, int vbits, int strict,
                        uint64_t* keys, unsigned* err) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= np) return;
    const int64_t a = src[i], b = dst[i];
    const uint64_t sentinel = ((uint64_t)n << vbits) | (uint64_t)n;
    uint64_t k0 = sentinel, k1 = sentinel;
    if (a < 0 || b < 0 || a >= n || b >= n) {
        atomicOr(err, 1u);
    } else if (a == b) {
        if (strict) atomicOr(err, 2u);
    } else {
        k0 = ((uint64_t)a << vbits) | (uint64_t)b;
        k1 = ((uint64_t)b << vbits) | (uint64_t)a;
    }
    keys[2 * i] = k0;
    keys[2 * i + 1] = k1;
}

__global__ void k_unique_flags(const uint64_t* keys, int64_t np, uint64_t sentinel, int strict, uint32_t* flag,
                               unsigned* err) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= np) return;
    const uint64_t k = keys[i];
    uint32_t f = (k != sentinel) && (i == 0 || keys[i - 1] != k);
    if (strict && k != sentinel && i > 0 && keys[i - 1] == k) atomicOr(err, 4u);
    flag[i] = f;
}

__global__ void k_compact(const uint64_t* keys, const uint32_t* flag, const uint64_t* pos, int64_t np,
                          uint64_t* out) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= np || !flag[i]) return;
    out[pos[i]] = keys[i];
}

// run boundaries of the sorted symmetric keys: first slot and one-past-last
// slot of every row that has slots
__global__ void k_row_bounds(const uint64_t* sk, int64_t ns, int vbits, int64_t* rstart, int64_t* rend) {
    const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= ns) return;
    const uint64_t row = sk[j] >> vbits;
    if (j == 0 || (sk[j - 1] >> vbits) != row) rstart[row] = j;
    if (j == ns - 1 || (sk[j + 1] >> vbits) != row) rend[row] = j + 1;
}

__global__ void k_row_deg(const int64_t* rstart, const int64_t* rend, int64_t n, int32_t* deg) {
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    deg[v] = (int32_t)(rend[v] - rstart[v]);
}

__global__ void k_maxdeg(const int32_t* deg, int64_t n, int* out, unsigned long long* nz) {
    // grid-stride (the launch is capped at kReduceWG workgroups): one atomic
    // per wave on each of the two counters; with a wave per 64 entries the
    // waves of a 4M-entry array queued ~125k atomics on two addresses (0.75 ms)
    int d = 0;
    unsigned c = 0;  // entries > 0 (fewer than 2^32)
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        const int x = deg[i];
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

// renumber key: degree descending, original id ascending
__global__ void k_relabel_keys(const int32_t* deg, int64_t n, int vbits, int32_t dmax, uint64_t* keys) {
    const int64_t v = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (v >= n) return;
    keys[v] = ((uint64_t)(dmax - deg[v]) << vbits) | (uint64_t)v;
}

__global__ void k_relabel_apply(const uint64_t* keys, int64_t n, int vbits, const int32_t* deg_orig,
                                int32_t* orig_of, int32_t* int_of, int32_t* deg_int) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i >= n) return;
    const int32_t o = (int32_t)(keys[i] & ((1ull << vbits) - 1));
    orig_of[i] = o;
    int_of[o] = (int32_t)i;
    deg_int[i] = deg_orig[o];
}

// slot j of original row o moves to internal row int_of[o], same offset
// within the row; its column is renumbered
__global__ void k_permute(const uint64_t* sk, int64_t ns, int vbits, const int64_t* rstart, const int32_t* int_of,
                          const int64_t* rowptr, int32_t* col) {
    const int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (j >= ns) return;
    const uint64_t k = sk[j], mask = (1ull << vbits) - 1;
    const int64_t o = (int64_t)(k >> vbits);
    const int32_t i = int_of[o];
    col[rowptr[i] + (j - rstart[o])] = int_of[k & mask];
}

// (row, col) keys of the internal CSR, for sorting every row ascending
__global__ void k_set_last(int64_t* rowptr, int64_t idx, const uint64_t* total) { rowptr[idx] = (int64_t)*total; }

// ------------------------------------------------------------- sweep plan
__global__ void k_hub_words(const int64_t* rp, int64_t n_hub, uint64_t* words) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= n_hub) return;
    words[r] = (uint64_t)((rp[r + 1] - rp[r] + 63) / 64);
}

// pieces of the hub rows: of each whole row, or (pre given) of its first
// pre[r] slots
__global__ void k_hub_pieces(const int64_t* rp, int64_t n_hub, const int32_t* pre, uint32_t* np) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r < n_hub) np[r] = (uint32_t)(((pre ? (int64_t)pre[r] : rp[r + 1] - rp[r]) + kPiece - 1) / kPiece);
}

__global__ void k_hub_piece_fill(const int64_t* rp, int64_t n_hub, const int32_t* pre, const uint64_t* first,
                                 int32_t* hp_row, int32_t* hp_off) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= n_hub) return;
    const int64_t len = pre ? (int64_t)pre[r] : rp[r + 1] - rp[r];
    int64_t k = (int64_t)first[r];
    for (int64_t o = 0; o < len; o += kPiece, ++k) {
        hp_row[k] = (int32_t)r;
        hp_off[k] = (int32_t)o;
    }
}

// hub push: the slots of hub row r whose neighbour is a hub row (a prefix:
// the row is sorted by neighbour id)
__global__ void k_hub_prefix(const int64_t* rp, const int32_t* col, int64_t n_hub, int32_t* pre) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= n_hub) return;
    int64_t lo = rp[r], hi = rp[r + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < (int32_t)n_hub)
            lo = mid + 1;
        else
            hi = mid;
    }
    pre[r] = (int32_t)(lo - rp[r]);
}

__global__ void k_chunk_rows(const int64_t* rp, int64_t nrows, int64_t n_hub, int64_t n_chunks, int64_t* chunk_row) {
    const int64_t r = n_hub + (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r > nrows) return;
    const int64_t base = rp[n_hub];
    const int64_t cr = (r < nrows) ? (rp[r] - base) / kChunk : n_chunks;  // r == nrows: close every chunk
    const int64_t cp = (r == n_hub) ? -1 : (rp[r - 1] - base) / kChunk;
    for (int64_t c = cp + 1; c <= cr; ++c) chunk_row[c] = r;
}

__global__ void k_chunk_words(const int64_t* rp, const int64_t* chunk_row, int64_t n_chunks, uint64_t* words) {
    const int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (c >= n_chunks) return;
    words[c] = (uint64_t)((rp[chunk_row[c + 1]] - rp[chunk_row[c]] + 63) / 64);
}

__global__ void k_head(const int64_t* rp, int64_t nrows, int64_t n_hub, const int64_t* chunk_row,
                       const int64_t* cwo, unsigned long long* head) {
    const int64_t r = n_hub + (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= nrows) return;
    const int64_t base = rp[n_hub];
    const int64_t c = (rp[r] - base) / kChunk;
    const int64_t pos = rp[r] - rp[chunk_row[c]];
    atomicOr(&head[cwo[c] + pos / 64], 1ull << (pos % 64));
}

__global__ void k_bitbase(const int64_t* rp, int64_t nrows, int64_t n_hub, const int64_t* chunk_row,
                          const int64_t* cwo, const int64_t* hwo, int64_t chunk_words, bool heavy, int64_t* bitbase) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= nrows) return;
    if (r < n_hub) {
        bitbase[r] = heavy ? -1 : (chunk_words + hwo[r]) * 64;
    } else {
        const int64_t base = rp[n_hub];
        const int64_t c = (rp[r] - base) / kChunk;
        bitbase[r] = cwo[c] * 64 + (rp[r] - rp[chunk_row[c]]);
    }
}

// ------------------------------------------------------------- row sort
// Every CSR row sorted ascending, by row length (rows are ordered by length,
// descending, so each class is a range of rows): rows of at most S <= 64
// slots by a bitonic network over S lanes of a wave (64 / S rows per wave);
// rows of up to 4096 slots by one workgroup with a bitonic network in LDS;
// longer rows by the library's radix sort of (row, column) keys.
template <int S>
__global__ void k_sort_rows_lanes(const int64_t* rp, int64_t r0, int64_t r1, int32_t* col) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 6;
    const int64_t r = r0 + wave * (64 / S) + lane / S;
    const int e = lane % S;
    int64_t s0 = 0, len = 0;
    if (r < r1) {
        s0 = rp[r];
        len = rp[r + 1] - s0;
    }
    int32_t x = (e < len) ? col[s0 + e] : INT32_MAX;
#pragma unroll
    for (int k = 2; k <= S; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const int32_t y = __shfl_xor(x, j, 64);
            x = (((e & j) == 0) == ((e & k) == 0)) ? min(x, y) : max(x, y);
        }
    }
    if (e < len) col[s0 + e] = x;
}

// rows of at most MAXP slots, one workgroup of NT threads each; the row
// classes (65-128, 129-512, 513-4096 slots) get workgroups and LDS sized to
// them, so that a short row neither idles a 256-thread workgroup nor holds
// 16 KB of LDS
template <int NT, int MAXP>
__global__ __launch_bounds__(NT) void k_sort_rows_block(const int64_t* rp, int64_t r0, int32_t* col) {
    __shared__ int32_t v[MAXP];
    const int64_t r = r0 + blockIdx.x;
    const int64_t s0 = rp[r];
    const int len = (int)(rp[r + 1] - s0);
    int P = 1;
    while (P < len) P <<= 1;
    for (int i = threadIdx.x; i < P; i += NT) v[i] = (i < len) ? col[s0 + i] : INT32_MAX;
    __syncthreads();
    for (int k = 2; k <= P; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < P; i += NT) {
                const int q = i ^ j;
                if (q > i) {
                    const int32_t a = v[i], b = v[q];
                    if ((a > b) == ((i & k) == 0)) {
                        v[i] = b;
                        v[q] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < len; i += NT) col[s0 + i] = v[i];
}

// keys (row << 32 | column) of the slots of rows [0, r1) and back
__global__ void k_row_keys(const int64_t* rp, int64_t r1, const int32_t* col, uint64_t* keys) {
    for (int64_t r = blockIdx.x; r < r1; r += gridDim.x)
        for (int64_t q = rp[r] + threadIdx.x; q < rp[r + 1]; q += kT)
            keys[q - rp[0]] = ((uint64_t)r << 32) | (uint32_t)col[q];
}

__global__ void k_row_unkeys(const uint64_t* keys, int64_t n, int32_t* col) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) col[i] = (int32_t)(uint32_t)keys[i];
}

// ------------------------------------------------------ heavy 2D part
// rows with at least deg_min slots: a prefix (rows are ordered by slot count)
__global__ void k_count_deg(const int64_t* rp, int64_t nrows, int64_t deg_min, unsigned long long* cnt) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    const bool h = r < nrows && (rp[r + 1] - rp[r]) >= deg_min;
    unsigned long long c = __popcll(__ballot(h));
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

// rows longer than each of a few thresholds: rows are ordered by slot count,
// descending, so each count is the end of a prefix, found by binary search
// (one thread per threshold; a count over every row with one atomic per
// wave spent ~0.3 ms per threshold on the one contended counter)
constexpr int kLongerThresholds = 9;
struct LongerThan {
    int64_t t[kLongerThresholds];
};
__global__ void k_rows_longer(const int64_t* rp, int64_t nrows, LongerThan lt, int64_t* cnt) {
    const int i = threadIdx.x;
    if (i >= kLongerThresholds) return;
    int64_t lo = 0, hi = nrows;  // first row with at most t slots
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (rp[mid + 1] - rp[mid] > lt.t[i]) lo = mid + 1;
        else hi = mid;
    }
    cnt[i] = lo;
}

// One wave per heavy row walks the row's slots (sorted by neighbour, so each
// slab's slots form one run).  FILL = false: the length of the run of every
// (row, slab) pair into len[(b P + j) R + row in block].  FILL = true: with
// len scanned per (b, j), every slot's position seg + len + index in run, its
// packed (row, neighbour) and its CSR slot.
template <bool FILL>
__global__ void k_heavy_rows(const int64_t* rp, const int32_t* col, int64_t n_heavy, const int32_t* row_blk,
                             const int64_t* blk_row, int R, int C, int64_t P, uint32_t* len, const int64_t* seg,
                             uint32_t* pay, uint32_t* csr) {
    const int lane = threadIdx.x & 63;
    const int64_t u = ((int64_t)blockIdx.x * kT + threadIdx.x) >> 6;
    if (u >= n_heavy) return;
    const int64_t b = row_blk[u], ul = u - blk_row[b];
    const int64_t s0 = rp[u], s1 = rp[u + 1];
    int64_t carry_start = s0;  // first slot of the run that continues into this chunk
    int32_t carry_j = -1;
    for (int64_t base = s0; base < s1; base += 64) {
        const int64_t sl = base + lane;
        const bool valid = sl < s1;
        const int32_t v = valid ? col[sl] : 0;
        const int32_t j = valid ? v / C : INT32_MAX;
        int32_t jprev = __shfl_up(j, 1, 64);
        if (lane == 0) jprev = carry_j;
        const bool head = valid && j != jprev;
        const uint64_t H = __ballot(head);
        const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
        const uint64_t m = H & le;
        const int64_t rs = m ? base + (63 - __clzll(m)) : carry_start;
        if (FILL) {
            if (valid) {
                const int64_t k = (b * P + j);
                const int64_t pos = seg[k] + (int64_t)len[k * R + ul] + (sl - rs);
                pay[pos] = (((uint32_t)ul | (sl == rs ? 0x8000u : 0u)) << 16) | (uint32_t)(v - j * C);
                csr[pos] = (uint32_t)sl;
            }
        } else {
            int32_t jnext = __shfl_down(j, 1, 64);
            if (lane == 63) jnext = (sl + 1 < s1) ? col[sl + 1] / C : INT32_MAX;
            if (valid && (sl + 1 == s1 || jnext != j)) len[(b * P + j) * R + ul] = (uint32_t)(sl - rs + 1);
        }
        carry_start = __shfl(rs, 63, 64);
        carry_j = __shfl(j, 63, 64);
    }
}

// exclusive scan of each (b, j) row of len (R entries, in place); the
// segment's slot count padded to whole words into segsz[b P + j]
__global__ __launch_bounds__(256) void k_heavy_scan(uint32_t* len, int R, uint64_t* segsz) {
    __shared__ uint32_t part[256];
    uint32_t* row = len + (int64_t)blockIdx.x * R;
    const int per = (R + 255) / 256, t = threadIdx.x;
    uint32_t sum = 0;
    for (int i = 0; i < per; ++i) {
        const int k = t * per + i;
        if (k < R) sum += row[k];
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t x = (t >= off) ? part[t - off] : 0u;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int i = 0; i < per; ++i) {
        const int k = t * per + i;
        if (k < R) {
            const uint32_t x = row[k];
            row[k] = run;
            run += x;
        }
    }
    if (t == 255) segsz[blockIdx.x] = ((uint64_t)part[255] + 63) / 64 * 64;
}

__global__ void k_fill_u32v(uint32_t* p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (i < n) p[i] = v;
}

template <class T>
T d2h(const T* p, hipStream_t s) {
    T v;
    LDS_HIP(hipMemcpyAsync(&v, p, sizeof(T), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    return v;
}

}  // namespace

namespace {

int64_t env_int(const char* name, int64_t dflt) {
    const char* e = std::getenv(name);
    if (!e || !*e) return dflt;
    return std::strtoll(e, nullptr, 10);
}

// The 2D part of a large edge plan (see HeavyPlan), built only when
// LDS_HEAVY_DEG is set: on the 4M-vertex power-law workload it measured
// slower than the one-dimensional sweep (1.01 against 0.945 ms per launch
// with rows of degree >= 128 in it), so it is off by default.  Rows of degree
// >= LDS_HEAVY_DEG are heavy when their slots number at least
// LDS_HEAVY_MIN_SLOTS (default 2^22) and the graph has more than one slab;
// LDS_HEAVY_ROWS (<= 8192) and LDS_HEAVY_SLAB (<= 24576, a multiple of 8)
// override the block and slab sizes, LDS_HEAVY_PART the positions of a part
// (default: a quarter of the positions per compute unit, at least 4096).
// Returns the heavy row count (0: none).
int64_t build_heavy(SweepPlan& p, int64_t n, hipStream_t s) {
    HeavyPlan& h = p.heavy;
    h = HeavyPlan{};
    if (p.h != 2 || p.rid != nullptr || n <= 0 || p.nrows == 0) return 0;
    // every row with more than a chunk's slots must be heavy (no hub pieces
    // then), so the threshold is at most kChunk + 1
    const int64_t deg_env = env_int("LDS_HEAVY_DEG", 0);
    if (deg_env <= 0) return 0;  // off unless asked for (see the header comment)
    const int64_t deg_min = std::min<int64_t>(deg_env, kChunk + 1);
    const int64_t min_slots = env_int("LDS_HEAVY_MIN_SLOTS", (int64_t)1 << 22);
    const int R = (int)(std::min<int64_t>(std::max<int64_t>(64, env_int("LDS_HEAVY_ROWS", kHeavyRows)), kHeavyRows) /
                        64 * 64);
    const int C = (int)(std::min<int64_t>(std::max<int64_t>(64, env_int("LDS_HEAVY_SLAB", kHeavySlab)), kHeavySlab) /
                        8 * 8);
    if (n <= C) return 0;
    DBuf<unsigned long long> cnt;
    cnt.alloc(1, s);
    LDS_HIP(hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), s));
    k_count_deg<<<grid_for(p.nrows, kT), kT, 0, s>>>(p.rp, p.nrows, deg_min, cnt.p);
    LDS_HIP(hipGetLastError());
    const int64_t nh = (int64_t)d2h(cnt.p, s);
    if (nh == 0) return 0;
    int64_t hslots = 0;
    LDS_HIP(hipMemcpyAsync(&hslots, p.rp + nh, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    if (hslots < min_slots) return 0;
    h.n_heavy = nh;
    h.R = R;
    h.C = C;
    h.P = (n + C - 1) / C;
    // blocks: consecutive rows, at most R of them and, for long rows, at most
    // LDS_HEAVY_BLOCK_SLOTS (default 2^22) slots, so that no block needs a
    // great many parts
    const int64_t cap = std::max<int64_t>(1, env_int("LDS_HEAVY_BLOCK_SLOTS", (int64_t)1 << 22));
    std::vector<int64_t> hrp(nh + 1);
    LDS_HIP(hipMemcpyAsync(hrp.data(), p.rp, hrp.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    std::vector<int64_t> brow{0};
    std::vector<int32_t> rblk(nh);
    for (int64_t u = 0; u < nh; ++u) {
        const int64_t b0 = brow.back();
        if (u > b0 && (u - b0 >= R || hrp[u + 1] - hrp[b0] > cap)) brow.push_back(u);
        rblk[u] = (int32_t)(brow.size() - 1);
    }
    brow.push_back(nh);
    h.n_blocks = (int64_t)brow.size() - 1;
    h.blk_row.alloc(brow.size(), s);
    h.row_blk.alloc(nh, s);
    LDS_HIP(hipMemcpyAsync(h.blk_row.p, brow.data(), brow.size() * 8, hipMemcpyHostToDevice, s));
    LDS_HIP(hipMemcpyAsync(h.row_blk.p, rblk.data(), rblk.size() * 4, hipMemcpyHostToDevice, s));
    const int64_t nseg = h.n_blocks * h.P;
    // run lengths per (block, slab, row), scanned per (block, slab)
    DBuf<uint32_t> len;
    len.alloc((size_t)nseg * R, s);
    LDS_HIP(hipMemsetAsync(len.p, 0, len.bytes(), s));
    k_heavy_rows<false><<<grid_for(nh * 64, kT), kT, 0, s>>>(p.rp, p.py, nh, h.row_blk.p, h.blk_row.p, R, C, h.P,
                                                             len.p, nullptr, nullptr, nullptr);
    LDS_HIP(hipGetLastError());
    h.seg.alloc(nseg + 1, s);
    k_heavy_scan<<<(unsigned)nseg, 256, 0, s>>>(len.p, R, (uint64_t*)h.seg.p);
    LDS_HIP(hipGetLastError());
    DBuf<uint64_t> tot;
    tot.alloc(1, s);
    exclusive_scan_u64((uint64_t*)h.seg.p, (uint64_t*)h.seg.p, nseg, tot.p, s);
    k_set_last<<<1, 1, 0, s>>>(h.seg.p, nseg, tot.p);
    LDS_HIP(hipGetLastError());
    h.positions = (int64_t)d2h(tot.p, s);
    h.pay.alloc(h.positions, s);
    h.csr.alloc(h.positions, s);
    if (h.positions > 0) {
        k_fill_u32v<<<grid_for(h.positions, kT), kT, 0, s>>>(h.pay.p, h.positions, 0xffffffffu);
        k_fill_u32v<<<grid_for(h.positions, kT), kT, 0, s>>>(h.csr.p, h.positions, 0xffffffffu);
        LDS_HIP(hipGetLastError());
    }
    k_heavy_rows<true><<<grid_for(nh * 64, kT), kT, 0, s>>>(p.rp, p.py, nh, h.row_blk.p, h.blk_row.p, R, C, h.P,
                                                            len.p, h.seg.p, h.pay.p, h.csr.p);
    LDS_HIP(hipGetLastError());
    // parts: each block's positions cut into near-equal word-aligned ranges
    std::vector<int64_t> seg(nseg + 1);
    LDS_HIP(hipMemcpyAsync(seg.data(), h.seg.p, seg.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    int dev = 0, cus = 0;
    LDS_HIP(hipGetDevice(&dev));
    LDS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t dflt = (h.positions / std::max<int64_t>(1, 4 * (int64_t)std::max(cus, 1)) + 63) / 64 * 64;
    const int64_t target = std::max<int64_t>(64, env_int("LDS_HEAVY_PART", std::max<int64_t>(64 * 64, dflt))) / 64 * 64;
    std::vector<int32_t> pb, pj0, pj1, bp(h.n_blocks + 1, 0);
    std::vector<int64_t> ps, pe;
    for (int64_t b = 0; b < h.n_blocks; ++b) {
        bp[b] = (int32_t)pb.size();
        const int64_t B0 = seg[b * h.P], B1 = seg[(b + 1) * h.P];
        const int64_t np = std::max<int64_t>(1, (B1 - B0 + target - 1) / target);
        for (int64_t k = 0; k < np; ++k) {
            const int64_t q0 = B0 + (B1 - B0) * k / np / 64 * 64;
            const int64_t q1 = (k + 1 == np) ? B1 : B0 + (B1 - B0) * (k + 1) / np / 64 * 64;
            if (q1 <= q0) continue;
            // slabs whose segments meet [q0, q1)
            int64_t j0 = 0, j1 = h.P;
            while (j0 < h.P && seg[b * h.P + j0 + 1] <= q0) ++j0;
            while (j1 > j0 && seg[b * h.P + j1 - 1] >= q1) --j1;
            pb.push_back((int32_t)b);
            pj0.push_back((int32_t)j0);
            pj1.push_back((int32_t)j1);
            ps.push_back(q0);
            pe.push_back(q1);
        }
    }
    bp[h.n_blocks] = (int32_t)pb.size();
    h.n_parts = (int64_t)pb.size();
    LDS_CHECK(h.n_parts < INT32_MAX / 2, ST_INVALID, "too many parts in the heavy sweep plan");
    h.part_blk.alloc(h.n_parts, s);
    h.part_j0.alloc(h.n_parts, s);
    h.part_j1.alloc(h.n_parts, s);
    h.blk_part.alloc(h.n_blocks + 1, s);
    h.part_cnt.alloc((size_t)h.n_parts * R, s);
    h.part_lo.alloc(h.n_parts, s);
    h.part_hi.alloc(h.n_parts, s);
    LDS_HIP(hipMemcpyAsync(h.part_blk.p, pb.data(), pb.size() * 4, hipMemcpyHostToDevice, s));
    LDS_HIP(hipMemcpyAsync(h.part_j0.p, pj0.data(), pj0.size() * 4, hipMemcpyHostToDevice, s));
    LDS_HIP(hipMemcpyAsync(h.part_j1.p, pj1.data(), pj1.size() * 4, hipMemcpyHostToDevice, s));
    LDS_HIP(hipMemcpyAsync(h.part_lo.p, ps.data(), ps.size() * 8, hipMemcpyHostToDevice, s));
    LDS_HIP(hipMemcpyAsync(h.part_hi.p, pe.data(), pe.size() * 8, hipMemcpyHostToDevice, s));
    LDS_HIP(hipMemcpyAsync(h.blk_part.p, bp.data(), bp.size() * 4, hipMemcpyHostToDevice, s));
    LDS_HIP(hipStreamSynchronize(s));
    return nh;
}

}  // namespace

void build_sweep_plan(SweepPlan& p, hipStream_t s, int64_t n_vertices) {
    const int64_t nrows = p.nrows;
    const int64_t n_heavy = n_vertices > 0 ? build_heavy(p, n_vertices, s) : 0;
    // hub rows (more than a chunk's slots) and big rows (at least 64 slots):
    // prefixes of the rows, which are ordered by slot count
    int64_t hub_big[kLongerThresholds] = {0, 0};
    if (nrows > 0) {
        const LongerThan lt{{(int64_t)kChunk, 63, 0, 0, 0, 0, 0, 0, 0}};
        DBuf<int64_t> cnt;
        cnt.alloc(kLongerThresholds, s);
        k_rows_longer<<<1, 64, 0, s>>>(p.rp, nrows, lt, cnt.p);
        LDS_HIP(hipGetLastError());
        LDS_HIP(hipMemcpyAsync(hub_big, cnt.p, sizeof(hub_big), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
    }
    p.n_hub = hub_big[0];
    // with a 2D part, every row of more than a chunk's slots is heavy: the
    // chunks start after the heavy rows and there are no hub pieces
    if (n_heavy > 0) {
        LDS_CHECK(n_heavy >= p.n_hub, ST_INVALID, "heavy rows must include every hub row");
        p.n_hub = n_heavy;
    }
    p.n_big = hub_big[1];
    // hub word offsets (none with a 2D part: its rows have no words there)
    p.hwo.alloc(p.n_hub + 1, s);
    if (n_heavy > 0) {
        LDS_HIP(hipMemsetAsync(p.hwo.p, 0, p.hwo.bytes(), s));
    } else if (p.n_hub > 0) {
        k_hub_words<<<grid_for(p.n_hub, kT), kT, 0, s>>>(p.rp, p.n_hub, (uint64_t*)p.hwo.p);
        LDS_HIP(hipGetLastError());
    }
    DBuf<uint64_t> tot;
    tot.alloc(1, s);
    if (n_heavy == 0) {
        exclusive_scan_u64((uint64_t*)p.hwo.p, (uint64_t*)p.hwo.p, p.n_hub, tot.p, s);
        k_set_last<<<1, 1, 0, s>>>(p.hwo.p, p.n_hub, tot.p);
        LDS_HIP(hipGetLastError());
        p.hub_words = (int64_t)d2h(tot.p, s);
    } else {
        p.hub_words = 0;
    }
    // hub pieces and their per-row counters
    p.n_pieces = 0;
    if (p.n_hub > 0 && n_heavy == 0) {
        DBuf<uint32_t> npc;
        DBuf<uint64_t> first;
        npc.alloc(p.n_hub, s);
        first.alloc(p.n_hub, s);
        k_hub_pieces<<<grid_for(p.n_hub, kT), kT, 0, s>>>(p.rp, p.n_hub, nullptr, npc.p);
        LDS_HIP(hipGetLastError());
        exclusive_scan_u32_to_u64(npc.p, first.p, p.n_hub, tot.p, s);
        p.n_pieces = (int64_t)d2h(tot.p, s);
        LDS_CHECK(p.n_pieces < INT32_MAX, ST_INVALID, "too many hub pieces");
        p.hp_row.alloc(p.n_pieces, s);
        p.hp_off.alloc(p.n_pieces, s);
        k_hub_piece_fill<<<grid_for(p.n_hub, kT), kT, 0, s>>>(p.rp, p.n_hub, nullptr, first.p, p.hp_row.p,
                                                              p.hp_off.p);
        LDS_HIP(hipGetLastError());
        p.hub_ctr.alloc(p.n_hub, s);
        LDS_HIP(hipMemsetAsync(p.hub_ctr.p, 0, p.hub_ctr.bytes(), s));
    }
    // hub push (edge plans in internal order): the hub rows' codes and their
    // 16-bit per-workgroup counters must fit the sweep's LDS beside each other,
    // and no hub row may have 2^16 slots (a counter never wraps into the next)
    p.n_push = p.push_nc = p.n_ppieces = 0;
    if (p.h == 2 && p.rid == nullptr && n_heavy == 0 && p.n_hub > 0) {
        int64_t r01[2] = {0, 0};
        LDS_HIP(hipMemcpyAsync(r01, p.rp, sizeof(r01), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
        const int64_t nc = ((kSweepLds - 4 * ((p.n_hub + 1) / 2)) / 2) & ~(int64_t)1;
        const int64_t ncache = std::min<int64_t>(n_vertices, nc);
        if (r01[1] - r01[0] < 65536 && ncache >= std::min<int64_t>(n_vertices, p.n_hub)) {
            p.n_push = p.n_hub;
            p.push_nc = ncache;
            p.hub_pre.alloc(p.n_hub, s);
            k_hub_prefix<<<grid_for(p.n_hub, kT), kT, 0, s>>>(p.rp, p.py, p.n_hub, p.hub_pre.p);
            LDS_HIP(hipGetLastError());
            DBuf<uint32_t> npc;
            DBuf<uint64_t> first;
            npc.alloc(p.n_hub, s);
            first.alloc(p.n_hub, s);
            k_hub_pieces<<<grid_for(p.n_hub, kT), kT, 0, s>>>(p.rp, p.n_hub, p.hub_pre.p, npc.p);
            LDS_HIP(hipGetLastError());
            exclusive_scan_u32_to_u64(npc.p, first.p, p.n_hub, tot.p, s);
            p.n_ppieces = (int64_t)d2h(tot.p, s);
            p.pp_row.alloc(p.n_ppieces, s);
            p.pp_off.alloc(p.n_ppieces, s);
            if (p.n_ppieces > 0) {
                k_hub_piece_fill<<<grid_for(p.n_hub, kT), kT, 0, s>>>(p.rp, p.n_hub, p.hub_pre.p, first.p,
                                                                      p.pp_row.p, p.pp_off.p);
                LDS_HIP(hipGetLastError());
            }
        }
    }
    // chunks
    int64_t base = 0;
    LDS_HIP(hipMemcpyAsync(&base, p.rp + p.n_hub, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    const int64_t nonhub = p.nslots - base;
    p.n_chunks = (nonhub + kChunk - 1) / kChunk;
    p.chunk_row.alloc(p.n_chunks + 1, s);
    p.cwo.alloc(p.n_chunks + 1, s);
    if (p.n_chunks > 0) {
        k_chunk_rows<<<grid_for(nrows - p.n_hub + 1, kT), kT, 0, s>>>(p.rp, nrows, p.n_hub, p.n_chunks,
                                                                       p.chunk_row.p);
        LDS_HIP(hipGetLastError());
        k_chunk_words<<<grid_for(p.n_chunks, kT), kT, 0, s>>>(p.rp, p.chunk_row.p, p.n_chunks,
                                                             (uint64_t*)p.cwo.p);
        LDS_HIP(hipGetLastError());
    } else {
        LDS_HIP(hipMemcpyAsync(p.chunk_row.p, &nrows, sizeof(int64_t), hipMemcpyHostToDevice, s));
    }
    exclusive_scan_u64((uint64_t*)p.cwo.p, (uint64_t*)p.cwo.p, p.n_chunks, tot.p, s);
    k_set_last<<<1, 1, 0, s>>>(p.cwo.p, p.n_chunks, tot.p);
    LDS_HIP(hipGetLastError());
    p.chunk_words = (int64_t)d2h(tot.p, s);
    p.heavy.word0 = p.chunk_words + p.hub_words;
    p.total_words = p.chunk_words + p.hub_words + p.heavy.positions / 64;
    p.head.alloc(p.chunk_words, s);
    if (p.chunk_words) LDS_HIP(hipMemsetAsync(p.head.p, 0, p.head.bytes(), s));
    if (nrows > p.n_hub) {
        k_head<<<grid_for(nrows - p.n_hub, kT), kT, 0, s>>>(p.rp, nrows, p.n_hub, p.chunk_row.p, p.cwo.p,
                                                           (unsigned long long*)p.head.p);
        LDS_HIP(hipGetLastError());
    }
    p.bitbase.alloc(nrows, s);
    if (nrows > 0) {
        k_bitbase<<<grid_for(nrows, kT), kT, 0, s>>>(p.rp, nrows, p.n_hub, p.chunk_row.p, p.cwo.p, p.hwo.p,
                                                    p.chunk_words, n_heavy > 0, p.bitbase.p);
        LDS_HIP(hipGetLastError());
    }
    LDS_HIP(hipStreamSynchronize(s));
}

void build_graph(Graph& g, int64_t n, int64_t npairs, const int32_t* src, const int32_t* dst, bool on_device,
                 bool strict, hipStream_t s) {
    LDS_CHECK(n >= 0 && n <= 0x7fffffffLL, ST_INVALID, "n must be in [0, 2^31)");
    LDS_CHECK(npairs >= 0, ST_INVALID, "npairs must be >= 0");
    LDS_CHECK(npairs == 0 || (src && dst), ST_INVALID, "src/dst must not be NULL");
    g.n = n;
    g.stream = s;
    g.vbits = bits_for((uint64_t)n);
    if (g.vbits < 1) g.vbits = 1;
    g.idbits = bits_for(n > 0 ? (uint64_t)(n - 1) : 0);
    if (g.idbits < 1) g.idbits = 1;
    const int vb = g.vbits;
    const uint64_t sentinel = ((uint64_t)n << vb) | (uint64_t)n;

    // 1. both orientations of every pair -> sort -> drop duplicates and
    //    self-loops: the symmetric CSR in original ids, rows ascending
    DBuf<int32_t> dsrc, ddst;
    const int32_t *ps = src, *pd = dst;
    if (!on_device && npairs > 0) {
        dsrc.alloc(npairs, s);
        ddst.alloc(npairs, s);
        LDS_HIP(hipMemcpyAsync(dsrc.p, src, npairs * sizeof(int32_t), hipMemcpyHostToDevice, s));
        LDS_HIP(hipMemcpyAsync(ddst.p, dst, npairs * sizeof(int32_t), hipMemcpyHostToDevice, s));
        ps = dsrc.p;
        pd = ddst.p;
    }
    DBuf<unsigned> err;
    err.alloc(1, s);
    LDS_HIP(hipMemsetAsync(err.p, 0, sizeof(unsigned), s));
    DBuf<uint64_t> skeys;
    int64_t ns = 0;
    if (npairs > 0) {
        const int64_t nk = 2 * npairs;
        DBuf<uint64_t> keys, tmp;
        keys.alloc(nk, s);
        tmp.alloc(nk, s);
        k_canon<<<grid_for(npairs, kT), kT, 0, s>>>(ps, pd, npairs, n, vb, strict, keys.p, err.p);
        LDS_HIP(hipGetLastError());
        dsrc.release();
        ddst.release();
        radix_sort_u64(keys.p, nullptr, nk, 2 * vb, tmp.p, nullptr, s);
        DBuf<uint32_t> flag;
        flag.alloc(nk, s);
        k_unique_flags<<<grid_for(nk, kT), kT, 0, s>>>(keys.p, nk, sentinel, strict, flag.p, err.p);
        LDS_HIP(hipGetLastError());
        DBuf<uint64_t> total;
        total.alloc(1, s);
        exclusive_scan_u32_to_u64(flag.p, tmp.p, nk, total.p, s);
        ns = (int64_t)d2h(total.p, s);
        skeys.alloc(ns, s);
        k_compact<<<grid_for(nk, kT), kT, 0, s>>>(keys.p, flag.p, tmp.p, nk, skeys.p);
        LDS_HIP(hipGetLastError());
    }
    const unsigned e = d2h(err.p, s);
    LDS_CHECK(!(e & 1u), ST_INVALID, "vertex id out of range [0, n)");
    LDS_CHECK(!(e & 2u), ST_INVALID, "self-loop in strict mode");
    LDS_CHECK(!(e & 4u), ST_INVALID, "duplicate pair in strict mode");
    g.m = ns / 2;

    // 2. degrees from the row runs (no atomics), renumbering by degree desc,
    //    original id asc
    DBuf<int32_t> deg_orig;
    DBuf<int64_t> rstart, rend;
    deg_orig.alloc(n, s);
    rstart.alloc(n, s);
    rend.alloc(n, s);
    if (n) {
        LDS_HIP(hipMemsetAsync(rstart.p, 0, n * sizeof(int64_t), s));
        LDS_HIP(hipMemsetAsync(rend.p, 0, n * sizeof(int64_t), s));
    }
    if (ns > 0) {
        k_row_bounds<<<grid_for(ns, kT), kT, 0, s>>>(skeys.p, ns, vb, rstart.p, rend.p);
        LDS_HIP(hipGetLastError());
    }
    if (n > 0) {
        k_row_deg<<<grid_for(n, kT), kT, 0, s>>>(rstart.p, rend.p, n, deg_orig.p);
        LDS_HIP(hipGetLastError());
    }
    rend.release();
    DBuf<int> dmax;
    DBuf<unsigned long long> nz;
    dmax.alloc(1, s);
    nz.alloc(1, s);
    LDS_HIP(hipMemsetAsync(dmax.p, 0, sizeof(int), s));
    LDS_HIP(hipMemsetAsync(nz.p, 0, sizeof(unsigned long long), s));
    if (n > 0) {
        k_maxdeg<<<std::min(grid_for(n, kT), kReduceWG), kT, 0, s>>>(deg_orig.p, n, dmax.p, nz.p);
        LDS_HIP(hipGetLastError());
    }
    g.max_deg = d2h(dmax.p, s);
    g.n_nz = (int64_t)d2h(nz.p, s);
    g.orig_of.alloc(n, s);
    g.int_of.alloc(n, s);
    g.deg.alloc(n, s);
    if (n > 0) {
        DBuf<uint64_t> rk, rt;
        rk.alloc(n, s);
        rt.alloc(n, s);
        k_relabel_keys<<<grid_for(n, kT), kT, 0, s>>>(deg_orig.p, n, vb, g.max_deg, rk.p);
        LDS_HIP(hipGetLastError());
        radix_sort_u64(rk.p, nullptr, n, vb + bits_for((uint64_t)g.max_deg), rt.p, nullptr, s);
        k_relabel_apply<<<grid_for(n, kT), kT, 0, s>>>(rk.p, n, vb, deg_orig.p, g.orig_of.p, g.int_of.p,
                                                      g.deg.p);
        LDS_HIP(hipGetLastError());
    }

    // 3. symmetric CSR in internal ids, every row sorted ascending (the
    //    triangle listing needs sorted rows; sorting here, once, means that the
    //    slot order of the edge sweep never changes after ingest, so FW state
    //    stays valid whatever runs later on the graph)
    g.rowptr.alloc(n + 1, s);
    g.col.alloc(ns, s);
    g.col_sorted = false;
    {
        DBuf<uint64_t> total;
        total.alloc(1, s);
        exclusive_scan_u32_to_u64((const uint32_t*)g.deg.p, (uint64_t*)g.rowptr.p, n, total.p, s);
        k_set_last<<<1, 1, 0, s>>>(g.rowptr.p, n, total.p);
        LDS_HIP(hipGetLastError());
    }
    if (ns > 0) {
        k_permute<<<grid_for(ns, kT), kT, 0, s>>>(skeys.p, ns, vb, rstart.p, g.int_of.p, g.rowptr.p, g.col.p);
        LDS_HIP(hipGetLastError());
    }
    skeys.release();
    sort_rows(g, s);

    // 4. edge sweep plan: rows are internal vertices [0, n_nz), degree-sorted
    SweepPlan& p = g.edge_plan;
    p.h = 2;
    p.nrows = g.n_nz;
    p.nslots = ns;
    p.rid = nullptr;
    p.rp = g.rowptr.p;
    p.py = g.col.p;
    build_sweep_plan(p, s, n);
}

void sort_rows(Graph& g, hipStream_t s) {
    if (g.col_sorted) return;
    const int64_t ns = 2 * g.m, n = g.n;
    if (ns > 0) {
        // rows with more than T slots form a prefix (rows are ordered by
        // length): the prefix lengths for every threshold in one pass
        LongerThan lt{{4096, 512, 128, 64, 32, 16, 8, 4, 1}};
        DBuf<int64_t> cnt;
        cnt.alloc(kLongerThresholds, s);
        k_rows_longer<<<1, 64, 0, s>>>(g.rowptr.p, n, lt, cnt.p);
        LDS_HIP(hipGetLastError());
        int64_t hc[kLongerThresholds];
        LDS_HIP(hipMemcpyAsync(hc, cnt.p, sizeof(hc), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
        const int64_t rb = hc[0], r512 = hc[1], r128 = hc[2], r64 = hc[3], r32 = hc[4], r16 = hc[5], r8 = hc[6],
                      r4 = hc[7], r1 = hc[8];
        if (rb > 0) {  // long rows: radix sort of (row, column) keys
            int64_t nk = 0;
            LDS_HIP(hipMemcpyAsync(&nk, g.rowptr.p + rb, sizeof(int64_t), hipMemcpyDeviceToHost, s));
            LDS_HIP(hipStreamSynchronize(s));
            DBuf<uint64_t> keys, tmp;
            keys.alloc(nk, s);
            tmp.alloc(nk, s);
            k_row_keys<<<(unsigned)std::min<int64_t>(rb, 65535), kT, 0, s>>>(g.rowptr.p, rb, g.col.p, keys.p);
            LDS_HIP(hipGetLastError());
            radix_sort_u64(keys.p, nullptr, nk, 32 + bits_for((uint64_t)rb), tmp.p, nullptr, s);
            k_row_unkeys<<<grid_for(nk, kT), kT, 0, s>>>(keys.p, nk, g.col.p);
            LDS_HIP(hipGetLastError());
        }
        if (r512 > rb) k_sort_rows_block<256, 4096><<<(unsigned)(r512 - rb), 256, 0, s>>>(g.rowptr.p, rb, g.col.p);
        if (r128 > r512) k_sort_rows_block<128, 512><<<(unsigned)(r128 - r512), 128, 0, s>>>(g.rowptr.p, r512, g.col.p);
        if (r64 > r128) k_sort_rows_block<64, 128><<<(unsigned)(r64 - r128), 64, 0, s>>>(g.rowptr.p, r128, g.col.p);
        LDS_HIP(hipGetLastError());
        auto lanes = [&](auto tag, int64_t a, int64_t b) {
            constexpr int S = decltype(tag)::value;
            if (b > a)
                k_sort_rows_lanes<S><<<grid_for((b - a + 64 / S - 1) / (64 / S) * 64, kT), kT, 0, s>>>(
                    g.rowptr.p, a, b, g.col.p);
            LDS_HIP(hipGetLastError());
        };
        lanes(std::integral_constant<int, 64>(), r64, r32);
        lanes(std::integral_constant<int, 32>(), r32, r16);
        lanes(std::integral_constant<int, 16>(), r16, r8);
        lanes(std::integral_constant<int, 8>(), r8, r4);
        lanes(std::integral_constant<int, 4>(), r4, r1);
    }
    g.col_sorted = true;
}

namespace {

void view_plan(SweepPlan& d, const SweepPlan& p, hipStream_t s) {
    d.h = p.h;
    d.nrows = p.nrows;
    d.nslots = p.nslots;
    d.rid = p.rid;
    d.rp = p.rp;
    d.py = p.py;
    d.own_rid.borrow(p.own_rid);
    d.own_rp.borrow(p.own_rp);
    d.own_py.borrow(p.own_py);
    d.own_tos.borrow(p.own_tos);
    d.own_row_of.borrow(p.own_row_of);
    d.n_big = p.n_big;
    d.n_hub = p.n_hub;
    d.hwo.borrow(p.hwo);
    d.n_pieces = p.n_pieces;
    d.hp_row.borrow(p.hp_row);
    d.hp_off.borrow(p.hp_off);
    d.n_push = p.n_push;
    d.push_nc = p.push_nc;
    d.hub_pre.borrow(p.hub_pre);
    d.n_ppieces = p.n_ppieces;
    d.pp_row.borrow(p.pp_row);
    d.pp_off.borrow(p.pp_off);
    if (p.hub_ctr.n) {  // written by every sweep: the view's own, zero between sweeps
        d.hub_ctr.alloc(p.hub_ctr.n, s);
        LDS_HIP(hipMemsetAsync(d.hub_ctr.p, 0, d.hub_ctr.bytes(), s));
    }
    d.n_chunks = p.n_chunks;
    d.chunk_row.borrow(p.chunk_row);
    d.cwo.borrow(p.cwo);
    d.head.borrow(p.head);
    d.chunk_words = p.chunk_words;
    d.hub_words = p.hub_words;
    d.total_words = p.total_words;
    d.bitbase.borrow(p.bitbase);
    const HeavyPlan& h = p.heavy;
    HeavyPlan& e = d.heavy;
    e.n_heavy = h.n_heavy;
    e.R = h.R;
    e.C = h.C;
    e.P = h.P;
    e.n_blocks = h.n_blocks;
    e.n_parts = h.n_parts;
    e.positions = h.positions;
    e.word0 = h.word0;
    e.seg.borrow(h.seg);
    e.pay.borrow(h.pay);
    e.csr.borrow(h.csr);
    e.part_blk.borrow(h.part_blk);
    e.part_j0.borrow(h.part_j0);
    e.part_j1.borrow(h.part_j1);
    e.part_lo.borrow(h.part_lo);
    e.part_hi.borrow(h.part_hi);
    e.blk_part.borrow(h.blk_part);
    e.blk_row.borrow(h.blk_row);
    e.row_blk.borrow(h.row_blk);
    if (h.part_cnt.n) e.part_cnt.alloc(h.part_cnt.n, s);  // rewritten by every sweep
}

}  // namespace

std::unique_ptr<Graph> graph_view(Graph& g, hipStream_t s) {
    auto v = std::make_unique<Graph>();
    v->n = g.n;
    v->m = g.m;
    v->n_nz = g.n_nz;
    v->idbits = g.idbits;
    v->vbits = g.vbits;
    v->max_deg = g.max_deg;
    v->orig_of.borrow(g.orig_of);
    v->int_of.borrow(g.int_of);
    v->deg.borrow(g.deg);
    v->rowptr.borrow(g.rowptr);
    v->col.borrow(g.col);
    v->col_sorted = g.col_sorted;
    view_plan(v->edge_plan, g.edge_plan, s);
    v->T = g.T;
    v->tri.borrow(g.tri);
    v->tcount.borrow(g.tcount);
    v->t_max = g.t_max;
    if (g.T >= 0) view_plan(v->tri_plan, g.tri_plan, s);
    v->Q4 = g.Q4;
    v->q4.borrow(g.q4);
    v->qcount.borrow(g.qcount);
    v->q_max = g.q_max;
    if (g.Q4 >= 0) view_plan(v->clique_plan, g.clique_plan, s);
    v->origin = g.origin ? g.origin : &g;
    v->stream = s;
    return v;
}

Graph::~Graph() {
    for (auto& f : fw)
        for (auto& e : f.ev)
            if (e) (void)hipEventDestroy(e);
}

size_t Graph::device_bytes() const {
    size_t b = orig_of.bytes() + int_of.bytes() + deg.bytes() + rowptr.bytes() + col.bytes() +
               edge_plan.device_bytes() + tri.bytes() + tcount.bytes() + tri_plan.device_bytes() + q4.bytes() +
               qcount.bytes() + clique_plan.device_bytes();
    for (const auto& f : fw) b += f.device_bytes();
    for (const auto& x : sg) b += x.device_bytes();
    return b;
}

}  // namespace lds
