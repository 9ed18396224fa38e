// Batched Frank-Wolfe (Alg. 1 / Alg. 6) over many independent graphs in one
// persistent kernel launch, captured once into a hipGraph and replayed.
//
// Each workgroup takes whole graphs from a device work queue (an atomic
// counter over the items, which are ordered longest-first) and runs all the
// iterations of a graph by itself: the iteration barrier is a workgroup
// barrier instead of a kernel boundary, and the keys of a graph with at most
// `kmax` vertices live in LDS for the whole run (two ping-pong buffers), so
// every gather of a neighbour's key is an LDS read.  Larger graphs keep their
// keys in their own device buffers (L2-resident for the sizes admitted here).
//
// The arithmetic, the slot layout and the decision-word layout are those of
// the per-graph sweep: a vertex wins a slot iff its packed key
// (A << B) | (2^B - 1 - orig_id) is below the keys of the pattern's other
// vertices; wins of a row are counted from the decision words; A += inc_i * b.
// So a batched run leaves every graph in exactly the state a per-graph run of
// the same iteration count leaves (keys, decision words, gap sums), and every
// later call (loads, splits, stable groups, top-k) reads it unchanged.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>

#include "batch.hpp"

namespace lds {

namespace {

typedef unsigned __int128 u128;

struct BItem {
    const int32_t* rid;  // compact row -> vertex (nullptr: identity)
    const int64_t* rp;
    const int32_t* py;
    const int64_t* hwo;
    const int64_t* chunk_row;
    const int64_t* cwo;
    const uint64_t* head;
    const int32_t* cnt;     // deg (edges) or triangle count per vertex
    const int32_t* orig_of;
    uint64_t* K0;           // the graph's key buffers
    uint64_t* K1;
    uint64_t* bits;         // iters * total_words decision words
    uint64_t* sums;         // iters * 4 exact gap sums, or nullptr
    float* r_out;           // n loads by caller id, or nullptr
    int64_t n_hub, n_chunks, chunk_words, total_words, nrows;
    int32_t n, h, mult, B, iters, lds_keys;
};

__device__ inline u128 wave_sum128(u128 x) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        const uint64_t lo = (uint64_t)x, hi = (uint64_t)(x >> 64);
        const uint64_t lo2 = ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(lo >> 32), m, 64) << 32) |
                             (uint32_t)__shfl_xor((int)(uint32_t)lo, m, 64);
        const uint64_t hi2 = ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(hi >> 32), m, 64) << 32) |
                             (uint32_t)__shfl_xor((int)(uint32_t)hi, m, 64);
        x += ((u128)hi2 << 64) | lo2;
    }
    return x;
}

__device__ inline uint64_t readlane64(uint64_t v, int lane) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t fw_inc(int h, int i) {  // D_i - D_{i-1}
    return (uint64_t)(h == 3 ? 6 : 2) * (uint64_t)(i + 1);
}

// does the vertex with key ku beat the other vertices of the pattern at slot s?
template <int H>
__device__ inline bool wins(uint64_t ku, const uint64_t* K, const int32_t* __restrict__ py, int64_t s) {
    if (H == 2) return ku < K[py[s]];
    const int2 v = reinterpret_cast<const int2*>(py)[s];
    return ku < K[v.x] && ku < K[v.y];
}

template <int H, int NT>
__device__ void run_graph(const BItem& it, uint64_t* Ka, uint64_t* Kb, uint64_t (*words)[32], uint64_t (*red)[4],
                          uint32_t* hcnt) {
    constexpr int NW = NT / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int B = it.B;
    const uint64_t idm = (1ull << B) - 1ull;
    // initial keys in both buffers: vertices without slots never change
    for (int u = threadIdx.x; u < it.n; u += NT) {
        const uint64_t k = (((uint64_t)it.cnt[u] * (uint64_t)it.mult) << B) | (idm - (uint64_t)it.orig_of[u]);
        Ka[u] = k;
        Kb[u] = k;
    }
    __syncthreads();
    uint64_t* Kin = Ka;
    uint64_t* Kout = Kb;
    for (int i = 1; i <= it.iters; ++i) {
        const uint64_t inc = fw_inc(H, i);
        uint64_t* bits = it.bits + (int64_t)(i - 1) * it.total_words;
        u128 sq = 0, mn = 0;
        // hub rows: the whole workgroup, one row at a time
        for (int64_t r = 0; r < it.n_hub; ++r) {
            const int32_t u = it.rid ? it.rid[r] : (int32_t)r;
            const int64_t s0 = it.rp[r], s1 = it.rp[r + 1];
            const uint64_t Ku = Kin[u];
            uint64_t* bw = bits + it.chunk_words + it.hwo[r];
            uint32_t cnt = 0;
            for (int64_t base = s0; base < s1; base += NT) {
                const int64_t s = base + threadIdx.x;
                const bool win = s < s1 && wins<H>(Ku, Kin, it.py, s);
                const uint64_t W = __ballot(win);
                const int64_t wb = base + 64 * w;
                if (lane == 0 && wb < s1) bw[(wb - s0) / 64] = W;
                cnt += (uint32_t)__popcll(W);
            }
            if (lane == 0) hcnt[w] = cnt;
            __syncthreads();
            if (threadIdx.x == 0) {
                uint64_t tot = 0;
                for (int q = 0; q < NW; ++q) tot += hcnt[q];
                Kout[u] = Ku + ((tot * inc) << B);
                if (it.sums) {
                    const uint64_t A = Ku >> B;
                    sq += (u128)A * A;
                    mn += (u128)A * tot;
                }
            }
            __syncthreads();
        }
        // chunks: one wave each; decision words, then one lane per row
        for (int64_t c = w; c < it.n_chunks; c += NW) {
            const int64_t r0 = it.chunk_row[c], r1 = it.chunk_row[c + 1];
            if (r0 >= r1) continue;
            const int64_t s0 = it.rp[r0], s1 = it.rp[r1];
            const int64_t w0 = it.cwo[c];
            const int nw = (int)(it.cwo[c + 1] - w0);  // <= 32
            const int nsl = (int)(s1 - s0);
            const uint64_t hreg = (lane < nw) ? it.head[w0 + lane] : 0ull;
            const uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
            int32_t rb = -1;  // chunk-relative row of the slot before the current word
            uint64_t mybits = 0;
            for (int t = 0; t < nw; ++t) {
                const uint64_t Hw = readlane64(hreg, t);
                const int off = t * 64 + lane;
                const int32_t row = rb + (int32_t)__popcll(Hw & le);
                rb += (int32_t)__popcll(Hw);
                bool win = false;
                if (off < nsl) {
                    const int32_t u = it.rid ? it.rid[r0 + row] : (int32_t)(r0 + row);
                    win = wins<H>(Kin[u], Kin, it.py, s0 + off);
                }
                const uint64_t W = __ballot(win);
                if (lane == t) mybits = W;
            }
            if (lane < nw) {
                bits[w0 + lane] = mybits;
                words[w][lane] = mybits;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            for (int64_t rbase = r0; rbase < r1; rbase += 64) {
                const int64_t r = rbase + lane;
                if (r < r1) {
                    const int sa = (int)(it.rp[r] - s0), sb = (int)(it.rp[r + 1] - s0);
                    uint32_t cnt = 0;
                    for (int wd = sa >> 6; wd <= ((sb - 1) >> 6); ++wd) {
                        const int lo = max(sa - wd * 64, 0), hi = min(sb - wd * 64, 64);
                        const uint64_t mk = ((hi >= 64) ? ~0ull : ((1ull << hi) - 1ull)) & (~0ull << lo);
                        cnt += (uint32_t)__popcll(words[w][wd] & mk);
                    }
                    const int32_t u = it.rid ? it.rid[r] : (int32_t)r;
                    const uint64_t Ku = Kin[u];
                    Kout[u] = Ku + (((uint64_t)cnt * inc) << B);
                    if (it.sums) {
                        const uint64_t A = Ku >> B;
                        sq += (u128)A * A;
                        mn += (u128)A * cnt;
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();  // words[w] is rewritten by the next chunk
        }
        if (it.sums) {
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
                for (int q = 0; q < NW; ++q) {
                    S += ((u128)red[q][1] << 64) | red[q][0];
                    M += ((u128)red[q][3] << 64) | red[q][2];
                }
                uint64_t* o = it.sums + 4 * (int64_t)(i - 1);
                o[0] = (uint64_t)S;
                o[1] = (uint64_t)(S >> 64);
                o[2] = (uint64_t)M;
                o[3] = (uint64_t)(M >> 64);
            }
        }
        __syncthreads();  // all keys of iteration i written before iteration i+1 reads them
        uint64_t* t = Kin;
        Kin = Kout;
        Kout = t;
    }
    // final keys into the graph's buffer number (iters & 1), loads by caller id
    uint64_t* Kfin = (it.iters & 1) ? it.K1 : it.K0;
    const double D = (double)((uint64_t)(H == 3 ? 3 : 1) * (uint64_t)(it.iters + 1) * (uint64_t)(it.iters + 2));
    for (int u = threadIdx.x; u < it.n; u += NT) {
        const uint64_t k = Kin[u];
        if (it.lds_keys) Kfin[u] = k;
        if (it.r_out) it.r_out[it.orig_of[u]] = (float)((double)(k >> B) / D);
    }
    __syncthreads();  // LDS keys are reused by the next graph
}

template <int NT>
__global__ __launch_bounds__(NT) void k_fw_batch(const BItem* __restrict__ items, int32_t count, int32_t* queue,
                                                int32_t kmax) {
    extern __shared__ uint64_t skeys[];  // 2 * kmax
    constexpr int NW = NT / 64;
    __shared__ uint64_t words[NW][32];
    __shared__ uint64_t red[NW][4];
    __shared__ uint32_t hcnt[NW];
    __shared__ int32_t next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(queue, 1);
        __syncthreads();
        const int32_t idx = next;
        __syncthreads();  // every thread has read `next`
        if (idx >= count) break;
        const BItem it = items[idx];
        uint64_t* Ka = it.lds_keys ? skeys : it.K0;
        uint64_t* Kb = it.lds_keys ? skeys + kmax : it.K1;
        if (it.h == 2)
            run_graph<2, NT>(it, Ka, Kb, words, red, hcnt);
        else
            run_graph<3, NT>(it, Ka, Kb, words, red, hcnt);
    }
}

__global__ void k_zero_i32(int32_t* p) { *p = 0; }

template <int NT>
void set_lds_limit(size_t bytes) {
    LDS_HIP(hipFuncSetAttribute((const void*)k_fw_batch<NT>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
}

template <int NT>
void launch_batch(unsigned grid, size_t lds, hipStream_t s, const BItem* items, int32_t count, int32_t* queue,
                  int32_t kmax) {
    k_fw_batch<NT><<<grid, NT, lds, s>>>(items, count, queue, kmax);
}

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        LDS_HIP(hipGetDevice(&dev));
        LDS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        if (cus <= 0) cus = 1;
    }
    return cus;
}

}  // namespace

int64_t batch_cost(const Graph& g, int mode, int iters) {
    const SweepPlan& p = (mode == 2) ? g.edge_plan : g.tri_plan;
    return (p.nslots + g.n) * (int64_t)std::max(iters, 1);
}

Batch::~Batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap) (void)hipStreamDestroy(cap);
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    if (ev[1]) (void)hipEventDestroy(ev[1]);
}

void batch_build(Batch& b, hipStream_t s) {
    const int count = (int)b.gs.size();
    const BatchTune& t = b.tune;
    LDS_CHECK(t.threads == 256 || t.threads == 512 || t.threads == 1024, ST_INVALID, "threads must be 256, 512 or 1024");
    LDS_CHECK(t.wg_per_cu >= 1 && t.wg_per_cu <= 8, ST_INVALID, "wg_per_cu must be in [1, 8]");
    LDS_CHECK(t.lds_vertices >= 0 && t.lds_vertices <= 8192, ST_INVALID, "lds_vertices must be in [0, 8192]");
    // FW buffers of every graph, triangle lists, key-width checks
    for (int i = 0; i < count; ++i) fw_prepare(*b.gs[i], b.modes[i], b.iters[i], s);
    // kernel items vs per-graph runs
    b.kernel_items.clear();
    b.plain_items.clear();
    for (int i = 0; i < count; ++i) {
        // graphs with a 2D part (large edge plans) take their own launches
        if (batch_cost(*b.gs[i], b.modes[i], b.iters[i]) <= t.max_kernel_cost &&
            plan_of(*b.gs[i], b.modes[i]).heavy.n_parts == 0)
            b.kernel_items.push_back(i);
        else
            b.plain_items.push_back(i);
    }
    if (t.longest_first)
        std::stable_sort(b.kernel_items.begin(), b.kernel_items.end(), [&](int x, int y) {
            return batch_cost(*b.gs[x], b.modes[x], b.iters[x]) > batch_cost(*b.gs[y], b.modes[y], b.iters[y]);
        });
    int32_t kmax = 0;
    for (int i : b.kernel_items)
        if (b.gs[i]->n <= t.lds_vertices) kmax = std::max<int32_t>(kmax, (int32_t)b.gs[i]->n);
    b.kmax = kmax;
    const size_t nk = b.kernel_items.size();
    b.sums.release();
    if (b.want_gap) {
        int64_t tot = 0;
        for (int i : b.kernel_items) tot += 4 * (int64_t)b.iters[i];
        b.sums.alloc((size_t)std::max<int64_t>(tot, 1), s);
    }
    std::vector<BItem> h(nk);
    int64_t soff = 0;
    b.sum_off.assign(nk, 0);
    for (size_t j = 0; j < nk; ++j) {
        const int i = b.kernel_items[j];
        Graph& g = *b.gs[i];
        const int mode = b.modes[i];
        const SweepPlan& p = (mode == 2) ? g.edge_plan : g.tri_plan;
        FwState& f = g.fw[mode == 2 ? 0 : 1];
        BItem& x = h[j];
        std::memset(&x, 0, sizeof(x));
        x.rid = p.rid;
        x.rp = p.rp;
        x.py = p.py;
        x.hwo = p.hwo.p;
        x.chunk_row = p.chunk_row.p;
        x.cwo = p.cwo.p;
        x.head = p.head.p;
        x.cnt = (mode == 2) ? g.deg.p : g.tcount.p;
        x.orig_of = g.orig_of.p;
        x.K0 = f.K[0].p;
        x.K1 = f.K[1].p;
        x.bits = f.bits.p;
        x.sums = b.want_gap ? b.sums.p + soff : nullptr;
        b.sum_off[j] = soff;
        if (b.want_gap) soff += 4 * (int64_t)b.iters[i];
        x.r_out = b.r_out.empty() ? nullptr : b.r_out[i];
        x.n_hub = p.n_hub;
        x.n_chunks = p.n_chunks;
        x.chunk_words = p.chunk_words;
        x.total_words = p.total_words;
        x.nrows = p.nrows;
        x.n = (int32_t)g.n;
        x.h = mode;
        x.mult = (mode == 2) ? 1 : 2;
        x.B = g.idbits;
        x.iters = (p.nrows > 0) ? b.iters[i] : 0;
        x.lds_keys = (g.n <= t.lds_vertices) ? 1 : 0;
        // a graph without patterns keeps its initial keys; its state still
        // records the requested iteration count
    }
    b.items.alloc(std::max<size_t>(nk, 1) * sizeof(BItem), s);
    if (nk) LDS_HIP(hipMemcpyAsync(b.items.p, h.data(), nk * sizeof(BItem), hipMemcpyHostToDevice, s));
    const BItem* items = reinterpret_cast<const BItem*>(b.items.p);
    b.queue.alloc(1, s);
    LDS_HIP(hipStreamSynchronize(s));
    // capture: reset the queue, run the batch kernel
    if (b.exec) {
        (void)hipGraphExecDestroy(b.exec);
        b.exec = nullptr;
    }
    if (b.graph) {
        (void)hipGraphDestroy(b.graph);
        b.graph = nullptr;
    }
    if (b.capture && !b.cap) LDS_HIP(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
    if (!b.ev[0]) {
        LDS_HIP(hipEventCreate(&b.ev[0]));
        LDS_HIP(hipEventCreate(&b.ev[1]));
    }
    if (nk == 0) return;
    const size_t lds = (size_t)2 * (size_t)kmax * sizeof(uint64_t);
    const unsigned grid =
        (unsigned)std::min<int64_t>((int64_t)device_cus() * t.wg_per_cu, (int64_t)nk);
    switch (t.threads) {
        case 256: set_lds_limit<256>(lds); break;
        case 512: set_lds_limit<512>(lds); break;
        default: set_lds_limit<1024>(lds); break;
    }
    b.grid = grid;
    b.lds_bytes = lds;
    if (!b.capture) return;
    LDS_HIP(hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal));
    k_zero_i32<<<1, 1, 0, b.cap>>>(b.queue.p);
    switch (t.threads) {
        case 256: launch_batch<256>(grid, lds, b.cap, items, (int32_t)nk, b.queue.p, kmax); break;
        case 512: launch_batch<512>(grid, lds, b.cap, items, (int32_t)nk, b.queue.p, kmax); break;
        default: launch_batch<1024>(grid, lds, b.cap, items, (int32_t)nk, b.queue.p, kmax); break;
    }
    const hipError_t le = hipGetLastError();
    hipGraph_t gr = nullptr;
    const hipError_t ce = hipStreamEndCapture(b.cap, &gr);
    LDS_HIP(le);
    LDS_HIP(ce);
    b.graph = gr;
    LDS_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
}

namespace {
void launch_direct(Batch& b, hipStream_t s) {
    const int32_t nk = (int32_t)b.kernel_items.size();
    if (nk == 0) return;
    const BItem* items = reinterpret_cast<const BItem*>(b.items.p);
    k_zero_i32<<<1, 1, 0, s>>>(b.queue.p);
    switch (b.tune.threads) {
        case 256: launch_batch<256>(b.grid, b.lds_bytes, s, items, nk, b.queue.p, b.kmax); break;
        case 512: launch_batch<512>(b.grid, b.lds_bytes, s, items, nk, b.queue.p, b.kmax); break;
        default: launch_batch<1024>(b.grid, b.lds_bytes, s, items, nk, b.queue.p, b.kmax); break;
    }
    LDS_HIP(hipGetLastError());
}
}  // namespace

void batch_run(Batch& b, hipStream_t s) {
    const int count = (int)b.gs.size();
    // graphs too large for one workgroup: per-graph runs on the same stream
    for (int i : b.plain_items) {
        fw_run(*b.gs[i], b.modes[i], b.iters[i], b.want_gap, s);
        if (!b.r_out.empty() && b.r_out[i]) fw_loads(*b.gs[i], b.modes[i], b.r_out[i], nullptr, nullptr, s);
    }
    LDS_HIP(hipEventRecord(b.ev[0], s));
    if (b.capture) {
        if (b.exec) LDS_HIP(hipGraphLaunch(b.exec, s));
    } else {
        launch_direct(b, s);
    }
    LDS_HIP(hipEventRecord(b.ev[1], s));
    for (size_t j = 0; j < b.kernel_items.size(); ++j) {
        const int i = b.kernel_items[j];
        Graph& g = *b.gs[i];
        const int mode = b.modes[i];
        FwState& f = g.fw[mode == 2 ? 0 : 1];
        f.iters = b.iters[i];
        const SweepPlan& p = (mode == 2) ? g.edge_plan : g.tri_plan;
        f.cur = (p.nrows > 0) ? (b.iters[i] & 1) : 0;
        f.ran = true;
        f.timed = false;
        f.gap.clear();
        f.lb.clear();
        f.fval.clear();
        g.sg[mode == 2 ? 0 : 1].valid = false;
    }
    b.runs++;
    (void)count;
    if (b.want_gap && !b.kernel_items.empty()) {
        std::vector<uint64_t> hs(b.sums.n);
        LDS_HIP(hipMemcpyAsync(hs.data(), b.sums.p, b.sums.bytes(), hipMemcpyDeviceToHost, s));
        LDS_HIP(hipStreamSynchronize(s));
        for (size_t j = 0; j < b.kernel_items.size(); ++j) {
            const int i = b.kernel_items[j];
            Graph& g = *b.gs[i];
            const int mode = b.modes[i];
            const SweepPlan& p = (mode == 2) ? g.edge_plan : g.tri_plan;
            if (p.nrows == 0) {
                std::vector<uint64_t> z((size_t)4 * b.iters[i], 0);
                fw_gap_from_sums(g.fw[mode == 2 ? 0 : 1], mode, b.iters[i], z.data());
            } else {
                fw_gap_from_sums(g.fw[mode == 2 ? 0 : 1], mode, b.iters[i], hs.data() + b.sum_off[j]);
            }
        }
    }
}

}  // namespace lds
