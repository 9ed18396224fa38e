// Graph ingest on the device: canonical simple graph (Section 3 assumes an
// undirected simple graph), degree renumbering, symmetric CSR and the sweep
// plan (hub rows, row-aligned chunks, word offsets and row-start flags) that
// the Frank-Wolfe kernels stream over.
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "graph.hpp"

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
    const int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x;
    int d = (i < n) ? deg[i] : 0;
    // wave-level reduction first, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) d = max(d, __shfl_xor(d, off, 64));
    unsigned long long c = __popcll(__ballot(i < n && deg[i] > 0));
    if ((threadIdx.x & 63) == 0) {
        atomicMax(out, d);
        if (c) atomicAdd(nz, c);
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
__global__ void k_count_hubs(const int64_t* rp, int64_t nrows, unsigned long long* cnt) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    const bool hub = r < nrows && (rp[r + 1] - rp[r]) > kChunk;
    unsigned long long c = __popcll(__ballot(hub));
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

__global__ void k_count_big(const int64_t* rp, int64_t nrows, unsigned long long* cnt) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    const bool big = r < nrows && (rp[r + 1] - rp[r]) >= 64;
    unsigned long long c = __popcll(__ballot(big));
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(cnt, c);
}

__global__ void k_hub_words(const int64_t* rp, int64_t n_hub, uint64_t* words) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= n_hub) return;
    words[r] = (uint64_t)((rp[r + 1] - rp[r] + 63) / 64);
}

__global__ void k_hub_pieces(const int64_t* rp, int64_t n_hub, uint32_t* np) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r < n_hub) np[r] = (uint32_t)((rp[r + 1] - rp[r] + kPiece - 1) / kPiece);
}

__global__ void k_hub_piece_fill(const int64_t* rp, int64_t n_hub, const uint64_t* first, int32_t* hp_row,
                                 int32_t* hp_off) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= n_hub) return;
    const int64_t len = rp[r + 1] - rp[r];
    int64_t k = (int64_t)first[r];
    for (int64_t o = 0; o < len; o += kPiece, ++k) {
        hp_row[k] = (int32_t)r;
        hp_off[k] = (int32_t)o;
    }
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
                          const int64_t* cwo, const int64_t* hwo, int64_t chunk_words, int64_t* bitbase) {
    const int64_t r = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (r >= nrows) return;
    if (r < n_hub) {
        bitbase[r] = (chunk_words + hwo[r]) * 64;
    } else {
        const int64_t base = rp[n_hub];
        const int64_t c = (rp[r] - base) / kChunk;
        bitbase[r] = cwo[c] * 64 + (rp[r] - rp[chunk_row[c]]);
    }
}

template <class T>
T d2h(const T* p, hipStream_t s) {
    T v;
    LDS_HIP(hipMemcpyAsync(&v, p, sizeof(T), hipMemcpyDeviceToHost, s));
    LDS_HIP(hipStreamSynchronize(s));
    return v;
}

}  // namespace

void build_sweep_plan(SweepPlan& p, hipStream_t s) {
    const int64_t nrows = p.nrows;
    DBuf<unsigned long long> cnt;
    cnt.alloc(1, s);
    LDS_HIP(hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), s));
    if (nrows > 0) k_count_hubs<<<grid_for(nrows, kT), kT, 0, s>>>(p.rp, nrows, cnt.p);
    LDS_HIP(hipGetLastError());
    p.n_hub = (int64_t)d2h(cnt.p, s);
    LDS_HIP(hipMemsetAsync(cnt.p, 0, sizeof(unsigned long long), s));
    if (nrows > 0) k_count_big<<<grid_for(nrows, kT), kT, 0, s>>>(p.rp, nrows, cnt.p);
    LDS_HIP(hipGetLastError());
    p.n_big = (int64_t)d2h(cnt.p, s);
    // hub word offsets
    p.hwo.alloc(p.n_hub + 1, s);
    if (p.n_hub > 0) {
        k_hub_words<<<grid_for(p.n_hub, kT), kT, 0, s>>>(p.rp, p.n_hub, (uint64_t*)p.hwo.p);
        LDS_HIP(hipGetLastError());
    }
    DBuf<uint64_t> tot;
    tot.alloc(1, s);
    exclusive_scan_u64((uint64_t*)p.hwo.p, (uint64_t*)p.hwo.p, p.n_hub, tot.p, s);
    k_set_last<<<1, 1, 0, s>>>(p.hwo.p, p.n_hub, tot.p);
    LDS_HIP(hipGetLastError());
    p.hub_words = (int64_t)d2h(tot.p, s);
    // hub pieces and their per-row counters
    p.n_pieces = 0;
    if (p.n_hub > 0) {
        DBuf<uint32_t> npc;
        DBuf<uint64_t> first;
        npc.alloc(p.n_hub, s);
        first.alloc(p.n_hub, s);
        k_hub_pieces<<<grid_for(p.n_hub, kT), kT, 0, s>>>(p.rp, p.n_hub, npc.p);
        LDS_HIP(hipGetLastError());
        exclusive_scan_u32_to_u64(npc.p, first.p, p.n_hub, tot.p, s);
        p.n_pieces = (int64_t)d2h(tot.p, s);
        LDS_CHECK(p.n_pieces < INT32_MAX, ST_INVALID, "too many hub pieces");
        p.hp_row.alloc(p.n_pieces, s);
        p.hp_off.alloc(p.n_pieces, s);
        k_hub_piece_fill<<<grid_for(p.n_hub, kT), kT, 0, s>>>(p.rp, p.n_hub, first.p, p.hp_row.p, p.hp_off.p);
        LDS_HIP(hipGetLastError());
        p.hub_ctr.alloc(p.n_hub, s);
        LDS_HIP(hipMemsetAsync(p.hub_ctr.p, 0, p.hub_ctr.bytes(), s));
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
    p.total_words = p.chunk_words + p.hub_words;
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
                                                    p.chunk_words, p.bitbase.p);
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
        k_maxdeg<<<grid_for(n, kT), kT, 0, s>>>(deg_orig.p, n, dmax.p, nz.p);
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
    build_sweep_plan(p, s);
}

void sort_rows(Graph& g, hipStream_t s) {
    if (g.col_sorted) return;
    const int64_t ns = 2 * g.m;
    if (ns > 0) {
        // each row is a segment of keys below 2^vbits: a segmented radix sort
        // (small segments sorted in registers / LDS, large ones by passes)
        // instead of a global sort of (row, column) keys
        LDS_CHECK(ns < (int64_t)UINT32_MAX, ST_OVERFLOW, "too many slots for the row sort");
        DBuf<int32_t> out;
        out.alloc(ns, s);
        size_t bytes = 0;
        LDS_HIP(rocprim::segmented_radix_sort_keys(nullptr, bytes, (const uint32_t*)g.col.p, (uint32_t*)out.p,
                                                   (unsigned)ns, (unsigned)g.n, g.rowptr.p, g.rowptr.p + 1, 0u,
                                                   (unsigned)g.vbits, s));
        DBuf<uint8_t> tmp;
        tmp.alloc(bytes > 0 ? bytes : 1, s);
        LDS_HIP(rocprim::segmented_radix_sort_keys(tmp.p, bytes, (const uint32_t*)g.col.p, (uint32_t*)out.p,
                                                   (unsigned)ns, (unsigned)g.n, g.rowptr.p, g.rowptr.p + 1, 0u,
                                                   (unsigned)g.vbits, s));
        std::swap(g.col, out);
    }
    g.col_sorted = true;
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
