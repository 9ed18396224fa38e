// Device primitives for gfx950: exclusive prefix sums and a stable LSD radix
// sort (8-bit digits, 4096-key tiles, wave64 ballot matching for the stable
// in-tile ranks).  Used by graph ingest, the triangle incidence build and the
// sort of converged loads (the first step of Alg. 2).
#include "common.hpp"

namespace lds {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // 4096

__device__ inline uint64_t wave_incl_scan(uint64_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// inclusive scan over the 256 threads of a block; `total` gets the block sum
__device__ inline uint64_t block_incl_scan(uint64_t x, uint64_t* sh, uint64_t& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    x = wave_incl_scan(x);
    if (lane == 63) sh[w] = x;
    __syncthreads();
    uint64_t pre = 0;
    for (int i = 0; i < w; ++i) pre += sh[i];
    total = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    return x + pre;
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_tile_sums(const T* in, int64_t n, uint64_t* sums) {
    __shared__ uint64_t sh[4];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint64_t acc = 0;
    for (int k = 0; k < kItems; ++k) {
        int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
        if (i < n) acc += (uint64_t)in[i];
    }
    uint64_t tot;
    block_incl_scan(acc, sh, tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class T>
__global__ __launch_bounds__(kThreads) void k_tile_scan(const T* in, uint64_t* out, int64_t n,
                                                        const uint64_t* tile_off, uint64_t* total_dev,
                                                        int64_t ntiles) {
    __shared__ uint64_t sh[4];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint64_t carry = tile_off ? tile_off[blockIdx.x] : 0;
    for (int k = 0; k < kItems; ++k) {
        int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
        uint64_t x = (i < n) ? (uint64_t)in[i] : 0;
        uint64_t tot;
        uint64_t inc = block_incl_scan(x, sh, tot);
        if (i < n) out[i] = carry + inc - x;
        carry += tot;
    }
    if (total_dev && blockIdx.x == ntiles - 1 && threadIdx.x == 0) *total_dev = carry;
}

template <class T>
void scan_impl(const T* in, uint64_t* out, int64_t n, uint64_t* total_dev, hipStream_t s) {
    if (n <= 0) {
        if (total_dev) LDS_HIP(hipMemsetAsync(total_dev, 0, sizeof(uint64_t), s));
        return;
    }
    int64_t ntiles = (n + kTile - 1) / kTile;
    if (ntiles == 1) {
        k_tile_scan<T><<<1, kThreads, 0, s>>>(in, out, n, nullptr, total_dev, 1);
        LDS_HIP(hipGetLastError());
        return;
    }
    DBuf<uint64_t> sums;
    sums.alloc(ntiles, s);
    k_tile_sums<T><<<grid_for(ntiles, 1), kThreads, 0, s>>>(in, n, sums.p);
    LDS_HIP(hipGetLastError());
    scan_impl<uint64_t>(sums.p, sums.p, ntiles, nullptr, s);
    k_tile_scan<T><<<grid_for(ntiles, 1), kThreads, 0, s>>>(in, out, n, sums.p, total_dev, ntiles);
    LDS_HIP(hipGetLastError());
}

// ------------------------------------------------------------- radix sort
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint64_t* keys, int64_t n, int shift,
                                                         uint64_t* hist, int64_t nblocks) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int k = 0; k < kItems; ++k) {
        int64_t i = base + (int64_t)k * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

template <bool VALS>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const uint64_t* kin, const uint32_t* vin,
                                                            uint64_t* kout, uint32_t* vout, int64_t n,
                                                            int shift, const uint64_t* offs,
                                                            int64_t nblocks) {
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint64_t gofs[256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < 4 * 256; i += kThreads) (&wcnt[0][0])[i] = 0;
    gofs[threadIdx.x] = offs[(int64_t)threadIdx.x * nblocks + blockIdx.x];
    __syncthreads();
    // wave w owns the contiguous range [base, base + 1024) of the tile and
    // walks it in 16 rounds of 64 consecutive keys: rank order = key order
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)w * (kItems * 64);
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint64_t key[kItems];
    uint32_t val[kItems];
    uint32_t rank[kItems];
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + (int64_t)k * 64 + lane;
        const bool valid = i < n;
        key[k] = valid ? kin[i] : 0;
        if (VALS) val[k] = valid ? vin[i] : 0;
        const uint32_t d = (uint32_t)(key[k] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t r = (uint32_t)__popcll(peers & lt);
        uint32_t c = 0;
        if (valid) c = wcnt[w][d];
        rank[k] = c + r;
        if (valid && r == 0) wcnt[w][d] = c + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;
        uint32_t run = 0;
        for (int q = 0; q < 4; ++q) {
            uint32_t t = wcnt[q][d];
            wcnt[q][d] = run;
            run += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t i = base + (int64_t)k * 64 + lane;
        if (i < n) {
            const uint32_t d = (uint32_t)(key[k] >> shift) & 255u;
            const uint64_t pos = gofs[d] + wcnt[w][d] + rank[k];
            kout[pos] = key[k];
            if (VALS) vout[pos] = val[k];
        }
    }
}

}  // namespace

void exclusive_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total_dev, hipStream_t s) {
    scan_impl<uint64_t>(in, out, n, total_dev, s);
}
void exclusive_scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* total_dev,
                               hipStream_t s) {
    scan_impl<uint32_t>(in, out, n, total_dev, s);
}

void radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int end_bit, uint64_t* tmp_keys,
                    uint32_t* tmp_vals, hipStream_t s) {
    if (n <= 1 || end_bit <= 0) return;
    const int64_t nblocks = (n + kTile - 1) / kTile;
    DBuf<uint64_t> hist;
    hist.alloc((size_t)256 * nblocks, s);
    uint64_t *ka = keys, *kb = tmp_keys;
    uint32_t *va = vals, *vb = tmp_vals;
    int passes = 0;
    for (int shift = 0; shift < end_bit; shift += 8, ++passes) {
        k_radix_hist<<<grid_for(nblocks, 1), kThreads, 0, s>>>(ka, n, shift, hist.p, nblocks);
        LDS_HIP(hipGetLastError());
        exclusive_scan_u64(hist.p, hist.p, 256 * nblocks, nullptr, s);
        if (vals)
            k_radix_scatter<true><<<grid_for(nblocks, 1), kThreads, 0, s>>>(ka, va, kb, vb, n, shift, hist.p,
                                                                           nblocks);
        else
            k_radix_scatter<false><<<grid_for(nblocks, 1), kThreads, 0, s>>>(ka, nullptr, kb, nullptr, n,
                                                                            shift, hist.p, nblocks);
        LDS_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (passes & 1) {
        LDS_HIP(hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        if (vals) LDS_HIP(hipMemcpyAsync(vals, va, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }
    // hist is released at scope exit: either to the stream-ordered caching
    // allocator of the caller, or through hipFree, which synchronises.
}

}  // namespace lds
