// Reference kernels for the roofline.  A plain streaming copy on gfx950, the
// achievable bandwidth the HBM-bound kernels are read against: every thread moves
// 16-byte vectors, eight in flight, grid-strided, non-temporal on both
// sides, over sixteen workgroups per compute unit.  And random 2-byte gathers
// from a table, the rate the Frank-Wolfe sweep's code gathers are read
// against.
#include "graph.hpp"

namespace lds {

namespace {

typedef unsigned int v4u __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_copy16(v4u* __restrict__ dst, const v4u* __restrict__ src, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    // eight vectors in flight per thread
    for (; i + 7 * stride < n; i += 8 * stride) {
        v4u v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = __builtin_nontemporal_load(src + i + k * stride);
#pragma unroll
        for (int k = 0; k < 8; ++k) __builtin_nontemporal_store(v[k], dst + i + k * stride);
    }
    for (; i < n; i += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// random 2-byte gathers: every thread streams eight indices, then gathers
// the eight table entries they name; the sum keeps the loads alive
__global__ __launch_bounds__(256) void k_gather16(const int32_t* __restrict__ idx, int64_t n,
                                                  const uint16_t* __restrict__ table, uint32_t* sink) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    uint32_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += 8 * stride) {
        int32_t v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = (i + k * stride < n) ? __builtin_nontemporal_load(idx + i + k * stride) : 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) acc += table[v[k]];
    }
    sink[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc;
}

}  // namespace

float gather_rate(const int32_t* idx, int64_t n, const uint16_t* table, int64_t entries, uint32_t* sink,
                  int reps, hipStream_t s) {
    LDS_CHECK(idx != nullptr && table != nullptr && sink != nullptr, ST_INVALID, "pointers must not be NULL");
    LDS_CHECK(n > 0 && entries > 0 && reps >= 1, ST_INVALID, "n, entries and reps must be positive");
    int dev = 0, cus = 0;
    LDS_HIP(hipGetDevice(&dev));
    LDS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * 8, (n + 255) / 256));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LDS_HIP(hipEventCreate(&e0));
    LDS_HIP(hipEventCreate(&e1));
    float ms = 0.0f;
    try {
        k_gather16<<<grid, 256, 0, s>>>(idx, n, table, sink);
        LDS_HIP(hipGetLastError());
        LDS_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) k_gather16<<<grid, 256, 0, s>>>(idx, n, table, sink);
        LDS_HIP(hipGetLastError());
        LDS_HIP(hipEventRecord(e1, s));
        LDS_HIP(hipEventSynchronize(e1));
        LDS_HIP(hipEventElapsedTime(&ms, e0, e1));
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / (float)reps;
}

float copy_bandwidth(void* dst, const void* src, size_t bytes, int reps, hipStream_t s) {
    LDS_CHECK(dst != nullptr && src != nullptr, ST_INVALID, "dst and src must not be NULL");
    LDS_CHECK(bytes % 16 == 0 && bytes > 0, ST_INVALID, "bytes must be a positive multiple of 16");
    LDS_CHECK(((uintptr_t)dst | (uintptr_t)src) % 16 == 0, ST_INVALID, "dst and src must be 16-byte aligned");
    LDS_CHECK(reps >= 1, ST_INVALID, "reps must be >= 1");
    const int64_t n = (int64_t)(bytes / 16);
    int dev = 0, cus = 0;
    LDS_HIP(hipGetDevice(&dev));
    LDS_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * 16, (n + 255) / 256));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    LDS_HIP(hipEventCreate(&e0));
    LDS_HIP(hipEventCreate(&e1));
    float ms = 0.0f;
    try {
        k_copy16<<<grid, 256, 0, s>>>((v4u*)dst, (const v4u*)src, n);  // warm-up
        LDS_HIP(hipGetLastError());
        LDS_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < reps; ++r) k_copy16<<<grid, 256, 0, s>>>((v4u*)dst, (const v4u*)src, n);
        LDS_HIP(hipGetLastError());
        LDS_HIP(hipEventRecord(e1, s));
        LDS_HIP(hipEventSynchronize(e1));
        LDS_HIP(hipEventElapsedTime(&ms, e0, e1));
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ms / (float)reps;
}

}  // namespace lds
