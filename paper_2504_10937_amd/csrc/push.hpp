// Hub push of the edge sweep (k_fw_sweep, k_push_finish): a hub row only
// compares itself with the other hub rows (its hub prefix); every other row
// that loses a slot to a hub neighbour adds 1 to that hub's 16-bit
// per-workgroup counter in LDS, and k_push_finish sums the counters and
// writes the hub rows' keys.  The hub rows' slots against non-hub vertices
// are thus neither streamed nor gathered and carry no decision bits, so
// their split numerators follow from the mirror slot: the two shares of an
// edge sum to D.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lds {

// a[s] = D - a[mirror(s)] for every slot s of a hub row r < n_push past its
// hub prefix (rp[r] + hub_pre[r] .. rp[r + 1]); the mirror is r's slot in
// the row of s's neighbour v, found by binary search (rows are sorted by
// neighbour id, and v's row is not a hub row, so the kernel never writes a
// slot it reads).  One workgroup per hub row at a time; each thread runs
// kMirrorU searches side by side, so that their dependent loads overlap
// (6.0 ms on lds_large with one search at a time, 3.2 ms with 8; 16 gave the
// same, and loading the first 16 entries of v's row before searching was
// slower: the per-lane loads, not their latency, then set the time).
constexpr int kMirrorU = 8;
template <class T>
__global__ void k_push_mirror(const int64_t* rp, const int32_t* py, const int32_t* hub_pre, int64_t n_push,
                              uint64_t D, T* a) {
    for (int64_t r = blockIdx.x; r < n_push; r += gridDim.x) {
        const int64_t s0 = rp[r] + hub_pre[r], s1 = rp[r + 1];
        for (int64_t base = s0 + threadIdx.x; base < s1; base += (int64_t)blockDim.x * kMirrorU) {
            int64_t lo[kMirrorU], hi[kMirrorU];
#pragma unroll
            for (int u = 0; u < kMirrorU; ++u) {
                const int64_t s = base + (int64_t)u * blockDim.x;
                lo[u] = hi[u] = 0;
                if (s < s1) {
                    const int32_t v = py[s];
                    lo[u] = rp[v];
                    hi[u] = rp[v + 1];
                }
            }
            for (bool more = true; more;) {
                more = false;
#pragma unroll
                for (int u = 0; u < kMirrorU; ++u) {
                    if (lo[u] < hi[u]) {
                        const int64_t mid = (lo[u] + hi[u]) >> 1;
                        if (py[mid] < (int32_t)r)
                            lo[u] = mid + 1;
                        else
                            hi[u] = mid;
                        more = more || lo[u] < hi[u];
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kMirrorU; ++u) {
                const int64_t s = base + (int64_t)u * blockDim.x;
                if (s < s1) a[s] = (T)(D - (uint64_t)a[lo[u]]);
            }
        }
    }
}

}  // namespace lds
