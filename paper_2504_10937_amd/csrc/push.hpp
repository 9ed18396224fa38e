// Hub push of the edge sweep: the hub rows' slots against non-hub vertices
// carry no decision bits (the other row of the pair decides and adds the
// hub's wins to its counter), so their split numerators follow from the
// mirror slot: the two shares of an edge sum to D.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lds {

// a[s] = D - a[mirror(s)] for every slot s of a hub row r < n_push past its
// hub prefix (rp[r] + hub_pre[r] .. rp[r + 1]); the mirror is r's slot in
// the row of s's neighbour v, found by binary search (rows are sorted by
// neighbour id, and v's row is not a hub row, so the kernel never writes a
// slot it reads).  One workgroup per hub row at a time.
template <class T>
__global__ void k_push_mirror(const int64_t* rp, const int32_t* py, const int32_t* hub_pre, int64_t n_push,
                              uint64_t D, T* a) {
    for (int64_t r = blockIdx.x; r < n_push; r += gridDim.x) {
        const int64_t s0 = rp[r] + hub_pre[r], s1 = rp[r + 1];
        for (int64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
            const int32_t v = py[s];
            int64_t lo = rp[v], hi = rp[v + 1];
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (py[mid] < (int32_t)r)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            a[s] = (T)(D - (uint64_t)a[lo]);
        }
    }
}

}  // namespace lds
