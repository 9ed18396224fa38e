// Grid-wide barrier for cooperative launches (every workgroup resident).
//
// Only thread 0 of a workgroup makes the device-scope release / acquire: on
// a chip with several L2s these write back and invalidate the caches, which
// the workgroup's threads share; the others order their accesses against it
// with the workgroup barrier.  The arrival counter only grows (zeroed before
// the launch): a workgroup arriving at the k-th barrier draws a value in
// [k nwg, (k+1) nwg) and waits until the counter reaches (k+1) nwg, so one
// atomic per arrival and no separate generation word.  The wait is bounded:
// past the spin limit thread 0 sets *err (shared by the workgroup) and the
// barrier returns without the other workgroups.  Values that other
// workgroups wrote before the barrier (list counts, frontiers) are then not
// complete, so every caller tests *err after each barrier before it uses
// them and leaves its loop when it is set; the kernel ends and its host
// reports the error.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace lds {

constexpr unsigned kGridSpinLimit = 1u << 26;

__device__ inline void grid_sync(unsigned* counter, unsigned nwg, int64_t* err) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    if (nwg == 1) {  // one workgroup: its own barrier is enough
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        return;
    }
    if (threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned arrived = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = (arrived / nwg + 1) * nwg;
        unsigned spins = 0;
        while ((int)(__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
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

}  // namespace lds
