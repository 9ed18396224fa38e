// Wave64 reductions and segmented scans on the data-parallel primitives of
// gfx9 (DPP): shifts inside 16-lane rows, then broadcasts of a row's last lane
// to the rows after it.  Each step is a VALU operation with a DPP source, a
// few cycles, where a lane shuffle (an LDS permute) takes tens; the
// latency-bound loops of the stable-group scan run one such chain per
// phase.  Every function must be called with all 64 lanes of the wave active.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

namespace lds {
namespace wave {

// DPP controls of gfx9
constexpr int kRowShr1 = 0x111, kRowShr2 = 0x112, kRowShr4 = 0x114, kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142;  // lane 15 of a row to the next row (row mask 0xa: rows 1 and 3)
constexpr int kRowBcast31 = 0x143;  // lane 31 to rows 2 and 3 (row mask 0xc)
constexpr int kWaveShl1 = 0x130;    // lane i reads lane i + 1

// lane i reads the lane that CTRL names; a lane without a source (outside
// its row, or outside ROWS) keeps `old`
template <int CTRL, int ROWS>
__device__ inline int32_t dpp(int32_t v, int32_t old) {
    return __builtin_amdgcn_update_dpp(old, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ inline int64_t dpp(int64_t v, int64_t old) {
    const uint64_t u = (uint64_t)v, o = (uint64_t)old;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)u, CTRL, ROWS, 0xf, false);
    const uint32_t hi =
        (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(u >> 32), CTRL, ROWS, 0xf, false);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ inline int64_t lane63(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), 63);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// inclusive scan: lane i ends with op over lanes 0..i (id: op's identity)
template <class Op>
__device__ inline int64_t scan(int64_t v, int64_t id, Op op) {
    v = op(v, dpp<kRowShr1, 0xf>(v, id));
    v = op(v, dpp<kRowShr2, 0xf>(v, id));
    v = op(v, dpp<kRowShr4, 0xf>(v, id));
    v = op(v, dpp<kRowShr8, 0xf>(v, id));
    v = op(v, dpp<kRowBcast15, 0xa>(v, id));
    v = op(v, dpp<kRowBcast31, 0xc>(v, id));
    return v;
}

// the wave's maximum / minimum, the same in every lane
__device__ inline long long max_all(long long v) {
    return (long long)lane63(scan((int64_t)v, (int64_t)LLONG_MIN,
                                  [](int64_t a, int64_t b) { return a > b ? a : b; }));
}
__device__ inline long long min_all(long long v) {
    return (long long)lane63(scan((int64_t)v, (int64_t)LLONG_MAX,
                                  [](int64_t a, int64_t b) { return a < b ? a : b; }));
}

// Segmented inclusive prefix sum: lanes with equal keys must be contiguous
// (runs); lane i ends with the sum of its run's values up to lane i, so the
// last lane of a run holds the run's total.  A lane adds a shifted partial
// only when it comes from the same run: runs are contiguous, so every lane
// between the two carries that key too.
__device__ inline int64_t seg_prefix_sum(int32_t key, int64_t v) {
#define LDS_SEG_STEP(C, R)                                    \
    {                                                         \
        const int64_t o = dpp<C, R>(v, (int64_t)0);           \
        if (dpp<C, R>(key, (int32_t)INT_MIN) == key) v += o;  \
    }
    LDS_SEG_STEP(kRowShr1, 0xf)
    LDS_SEG_STEP(kRowShr2, 0xf)
    LDS_SEG_STEP(kRowShr4, 0xf)
    LDS_SEG_STEP(kRowShr8, 0xf)
    LDS_SEG_STEP(kRowBcast15, 0xa)
    LDS_SEG_STEP(kRowBcast31, 0xc)
#undef LDS_SEG_STEP
    return v;
}

// true on the last lane of each run of equal keys
__device__ inline bool run_tail(int32_t key) { return dpp<kWaveShl1, 0xf>(key, (int32_t)INT_MIN) != key; }

}  // namespace wave
}  // namespace lds
