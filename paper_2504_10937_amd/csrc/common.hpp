// Internal helpers shared by the gfx950 kernels and the host runtime of the
// LDS / LTDS library.  Not part of the public C ABI (see include/lds.h).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cmath>
#include <cstdio>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

namespace lds {

// Thrown inside the library and turned into an lds_status at the C ABI.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

enum : int { ST_OK = 0, ST_INVALID = 1, ST_NOMEM = 2, ST_DEVICE = 3, ST_OVERFLOW = 4, ST_BUSY = 5 };

void set_last_error(const std::string& msg);

#define LDS_HIP(call)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            throw ::lds::Error(e_ == hipErrorOutOfMemory ? ::lds::ST_NOMEM : ::lds::ST_DEVICE, \
                               std::string(#call) + ": " + hipGetErrorString(e_));           \
        }                                                                                     \
    } while (0)

#define LDS_CHECK(cond, code, msg)                       \
    do {                                                 \
        if (!(cond)) throw ::lds::Error((code), (msg));  \
    } while (0)

// Device allocation through an optional caller-registered allocator (the
// Python binding registers PyTorch's caching allocator); hipMalloc otherwise.
void* dev_alloc(size_t bytes, hipStream_t s);
void dev_free(void* p);

// Device buffer (RAII); memory comes from dev_alloc.  A buffer may instead
// borrow another's memory (a per-query view of a resident graph): it is then
// never freed through it, and its owner must outlive it.
template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    bool own = true;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), n(o.n), own(o.own) { o.p = nullptr; o.n = 0; o.own = true; }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            own = o.own;
            o.p = nullptr;
            o.n = 0;
            o.own = true;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count, hipStream_t s) {
        release();
        n = count;
        p = count ? static_cast<T*>(dev_alloc(count * sizeof(T), s)) : nullptr;
    }
    void borrow(const DBuf& o) {
        release();
        p = o.p;
        n = o.n;
        own = false;
    }
    void release() {
        if (p && own) dev_free(p);
        p = nullptr;
        n = 0;
        own = true;
    }
    size_t bytes() const { return n * sizeof(T); }
};

inline int bits_for(uint64_t v) {  // number of bits to hold values 0..v
    int b = 0;
    while (b < 64 && (v >> b)) ++b;
    return b;
}

inline unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 0x7fffffff) throw Error(ST_INVALID, "launch too large");
    return static_cast<unsigned>(g);
}

// workgroups of a grid-stride reduction into a few global counters (one
// atomic per wave): enough to fill the chip, few enough that the atomics on
// one address stay cheap
constexpr unsigned kReduceWG = 256;

// ---------------------------------------------------------------- scan/sort
// Exclusive prefix sum out[i] = sum_{j<i} in[i]; returns nothing, total is
// written to *total_dev when non-null.  in and out may alias.
void exclusive_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* total_dev, hipStream_t s);
void exclusive_scan_u32_to_u64(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* total_dev,
                               hipStream_t s);

// Stable LSD radix sort of 64-bit keys over bits [0, end_bit), with an
// optional 32-bit payload.  Result is left in keys/vals (buffers swapped
// internally through the provided temporaries of the same size).
void radix_sort_u64(uint64_t* keys, uint32_t* vals, int64_t n, int end_bit, uint64_t* tmp_keys,
                    uint32_t* tmp_vals, hipStream_t s);

}  // namespace lds
