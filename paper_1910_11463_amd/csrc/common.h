// Shared host/device helpers of the pAIR transport library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

namespace pair {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

enum : int {
    OK = 0,
    E_INVALID = -1,
    E_HIP = -2,
    E_OOM = -3,
    E_NOCONV = -4,
    E_STATE = -5,
};

#define PAIR_HIP(expr)                                                                  \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess) {                                                         \
            throw ::pair::Error(_e == hipErrorOutOfMemory ? ::pair::E_OOM : ::pair::E_HIP, \
                                std::string(#expr) + ": " + hipGetErrorString(_e) +     \
                                    " (" + __FILE__ + ":" + std::to_string(__LINE__) + ")"); \
        }                                                                               \
    } while (0)

#define PAIR_CHECK(cond, msg)                                                           \
    do {                                                                                \
        if (!(cond)) throw ::pair::Error(::pair::E_INVALID, std::string(msg));          \
    } while (0)

#define PAIR_LAUNCH_CHECK() PAIR_HIP(hipGetLastError())

// ---------------------------------------------------------------- device memory
// Caching allocator: freed blocks are kept in bins by size (rounded up to a
// power of two) and by the stream their owner works on, and are handed out again
// only to allocations for that same stream, so stream order makes reuse safe
// without synchronisation while several streams work at once.  The stream of an
// allocation is the calling thread's pool stream (PoolStream).  All cached
// memory is returned by pool_release_all() (hipFree synchronises the device),
// which destroying a context or an AMG handle calls.
void* pool_alloc(size_t bytes);
void pool_free(void* p);
void pool_release_all();
size_t pool_bytes_in_use();
// Call once s is synchronised and no longer used: its cached blocks become
// available to every stream.
void pool_retire_stream(hipStream_t s);

// Sets the calling thread's pool stream for its lifetime (restored after).
struct PoolStream {
    explicit PoolStream(hipStream_t s);
    ~PoolStream();
    PoolStream(const PoolStream&) = delete;
    PoolStream& operator=(const PoolStream&) = delete;
    hipStream_t prev;
};

template <class T>
struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf& operator=(DBuf&& o) noexcept {
        if (this != &o) { reset(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { reset(); }
    void alloc(size_t count) {
        reset();
        n = count;
        if (count) p = static_cast<T*>(pool_alloc(count * sizeof(T)));
    }
    void reset() {
        if (p) pool_free(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

template <class T>
inline void h2d(T* d, const T* h, size_t n, hipStream_t s) {
    if (n) PAIR_HIP(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, s));
}
template <class T>
inline void d2h(T* h, const T* d, size_t n, hipStream_t s) {
    if (n) PAIR_HIP(hipMemcpyAsync(h, d, n * sizeof(T), hipMemcpyDeviceToHost, s));
}
template <class T>
inline void d2d(T* dst, const T* src, size_t n, hipStream_t s) {
    if (n) PAIR_HIP(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, s));
}

inline unsigned grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    return static_cast<unsigned>(g);
}

// Grids padded to a multiple of the XCD count so that xcd_block() can hand each
// XCD one contiguous range of logical blocks.
constexpr int kNumXcd = 8;
inline unsigned grid_xcd(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    g = (g + kNumXcd - 1) / kNumXcd * kNumXcd;
    return static_cast<unsigned>(g);
}

#ifdef __HIPCC__
// Workgroups are dispatched round-robin over the 8 XCDs (physical block b runs
// on XCD b % 8).  Remapping b -> (b % 8) * (G / 8) + b / 8 gives every XCD a
// contiguous slice of the row space, so neighbouring rows (which gather the same
// x entries) share one XCD's L2.  Requires gridDim.x % 8 == 0 (grid_xcd()).
__device__ __forceinline__ unsigned xcd_block() {
    unsigned G = gridDim.x, b = blockIdx.x;
    return (b % kNumXcd) * (G / kNumXcd) + b / kNumXcd;
}
#endif

}  // namespace pair
