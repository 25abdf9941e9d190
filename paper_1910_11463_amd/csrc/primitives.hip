// Device primitives: caching allocator, exclusive scan, member-id fill.
#include <map>
#include <mutex>
#include <unordered_map>

#include "amg.h"
#include "kernels_common.h"

namespace pair {

// ---------------------------------------------------------------- allocator
namespace {
struct Block {
    size_t size;
    hipStream_t stream;
};
struct Pool {
    std::mutex mu;
    std::multimap<std::pair<hipStream_t, size_t>, void*> free_blocks;   // (stream, size) -> ptr
    std::unordered_map<void*, Block> live;
    size_t in_use = 0;
};
Pool& pool() {
    static Pool* p = new Pool();   // intentionally leaked: outlives static destructors
    return *p;
}
thread_local hipStream_t t_pool_stream = nullptr;
// blocks of retired streams, usable by all
hipStream_t const kShared = reinterpret_cast<hipStream_t>(~uintptr_t(0));
size_t round_size(size_t b) {
    size_t r = 256;
    while (r < b) r <<= 1;
    return r;
}
}  // namespace

PoolStream::PoolStream(hipStream_t s) : prev(t_pool_stream) { t_pool_stream = s; }
PoolStream::~PoolStream() { t_pool_stream = prev; }

void* pool_alloc(size_t bytes) {
    Pool& P = pool();
    const size_t sz = round_size(bytes);
    const hipStream_t st = t_pool_stream;
    {
        std::lock_guard<std::mutex> g(P.mu);
        for (hipStream_t key : {st, kShared}) {
            auto it = P.free_blocks.find({key, sz});
            if (it != P.free_blocks.end()) {
                void* p = it->second;
                P.free_blocks.erase(it);
                P.live[p] = Block{sz, st};
                P.in_use += sz;
                return p;
            }
        }
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
        // release cached blocks and retry once
        pool_release_all();
        (void)hipGetLastError();
        e = hipMalloc(&p, sz);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw Error(E_OOM, "device allocation of " + std::to_string(sz) + " bytes failed");
        }
    }
    std::lock_guard<std::mutex> g(P.mu);
    P.live[p] = Block{sz, st};
    P.in_use += sz;
    return p;
}

void pool_free(void* p) {
    if (!p) return;
    Pool& P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    auto it = P.live.find(p);
    if (it == P.live.end()) return;
    P.free_blocks.emplace(std::make_pair(it->second.stream, it->second.size), p);
    P.in_use -= it->second.size;
    P.live.erase(it);
}

void pool_retire_stream(hipStream_t s) {
    Pool& P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    for (auto it = P.free_blocks.begin(); it != P.free_blocks.end();) {
        if (it->first.first == s) {
            P.free_blocks.emplace(std::make_pair(kShared, it->first.second), it->second);
            it = P.free_blocks.erase(it);
        } else {
            ++it;
        }
    }
    for (auto& kv : P.live)
        if (kv.second.stream == s) kv.second.stream = kShared;
}

void pool_release_all() {
    Pool& P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    for (auto& kv : P.free_blocks) (void)hipFree(kv.second);
    P.free_blocks.clear();
}

size_t pool_bytes_in_use() { return pool().in_use; }

// ---------------------------------------------------------------- scan
namespace {
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

__global__ void __launch_bounds__(kScanBlock)
k_scan_tiles(const int64_t* __restrict__ in, int64_t* __restrict__ out, int64_t n,
             int64_t* __restrict__ tile_sums) {
    __shared__ int64_t sh[kScanTile];
    __shared__ int64_t wsum[kScanBlock / 64];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    for (int i = threadIdx.x; i < kScanTile; i += kScanBlock) {
        int64_t g = base + i;
        sh[i] = g < n ? in[g] : 0;
    }
    __syncthreads();
    int64_t v[kScanItems];
    int64_t run = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = run;
        run += sh[threadIdx.x * kScanItems + k];
    }
    // exclusive scan of the per-thread totals across the block
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t incl = wave_inclusive_scan(run);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    int64_t woff = 0;
    for (int w = 0; w < wid; ++w) woff += wsum[w];
    int64_t excl = woff + incl - run;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) sh[threadIdx.x * kScanItems + k] = v[k] + excl;
    __syncthreads();
    for (int i = threadIdx.x; i < kScanTile; i += kScanBlock) {
        int64_t g = base + i;
        if (g < n) out[g] = sh[i];
    }
    if (threadIdx.x == kScanBlock - 1) tile_sums[blockIdx.x] = excl + run;
}

__global__ void k_add_tile_offsets(int64_t* __restrict__ out, int64_t n,
                                   const int64_t* __restrict__ off) {
    int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g < n) out[g] += off[g / kScanTile];
}

__global__ void k_set_total(int64_t* out, int64_t n, const int64_t* in_last, const int64_t* out_last) {
    out[n] = (n > 0) ? (*out_last + *in_last) : 0;
}
}  // namespace

int64_t exclusive_scan(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
    if (n <= 0) {
        int64_t z = 0;
        PAIR_HIP(hipMemcpyAsync(out, &z, sizeof(int64_t), hipMemcpyHostToDevice, s));
        PAIR_HIP(hipStreamSynchronize(s));
        return 0;
    }
    int64_t ntiles = (n + kScanTile - 1) / kScanTile;
    DBuf<int64_t> sums(ntiles), offs(ntiles + 1);
    hipLaunchKernelGGL(k_scan_tiles, dim3(static_cast<unsigned>(ntiles)), dim3(kScanBlock), 0, s,
                       in, out, n, sums.p);
    PAIR_LAUNCH_CHECK();
    if (ntiles > 1) {
        exclusive_scan(sums.p, offs.p, ntiles, s);
        hipLaunchKernelGGL(k_add_tile_offsets, dim3(grid_for(n, 256)), dim3(256), 0, s, out, n,
                           offs.p);
        PAIR_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_set_total, dim3(1), dim3(1), 0, s, out, n, in + (n - 1), out + (n - 1));
    PAIR_LAUNCH_CHECK();
    int64_t total = 0;
    PAIR_HIP(hipMemcpyAsync(&total, out + n, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PAIR_HIP(hipStreamSynchronize(s));
    return total;
}

// ---------------------------------------------------------------- segments
namespace {
__global__ void k_fill_seg(uint16_t* seg, int64_t begin, int64_t count, uint16_t id) {
    int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g < count) seg[begin + g] = id;
}
}  // namespace

void fill_segments(uint16_t* seg, int64_t n, const std::vector<int64_t>& off,
                   const std::vector<int64_t>& cnt, hipStream_t s) {
    (void)n;
    for (size_t b = 0; b < off.size(); ++b) {
        if (off[b] < 0 || cnt[b] == 0) continue;
        hipLaunchKernelGGL(k_fill_seg, dim3(grid_for(cnt[b], 256)), dim3(256), 0, s, seg, off[b],
                           cnt[b], static_cast<uint16_t>(b));
        PAIR_LAUNCH_CHECK();
    }
}

int choose_lpr(double avg) {
    int l = 1;
    while (l < 64 && l * 1.5 < avg) l <<= 1;
    return l;
}

}  // namespace pair
