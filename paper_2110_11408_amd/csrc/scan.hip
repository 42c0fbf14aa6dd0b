// Device-wide exclusive prefix sum of uint32 arrays and fill kernels.
//
// One pass with decoupled look-back: every tile of 256 threads x 16 items
// takes a ticket in launch order, scans its items staged through LDS,
// publishes its sum, and adds the sum of all earlier tiles, read back from
// their published sums and inclusive prefixes (each status word holds a flag
// and a value).  A tile only waits for tiles with smaller tickets, which have
// started before it, so every wait ends; the wait is bounded anyway and a
// timeout is reported through the error word.  LDS indices are padded by one
// word per 32 to keep the per-thread runs of 16 words off a single bank.
#include "hf_internal.h"

namespace hf {

namespace {

constexpr int kIpt = 16;
constexpr int kTile = kBlock * kIpt;

__device__ __forceinline__ int pad(int i) { return i + (i >> 5); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(v, d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread across the 256-thread block; *total
// receives the block sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wsum[kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; k++) {
        if (k < wid) pre += wsum[k];
        tot += wsum[k];
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

__global__ __launch_bounds__(kBlock) void k_tile_scan(const uint32_t *__restrict__ in,
                                                      uint32_t *__restrict__ out, int64_t n,
                                                      const uint32_t *__restrict__ tile_off) {
    __shared__ uint32_t buf[kTile + kTile / 32];
    int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
    for (int k = 0; k < kIpt; k++) {
        int idx = k * kBlock + threadIdx.x;
        int64_t i = base + idx;
        buf[pad(idx)] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t v[kIpt];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kIpt; k++) {
        v[k] = buf[pad(threadIdx.x * kIpt + k)];
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, &tot);
    uint32_t toff = tile_off ? tile_off[blockIdx.x] : 0u;
    run += toff;
#pragma unroll
    for (int k = 0; k < kIpt; k++) {
        buf[pad(threadIdx.x * kIpt + k)] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kIpt; k++) {
        int idx = k * kBlock + threadIdx.x;
        int64_t i = base + idx;
        if (i < n) out[i] = buf[pad(idx)];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = toff + tot;
}

constexpr uint64_t kAggregate = 1ull << 32;  // status flag: the tile's own sum
constexpr uint64_t kInclusive = 2ull << 32;  // status flag: sum of the tiles up to this one
constexpr uint32_t kSpinLimit = 1u << 22;

__global__ __launch_bounds__(kBlock) void k_scan_onepass(const uint32_t *in, uint32_t *out, int64_t n,
                                                         uint32_t *__restrict__ ticket,
                                                         uint64_t *__restrict__ status,
                                                         int32_t *__restrict__ err) {
    __shared__ uint32_t buf[kTile + kTile / 32];
    __shared__ uint32_t s_tile, s_prefix;
    if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t base = (int64_t)tile * kTile;
#pragma unroll
    for (int k = 0; k < kIpt; k++) {
        const int idx = k * kBlock + threadIdx.x;
        const int64_t i = base + idx;
        buf[pad(idx)] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t v[kIpt];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kIpt; k++) {
        v[k] = buf[pad(threadIdx.x * kIpt + k)];
        sum += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(sum, &tot);
    if (threadIdx.x == 0) {
        uint32_t prefix = 0;
        if (tile == 0) {
            __hip_atomic_store(status, kInclusive | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(status + tile, kAggregate | tot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t j = (int64_t)tile - 1;
            uint32_t spins = 0;
            while (j >= 0) {
                const uint64_t st = __hip_atomic_load(status + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t flag = st & (3ull << 32);
                if (flag == 0) {
                    if (++spins > kSpinLimit) {
                        if (err) atomicOr(err, 8);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                prefix += (uint32_t)st;
                if (flag == kInclusive) break;
                j--;
            }
            __hip_atomic_store(status + tile, kInclusive | (uint32_t)(prefix + tot), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        }
        s_prefix = prefix;
    }
    __syncthreads();
    run += s_prefix;
#pragma unroll
    for (int k = 0; k < kIpt; k++) {
        buf[pad(threadIdx.x * kIpt + k)] = run;
        run += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kIpt; k++) {
        const int idx = k * kBlock + threadIdx.x;
        const int64_t i = base + idx;
        if (i < n) out[i] = buf[pad(idx)];
    }
    if (base + kTile >= n && threadIdx.x == 0) out[n] = s_prefix + tot;
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_fill_i32(int32_t *p, int32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Copies k device words into pinned host memory with system-scope stores, so
// the host sees them once the stream has drained.
__global__ void k_publish(WordSrc src, int k, uint32_t *host) {
    const int t = threadIdx.x;
    if (t < k) __hip_atomic_store(host + t, *src.p[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

int64_t grid_for(int64_t n, int64_t cap = 1 << 20) {
    int64_t b = (n + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    return b < cap ? b : cap;
}

}  // namespace

void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
}

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
}

hipError_t read_words(const WordSrc &src, int k, uint32_t *host, uint32_t *out, hipStream_t s) {
    if (k < 1 || k > WordSrc::kMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, src, k, host);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    for (int i = 0; i < k; i++) out[i] = __atomic_load_n(host + i, __ATOMIC_ACQUIRE);
    return hipSuccess;
}

int64_t scan_tmp_words(int64_t n) {
    // ticket (padded to 8 bytes) and one 64-bit status word per tile
    const int64_t tiles = (n + kTile - 1) / kTile;
    return 2 * (tiles + 1) + 16;
}

void scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s, int32_t *err) {
    int64_t tiles = (n + kTile - 1) / kTile;
    if (tiles < 1) tiles = 1;
    if (tiles == 1) {
        hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kBlock), 0, s, in, out, n, nullptr);
        return;
    }
    // tmp (256-byte aligned): ticket in word 0, status words from word 2
    fill_u32(tmp, 0u, 2 * (tiles + 1), s);
    hipLaunchKernelGGL(k_scan_onepass, dim3((unsigned)tiles), dim3(kBlock), 0, s, in, out, n, tmp,
                       reinterpret_cast<uint64_t *>(tmp + 2), err);
}

}  // namespace hf
