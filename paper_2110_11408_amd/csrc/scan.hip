// Device-wide exclusive prefix sum of uint32 arrays and fill kernels.
//
// Three passes per level: tile sums (coalesced reads), a recursive scan of the
// tile sums, and a tile scan staged through LDS that adds each tile's offset.
// (A single pass with decoupled look-back was slower here: on this chip the
// chain of status words between thousands of tiles goes through memory that
// every XCD must see, a few microseconds per link.)
// Tiles are 256 threads x 16 items; LDS indices are padded by one word per 32
// to keep the per-thread runs of 16 words off a single bank.
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

// Full tiles are moved as 16-byte vectors (in and out are 16-byte aligned:
// arena arrays, and the tile-sum arrays below are padded to four words); the
// last, partial tile word by word.
// kNz: scan the indicator in[i] != 0 instead of the values.
template <bool kNz>
__device__ __forceinline__ uint32_t val(uint32_t x) { return kNz ? (x != 0u ? 1u : 0u) : x; }

template <bool kNz>
__global__ __launch_bounds__(kBlock) void k_tile_sums(const uint32_t *__restrict__ in, int64_t n,
                                                      uint32_t *__restrict__ sums) {
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t s = 0;
    if (base + kTile <= n) {
        const uint4 *p = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
        for (int k = 0; k < kIpt / 4; k++) {
            const uint4 v = p[k * kBlock + threadIdx.x];
            s += (val<kNz>(v.x) + val<kNz>(v.y)) + (val<kNz>(v.z) + val<kNz>(v.w));
        }
    } else {
#pragma unroll
        for (int k = 0; k < kIpt; k++) {
            const int64_t i = base + k * kBlock + threadIdx.x;
            if (i < n) s += val<kNz>(in[i]);
        }
    }
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <bool kNz>
__global__ __launch_bounds__(kBlock) void k_tile_scan(const uint32_t *__restrict__ in,
                                                      uint32_t *__restrict__ out, int64_t n,
                                                      const uint32_t *__restrict__ tile_off) {
    __shared__ uint32_t buf[kTile + kTile / 32];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    const bool full = base + kTile <= n;
    if (full) {
        const uint4 *p = reinterpret_cast<const uint4 *>(in + base);
#pragma unroll
        for (int k = 0; k < kIpt / 4; k++) {
            const int q = k * kBlock + threadIdx.x;
            const uint4 v = p[q];
            buf[pad(4 * q + 0)] = val<kNz>(v.x);
            buf[pad(4 * q + 1)] = val<kNz>(v.y);
            buf[pad(4 * q + 2)] = val<kNz>(v.z);
            buf[pad(4 * q + 3)] = val<kNz>(v.w);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kIpt; k++) {
            const int idx = k * kBlock + threadIdx.x;
            const int64_t i = base + idx;
            buf[pad(idx)] = i < n ? val<kNz>(in[i]) : 0u;
        }
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
    const uint32_t toff = tile_off ? tile_off[blockIdx.x] : 0u;
    run += toff;
#pragma unroll
    for (int k = 0; k < kIpt; k++) {
        buf[pad(threadIdx.x * kIpt + k)] = run;
        run += v[k];
    }
    __syncthreads();
    if (full) {
        uint4 *p = reinterpret_cast<uint4 *>(out + base);
#pragma unroll
        for (int k = 0; k < kIpt / 4; k++) {
            const int q = k * kBlock + threadIdx.x;
            p[q] = make_uint4(buf[pad(4 * q + 0)], buf[pad(4 * q + 1)], buf[pad(4 * q + 2)], buf[pad(4 * q + 3)]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < kIpt; k++) {
            const int idx = k * kBlock + threadIdx.x;
            const int64_t i = base + idx;
            if (i < n) out[i] = buf[pad(idx)];
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = toff + tot;
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// 16-byte stores for a 16-byte-aligned array of n4 words x4, then the tail.
__global__ __launch_bounds__(kBlock) void k_fill_u32x4(uint4 *p, uint32_t v, int64_t n4, uint32_t *tail,
                                                       int ntail) {
    const uint4 q = make_uint4(v, v, v, v);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = q;
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = v;
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
    if ((reinterpret_cast<uintptr_t>(p) & 15u) == 0 && n >= 1024) {
        const int64_t n4 = n / 4;
        hipLaunchKernelGGL(k_fill_u32x4, dim3(grid_for(n4)), dim3(kBlock), 0, s, reinterpret_cast<uint4 *>(p), v, n4,
                           p + 4 * n4, (int)(n - 4 * n4));
        return;
    }
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
}

void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s) {
    fill_u32(reinterpret_cast<uint32_t *>(p), (uint32_t)v, n, s);
}

hipError_t publish_words(const WordSrc &src, int k, uint32_t *host, hipStream_t s) {
    if (k < 1 || k > WordSrc::kMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, src, k, host);
    return hipGetLastError();
}

void collect_words(const uint32_t *host, int k, uint32_t *out) {
    for (int i = 0; i < k; i++) out[i] = __atomic_load_n(host + i, __ATOMIC_ACQUIRE);
}

hipError_t read_words(const WordSrc &src, int k, uint32_t *host, uint32_t *out, hipStream_t s) {
    hipError_t e = publish_words(src, k, host, s);
    if (e != hipSuccess) return e;
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    collect_words(host, k, out);
    return hipSuccess;
}

// Words of one tile-sum array (tiles + 1), rounded up to keep 16-byte alignment.
static int64_t sums_words(int64_t tiles) { return (tiles + 1 + 3) & ~(int64_t)3; }

int64_t scan_tmp_words(int64_t n) {
    int64_t w = 0;
    while (n > kTile) {
        int64_t t = (n + kTile - 1) / kTile;
        w += 2 * sums_words(t);
        n = t;
    }
    return w + 16;
}

template <bool kNz>
void scan_impl(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s) {
    int64_t tiles = (n + kTile - 1) / kTile;
    if (tiles < 1) tiles = 1;
    if (tiles == 1) {
        hipLaunchKernelGGL(k_tile_scan<kNz>, dim3(1), dim3(kBlock), 0, s, in, out, n, nullptr);
        return;
    }
    uint32_t *sums = tmp;
    uint32_t *sums_scan = tmp + sums_words(tiles);
    hipLaunchKernelGGL(k_tile_sums<kNz>, dim3(tiles), dim3(kBlock), 0, s, in, n, sums);
    scan_impl<false>(sums, sums_scan, tiles, tmp + 2 * sums_words(tiles), s);
    hipLaunchKernelGGL(k_tile_scan<kNz>, dim3(tiles), dim3(kBlock), 0, s, in, out, n, sums_scan);
}

void scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s) {
    scan_impl<false>(in, out, n, tmp, s);
}

void scan_nz_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s) {
    scan_impl<true>(in, out, n, tmp, s);
}

}  // namespace hf
