// Kernel density (Sec. 2.2.1): Delta_i = norm * sum_{j != i, r_ij < b} (1 - r_ij^2/b^2),
// norm = 15 / (8 pi b^3 nbar) so that a uniform field has Delta = 1 (App. B.2).
//
// Coordinates are the cell-local FP32 values in units of b; the periodic image
// of a neighbour cell is the exact cell offset, so W = 1 - d^2 is three FMAs on
// (dx, dy, dz) clamped at 0 (which also removes pairs beyond b).  The self pair
// contributes exactly 1 and is subtracted at the end.  Partial sums run over at
// most 64 neighbours in FP32 and are accumulated in FP64, in cell order, so the
// result does not depend on the launch shape.
//
// Dense cells: one wavefront per chunk of <= 64 particles of the cell (one per
// lane), or per pair of small x-adjacent dense cells; the neighbour cells are
// streamed in the same order by all lanes, so neighbour coordinates are
// wave-uniform and come through the scalar cache as SGPR operands of the FP32
// FMAs.  Sparse cells: one thread per particle.
#include "hf_internal.h"

namespace hf {

namespace {

// Accumulate one neighbour cell [a, b) for an i-particle at shifted local
// coordinates (xs, ys, zs).  `a`, `b` are uniform in the dense kernel.
__device__ __forceinline__ void accum_range(const float4 *__restrict__ sloc, uint32_t a, uint32_t b,
                                            float xs, float ys, float zs, double &acc) {
    for (uint32_t j0 = a; j0 < b; j0 += 64) {
        const uint32_t e = min(j0 + 64u, b);
        float p = 0.0f;
        uint32_t j = j0;
        for (; j + 4 <= e; j += 4) {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const float4 lj = sloc[j + u];
                const float dx = lj.x - xs, dy = lj.y - ys, dz = lj.z - zs;
                float t = fmaf(-dx, dx, 1.0f);
                t = fmaf(-dy, dy, t);
                t = fmaf(-dz, dz, t);
                p += fmaxf(t, 0.0f);
            }
        }
        for (; j < e; j++) {
            const float4 lj = sloc[j];
            const float dx = lj.x - xs, dy = lj.y - ys, dz = lj.z - zs;
            float t = fmaf(-dx, dx, 1.0f);
            t = fmaf(-dy, dy, t);
            t = fmaf(-dz, dz, t);
            p += fmaxf(t, 0.0f);
        }
        acc += (double)p;
    }
}

// accum_range for a wave-uniform range: the neighbours are read through a
// pointer with constant offsets so that eight of them arrive in two 64-byte
// scalar loads behind one wait.
__device__ __forceinline__ void accum_range_uniform(const float4 *__restrict__ sloc, uint32_t a, uint32_t b,
                                                    float xs, float ys, float zs, double &acc) {
    for (uint32_t j0 = a; j0 < b; j0 += 64) {
        const float4 *pj = sloc + j0;
        uint32_t m = min(64u, b - j0);
        float p = 0.0f;
        for (; m >= 8; m -= 8, pj += 8) {
#pragma unroll
            for (int u = 0; u < 8; u++) {
                const float4 lj = pj[u];
                const float dx = lj.x - xs, dy = lj.y - ys, dz = lj.z - zs;
                float t = fmaf(-dx, dx, 1.0f);
                t = fmaf(-dy, dy, t);
                t = fmaf(-dz, dz, t);
                p += fmaxf(t, 0.0f);
            }
        }
        for (; m > 0; m--, pj++) {
            const float4 lj = *pj;
            const float dx = lj.x - xs, dy = lj.y - ys, dz = lj.z - zs;
            float t = fmaf(-dx, dx, 1.0f);
            t = fmaf(-dy, dy, t);
            t = fmaf(-dz, dz, t);
            p += fmaxf(t, 0.0f);
        }
        acc += (double)p;
    }
}

// Sum of v over the wavefront in a fixed order, wave-uniform: inclusive sums of
// each 16-lane row by DPP row shifts, then the four row totals in row order.
__device__ __forceinline__ float wave_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x111, 0xf, 0xf, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x112, 0xf, 0xf, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x114, 0xf, 0xf, true));
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x118, 0xf, 0xf, true));
    const int b = __float_as_int(v);
    return ((__int_as_float(__builtin_amdgcn_readlane(b, 15)) + __int_as_float(__builtin_amdgcn_readlane(b, 31))) +
            __int_as_float(__builtin_amdgcn_readlane(b, 47))) +
           __int_as_float(__builtin_amdgcn_readlane(b, 63));
}

// Dense-neighbour contributions of sparse particles are added in fixed point
// (2^-32), so their order does not change the result.
constexpr double kFixScale = 4294967296.0;

__device__ __forceinline__ void write_density(int64_t i, double acc, const Geo &g,
                                              const float4 *__restrict__ spos,
                                              float *__restrict__ dens_s, float *__restrict__ dens_out) {
    const double S = acc - (g.self_count ? 0.0 : 1.0);
    const float d = (float)(g.norm * S);
    dens_s[i] = d;
    if (dens_out) dens_out[orig_of(spos[i])] = d;
}

__global__ __launch_bounds__(kBlock) void k_density_dense(int64_t nchunks, Geo g,
                                                          const int32_t *__restrict__ chunks,
                                                          const float4 *__restrict__ sloc,
                                                          const float4 *__restrict__ spos,
                                                          const uint32_t *__restrict__ off,
                                                          const uint32_t *__restrict__ s_sparse,
                                                          uint64_t *__restrict__ dfx,
                                                          float *__restrict__ dens_s,
                                                          float *__restrict__ dens_out) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t q = (int64_t)xcd_block() * (kBlock / 64) + wave;
    if (q >= nchunks) return;
    const int lane = threadIdx.x & 63;
    const uint32_t h = (uint32_t)__builtin_amdgcn_readfirstlane(chunks[q]);
    const uint32_t c = __builtin_amdgcn_readfirstlane(__float_as_uint(sloc[h].w));
    const uint32_t cend = __builtin_amdgcn_readfirstlane(off[c + 1]);
    const int nc = g.nc;
    const int cx = (int)(c % (uint32_t)nc), cy = (int)((c / (uint32_t)nc) % (uint32_t)nc),
              cz = (int)(c / ((uint32_t)nc * (uint32_t)nc));
    uint32_t end = min(h + 64u, cend);
    // Two x-adjacent cells (even x, and x + 1 in the same row) that are both
    // dense and together hold at most 64 particles share one wavefront: their
    // particles are consecutive, the stream covers x offsets -1..2 from the
    // even cell, and each lane shifts the neighbours by its own cell's offset
    // (a pair outside a lane's 27 cells is at least one cell width apart and
    // weighs exactly 0).  The odd cell's wavefront finds the same pair and exits.
    int xmax = 1;
    // only a cell that is a single chunk pairs (the chunk starts the cell)
    if (cend - h <= 64u && h == (uint32_t)__builtin_amdgcn_readfirstlane(off[c])) {
        const uint32_t mine = cend - h;
        if (cx & 1) {
            const uint32_t left = h - (uint32_t)__builtin_amdgcn_readfirstlane(off[c - 1]);
            if (left >= (uint32_t)kDenseMin && left <= 64u && left + mine <= 64u) return;
        } else if (cx + 1 < nc) {
            const uint32_t e2 = (uint32_t)__builtin_amdgcn_readfirstlane(off[c + 2]);
            const uint32_t right = e2 - cend;
            if (right >= (uint32_t)kDenseMin && right <= 64u && mine + right <= 64u) {
                end = e2;
                xmax = 2;
            }
        }
    }
    const uint32_t i = h + (uint32_t)lane;
    const bool active = i < end;
    const float4 li = sloc[active ? i : h];
    const float du = i >= cend ? 1.0f : 0.0f;  // x offset of the lane's cell in a pair
    double acc = 0.0;
    for (int oz = -1; oz <= 1; oz++) {
        const int z = wrapc(cz + oz, nc);
        const float zs = li.z - (float)oz * g.cellb;
        for (int oy = -1; oy <= 1; oy++) {
            const int y = wrapc(cy + oy, nc);
            const float ys = li.y - (float)oy * g.cellb;
            const uint32_t row = ((uint32_t)z * (uint32_t)nc + (uint32_t)y) * (uint32_t)nc;
            for (int ox = -1; ox <= xmax; ox++) {
                const uint32_t nb = row + (uint32_t)wrapc(cx + ox, nc);
                const float xs = li.x - ((float)ox - du) * g.cellb;
                const uint32_t a = __builtin_amdgcn_readfirstlane(off[nb]);
                const uint32_t b = __builtin_amdgcn_readfirstlane(off[nb + 1]);
                if (b - a >= (uint32_t)kDenseMin) {
                    accum_range_uniform(sloc, a, b, xs, ys, zs, acc);
                    continue;
                }
                // sparse neighbour cell: the pair weights also go to the
                // sparse particle, summed over the chunk in a fixed order
                float p = 0.0f;
                for (uint32_t j = a; j < b; j++) {
                    const float4 lj = sloc[j];
                    const float dx = lj.x - xs, dy = lj.y - ys, dz = lj.z - zs;
                    float t = fmaf(-dx, dx, 1.0f);
                    t = fmaf(-dy, dy, t);
                    t = fmaf(-dz, dz, t);
                    t = active ? fmaxf(t, 0.0f) : 0.0f;
                    p += t;
                    const float sum = wave_sum(t);
                    if (lane == 0 && sum > 0.0f)
                        atomicAdd(reinterpret_cast<unsigned long long *>(&dfx[s_sparse[j]]),
                                  (unsigned long long)__double2ll_rn((double)sum * kFixScale));
                }
                acc += (double)p;
            }
        }
    }
    if (active) write_density(i, acc, g, spos, dens_s, dens_out);
}

// Sparse cells: one particle per lane, sparse neighbour cells only; the pairs
// with dense neighbour cells were summed by the dense kernel into dfx.
__global__ __launch_bounds__(kBlock) void k_density_sparse(int64_t nsparse, Geo g,
                                                           const int32_t *__restrict__ sparse,
                                                           const float4 *__restrict__ sloc,
                                                           const float4 *__restrict__ spos,
                                                           const uint32_t *__restrict__ off,
                                                           const uint64_t *__restrict__ dfx,
                                                           float *__restrict__ dens_s,
                                                           float *__restrict__ dens_out) {
    const int64_t t = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    if (t >= nsparse) return;
    const int64_t i = sparse[t];
    const float4 li = sloc[i];
    const uint32_t c = __float_as_uint(li.w);
    const int nc = g.nc;
    const int cx = (int)(c % (uint32_t)nc), cy = (int)((c / (uint32_t)nc) % (uint32_t)nc),
              cz = (int)(c / ((uint32_t)nc * (uint32_t)nc));
    const uint32_t x0 = (uint32_t)wrapc(cx - 1, nc), x1 = (uint32_t)cx, x2 = (uint32_t)wrapc(cx + 1, nc);
    // away from the periodic x edges the three cells of a stencil row are
    // consecutive: their four bounding offsets are one 16-byte load
    const bool inner = cx > 0 && cx < nc - 1;
    double acc = 0.0;
    for (int oz = -1; oz <= 1; oz++) {
        const int z = wrapc(cz + oz, nc);
        const float zs = li.z - (float)oz * g.cellb;
        // the offsets of this plane are loaded together so their latencies overlap
        uint32_t ra[9], rb[9];
#pragma unroll
        for (int oy = -1; oy <= 1; oy++) {
            const uint32_t row = ((uint32_t)z * (uint32_t)nc + (uint32_t)wrapc(cy + oy, nc)) * (uint32_t)nc;
            const int r = (oy + 1) * 3;
            if (inner) {
                const uint32_t *p = off + row + x0;
                const uint32_t o0 = p[0], o1 = p[1], o2 = p[2], o3 = p[3];
                ra[r + 0] = o0;
                rb[r + 0] = o1;
                ra[r + 1] = o1;
                rb[r + 1] = o2;
                ra[r + 2] = o2;
                rb[r + 2] = o3;
            } else {
                ra[r + 0] = off[row + x0];
                rb[r + 0] = off[row + x0 + 1];
                ra[r + 1] = off[row + x1];
                rb[r + 1] = off[row + x1 + 1];
                ra[r + 2] = off[row + x2];
                rb[r + 2] = off[row + x2 + 1];
            }
        }
#pragma unroll
        for (int oy = -1; oy <= 1; oy++) {
            const float ys = li.y - (float)oy * g.cellb;
#pragma unroll
            for (int ox = -1; ox <= 1; ox++) {
                const int r = (oy + 1) * 3 + (ox + 1);
                if (rb[r] - ra[r] >= (uint32_t)kDenseMin) continue;
                const float xs = li.x - (float)ox * g.cellb;
                accum_range(sloc, ra[r], rb[r], xs, ys, zs, acc);
            }
        }
    }
    acc += (double)dfx[t] * (1.0 / kFixScale);
    write_density(i, acc, g, spos, dens_s, dens_out);
}

// Number of ordered pairs (i, j != i) closer than b, for the roofline's
// algorithmic pair count (evaluated in the same FP32 local coordinates).
__global__ __launch_bounds__(kBlock) void k_count_pairs(int64_t n, Geo g,
                                                        const float4 *__restrict__ sloc,
                                                        const uint32_t *__restrict__ off,
                                                        unsigned long long *__restrict__ total) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t cnt = 0;
    if (i < n) {
        const float4 li = sloc[i];
        const uint32_t c = __float_as_uint(li.w);
        const int nc = g.nc;
        const int cx = (int)(c % (uint32_t)nc), cy = (int)((c / (uint32_t)nc) % (uint32_t)nc),
                  cz = (int)(c / ((uint32_t)nc * (uint32_t)nc));
        for (int oz = -1; oz <= 1; oz++)
            for (int oy = -1; oy <= 1; oy++)
                for (int ox = -1; ox <= 1; ox++) {
                    const uint32_t nb = ((uint32_t)wrapc(cz + oz, nc) * (uint32_t)nc +
                                         (uint32_t)wrapc(cy + oy, nc)) * (uint32_t)nc +
                                        (uint32_t)wrapc(cx + ox, nc);
                    const float xs = li.x - (float)ox * g.cellb, ys = li.y - (float)oy * g.cellb,
                                zs = li.z - (float)oz * g.cellb;
                    for (uint32_t j = off[nb]; j < off[nb + 1]; j++) {
                        const float4 lj = sloc[j];
                        const float dx = lj.x - xs, dy = lj.y - ys, dz = lj.z - zs;
                        cnt += (dx * dx + dy * dy + dz * dz < 1.0f) ? 1u : 0u;
                    }
                }
        cnt -= 1;  // the particle itself
    }
    for (int d = 32; d >= 1; d >>= 1) cnt += __shfl_xor(cnt, d, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(total, (unsigned long long)cnt);
}

__global__ __launch_bounds__(kBlock) void k_gather_density(int64_t n, const float4 *__restrict__ spos,
                                                           const float *__restrict__ dens_in,
                                                           float *__restrict__ dens_s) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    dens_s[i] = dens_in[orig_of(spos[i])];
}

}  // namespace

void launch_density(int64_t n, const Geo &g, Work &w, float *dens_out, hipStream_t s) {
    // dfx: dense-neighbour sums of the sparse particles (fixed point), in the
    // radix key array that binning no longer needs
    uint64_t *dfx = w.rkey[0];
    if (w.nsparse > 0) fill_u32(reinterpret_cast<uint32_t *>(dfx), 0u, 2 * w.nsparse, s);
    if (w.nchunks > 0)
        hipLaunchKernelGGL(k_density_dense, dim3((unsigned)((w.nchunks + 3) / 4)), dim3(kBlock), 0, s,
                           w.nchunks, g, w.chunks, w.sloc, w.spos, w.off, w.s_sparse, dfx, w.dens_s,
                           dens_out);
    if (w.nsparse > 0)
        hipLaunchKernelGGL(k_density_sparse, dim3((unsigned)((w.nsparse + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, s, w.nsparse, g, w.sparse, w.sloc, w.spos, w.off, dfx, w.dens_s,
                           dens_out);
}

void launch_count_pairs(int64_t n, const Geo &g, Work &w, unsigned long long *total, hipStream_t s) {
    hipLaunchKernelGGL(k_count_pairs, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, g, w.sloc,
                       w.off, total);
}

void launch_gather_density(const float *dens_in, int64_t n, Work &w, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_density, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n,
                       w.spos, dens_in, w.dens_s);
}

}  // namespace hf
