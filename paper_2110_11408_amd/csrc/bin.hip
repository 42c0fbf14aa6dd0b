// Cell binning: a stable counting sort of the particles by cell.
//
// The paper's host code receives particles already ordered by cell from the
// N-body engine (Sec. 2.3.4); here the caller hands over an unordered float32
// [n][3] array, so the library builds the order itself:
//   1. cell key per particle and an atomic ticket inside its cell (counts);
//   2. exclusive scan of the per-cell counts (cell offsets);
//   3. scatter of the particle index to offset + ticket (unstable);
//   4. stable rank inside the cell (number of smaller original indices in the
//      same cell), and the final write of two float4 streams per particle:
//        spos = (x, y, z, original index bits)    -- the paper's float quad with
//               the index stored bitwise (Sec. 2.3.3), used by FP64 predicates;
//        sloc = (x, y, z relative to the cell corner, in units of b; cell id
//               bits) -- FP32 coordinates whose differences across a periodic
//               face stay exact, used by the density loop and prefilters.
// The in-cell order is the original index order, so every later summation
// order is independent of thread scheduling.
#include "hf_internal.h"

namespace hf {

namespace {

__device__ __forceinline__ int cell_coord(float x, const Geo &g) {
    int c = (int)floor((double)x * g.inv_cell);
    return c < 0 ? 0 : (c >= g.nc ? g.nc - 1 : c);
}

__global__ __launch_bounds__(kBlock) void k_bin_key(const float *__restrict__ pos, int64_t n, Geo g,
                                                    uint32_t *__restrict__ key,
                                                    uint32_t *__restrict__ ticket,
                                                    uint32_t *__restrict__ cnt,
                                                    int32_t *__restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x = pos[3 * i + 0], y = pos[3 * i + 1], z = pos[3 * i + 2];
    float Lf = (float)g.L;
    bool ok = x >= 0.0f && x < Lf && y >= 0.0f && y < Lf && z >= 0.0f && z < Lf;
    if (!ok) atomicOr(err, 1);
    uint32_t c = ((uint32_t)cell_coord(z, g) * (uint32_t)g.nc + (uint32_t)cell_coord(y, g)) *
                     (uint32_t)g.nc + (uint32_t)cell_coord(x, g);
    key[i] = c;
    ticket[i] = atomicAdd(&cnt[c], 1u);
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(int64_t n, const uint32_t *__restrict__ key,
                                                        const uint32_t *__restrict__ ticket,
                                                        const uint32_t *__restrict__ off,
                                                        uint32_t *__restrict__ tmp) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    tmp[off[key[i]] + ticket[i]] = (uint32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_bin_stable(const float *__restrict__ pos, int64_t n, Geo g,
                                                       const uint32_t *__restrict__ key,
                                                       const uint32_t *__restrict__ off,
                                                       const uint32_t *__restrict__ tmp,
                                                       float4 *__restrict__ spos,
                                                       float4 *__restrict__ sloc) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    uint32_t o = tmp[s];
    uint32_t c = key[o];
    uint32_t a = off[c], b = off[c + 1];
    uint32_t rank = 0;
    for (uint32_t t = a; t < b; t++) rank += tmp[t] < o ? 1u : 0u;
    uint32_t d = a + rank;
    float x = pos[3 * (int64_t)o + 0], y = pos[3 * (int64_t)o + 1], z = pos[3 * (int64_t)o + 2];
    spos[d] = make_float4(x, y, z, __uint_as_float(o));
    uint32_t nc = (uint32_t)g.nc;
    uint32_t cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
    float xl = (float)(((double)x - (double)cx * g.cell) * g.inv_b);
    float yl = (float)(((double)y - (double)cy * g.cell) * g.inv_b);
    float zl = (float)(((double)z - (double)cz * g.cell) * g.inv_b);
    sloc[d] = make_float4(xl, yl, zl, __uint_as_float(c));
}

inline int64_t blocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

}  // namespace

void launch_bin(const float *pos, int64_t n, const Geo &g, Work &w, hipStream_t s) {
    int64_t ncell = (int64_t)g.nc * g.nc * g.nc;
    fill_u32(w.cnt, 0u, ncell, s);
    hipLaunchKernelGGL(k_bin_key, dim3(blocks(n)), dim3(kBlock), 0, s, pos, n, g, w.key, w.ticket,
                       w.cnt, w.err);
    scan_u32(w.cnt, w.off, ncell, w.scan_tmp, s);
    hipLaunchKernelGGL(k_bin_scatter, dim3(blocks(n)), dim3(kBlock), 0, s, n, w.key, w.ticket,
                       w.off, w.tmp);
    hipLaunchKernelGGL(k_bin_stable, dim3(blocks(n)), dim3(kBlock), 0, s, pos, n, g, w.key, w.off,
                       w.tmp, w.spos, w.sloc);
}

}  // namespace hf
