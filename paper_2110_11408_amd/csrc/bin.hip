// Cell binning: a stable counting sort of the particles by (cell, sub-cell).
//
// The paper's host code receives particles already ordered by cell from the
// N-body engine (Sec. 2.3.4); here the caller hands over an unordered float32
// [n][3] array, so the library builds the order itself:
//   1. cell key, sub-cell index and an atomic ticket inside the cell (counts);
//   2. exclusive scan of the per-cell counts (cell offsets);
//   3. scatter of (sub-cell, original index) to offset + ticket (unstable);
//   4. stable rank inside the cell by (sub-cell, original index), and the final
//      write of two float4 streams per particle:
//        spos = (x, y, z, original index bits)    -- the paper's float quad with
//               the index stored bitwise (Sec. 2.3.3), used by FP64 predicates;
//        sloc = (x, y, z relative to the cell corner, in units of b; cell id
//               bits) -- FP32 coordinates whose differences across a periodic
//               face stay exact, used by the density loop and prefilters.
// Cells are at least max(b, l) wide; each is split into k^3 sub-cells whose
// diagonal is below l, so all particles of one sub-cell are friends.
//
// Work decomposition shared by the neighbour-loop kernels: a cell holding at
// least kDenseMin particles is "dense".  Dense cells get a table of their
// sub-cell offsets and are cut into chunks of at most 64 consecutive particles
// (one wavefront each); particles of the other cells form the "sparse" list
// (one thread each).  The in-cell order, and therefore every summation order,
// is fixed by the data, never by thread scheduling.
#include "hf_internal.h"

namespace hf {

namespace {

inline int64_t blocks(int64_t n) { return (n + kBlock - 1) / kBlock; }

__device__ __forceinline__ int cell_coord(float x, const Geo &g) {
    int c = (int)floor((double)x * g.inv_cell);
    return c < 0 ? 0 : (c >= g.nc ? g.nc - 1 : c);
}

__device__ __forceinline__ int sub_coord(float x, int c, const Geo &g) {
    int s = (int)floor(((double)x - (double)c * g.cell) * g.inv_sub);
    return s < 0 ? 0 : (s >= g.ksub ? g.ksub - 1 : s);
}

__global__ __launch_bounds__(kBlock) void k_bin_key(const float *__restrict__ pos, int64_t n, Geo g,
                                                    uint32_t *__restrict__ key,
                                                    uint32_t *__restrict__ ticket,
                                                    uint16_t *__restrict__ subk,
                                                    uint32_t *__restrict__ cnt,
                                                    int32_t *__restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x = pos[3 * i + 0], y = pos[3 * i + 1], z = pos[3 * i + 2];
    float Lf = (float)g.L;
    bool ok = x >= 0.0f && x < Lf && y >= 0.0f && y < Lf && z >= 0.0f && z < Lf;
    if (!ok) atomicOr(err, 1);
    int cx = cell_coord(x, g), cy = cell_coord(y, g), cz = cell_coord(z, g);
    uint32_t c = ((uint32_t)cz * (uint32_t)g.nc + (uint32_t)cy) * (uint32_t)g.nc + (uint32_t)cx;
    int k = g.ksub;
    key[i] = c;
    subk[i] = (uint16_t)((sub_coord(z, cz, g) * k + sub_coord(y, cy, g)) * k + sub_coord(x, cx, g));
    ticket[i] = atomicAdd(&cnt[c], 1u);
}

__global__ __launch_bounds__(kBlock) void k_bin_scatter(int64_t n, const uint32_t *__restrict__ key,
                                                        const uint32_t *__restrict__ ticket,
                                                        const uint16_t *__restrict__ subk,
                                                        const uint32_t *__restrict__ off,
                                                        uint64_t *__restrict__ tmp) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    tmp[off[key[i]] + ticket[i]] = ((uint64_t)subk[i] << 32) | (uint64_t)i;
}

__global__ __launch_bounds__(kBlock) void k_bin_stable(const float *__restrict__ pos, int64_t n, Geo g,
                                                       const uint32_t *__restrict__ key,
                                                       const uint32_t *__restrict__ off,
                                                       const uint64_t *__restrict__ tmp,
                                                       float4 *__restrict__ spos,
                                                       float4 *__restrict__ sloc,
                                                       uint16_t *__restrict__ ssub) {
    int64_t s = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const uint64_t me = tmp[s];
    const uint32_t o = (uint32_t)me;
    const uint32_t c = key[o];
    const uint32_t a = off[c], b = off[c + 1];
    uint32_t rank = 0;
    // a wavefront whose slots all lie in one cell streams that cell once
    // (wave-uniform loads); otherwise every lane walks its own cell
    const uint32_t c0 = __builtin_amdgcn_readfirstlane(c);
    if (__ballot(c != c0) == 0ull && s - (threadIdx.x & 63) + 63 < n) {
        const uint32_t ua = __builtin_amdgcn_readfirstlane(a), ub = __builtin_amdgcn_readfirstlane(b);
        for (uint32_t t = ua; t < ub; t++) rank += tmp[t] < me ? 1u : 0u;
    } else {
        for (uint32_t t = a; t < b; t++) rank += tmp[t] < me ? 1u : 0u;
    }
    const uint32_t d = a + rank;
    float x = pos[3 * (int64_t)o + 0], y = pos[3 * (int64_t)o + 1], z = pos[3 * (int64_t)o + 2];
    spos[d] = make_float4(x, y, z, __uint_as_float(o));
    uint32_t nc = (uint32_t)g.nc;
    uint32_t cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
    float xl = (float)(((double)x - (double)cx * g.cell) * g.inv_b);
    float yl = (float)(((double)y - (double)cy * g.cell) * g.inv_b);
    float zl = (float)(((double)z - (double)cz * g.cell) * g.inv_b);
    sloc[d] = make_float4(xl, yl, zl, __uint_as_float(c));
    ssub[d] = (uint16_t)(me >> 32);
}

// Flags per sorted particle: head of a dense chunk, head of a dense cell, sparse.
__global__ __launch_bounds__(kBlock) void k_bin_flags(int64_t n, const float4 *__restrict__ sloc,
                                                      const uint32_t *__restrict__ off,
                                                      uint32_t *__restrict__ f_chunk,
                                                      uint32_t *__restrict__ f_dcell,
                                                      uint32_t *__restrict__ f_sparse) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = __float_as_uint(sloc[i].w);
    const uint32_t a = off[c], b = off[c + 1];
    const bool dense = b - a >= (uint32_t)kDenseMin;
    f_chunk[i] = dense && (((uint32_t)i - a) % 64u == 0u);
    f_dcell[i] = dense && (uint32_t)i == a;
    f_sparse[i] = !dense;
}

__global__ __launch_bounds__(kBlock) void k_bin_lists(int64_t n, const uint32_t *__restrict__ f_chunk,
                                                      const uint32_t *__restrict__ s_chunk,
                                                      const uint32_t *__restrict__ f_dcell,
                                                      const uint32_t *__restrict__ s_dcell,
                                                      const uint32_t *__restrict__ f_sparse,
                                                      const uint32_t *__restrict__ s_sparse,
                                                      const float4 *__restrict__ sloc,
                                                      int32_t *__restrict__ chunks,
                                                      uint32_t *__restrict__ dcells,
                                                      int32_t *__restrict__ sparse,
                                                      uint32_t *__restrict__ cellmap) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (f_chunk[i]) chunks[s_chunk[i]] = (int32_t)i;
    if (f_sparse[i]) sparse[s_sparse[i]] = (int32_t)i;
    if (f_dcell[i]) {
        const uint32_t c = __float_as_uint(sloc[i].w);
        const uint32_t d = s_dcell[i];
        dcells[d] = c;
        cellmap[c] = d;  // the cell-count array is reused as cell -> dense-cell map
    }
}

// Sub-cell offsets of every dense cell: entry s is the first particle of
// sub-cell s (the next non-empty one for empty sub-cells), entry k^3 the cell end.
__global__ __launch_bounds__(kBlock) void k_sub_init(int64_t ndc, int nsub,
                                                     const uint32_t *__restrict__ dcells,
                                                     const uint32_t *__restrict__ off,
                                                     uint32_t *__restrict__ subtab) {
    int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= ndc) return;
    const uint32_t end = off[dcells[d] + 1];
    for (int s = 0; s <= nsub; s++) subtab[d * (nsub + 1) + s] = end;
}

__global__ __launch_bounds__(kBlock) void k_sub_starts(int64_t n, int nsub,
                                                       const float4 *__restrict__ sloc,
                                                       const uint32_t *__restrict__ off,
                                                       const uint16_t *__restrict__ ssub,
                                                       const uint32_t *__restrict__ cellmap,
                                                       uint32_t *__restrict__ subtab) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t c = __float_as_uint(sloc[i].w);
    const uint32_t a = off[c], b = off[c + 1];
    if (b - a < (uint32_t)kDenseMin) return;
    const uint16_t s = ssub[i];
    if ((uint32_t)i == a || ssub[i - 1] != s) subtab[(int64_t)cellmap[c] * (nsub + 1) + s] = (uint32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_sub_fix(int64_t ndc, int nsub, uint32_t *__restrict__ subtab) {
    int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= ndc) return;
    uint32_t *t = subtab + d * (nsub + 1);
    for (int s = nsub - 1; s >= 0; s--)
        if (t[s] > t[s + 1]) t[s] = t[s + 1];
}

}  // namespace

void launch_bin(const float *pos, int64_t n, const Geo &g, Work &w, hipStream_t s) {
    int64_t ncell = (int64_t)g.nc * g.nc * g.nc;
    fill_u32(w.cnt, 0u, ncell, s);
    hipLaunchKernelGGL(k_bin_key, dim3(blocks(n)), dim3(kBlock), 0, s, pos, n, g, w.key, w.ticket,
                       w.subk, w.cnt, w.err);
    scan_u32(w.cnt, w.off, ncell, w.scan_tmp, s);
    hipLaunchKernelGGL(k_bin_scatter, dim3(blocks(n)), dim3(kBlock), 0, s, n, w.key, w.ticket, w.subk,
                       w.off, w.tmp);
    hipLaunchKernelGGL(k_bin_stable, dim3(blocks(n)), dim3(kBlock), 0, s, pos, n, g, w.key, w.off,
                       w.tmp, w.spos, w.sloc, w.ssub);
    hipLaunchKernelGGL(k_bin_flags, dim3(blocks(n)), dim3(kBlock), 0, s, n, w.sloc, w.off, w.f_chunk,
                       w.f_dcell, w.f_sparse);
    scan_u32(w.f_chunk, w.s_chunk, n, w.scan_tmp, s);
    scan_u32(w.f_dcell, w.s_dcell, n, w.scan_tmp, s);
    scan_u32(w.f_sparse, w.s_sparse, n, w.scan_tmp, s);
    hipLaunchKernelGGL(k_bin_lists, dim3(blocks(n)), dim3(kBlock), 0, s, n, w.f_chunk, w.s_chunk,
                       w.f_dcell, w.s_dcell, w.f_sparse, w.s_sparse, w.sloc, w.chunks, w.dcells,
                       w.sparse, w.cnt);
}

void launch_subtab(int64_t n, int64_t ndc, const Geo &g, Work &w, hipStream_t s) {
    if (ndc <= 0) return;
    const int nsub = g.ksub * g.ksub * g.ksub;
    hipLaunchKernelGGL(k_sub_init, dim3(blocks(ndc)), dim3(kBlock), 0, s, ndc, nsub, w.dcells, w.off,
                       w.subtab);
    hipLaunchKernelGGL(k_sub_starts, dim3(blocks(n)), dim3(kBlock), 0, s, n, nsub, w.sloc, w.off, w.ssub,
                       w.cnt, w.subtab);
    hipLaunchKernelGGL(k_sub_fix, dim3(blocks(ndc)), dim3(kBlock), 0, s, ndc, nsub, w.subtab);
}

}  // namespace hf
