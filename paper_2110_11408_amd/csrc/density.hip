// Kernel density (Sec. 2.2.1): Delta_i = norm * sum_{j != i, r_ij < b} (1 - r_ij^2/b^2),
// norm = 15 / (8 pi b^3 nbar) so that a uniform field has Delta = 1 (App. B.2).
//
// Coordinates are the cell-local FP32 values in units of b; the periodic image
// of a neighbour cell is the exact cell offset, so a pair's weight is
// 1 - d^2 clamped at 0 (which also removes pairs beyond b).
//
// Dense cells (>= 8 particles): one wavefront per chunk of <= 64 consecutive
// particles of the cell.  The weights of 16 i-particles against 16 neighbours
// come from one FP32 matrix-core product (the squared distance expanded into
// a rank-4 inner product), so the vector ALU only clamps and sums; blocks of
// 16 lanes that hold no particle are skipped, and the few particles of the
// sparse neighbour cells are packed 16 to a block.  The self pair is masked out and
// added back as exactly 1 when it counts.  Partial sums run in FP32 over
// bounded stretches and are accumulated in FP64 in a fixed order, so the
// result does not depend on the launch shape.
//
// Particles of sparse cells have few neighbours, often near r = b where the
// weights are small, so the tolerance of their density is only about 1e-6 in
// the weight sum: the density of a sparse-cell particle is a sum of FP64
// weights from the original float positions (1 - d^2/b^2, the periodic image
// of a neighbour cell taken once per cell), by one thread per sparse particle
// for its sparse neighbour cells, and by the dense chunks for the sparse
// particles around them (one lane per sparse particle, summing over the
// chunk's particles, added in fixed point).  The
// rank-4 form has terms up to about 6 in magnitude, so its weights are only
// good to a few 1e-7 each; that suffices for dense-cell particles, whose sums
// have many terms.
#include <stdlib.h>

#include "hf_internal.h"

namespace hf {

namespace {

// FP64 position of particle p as seen from a particle whose neighbour cell it
// is through stencil offset (ox, oy, oz) from cell (cx, cy, cz): the periodic
// image across a box face is taken by adding or subtracting L once per cell
// (a stencil cell that wraps), so no pair needs a minimum-image fold.  Where
// a weight is nonzero (r < b <= the cell side < L/2) this is the minimum
// image.
struct Pos64 {
    double x, y, z;
};
__device__ __forceinline__ double image_shift(int c, int o, int nc, double L) {
    return c + o < 0 ? -L : (c + o >= nc ? L : 0.0);
}

// Weight 1 - d^2/b^2 (0 beyond b) of the pair (a, q) in FP64, with q a float
// position and a an FP64 position in q's frame.
__device__ __forceinline__ double weight64(const Pos64 &a, const float4 &q, double inv_b2) {
    const double dx = (double)q.x - a.x, dy = (double)q.y - a.y, dz = (double)q.z - a.z;
    const double t = 1.0 - (dx * dx + dy * dy + dz * dz) * inv_b2;
    return fmax(t, 0.0);
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

typedef float f32x4 __attribute__((ext_vector_type(4)));

// max(x, 0) for a finite float as one integer maximum: negative values (and
// -0) have the sign bit set.
__device__ __forceinline__ float clamp0(float x) { return __int_as_float(max(__float_as_int(x), 0)); }

// Dense chunk with R = ceil(active lanes / 16) row blocks of 16 i-particles.
//
// pq holds per sorted particle the cell-centred coordinates x_c (units of b)
// and -|x_c|^2.  For a neighbour cell at image offset s (a multiple of the
// cell width) the pair weight before clamping is
//   1 - |x_i - s - x_j|^2 = (1 - |x_i - s|^2) + 2 (x_i - s).x_j - |x_j|^2,
// a rank-4 product: one v_mfma_f32_16x16x4_f32 per 16x16 block of pairs with
// A = (2 (x_i - s), 1), B = (x_j, -|x_j|^2) straight from pq and the
// accumulator input 1 - |x_i - s|^2, itself one product per cell
// ((2 x_i, 1) against (s, -|s|^2) added to 1 - |x_i|^2).  The vector ALU only
// clamps and sums.  For the pairs that count every term is below about 4 in
// magnitude, so a weight is within a few 1e-7 of the difference form.
//
// Layouts of the 16x16x4 FP32 instruction (one block): lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; result register v of lane l is
// D[4 (l / 16) + v][l % 16].  Lane l therefore sums, for the rows
// 16 r + 4 (l / 16) + v, the neighbours in column l % 16; the 16 lanes of a
// row group are reduced at the end.  The neighbours of dense cells stream in
// blocks of 16 consecutive sorted particles per cell; a column past the cell's
// end gets B = (., ., ., -1e30) and weighs 0 (pq is padded so that the load
// stays in bounds).  The particles of the sparse neighbour cells (fewer than
// 8 each) share blocks instead, with the shift on their side.
template <int R, bool kNarrow>
__device__ __forceinline__ void density_chunk(const Geo &g, uint32_t h, uint32_t c, uint32_t end,
                                              const float *__restrict__ pq,
                                              const float4 *__restrict__ spos,
                                              const uint32_t *__restrict__ off,
                                              const uint32_t *__restrict__ s_sparse,
                                              uint64_t *__restrict__ dfx, float *__restrict__ dens_s,
                                              float *__restrict__ dens_out, float *__restrict__ cl,
                                              float4 *__restrict__ s_pk) {
    const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
    const int loff = 4 * col + grp;  // this lane's word of a block of 16 pq records
    // this lane's word of the block of 16 records from j0, as a buffer load
    // (scalar address arithmetic only; the lane offset is a constant VGPR):
    // one descriptor at pq with the block's byte offset in an SGPR while the
    // offsets fit in 32 bits, else a descriptor at the block itself
    const __amdgpu_buffer_rsrc_t rs0 =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(pq), 0, (int)0xffffffffu, 0x00020000);
    auto ld = [&](uint32_t j0) -> float {
        if (kNarrow)
            return __builtin_bit_cast(float,
                                      __builtin_amdgcn_raw_buffer_load_b32(rs0, loff * 4, (int)(j0 * 16u), 0));
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float *>(pq + 4 * (size_t)j0), 0, 256, 0x00020000);
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, loff * 4, 0, 0));
    };
    int cx, cy, cz;
    cell_xyz(g, c, cx, cy, cz);
    // the chunk's rows: A = (2 x_i, 1), accumulator input 1 - |x_i|^2; rows
    // past the chunk get A = (0, 0, 0, 1) and -1, so all their weights clamp
    // to exactly 0
    float A[R];
    // the accumulator inputs 1 - |x_i|^2 stay in LDS (read once per stencil
    // cell), which keeps the kernel at six wavefronts per SIMD
    auto Cget = [&](int r) -> f32x4 {
        f32x4 v;
#pragma unroll
        for (int u = 0; u < 4; u++) v[u] = cl[(4 * r + u) * 64 + lane];
        return v;
    };
#pragma unroll
    for (int r = 0; r < R; r++) {
        const uint32_t ir = h + 16u * (uint32_t)r + (uint32_t)col;
        const float v = pq[4 * (size_t)min(ir, end - 1u) + grp];
        A[r] = grp == 3 ? 1.0f : (ir < end ? v + v : 0.0f);
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const uint32_t iu = h + 16u * (uint32_t)r + 4u * (uint32_t)grp + (uint32_t)u;
            const float q = pq[4 * (size_t)min(iu, end - 1u) + 3];
            cl[(4 * r + u) * 64 + lane] = iu < end ? 1.0f + q : -1.0f;
        }
    }
    // neighbour ranges, one per lane: lanes 0..26 the stencil cells (lane
    // 9 (oz+1) + 3 (oy+1) + ox+1); the chunk's own cell (lane 13) is cut
    // around the chunk's diagonal blocks, its tail is range 27
    uint32_t ra = 0, rb = 0, sb = 0;
    bool sp = false;
    if (lane < 27) {
        const int ox = lane % 3 - 1, oy = (lane / 3) % 3 - 1, oz = lane / 9 - 1;
        const uint32_t nb = cell_id(g, cx + ox, cy + oy, cz + oz);
        ra = off[nb];
        rb = off[nb + 1];
        // a sparse cell's particles have consecutive sparse ordinals
        sp = rb > ra && rb - ra < (uint32_t)kDenseMin;
        if (sp) sb = s_sparse[ra];
    }
    const uint32_t cend = (uint32_t)__builtin_amdgcn_readlane((int)rb, 13);
    const uint32_t tail = h + 16u * (uint32_t)R;
    if (lane == 13) rb = h;
    if (lane == 27) {
        ra = tail;
        rb = cend > tail ? cend : tail;
    }
    const uint64_t spm = __ballot(sp);
    // the dense ranges stream block by block; the sparse cells' few particles
    // are packed 16 to a block below
    uint64_t todo = __ballot(lane < 28 && rb > ra && !sp);

    // FP32 partials over at most 32 blocks.  A flush sums them over the 16
    // lanes of each row group (halving exchanges in a fixed order; afterwards
    // lane col holds entry m = col: row block m / 4, register m % 4) and adds
    // that row total to the lane's FP64 sum.
    float pf[4 * R];
#pragma unroll
    for (int m = 0; m < 4 * R; m++) pf[m] = 0.0f;
    double acc = 0.0;
    auto reduce = [&]() {
        float t[16];
#pragma unroll
        for (int m = 0; m < 16; m++) t[m] = m < 4 * R ? pf[m] : 0.0f;
#pragma unroll
        for (int half = 8; half >= 1; half >>= 1) {
            const bool upper = (col & half) != 0;
#pragma unroll
            for (int m = 0; m < half; m++) {
                if (m >= 4 * R && m + half >= 4 * R) continue;  // both zero
                const float keep = upper ? t[m + half] : t[m];
                const float send = upper ? t[m] : t[m + half];
                t[m] = keep + __shfl_xor(send, half);
            }
        }
        acc += (double)t[0];
#pragma unroll
        for (int m = 0; m < 4 * R; m++) pf[m] = 0.0f;
    };
    int nt = 0;
    auto flush = [&]() {
        if (++nt == 32) {
            reduce();
            nt = 0;
        }
    };

    // the chunk's own blocks: the self pairs sit on the diagonal of block
    // r = rd; their accumulator input is -1e30 so they weigh 0
    const int dv = col - 4 * grp;
#pragma unroll
    for (int rd = 0; rd < R; rd++) {
        const uint32_t j0 = h + 16u * (uint32_t)rd;
        const float val = ld(j0);
        const float bv = (grp == 3 && (uint32_t)col >= cend - j0) ? -1e30f : val;
#pragma unroll
        for (int r = 0; r < R; r++) {
            f32x4 cin = Cget(r);
            if (r == rd) {
#pragma unroll
                for (int u = 0; u < 4; u++) cin[u] = dv == u ? -1e30f : cin[u];
            }
            const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(A[r], bv, cin, 0, 0, 0);
#pragma unroll
            for (int u = 0; u < 4; u++) pf[4 * r + u] += clamp0(d[u]);
        }
        flush();
    }

    if (todo) {
        float As[R];
        f32x4 Cs[R];
        int k = __builtin_ctzll(todo);
        todo &= todo - 1;
        uint32_t j0 = (uint32_t)__builtin_amdgcn_readlane((int)ra, k);
        uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)rb, k);
        auto setup = [&](int kk) {
            const int ks = kk == 27 ? 13 : kk;
            const float sx = (float)(ks % 3 - 1) * g.cellb, sy = (float)((ks / 3) % 3 - 1) * g.cellb,
                        sz = (float)(ks / 9 - 1) * g.cellb;
            const float sg = grp == 0 ? sx : (grp == 1 ? sy : sz);
            const float bs = grp == 3 ? -(sx * sx + sy * sy + sz * sz) : sg;
#pragma unroll
            for (int r = 0; r < R; r++) {
                As[r] = grp == 3 ? 1.0f : A[r] - (sg + sg);
                Cs[r] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[r], bs, Cget(r), 0, 0, 0);
            }
        };
        setup(k);
        // one block: 16 neighbours [j0, j0 + 16) of range k (ending at b),
        // this lane's component val
        auto block = [&](uint32_t j0, uint32_t b, float val) {
            const uint32_t rem = b - j0;
            const float bv = (grp == 3 && (uint32_t)col >= rem) ? -1e30f : val;
#pragma unroll
            for (int r = 0; r < R; r++) {
                const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(As[r], bv, Cs[r], 0, 0, 0);
#pragma unroll
                for (int u = 0; u < 4; u++) pf[4 * r + u] += clamp0(d[u]);
            }
            flush();
        };
        // The blocks in stream order come from a generator (range gk, next
        // block gj, range end gb); four of them are loaded ahead in a ring.
        int gk = k;
        uint32_t gj = j0, gb = b;
        auto gen = [&](int &ko, uint32_t &jo) {
            ko = gk;
            jo = gj;
            if (gk < 0) return;
            gj += 16u;
            if (gj >= gb) {
                if (todo) {
                    gk = __builtin_ctzll(todo);
                    todo &= todo - 1;
                    gj = (uint32_t)__builtin_amdgcn_readlane((int)ra, gk);
                    gb = (uint32_t)__builtin_amdgcn_readlane((int)rb, gk);
                } else {
                    gk = -1;
                }
            }
        };
        // Blocks go in batches of two: the loads of the next batch are
        // issued before the current one is summed (two register sets in
        // turn; longer batches would cost the sixth wavefront per SIMD).  A
        // position past the stream's end loads the chunk's own first block
        // instead and is skipped.
        auto use = [&](int bk, uint32_t bj, float v) {
            if (bk < 0) return;
            if (bk != k) {
                k = bk;
                b = (uint32_t)__builtin_amdgcn_readlane((int)rb, k);
                setup(k);
            }
            block(bj, b, v);
        };
        constexpr int kB = 2;  // blocks per batch
        int ka[kB], kb[kB];
        uint32_t ja[kB], jb[kB];
        float va[kB], vb[kB];
#pragma unroll
        for (int t = 0; t < kB; t++) {
            gen(ka[t], ja[t]);
            va[t] = ld(ka[t] >= 0 ? ja[t] : h);
        }
        while (true) {
#pragma unroll
            for (int t = 0; t < kB; t++) {
                gen(kb[t], jb[t]);
                vb[t] = ld(kb[t] >= 0 ? jb[t] : h);
            }
#pragma unroll
            for (int t = 0; t < kB; t++) use(ka[t], ja[t], va[t]);
            if (kb[0] < 0) break;
#pragma unroll
            for (int t = 0; t < kB; t++) {
                gen(ka[t], ja[t]);
                va[t] = ld(ka[t] >= 0 ? ja[t] : h);
            }
#pragma unroll
            for (int t = 0; t < kB; t++) use(kb[t], jb[t], vb[t]);
            if (ka[0] < 0) break;
        }
    }
    // The sparse particles' shares from this chunk, in FP64 and added in fixed
    // point: the particles of all sparse ranges are numbered in range order
    // and handled 64 per pass, one per lane (its range and column found by one
    // scalar walk over the ranges); each lane sums the weights of the chunk's
    // particles in order (wave-uniform loads), then adds its total with one
    // atomic.
    uint32_t ntot = 0;
    for (uint64_t m = spm; m; m &= m - 1) {
        const int k = __builtin_ctzll(m);
        ntot += (uint32_t)__builtin_amdgcn_readlane((int)rb, k) - (uint32_t)__builtin_amdgcn_readlane((int)ra, k);
    }
    for (uint32_t p0 = 0; p0 < ntot; p0 += 64) {
        const uint32_t q = p0 + (uint32_t)lane;  // this lane's column number
        uint32_t js = h, dst = 0;                 // its particle and sparse ordinal
        int kc = 13;                              // and its stencil cell
        uint32_t pre = 0;
        for (uint64_t m = spm; m; m &= m - 1) {
            const int k = __builtin_ctzll(m);
            const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)ra, k);
            const uint32_t cnt = (uint32_t)__builtin_amdgcn_readlane((int)rb, k) - a;
            if (q >= pre && q < pre + cnt) {
                js = a + (q - pre);
                dst = (uint32_t)__builtin_amdgcn_readlane((int)sb, k) + (q - pre);
                kc = k;
            }
            pre += cnt;
        }
        // The chunk's rows against the sparse particles packed 16 to a block:
        // the image shift goes to the neighbour side, B = (x_j + s, -|x_j +
        // s|^2) in the chunk's cell-centred frame (staged in LDS, one particle
        // per lane), A and the accumulator input are the rows' unshifted ones.
        // For the pairs that count the terms stay below about 4 in magnitude,
        // as in the blocks above.
        {
            const float4 qj = reinterpret_cast<const float4 *>(pq)[js];
            const float x = qj.x + (float)(kc % 3 - 1) * g.cellb, y = qj.y + (float)((kc / 3) % 3 - 1) * g.cellb,
                        z = qj.z + (float)(kc / 9 - 1) * g.cellb;
            s_pk[lane] = make_float4(x, y, z, q < ntot ? -(x * x + y * y + z * z) : -1e30f);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            __builtin_amdgcn_wave_barrier();
            const uint32_t nb = min(ntot - p0, 64u);
            for (uint32_t b0 = 0; b0 < nb; b0 += 16) {
                const float4 e = s_pk[b0 + (uint32_t)col];
                const float bv = grp == 0 ? e.x : (grp == 1 ? e.y : (grp == 2 ? e.z : e.w));
#pragma unroll
                for (int r = 0; r < R; r++) {
                    const f32x4 d = __builtin_amdgcn_mfma_f32_16x16x4f32(A[r], bv, Cget(r), 0, 0, 0);
#pragma unroll
                    for (int u = 0; u < 4; u++) pf[4 * r + u] += clamp0(d[u]);
                }
                flush();
            }
            __builtin_amdgcn_wave_barrier();
        }
        // the sparse particle's image in the chunk's frame
        const float4 pj = spos[js];
        const Pos64 pjm{(double)pj.x + image_shift(cx, kc % 3 - 1, g.nc, g.L),
                        (double)pj.y + image_shift(cy, (kc / 3) % 3 - 1, g.nc, g.L),
                        (double)pj.z + image_shift(cz, kc / 9 - 1, g.nc, g.L)};
        double v = 0.0;
        for (uint32_t r = h; r < end; r++) v += weight64(pjm, spos[r], g.inv_b2);
        if (q < ntot && v > 0.0)
            atomicAdd(reinterpret_cast<unsigned long long *>(&dfx[dst]),
                      (unsigned long long)__double2ll_rn(v * kFixScale));
    }
    reduce();
    const uint32_t ii = h + 16u * (uint32_t)(col >> 2) + 4u * (uint32_t)grp + (uint32_t)(col & 3);
    if (ii < end) {
        // the self pair weighs exactly 1 when it counts
        const double S = acc + (g.self_count ? 1.0 : 0.0);
        const float dd = (float)(g.norm * S);
        dens_s[ii] = dd;
        if (dens_out) dens_out[orig_of(spos[ii])] = dd;
    }
}

// One wavefront per workgroup: chunk costs differ widely, and a finished
// wavefront frees its slot at once.
__global__ __launch_bounds__(64, 6) void k_density_dense(int64_t nchunks, Boxes bx, bool narrow,
                                                      const int32_t *__restrict__ chunks,
                                                      const float4 *__restrict__ sloc,
                                                      const float4 *__restrict__ pq,
                                                      const float4 *__restrict__ spos,
                                                      const uint32_t *__restrict__ off,
                                                      const uint32_t *__restrict__ s_sparse,
                                                      uint64_t *__restrict__ dfx,
                                                      float *__restrict__ dens_s,
                                                      float *__restrict__ dens_out) {
    const int64_t q = (int64_t)xcd_block();
    if (q >= nchunks) return;
    const uint32_t h = (uint32_t)__builtin_amdgcn_readfirstlane(chunks[q]);
    const Geo &g = bx.geo[__builtin_amdgcn_readfirstlane(box_of(bx, h))];
    const uint32_t c = __builtin_amdgcn_readfirstlane(__float_as_uint(sloc[h].w));
    const uint32_t cend = __builtin_amdgcn_readfirstlane(off[c + 1]);
    const uint32_t end = min(h + 64u, cend);
    const float *p = reinterpret_cast<const float *>(pq);
    // the rows' accumulator inputs, and the packed sparse neighbours
    __shared__ float cl[16 * 64];
    __shared__ float4 s_pk[64];
#define HF_DENSITY_CHUNK(RR)                                                                        \
    (narrow ? density_chunk<RR, true>(g, h, c, end, p, spos, off, s_sparse, dfx, dens_s, dens_out, cl, s_pk) \
            : density_chunk<RR, false>(g, h, c, end, p, spos, off, s_sparse, dfx, dens_s, dens_out, cl, s_pk))
    switch ((end - h + 15u) >> 4) {
    case 1: HF_DENSITY_CHUNK(1); break;
    case 2: HF_DENSITY_CHUNK(2); break;
    case 3: HF_DENSITY_CHUNK(3); break;
    default: HF_DENSITY_CHUNK(4); break;
    }
#undef HF_DENSITY_CHUNK
}

// Sparse cells: one particle per lane, sparse neighbour cells only; the pairs
// with dense neighbour cells were summed by the dense kernel into dfx.  This
// is particle i (entry t of the sparse list) of box g.
__device__ __forceinline__ void density_sparse_one(const Geo &g, int64_t t, int64_t i,
                                                   const float4 *__restrict__ sloc,
                                                   const float4 *__restrict__ spos,
                                                   const uint32_t *__restrict__ off,
                                                   const uint64_t *__restrict__ dfx,
                                                   float *__restrict__ dens_s, float *__restrict__ dens_out) {
    const float4 li = sloc[i];
    const float4 pi = spos[i];
    const uint32_t c = __float_as_uint(li.w);
    const int nc = g.nc;
    int cx, cy, cz;
    cell_xyz(g, c, cx, cy, cz);
    const uint32_t x0 = (uint32_t)wrapc(cx - 1, nc), x1 = (uint32_t)cx, x2 = (uint32_t)wrapc(cx + 1, nc);
    // away from the periodic x edges the three cells of a stencil row are
    // consecutive: their four bounding offsets are one 16-byte load
    const bool inner = cx > 0 && cx < nc - 1;
    double acc = 0.0;
#pragma unroll 1
    for (int oz = -1; oz <= 1; oz++) {
        const int z = wrapc(cz + oz, nc);
        const float gz = oz < 0 ? li.z : (oz > 0 ? g.cellb - li.z : 0.0f);
        // the offsets of this plane are loaded together so their latencies
        // overlap; the cells to visit are kept as their starts and, packed
        // three bits each, their particle counts (0: dense, empty or out of
        // reach)
        uint32_t ra[9], cnts = 0;
#pragma unroll
        for (int oy = -1; oy <= 1; oy++) {
            const uint32_t row =
                g.cell_base + ((uint32_t)z * (uint32_t)nc + (uint32_t)wrapc(cy + oy, nc)) * (uint32_t)nc;
            const int r = (oy + 1) * 3;
            uint32_t o[6];
            if (inner) {
                const uint32_t *p = off + row + x0;
                o[0] = p[0];
                o[1] = p[1];
                o[2] = p[1];
                o[3] = p[2];
                o[4] = p[2];
                o[5] = p[3];
            } else {
                o[0] = off[row + x0];
                o[1] = off[row + x0 + 1];
                o[2] = off[row + x1];
                o[3] = off[row + x1 + 1];
                o[4] = off[row + x2];
                o[5] = off[row + x2 + 1];
            }
            const float gy = oy < 0 ? li.y : (oy > 0 ? g.cellb - li.y : 0.0f);
#pragma unroll
            for (int ox = -1; ox <= 1; ox++) {
                const uint32_t a = o[2 * (ox + 1)], cnt = o[2 * (ox + 1) + 1] - a;
                // a cell whose nearest face is b or more away (by a margin far
                // above the rounding of the local coordinates) weighs nothing
                const float gx = ox < 0 ? li.x : (ox > 0 ? g.cellb - li.x : 0.0f);
                const bool use = cnt < (uint32_t)kDenseMin && gx * gx + gy * gy + gz * gz < 1.0f + 1e-5f;
                ra[r + ox + 1] = a;
                cnts |= (use ? cnt : 0u) << (3 * (r + ox + 1));
            }
        }
        // the plane's cells walked as one sequence of particles (cell after
        // cell in stencil order, so the summation order is that of a loop per
        // cell): every lane runs through its own particles, and the wavefront
        // waits on the longest lane's count for the whole plane rather than on
        // the longest count of each cell
        uint32_t j = 0, e = 0;
        Pos64 pim{0.0, 0.0, 0.0};
        for (;;) {
            if (j == e) {
                if (cnts == 0u) break;
                const int r = __builtin_ctz(cnts) / 3;
                const uint32_t cnt = (cnts >> (3 * r)) & 7u;
                cnts &= ~(7u << (3 * r));
                uint32_t a = ra[0];
#pragma unroll
                for (int u = 1; u < 9; u++) a = r == u ? ra[u] : a;
                j = a;
                e = a + cnt;
                // i's position in this cell's frame
                const int ox = r % 3 - 1, oy = r / 3 - 1;
                pim = Pos64{(double)pi.x - image_shift(cx, ox, nc, g.L), (double)pi.y - image_shift(cy, oy, nc, g.L),
                            (double)pi.z - image_shift(cz, oz, nc, g.L)};
            }
            acc += weight64(pim, spos[j], g.inv_b2);
            j++;
        }
    }
    acc += (double)dfx[t] * (1.0 / kFixScale);
    write_density(i, acc, g, spos, dens_s, dens_out);
}

// The sparse-cell particles whose wavefront lies in one box (nearly all): the
// box's constants are read with a box index uniform over the wavefront, so
// they come with scalar loads into scalar registers.  A wavefront that spans
// a box boundary (one per boundary at most) is listed in mixed[] and left to
// k_density_sparse_mixed.  The kernel waits on memory, so it is held to 64
// VGPRs (eight wavefronts per SIMD, the most a SIMD runs).
__global__ __launch_bounds__(kBlock, 8) void k_density_sparse(int64_t nsparse, Boxes bx,
                                                           const int32_t *__restrict__ sparse,
                                                           const float4 *__restrict__ sloc,
                                                           const float4 *__restrict__ spos,
                                                           const uint32_t *__restrict__ off,
                                                           const uint64_t *__restrict__ dfx,
                                                           float *__restrict__ dens_s,
                                                           float *__restrict__ dens_out,
                                                           int32_t *__restrict__ mixed,
                                                           uint32_t *__restrict__ nmixed) {
    const int64_t t = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    if (t >= nsparse) return;
    const int lane = threadIdx.x & 63;
    const int64_t i = sparse[t];
    const int b = box_of(bx, (uint32_t)i);
    const int b0 = __builtin_amdgcn_readfirstlane(b);
    if (__ballot(b != b0) != 0ull) {
        const uint64_t act = __ballot(true);
        if (lane == __ffsll((unsigned long long)act) - 1) mixed[atomicAdd(nmixed, 1u)] = (int32_t)(t - lane);
        return;
    }
    density_sparse_one(bx.geo[b0], t, i, sloc, spos, off, dfx, dens_s, dens_out);
}

// The wavefronts of the sparse list that span a box boundary: each lane reads
// its own box's constants.
__global__ __launch_bounds__(64) void k_density_sparse_mixed(int64_t nsparse, Boxes bx,
                                                             const uint32_t *__restrict__ nmixed,
                                                             const int32_t *__restrict__ mixed,
                                                             const int32_t *__restrict__ sparse,
                                                             const float4 *__restrict__ sloc,
                                                             const float4 *__restrict__ spos,
                                                             const uint32_t *__restrict__ off,
                                                             const uint64_t *__restrict__ dfx,
                                                             float *__restrict__ dens_s,
                                                             float *__restrict__ dens_out) {
    if (blockIdx.x >= *nmixed) return;
    const int64_t t = (int64_t)mixed[blockIdx.x] + threadIdx.x;
    if (t >= nsparse) return;
    const int64_t i = sparse[t];
    density_sparse_one(bx.geo[box_of(bx, (uint32_t)i)], t, i, sloc, spos, off, dfx, dens_s, dens_out);
}

// Number of ordered pairs (i, j != i) closer than b, for the roofline's
// algorithmic pair count (evaluated in the same FP32 local coordinates).
__global__ __launch_bounds__(kBlock) void k_count_pairs(int64_t n, Boxes bx,
                                                        const float4 *__restrict__ sloc,
                                                        const uint32_t *__restrict__ off,
                                                        unsigned long long *__restrict__ total) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t cnt = 0;
    if (i < n) {
        const Geo &g = bx.geo[box_of(bx, (uint32_t)i)];
        const float4 li = sloc[i];
        const uint32_t c = __float_as_uint(li.w);
        int cx, cy, cz;
        cell_xyz(g, c, cx, cy, cz);
        for (int oz = -1; oz <= 1; oz++)
            for (int oy = -1; oy <= 1; oy++)
                for (int ox = -1; ox <= 1; ox++) {
                    const uint32_t nb = cell_id(g, cx + ox, cy + oy, cz + oz);
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

void launch_density(int64_t n, const Boxes &bx, Work &w, float *dens_out, hipStream_t s) {
    // dfx: dense-neighbour sums of the sparse particles (fixed point), in the
    // radix key array that binning no longer needs
    uint64_t *dfx = w.rkey[0];
    if (w.nsparse > 0) fill_u32(reinterpret_cast<uint32_t *>(dfx), 0u, 2 * w.nsparse, s);
    if (w.nchunks > 0) {
        // one buffer descriptor for all record loads while the byte offsets
        // fit in 32 bits; HF_DENSITY_WIDE=1 forces the per-block descriptors
        // of larger inputs (used by tests)
        bool narrow = (n + 32) * 16 <= (int64_t)0xffffff00;
        const char *force = getenv("HF_DENSITY_WIDE");
        if (force && force[0] == '1') narrow = false;
        hipLaunchKernelGGL(k_density_dense, dim3((unsigned)w.nchunks), dim3(64), 0, s, w.nchunks, bx, narrow,
                           w.chunks, w.sloc, w.pq, w.spos, w.off, w.s_sparse, dfx, w.dens_s, dens_out);
    }
    if (w.nsparse > 0) {
        // the wavefronts that span a box boundary: at most nbox - 1, listed
        // in the table-flag array (free until the output stage), their count
        // in counters[14] (zero since the call began)
        int32_t *mixed = reinterpret_cast<int32_t *>(w.tflag);
        uint32_t *nmixed = reinterpret_cast<uint32_t *>(w.counters + 14);
        hipLaunchKernelGGL(k_density_sparse, dim3((unsigned)((w.nsparse + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, s, w.nsparse, bx, w.sparse, w.sloc, w.spos, w.off, dfx, w.dens_s,
                           dens_out, mixed, nmixed);
        if (bx.nbox > 1)
            hipLaunchKernelGGL(k_density_sparse_mixed, dim3((unsigned)bx.nbox), dim3(64), 0, s, w.nsparse, bx,
                               nmixed, mixed, w.sparse, w.sloc, w.spos, w.off, dfx, w.dens_s, dens_out);
    }
}

void launch_count_pairs(int64_t n, const Boxes &bx, Work &w, unsigned long long *total, hipStream_t s) {
    hipLaunchKernelGGL(k_count_pairs, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, bx, w.sloc,
                       w.off, total);
}

void launch_gather_density(const float *dens_in, int64_t n, Work &w, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_density, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n,
                       w.spos, dens_in, w.dens_s);
}

}  // namespace hf
