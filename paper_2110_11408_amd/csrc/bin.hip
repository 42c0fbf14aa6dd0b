// Cell binning: a stable sort of the particles by (cell, sub-cell), ties in
// original index order.
//
// The paper's host code receives particles already ordered by cell from the
// N-body engine (Sec. 2.3.4); here the caller hands over an unordered float32
// [n][3] array, so the library builds the order itself:
//   1. key = cell * k^3 + sub-cell per particle (range check of the input);
//   2. least-significant-digit radix sort of (key, original index), digits of
//      at most 8 bits; key and index share one 64-bit word when they fit.
//      Each pass: a block counts the digits of its tile of 2048 consecutive
//      elements; an exclusive scan of the digit-major [digit][tile] counts
//      gives every (digit, tile) its output offset; the tile is then walked
//      again in order, each element's rank among equal digits coming from the
//      ballots of its digit bits (lower lanes first), so the pass is stable,
//      and written out through LDS in digit order (coalesced runs).
//      Consecutive tiles run on one XCD, so the runs that consecutive tiles
//      write for a digit (adjacent in the output) meet in one L2;
//   3. the sorted order writes two float4 streams per particle:
//        spos = (x, y, z, original index bits)    -- the paper's float quad with
//               the index stored bitwise (Sec. 2.3.3), used by FP64 predicates;
//        sloc = (x, y, z relative to the cell corner, in units of b; cell id
//               bits) -- FP32 coordinates whose differences across a periodic
//               face stay exact, used by the density loop and prefilters;
//   4. cell offsets for every cell of the grid, written by the sorted
//      particles that end each run of cells (coalesced, one wavefront per 64).
// Cells are at least max(b, l) wide; each is split into k^3 sub-cells whose
// diagonal is below l, so all particles of one sub-cell are friends.  The
// boxes of one call are binned together: their cells are numbered box after
// box, so the sorted order is box-major and box b keeps the slots of its
// input range.
//
// Work decomposition shared by the neighbour-loop kernels: a cell holding at
// least kDenseMin particles is "dense".  Dense cells get a table of their
// sub-cell offsets and are cut into chunks of at most 64 consecutive particles
// (one wavefront each); particles of the other cells form the "sparse" list
// (one thread each).  The in-cell order, and therefore every summation order,
// is fixed by the data, never by thread scheduling.
#include <stdlib.h>

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

// Sort key of particle i: cell * nsub_max + sub-cell, the cell numbered in the
// call's numbering (box after box).  Packed mode stores (key << ib) | i in one
// word (ib bits hold the index); otherwise the index travels in a separate
// payload array.
// A thread keys kKeyIlp particles (i0, i0 + kBlock, ...), their positions
// loaded together (one load in flight per thread leaves most of the
// bandwidth unused).
constexpr int kKeyIlp = 4;
__global__ __launch_bounds__(kBlock) void k_bin_key(const float *__restrict__ pos, int64_t n, Boxes bx, int ib,
                                                    uint64_t *__restrict__ key,
                                                    int32_t *__restrict__ err) {
    const int64_t i0 = (int64_t)blockIdx.x * (kBlock * kKeyIlp) + threadIdx.x;
    float px[kKeyIlp], py[kKeyIlp], pz[kKeyIlp];
#pragma unroll
    for (int u = 0; u < kKeyIlp; u++) {
        const int64_t i = i0 + (int64_t)u * kBlock;
        px[u] = i < n ? pos[3 * i + 0] : 0.0f;
        py[u] = i < n ? pos[3 * i + 1] : 0.0f;
        pz[u] = i < n ? pos[3 * i + 2] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kKeyIlp; u++) {
        const int64_t i = i0 + (int64_t)u * kBlock;
        if (i >= n) break;
        const int box = box_of(bx, (uint32_t)i);
        const Geo &g = bx.geo[box];
        const float x = px[u], y = py[u], z = pz[u];
        const float Lf = (float)g.L;
        const bool ok = x >= 0.0f && x < Lf && y >= 0.0f && y < Lf && z >= 0.0f && z < Lf;
        if (!ok) flag_error(err, 1, box);
        const int cx = cell_coord(x, g), cy = cell_coord(y, g), cz = cell_coord(z, g);
        const uint32_t c =
            g.cell_base + ((uint32_t)cz * (uint32_t)g.nc + (uint32_t)cy) * (uint32_t)g.nc + (uint32_t)cx;
        const int k = g.ksub;
        const uint32_t sub = (uint32_t)((sub_coord(z, cz, g) * k + sub_coord(y, cy, g)) * k + sub_coord(x, cx, g));
        const uint64_t kk = (uint64_t)c * (uint64_t)bx.nsub_max + sub;
        key[i] = ib > 0 ? (kk << ib) | (uint64_t)i : kk;
    }
}

constexpr int kRadixMaxBits = 8;
// k_radix_scatter scans the digit counts with one digit per thread of its 256
static_assert((1 << kRadixMaxBits) <= 256, "at most 256 digits per radix pass");
constexpr int kRadixWaves = 4;                      // wavefronts per tile
constexpr int kRadixIters = 8;                      // 64-element steps per wavefront
// 2048 elements per tile: the scatter's LDS tile (16 KB of keys) then lets
// seven blocks share a CU, twice as many as with 4096
constexpr int64_t kTile = 64 * kRadixWaves * kRadixIters;

// Lanes holding the same D-bit digit as this lane (within `active`).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, int D, uint64_t active) {
    uint64_t m = active;
    for (int b = 0; b < D; b++) {
        const uint64_t bal = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return m;
}

__device__ __forceinline__ uint64_t lanes_below(int lane) {
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Digit counts of one tile, stored digit-major ([digit][tile]).  Wavefront w
// of the tile owns elements [w * 512, (w + 1) * 512) of it and loads all 8 of
// its steps before counting.
__global__ __launch_bounds__(256) void k_radix_count(const uint64_t *__restrict__ key, int64_t n, int shift,
                                                     int D, int64_t ntiles, uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[1 << kRadixMaxBits];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t t = xcd_block();
    const int nd = 1 << D;
    for (int d = threadIdx.x; d < nd; d += 256) h[d] = 0u;
    const int64_t base = t * kTile + (int64_t)w * (64 * kRadixIters) + lane;
    uint64_t k[kRadixIters];
#pragma unroll
    for (int it = 0; it < kRadixIters; it++) {
        const int64_t e = base + it * 64;
        k[it] = e < n ? key[e] : 0ull;
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRadixIters; it++) {
        const bool act = base + it * 64 < n;
        const uint32_t d = (uint32_t)(k[it] >> shift) & (uint32_t)(nd - 1);
        const uint64_t m = digit_peers(d, D, __ballot(act));
        if (act && (m & lanes_below(lane)) == 0ull) atomicAdd(&h[d], (uint32_t)__popcll(m));
    }
    __syncthreads();
    for (int d = threadIdx.x; d < nd; d += 256) hist[(int64_t)d * ntiles + t] = h[d];
}

// Block-wide exclusive scan of one value per thread (256 threads).
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t *s_tot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) s_tot[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (int x = 0; x < w; x++) pre += s_tot[x];
    return pre + inc - v;
}

// Stable scatter of one tile.  Every element's position inside the tile's
// digit-sorted order is its digit's start in the tile plus the count of equal
// digits before it (earlier wavefronts, earlier steps, lower lanes); the tile
// is first placed in LDS in that order and then written out in order, so
// consecutive threads write consecutive addresses of one digit's run (the
// digit's global offset for this tile comes from the scanned counts).
template <bool kPacked>
__global__ __launch_bounds__(256) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                       const uint32_t *__restrict__ vin, int64_t n, int shift,
                                                       int D, int64_t ntiles, const uint32_t *__restrict__ hscan,
                                                       uint64_t *__restrict__ kout, uint32_t *__restrict__ vout) {
    __shared__ uint32_t o[kRadixWaves][1 << kRadixMaxBits];
    __shared__ uint32_t lstart[1 << kRadixMaxBits], gbase[1 << kRadixMaxBits];
    __shared__ uint32_t s_tot[kRadixWaves];
    __shared__ uint64_t sk[kTile];
    __shared__ uint32_t sv[kPacked ? 1 : kTile];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, tid = threadIdx.x;
    const int64_t t = xcd_block();
    const int nd = 1 << D;
    const uint32_t dmask = (uint32_t)(nd - 1);
    for (int d = lane; d < nd; d += 64) o[w][d] = 0u;
    const int64_t base = t * kTile + (int64_t)w * (64 * kRadixIters) + lane;
    uint64_t k[kRadixIters];
    uint32_t v[kPacked ? 1 : kRadixIters];
#pragma unroll
    for (int it = 0; it < kRadixIters; it++) {
        const int64_t e = base + it * 64;
        k[it] = e < n ? kin[e] : 0ull;
        if (!kPacked) v[it] = e < n ? (vin ? vin[e] : (uint32_t)e) : 0u;
    }
    // counts of this wavefront (its own LDS row; leaders only, in step order)
#pragma unroll
    for (int it = 0; it < kRadixIters; it++) {
        const bool act = base + it * 64 < n;
        const uint32_t d = (uint32_t)(k[it] >> shift) & dmask;
        const uint64_t m = digit_peers(d, D, __ballot(act));
        if (act && (m & lanes_below(lane)) == 0ull) o[w][d] += (uint32_t)__popcll(m);
    }
    __syncthreads();
    // digit starts inside the tile, then every wavefront's start per digit
    uint32_t tot = 0;
    if (tid < nd)
        for (int x = 0; x < kRadixWaves; x++) tot += o[x][tid];
    const uint32_t ex = block_scan_excl(tot, s_tot);
    if (tid < nd) {
        lstart[tid] = ex;
        gbase[tid] = hscan[(int64_t)tid * ntiles + t];
        uint32_t b = ex;
        for (int x = 0; x < kRadixWaves; x++) {
            const uint32_t c = o[x][tid];
            o[x][tid] = b;
            b += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRadixIters; it++) {
        const bool act = base + it * 64 < n;
        const uint32_t d = (uint32_t)(k[it] >> shift) & dmask;
        const uint64_t m = digit_peers(d, D, __ballot(act));
        const uint32_t start = act ? o[w][d] : 0u;
        if (act) {
            const uint32_t lp = start + (uint32_t)__popcll(m & lanes_below(lane));
            sk[lp] = k[it];
            if (!kPacked) sv[lp] = v[it];
        }
        // LDS operations of one wavefront complete in order: every lane of the
        // group has read `start` before the leader's update lands
        if (act && (m & lanes_below(lane)) == 0ull) o[w][d] = start + (uint32_t)__popcll(m);
    }
    __syncthreads();
    const int64_t rem = n - t * kTile;
    const int cnt = rem < kTile ? (int)rem : (int)kTile;
    for (int lp = tid; lp < cnt; lp += 256) {
        const uint64_t key = sk[lp];
        const uint32_t d = (uint32_t)(key >> shift) & dmask;
        const uint32_t dst = gbase[d] + ((uint32_t)lp - lstart[d]);
        kout[dst] = key;
        if (!kPacked) vout[dst] = sv[lp];
    }
}

// Sorted slot s: the particle's two float4 records, its sub-cell and, when
// densities follow, its density record.
template <bool kPacked>
__global__ __launch_bounds__(kBlock) void k_bin_place(const float *__restrict__ pos, int64_t n, Boxes bx, int ib,
                                                      const uint64_t *__restrict__ key,
                                                      const uint32_t *__restrict__ idx,
                                                      float4 *__restrict__ spos, float4 *__restrict__ sloc,
                                                      float4 *__restrict__ pq, uint16_t *__restrict__ ssub) {
    const int64_t s = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    // pq's padding (read past a cell's end by the density kernel, never used)
    if (pq && s < 32) pq[n + s] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (s >= n) return;
    const uint64_t kw = key[s];
    const uint64_t k = kPacked ? kw >> ib : kw;
    const uint32_t o = kPacked ? (uint32_t)(kw & ((1ull << ib) - 1ull)) : idx[s];
    const uint32_t nsub = (uint32_t)bx.nsub_max;
    const uint32_t c = (uint32_t)(k / nsub);
    const uint32_t sub = (uint32_t)(k - (uint64_t)c * nsub);
    const Geo &g = bx.geo[box_of(bx, (uint32_t)s)];
    const float x = pos[3 * (int64_t)o + 0], y = pos[3 * (int64_t)o + 1], z = pos[3 * (int64_t)o + 2];
    spos[s] = make_float4(x, y, z, __uint_as_float(o));
    const uint32_t nc = (uint32_t)g.nc, lc = c - g.cell_base;
    const uint32_t cx = lc % nc, cy = (lc / nc) % nc, cz = lc / (nc * nc);
    const float xl = (float)(((double)x - (double)cx * g.cell) * g.inv_b);
    const float yl = (float)(((double)y - (double)cy * g.cell) * g.inv_b);
    const float zl = (float)(((double)z - (double)cz * g.cell) * g.inv_b);
    sloc[s] = make_float4(xl, yl, zl, __uint_as_float(c));
    if (pq) {
        // coordinates about the cell centre and minus their squared norm
        const float c0 = 0.5f * g.cellb;
        const float xc = xl - c0, yc = yl - c0, zc = zl - c0;
        pq[s] = make_float4(xc, yc, zc, -(xc * xc + yc * yc + zc * zc));
    }
    ssub[s] = (uint16_t)sub;
}

// Cell offsets: off[c] = first sorted particle of cell c (the next cell's
// start when c is empty), off[ncell] = n.  With C(s) = cell of slot s,
// C(-1) = -1 and C(n) = ncell, slot s owns the cells (C(s-1), C(s)].  Each
// wavefront takes 64 consecutive slots (the last one slot n) and writes the
// cells they own with consecutive lanes on consecutive cells (16-byte stores);
// the owner of a cell is the last slot that owns cells and starts at or before
// it, found from a bitmask of the starts in each 256-cell window (a count of
// set bits gives its rank among those slots) and a rank -> slot table.
__global__ __launch_bounds__(kBlock) void k_cell_offsets(int64_t n, int64_t ncell,
                                                         const float4 *__restrict__ sloc,
                                                         uint32_t *__restrict__ off) {
    __shared__ uint64_t s_bits[kBlock / 64][4];   // starts inside the current 256-cell window
    __shared__ uint8_t s_slot[kBlock / 64][64];   // slot of each rank
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t s0 = ((int64_t)blockIdx.x * (kBlock / 64) + w) * 64;
    if (s0 > n) return;  // whole wavefront past slot n (uniform)
    const int64_t s = s0 + lane;
    auto C = [&](int64_t q) -> int64_t {
        return q < 0 ? -1 : (q >= n ? ncell : (int64_t)__float_as_uint(sloc[q].w));
    };
    const int64_t hi = s <= n ? C(s) : ncell;
    const int64_t lo = s <= n ? C(s - 1) : ncell;
    // cells owned by this slot, and their exclusive prefix over the wavefront
    // (32-bit: the grid has fewer than 2^32 cells)
    const uint32_t g = (uint32_t)(hi - lo);
    uint32_t incl = g;
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    const uint32_t pre = incl - g;
    const uint32_t G = lane_get(incl, 63);
    // first cell owned by the wavefront: one past the cell of the slot before
    // it, which lane 0 holds as lo (a cell id below 2^32 when s0 > 0)
    const int64_t first =
        s0 == 0 ? 0 : (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)lo) + 1;
    const int64_t end = first + (int64_t)G;
    // the slots that own cells, in order: rank -> slot
    const uint64_t owners = __ballot(g > 0);
    if (g > 0) s_slot[w][__popcll(owners & lanes_below(lane))] = (uint8_t)lane;
    // windows of 256 cells aligned to 4, four consecutive cells per lane; the
    // owner of a cell is the slot of rank (number of owned starts at or before
    // it) - 1, counted from a bitmask of the starts in the window
    uint32_t before = 0;  // starts in earlier windows
    for (int64_t w0 = first & ~(int64_t)3; w0 < end; w0 += 256) {
        if (lane < 4) s_bits[w][lane] = 0ull;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        const int64_t st = first + (int64_t)pre;
        if (g > 0 && st >= w0 && st < w0 + 256) {
            const int r = (int)(st - w0);
            atomicOr(reinterpret_cast<unsigned long long *>(&s_bits[w][r >> 6]), 1ull << (r & 63));
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        const uint64_t b0 = s_bits[w][0], b1 = s_bits[w][1], b2 = s_bits[w][2], b3 = s_bits[w][3];
        const int p = 4 * lane, k = p >> 6;
        const uint64_t wk = k == 0 ? b0 : (k == 1 ? b1 : (k == 2 ? b2 : b3));
        const uint32_t lower = before + (k > 0 ? (uint32_t)__popcll(b0) : 0u) + (k > 1 ? (uint32_t)__popcll(b1) : 0u) +
                               (k > 2 ? (uint32_t)__popcll(b2) : 0u);
        uint32_t v[4];
        bool all = true;
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int pu = (p + u) & 63;
            const uint64_t upto = pu == 63 ? ~0ull : ((2ull << pu) - 1ull);
            const uint32_t cnt = lower + (uint32_t)__popcll(wk & upto);
            const int64_t cell = w0 + p + u;
            const bool valid = cell >= first && cell < end;
            all = all && valid;
            // read for every cell (the rank is at most 64), so that the four
            // reads are issued together
            const uint32_t sl = s_slot[w][(cnt > 0u ? cnt - 1u : 0u) & 63u];
            v[u] = valid ? (uint32_t)s0 + sl : 0u;
        }
        if (all) {
            *reinterpret_cast<uint4 *>(off + w0 + p) = make_uint4(v[0], v[1], v[2], v[3]);
        } else {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int64_t cell = w0 + p + u;
                if (cell >= first && cell < end) off[cell] = v[u];
            }
        }
        before += (uint32_t)(__popcll(b0) + __popcll(b1) + __popcll(b2) + __popcll(b3));
    }
}

// Flags per sorted particle: head of a dense chunk, head of a dense cell,
// sparse.  A wavefront takes 64 consecutive particles and finds the bounds of
// their cells from the cell ids of neighbouring particles (cell changes are
// found by ballot); only a cell that starts before, or ends after, the
// wavefront's particles reads its offset from the grid.
__global__ __launch_bounds__(kBlock) void k_bin_flags(int64_t n, const float4 *__restrict__ sloc,
                                                      const uint32_t *__restrict__ off,
                                                      uint32_t *__restrict__ f_chunk,
                                                      uint32_t *__restrict__ f_dcell,
                                                      uint32_t *__restrict__ f_sparse) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const int64_t s0 = i - lane;
    const bool act = i < n;
    // the cells beyond the wavefront's two ends are loaded with the lanes'
    // own (lane 0: slot s0 - 1, lane 63: slot s0 + 64)
    const int64_t e = lane == 0 ? s0 - 1 : (lane == 63 ? s0 + 64 : -1);
    const uint32_t c = act ? __float_as_uint(sloc[i].w) : 0xffffffffu;
    const uint32_t ce = e >= 0 && e < n ? __float_as_uint(sloc[e].w) : 0u;
    uint32_t cprev = __shfl_up(c, 1, 64), cnext = __shfl_down(c, 1, 64);
    if (lane == 0) cprev = s0 > 0 ? ce : 0xfffffffeu;
    if (lane == 63) cnext = s0 + 64 < n ? ce : 0xfffffffdu;
    const uint64_t heads = __ballot(act && c != cprev);
    const uint64_t tails = __ballot(act && c != cnext);
    if (!act) return;
    const uint64_t le = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const uint64_t h = heads & le, t = tails & ~(le >> 1);  // heads at or below, tails at or above
    const uint32_t a = h ? (uint32_t)(s0 + 63 - __clzll((long long)h)) : off[c];
    const uint32_t b = t ? (uint32_t)(s0 + __ffsll((unsigned long long)t)) : off[c + 1];
    const bool dense = b - a >= (uint32_t)kDenseMin;
    f_chunk[i] = dense && (((uint32_t)i - a) % 64u == 0u);
    f_dcell[i] = dense && (uint32_t)i == a;
    f_sparse[i] = !dense;
}

constexpr int kListIlp = 4;
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
    // kListIlp particles per thread (i0, i0 + kBlock, ...): their flags and
    // list positions loaded together, the positions whatever the flags (one
    // round of loads instead of two)
    const int64_t i0 = (int64_t)blockIdx.x * (kBlock * kListIlp) + threadIdx.x;
    uint32_t fc[kListIlp], sc[kListIlp], fs[kListIlp], ss[kListIlp], fd[kListIlp];
#pragma unroll
    for (int u = 0; u < kListIlp; u++) {
        const int64_t i = i0 + (int64_t)u * kBlock;
        const bool in = i < n;
        fc[u] = in ? f_chunk[i] : 0u;
        sc[u] = in ? s_chunk[i] : 0u;
        fs[u] = in ? f_sparse[i] : 0u;
        ss[u] = in ? s_sparse[i] : 0u;
        fd[u] = in ? f_dcell[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kListIlp; u++) {
        const int64_t i = i0 + (int64_t)u * kBlock;
        if (fc[u]) chunks[sc[u]] = (int32_t)i;
        if (fs[u]) sparse[ss[u]] = (int32_t)i;
        if (fd[u]) {
            const uint32_t c = __float_as_uint(sloc[i].w);
            const uint32_t d = s_dcell[i];
            dcells[d] = c;
            cellmap[c] = d;  // the cell-count array is reused as cell -> dense-cell map
        }
    }
}

// Sub-cell table of one dense cell d, by one wavefront: entry s is the first
// particle of the cell whose sub-cell is s or later (an empty sub-cell gets
// the start of the next non-empty one; entry nsub is the cell end).  The
// cell's particles are sorted by sub-cell, so particle j writes the entries
// after its predecessor's sub-cell up to its own, and the entries after the
// last particle's sub-cell get the cell end; every entry is written once.
__device__ __forceinline__ void sub_table_cell(int64_t d, const Boxes &bx, const uint32_t *__restrict__ dcells,
                                               const uint32_t *__restrict__ off,
                                               const uint16_t *__restrict__ ssub,
                                               uint32_t *__restrict__ subtab) {
    const int lane = threadIdx.x & 63;
    const uint32_t c = (uint32_t)__builtin_amdgcn_readfirstlane(dcells[d]);
    const uint32_t a = (uint32_t)__builtin_amdgcn_readfirstlane(off[c]);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readfirstlane(off[c + 1]);
    const int nsub = __builtin_amdgcn_readfirstlane(bx.geo[box_of(bx, a)].nsub);
    uint32_t *t = subtab + d * (bx.nsub_max + 1);
    for (uint32_t j0 = a; j0 < b; j0 += 64) {
        const uint32_t j = j0 + (uint32_t)lane;
        if (j < b) {
            const int cur = ssub[j];
            const int prev = j > a ? (int)ssub[j - 1] : -1;
            for (int s2 = prev + 1; s2 <= cur; s2++) t[s2] = j;
            if (j + 1 == b)
                for (int s2 = cur + 1; s2 <= nsub; s2++) t[s2] = b;
        }
    }
}

// The sub-cell tables of all dense cells, one wavefront per cell over a grid
// that strides the cells; the cell count *ndc_p is read on the device.
__global__ __launch_bounds__(kBlock) void k_sub_table(const uint32_t *__restrict__ ndc_p, Boxes bx,
                                                      const uint32_t *__restrict__ dcells,
                                                      const uint32_t *__restrict__ off,
                                                      const uint16_t *__restrict__ ssub,
                                                      uint32_t *__restrict__ subtab) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t ndc = *ndc_p;
    const int64_t stride = (int64_t)gridDim.x * (kBlock / 64);
    for (int64_t d = (int64_t)blockIdx.x * (kBlock / 64) + wave; d < ndc; d += stride)
        sub_table_cell(d, bx, dcells, off, ssub, subtab);
}

}  // namespace

int bit_width(uint64_t x) {
    int b = 0;
    while (b < 64 && (x >> b)) b++;
    return b;
}

// Radix pass plan: key bits, index bits when packed (0 = separate payload).
struct RadixPlan {
    int passes, D, ib;
};

RadixPlan radix_plan(int64_t n, int64_t ncell, int nsub_max) {
    const uint64_t nkeys = (uint64_t)ncell * (uint64_t)nsub_max;
    int bits = bit_width(nkeys - 1);
    if (bits < 1) bits = 1;
    RadixPlan r;
    r.passes = (bits + kRadixMaxBits - 1) / kRadixMaxBits;
    r.D = (bits + r.passes - 1) / r.passes;
    int ib = bit_width((uint64_t)(n > 1 ? n - 1 : 1));
    r.ib = ib + bits <= 64 ? ib : 0;
    // HF_RADIX_PAYLOAD=1 forces the separate-payload form (used by tests; it
    // is otherwise taken only when key and index need more than 64 bits)
    const char *force = getenv("HF_RADIX_PAYLOAD");
    if (force && force[0] == '1') r.ib = 0;
    return r;
}

int64_t radix_hist_len(int64_t n) {
    // room for the widest digit, so that every sort of up to n keys fits
    const int64_t ntiles = (n + kTile - 1) / kTile;
    return ((int64_t)1 << kRadixMaxBits) * (ntiles > 0 ? ntiles : 1) + 1;
}

uint64_t *radix_sort_keys(uint64_t *a, uint64_t *b, int64_t n, int lo, int bits, Work &w, hipStream_t s) {
    if (n <= 1 || bits <= 0) return a;
    const int passes = (bits + kRadixMaxBits - 1) / kRadixMaxBits;
    const int D = (bits + passes - 1) / passes;
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const int64_t hl = ((int64_t)1 << D) * ntiles;
    uint64_t *cur = a, *nxt = b;
    for (int p = 0; p < passes; p++) {
        const int shift = lo + p * D;
        hipLaunchKernelGGL(k_radix_count, dim3((unsigned)ntiles), dim3(256), 0, s, cur, n, shift, D, ntiles,
                           w.rhist);
        scan_u32(w.rhist, w.rscan, hl, w.scan_tmp, s);
        hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)ntiles), dim3(256), 0, s, cur, nullptr, n, shift,
                           D, ntiles, w.rscan, nxt, nullptr);
        uint64_t *t = cur;
        cur = nxt;
        nxt = t;
    }
    return cur;
}

void launch_bin(const float *pos, int64_t n, int64_t ncell, const Boxes &bx, Work &w, hipStream_t s) {
    const RadixPlan r = radix_plan(n, ncell, bx.nsub_max);
    const bool packed = r.ib > 0;
    hipLaunchKernelGGL(k_bin_key, dim3(blocks((n + kKeyIlp - 1) / kKeyIlp)), dim3(kBlock), 0, s, pos, n, bx, r.ib,
                       w.rkey[0], w.err);
    const int64_t ntiles = (n + kTile - 1) / kTile;
    const int64_t hl = ((int64_t)1 << r.D) * ntiles;
    int cur = 0;
    for (int p = 0; p < r.passes; p++) {
        const int shift = r.ib + p * r.D;
        hipLaunchKernelGGL(k_radix_count, dim3((unsigned)ntiles), dim3(256), 0, s, w.rkey[cur], n, shift, r.D,
                           ntiles, w.rhist);
        scan_u32(w.rhist, w.rscan, hl, w.scan_tmp, s);
        if (packed)
            hipLaunchKernelGGL(k_radix_scatter<true>, dim3((unsigned)ntiles), dim3(256), 0, s, w.rkey[cur],
                               nullptr, n, shift, r.D, ntiles, w.rscan, w.rkey[cur ^ 1], nullptr);
        else
            hipLaunchKernelGGL(k_radix_scatter<false>, dim3((unsigned)ntiles), dim3(256), 0, s, w.rkey[cur],
                               p == 0 ? nullptr : w.rval[cur], n, shift, r.D, ntiles, w.rscan,
                               w.rkey[cur ^ 1], w.rval[cur ^ 1]);
        cur ^= 1;
    }
    if (packed)
        hipLaunchKernelGGL(k_bin_place<true>, dim3(blocks(n)), dim3(kBlock), 0, s, pos, n, bx, r.ib, w.rkey[cur],
                           nullptr, w.spos, w.sloc, w.pq, w.ssub);
    else
        hipLaunchKernelGGL(k_bin_place<false>, dim3(blocks(n)), dim3(kBlock), 0, s, pos, n, bx, 0, w.rkey[cur],
                           w.rval[cur], w.spos, w.sloc, w.pq, w.ssub);
    // slots 0..n (slot n closes the grid): one wavefront per 64
    hipLaunchKernelGGL(k_cell_offsets, dim3((unsigned)((n + 1 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, n,
                       ncell, w.sloc, w.off);
    hipLaunchKernelGGL(k_bin_flags, dim3(blocks(n)), dim3(kBlock), 0, s, n, w.sloc, w.off, w.f_chunk,
                       w.f_dcell, w.f_sparse);
    scan_u32(w.f_chunk, w.s_chunk, n, w.scan_tmp, s);
    scan_u32(w.f_dcell, w.s_dcell, n, w.scan_tmp, s);
    scan_u32(w.f_sparse, w.s_sparse, n, w.scan_tmp, s);
    hipLaunchKernelGGL(k_bin_lists, dim3(blocks((n + kListIlp - 1) / kListIlp)), dim3(kBlock), 0, s, n, w.f_chunk,
                       w.s_chunk,
                       w.f_dcell, w.s_dcell, w.f_sparse, w.s_sparse, w.sloc, w.chunks, w.dcells,
                       w.sparse, w.cnt);
}

void launch_subtab(int64_t n, const uint32_t *ndc_p, const Boxes &bx, Work &w, hipStream_t s) {
    if (n <= 0) return;
    // the count is read on the device; a dense cell holds at least kDenseMin
    // particles, and a grid of at most 16384 workgroups strides over the cells
    const int64_t ub = n / kDenseMin + 1;
    int64_t blocks = (ub + kBlock / 64 - 1) / (kBlock / 64);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_sub_table, dim3((unsigned)blocks), dim3(kBlock), 0, s, ndc_p, bx, w.dcells, w.off,
                       w.ssub, w.subtab);
}

}  // namespace hf
