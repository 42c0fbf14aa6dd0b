// Internal declarations of libhf: the geometry/constant block passed to every
// kernel, device helpers for the canonical predicates, and the stage launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hf.h"

namespace hf {

constexpr int kBlock = 256;
constexpr int kDenseMin = 8;   // a cell with at least this many particles is "dense"
constexpr int kRadBins = 2048; // radial bins of the threshold-radius search by bins

// Constants of one periodic box, computed on the host (see hf_derived).
struct Geo {
    double L, half;        // periodic side and L/2 (minimum-image test)
    double cell, inv_cell; // binning cell side (>= max(b, l)) and its inverse
    double inv_b;          // 1/b: local coordinates are stored in units of b
    double inv_b2;         // 1/b^2: FP64 kernel weights 1 - r^2/b^2
    float cellb;           // cell / b in FP32 (image offset of a neighbour cell)
    int nc;                // cells per side (>= 3)
    double inv_nc;         // 1 / nc (cell coordinates from a cell id)
    int ksub;              // sub-cells per cell side (sub-cell diagonal < l)
    int nsub;              // ksub^3
    int rsub;              // FoF reach in sub-cells: ceil(l / sub-cell side)
    double inv_sub;        // ksub / cell
    double sub2;           // squared sub-cell side
    int face_sub_in_b;     // any two points of face-adjacent sub-cells are closer than b
    double b2, l2;         // FP64 squared radii of the peak test and of FoF links
    float l2b_lo, l2b_hi;  // (l/b)^2 shrunk / grown by the FP32 prefilter margin
    float b2b_lo, b2b_hi;  // 1 shrunk / grown by the same margin (peak test, units of b^2)
    double norm;           // density normalisation 15/(8 pi b^3 nbar)
    int self_count;
    double dl0;            // L0 density threshold
    double floor_nuc;      // nucleation floor
    double K, K2, A6, C3;  // R^3 = i/K; alpha^6; c_Roche^3
    double rbin;           // radial bin width of the threshold-radius search by bins
    int n_l1_min;
    float particle_mass;
    // the box's place among the boxes of one call
    uint32_t cell_base;    // its first cell in the call's cell numbering
    uint32_t orig_base;    // its first particle (input and sorted order alike)
    int64_t n;             // its particles
    hf_halo *halos;        // its halo table (device), or null
    int64_t halo_cap;      // rows of that table
};

// The boxes of one call.  Particles and cells of all boxes are numbered
// together, box after box, so box b holds particles [base[b], base[b + 1])
// both in input order and after the sort (the sort key leads with the cell,
// and box b's cells follow box b - 1's), and cells
// [geo[b].cell_base, geo[b + 1].cell_base).  Labels are 1 + an index inside
// the box.
struct Boxes {
    const Geo *geo;        // device [nbox]
    const uint32_t *base;  // device [nbox + 1]: first particle of each box, then the total
    int nbox;
    int nsub_max;          // largest ksub^3: the sort-key stride of a cell and the row
                           // length - 1 of the dense-cell sub-tables
    const int32_t *btab;   // device (nbox > 1): btab[k] = box of particle k << bshift
    int bshift;
};

// Box of particle i (input or sorted order): the box of the table bucket that
// holds i, then forward over the box starts inside the bucket (a step or two:
// the table has several buckets per box on average).  No load when there is
// one box.
__device__ __forceinline__ int box_of(const Boxes &bx, uint32_t i) {
    if (bx.nbox <= 1) return 0;
    int b = bx.btab[i >> bx.bshift];
    while (b + 1 < bx.nbox && bx.base[b + 1] <= i) b++;
    return b;
}

// ---------------------------------------------------------------- predicates
// Canonical minimum-image squared distance in FP64: the same sequence of IEEE
// operations as the definition (differences of the float32 inputs promoted to
// double, one image fold per axis, (xx + yy) + zz) with no fused multiply-add.
__device__ __forceinline__ double d2_exact(float4 a, float4 b, double L, double half) {
#pragma clang fp contract(off)
    double dx = (double)b.x - (double)a.x;
    double dy = (double)b.y - (double)a.y;
    double dz = (double)b.z - (double)a.z;
    if (dx > half) dx -= L; else if (dx < -half) dx += L;
    if (dy > half) dy -= L; else if (dy < -half) dy += L;
    if (dz > half) dz -= L; else if (dz < -half) dz += L;
    double xx = dx * dx;
    double yy = dy * dy;
    double zz = dz * dz;
    double s = xx + yy;
    return s + zz;
}

__device__ __forceinline__ double e3(double e) {
#pragma clang fp contract(off)
    double ee = e * e;
    return ee * e;
}

__device__ __forceinline__ double ii(int64_t k) {
#pragma clang fp contract(off)
    double x = (double)k;
    return x * x;
}

__device__ __forceinline__ uint32_t orig_of(float4 p) { return __float_as_uint(p.w); }

// "Denser" total order of nuclei: higher density, ties to the lower index.
__device__ __forceinline__ bool denser(float da, uint32_t ia, float db, uint32_t ib) {
    return da > db || (da == db && ia < ib);
}

// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8), and each XCD has its own L2.  Work lists are in spatial order, so a
// kernel whose neighbours overlap maps workgroup b to a logical index such that
// every XCD gets one contiguous slice of the list and its L2 sees the reuse.
constexpr unsigned kXcds = 8;

__device__ __forceinline__ unsigned xcd_block() {
    const unsigned b = blockIdx.x, nb = gridDim.x;
    const unsigned per = nb / kXcds, rem = nb % kXcds;
    const unsigned x = b % kXcds, k = b / kXcds;
    const unsigned start = x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
    return start + k;
}

// FP32 squared distance for the prefilters (one multiply and two fused
// multiply-adds); their margins are far above the rounding of either form.
__device__ __forceinline__ float d2_f32(float dx, float dy, float dz) {
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// Value of lane L (L wave-uniform): a v_readlane into a scalar register,
// without the LDS round trip of a general shuffle.
__device__ __forceinline__ int lane_get(int v, int L) { return __builtin_amdgcn_readlane(v, L); }
__device__ __forceinline__ uint32_t lane_get(uint32_t v, int L) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, L);
}
__device__ __forceinline__ float lane_get(float v, int L) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), L));
}

// a / d for 0 <= a < 2^16 and 1 <= d <= 256 from FP32, given inv_d = 1/d:
// (a + 1/2) / d is at least 1/(2d) away from every integer and its FP32
// product with inv_d is within a few ulps of it, far less, so the truncation
// is the integer quotient (a few instructions instead of an integer division
// by a variable; checked exhaustively over that range).
__device__ __forceinline__ int div_small(int a, float inv_d) { return (int)(((float)a + 0.5f) * inv_d); }

__device__ __forceinline__ int wrapc(int c, int nc) {
    return c < 0 ? c + nc : (c >= nc ? c - nc : c);
}

// x / nc for a cell id x < 2^32: the FP64 product with 1/nc is within far
// less than one of x / nc (x is exact in FP64), so its truncation is the
// quotient or one below it; one comparison corrects that (and, for safety, one
// above).
__device__ __forceinline__ uint32_t div_nc(uint32_t x, const Geo &g) {
    uint32_t q = (uint32_t)((double)x * g.inv_nc);
    const uint64_t nc = (uint64_t)g.nc;
    if ((uint64_t)(q + 1) * nc <= (uint64_t)x) q++;
    else if ((uint64_t)q * nc > (uint64_t)x) q--;
    return q;
}

// Coordinates inside its box of cell c (the call's numbering) of box g.
__device__ __forceinline__ void cell_xyz(const Geo &g, uint32_t c, int &cx, int &cy, int &cz) {
    const uint32_t lc = c - g.cell_base, nc = (uint32_t)g.nc;
    const uint32_t q = div_nc(lc, g), q2 = div_nc(q, g);
    cx = (int)(lc - q * nc);
    cy = (int)(q - q2 * nc);
    cz = (int)q2;
}

// The cell at coordinates (x, y, z) of box g, each wrapped once (one cell
// beyond a face at most), in the call's numbering.
__device__ __forceinline__ uint32_t cell_id(const Geo &g, int x, int y, int z) {
    const int nc = g.nc;
    return g.cell_base + ((uint32_t)wrapc(z, nc) * (uint32_t)nc + (uint32_t)wrapc(y, nc)) * (uint32_t)nc +
           (uint32_t)wrapc(x, nc);
}

// Record error bit `bit` for box `box` (err[0] collects the bits, err[1] the
// smallest box that raised one).
__device__ __forceinline__ void flag_error(int32_t *err, int32_t bit, int box) {
    atomicOr(err, bit);
    atomicMin(err + 1, box);
}

__device__ __forceinline__ bool is_member(const float *dens_s, int64_t j, double dl0) {
    return (double)dens_s[j] > dl0;
}

// Runs of equal keys among consecutive lanes of a wavefront: the lane of the
// run's first element, this lane's rank in the run, and the run length.  Used
// to aggregate atomics on sorted data (one atomic per run instead of per lane).
struct WaveRun {
    int head, rank, len;
};

__device__ __forceinline__ WaveRun wave_run(int key) {
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(key, 1, 64);
    const bool is_head = lane == 0 || prev != key;
    const uint64_t heads = __ballot(is_head);
    const uint64_t le = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const int head = 63 - __clzll(heads & le);
    const uint64_t upto_head = head == 63 ? ~0ull : ((2ull << head) - 1ull);
    const uint64_t above = heads & ~upto_head;
    const int next = above ? __ffsll((unsigned long long)above) - 1 : 64;
    return WaveRun{head, lane - head, next - head};
}

// Minimum of v over the lane's run (valid in the run's head lane).
__device__ __forceinline__ int32_t wave_run_min(int32_t v, const WaveRun &r) {
    const int lane = threadIdx.x & 63;
    const int end = r.head + r.len;
    for (int d = 1; d < 64; d <<= 1) {
        int32_t o = __shfl_down(v, d, 64);
        if (lane + d < end) v = min(v, o);
    }
    return v;
}

// --------------------------------------------------------------- workspace
struct Work {
    // binning
    uint32_t *cnt, *off;             // cnt: cell -> dense-cell ordinal (dense cells only)
    uint64_t *rkey[2];               // radix sort keys (ping-pong, rkey[1] = rkey[0] + n); reused after binning
    uint32_t *rval[2];               // radix sort payload: original index
    uint32_t *rhist, *rscan;         // per-pass [digit][tile] counts and their scan
    uint16_t *ssub;
    float4 *spos, *sloc;
    float4 *pq;                      // density only: cell-centred (x, y, z, -|x|^2), n + 32 entries
    // work decomposition (dense chunks, dense cells, sparse particles)
    uint32_t *f_chunk, *s_chunk, *f_dcell, *s_dcell, *f_sparse, *s_sparse;
    int32_t *chunks, *sparse;
    uint32_t *dcells, *subtab;
    uint64_t *submax;                                  // densest particle per dense sub-cell
    int32_t *subarg;
    int32_t *hardlist;                                 // candidate tests left after stage 1
    int64_t nchunks, ndcells, nsparse, nhard;
    int ncu;                         // compute units (grids of the persistent kernels)
    bool radius_bins;                // R_L1 by radial bins instead of the whole-group histogram
    // density / FoF / groups (sorted order unless noted)
    float *dens_s;
    int32_t *parent, *minorig, *gkey, *gid_of, *owner;
    uint32_t *gcnt, *goff, *gidx;                     // key space [0, n]
    int32_t *mem;                                     // members grouped by group
    int32_t *g_start, *g_size, *g_label;              // per group
    uint32_t *gccnt, *gcoff, *gcfill, *gcidx;          // candidates per group
    int32_t *glist;                                    // groups with candidates
    int32_t *cand, *cand_sorted;                       // candidates
    int32_t *h_nuc, *h_ienc, *h_gid, *g_nh;            // halo slots (= candidate slots)
    uint32_t *h_count;
    uint32_t *tflag, *tpos;                            // table rows (original index space)
    uint32_t *hist;                                    // R search histograms
    uint32_t *scan_tmp;
    double *gcom;                    // halo statistics only: centres per group (6 doubles)
    int32_t *ordk;                   // halo statistics only: group ordinal per key
    int32_t *counters;                                 // small device counters
    int32_t *err;                    // [0] error bits, [1] smallest box with an error
    Geo *geo, *geo2;                 // the boxes' constants (geo2: level 2, halo statistics only)
    uint32_t *base;                  // first particle of every box, then the total
    int32_t *btab;                   // box of every 2^bshift-th particle (Boxes::btab)
    int64_t *box_rows;               // halo-table rows of every box
    uint32_t *host;                                    // the lane's pinned host words (read_words)
};

// ------------------------------------------------------------------ launchers
// Device words to read back to the host in one go.
struct WordSrc {
    static constexpr int kMax = 8;
    const uint32_t *p[kMax];
};
// One small kernel copies *src.p[0..k) into the pinned host buffer `host`
// (at least kMax words), the stream is synchronized and out[0..k) receives
// the values: one dispatch and one wait for all the counts a step needs.
hipError_t read_words(const WordSrc &src, int k, uint32_t *host, uint32_t *out, hipStream_t s);
// The same in two halves: the copy is enqueued on s, and the words are read
// once the caller has waited for it (an event recorded right after it), so
// that later work can be enqueued first.
hipError_t publish_words(const WordSrc &src, int k, uint32_t *host, hipStream_t s);
void collect_words(const uint32_t *host, int k, uint32_t *out);
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void fill_i32(int32_t *p, int32_t v, int64_t n, hipStream_t s);
// Exclusive scan: out[0..n] with out[n] = total.  tmp: scan_tmp_words(n) words.
void scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s);
// Exclusive scan of the indicator in[i] != 0 (same layout and tmp as scan_u32).
void scan_nz_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s);
int64_t scan_tmp_words(int64_t n);

// Every launcher works on all boxes of the call at once: n is the particle
// total, bx the boxes (device tables), ncell the cell total.
void launch_bin(const float *pos, int64_t n, int64_t ncell, const Boxes &bx, Work &w, hipStream_t s);
// Level 2 summaries and position statistics after an L2 pass (stats.hip; one
// box, g its constants).
void launch_halo_stats(int64_t n, int64_t G, int64_t M, const Geo &g, double particle_mass, const float *pos,
                       const int32_t *halo_id, Work &w, hf_halo_summary *out, int32_t *group_start,
                       int32_t *group_members, hipStream_t s);
// Length of the radix count arrays for n particles.
int64_t radix_hist_len(int64_t n);
// Stable LSD radix sort of n 64-bit keys a[] by their bits [lo, lo + bits),
// using b[] as the second buffer and w's count arrays; returns the buffer
// (a or b) that holds the result.
uint64_t *radix_sort_keys(uint64_t *a, uint64_t *b, int64_t n, int lo, int bits, Work &w, hipStream_t s);
void launch_subtab(int64_t n, const uint32_t *ndc_p, const Boxes &bx, Work &w, hipStream_t s);
void launch_density(int64_t n, const Boxes &bx, Work &w, float *dens_out, hipStream_t s);
void launch_count_pairs(int64_t n, const Boxes &bx, Work &w, unsigned long long *total, hipStream_t s);
void launch_gather_density(const float *dens_in, int64_t n, Work &w, hipStream_t s);
void launch_fof(int64_t n, const Boxes &bx, Work &w, hipStream_t s);
void launch_fof_labels(int64_t n, const Boxes &bx, Work &w, int32_t *l0_out, hipStream_t s);
void launch_keys_from_labels(const int32_t *l0_in, const float *dens_in, int64_t n, const Boxes &bx, Work &w,
                             hipStream_t s);
void launch_segment(int64_t n, Work &w, hipStream_t s);
void launch_segment_groups(int64_t n, int64_t G, Work &w, hipStream_t s);
// Extent check of the L0 groups (sets err bit 8 when a group spans half its
// box or more along an axis); M members in G groups.
void launch_extent(int64_t G, int64_t M, const Boxes &bx, Work &w, hipStream_t s);
void launch_candidates(int64_t n, const Boxes &bx, Work &w, hipStream_t s);   // candidates.hip
// Candidates in descending density per group; the groups with candidates in
// descending size (the largest first, over all boxes).
void launch_candidates_sort(int64_t n, int64_t G, int64_t NC, Work &w, hipStream_t s);
// Groups with candidates (their count is read on the device; grid bound
// min(G, NC)); M = members of all groups, n = particles.
void launch_accept(int64_t n, int64_t G, int64_t NC, int64_t M, const Boxes &bx, Work &w, hipStream_t s);
void launch_assign(int64_t n, const Boxes &bx, Work &w, hipStream_t s);
void launch_output_flags(int64_t n, int64_t NC, const Boxes &bx, Work &w, hipStream_t s);
// halo_id / l0_out: device [n], box-local labels; dens_out: device [n], the
// densities (l0_out and dens_out may be null).  Each box's table goes to its
// Geo::halos when its rows fit in Geo::halo_cap; box_rows (device [nbox])
// receives every box's row count.
void launch_output(int64_t n, int64_t NC, const Boxes &bx, Work &w, int32_t *halo_id, int32_t *l0_out,
                   float *dens_out, int64_t *box_rows, hipStream_t s);
// One box after launch_output: its n particles by table row of their halo
// (nrows rows, then the particles of no halo), ascending index within a row,
// into members [n]; halo_start [nrows + 1] receives each row's first position.
void launch_group_order(int64_t n, int64_t nrows, const int32_t *halo_id, Work &w, int32_t *members,
                        int64_t *halo_start, hipStream_t s);

}  // namespace hf
