// CompaSO L1 inside every L0 group (Sec. 2.2.2) and the output cut.
//
// The paper's per-group loop is sequential (find a nucleus, assign, mark
// ineligible, repeat).  It decomposes exactly into data-parallel stages because
//   - the peak condition and the nucleation floor depend only on the densities
//     (steps 2 and 4), so the candidate set is fixed before the loop;
//   - R_L1 of a nucleus uses ALL particles of the L0 group and is independent of
//     earlier assignments (steps 1-2);
//   - eligibility depends only on earlier nuclei and their R (step 1);
//   - a particle's reassignment depends only on its current halo (step 3).
// Hence: candidates are found in parallel; one workgroup per group walks its
// candidates in descending density, rejects those inside alpha R of an
// accepted nucleus and computes R for the accepted ones; finally every
// particle folds over its group's accepted halos in creation order.
//
// R without sorting (Sec. 2.3.3: the enclosed mass at sorted position k is k,
// R_L1 is where the enclosed density first drops below Delta_L1).  With
// T(e) = K^2 e^3 for a squared distance e (R^3 = i/K), the sorted definition
// "first k >= 1 whose k-th smallest T exceeds k^2" is equivalent to
// "first k >= 1 with C(k) <= k", where C(k) counts particles with T <= k^2.
// C is the prefix sum of a histogram over integer buckets
// ceil(sqrt(T)) (computed exactly with integer-square comparisons), so each
// accepted nucleus costs one pass over the group plus a prefix scan.
#include "hf_internal.h"

namespace hf {

namespace {

inline dim3 grid(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

__device__ __forceinline__ int32_t ldi(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ldu(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stu(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ segmentation

__global__ __launch_bounds__(kBlock) void k_seg_count(int64_t n, const int32_t *__restrict__ gkey,
                                                      uint32_t *__restrict__ gcnt) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = i < n ? gkey[i] : -1;
    const WaveRun r = wave_run(k);
    if (k >= 0 && r.rank == 0) atomicAdd(&gcnt[k], (uint32_t)r.len);
}

__global__ __launch_bounds__(kBlock) void k_seg_groups(int64_t n, const uint32_t *__restrict__ gcnt,
                                                       const uint32_t *__restrict__ goff,
                                                       const uint32_t *__restrict__ gidx,
                                                       int32_t *__restrict__ g_start,
                                                       int32_t *__restrict__ g_size,
                                                       int32_t *__restrict__ g_label) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    uint32_t c = gcnt[k];
    if (!c) return;
    uint32_t g = gidx[k];
    g_start[g] = (int32_t)goff[k];
    g_size[g] = (int32_t)c;
    g_label[g] = (int32_t)k + 1;
}

// Members into group order: each run of equal keys among consecutive lanes
// takes a slice of its group by counting the group's count down (the order of
// members inside a group is not used).
__global__ __launch_bounds__(kBlock) void k_seg_scatter(int64_t n, const int32_t *__restrict__ gkey,
                                                        const uint32_t *__restrict__ goff,
                                                        const uint32_t *__restrict__ gidx,
                                                        uint32_t *__restrict__ gcnt,
                                                        int32_t *__restrict__ mem,
                                                        int32_t *__restrict__ gid_of) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = i < n ? gkey[i] : -1;
    const WaveRun r = wave_run(k);
    uint32_t base = 0;
    if (k >= 0 && r.rank == 0) base = atomicSub(&gcnt[k], (uint32_t)r.len) - (uint32_t)r.len;
    base = __shfl(base, r.head, 64);
    if (i >= n) return;
    if (k < 0) {
        gid_of[i] = -1;
        return;
    }
    mem[goff[k] + base + (uint32_t)r.rank] = (int32_t)i;
    gid_of[i] = (int32_t)gidx[k];
}

__global__ __launch_bounds__(kBlock) void k_cand_scatter(int64_t n, const int32_t *__restrict__ cflag,
                                                         const int32_t *__restrict__ gid_of,
                                                         const uint32_t *__restrict__ gcoff,
                                                         uint32_t *__restrict__ gcfill,
                                                         int32_t *__restrict__ cand) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !cflag[i]) return;
    int gi = gid_of[i];
    cand[gcoff[gi] + atomicAdd(&gcfill[gi], 1u)] = (int32_t)i;
}

// Candidate slot -> group, via a marker per group start and a max-scan would be
// heavier than a binary search over the group candidate offsets.
__device__ __forceinline__ int group_of_slot(const uint32_t *gcoff, int G, uint32_t s) {
    int lo = 0, hi = G - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (gcoff[mid] <= s) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Order candidates of a group by "denser" (density desc, original index asc):
// the rank of a candidate is the number of denser candidates in its group.
__global__ __launch_bounds__(kBlock) void k_cand_rank(int64_t NC, int G, const uint32_t *__restrict__ gcoff,
                                                      const int32_t *__restrict__ cand,
                                                      const float *__restrict__ dens_s,
                                                      const float4 *__restrict__ spos,
                                                      int32_t *__restrict__ cand_sorted) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= NC) return;
    int gi = group_of_slot(gcoff, G, (uint32_t)s);
    uint32_t a = gcoff[gi], b = gcoff[gi + 1];
    int me = cand[s];
    float dm = dens_s[me];
    uint32_t om = orig_of(spos[me]);
    uint32_t rank = 0;
    for (uint32_t t = a; t < b; t++) {
        int o = cand[t];
        rank += denser(dens_s[o], orig_of(spos[o]), dm, om) ? 1u : 0u;
    }
    cand_sorted[a + rank] = me;
}

__global__ __launch_bounds__(kBlock) void k_glist(int G, const uint32_t *__restrict__ gccnt,
                                                  const uint32_t *__restrict__ idx,
                                                  int32_t *__restrict__ glist) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    if (gccnt[g]) glist[idx[g]] = g;
}

// ------------------------------------------------------- group extent
// Every distance is a minimum image, which stands for the distance inside an
// L0 group only while the group spans less than half the box along each axis.
// A group whose extent reaches L/2 makes the call fail (HF_ERR_INVALID) rather
// than return labels computed with the wrong images.  The extent is measured
// from the group's first member r: with o_q the minimum-image offset of member
// q from r along an axis, extent = max o - min o.  Offsets below L/4 in every
// axis bound it below L/2, so a first pass flags the groups with a member at
// L/4 or more and the exact extent is taken for those only.

// Minimum-image offset b - a along one axis (the canonical fold).
__device__ __forceinline__ double mi_off(float a, float b, double L, double half) {
    double d = (double)b - (double)a;
    if (d > half) d -= L; else if (d < -half) d += L;
    return d;
}

__global__ __launch_bounds__(kBlock) void k_extent_far(int64_t M, Boxes bx, const int32_t *__restrict__ mem,
                                                       const int32_t *__restrict__ gid_of,
                                                       const int32_t *__restrict__ g_start,
                                                       const float4 *__restrict__ spos,
                                                       int32_t *__restrict__ gflag,
                                                       int32_t *__restrict__ farlist,
                                                       uint32_t *__restrict__ nfar) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M) return;
    const int i = mem[t];
    const Geo &g = bx.geo[box_of(bx, (uint32_t)i)];
    const int gi = gid_of[i];
    const float4 pr = spos[mem[g_start[gi]]];
    const float4 pi = spos[i];
    const double q = 0.25 * g.L;
    const bool far = fabs(mi_off(pr.x, pi.x, g.L, g.half)) >= q || fabs(mi_off(pr.y, pi.y, g.L, g.half)) >= q ||
                     fabs(mi_off(pr.z, pi.z, g.L, g.half)) >= q;
    if (far && atomicCAS(&gflag[gi], 0, 1) == 0) farlist[atomicAdd(nfar, 1u)] = gi;
}

// The exact extent of the flagged groups, one workgroup per group (grid-stride
// over the list, its length read on the device).
__global__ __launch_bounds__(kBlock) void k_extent_span(const uint32_t *__restrict__ nfar_p, Boxes bx,
                                                        const int32_t *__restrict__ farlist,
                                                        const int32_t *__restrict__ g_start,
                                                        const int32_t *__restrict__ g_size,
                                                        const int32_t *__restrict__ mem,
                                                        const float4 *__restrict__ spos,
                                                        int32_t *__restrict__ err) {
    __shared__ double s_lo[3][kBlock / 64], s_hi[3][kBlock / 64];
    const uint32_t nfar = *nfar_p;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (uint32_t f = blockIdx.x; f < nfar; f += gridDim.x) {
        const int gi = farlist[f];
        const int64_t start = g_start[gi], m = g_size[gi];
        const int box = __builtin_amdgcn_readfirstlane(box_of(bx, (uint32_t)mem[start]));
        const Geo &g = bx.geo[box];
        const float4 pr = spos[mem[start]];
        double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
        for (int64_t t = threadIdx.x; t < m; t += blockDim.x) {
            const float4 pq = spos[mem[start + t]];
            const double o[3] = {mi_off(pr.x, pq.x, g.L, g.half), mi_off(pr.y, pq.y, g.L, g.half),
                                 mi_off(pr.z, pq.z, g.L, g.half)};
#pragma unroll
            for (int a = 0; a < 3; a++) {
                lo[a] = fmin(lo[a], o[a]);
                hi[a] = fmax(hi[a], o[a]);
            }
        }
#pragma unroll
        for (int a = 0; a < 3; a++) {
            for (int d = 32; d >= 1; d >>= 1) {
                lo[a] = fmin(lo[a], __shfl_xor(lo[a], d, 64));
                hi[a] = fmax(hi[a], __shfl_xor(hi[a], d, 64));
            }
            if (lane == 0) {
                s_lo[a][wid] = lo[a];
                s_hi[a][wid] = hi[a];
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            bool wide = false;
            for (int a = 0; a < 3; a++) {
                double l = s_lo[a][0], h = s_hi[a][0];
                for (int w = 1; w < kBlock / 64; w++) {
                    l = fmin(l, s_lo[a][w]);
                    h = fmax(h, s_hi[a][w]);
                }
                wide = wide || h - l >= g.half;
            }
            if (wide) flag_error(err, 8, box);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------ acceptance and R
// Smallest integer k >= 0 with T <= k^2 (both sides as the FP64 expressions
// T and ii(k)); m when T > ii(m - 1) (beyond every k the search inspects).
__device__ __forceinline__ int64_t bucket_of(double T, int64_t m) {
    if (!(T > 0.0)) return 0;
    if (m <= 1 || T > ii(m - 1)) return m;
    // the loops below reach the exact k from any start in [0, m - 1]: the
    // start only sets their length, so it comes from the FP32 square root
    // (T < 2^62 here; within a few units of k below 2^23, one or two steps),
    // not from the much longer FP64 one
    int64_t k = (int64_t)ceilf(__builtin_amdgcn_sqrtf((float)T));
    if (k > m - 1) k = m - 1;
    if (k < 0) k = 0;
    while (k > 0 && T <= ii(k - 1)) k--;
    while (T > ii(k)) k++;
    return k;
}

constexpr int kHistMid = 12288;   // histogram buckets of a medium group counted in LDS (48 KB)
constexpr int kHistBig = 36864;   // histogram buckets of a large group counted in LDS (144 KB)
constexpr int kScanIpt = 16;      // buckets per thread per scan step

// Block-wide exclusive scan of one value per thread (NT threads).
template <int NT>
__device__ __forceinline__ uint32_t block_excl(uint32_t v, uint32_t *s_red, uint32_t *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t inc = v;
    for (int d = 1; d < 64; d <<= 1) {
        uint32_t t = __shfl_up(inc, d, 64);
        if (lane >= d) inc += t;
    }
    if (lane == 63) s_red[wid] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (int w = 0; w < NT / 64; w++) {
        if (w < wid) pre += s_red[w];
        tot += s_red[w];
    }
    __syncthreads();
    *total = tot;
    return pre + inc - v;
}

template <int NT>
__device__ __forceinline__ int block_min(int v, int *s_min) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int d = 32; d >= 1; d >>= 1) v = min(v, __shfl_xor(v, d, 64));
    if (lane == 0) s_min[wid] = v;
    __syncthreads();
    int best = s_min[0];
    for (int w = 1; w < NT / 64; w++) best = min(best, s_min[w]);
    __syncthreads();
    return best;
}

constexpr int kWaveHist = 1024;   // groups below this size run one per wavefront
constexpr int kWaveNuc = 64;      // ... when they have at most this many candidates

// Groups with candidates (all boxes, largest first), one wavefront at a time
// each: a persistent grid of W wavefronts in which wavefront w takes groups
// w, w + W, w + 2W, ... of the list (its length read on the device), so that
// every wavefront gets one group of each size tier.  (A shared counter that
// every wavefront increments per group serialises on its one address: tens of
// thousands of groups cost more in atomics than in work.)  Groups of fewer
// than kWaveHist particles with at
// most kWaveNuc candidates run here: the same walk as k_accept with the
// histogram, the accepted nuclei and their positions in the wavefront's LDS
// and wave-level scans instead of workgroup barriers, so that many small
// groups run on a CU at once.  The other groups are appended to mid_list
// (fewer than kHistMid particles) or big_list, with their counts in
// *mid_count and *big_count, for k_accept (route_all: every group, when R is
// searched by radial bins).
__global__ __launch_bounds__(kBlock) void k_accept_small(const uint32_t *__restrict__ ngc_p, bool route_all,
                                                         Boxes bx,
                                                         const int32_t *__restrict__ glist,
                                                         const int32_t *__restrict__ g_start,
                                                         const int32_t *__restrict__ g_size,
                                                         const uint32_t *__restrict__ gcoff,
                                                         const int32_t *__restrict__ cand_sorted,
                                                         const int32_t *__restrict__ mem,
                                                         const float4 *__restrict__ spos,
                                                         int32_t *__restrict__ h_nuc,
                                                         int32_t *__restrict__ h_ienc,
                                                         int32_t *__restrict__ h_gid,
                                                         int32_t *__restrict__ g_nh,
                                                         int32_t *__restrict__ mid_list,
                                                         uint32_t *__restrict__ mid_count,
                                                         int32_t *__restrict__ big_list,
                                                         uint32_t *__restrict__ big_count) {
#pragma clang fp contract(off)
    __shared__ uint32_t s_hist[kBlock / 64][kWaveHist];
    __shared__ float4 s_hp[kBlock / 64][kWaveNuc];
    __shared__ int32_t s_hi[kBlock / 64][kWaveNuc];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const uint32_t ngc = __builtin_amdgcn_readfirstlane(*ngc_p);
    const uint32_t nw = gridDim.x * (kBlock / 64);
    uint32_t *hist = s_hist[wave];
    for (uint32_t q = blockIdx.x * (kBlock / 64) + (uint32_t)wave; q < ngc; q += nw) {
        const int gi = glist[q];
        const int64_t start = g_start[gi];
        const int64_t m = g_size[gi];
        const Geo &g = bx.geo[__builtin_amdgcn_readfirstlane(box_of(bx, (uint32_t)mem[start]))];
        const uint32_t cs = gcoff[gi], ce = gcoff[gi + 1];
        if (route_all || m + 1 > kWaveHist || ce - cs > (uint32_t)kWaveNuc) {
            if (lane == 0) {
                if (m + 1 <= kHistMid) mid_list[atomicAdd(mid_count, 1u)] = gi;
                else big_list[atomicAdd(big_count, 1u)] = gi;
            }
            continue;
        }
        int nh = 0;
        for (uint32_t r = cs; r < ce; r++) {
            const int c = cand_sorted[r];
            const float4 pc = spos[c];
            // eligibility: not inside alpha R of any accepted nucleus (nh <= 64)
            bool inel = false;
            if (lane < nh) {
                const double e = d2_exact(pc, s_hp[wave][lane], g.L, g.half);
                inel = g.K2 * e3(e) < g.A6 * ii(s_hi[wave][lane]);
            }
            if (__ballot(inel)) continue;
            // bucket histogram over all m particles of the group
            for (int64_t k = lane; k <= m; k += 64) hist[k] = 0u;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            for (int64_t t = lane; t < m; t += 64) {
                const double e = d2_exact(pc, spos[mem[start + t]], g.L, g.half);
                atomicAdd(&hist[bucket_of(g.K2 * e3(e), m)], 1u);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
            __builtin_amdgcn_wave_barrier();
            // first k in [1, m-1] with C(k) <= k, C(k) = sum of buckets 0..k;
            // lane L covers buckets 16L .. 16L + 15 (m < 1024)
            uint32_t v[16];
            uint32_t sum = 0;
    #pragma unroll
            for (int u = 0; u < 16; u++) {
                const int64_t k = (int64_t)lane * 16 + u;
                v[u] = k < m ? hist[k] : 0u;
                sum += v[u];
            }
            uint32_t incl = sum;
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t y = __shfl_up(incl, d, 64);
                if (lane >= d) incl += y;
            }
            uint32_t C = incl - sum;
            int hit = -1;
    #pragma unroll
            for (int u = 0; u < 16; u++) {
                const int64_t k = (int64_t)lane * 16 + u;
                C += v[u];
                if (hit < 0 && k >= 1 && k < m && (int64_t)C <= k) hit = (int)k;
            }
            const uint64_t hm = __ballot(hit >= 0);
            const int64_t found = hm ? (int64_t)lane_get(hit, __ffsll((unsigned long long)hm) - 1) : m;
            if (lane == 0) {
                h_nuc[cs + nh] = c;
                h_ienc[cs + nh] = (int32_t)found;
                h_gid[cs + nh] = gi;
                s_hp[wave][nh] = pc;
                s_hi[wave][nh] = (int32_t)found;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            nh++;
        }
        if (lane == 0) g_nh[gi] = nh;
    }
}

// Squared outer edge of radial bin j of width w: ((j + 1) w)^2; bin j holds
// the squared distances e with edge(j - 1) <= e < edge(j).
__device__ __forceinline__ double rbin_edge2(int j, double w) {
    const double r = (double)(j + 1) * w;
    return r * r;
}

// The bin of e (the bin width is such that every minimum-image distance lies
// inside the last edge).
__device__ __forceinline__ int rbin_of(double e, double w) {
    int j = (int)(sqrt(e) / w);
    if (j > kRadBins - 1) j = kRadBins - 1;
    while (j > 0 && e < rbin_edge2(j - 1, w)) j--;
    while (j < kRadBins - 1 && !(e < rbin_edge2(j, w))) j++;
    return j;
}

// f(e) for the squared distance e of every member of the group to pc, the
// members spread over the workgroup (UB per thread and round, their loads
// issued together).
template <int NT, class F>
__device__ __forceinline__ void for_members(int64_t m, int64_t start, const int32_t *__restrict__ mem,
                                            const float4 *__restrict__ spos, const float4 &pc, const Geo &g,
                                            F f) {
    constexpr int UB = NT >= 1024 ? 4 : 8;
    for (int64_t t0 = threadIdx.x; t0 < m; t0 += UB * NT) {
        int32_t id[UB];
#pragma unroll
        for (int u = 0; u < UB; u++) {
            const int64_t t = t0 + (int64_t)u * NT;
            id[u] = t < m ? mem[start + t] : -1;
        }
        float4 pm[UB];
#pragma unroll
        for (int u = 0; u < UB; u++) pm[u] = id[u] >= 0 ? spos[id[u]] : pc;
#pragma unroll
        for (int u = 0; u < UB; u++)
            if (id[u] >= 0) f(d2_exact(pc, pm[u], g.L, g.half));
    }
}

// Zero hist[0..len]: LDS below HL, the group's global region gh beyond.
template <int NT, int HL>
__device__ __forceinline__ void hist_clear(uint32_t *s_hist, uint32_t *gh, int64_t len) {
    for (int64_t k = threadIdx.x; k <= len && k < HL; k += NT) s_hist[k] = 0u;
    if (len + 1 > HL) {
        for (int64_t k = HL + threadIdx.x; k <= len; k += NT) stu(gh + k, 0u);
        __threadfence();
    }
}

__device__ __forceinline__ void hist_add(uint32_t *s_hist, uint32_t *gh, int64_t k, int hl) {
    if (k < hl) atomicAdd(&s_hist[k], 1u);
    else atomicAdd(gh + k, 1u);
}

// First t in [0, len) with C(t) <= t and 1 <= base + t <= m - 1, where
// C(t) = hist[0] + ... + hist[t]; -1 when there is none.
template <int NT, int HL>
__device__ __forceinline__ int64_t first_crossing(const uint32_t *s_hist, const uint32_t *gh, int64_t len,
                                                  int64_t base, int64_t m, uint32_t *s_red, int *s_min) {
    constexpr int SI = NT >= 1024 ? kScanIpt / 2 : kScanIpt;
    uint32_t run = 0;
    for (int64_t b0 = 0; b0 < len; b0 += (int64_t)NT * SI) {
        const int64_t k0 = b0 + (int64_t)threadIdx.x * SI;
        uint32_t v[SI];
        uint32_t sum = 0;
#pragma unroll
        for (int u = 0; u < SI; u++) {
            const int64_t k = k0 + u;
            v[u] = k < len ? (k < HL ? s_hist[k] : ldu(gh + k)) : 0u;
            sum += v[u];
        }
        uint32_t tot;
        uint32_t C = run + block_excl<NT>(sum, s_red, &tot);
        int hit = 0x7fffffff;
#pragma unroll
        for (int u = 0; u < SI; u++) {
            const int64_t k = k0 + u;
            C += v[u];
            if (hit == 0x7fffffff && k < len && base + k >= 1 && base + k < m && (int64_t)C <= k)
                hit = (int)(k - b0);
        }
        const int best = block_min<NT>(hit, s_min);
        run += tot;
        if (best != 0x7fffffff) return b0 + best;
    }
    return -1;
}

// One workgroup per L0 group in `glist` (count on the device; the grid is an
// upper bound).  No persistent loop here: a group index broadcast through LDS
// by one thread, with a barrier inside a loop whose exit depends on it, is a
// form the compiler may restructure so that the other threads pass the barrier
// again before that thread has written the next index.  Walk the candidates
// in descending density; a
// candidate inside alpha R of an accepted nucleus is ineligible; an eligible
// one is accepted and its enclosed count i found
//   BINS = false: from the bucket histogram of all particles of the group;
//   BINS = true:  by the radial bins of Sec. 2.3.4.  Counts of the members per
//                 radial bin (width g.rbin, in LDS) give C_j, the members
//                 inside bin j's inner edge.  A bin whose C_j members, placed
//                 at its outer edge, still meet the threshold
//                 (K^2 edge^3 <= C_j^2) holds no crossing: every member in it
//                 is inside that edge at a sorted position >= C_j.  The first
//                 bin that is not passed over is searched with the bucket
//                 histogram of its own members (positions C_j .. C_j + c_j - 1
//                 of the sorted order: the crossing is the first t with
//                 #{bin members with bucket <= C_j + t} <= t), and the search
//                 moves outwards while a bin holds no crossing.
template <int NT, int HL, bool BINS>
__global__ __launch_bounds__(NT) void k_accept(const uint32_t *__restrict__ ngc_p,
                                               Boxes bx,
                                               const int32_t *__restrict__ glist,
                                               const int32_t *__restrict__ g_start,
                                               const int32_t *__restrict__ g_size,
                                               const uint32_t *__restrict__ gcoff,
                                               const int32_t *__restrict__ cand_sorted,
                                               const int32_t *__restrict__ mem,
                                               const float4 *__restrict__ spos,
                                               uint32_t *__restrict__ hist_all,
                                               int32_t *__restrict__ h_nuc,
                                               int32_t *__restrict__ h_ienc,
                                               int32_t *__restrict__ h_gid,
                                               int32_t *__restrict__ g_nh) {
#pragma clang fp contract(off)
    __shared__ uint32_t s_hist[HL + 1];
    __shared__ uint32_t s_rb[BINS ? kRadBins : 1];
    __shared__ int s_nh;
    __shared__ uint32_t s_red[NT / 64];
    __shared__ int s_min[NT / 64];
    if (blockIdx.x >= *ngc_p) return;
    const int tid = threadIdx.x;
    const int gi = glist[blockIdx.x];
    const int64_t start = g_start[gi];
    const int64_t m = g_size[gi];
    const uint32_t cs = gcoff[gi], ce = gcoff[gi + 1];
    const Geo &g = bx.geo[__builtin_amdgcn_readfirstlane(box_of(bx, (uint32_t)mem[start]))];
    // buckets below HL live in LDS; a group with more buckets keeps the
    // rest in its own global region (m + 1 words, disjoint per group).  The
    // small buckets are where the particles of a dense core pile up, so the
    // global atomics are only the sparse outer ones.
    uint32_t *ghist = hist_all + start + gi;
    if (tid == 0) s_nh = 0;
    __syncthreads();
    for (uint32_t r = cs; r < ce; r++) {
        const int nh = s_nh;
        // the next candidate from r on that is eligible (not inside alpha R of
        // any nucleus accepted so far), NT candidates tested at once, one per
        // thread: the ones passed over are ineligible in the serial order too,
        // since the nuclei change only when a candidate is accepted
        int next = 0x7fffffff;
        for (uint32_t r0 = r; r0 < ce; r0 += NT) {
            const uint32_t q = r0 + (uint32_t)tid;
            int hit = 0x7fffffff;
            if (q < ce) {
                const float4 pq = spos[cand_sorted[q]];
                bool el = true;
                for (int h = 0; h < nh && el; h++) {
                    const double e = d2_exact(pq, spos[ldi(h_nuc + cs + h)], g.L, g.half);
                    el = !(g.K2 * e3(e) < g.A6 * ii(ldi(h_ienc + cs + h)));
                }
                if (el) hit = (int)(q - r);
            }
            next = block_min<NT>(hit, s_min);
            if (next != 0x7fffffff) break;
        }
        if (next == 0x7fffffff) break;
        r += (uint32_t)next;
        const int c = cand_sorted[r];
        const float4 pc = spos[c];
        int64_t found = m;
        if constexpr (BINS) {
            // members per radial bin, then their inclusive prefix in place
            for (int k = tid; k < kRadBins; k += NT) s_rb[k] = 0u;
            __syncthreads();
            for_members<NT>(m, start, mem, spos, pc, g,
                            [&](double e) { atomicAdd(&s_rb[rbin_of(e, g.rbin)], 1u); });
            __syncthreads();
            constexpr int BI = kRadBins / NT;
            uint32_t v[BI];
            uint32_t sum = 0;
#pragma unroll
            for (int u = 0; u < BI; u++) {
                v[u] = s_rb[tid * BI + u];
                sum += v[u];
            }
            uint32_t tot;
            uint32_t P = block_excl<NT>(sum, s_red, &tot);
#pragma unroll
            for (int u = 0; u < BI; u++) {
                P += v[u];
                s_rb[tid * BI + u] = P;
            }
            __syncthreads();
            for (int j0 = 0;;) {
                // the innermost occupied bin from j0 on that is not passed over
                int jb = 0x7fffffff;
                for (int j = j0 + tid; j < kRadBins; j += NT) {
                    const uint32_t Cj = j ? s_rb[j - 1] : 0u;
                    if (s_rb[j] > Cj && !(g.K2 * e3(rbin_edge2(j, g.rbin)) <= ii(Cj))) {
                        jb = j;
                        break;
                    }
                }
                const int js = block_min<NT>(jb, s_min);
                if (js == 0x7fffffff) break;  // no crossing inside the group
                const int64_t C = js ? s_rb[js - 1] : 0u;
                const int64_t cnt = (int64_t)s_rb[js] - C;
                const double lo = js ? rbin_edge2(js - 1, g.rbin) : -1.0, hi = rbin_edge2(js, g.rbin);
                hist_clear<NT, HL>(s_hist, ghist, cnt);
                __syncthreads();
                for_members<NT>(m, start, mem, spos, pc, g, [&](double e) {
                    if (e >= lo && e < hi) {
                        int64_t k = bucket_of(g.K2 * e3(e), m) - C;
                        k = k < 0 ? 0 : (k > cnt ? cnt : k);
                        hist_add(s_hist, ghist, k, HL);
                    }
                });
                if (cnt + 1 > HL) __threadfence();
                __syncthreads();
                const int64_t t = first_crossing<NT, HL>(s_hist, ghist, cnt, C, m, s_red, s_min);
                if (t >= 0) {
                    found = C + t;
                    break;
                }
                j0 = js + 1;
            }
        } else {
            // histogram of buckets over all particles of the group
            hist_clear<NT, HL>(s_hist, ghist, m);
            __syncthreads();
            for_members<NT>(m, start, mem, spos, pc, g,
                            [&](double e) { hist_add(s_hist, ghist, bucket_of(g.K2 * e3(e), m), HL); });
            if (m + 1 > HL) __threadfence();
            __syncthreads();
            // first k in [1, m-1] with C(k) <= k, C(k) = sum of buckets 0..k
            const int64_t t = first_crossing<NT, HL>(s_hist, ghist, m, 0, m, s_red, s_min);
            if (t >= 0) found = t;
        }
        if (tid == 0) {
            h_nuc[cs + nh] = c;
            h_ienc[cs + nh] = (int32_t)found;
            h_gid[cs + nh] = gi;
            s_nh = nh + 1;
        }
        __syncthreads();
    }
    if (tid == 0) g_nh[gi] = s_nh;
}

// --------------------------------------------------------------- assignment
// Step 3 as a per-particle fold over the group's halos in creation order, with
// the flat-rotation-curve enclosed density Delta_L1 R^2 / r^2 (Sec. 2.3.2)
// compared in cubed form: i_new^2 e_own^3 >= c^3 i_own^2 e_new^3.
__global__ __launch_bounds__(kBlock) void k_assign(int64_t n, Boxes bx, const int32_t *__restrict__ gid_of,
                                                   const uint32_t *__restrict__ gcoff,
                                                   const int32_t *__restrict__ g_nh,
                                                   const int32_t *__restrict__ h_nuc,
                                                   const int32_t *__restrict__ h_ienc,
                                                   const float4 *__restrict__ spos,
                                                   int32_t *__restrict__ owner,
                                                   uint32_t *__restrict__ h_count) {
#pragma clang fp contract(off)
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int gi = i < n ? gid_of[i] : -1;
    int own = -1;
    if (gi >= 0) {
        const Geo &g = bx.geo[box_of(bx, (uint32_t)i)];
        const uint32_t cs = gcoff[gi];
        const int nh = g_nh[gi];
        const float4 pi = spos[i];
        double eown = 0.0, iown = 0.0;
        // the halos in creation order, four per round of loads (their
        // nuclei, then the nuclei's positions)
        for (int h0 = 0; h0 < nh; h0 += 4) {
            int nuc[4], ienc[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                nuc[u] = h0 + u < nh ? h_nuc[cs + h0 + u] : 0;
                ienc[u] = h0 + u < nh ? h_ienc[cs + h0 + u] : 0;
            }
            float4 pn[4];
#pragma unroll
            for (int u = 0; u < 4; u++) pn[u] = h0 + u < nh ? spos[nuc[u]] : pi;
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (h0 + u >= nh) break;
                const double e = d2_exact(pi, pn[u], g.L, g.half);
                const double ih = ii(ienc[u]);
                if (!(g.K2 * e3(e) < ih)) continue;
                bool take;
                if (own < 0) {
                    take = true;
                } else {
                    const double lhs = ih * e3(eown);
                    const double rhs = (g.C3 * iown) * e3(e);
                    take = lhs >= rhs;
                }
                if (take) {
                    own = (int)cs + h0 + u;
                    eown = e;
                    iown = ih;
                }
            }
        }
    }
    const WaveRun r = wave_run(own);
    if (own >= 0 && r.rank == 0) atomicAdd(&h_count[own], (uint32_t)r.len);
    if (i < n) owner[i] = own;
}

// ------------------------------------------------------------------- output

__global__ __launch_bounds__(kBlock) void k_out_flags(int64_t NC, Boxes bx, const int32_t *__restrict__ h_nuc,
                                                      const uint32_t *__restrict__ h_count,
                                                      const float4 *__restrict__ spos,
                                                      uint32_t *__restrict__ tflag,
                                                      int32_t *__restrict__ h_label,
                                                      int32_t *__restrict__ counters) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nuc = s < NC ? h_nuc[s] : -1;
    const uint64_t b = __ballot(nuc >= 0);
    if ((threadIdx.x & 63) == 0 && b) atomicAdd(&counters[2], __popcll(b));
    if (s >= NC) return;
    // the label every member of this halo gets: 1 + its nucleus's index in
    // the box when the halo is kept, else 0
    int32_t lab = 0;
    if (nuc >= 0) {
        const Geo &g = bx.geo[box_of(bx, (uint32_t)nuc)];
        if (h_count[s] >= (uint32_t)g.n_l1_min) {
            const uint32_t o = orig_of(spos[nuc]);
            tflag[o] = 1u;
            lab = (int32_t)(o - g.orig_base) + 1;
        }
    }
    h_label[s] = lab;
}

// Rows of the halo table of every box: the kept halos are flagged at their
// nucleus's original index, so a box's rows are the flags in its index range.
__global__ __launch_bounds__(kBlock) void k_box_rows(Boxes bx, const uint32_t *__restrict__ tpos,
                                                     int64_t *__restrict__ box_rows) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= bx.nbox) return;
    box_rows[b] = (int64_t)tpos[bx.base[b + 1]] - (int64_t)tpos[bx.base[b]];
}

// A halo's row in its box's table (ascending id); a box whose rows exceed its
// table's capacity gets none written.  Ids and labels are box-local.
__global__ __launch_bounds__(kBlock) void k_out_table(int64_t NC, Boxes bx, const int32_t *__restrict__ h_nuc,
                                                      const int32_t *__restrict__ h_ienc,
                                                      const int32_t *__restrict__ h_gid,
                                                      const uint32_t *__restrict__ h_count,
                                                      const int32_t *__restrict__ g_label,
                                                      const float4 *__restrict__ spos,
                                                      const uint32_t *__restrict__ tpos) {
    int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= NC) return;
    int nuc = h_nuc[s];
    if (nuc < 0) return;
    const int box = box_of(bx, (uint32_t)nuc);
    const Geo &g = bx.geo[box];
    if (h_count[s] < (uint32_t)g.n_l1_min || !g.halos) return;
    const uint32_t b0 = tpos[bx.base[box]];
    if ((int64_t)(tpos[bx.base[box + 1]] - b0) > g.halo_cap) return;
    float4 p = spos[nuc];
    uint32_t o = orig_of(p);
    const int32_t lo = (int32_t)(o - g.orig_base);
    hf_halo h;
    h.id = lo + 1;
    h.nucleus = lo;
    h.l0_id = g_label[h_gid[s]] - (int32_t)g.orig_base;
    h.n = (int32_t)h_count[s];
    h.n_enclosed = h_ienc[s];
    h.x = p.x;
    h.y = p.y;
    h.z = p.z;
    h.r = (float)cbrt((double)h_ienc[s] / g.K);
    h.mass = (float)h_count[s] * g.particle_mass;
    g.halos[tpos[o] - b0] = h;
}

// Only the halo labels to return: halo_id was filled with 0, and only the
// members of kept halos are written (scattered stores into the input order,
// so the fewer the better; their original index is read only for them).
__global__ __launch_bounds__(kBlock) void k_out_particles(int64_t n, const int32_t *__restrict__ owner,
                                                          const int32_t *__restrict__ h_label,
                                                          const float4 *__restrict__ spos,
                                                          int32_t *__restrict__ halo_id) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int own = owner[i];
    const int32_t lab = own >= 0 ? h_label[own] : 0;
    if (lab) halo_id[orig_of(spos[i])] = lab;
}

// With more than the halo labels to return: the record (density, L0 label,
// halo label) of every sorted particle stored at its original index, one
// scattered 16-byte store (one cache line) per particle instead of one per
// output array; k_out_split then writes the arrays in input order.
__global__ __launch_bounds__(kBlock) void k_out_records(int64_t n, Boxes bx, const int32_t *__restrict__ owner,
                                                        const int32_t *__restrict__ h_label,
                                                        const int32_t *__restrict__ gkey,
                                                        const float4 *__restrict__ spos,
                                                        const float *__restrict__ dens_s,
                                                        uint4 *__restrict__ rec) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int own = owner[i];
    const int32_t lab = own >= 0 ? h_label[own] : 0;
    const int32_t key = gkey[i];
    const Geo &g = bx.geo[box_of(bx, (uint32_t)i)];
    const int32_t l0 = key < 0 ? 0 : key + 1 - (int32_t)g.orig_base;
    rec[orig_of(spos[i])] = make_uint4(__float_as_uint(dens_s[i]), (uint32_t)l0, (uint32_t)lab, 0u);
}

__global__ __launch_bounds__(kBlock) void k_out_split(int64_t n, const uint4 *__restrict__ rec,
                                                      float *__restrict__ dens_out, int32_t *__restrict__ l0_out,
                                                      int32_t *__restrict__ halo_id) {
    int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    const uint4 r = rec[o];
    if (dens_out) dens_out[o] = __uint_as_float(r.x);
    if (l0_out) l0_out[o] = (int32_t)r.y;
    halo_id[o] = (int32_t)r.z;
}

// Groups with candidates in descending size, for the acceptance kernels: keys
// (~size, group) of the groups listed, padding keys sort last.
__global__ __launch_bounds__(kBlock) void k_glist_keys(int64_t len, const uint32_t *__restrict__ ngc_p,
                                                       const int32_t *__restrict__ glist,
                                                       const int32_t *__restrict__ g_size,
                                                       uint64_t *__restrict__ keys) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= len) return;
    uint64_t k = ~0ull;
    if (t < (int64_t)*ngc_p) {
        const int gi = glist[t];
        k = ((uint64_t)(0xffffffffu - (uint32_t)g_size[gi]) << 32) | (uint32_t)gi;
    }
    keys[t] = k;
}

__global__ __launch_bounds__(kBlock) void k_glist_from_keys(int64_t len, const uint32_t *__restrict__ ngc_p,
                                                            const uint64_t *__restrict__ keys,
                                                            int32_t *__restrict__ glist) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < len && t < (int64_t)*ngc_p) glist[t] = (int32_t)(keys[t] & 0xffffffffu);
}

// ------------------------------------------------------------ group order
// Members collected into group order (Sec. 2.3.5): the particles sorted by the
// table row of their halo (particles of no halo after the last row), ascending
// original index within a row.  The paper sweeps the particles with in-place
// partitions, the largest halo and the unassigned ones first; here one stable
// sort by row gives every run at once.

// key = (row, original index); row = nrows for particles of no halo.  halo_id
// is in original order with labels 1 + nucleus index; tpos maps a kept
// nucleus to its table row.
__global__ __launch_bounds__(kBlock) void k_order_keys(int64_t n, int64_t nrows,
                                                       const int32_t *__restrict__ halo_id,
                                                       const uint32_t *__restrict__ tpos,
                                                       uint64_t *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t h = halo_id[i];
    const uint64_t row = h > 0 ? (uint64_t)tpos[h - 1] : (uint64_t)nrows;
    keys[i] = (row << 32) | (uint64_t)i;
}

// members[t] from the sorted keys; halo_start[r] = first position of row r
// (the rows between two consecutive keys' rows start at the later key).
__global__ __launch_bounds__(kBlock) void k_order_out(int64_t n, int64_t nrows, const uint64_t *__restrict__ keys,
                                                      int32_t *__restrict__ members,
                                                      int64_t *__restrict__ halo_start) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > n) return;
    if (t < n) members[t] = (int32_t)(keys[t] & 0xffffffffu);
    const int64_t rp = t > 0 ? (int64_t)(keys[t - 1] >> 32) : -1;
    const int64_t rc = t < n ? (int64_t)(keys[t] >> 32) : nrows + 1;
    for (int64_t r = rp + 1; r <= rc && r <= nrows; r++) halo_start[r] = t;
}

}  // namespace

void launch_segment(int64_t n, Work &w, hipStream_t s) {
    fill_u32(w.gcnt, 0u, n + 1, s);
    hipLaunchKernelGGL(k_seg_count, grid(n), dim3(kBlock), 0, s, n, w.gkey, w.gcnt);
    scan_u32(w.gcnt, w.goff, n, w.scan_tmp, s);
    scan_nz_u32(w.gcnt, w.gidx, n, w.scan_tmp, s);  // group ordinal of every key
}

void launch_segment_groups(int64_t n, int64_t G, Work &w, hipStream_t s) {
    hipLaunchKernelGGL(k_seg_groups, grid(n), dim3(kBlock), 0, s, n, w.gcnt, w.goff, w.gidx, w.g_start,
                       w.g_size, w.g_label);
    hipLaunchKernelGGL(k_seg_scatter, grid(n), dim3(kBlock), 0, s, n, w.gkey, w.goff, w.gidx, w.gcnt,
                       w.mem, w.gid_of);
    fill_u32(w.gccnt, 0u, G + 1, s);
    fill_u32(w.gcfill, 0u, G + 1, s);
}

void launch_extent(int64_t G, int64_t M, const Boxes &bx, Work &w, hipStream_t s) {
    if (M <= 0) return;
    // flags per group in g_nh and the flagged groups in glist (both free until
    // the candidate stage fills them), their count in counters[12]
    fill_i32(w.g_nh, 0, G + 1, s);
    hipLaunchKernelGGL(k_extent_far, grid(M), dim3(kBlock), 0, s, M, bx, w.mem, w.gid_of, w.g_start, w.spos,
                       w.g_nh, w.glist, reinterpret_cast<uint32_t *>(w.counters + 12));
    const int64_t blocks = G < 1024 ? G : 1024;
    hipLaunchKernelGGL(k_extent_span, dim3((unsigned)blocks), dim3(kBlock), 0, s,
                       reinterpret_cast<const uint32_t *>(w.counters + 12), bx, w.glist, w.g_start, w.g_size,
                       w.mem, w.spos, w.err);
}

static int bits_for(int64_t x) {
    int b = 1;
    while (b < 32 && (x >> b) != 0) b++;
    return b;
}

void launch_candidates_sort(int64_t n, int64_t G, int64_t NC, Work &w, hipStream_t s) {
    // gcoff already holds the exclusive scan of gccnt
    hipLaunchKernelGGL(k_cand_scatter, grid(n), dim3(kBlock), 0, s, n, w.owner, w.gid_of, w.gcoff,
                       w.gcfill, w.cand);
    if (NC > 0)
        hipLaunchKernelGGL(k_cand_rank, grid(NC), dim3(kBlock), 0, s, NC, (int)G, w.gcoff, w.cand,
                           w.dens_s, w.spos, w.cand_sorted);
    scan_nz_u32(w.gccnt, w.gcidx, G, w.scan_tmp, s);  // ordinal of every group with candidates
    if (G > 0)
        hipLaunchKernelGGL(k_glist, grid(G), dim3(kBlock), 0, s, (int)G, w.gccnt, w.gcidx, w.glist);
    // the groups with candidates (of every box) in descending size, so that the
    // acceptance kernels start the longest walks first: a stable sort of
    // (~size, group) on the size bits (sizes are below n); the radix key
    // arrays are free at this point
    const int64_t len = G < NC ? G : NC;
    if (len > 1) {
        hipLaunchKernelGGL(k_glist_keys, grid(len), dim3(kBlock), 0, s, len, w.gcidx + G, w.glist, w.g_size,
                           w.rkey[0]);
        const uint64_t *sorted = radix_sort_keys(w.rkey[0], w.rkey[1], len, 32, bits_for(n), w, s);
        hipLaunchKernelGGL(k_glist_from_keys, grid(len), dim3(kBlock), 0, s, len, w.gcidx + G, sorted, w.glist);
    }
    fill_i32(w.h_nuc, -1, NC + 1, s);
    fill_u32(w.h_count, 0u, NC + 1, s);
    fill_i32(w.g_nh, 0, G + 1, s);
}

void launch_accept(int64_t n, int64_t G, int64_t NC, int64_t M, const Boxes &bx, Work &w, hipStream_t s) {
    // groups with candidates (at most min(G, NC)), one wavefront each; the
    // others are listed (in the free chunk-flag array, counts in counters[9]
    // and [11]) for one workgroup each: medium groups (at most M / kWaveHist
    // of kWaveHist particles or more, and NC / (kWaveNuc + 1) with more than
    // kWaveNuc candidates) and large ones (at most M / kHistMid), whose list
    // starts halfway through the array.  The first kernel is a persistent
    // grid (as many wavefronts as fit on the chip at once) striding over the
    // list; the others run one workgroup per listed group.  The counts are
    // zero since the call began.
    const int64_t bound = G < NC ? G : NC;
    if (bound <= 0) return;
    int32_t *mid_list = reinterpret_cast<int32_t *>(w.f_chunk);
    int32_t *big_list = reinterpret_cast<int32_t *>(w.f_chunk) + n / 2;
    uint32_t *mid_count = reinterpret_cast<uint32_t *>(w.counters + 9);
    uint32_t *big_count = reinterpret_cast<uint32_t *>(w.counters + 11);
    const int64_t ncu = w.ncu > 0 ? w.ncu : 1;
    auto cap = [](int64_t a, int64_t b) { return (unsigned)(a < b ? a : b); };
    const bool bins = w.radius_bins;
    // six wavefronts per SIMD (its register use): 6 workgroups of 4 per CU
    hipLaunchKernelGGL(k_accept_small, dim3(cap((bound + kBlock / 64 - 1) / (kBlock / 64), 6 * ncu)), dim3(kBlock),
                       0, s, w.gcidx + G, bins, bx, w.glist, w.g_start, w.g_size, w.gcoff, w.cand_sorted,
                       w.mem, w.spos, w.h_nuc, w.h_ienc, w.h_gid, w.g_nh, mid_list, mid_count, big_list, big_count);
    // with radial bins every group is listed: at most bound medium groups
    const int64_t nmid = bins ? bound : M / kWaveHist + NC / (kWaveNuc + 1) + 1;
    const dim3 gmid(cap(nmid, bound));
    // the large groups are few and each is a serial walk: 1024 threads and a
    // 144 KB LDS histogram each (one workgroup per CU)
    const int64_t nbig = M / kHistMid + 1;
    const dim3 gbig(cap(nbig, bound));
    if (bins) {
        hipLaunchKernelGGL((k_accept<kBlock, kHistMid, true>), gmid, dim3(kBlock), 0, s, mid_count, bx,
                           mid_list, w.g_start, w.g_size, w.gcoff, w.cand_sorted, w.mem, w.spos, w.hist, w.h_nuc,
                           w.h_ienc, w.h_gid, w.g_nh);
        hipLaunchKernelGGL((k_accept<1024, kHistBig, true>), gbig, dim3(1024), 0, s, big_count, bx,
                           big_list, w.g_start, w.g_size, w.gcoff, w.cand_sorted, w.mem, w.spos, w.hist, w.h_nuc,
                           w.h_ienc, w.h_gid, w.g_nh);
    } else {
        hipLaunchKernelGGL((k_accept<kBlock, kHistMid, false>), gmid, dim3(kBlock), 0, s, mid_count, bx,
                           mid_list, w.g_start, w.g_size, w.gcoff, w.cand_sorted, w.mem, w.spos, w.hist, w.h_nuc,
                           w.h_ienc, w.h_gid, w.g_nh);
        hipLaunchKernelGGL((k_accept<1024, kHistBig, false>), gbig, dim3(1024), 0, s, big_count, bx,
                           big_list, w.g_start, w.g_size, w.gcoff, w.cand_sorted, w.mem, w.spos, w.hist, w.h_nuc,
                           w.h_ienc, w.h_gid, w.g_nh);
    }
}

void launch_assign(int64_t n, const Boxes &bx, Work &w, hipStream_t s) {
    hipLaunchKernelGGL(k_assign, grid(n), dim3(kBlock), 0, s, n, bx, w.gid_of, w.gcoff, w.g_nh, w.h_nuc,
                       w.h_ienc, w.spos, w.owner, w.h_count);
}

void launch_output_flags(int64_t n, int64_t NC, const Boxes &bx, Work &w, hipStream_t s) {
    fill_u32(w.tflag, 0u, n + 1, s);
    if (NC > 0)
        // the candidates' member labels go to the hard-case list (free after
        // the candidate stage)
        hipLaunchKernelGGL(k_out_flags, grid(NC), dim3(kBlock), 0, s, NC, bx, w.h_nuc, w.h_count, w.spos,
                           w.tflag, w.hardlist, w.counters);
    scan_u32(w.tflag, w.tpos, n, w.scan_tmp, s);
}

void launch_output(int64_t n, int64_t NC, const Boxes &bx, Work &w, int32_t *halo_id, int32_t *l0_out,
                   float *dens_out, int64_t *box_rows, hipStream_t s) {
    if (NC > 0)
        hipLaunchKernelGGL(k_out_table, grid(NC), dim3(kBlock), 0, s, NC, bx, w.h_nuc, w.h_ienc, w.h_gid,
                           w.h_count, w.g_label, w.spos, w.tpos);
    if (box_rows)
        hipLaunchKernelGGL(k_box_rows, grid(bx.nbox), dim3(kBlock), 0, s, bx, w.tpos, box_rows);
    if (!l0_out && !dens_out) {
        fill_i32(halo_id, 0, n, s);
        hipLaunchKernelGGL(k_out_particles, grid(n), dim3(kBlock), 0, s, n, w.owner, w.hardlist, w.spos,
                           halo_id);
        return;
    }
    // records in the radix key block (2n words, free at this point)
    uint4 *rec = reinterpret_cast<uint4 *>(w.rkey[0]);
    hipLaunchKernelGGL(k_out_records, grid(n), dim3(kBlock), 0, s, n, bx, w.owner, w.hardlist, w.gkey, w.spos,
                       w.dens_s, rec);
    hipLaunchKernelGGL(k_out_split, grid(n), dim3(kBlock), 0, s, n, rec, dens_out, l0_out, halo_id);
}

void launch_group_order(int64_t n, int64_t nrows, const int32_t *halo_id, Work &w, int32_t *members,
                        int64_t *halo_start, hipStream_t s) {
    // the radix key arrays are free once the output is written
    hipLaunchKernelGGL(k_order_keys, grid(n), dim3(kBlock), 0, s, n, nrows, halo_id, w.tpos, w.rkey[0]);
    const uint64_t *sorted = radix_sort_keys(w.rkey[0], w.rkey[1], n, 32, bits_for(nrows + 1), w, s);
    hipLaunchKernelGGL(k_order_out, grid(n + 1), dim3(kBlock), 0, s, n, nrows, sorted, members, halo_start);
}

}  // namespace hf
