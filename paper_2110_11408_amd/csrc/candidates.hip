// Nucleus candidates (Sec. 2.2.2, steps 2 and 4): a member of an L0 group is a
// candidate when its density is at least the nucleation floor and no denser
// particle of the same group (eligible or not) lies within b.  "Denser" is the
// total order (density, then lower original index).  Candidacy depends only on
// the densities and the groups, so it is decided for all particles at once,
// before the sequential part of CompaSO.
//
// Two stages: most particles are settled by the densest particle of their own
// sub-cell; the rest (sub-cell maxima and particles of sparse cells) search
// their neighbourhood with sub-cell pruning.
#include "hf_internal.h"

namespace hf {

namespace {

// Neighbour cell t of 27 in order of distance: own cell, the 6 face
// neighbours, the 12 edge neighbours, the 8 corners.
__constant__ int8_t kStencil[27] = {13, 4, 10, 12, 14, 16, 22, 1,  3,  5,  7,  9,  11, 15,
                                    17, 19, 21, 23, 25, 0, 2,  6,  8,  18, 20, 24, 26};

__device__ __forceinline__ void stencil_offset(int t, int &ox, int &oy, int &oz) {
    const int u = kStencil[t];
    ox = u % 3 - 1;
    oy = (u / 3) % 3 - 1;
    oz = u / 9 - 1;
}

// j is a denser particle of the same group within b.  Its group key and
// position are loaded together (one round trip: the searches wait on memory,
// not on arithmetic), and the distance is the canonical FP64 one.
__device__ __forceinline__ bool denser_within_b(int64_t j, const float *__restrict__ dens_s,
                                                const int32_t *__restrict__ gkey,
                                                const float4 *__restrict__ spos, int key, float di,
                                                uint32_t oi, const float4 &pi, const Geo &g) {
    const float dj = dens_s[j];
    const int kj = gkey[j];
    const float4 pj = spos[j];
    if (dj < di || kj != key) return false;
    if (!denser(dj, orig_of(pj), di, oi)) return false;
    return d2_exact(pi, pj, g.L, g.half) < g.b2;
}

// Densest particle of every sub-cell of a dense cell, as a packed key
// (density bits, inverted original index): larger key = denser in the total
// order (densities are >= 0, so their bit patterns order like the values).
__device__ __forceinline__ uint64_t dkey(float d, uint32_t orig) {
    return ((uint64_t)__float_as_uint(d) << 32) | (uint64_t)(0xffffffffu - orig);
}

// Slot t = (dense cell d, sub-cell s < nsub_max); sub-cells beyond the cell's
// own box's count are left alone.
__global__ __launch_bounds__(kBlock) void k_submax(int64_t nslots, Boxes bx,
                                                   const uint32_t *__restrict__ dcells,
                                                   const uint32_t *__restrict__ off,
                                                   const uint32_t *__restrict__ subtab,
                                                   const float *__restrict__ dens_s,
                                                   const float4 *__restrict__ spos,
                                                   uint64_t *__restrict__ submax,
                                                   int32_t *__restrict__ subarg) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslots) return;
    const int nsub = bx.nsub_max;
    const int64_t d = t / nsub;
    const int s = (int)(t - d * nsub);
    if (s >= bx.geo[box_of(bx, off[dcells[d]])].nsub) return;
    const uint32_t *tab = subtab + d * (nsub + 1);
    uint64_t best = 0;
    int32_t arg = -1;
    for (uint32_t j = tab[s]; j < tab[s + 1]; j++) {
        const uint64_t kk = dkey(dens_s[j], orig_of(spos[j]));
        if (arg < 0 || kk > best) {
            best = kk;
            arg = (int32_t)j;
        }
    }
    submax[d * (nsub + 1) + s] = best;
    subarg[d * (nsub + 1) + s] = arg;
}

// The same table with one wavefront per dense cell, for at most 64 sub-cells:
// the cell's particles are sorted by sub-cell, so each 64-particle step
// reduces the runs of equal sub-cells (maximum key and its particle) and the
// first lane of each run merges the result into the cell's row in LDS.
__global__ __launch_bounds__(kBlock) void k_submax_wave(int64_t ndc, Boxes bx,
                                                        const uint32_t *__restrict__ dcells,
                                                        const uint32_t *__restrict__ off,
                                                        const uint16_t *__restrict__ ssub,
                                                        const float *__restrict__ dens_s,
                                                        const float4 *__restrict__ spos,
                                                        uint64_t *__restrict__ submax,
                                                        int32_t *__restrict__ subarg) {
    __shared__ uint64_t s_best[kBlock / 64][64];
    __shared__ int32_t s_arg[kBlock / 64][64];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t d = (int64_t)blockIdx.x * (kBlock / 64) + wave;
    if (d >= ndc) return;
    const int lane = threadIdx.x & 63;
    const uint32_t c = (uint32_t)__builtin_amdgcn_readfirstlane(dcells[d]);
    const uint32_t a = (uint32_t)__builtin_amdgcn_readfirstlane(off[c]);
    const uint32_t b = (uint32_t)__builtin_amdgcn_readfirstlane(off[c + 1]);
    const int nsub = __builtin_amdgcn_readfirstlane(bx.geo[box_of(bx, a)].nsub);
    const int64_t row = d * (bx.nsub_max + 1);
    s_best[wave][lane] = 0ull;
    s_arg[wave][lane] = -1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (uint32_t j0 = a; j0 < b; j0 += 64) {
        const uint32_t j = j0 + (uint32_t)lane;
        const bool act = j < b;
        const int v = act ? (int)ssub[j] : -1 - lane;  // inactive lanes: runs of their own
        uint64_t kk = act ? dkey(dens_s[j], orig_of(spos[j])) : 0ull;
        int32_t jj = (int32_t)j;
        const WaveRun run = wave_run(v);
        const int end = run.head + run.len;
        for (int dd = 1; dd < 64; dd <<= 1) {
            const uint32_t olo = __shfl_down((uint32_t)kk, dd, 64), ohi = __shfl_down((uint32_t)(kk >> 32), dd, 64);
            const int32_t oj = __shfl_down(jj, dd, 64);
            const uint64_t ok = ((uint64_t)ohi << 32) | olo;
            if (lane + dd < end && ok > kk) {
                kk = ok;
                jj = oj;
            }
        }
        if (act && run.rank == 0 && (s_arg[wave][v] < 0 || kk > s_best[wave][v])) {
            s_best[wave][v] = kk;
            s_arg[wave][v] = jj;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
    if (lane < nsub) {
        submax[row + lane] = s_best[wave][lane];
        subarg[row + lane] = s_arg[wave][lane];
    }
}

// Stage 1, one thread per particle: a member at or above the floor that is not
// the densest particle of its sub-cell is decided at once when that densest
// particle belongs to its group and lies within b (the usual case inside an L0
// group, the sub-cell diagonal being below l).  A member that is its
// sub-cell's densest is decided when the densest particle of a face-adjacent
// sub-cell of the same cell is denser and in its group, where such sub-cells
// lie within b of each other entirely (s sqrt(6) < b).  Every other member at
// or above the floor is flagged as a hard case.
__global__ __launch_bounds__(kBlock) void k_cand_quick(int64_t n, Boxes bx, const float4 *__restrict__ sloc,
                                                       const float4 *__restrict__ spos,
                                                       const uint32_t *__restrict__ f_sparse,
                                                       const uint16_t *__restrict__ ssub,
                                                       const uint32_t *__restrict__ cellmap,
                                                       const uint64_t *__restrict__ submax,
                                                       const int32_t *__restrict__ subarg,
                                                       const float *__restrict__ dens_s,
                                                       const int32_t *__restrict__ gkey,
                                                       int32_t *__restrict__ cflag,
                                                       uint32_t *__restrict__ f_hard) {
    const int64_t i = (int64_t)xcd_block() * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Geo &g = bx.geo[box_of(bx, (uint32_t)i)];
    bool is_hard = false;
    cflag[i] = 0;
    const int key = gkey[i];
    const float di = dens_s[i];
    if (key >= 0 && (double)di >= g.floor_nuc) {
        is_hard = true;
        // everything indexed by i in one round of loads
        const uint32_t c = __float_as_uint(sloc[i].w);
        const uint32_t sparse_i = f_sparse[i];
        const int si = ssub[i];
        const float4 pi = spos[i];
        if (!sparse_i) {
            const int64_t base = (int64_t)cellmap[c] * (bx.nsub_max + 1);
            const int32_t top = subarg[base + si];
            const uint32_t oi = orig_of(pi);
            if (top != (int32_t)i) {
                // top, the maximum of i's sub-cell, is denser than i (the bit
                // order of the key matches the values for the non-negative
                // densities the stage works on; checked anyway); its key,
                // density and position are loaded together
                const int kt = gkey[top];
                const float dt = dens_s[top];
                const float4 pt = spos[top];
                if (kt == key && denser(dt, orig_of(pt), di, oi) && d2_exact(pi, pt, g.L, g.half) < g.b2)
                    is_hard = false;
            } else if (g.face_sub_in_b) {
                // the six face-adjacent sub-cells at once: their maxima, then
                // the particles that hold them, then those particles' keys
                const int k = g.ksub;
                const int sz = div_small(si, 1.0f / (float)(k * k)), syx = si - sz * k * k,
                          sy = div_small(syx, 1.0f / (float)k), sx = syx - sy * k;
                const uint64_t mykey = dkey(di, oi);
                int s2[6];
                uint64_t mx[6];
#pragma unroll
                for (int f = 0; f < 6; f++) {
                    const int ax = f >> 1, dir = (f & 1) ? 1 : -1;
                    const int nx = sx + (ax == 0 ? dir : 0), ny = sy + (ax == 1 ? dir : 0),
                              nz = sz + (ax == 2 ? dir : 0);
                    const bool in = nx >= 0 && nx < k && ny >= 0 && ny < k && nz >= 0 && nz < k;
                    s2[f] = in ? (nz * k + ny) * k + nx : -1;
                    mx[f] = in ? submax[base + s2[f]] : 0ull;
                }
                int32_t t2[6];
#pragma unroll
                for (int f = 0; f < 6; f++) t2[f] = mx[f] > mykey ? subarg[base + s2[f]] : -1;
                int kt[6];
                float dt[6];
                uint32_t ot[6];
#pragma unroll
                for (int f = 0; f < 6; f++) {
                    kt[f] = -1;
                    dt[f] = 0.0f;
                    ot[f] = 0u;
                    if (t2[f] >= 0) {
                        kt[f] = gkey[t2[f]];
                        dt[f] = dens_s[t2[f]];
                        ot[f] = orig_of(spos[t2[f]]);
                    }
                }
#pragma unroll
                for (int f = 0; f < 6; f++)
                    if (t2[f] >= 0 && kt[f] == key && denser(dt[f], ot[f], di, oi)) is_hard = false;
            }
        }
    }
    f_hard[i] = is_hard ? 1u : 0u;
}

// Four particles per thread (i0, i0 + kBlock, ...), their flags loaded
// together: the kernel streams the flags, and one load in flight per thread
// leaves most of the bandwidth unused.
constexpr int kHardIlp = 4;
__global__ __launch_bounds__(kBlock) void k_hard_list(int64_t n, const uint32_t *__restrict__ f_hard,
                                                      const uint32_t *__restrict__ s_hard,
                                                      int32_t *__restrict__ hard) {
    const int64_t i0 = (int64_t)blockIdx.x * (kBlock * kHardIlp) + threadIdx.x;
    uint32_t f[kHardIlp];
#pragma unroll
    for (int u = 0; u < kHardIlp; u++) {
        const int64_t i = i0 + (int64_t)u * kBlock;
        f[u] = i < n ? f_hard[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kHardIlp; u++) {
        const int64_t i = i0 + (int64_t)u * kBlock;
        if (f[u]) hard[s_hard[i]] = (int32_t)i;
    }
}

// Whether particle i has a denser particle of its group within b in the
// stencil cells tt0..tt1-1 (cell 0 of the order is its own).  In dense cells
// only sub-cells within b that hold a denser particle are visited, their
// densest particle first.
__device__ bool has_denser_within_b(int i, int tt0, int tt1, const Geo &g, int tstride,
                                    const float4 *__restrict__ sloc,
                                    const float4 *__restrict__ spos, const uint32_t *__restrict__ off,
                                    const uint32_t *__restrict__ cellmap, const uint32_t *__restrict__ subtab,
                                    const uint64_t *__restrict__ submax, const int32_t *__restrict__ subarg,
                                    const float *__restrict__ dens_s, const int32_t *__restrict__ gkey) {
    const int key = gkey[i];
    const float di = dens_s[i];
    const float4 li = sloc[i];
    const float4 pi = spos[i];
    const uint32_t oi = orig_of(pi);
    const uint64_t mykey = dkey(di, oi);
    const uint32_t c = __float_as_uint(li.w);
    const int k = g.ksub, nsub = g.nsub;
    const float subb = g.cellb / (float)k, inv_k = 1.0f / (float)k, inv_k2 = 1.0f / (float)(k * k);
    int cx, cy, cz;
    cell_xyz(g, c, cx, cy, cz);
    for (int tt = tt0; tt < tt1; tt++) {
        int ox, oy, oz;
        stencil_offset(tt, ox, oy, oz);
        const float xs = li.x - (float)ox * g.cellb, ys = li.y - (float)oy * g.cellb,
                    zs = li.z - (float)oz * g.cellb;
        // nothing of this cell lies within b
        const float gx = ox < 0 ? li.x : (ox > 0 ? g.cellb - li.x : 0.0f);
        const float gy = oy < 0 ? li.y : (oy > 0 ? g.cellb - li.y : 0.0f);
        const float gz = oz < 0 ? li.z : (oz > 0 ? g.cellb - li.z : 0.0f);
        if (gx * gx + gy * gy + gz * gz >= g.b2b_hi) continue;
        const uint32_t nb = cell_id(g, cx + ox, cy + oy, cz + oz);
        const uint32_t a = off[nb], b = off[nb + 1];
        if (b - a < (uint32_t)kDenseMin) {
            // sparse cell: densities four at a time (their loads together),
            // then the few denser ones in full
            for (uint32_t a0 = a; a0 < b; a0 += 4) {
                float dj[4];
#pragma unroll
                for (int u = 0; u < 4; u++) dj[u] = a0 + u < b ? dens_s[a0 + u] : -1.0f;
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const uint32_t j = a0 + u;
                    if (dj[u] < di || (int)j == i) continue;
                    if (denser_within_b(j, dens_s, gkey, spos, key, di, oi, pi, g)) return true;
                }
            }
            continue;
        }
        const int64_t base = (int64_t)cellmap[nb] * tstride;
        for (int s0 = 0; s0 < nsub; s0 += 3) {
            // three sub-cell maxima per round of loads (the thread-per-case
            // kernel waits on memory: small batches keep it at eight
            // wavefronts per SIMD, which hide more than longer batches would)
            uint64_t mx[3];
#pragma unroll
            for (int u = 0; u < 3; u++) mx[u] = s0 + u < nsub ? submax[base + s0 + u] : 0ull;
#pragma unroll
            for (int u = 0; u < 3; u++) {
                const int s2 = s0 + u;
                if (!(mx[u] > mykey)) continue;
                const int sz = div_small(s2, inv_k2), syx = s2 - sz * k * k, sy = div_small(syx, inv_k),
                          sx = syx - sy * k;
                const float ex = fmaxf(fmaxf(sx * subb - 1e-5f - xs, xs - (sx + 1) * subb - 1e-5f), 0.0f);
                const float ey = fmaxf(fmaxf(sy * subb - 1e-5f - ys, ys - (sy + 1) * subb - 1e-5f), 0.0f);
                const float ez = fmaxf(fmaxf(sz * subb - 1e-5f - zs, zs - (sz + 1) * subb - 1e-5f), 0.0f);
                if (ex * ex + ey * ey + ez * ez >= g.b2b_hi) continue;
                const int32_t top = subarg[base + s2];
                if (denser_within_b(top, dens_s, gkey, spos, key, di, oi, pi, g)) return true;
                // the rest of the sub-cell: densities four at a time, then the
                // denser ones in full
                const uint32_t u1 = subtab[base + s2 + 1];
                for (uint32_t j0 = subtab[base + s2]; j0 < u1; j0 += 4) {
                    float dj[4];
#pragma unroll
                    for (int v = 0; v < 4; v++) dj[v] = j0 + v < u1 ? dens_s[j0 + v] : -1.0f;
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const uint32_t j = j0 + v;
                        if (dj[v] < di || (int32_t)j == top || (int)j == i) continue;
                        if (denser_within_b(j, dens_s, gkey, spos, key, di, oi, pi, g))
                            return true;
                    }
                }
            }
        }
    }
    return false;
}

// Hard cases, one thread each, searching the stencil cells tt0..tt1-1: the
// particle's own cell (stage 1, where a denser neighbour is nearly always
// found), then the face neighbours (stage 2).  With `rest`, the cases left are
// appended to it (one atomic per wavefront), so that the few exhaustive
// searches (mostly the actual candidates) do not hold up waves of quick ones;
// without it, the cases left are candidates.  Held to 64 VGPRs (eight
// wavefronts per SIMD): a few values spill to scratch, which costs less than
// the two wavefronts per SIMD it buys.
__global__ __launch_bounds__(kBlock, 8) void k_cand_hard(const uint32_t *__restrict__ nhard_p, int stage, int tt0,
                                                      int tt1, Boxes bx,
                                                      const int32_t *__restrict__ hard,
                                                      const float4 *__restrict__ sloc,
                                                      const float4 *__restrict__ spos,
                                                      const uint32_t *__restrict__ off,
                                                      const uint32_t *__restrict__ cellmap,
                                                      const uint32_t *__restrict__ subtab,
                                                      const uint64_t *__restrict__ submax,
                                                      const int32_t *__restrict__ subarg,
                                                      const float *__restrict__ dens_s,
                                                      const int32_t *__restrict__ gkey,
                                                      const int32_t *__restrict__ gid_of,
                                                      uint32_t *__restrict__ gccnt,
                                                      int32_t *__restrict__ cflag,
                                                      int32_t *__restrict__ rest,
                                                      uint32_t *__restrict__ nrest) {
    // a list built on the device fills only the first blocks of its grid:
    // those are spread over all XCDs by the plain block order, not gathered
    // on one
    const int64_t t = (int64_t)(stage == 1 ? xcd_block() : blockIdx.x) * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = t < (int64_t)*nhard_p;
    const int i = valid ? hard[t] : -1;
    bool left = false;
    if (valid && !has_denser_within_b(i, tt0, tt1, bx.geo[box_of(bx, (uint32_t)i)], bx.nsub_max + 1, sloc, spos,
                                      off, cellmap, subtab, submax, subarg, dens_s, gkey)) {
        if (rest) {
            left = true;
        } else {
            cflag[i] = 1;
            atomicAdd(&gccnt[gid_of[i]], 1u);
        }
    }
    if (!rest) return;
    // append the cases left: one atomic per wavefront
    const uint64_t m = __ballot(left);
    if (m == 0ull) return;
    const int leader = __ffsll((unsigned long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(nrest, (uint32_t)__popcll(m));
    base = lane_get(base, leader);
    if (left) rest[base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = i;
}

// Stage 3, one wavefront per case (grid-stride over the list, its length read
// on the device): the stencil cells tt0..26 are searched by all lanes at once.
// A lane takes one stencil cell (its range; the particles of a sparse cell),
// then the sub-cells of the dense cells are taken 64 at a time (densest
// particle first, then the rest of the sub-cell); the wavefront stops at the
// first denser particle of the group within b.  The cases that reach this
// stage are mostly the true candidates, which need every cell.
__global__ __launch_bounds__(kBlock) void k_cand_wave(const uint32_t *__restrict__ ncase_p, int tt0, Boxes bx,
                                                      const int32_t *__restrict__ cases,
                                                      const float4 *__restrict__ sloc,
                                                      const float4 *__restrict__ spos,
                                                      const uint32_t *__restrict__ off,
                                                      const uint32_t *__restrict__ cellmap,
                                                      const uint32_t *__restrict__ subtab,
                                                      const uint64_t *__restrict__ submax,
                                                      const int32_t *__restrict__ subarg,
                                                      const float *__restrict__ dens_s,
                                                      const int32_t *__restrict__ gkey,
                                                      const int32_t *__restrict__ gid_of,
                                                      uint32_t *__restrict__ gccnt,
                                                      int32_t *__restrict__ cflag) {
    __shared__ int64_t s_base[kBlock / 64][27];  // sub-table base of the lane's dense cells
    __shared__ int8_t s_tt[kBlock / 64][27];     // and their stencil order index
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const uint32_t ncase = *ncase_p;
    const uint32_t nwaves = gridDim.x * (kBlock / 64);
    const int tstride = bx.nsub_max + 1;
    for (uint32_t q = blockIdx.x * (kBlock / 64) + (uint32_t)wave; q < ncase; q += nwaves) {
        const int i = __builtin_amdgcn_readfirstlane(cases[q]);
        const Geo &g = bx.geo[__builtin_amdgcn_readfirstlane(box_of(bx, (uint32_t)i))];
        const int k = g.ksub, nsub = g.nsub;
        const float subb = g.cellb / (float)k;
        const int key = gkey[i];
        const float di = dens_s[i];
        const float4 li = sloc[i];
        const float4 pi = spos[i];
        const uint32_t oi = orig_of(pi);
        const uint64_t mykey = dkey(di, oi);
        const uint32_t c = __float_as_uint(li.w);
        int cx, cy, cz;
        cell_xyz(g, c, cx, cy, cz);
        // one stencil cell per lane
        const int tt = tt0 + lane;
        bool in_reach = false, dense = false, found = false;
        float xs = 0.0f, ys = 0.0f, zs = 0.0f;
        uint32_t a = 0, b = 0, nb = 0;
        if (tt < 27) {
            int ox, oy, oz;
            stencil_offset(tt, ox, oy, oz);
            xs = li.x - (float)ox * g.cellb;
            ys = li.y - (float)oy * g.cellb;
            zs = li.z - (float)oz * g.cellb;
            const float gx = ox < 0 ? li.x : (ox > 0 ? g.cellb - li.x : 0.0f);
            const float gy = oy < 0 ? li.y : (oy > 0 ? g.cellb - li.y : 0.0f);
            const float gz = oz < 0 ? li.z : (oz > 0 ? g.cellb - li.z : 0.0f);
            in_reach = gx * gx + gy * gy + gz * gz < g.b2b_hi;
            if (in_reach) {
                nb = cell_id(g, cx + ox, cy + oy, cz + oz);
                a = off[nb];
                b = off[nb + 1];
                dense = b - a >= (uint32_t)kDenseMin;
            }
        }
        // sparse cells: the lane's own particles
        if (in_reach && !dense) {
            for (uint32_t j = a; j < b && !found; j++)
                if ((int)j != i && dens_s[j] >= di &&
                    denser_within_b(j, dens_s, gkey, spos, key, di, oi, pi, g))
                    found = true;
        }
        if (__ballot(found)) continue;
        // dense cells: their sub-table bases, then (cell, sub-cell) tasks
        const uint64_t dm = __ballot(in_reach && dense);
        if (dm == 0ull) {
            if (lane == 0) {
                cflag[i] = 1;
                atomicAdd(&gccnt[gid_of[i]], 1u);
            }
            continue;
        }
        if (in_reach && dense) {
            const int slot = __popcll(dm & ((1ull << lane) - 1ull));
            s_base[wave][slot] = (int64_t)cellmap[nb] * tstride;
            s_tt[wave][slot] = (int8_t)tt;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        const int ntask = __popcll(dm) * nsub;
        for (int t0 = 0; t0 < ntask; t0 += 64) {
            const int tq = t0 + lane;
            if (tq < ntask) {
                const int r = div_small(tq, 1.0f / (float)nsub), sl = tq - r * nsub;
                const int64_t base = s_base[wave][r];
                if (submax[base + sl] > mykey) {
                    int ox, oy, oz;
                    stencil_offset(s_tt[wave][r], ox, oy, oz);
                    const float txs = li.x - (float)ox * g.cellb, tys = li.y - (float)oy * g.cellb,
                                tzs = li.z - (float)oz * g.cellb;
                    const int sz = div_small(sl, 1.0f / (float)(k * k)), syx = sl - sz * k * k,
                              sy = div_small(syx, 1.0f / (float)k), sx = syx - sy * k;
                    const float ex = fmaxf(fmaxf(sx * subb - 1e-5f - txs, txs - (sx + 1) * subb - 1e-5f), 0.0f);
                    const float ey = fmaxf(fmaxf(sy * subb - 1e-5f - tys, tys - (sy + 1) * subb - 1e-5f), 0.0f);
                    const float ez = fmaxf(fmaxf(sz * subb - 1e-5f - tzs, tzs - (sz + 1) * subb - 1e-5f), 0.0f);
                    if (ex * ex + ey * ey + ez * ez < g.b2b_hi) {
                        const int32_t top = subarg[base + sl];
                        found = denser_within_b(top, dens_s, gkey, spos, key, di, oi, pi, g);
                        const uint32_t u1 = subtab[base + sl + 1];
                        for (uint32_t j = subtab[base + sl]; j < u1 && !found; j++)
                            if ((int32_t)j != top && (int)j != i && dens_s[j] >= di &&
                                denser_within_b(j, dens_s, gkey, spos, key, di, oi, pi, g))
                                found = true;
                    }
                }
            }
            if (__ballot(found)) break;
        }
        if (!__ballot(found) && lane == 0) {
            cflag[i] = 1;
            atomicAdd(&gccnt[gid_of[i]], 1u);
        }
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace

void launch_candidates(int64_t n, const Boxes &bx, Work &w, hipStream_t s) {
    const int nsub = bx.nsub_max;
    const int64_t nslots = w.ndcells * nsub;
    if (nslots > 0 && nsub <= 64)
        hipLaunchKernelGGL(k_submax_wave, dim3((unsigned)((w.ndcells + kBlock / 64 - 1) / (kBlock / 64))),
                           dim3(kBlock), 0, s, w.ndcells, bx, w.dcells, w.off, w.ssub, w.dens_s, w.spos, w.submax,
                           w.subarg);
    else if (nslots > 0)
        hipLaunchKernelGGL(k_submax, dim3((unsigned)((nslots + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           nslots, bx, w.dcells, w.off, w.subtab, w.dens_s, w.spos, w.submax, w.subarg);
    const unsigned blocks = (unsigned)((n + kBlock - 1) / kBlock);
    // candidate flags live in the owner array until the assignment overwrites
    // it; the hard-case flags and their scan reuse the dense-cell flag arrays
    hipLaunchKernelGGL(k_cand_quick, dim3(blocks), dim3(kBlock), 0, s, n, bx, w.sloc, w.spos, w.f_sparse, w.ssub,
                       w.cnt, w.submax, w.subarg, w.dens_s, w.gkey, w.owner, w.f_dcell);
    scan_u32(w.f_dcell, w.s_dcell, n, w.scan_tmp, s);
    hipLaunchKernelGGL(k_hard_list, dim3((unsigned)((n + kBlock * kHardIlp - 1) / (kBlock * kHardIlp))), dim3(kBlock),
                       0, s, n, w.f_dcell, w.s_dcell, w.hardlist);
    uint32_t nh = 0;
    WordSrc src{};
    src.p[0] = w.s_dcell + n;
    if (read_words(src, 1, w.host, &nh, s) != hipSuccess) nh = 0;  // the caller's next read reports it
    w.nhard = nh;
    if (nh > 0) {
        // three stages, each on the cases the one before left, listed on the
        // device (counts in counters[8] and [10]; surplus threads exit):
        // the own cell and the 6 face neighbours one thread per case, then the
        // 20 edge and corner neighbours one wavefront per case.  The first
        // list is kept in the (free) chunk-flag array, the second in the hard
        // list, which stage 1 has read by then.
        int32_t *rest1 = reinterpret_cast<int32_t *>(w.f_chunk);
        int32_t *rest2 = w.hardlist;
        uint32_t *n1 = reinterpret_cast<uint32_t *>(w.counters + 8);
        uint32_t *n2 = reinterpret_cast<uint32_t *>(w.counters + 10);
        fill_u32(n1, 0u, 3, s);  // counters 8..10 (9 is the acceptance's, also zero here)
        const dim3 grid((unsigned)((nh + kBlock - 1) / kBlock));
        hipLaunchKernelGGL(k_cand_hard, grid, dim3(kBlock), 0, s, w.s_dcell + n, 1, 0, 1, bx, w.hardlist, w.sloc,
                           w.spos, w.off, w.cnt, w.subtab, w.submax, w.subarg, w.dens_s, w.gkey, w.gid_of,
                           w.gccnt, w.owner, rest1, n1);
        hipLaunchKernelGGL(k_cand_hard, grid, dim3(kBlock), 0, s, n1, 2, 1, 7, bx, rest1, w.sloc, w.spos, w.off,
                           w.cnt, w.subtab, w.submax, w.subarg, w.dens_s, w.gkey, w.gid_of, w.gccnt, w.owner,
                           rest2, n2);
        // a fixed grid of wavefronts striding over the list
        const int64_t waves = nh < 8192 ? nh : 8192;
        hipLaunchKernelGGL(k_cand_wave, dim3((unsigned)((waves + kBlock / 64 - 1) / (kBlock / 64))), dim3(kBlock), 0,
                           s, n2, 7, bx, rest2, w.sloc, w.spos, w.off, w.cnt, w.subtab, w.submax, w.subarg,
                           w.dens_s, w.gkey, w.gid_of, w.gccnt, w.owner);
    }
}

}  // namespace hf
