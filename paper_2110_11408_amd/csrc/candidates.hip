// Nucleus candidates (Sec. 2.2.2, steps 2 and 4): a member of an L0 group is a
// candidate when its density is at least the nucleation floor and no denser
// particle of the same group (eligible or not) lies within b.  "Denser" is the
// total order (density, then lower original index).  Candidacy depends only on
// the densities and the groups, so it is decided for all particles at once,
// before the sequential part of CompaSO.
//
// Dense cells: one wavefront per chunk of <= 64 particles; every lane tests its
// own particle against the same neighbour stream (own cell first, where a
// denser neighbour is most likely), and the wave leaves as soon as every
// active lane has found a denser neighbour.  Sparse cells: one thread each.
#include "hf_internal.h"

namespace hf {

namespace {

// Neighbour cell t of 27, own cell first.
__device__ __forceinline__ void stencil_offset(int t, int &ox, int &oy, int &oz) {
    const int u = t == 0 ? 13 : (t <= 13 ? t - 1 : t);
    ox = u % 3 - 1;
    oy = (u / 3) % 3 - 1;
    oz = u / 9 - 1;
}

__device__ __forceinline__ bool denser_within_b(float dj, uint32_t oj, int kj, float4 lj, float4 pj,
                                                int key, float di, uint32_t oi, float xs, float ys,
                                                float zs, const float4 &pi, const Geo &g) {
    if (kj != key || !denser(dj, oj, di, oi)) return false;
    const float dx = lj.x - xs, dy = lj.y - ys, dz = lj.z - zs;
    const float d2f = dx * dx + dy * dy + dz * dz;
    if (d2f >= g.b2b_hi) return false;
    if (d2f < g.b2b_lo) return true;
    return d2_exact(pi, pj, g.L, g.half) < g.b2;
}

__global__ __launch_bounds__(kBlock) void k_cand_dense(int64_t nchunks, Geo g,
                                                       const int32_t *__restrict__ chunks,
                                                       const float4 *__restrict__ sloc,
                                                       const float4 *__restrict__ spos,
                                                       const uint32_t *__restrict__ off,
                                                       const float *__restrict__ dens_s,
                                                       const int32_t *__restrict__ gkey,
                                                       const int32_t *__restrict__ gid_of,
                                                       uint32_t *__restrict__ gccnt,
                                                       int32_t *__restrict__ cflag) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t q = (int64_t)blockIdx.x * (kBlock / 64) + wave;
    if (q >= nchunks) return;
    const int lane = threadIdx.x & 63;
    const uint32_t h = (uint32_t)__builtin_amdgcn_readfirstlane(chunks[q]);
    const uint32_t c = __builtin_amdgcn_readfirstlane(__float_as_uint(sloc[h].w));
    const uint32_t end = min(h + 64u, (uint32_t)__builtin_amdgcn_readfirstlane(off[c + 1]));
    const uint32_t i = h + (uint32_t)lane;
    const bool inrange = i < end;
    const uint32_t ii_ = inrange ? i : h;
    const int key = inrange ? gkey[ii_] : -1;
    const float di = dens_s[ii_];
    const bool active = key >= 0 && (double)di >= g.floor_nuc;
    if (inrange) cflag[i] = 0;
    if (!__ballot(active)) return;
    const float4 li = sloc[ii_];
    const float4 pi = spos[ii_];
    const uint32_t oi = orig_of(pi);
    const int nc = g.nc;
    const int cx = (int)(c % (uint32_t)nc), cy = (int)((c / (uint32_t)nc) % (uint32_t)nc),
              cz = (int)(c / ((uint32_t)nc * (uint32_t)nc));
    bool found = !active;
    for (int t = 0; t < 27; t++) {
        int ox, oy, oz;
        stencil_offset(t, ox, oy, oz);
        const uint32_t nb = ((uint32_t)wrapc(cz + oz, nc) * (uint32_t)nc + (uint32_t)wrapc(cy + oy, nc)) *
                                (uint32_t)nc + (uint32_t)wrapc(cx + ox, nc);
        const float xs = li.x - (float)ox * g.cellb, ys = li.y - (float)oy * g.cellb,
                    zs = li.z - (float)oz * g.cellb;
        const uint32_t a = __builtin_amdgcn_readfirstlane(off[nb]);
        const uint32_t b = __builtin_amdgcn_readfirstlane(off[nb + 1]);
        for (uint32_t j = a; j < b; j++) {
            const float dj = dens_s[j];
            const int kj = gkey[j];
            const float4 lj = sloc[j];
            const float4 pj = spos[j];
            if (!found && denser_within_b(dj, orig_of(pj), kj, lj, pj, key, di, oi, xs, ys, zs, pi, g))
                found = true;
            if (((j - a) & 15u) == 15u && !__ballot(!found)) break;
        }
        if (!__ballot(!found)) break;
    }
    if (active && !found) {
        cflag[i] = 1;
        atomicAdd(&gccnt[gid_of[i]], 1u);
    }
}

__global__ __launch_bounds__(kBlock) void k_cand_sparse(int64_t nsparse, Geo g,
                                                        const int32_t *__restrict__ sparse,
                                                        const float4 *__restrict__ sloc,
                                                        const float4 *__restrict__ spos,
                                                        const uint32_t *__restrict__ off,
                                                        const float *__restrict__ dens_s,
                                                        const int32_t *__restrict__ gkey,
                                                        const int32_t *__restrict__ gid_of,
                                                        uint32_t *__restrict__ gccnt,
                                                        int32_t *__restrict__ cflag) {
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t0 >= nsparse) return;
    const int i = sparse[t0];
    cflag[i] = 0;
    const int key = gkey[i];
    if (key < 0) return;
    const float di = dens_s[i];
    if (!((double)di >= g.floor_nuc)) return;
    const float4 li = sloc[i];
    const float4 pi = spos[i];
    const uint32_t oi = orig_of(pi);
    const uint32_t c = __float_as_uint(li.w);
    const int nc = g.nc;
    const int cx = (int)(c % (uint32_t)nc), cy = (int)((c / (uint32_t)nc) % (uint32_t)nc),
              cz = (int)(c / ((uint32_t)nc * (uint32_t)nc));
    for (int t = 0; t < 27; t++) {
        int ox, oy, oz;
        stencil_offset(t, ox, oy, oz);
        const uint32_t nb = ((uint32_t)wrapc(cz + oz, nc) * (uint32_t)nc + (uint32_t)wrapc(cy + oy, nc)) *
                                (uint32_t)nc + (uint32_t)wrapc(cx + ox, nc);
        const float xs = li.x - (float)ox * g.cellb, ys = li.y - (float)oy * g.cellb,
                    zs = li.z - (float)oz * g.cellb;
        for (uint32_t j = off[nb]; j < off[nb + 1]; j++) {
            const float dj = dens_s[j];
            if (dj < di) continue;
            const float4 pj = spos[j];
            if (denser_within_b(dj, orig_of(pj), gkey[j], sloc[j], pj, key, di, oi, xs, ys, zs, pi, g))
                return;
        }
    }
    cflag[i] = 1;
    atomicAdd(&gccnt[gid_of[i]], 1u);
}

}  // namespace

void launch_candidates(int64_t n, const Geo &g, Work &w, hipStream_t s) {
    if (w.nchunks > 0)
        hipLaunchKernelGGL(k_cand_dense, dim3((unsigned)((w.nchunks + 3) / 4)), dim3(kBlock), 0, s,
                           w.nchunks, g, w.chunks, w.sloc, w.spos, w.off, w.dens_s, w.gkey, w.gid_of,
                           w.gccnt, w.owner /* candidate flags */);
    if (w.nsparse > 0)
        hipLaunchKernelGGL(k_cand_sparse, dim3((unsigned)((w.nsparse + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, s, w.nsparse, g, w.sparse, w.sloc, w.spos, w.off, w.dens_s, w.gkey, w.gid_of,
                           w.gccnt, w.owner);
}

}  // namespace hf
