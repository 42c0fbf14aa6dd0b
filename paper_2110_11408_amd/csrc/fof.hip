// L0 friends-of-friends over the particles denser than Delta_L0,min (Sec. 2.2.1):
// two members are friends when their separation is less than l; L0 groups are
// the connected components.
//
// Lock-free union-find in sorted (cell) order:
//   init      parent[i] = i for members, -1 otherwise;
//   link      every member i visits the members j > i of its 27 neighbour cells;
//             an FP32 prefilter on the cell-local coordinates decides clear
//             cases (the margin exceeds the FP32 error bound of the local
//             coordinates by a factor of ten) and the canonical FP64 distance
//             decides the rest; linked pairs are united by hooking the larger
//             root under the smaller one with a compare-and-swap;
//   compress  parent[i] = root(i);
//   labels    the canonical label of a group is 1 + the smallest ORIGINAL index
//             of its members (atomicMin into the root's slot).
// The union-find is order-independent: the components, and therefore the
// labels, do not depend on thread scheduling.
#include "hf_internal.h"

namespace hf {

namespace {

__device__ __forceinline__ int ld(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root with path halving.  Only non-roots are rewritten and only ever to an
// ancestor, so the plain relaxed stores cannot undo a concurrent hook (hooks
// only change roots).
__device__ int uf_find(int32_t *parent, int x) {
    for (;;) {
        int p = ld(parent + x);
        if (p == x) return x;
        int gp = ld(parent + p);
        if (gp != p) st(parent + x, gp);
        x = gp;
    }
}

__device__ void uf_unite(int32_t *parent, int a, int b) {
    for (;;) {
        a = uf_find(parent, a);
        b = uf_find(parent, b);
        if (a == b) return;
        if (a > b) { int t = a; a = b; b = t; }
        int old = atomicCAS(parent + b, b, a);
        if (old == b) return;
    }
}

__global__ __launch_bounds__(kBlock) void k_fof_init(int64_t n, Geo g, const float *__restrict__ dens_s,
                                                     int32_t *__restrict__ parent,
                                                     int32_t *__restrict__ counters) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool m = (double)dens_s[i] > g.dl0;
    parent[i] = m ? (int32_t)i : -1;
    if (m) atomicAdd(&counters[0], 1);
}

__global__ __launch_bounds__(kBlock) void k_fof_link(int64_t n, Geo g, const float4 *__restrict__ sloc,
                                                     const float4 *__restrict__ spos,
                                                     const uint32_t *__restrict__ off,
                                                     const float *__restrict__ dens_s,
                                                     int32_t *parent) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!((double)dens_s[i] > g.dl0)) return;
    const float4 li = sloc[i];
    const float4 pi = spos[i];
    const uint32_t c = __float_as_uint(li.w);
    const int nc = g.nc;
    const int cx = (int)(c % (uint32_t)nc), cy = (int)((c / (uint32_t)nc) % (uint32_t)nc),
              cz = (int)(c / ((uint32_t)nc * (uint32_t)nc));
    for (int oz = -1; oz <= 1; oz++) {
        const int z = wrapc(cz + oz, nc);
        const float zs = li.z - (float)oz * g.cellb;
        for (int oy = -1; oy <= 1; oy++) {
            const int y = wrapc(cy + oy, nc);
            const float ys = li.y - (float)oy * g.cellb;
            const uint32_t row = ((uint32_t)z * (uint32_t)nc + (uint32_t)y) * (uint32_t)nc;
            for (int ox = -1; ox <= 1; ox++) {
                const int x = wrapc(cx + ox, nc);
                const float xs = li.x - (float)ox * g.cellb;
                const uint32_t nb = row + (uint32_t)x;
                uint32_t a = off[nb];
                const uint32_t b = off[nb + 1];
                if (a <= (uint32_t)i) a = (uint32_t)i + 1;
                for (uint32_t j = a; j < b; j++) {
                    const float4 lj = sloc[j];
                    const float dx = lj.x - xs, dy = lj.y - ys, dz = lj.z - zs;
                    const float d2f = dx * dx + dy * dy + dz * dz;
                    if (d2f >= g.l2b_hi) continue;
                    if (!((double)dens_s[j] > g.dl0)) continue;
                    if (d2f >= g.l2b_lo && !(d2_exact(pi, spos[j], g.L, g.half) < g.l2)) continue;
                    uf_unite(parent, (int)i, (int)j);
                }
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_fof_compress(int64_t n, int32_t *parent,
                                                         const float4 *__restrict__ spos,
                                                         int32_t *__restrict__ minorig,
                                                         int32_t *__restrict__ counters) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (ld(parent + i) < 0) return;
    int r = uf_find(parent, (int)i);
    st(parent + i, r);
    if (r == (int)i) atomicAdd(&counters[1], 1);
    atomicMin(&minorig[r], (int32_t)orig_of(spos[i]));
}

// Group key (smallest original index of the group) per sorted particle, and the
// L0 label in original order.
__global__ __launch_bounds__(kBlock) void k_fof_keys(int64_t n, const int32_t *__restrict__ parent,
                                                     const int32_t *__restrict__ minorig,
                                                     const float4 *__restrict__ spos,
                                                     int32_t *__restrict__ gkey,
                                                     int32_t *__restrict__ l0_out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int p = parent[i];
    int k = p < 0 ? -1 : minorig[p];
    gkey[i] = k;
    if (l0_out) l0_out[orig_of(spos[i])] = k + 1;
}

// Group keys from caller-provided labels (1..n, 0 = none), in sorted order.
__global__ __launch_bounds__(kBlock) void k_keys_from_labels(int64_t n, const int32_t *__restrict__ l0_in,
                                                             const float4 *__restrict__ spos,
                                                             int32_t *__restrict__ gkey,
                                                             int32_t *__restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t lab = l0_in[orig_of(spos[i])];
    if (lab < 0 || (int64_t)lab > n) {
        atomicOr(err, 2);
        lab = 0;
    }
    gkey[i] = lab - 1;
}

inline dim3 grid(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

}  // namespace

void launch_fof(int64_t n, const Geo &g, Work &w, hipStream_t s) {
    hipLaunchKernelGGL(k_fof_init, grid(n), dim3(kBlock), 0, s, n, g, w.dens_s, w.parent, w.counters);
    hipLaunchKernelGGL(k_fof_link, grid(n), dim3(kBlock), 0, s, n, g, w.sloc, w.spos, w.off, w.dens_s,
                       w.parent);
    fill_i32(w.minorig, 0x7fffffff, n, s);
    hipLaunchKernelGGL(k_fof_compress, grid(n), dim3(kBlock), 0, s, n, w.parent, w.spos, w.minorig,
                       w.counters);
}

void launch_fof_labels(int64_t n, const Geo &, Work &w, int32_t *l0_out, hipStream_t s) {
    hipLaunchKernelGGL(k_fof_keys, grid(n), dim3(kBlock), 0, s, n, w.parent, w.minorig, w.spos, w.gkey,
                       l0_out);
}

void launch_keys_from_labels(const int32_t *l0_in, int64_t n, Work &w, hipStream_t s) {
    hipLaunchKernelGGL(k_keys_from_labels, grid(n), dim3(kBlock), 0, s, n, l0_in, w.spos, w.gkey,
                       w.err);
}

}  // namespace hf
