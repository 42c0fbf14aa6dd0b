// L0 friends-of-friends over the particles denser than Delta_L0,min (Sec. 2.2.1):
// two members are friends when their separation is less than l; L0 groups are
// the connected components.
//
// Lock-free union-find in sorted (cell, sub-cell) order.  A sub-cell's diagonal
// is below l, so all members of a sub-cell are friends; the link work is done
// between sub-cells instead of between particles:
//   phase A  in dense cells every member points at the first member of its
//            sub-cell (a valid forest: parents never exceed their child);
//   phase B  one thread per sub-cell of a dense cell visits the sub-cells of
//            dense cells within reach (half stencil); if the two are not yet in
//            one set it searches for one friend pair (FP32 prefilter on the
//            cell-local coordinates, canonical FP64 distance for the undecided
//            band) and unites them.  A first pass over face neighbours plus a
//            compression makes most later checks a single root comparison;
//   sparse   members of sparse cells link particle by particle to every member
//            of a dense neighbour cell and to the later members of sparse ones;
//   labels   compression, then 1 + the smallest ORIGINAL index of each set.
// Hooks always attach the larger root under the smaller one, so the sets, and
// therefore the labels, do not depend on thread scheduling.
#include "hf_internal.h"

namespace hf {

namespace {

inline dim3 grid(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

__device__ __forceinline__ int ld(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root with path halving.  Only non-roots are rewritten and only ever to an
// ancestor, so the relaxed stores cannot undo a concurrent hook (hooks only
// change roots).
__device__ int uf_find(int32_t *parent, int x) {
    for (;;) {
        int p = ld(parent + x);
        if (p == x) return x;
        int gp = ld(parent + p);
        if (gp != p) st(parent + x, gp);
        x = gp;
    }
}

// Root by plain (cacheable) loads, for filters only: a stale parent is an
// earlier ancestor, so two particles reported in one set are in one set; a
// "different" answer may be stale and is then settled by uf_unite.
__device__ __forceinline__ int uf_find_hint(const int32_t *parent, int x) {
    for (;;) {
        const int p = parent[x];
        if (p == x) return x;
        x = p;
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

// Friends test of a (shifted local coordinates xs, ys, zs) and b: FP32 prefilter,
// canonical FP64 distance only in the undecided band.
__device__ __forceinline__ bool linked(float xs, float ys, float zs, const float4 &pa,
                                       const float4 *__restrict__ sloc, const float4 *__restrict__ spos,
                                       uint32_t b, const Geo &g) {
    const float4 lb = sloc[b];
    const float dx = lb.x - xs, dy = lb.y - ys, dz = lb.z - zs;
    const float d2f = dx * dx + dy * dy + dz * dz;
    if (d2f >= g.l2b_hi) return false;
    if (d2f < g.l2b_lo) return true;
    return d2_exact(pa, spos[b], g.L, g.half) < g.l2;
}

__global__ __launch_bounds__(kBlock) void k_fof_init(int64_t n, Geo g, const float *__restrict__ dens_s,
                                                     int32_t *__restrict__ parent) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    parent[i] = is_member(dens_s, i, g.dl0) ? (int32_t)i : -1;
}

// Phase A: members of dense cells point at the first member of their sub-cell.
__global__ __launch_bounds__(kBlock) void k_fof_phase_a(int64_t n, Geo g, const float4 *__restrict__ sloc,
                                                        const uint32_t *__restrict__ off,
                                                        const uint16_t *__restrict__ ssub,
                                                        const uint32_t *__restrict__ cellmap,
                                                        const uint32_t *__restrict__ subtab,
                                                        const float *__restrict__ dens_s,
                                                        int32_t *__restrict__ parent,
                                                        uint32_t *__restrict__ f_run) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    f_run[i] = 0;
    if (!is_member(dens_s, i, g.dl0)) return;
    const uint32_t c = __float_as_uint(sloc[i].w);
    if (off[c + 1] - off[c] < (uint32_t)kDenseMin) return;
    const int nsub = g.ksub * g.ksub * g.ksub;
    uint32_t f = subtab[(int64_t)cellmap[c] * (nsub + 1) + ssub[i]];
    while (f < (uint32_t)i && !is_member(dens_s, f, g.dl0)) f++;
    parent[i] = (int32_t)f;
    f_run[i] = f == (uint32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_list(int64_t n, const uint32_t *__restrict__ flag,
                                                 const uint32_t *__restrict__ pos,
                                                 int32_t *__restrict__ list) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    list[pos[i]] = (int32_t)i;
}

// Phase B: sub-cell to sub-cell links between dense cells.  pass 0 visits the
// three positive face neighbours, pass 1 the whole positive half of the reach.
__global__ __launch_bounds__(kBlock) void k_fof_runs(int64_t nruns, int pass, Geo g,
                                                     const int32_t *__restrict__ runlist,
                                                     const float4 *__restrict__ sloc,
                                                     const float4 *__restrict__ spos,
                                                     const uint32_t *__restrict__ off,
                                                     const uint16_t *__restrict__ ssub,
                                                     const uint32_t *__restrict__ cellmap,
                                                     const uint32_t *__restrict__ subtab,
                                                     const float *__restrict__ dens_s,
                                                     int32_t *parent) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nruns) return;
    const int f = runlist[t];
    const int k = g.ksub, nsub = k * k * k, R = g.rsub, nc = g.nc;
    const uint32_t c = __float_as_uint(sloc[f].w);
    const int cx = (int)(c % (uint32_t)nc), cy = (int)((c / (uint32_t)nc) % (uint32_t)nc),
              cz = (int)(c / ((uint32_t)nc * (uint32_t)nc));
    const int s = ssub[f];
    const int sx = s % k, sy = (s / k) % k, sz = s / (k * k);
    const uint32_t *tabA = subtab + (int64_t)cellmap[c] * (nsub + 1);
    const uint32_t A1 = tabA[s + 1];
    uint32_t last_c2 = 0xffffffffu;
    bool last_dense = false;
    const uint32_t *tabB = nullptr;
    for (int dz = 0; dz <= R; dz++) {
        for (int dy = (dz > 0 ? -R : 0); dy <= R; dy++) {
            for (int dx = (dz > 0 || dy > 0 ? -R : 1); dx <= R; dx++) {
                const int ax = dx < 0 ? -dx : dx, ay = dy < 0 ? -dy : dy, az = dz < 0 ? -dz : dz;
                if (pass == 0 && ax + ay + az != 1) continue;
                const int gx = ax > 0 ? ax - 1 : 0, gy = ay > 0 ? ay - 1 : 0, gz = az > 0 ? az - 1 : 0;
                if ((double)(gx * gx + gy * gy + gz * gz) * g.sub2 >= g.l2) continue;
                // neighbour sub-cell: cell offset (image) and sub index
                const int fx = sx + dx, fy = sy + dy, fz = sz + dz;
                const int ocx = fx < 0 ? -1 : (fx >= k ? 1 : 0);
                const int ocy = fy < 0 ? -1 : (fy >= k ? 1 : 0);
                const int ocz = fz < 0 ? -1 : (fz >= k ? 1 : 0);
                const uint32_t c2 = ((uint32_t)wrapc(cz + ocz, nc) * (uint32_t)nc +
                                     (uint32_t)wrapc(cy + ocy, nc)) * (uint32_t)nc +
                                    (uint32_t)wrapc(cx + ocx, nc);
                if (c2 != last_c2) {
                    last_c2 = c2;
                    last_dense = off[c2 + 1] - off[c2] >= (uint32_t)kDenseMin;
                    if (last_dense) tabB = subtab + (int64_t)cellmap[c2] * (nsub + 1);
                }
                if (!last_dense) continue;  // the sparse side links it
                const int s2 = ((fz - ocz * k) * k + (fy - ocy * k)) * k + (fx - ocx * k);
                uint32_t fb = tabB[s2];
                const uint32_t B1 = tabB[s2 + 1];
                while (fb < B1 && !is_member(dens_s, fb, g.dl0)) fb++;
                if (fb >= B1) continue;
                if (uf_find_hint(parent, f) == uf_find_hint(parent, (int)fb)) continue;
                const float ox = (float)ocx * g.cellb, oy = (float)ocy * g.cellb, oz = (float)ocz * g.cellb;
                bool hit = false;
                for (uint32_t a = (uint32_t)f; a < A1 && !hit; a++) {
                    if (!is_member(dens_s, a, g.dl0)) continue;
                    const float4 la = sloc[a];
                    const float4 pa = spos[a];
                    const float xs = la.x - ox, ys = la.y - oy, zs = la.z - oz;
                    for (uint32_t bb = fb; bb < B1; bb++) {
                        if (!is_member(dens_s, bb, g.dl0)) continue;
                        if (linked(xs, ys, zs, pa, sloc, spos, bb, g)) {
                            hit = true;
                            break;
                        }
                    }
                }
                if (hit) uf_unite(parent, f, (int)fb);
            }
        }
    }
}

// Members of sparse cells: link to the later members of sparse neighbour cells,
// and to one member of every reachable sub-cell of a dense neighbour cell (the
// members of a sub-cell are already one set).
__global__ __launch_bounds__(kBlock) void k_fof_sparse(int64_t nsparse, Geo g,
                                                       const int32_t *__restrict__ sparse,
                                                       const float4 *__restrict__ sloc,
                                                       const float4 *__restrict__ spos,
                                                       const uint32_t *__restrict__ off,
                                                       const uint32_t *__restrict__ cellmap,
                                                       const uint32_t *__restrict__ subtab,
                                                       const float *__restrict__ dens_s,
                                                       int32_t *parent) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsparse) return;
    const int i = sparse[t];
    if (!is_member(dens_s, i, g.dl0)) return;
    const float4 li = sloc[i];
    const float4 pi = spos[i];
    const uint32_t c = __float_as_uint(li.w);
    const int nc = g.nc, k = g.ksub, nsub = k * k * k;
    const float subb = g.cellb / (float)k;
    const int cx = (int)(c % (uint32_t)nc), cy = (int)((c / (uint32_t)nc) % (uint32_t)nc),
              cz = (int)(c / ((uint32_t)nc * (uint32_t)nc));
    int ri = uf_find_hint(parent, i);
    for (int oz = -1; oz <= 1; oz++) {
        const int z = wrapc(cz + oz, nc);
        const float zs = li.z - (float)oz * g.cellb;
        for (int oy = -1; oy <= 1; oy++) {
            const int y = wrapc(cy + oy, nc);
            const float ys = li.y - (float)oy * g.cellb;
            const uint32_t row = ((uint32_t)z * (uint32_t)nc + (uint32_t)y) * (uint32_t)nc;
            for (int ox = -1; ox <= 1; ox++) {
                // the neighbour cell must come closer than l to the particle
                const float gx = ox < 0 ? li.x : (ox > 0 ? g.cellb - li.x : 0.0f);
                const float gy = oy < 0 ? li.y : (oy > 0 ? g.cellb - li.y : 0.0f);
                const float gz = oz < 0 ? li.z : (oz > 0 ? g.cellb - li.z : 0.0f);
                if (gx * gx + gy * gy + gz * gz >= g.l2b_hi) continue;
                const uint32_t nb = row + (uint32_t)wrapc(cx + ox, nc);
                const float xs = li.x - (float)ox * g.cellb;
                const uint32_t a = off[nb], b = off[nb + 1];
                if (b - a < (uint32_t)kDenseMin) {
                    for (uint32_t j = a > (uint32_t)i ? a : (uint32_t)i + 1; j < b; j++) {
                        if (!is_member(dens_s, j, g.dl0)) continue;
                        if (linked(xs, ys, zs, pi, sloc, spos, j, g)) uf_unite(parent, i, (int)j);
                    }
                    continue;
                }
                const uint32_t *tab = subtab + (int64_t)cellmap[nb] * (nsub + 1);
                for (int sz = 0; sz < k; sz++) {
                    const float lz = sz * subb - 1e-5f, hz = lz + subb + 2e-5f;
                    const float gz = fmaxf(fmaxf(lz - zs, zs - hz), 0.0f);
                    if (gz * gz >= g.l2b_hi) continue;
                    for (int sy = 0; sy < k; sy++) {
                        const float ly = sy * subb - 1e-5f, hy = ly + subb + 2e-5f;
                        const float gy = fmaxf(fmaxf(ly - ys, ys - hy), 0.0f);
                        if (gz * gz + gy * gy >= g.l2b_hi) continue;
                        for (int sx = 0; sx < k; sx++) {
                            const float lx = sx * subb - 1e-5f, hx = lx + subb + 2e-5f;
                            const float gx = fmaxf(fmaxf(lx - xs, xs - hx), 0.0f);
                            if (gz * gz + gy * gy + gx * gx >= g.l2b_hi) continue;
                            const int s2 = (sz * k + sy) * k + sx;
                            const uint32_t u1 = tab[s2 + 1];
                            for (uint32_t j = tab[s2]; j < u1; j++) {
                                if (!is_member(dens_s, j, g.dl0)) continue;
                                if (ri == parent[j]) break;  // already one set
                                if (linked(xs, ys, zs, pi, sloc, spos, j, g)) {
                                    uf_unite(parent, i, (int)j);
                                    ri = uf_find_hint(parent, i);
                                    break;
                                }
                            }
                        }
                    }
                }
            }
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_fof_flatten(int64_t n, int32_t *parent) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (ld(parent + i) < 0) return;
    st(parent + i, uf_find(parent, (int)i));
}

// Final compression and the smallest original index of every set.
__global__ __launch_bounds__(kBlock) void k_fof_compress(int64_t n, int32_t *parent,
                                                         const float4 *__restrict__ spos,
                                                         int32_t *__restrict__ minorig) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int r = -1;
    if (i < n && ld(parent + i) >= 0) {
        r = uf_find(parent, (int)i);
        st(parent + i, r);
    }
    const WaveRun run = wave_run(r);
    const int32_t o = i < n ? (int32_t)orig_of(spos[i]) : 0x7fffffff;
    const int32_t m = wave_run_min(r >= 0 ? o : 0x7fffffff, run);
    if (r >= 0 && run.rank == 0) atomicMin(&minorig[r], m);
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

}  // namespace

void launch_fof(int64_t n, const Geo &g, Work &w, hipStream_t s) {
    hipLaunchKernelGGL(k_fof_init, grid(n), dim3(kBlock), 0, s, n, g, w.dens_s, w.parent);
    // phase A + list of sub-cell representatives (reuses the chunk flag arrays)
    hipLaunchKernelGGL(k_fof_phase_a, grid(n), dim3(kBlock), 0, s, n, g, w.sloc, w.off, w.ssub, w.cnt,
                       w.subtab, w.dens_s, w.parent, w.f_chunk);
    scan_u32(w.f_chunk, w.s_chunk, n, w.scan_tmp, s);
    hipLaunchKernelGGL(k_list, grid(n), dim3(kBlock), 0, s, n, w.f_chunk, w.s_chunk, w.runlist);
    // the run count is bounded by n; threads beyond it exit on the device count
    uint32_t nr = 0;
    (void)hipMemcpyAsync(&nr, w.s_chunk + n, sizeof(nr), hipMemcpyDeviceToHost, s);
    (void)hipStreamSynchronize(s);
    w.nruns = nr;
    if (w.nruns > 0) {
        hipLaunchKernelGGL(k_fof_runs, grid(w.nruns), dim3(kBlock), 0, s, w.nruns, 0, g, w.runlist, w.sloc,
                           w.spos, w.off, w.ssub, w.cnt, w.subtab, w.dens_s, w.parent);
        hipLaunchKernelGGL(k_fof_flatten, grid(n), dim3(kBlock), 0, s, n, w.parent);
        hipLaunchKernelGGL(k_fof_runs, grid(w.nruns), dim3(kBlock), 0, s, w.nruns, 1, g, w.runlist, w.sloc,
                           w.spos, w.off, w.ssub, w.cnt, w.subtab, w.dens_s, w.parent);
        hipLaunchKernelGGL(k_fof_flatten, grid(n), dim3(kBlock), 0, s, n, w.parent);
    }
    if (w.nsparse > 0)
        hipLaunchKernelGGL(k_fof_sparse, grid(w.nsparse), dim3(kBlock), 0, s, w.nsparse, g, w.sparse,
                           w.sloc, w.spos, w.off, w.cnt, w.subtab, w.dens_s, w.parent);
    fill_i32(w.minorig, 0x7fffffff, n, s);
    hipLaunchKernelGGL(k_fof_compress, grid(n), dim3(kBlock), 0, s, n, w.parent, w.spos, w.minorig);
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
