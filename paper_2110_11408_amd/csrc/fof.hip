// L0 friends-of-friends over the particles denser than Delta_L0,min (Sec. 2.2.1):
// two members are friends when their separation is less than l; L0 groups are
// the connected components.
//
// Lock-free union-find in sorted (cell, sub-cell) order:
//   phase A  a sub-cell's diagonal is below l, so all members of a sub-cell are
//            friends: in dense cells every member points at the first member of
//            its sub-cell;
//   dense    one wavefront per dense chunk streams the neighbour members within
//            reach (FP32 prefilter on the cell-local coordinates, canonical FP64
//            distance for the undecided band) and joins each linked member's set
//            to the sets of the lanes it links, with a per-lane root cache;
//   sparse   members of sparse cells link to the later members of sparse
//            neighbour cells;
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
    const float d2f = d2_f32(dx, dy, dz);
    if (d2f >= g.l2b_hi) return false;
    if (d2f < g.l2b_lo) return true;
    return d2_exact(pa, spos[b], g.L, g.half) < g.l2;
}

// Join the lanes linked to a member of the set rj (rj: any node of that set)
// to that set; every lane keeps the root of its own set in wr.  Returns the
// root of the joined set.
__device__ __forceinline__ int join_lanes(int32_t *parent, bool lk, int &wr, int rj) {
    const int lane = threadIdx.x & 63;
    bool need = lk && wr != rj;
    uint64_t m;
    while ((m = __ballot(need)) != 0ull) {
        const int L = __ffsll((unsigned long long)m) - 1;
        const int w = lane_get(wr, L);
        int r = 0;
        if (lane == L) {
            // fast path: both are usually current roots, so hooking the larger
            // under the smaller is one compare-and-swap; otherwise a full union
            const int lo = min(w, rj), hi = max(w, rj);
            if (atomicCAS(parent + hi, hi, lo) == hi) {
                r = lo;
            } else {
                uf_unite(parent, w, rj);
                r = uf_find(parent, w);
            }
        }
        r = lane_get(r, L);
        if (wr == w || wr == rj) wr = r;
        rj = r;
        need = lk && wr != rj;
    }
    return rj;
}

// Friends test from FP32 differences already taken in one frame (dx = x_b - x_a):
// FP32 prefilter, canonical FP64 distance of the original positions in the
// undecided band.
__device__ __forceinline__ bool linked_d(float dx, float dy, float dz, const float4 &pa,
                                         const float4 *__restrict__ spos, uint32_t b, const Geo &g) {
    const float d2f = d2_f32(dx, dy, dz);
    if (d2f >= g.l2b_hi) return false;
    if (d2f < g.l2b_lo) return true;
    return d2_exact(pa, spos[b], g.L, g.half) < g.l2;
}

// Joins the lanes linked to any member of [a, b) to that range's set rset
// (the range is one sub-cell, so its members are one set).  Every lane tests
// the members in order (wave-uniform loads, coordinates as scalar operands)
// and keeps whether it links to any of them, with the canonical FP64
// distance in the FP32 prefilter's undecided band.  The linked lanes are
// then joined in one go.  Returns whether any join was made.
__device__ __forceinline__ bool stream_range(int32_t *parent, const float *__restrict__ dens_s,
                                             const float4 *__restrict__ sloc,
                                             const float4 *__restrict__ spos, const Geo &g, bool active,
                                             const float4 &li, const float4 &pi, int &wr, uint32_t a,
                                             uint32_t b, int ox, int oy, int oz, int rset) {
    // the lane's coordinates in the neighbour cell's frame
    const float xs = li.x - (float)ox * g.cellb, ys = li.y - (float)oy * g.cellb,
                zs = li.z - (float)oz * g.cellb;
    const bool want = active && wr != rset;
    // the smallest FP32 squared distance to a member (one minimum per member,
    // no branch); only a lane whose minimum falls in the prefilter's
    // undecided band repeats the range with the canonical FP64 distance
    float mind = 3.0e38f;
    for (uint32_t j = a; j < b; j++) {
        if (!is_member(dens_s, j, g.dl0)) continue;
        const float4 lj = sloc[j];
        const float dx = lj.x - xs, dy = lj.y - ys, dz = lj.z - zs;
        mind = fminf(mind, d2_f32(dx, dy, dz));
    }
    bool any = mind < g.l2b_lo;
    if (want && !any && mind < g.l2b_hi) {
        for (uint32_t j = a; j < b && !any; j++)
            if (is_member(dens_s, j, g.dl0) && d2_exact(pi, spos[j], g.L, g.half) < g.l2) any = true;
    }
    const bool lk = want && any;
    if (!__ballot(lk)) return false;
    join_lanes(parent, lk, wr, rset);
    return true;
}

// All sparse neighbour cells of a chunk at once: lane t < 27 holds stencil
// cell t's range [la, lb) and whether it is to be visited; their particles are
// numbered through a prefix sum and loaded 64 at a time (each lane finds its
// particle's cell by one walk over the cells that hold particles), then
// broadcast in order and joined to the lanes they link.
__device__ __forceinline__ void stream_sparse_cells(int32_t *parent, const float *__restrict__ dens_s,
                                                    const float4 *__restrict__ sloc,
                                                    const float4 *__restrict__ spos, const Geo &g,
                                                    bool active, const float4 &li, const float4 &pi,
                                                    int &wr, bool visit, uint32_t la, uint32_t lb) {
    const int lane = threadIdx.x & 63;
    const int cntl = visit ? (int)(lb - la) : 0;
    int incl = cntl;
    for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(incl, d, 64);
        if (lane >= d) incl += y;
    }
    const int P = lane_get(incl, 63);
    if (P == 0) return;
    // the visited cells that hold particles (lane t for stencil cell t)
    const uint64_t cells = __ballot(cntl > 0);
    for (int p0 = 0; p0 < P; p0 += 64) {
        const int p = p0 + lane;
        bool mem = false;
        uint32_t j = 0;
        float xj = 0.0f, yj = 0.0f, zj = 0.0f;
        int rj = -1;
        // the visited cell whose particles include number p, found by one
        // walk over the cells with particles (their starts are scalars)
        int t = 0;
        uint32_t jt = 0;
        for (uint64_t m = cells; m; m &= m - 1) {
            const int u = __builtin_ctzll(m);
            const int st = lane_get(incl, u) - lane_get(cntl, u);
            if (p >= st) {
                t = u;
                jt = lane_get(la, u) + (uint32_t)(p - st);
            }
        }
        if (p < P) {
            j = jt;
            mem = is_member(dens_s, j, g.dl0);
            if (mem) {
                const float4 lj = sloc[j];
                xj = lj.x + (float)(t % 3 - 1) * g.cellb;
                yj = lj.y + (float)((t / 3) % 3 - 1) * g.cellb;
                zj = lj.z + (float)(t / 9 - 1) * g.cellb;
                rj = uf_find_hint(parent, (int)j);
            }
        }
        uint64_t mm = __ballot(mem);
        while (mm) {
            const int J = __ffsll((unsigned long long)mm) - 1;
            mm &= mm - 1;
            int r = lane_get(rj, J);
            if (!__ballot(active && wr != r)) continue;
            const uint32_t jj = lane_get(j, J);
            const float dx = lane_get(xj, J) - li.x, dy = lane_get(yj, J) - li.y,
                        dz = lane_get(zj, J) - li.z;
            const bool lk = active && wr != r && linked_d(dx, dy, dz, pi, spos, jj, g);
            if (!__ballot(lk)) continue;
            join_lanes(parent, lk, wr, r);
        }
    }
}

// Phase A, which also initializes the forest: non-members get -1, members of
// sparse cells are roots, and members of dense cells point at the first member
// of their sub-cell (a valid forest: every parent is a member with a smaller
// or equal sorted index).
__global__ __launch_bounds__(kBlock) void k_fof_phase_a(int64_t n, Boxes bx, const float4 *__restrict__ sloc,
                                                        const uint32_t *__restrict__ f_sparse,
                                                        const uint16_t *__restrict__ ssub,
                                                        const uint32_t *__restrict__ cellmap,
                                                        const uint32_t *__restrict__ subtab,
                                                        const float *__restrict__ dens_s,
                                                        int32_t *__restrict__ parent) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Geo &g = bx.geo[box_of(bx, (uint32_t)i)];
    if (!is_member(dens_s, i, g.dl0)) {
        parent[i] = -1;
        return;
    }
    if (f_sparse[i]) {
        parent[i] = (int32_t)i;
        return;
    }
    const uint32_t c = __float_as_uint(sloc[i].w);
    uint32_t f = subtab[(int64_t)cellmap[c] * (bx.nsub_max + 1) + ssub[i]];
    while (f < (uint32_t)i && !is_member(dens_s, f, g.dl0)) f++;
    parent[i] = (int32_t)f;
}

// Dense chunks, one wavefront each (lanes = the chunk's particles).  The wave
// visits the neighbour cells that come within l of some lane: sparse cells in
// all 26 directions, dense cells only in the forward half (the backward ones
// visit this cell themselves), and its own cell from the chunk start on.
// The 27 cell ranges are loaded at once (one stencil cell per lane); sparse
// cells are then streamed particle by particle.  The sub-cells of all visited
// dense cells are examined 64 at a time (one per lane): range, first member and
// that member's parent; a sub-cell already in the set every lane belongs to is
// skipped (all its members are one set), and the others are streamed as
// wave-uniform scalar loads and joined to the lanes they link.
__global__ __launch_bounds__(kBlock) void k_fof_dense(int64_t nchunks, Boxes bx,
                                                      const int32_t *__restrict__ chunks,
                                                      const float4 *__restrict__ sloc,
                                                      const float4 *__restrict__ spos,
                                                      const uint32_t *__restrict__ off,
                                                      const uint32_t *__restrict__ cellmap,
                                                      const uint32_t *__restrict__ subtab,
                                                      const float *__restrict__ dens_s,
                                                      int32_t *parent) {
    __shared__ int64_t dbase[kBlock / 64][27];  // visited dense cells: sub-table base
    __shared__ int8_t doff[kBlock / 64][27];    // and stencil index
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t q = (int64_t)xcd_block() * (int64_t)(blockDim.x >> 6) + wave;
    if (q >= nchunks) return;
    const int lane = threadIdx.x & 63;
    const uint32_t h = (uint32_t)__builtin_amdgcn_readfirstlane(chunks[q]);
    const Geo &g = bx.geo[__builtin_amdgcn_readfirstlane(box_of(bx, h))];
    const uint32_t c = __builtin_amdgcn_readfirstlane(__float_as_uint(sloc[h].w));
    const uint32_t cend = (uint32_t)__builtin_amdgcn_readfirstlane(off[c + 1]);
    const uint32_t end = min(h + 64u, cend);
    const uint32_t i = h + (uint32_t)lane;
    const uint32_t ic = i < end ? i : h;
    const bool active = i < end && is_member(dens_s, ic, g.dl0);
    if (!__ballot(active)) return;
    const float4 li = sloc[ic];
    const float4 pi = spos[ic];
    int wr = active ? uf_find_hint(parent, (int)ic) : -1;
    const int k = g.ksub, nsub = g.nsub, tstride = bx.nsub_max + 1;
    const float subb = g.cellb / (float)k;
    int cx, cy, cz;
    cell_xyz(g, c, cx, cy, cz);
    // chunk bounding box (active lanes), for the reach tests of stencil cells
    // and sub-cells
    float bx0 = active ? li.x : 1e30f, by0 = active ? li.y : 1e30f, bz0 = active ? li.z : 1e30f;
    float bx1 = active ? li.x : -1e30f, by1 = active ? li.y : -1e30f, bz1 = active ? li.z : -1e30f;
    for (int d = 32; d >= 1; d >>= 1) {
        bx0 = fminf(bx0, __shfl_xor(bx0, d, 64));
        by0 = fminf(by0, __shfl_xor(by0, d, 64));
        bz0 = fminf(bz0, __shfl_xor(bz0, d, 64));
        bx1 = fmaxf(bx1, __shfl_xor(bx1, d, 64));
        by1 = fmaxf(by1, __shfl_xor(by1, d, 64));
        bz1 = fmaxf(bz1, __shfl_xor(bz1, d, 64));
    }
    // one stencil cell per lane (offset (t % 3 - 1, t / 3 % 3 - 1, t / 9 - 1)):
    // its range, if it comes within l of the chunk's box
    const int tl = lane < 27 ? lane : 13;
    const int lx = tl % 3 - 1, ly = (tl / 3) % 3 - 1, lz = tl / 9 - 1;
    const uint32_t nbl = cell_id(g, cx + lx, cy + ly, cz + lz);
    const float gx = lx < 0 ? bx0 : (lx > 0 ? g.cellb - bx1 : 0.0f);
    const float gy = ly < 0 ? by0 : (ly > 0 ? g.cellb - by1 : 0.0f);
    const float gz = lz < 0 ? bz0 : (lz > 0 ? g.cellb - bz1 : 0.0f);
    const bool lreach = lane < 27 && gx * gx + gy * gy + gz * gz < g.l2b_hi;
    uint32_t la = 0, lb = 0;
    if (lreach) {
        la = off[nbl];
        lb = off[nbl + 1];
    }
    const bool ldense = lb - la >= (uint32_t)kDenseMin;
    const bool lforward = lz > 0 || (lz == 0 && (ly > 0 || (ly == 0 && lx >= 0)));  // own cell included
    const bool lvisit = lreach && ldense && lforward;
    if (lvisit) {
        const uint64_t vm = __ballot(lvisit);
        const int slot = __popcll(vm & ((1ull << lane) - 1ull));
        dbase[wave][slot] = (int64_t)cellmap[nbl] * tstride;
        doff[wave][slot] = (int8_t)lane;
    }
    const uint64_t visit = __ballot(lvisit);
    const int nvisit = __popcll(visit);
    // sparse neighbour cells, all together
    stream_sparse_cells(parent, dens_s, sloc, spos, g, active, li, pi, wr, lreach && !ldense && lb > la, la, lb);
    if (nvisit == 0) return;
    __builtin_amdgcn_wave_barrier();
    // (visited dense cell, sub-cell) pairs, 64 at a time
    const int ntask = nvisit * nsub;
    for (int t0 = 0; t0 < ntask; t0 += 64) {
        const int tq = t0 + lane;
        uint32_t u0 = 0, u1 = 0;
        int fs = -1, st = 0;
        if (tq < ntask) {
            const int r = tq / nsub, sl = tq - r * nsub;
            st = doff[wave][r];
            const int64_t base = dbase[wave][r];
            const int ox = st % 3 - 1, oy = (st / 3) % 3 - 1, oz = st / 9 - 1;
            u0 = subtab[base + sl];
            u1 = subtab[base + sl + 1];
            if (st == 13 && u0 < h) u0 = h;  // own cell: from the chunk start on
            const int sx = sl % k, sy = (sl / k) % k, sz = sl / (k * k);
            // sub-cell box (neighbour frame) shifted into the chunk's frame
            const float ex = fmaxf(fmaxf(sx * subb + (float)ox * g.cellb - bx1,
                                         bx0 - ((sx + 1) * subb + (float)ox * g.cellb)), 0.0f);
            const float ey = fmaxf(fmaxf(sy * subb + (float)oy * g.cellb - by1,
                                         by0 - ((sy + 1) * subb + (float)oy * g.cellb)), 0.0f);
            const float ez = fmaxf(fmaxf(sz * subb + (float)oz * g.cellb - bz1,
                                         bz0 - ((sz + 1) * subb + (float)oz * g.cellb)), 0.0f);
            if (ex * ex + ey * ey + ez * ez < g.l2b_hi + 1e-4f) {
                for (uint32_t j = u0; j < u1; j++)
                    if (is_member(dens_s, j, g.dl0)) {
                        fs = (int)j;
                        break;
                    }
            }
        }
        // root hints of all sub-cells at once; a sub-cell whose set is the one
        // every active lane belongs to needs nothing
        int rL = fs >= 0 ? uf_find_hint(parent, fs) : -1;
        const uint64_t am = __ballot(active);
        for (;;) {
            const int w0 = lane_get(wr, __ffsll((unsigned long long)am) - 1);
            const int wcommon = __ballot(active && wr != w0) ? -2 : w0;
            const uint64_t todo = __ballot(fs >= 0 && rL != wcommon);
            if (!todo) break;
            const int S = __ffsll((unsigned long long)todo) - 1;
            const int f = lane_get(fs, S);
            const uint32_t e = lane_get(u1, S);
            const int sts = lane_get(st, S);
            const int rS = lane_get(rL, S);
            if (lane == S) fs = -1;  // done with it
            if (!__ballot(active && wr != rS)) continue;
            const bool joined = stream_range(parent, dens_s, sloc, spos, g, active, li, pi, wr, (uint32_t)f, e,
                                             sts % 3 - 1, (sts / 3) % 3 - 1, sts / 9 - 1, rS);
            // after a join the remaining hints may be stale: refresh them
            if (joined && fs >= 0) rL = uf_find_hint(parent, fs);
        }
    }
}

// Members among the sparse-cell particles (about one in ten), compacted so
// that the linking kernel runs without idle lanes.
__global__ __launch_bounds__(kBlock) void k_fof_sparse_flags(int64_t nsparse, Boxes bx,
                                                             const int32_t *__restrict__ sparse,
                                                             const float *__restrict__ dens_s,
                                                             uint32_t *__restrict__ flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nsparse) return;
    const int i = sparse[t];
    flag[t] = is_member(dens_s, i, bx.geo[box_of(bx, (uint32_t)i)].dl0) ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_fof_sparse_list(int64_t nsparse, const int32_t *__restrict__ sparse,
                                                            const uint32_t *__restrict__ flag,
                                                            const uint32_t *__restrict__ at,
                                                            int32_t *__restrict__ list) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nsparse && flag[t]) list[at[t]] = sparse[t];
}

// Members of sparse cells (the compacted list, its length on the device):
// links to the later members of sparse neighbour cells (pairs with dense cells
// are found by the dense chunks).  The offsets of a stencil plane are loaded
// together.  The list fills only the first blocks of the grid, which the plain
// block order spreads over all XCDs.  The kernel waits on memory: it is held
// to 64 VGPRs (eight wavefronts per SIMD; the compiler fits it without
// spilling).
__global__ __launch_bounds__(kBlock, 8) void k_fof_sparse(const uint32_t *__restrict__ count_p, Boxes bx,
                                                       const int32_t *__restrict__ sparse,
                                                       const float4 *__restrict__ sloc,
                                                       const float4 *__restrict__ spos,
                                                       const uint32_t *__restrict__ off,
                                                       const float *__restrict__ dens_s,
                                                       int32_t *parent) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)*count_p) return;
    const int i = sparse[t];
    const Geo &g = bx.geo[box_of(bx, (uint32_t)i)];
    const float4 li = sloc[i];
    const float4 pi = spos[i];
    const uint32_t c = __float_as_uint(li.w);
    const int nc = g.nc;
    int cx, cy, cz;
    cell_xyz(g, c, cx, cy, cz);
    const uint32_t x0 = (uint32_t)wrapc(cx - 1, nc), x1 = (uint32_t)cx, x2 = (uint32_t)wrapc(cx + 1, nc);
    int ri = uf_find_hint(parent, i);
    for (int oz = -1; oz <= 1; oz++) {
        const float zs = li.z - (float)oz * g.cellb;
        const float gz = oz < 0 ? li.z : (oz > 0 ? g.cellb - li.z : 0.0f);
        if (gz * gz >= g.l2b_hi) continue;
        const int z = wrapc(cz + oz, nc);
        uint32_t ra[9], rb[9];
#pragma unroll
        for (int oy = -1; oy <= 1; oy++) {
            const uint32_t row =
                g.cell_base + ((uint32_t)z * (uint32_t)nc + (uint32_t)wrapc(cy + oy, nc)) * (uint32_t)nc;
            const int r = (oy + 1) * 3;
            ra[r + 0] = off[row + x0];
            rb[r + 0] = off[row + x0 + 1];
            ra[r + 1] = off[row + x1];
            rb[r + 1] = off[row + x1 + 1];
            ra[r + 2] = off[row + x2];
            rb[r + 2] = off[row + x2 + 1];
        }
#pragma unroll
        for (int oy = -1; oy <= 1; oy++) {
            const float ys = li.y - (float)oy * g.cellb;
#pragma unroll
            for (int ox = -1; ox <= 1; ox++) {
                const int r = (oy + 1) * 3 + (ox + 1);
                const float gx = ox < 0 ? li.x : (ox > 0 ? g.cellb - li.x : 0.0f);
                const float gy = oy < 0 ? li.y : (oy > 0 ? g.cellb - li.y : 0.0f);
                if (gx * gx + gy * gy + gz * gz >= g.l2b_hi) continue;
                uint32_t a = ra[r];
                const uint32_t b = rb[r];
                if (b - a >= (uint32_t)kDenseMin) continue;
                if (a <= (uint32_t)i) a = (uint32_t)i + 1;
                const float xs = li.x - (float)ox * g.cellb;
                for (uint32_t j = a; j < b; j++) {
                    if (!is_member(dens_s, j, g.dl0)) continue;
                    if (!linked(xs, ys, zs, pi, sloc, spos, j, g)) continue;
                    if (uf_find_hint(parent, (int)j) == ri) continue;
                    uf_unite(parent, i, (int)j);
                    ri = uf_find_hint(parent, i);
                }
            }
        }
    }
}

// Roots of all members, read-only: nothing writes the forest in this pass, so
// every stored root is final (a compressing writer could otherwise replace a
// stored root with an older ancestor).
// The root of every particle's set into root[], and the smallest original
// index of every set into minorig[root] (one atomic per run of equal roots
// among consecutive lanes).
__global__ __launch_bounds__(kBlock) void k_fof_roots(int64_t n, const int32_t *__restrict__ parent,
                                                      const float4 *__restrict__ spos,
                                                      int32_t *__restrict__ root,
                                                      int32_t *__restrict__ minorig) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int r = -1;
    if (i < n) {
        r = parent[i];
        if (r >= 0) {
            for (int p = parent[r]; p != r; p = parent[r]) r = p;
        }
        root[i] = r;
    }
    const WaveRun run = wave_run(r);
    const int32_t o = i < n ? (int32_t)orig_of(spos[i]) : 0x7fffffff;
    const int32_t m = wave_run_min(r >= 0 ? o : 0x7fffffff, run);
    if (r >= 0 && run.rank == 0) atomicMin(&minorig[r], m);
}

// Group key (smallest original index of the group, in the call's numbering)
// per sorted particle, and the L0 label (box-local) in original order.  A key
// outside [0, n) would be an internal error; it is flagged instead of being
// used as an index.
__global__ __launch_bounds__(kBlock) void k_fof_keys(int64_t n, Boxes bx, const int32_t *__restrict__ root,
                                                     const int32_t *__restrict__ minorig,
                                                     const float4 *__restrict__ spos,
                                                     int32_t *__restrict__ gkey,
                                                     int32_t *__restrict__ l0_out,
                                                     int32_t *__restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int box = box_of(bx, (uint32_t)i);
    const int r = root[i];
    int k = r < 0 ? -1 : minorig[r];
    if (k >= n) {
        flag_error(err, 4, box);
        k = -1;
    }
    gkey[i] = k;
    if (l0_out) l0_out[orig_of(spos[i])] = k < 0 ? 0 : k + 1 - (int)bx.geo[box].orig_base;
}

// Group keys from caller-provided labels (1..n, 0 = none), in sorted order,
// and with dens_in the caller's densities gathered into sorted order too (one
// pass over the sorted records for both).
// Label and density of each particle side by side, in input order (one
// coalesced pass), so that the gather into sorted order below reads one
// 8-byte element per particle instead of two random 4-byte ones.
__global__ __launch_bounds__(kBlock) void k_pack_labels(int64_t n, const int32_t *__restrict__ l0_in,
                                                        const float *__restrict__ dens_in,
                                                        uint2 *__restrict__ packed) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n) return;
    packed[o] = make_uint2((uint32_t)l0_in[o], __float_as_uint(dens_in[o]));
}

__global__ __launch_bounds__(kBlock) void k_keys_from_labels(int64_t n, Boxes bx,
                                                             const int32_t *__restrict__ l0_in,
                                                             const uint2 *__restrict__ packed,
                                                             const float4 *__restrict__ spos,
                                                             int32_t *__restrict__ gkey,
                                                             float *__restrict__ dens_s,
                                                             int32_t *__restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int box = box_of(bx, (uint32_t)i);
    const Geo &g = bx.geo[box];
    const uint32_t o = orig_of(spos[i]);
    int32_t lab;
    if (packed) {
        const uint2 v = packed[o];
        lab = (int32_t)v.x;
        // the candidate search orders densities by their bit patterns, which
        // matches their values for non-negative numbers only: -0 becomes +0
        // (the same value), NaN and negative values are rejected
        uint32_t db = v.y == 0x80000000u ? 0u : v.y;
        if ((db >> 31) != 0u || (db & 0x7fffffffu) > 0x7f800000u) {
            flag_error(err, 16, box);
            db = 0u;
        }
        dens_s[i] = __uint_as_float(db);
    } else {
        lab = l0_in[o];
    }
    // labels are box-local (1 .. box size, 0 = outside every group)
    if (lab < 0 || (int64_t)lab > g.n) {
        flag_error(err, 2, box);
        lab = 0;
    }
    gkey[i] = lab > 0 ? lab - 1 + (int32_t)g.orig_base : -1;
}

}  // namespace

void launch_fof(int64_t n, const Boxes &bx, Work &w, hipStream_t s) {
    hipLaunchKernelGGL(k_fof_phase_a, grid(n), dim3(kBlock), 0, s, n, bx, w.sloc, w.f_sparse, w.ssub, w.cnt,
                       w.subtab, w.dens_s, w.parent);
    if (w.nchunks > 0)
        // one wavefront per workgroup: chunk costs differ widely, and a
        // finished wavefront's slot is free at once
        hipLaunchKernelGGL(k_fof_dense, dim3((unsigned)w.nchunks), dim3(64), 0, s, w.nchunks, bx,
                           w.chunks, w.sloc, w.spos, w.off, w.cnt, w.subtab, w.dens_s, w.parent);
    if (w.nsparse > 0) {
        // sparse members: flags, positions and list in arrays that are free
        // during this stage (chunk flags of the binning, the hard-case list)
        hipLaunchKernelGGL(k_fof_sparse_flags, grid(w.nsparse), dim3(kBlock), 0, s, w.nsparse, bx, w.sparse,
                           w.dens_s, w.f_chunk);
        scan_u32(w.f_chunk, w.s_chunk, w.nsparse, w.scan_tmp, s);
        hipLaunchKernelGGL(k_fof_sparse_list, grid(w.nsparse), dim3(kBlock), 0, s, w.nsparse, w.sparse,
                           w.f_chunk, w.s_chunk, w.hardlist);
        hipLaunchKernelGGL(k_fof_sparse, grid(w.nsparse), dim3(kBlock), 0, s, w.s_chunk + w.nsparse, bx,
                           w.hardlist, w.sloc, w.spos, w.off, w.dens_s, w.parent);
    }
    // roots go to the owner array (free until the assignment stage)
    fill_i32(w.minorig, 0x7fffffff, n, s);
    hipLaunchKernelGGL(k_fof_roots, grid(n), dim3(kBlock), 0, s, n, w.parent, w.spos, w.owner, w.minorig);
}

void launch_fof_labels(int64_t n, const Boxes &bx, Work &w, int32_t *l0_out, hipStream_t s) {
    hipLaunchKernelGGL(k_fof_keys, grid(n), dim3(kBlock), 0, s, n, bx, w.owner, w.minorig, w.spos, w.gkey,
                       l0_out, w.err);
}

void launch_keys_from_labels(const int32_t *l0_in, const float *dens_in, int64_t n, const Boxes &bx, Work &w,
                             hipStream_t s) {
    // the packed copy lives in the second radix key array (free after binning)
    uint2 *packed = nullptr;
    if (dens_in) {
        packed = reinterpret_cast<uint2 *>(w.rkey[1]);
        hipLaunchKernelGGL(k_pack_labels, grid(n), dim3(kBlock), 0, s, n, l0_in, dens_in, packed);
    }
    hipLaunchKernelGGL(k_keys_from_labels, grid(n), dim3(kBlock), 0, s, n, bx, l0_in, packed, w.spos, w.gkey,
                       w.dens_s, w.err);
}

}  // namespace hf
