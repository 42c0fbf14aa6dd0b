// L0 friends-of-friends over the particles denser than Delta_L0,min (Sec. 2.2.1):
// two members are friends when their separation is less than l; L0 groups are
// the connected components.
//
// Lock-free union-find in sorted (cell, sub-cell) order:
//   phase A  a sub-cell's diagonal is below l, so all members of a sub-cell are
//            friends: in dense cells every member points at the first member of
//            its sub-cell;
//   dense    one wavefront per dense chunk gathers the neighbour members within
//            reach 64 at a time and tests them against its lanes (FP32
//            prefilter on the cell-local coordinates, canonical FP64 distance
//            for the undecided band); it joins sets in its own view of the
//            forest and applies the resulting hooks in bulk;
//   sparse   members of sparse cells link to the later members of sparse
//            neighbour cells;
//   labels   compression, then 1 + the smallest ORIGINAL index of each set.
// Hooks always attach the larger root under the smaller one, so the sets, and
// therefore the labels, do not depend on thread scheduling.
#include "hf_internal.h"

namespace hf {

namespace {

inline dim3 grid(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

// Particles of the dense sub-cells gathered per round of the dense kernel.
// Half a wavefront: after each round with joins the forest and the roots are
// refreshed, so more, smaller rounds pass over more of the sub-cells that the
// joins made common (k_fof_dense 5.76 -> 5.53 ms on the 96-box batch against
// 64; 16 was faster there but slower on the 256^3 box).
constexpr int kGather = 32;

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

// Hooks a wavefront has decided on but not yet applied to the forest: lane
// k < n holds hook k, a root c to be attached under p < c.  Deferring them
// takes the compare-and-swap round trips out of the serial candidate loop:
// the wavefront joins sets in its own registers and applies all hooks at
// once, one lane each.
struct Hooks {
    int c = -1, p = -1, n = 0;
};

// Applies every queued hook: a compare-and-swap while c is still a root,
// otherwise a full union (c was hooked elsewhere meanwhile).
__device__ __forceinline__ void hooks_apply(int32_t *parent, Hooks &h) {
    if ((int)(threadIdx.x & 63) < h.n && atomicCAS(parent + h.c, h.c, h.p) != h.c) uf_unite(parent, h.c, h.p);
    h.n = 0;
}

__device__ __forceinline__ void hooks_push(int32_t *parent, Hooks &h, int c, int p) {
    if (h.n == 64) hooks_apply(parent, h);
    if ((int)(threadIdx.x & 63) == h.n) {
        h.c = c;
        h.p = p;
    }
    h.n++;
}

// A root hint read from the forest, moved through the queued hooks in the
// order they were queued: a hook's parent was a root of the wavefront's view
// when queued, so only a later hook can move it again.
__device__ __forceinline__ int hooks_map(const Hooks &h, int x) {
    for (int k = 0; k < h.n; k++)
        if (x == lane_get(h.c, k)) x = lane_get(h.p, k);
    return x;
}

// A value equal in every lane, moved to a scalar register.
__device__ __forceinline__ float uniform(float v) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// The lanes lk are linked to a particle whose set has the local root r.  In
// the wavefront's view of the forest (every root it holds is a node of its
// set), the smallest of r and the lanes' roots becomes the root of all of
// them; the others are queued as hooks under it, and every reference the
// wavefront holds to one of them (lane roots wr, candidate roots rc, task
// roots rt) is moved to it.
__device__ __forceinline__ void join_local(int32_t *parent, Hooks &h, bool lk, int r, int &wr, int &rc, int &rt) {
    // the smallest root: one step per distinct root among the linked lanes
    // (rarely more than one or two), with no cross-lane shuffle
    int m = r;
    for (uint64_t mask = __ballot(lk); mask;) {
        const int x = lane_get(wr, (int)__builtin_ctzll(mask));
        m = min(m, x);
        mask &= ~__ballot(wr == x);
    }
    if (r != m) {
        hooks_push(parent, h, r, m);
        if (wr == r) wr = m;
        if (rc == r) rc = m;
        if (rt == r) rt = m;
    }
    uint64_t mask;
    while ((mask = __ballot(lk && wr != m)) != 0ull) {
        const int x = lane_get(wr, (int)__builtin_ctzll(mask));
        hooks_push(parent, h, x, m);
        if (wr == x) wr = m;
        if (rc == x) rc = m;
        if (rt == x) rt = m;
    }
}

// Tests the member candidates of a batch (lane p: candidate p) against the
// chunk's lanes and joins their sets.  A candidate holds whether it is a
// member, its coordinates in the chunk's cell frame (units of b), its index
// and its local root rc; a candidate already in the set of every lane needs no
// test.  The loop runs over the smaller side: with fewer candidates than chunk
// particles, each candidate is broadcast to the chunk's lanes and joined to
// the lanes it links at once; otherwise the candidates stay in the lanes, the
// chunk's particles are broadcast one after the other (each candidate
// collecting a bit mask of the lanes it links), and the linked candidates are
// joined one after the other.
__device__ __forceinline__ void test_candidates(int32_t *parent, Hooks &h, const float4 *__restrict__ spos,
                                                const Geo &g, bool active, const float4 &li, uint32_t h0,
                                                int &wr, bool cmem, float qx, float qy, float qz, uint32_t cj,
                                                int &rc, int &rt) {
    const int lane = threadIdx.x & 63;
    const uint64_t am = __ballot(active);
    const int w0 = lane_get(wr, (int)__builtin_ctzll(am));
    const bool common = !__ballot(active && wr != w0);
    const bool need = cmem && !(common && rc == w0);
    const uint64_t nm = __ballot(need);
    if (!nm) return;
    if (__popcll(nm) < __popcll(am)) {
        for (uint64_t mm = nm; mm; mm &= mm - 1) {
            const int J = (int)__builtin_ctzll(mm);
            const int r = lane_get(rc, J);
            if (!__ballot(active && wr != r)) continue;
            const float dx = lane_get(qx, J) - li.x, dy = lane_get(qy, J) - li.y, dz = lane_get(qz, J) - li.z;
            const float d2f = d2_f32(dx, dy, dz);
            bool lk = active && wr != r && d2f < g.l2b_hi;
            if (lk && !(d2f < g.l2b_lo)) lk = d2_exact(spos[h0 + (uint32_t)lane], spos[lane_get(cj, J)], g.L, g.half) < g.l2;
            if (__ballot(lk)) join_local(parent, h, lk, r, wr, rc, rt);
        }
        return;
    }
    uint32_t lo = 0u, hi = 0u;  // linked chunk lanes 0..31 and 32..63
    for (uint64_t m = am; m; m &= m - 1) {
        const int I = (int)__builtin_ctzll(m);
        const float dx = qx - lane_get(li.x, I), dy = qy - lane_get(li.y, I), dz = qz - lane_get(li.z, I);
        const float d2f = d2_f32(dx, dy, dz);
        bool lk = need && d2f < g.l2b_hi;
        if (lk && !(d2f < g.l2b_lo)) lk = d2_exact(spos[h0 + (uint32_t)I], spos[cj], g.L, g.half) < g.l2;
        if (I < 32)
            lo |= lk ? 1u << I : 0u;
        else
            hi |= lk ? 1u << (I - 32) : 0u;
    }
    for (uint64_t mm = __ballot((lo | hi) != 0u); mm; mm &= mm - 1) {
        const int J = (int)__builtin_ctzll(mm);
        const int r = lane_get(rc, J);
        const uint32_t bits = lane < 32 ? lane_get(lo, J) >> lane : lane_get(hi, J) >> (lane - 32);
        const bool lk = (bits & 1u) != 0u && wr != r;
        if (__ballot(lk)) join_local(parent, h, lk, r, wr, rc, rt);
    }
}

// Phase A, which also initializes the forest: non-members get -1, members of
// sparse cells are roots, and members of dense cells point at the first member
// of their sub-cell (a valid forest: every parent is a member with a smaller
// or equal sorted index).  The first particle of every dense sub-cell also
// records the sub-cell's first member (-1 if none) in submem, laid out like
// the sub-cell table.
__global__ __launch_bounds__(kBlock) void k_fof_phase_a(int64_t n, Boxes bx, const float4 *__restrict__ sloc,
                                                        const uint32_t *__restrict__ f_sparse,
                                                        const uint16_t *__restrict__ ssub,
                                                        const uint32_t *__restrict__ cellmap,
                                                        const uint32_t *__restrict__ subtab,
                                                        const float *__restrict__ dens_s,
                                                        int32_t *__restrict__ parent,
                                                        int32_t *__restrict__ submem) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const Geo &g = bx.geo[box_of(bx, (uint32_t)i)];
    const bool mem = is_member(dens_s, i, g.dl0);
    if (f_sparse[i]) {
        parent[i] = mem ? (int32_t)i : -1;
        return;
    }
    const uint32_t c = __float_as_uint(sloc[i].w);
    const int64_t row = (int64_t)cellmap[c] * (bx.nsub_max + 1) + ssub[i];
    const uint32_t u0 = subtab[row];
    if (mem) {
        uint32_t f = u0;
        while (f < (uint32_t)i && !is_member(dens_s, f, g.dl0)) f++;
        parent[i] = (int32_t)f;
    } else {
        parent[i] = -1;
    }
    if ((uint32_t)i == u0) {
        const uint32_t u1 = subtab[row + 1];
        uint32_t f = u0;
        while (f < u1 && !is_member(dens_s, f, g.dl0)) f++;
        submem[row] = f < u1 ? (int32_t)f : -1;
    }
}

// Dense chunks, one wavefront each (lanes = the chunk's particles).  The wave
// visits the neighbour cells that come within l of some lane: sparse cells in
// all 26 directions, dense cells only in the forward half (the backward ones
// visit this cell themselves), and its own cell from the chunk start on.
// The 27 cell ranges are loaded at once (one stencil cell per lane).
// Neighbour particles are gathered 64 at a time (one per lane, shifted into
// the chunk's cell frame) and tested one after the other against all lanes;
// sets are joined in the wavefront's registers and the hooks applied to the
// forest in bulk after every gather round with joins, before each round of
// sub-cells and at the end (root hints read meanwhile are moved through the
// queued hooks):
//   sparse cells  all their particles, each member with its root;
//   dense cells   their sub-cells, 64 at a time (one per lane): range, first
//                 member (recorded by phase A) and that member's root.  A
//                 sub-cell already in the set of every lane is passed over
//                 (its members are one set); the particles of the others are
//                 gathered in lane order.
__global__ __launch_bounds__(kBlock, 8) void k_fof_dense(int64_t nchunks, Boxes bx,
                                                      const int32_t *__restrict__ chunks,
                                                      const float4 *__restrict__ sloc,
                                                      const float4 *__restrict__ spos,
                                                      const uint32_t *__restrict__ off,
                                                      const uint32_t *__restrict__ cellmap,
                                                      const uint32_t *__restrict__ subtab,
                                                      const int32_t *__restrict__ submem,
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
    bx0 = uniform(bx0);
    by0 = uniform(by0);
    bz0 = uniform(bz0);
    bx1 = uniform(bx1);
    by1 = uniform(by1);
    bz1 = uniform(bz1);
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
    const int nvisit = __popcll(__ballot(lvisit));
    Hooks hk;
    int no_rt = -1;
    // sparse neighbour cells: their particles numbered through a prefix sum of
    // the cell sizes; lane p finds the cell of particle p by one walk over the
    // cells that hold particles (their starts are scalars)
    {
        const int cntl = lreach && !ldense ? (int)(lb - la) : 0;
        int incl = cntl;
        for (int d = 1; d < 64; d <<= 1) {
            const int y = __shfl_up(incl, d, 64);
            if (lane >= d) incl += y;
        }
        const int P = lane_get(incl, 63);
        const uint64_t cells = __ballot(cntl > 0);
        for (int p0 = 0; p0 < P; p0 += 64) {
            const int p = p0 + lane;
            int t = 0;
            uint32_t jt = 0;
            for (uint64_t m = cells; m; m &= m - 1) {
                const int u = (int)__builtin_ctzll(m);
                const int stt = lane_get(incl, u) - lane_get(cntl, u);
                if (p >= stt) {
                    t = u;
                    jt = lane_get(la, u) + (uint32_t)(p - stt);
                }
            }
            bool cmem = false;
            float qx = 0.0f, qy = 0.0f, qz = 0.0f;
            int rc = -1;
            if (p < P) {
                const float4 lj = sloc[jt];
                cmem = is_member(dens_s, jt, g.dl0);
                qx = lj.x + (float)(t % 3 - 1) * g.cellb;
                qy = lj.y + (float)((t / 3) % 3 - 1) * g.cellb;
                qz = lj.z + (float)(t / 9 - 1) * g.cellb;
            }
            if (cmem) rc = hooks_map(hk, uf_find_hint(parent, (int)jt));
            test_candidates(parent, hk, spos, g, active, li, h, wr, cmem, qx, qy, qz, jt, rc, no_rt);
        }
    }
    if (nvisit > 0) {
        __builtin_amdgcn_wave_barrier();
        const int a0 = (int)__builtin_ctzll(__ballot(active));
        const int ntask = nvisit * nsub;
        const float inv_nsub = 1.0f / (float)nsub, inv_k = 1.0f / (float)k, inv_k2 = 1.0f / (float)(k * k);
        // (visited dense cell, sub-cell) pairs, 64 at a time
        for (int t0 = 0; t0 < ntask; t0 += 64) {
            // the forest learns this chunk's joins so far, the lanes their
            // current roots (a sub-cell joined meanwhile, by any chunk, is
            // then passed over)
            hooks_apply(parent, hk);
            if (active) wr = uf_find_hint(parent, wr);
            const int tq = t0 + lane;
            uint32_t u1 = 0;
            int fs = -1, st = 0;
            if (tq < ntask) {
                const int r = div_small(tq, inv_nsub), sl = tq - r * nsub;
                st = doff[wave][r];
                const int64_t base = dbase[wave][r];
                const int ox = st % 3 - 1, oy = (st / 3) % 3 - 1, oz = st / 9 - 1;
                uint32_t u0 = subtab[base + sl];
                u1 = subtab[base + sl + 1];
                const int32_t fm = submem[base + sl];
                const bool cut = st == 13 && u0 < h;
                if (cut) u0 = h;  // own cell: from the chunk start on
                const int sz = div_small(sl, inv_k2), syx = sl - sz * k * k, sy = div_small(syx, inv_k),
                          sx = syx - sy * k;
                // sub-cell box (neighbour frame) shifted into the chunk's frame
                const float ex = fmaxf(fmaxf(sx * subb + (float)ox * g.cellb - bx1,
                                             bx0 - ((sx + 1) * subb + (float)ox * g.cellb)), 0.0f);
                const float ey = fmaxf(fmaxf(sy * subb + (float)oy * g.cellb - by1,
                                             by0 - ((sy + 1) * subb + (float)oy * g.cellb)), 0.0f);
                const float ez = fmaxf(fmaxf(sz * subb + (float)oz * g.cellb - bz1,
                                             bz0 - ((sz + 1) * subb + (float)oz * g.cellb)), 0.0f);
                if (ex * ex + ey * ey + ez * ez < g.l2b_hi + 1e-4f && u1 > u0) {
                    // first member: recorded by phase A, searched where the
                    // own cell's sub-cell is cut at the chunk start
                    if (!cut) {
                        fs = fm;
                    } else {
                        for (uint32_t j = u0; j < u1; j++)
                            if (is_member(dens_s, j, g.dl0)) {
                                fs = (int)j;
                                break;
                            }
                    }
                }
            }
            int rt = fs >= 0 ? hooks_map(hk, uf_find_hint(parent, fs)) : -1;
            uint32_t pos = fs >= 0 ? (uint32_t)fs : 0u;  // next particle of the sub-cell to gather
            for (int gr = 0;; gr++) {
                // after the joins of a gather round the forest learns them
                // and the lanes and sub-cells read their current roots, so
                // that sub-cells joined meanwhile (by this chunk or another)
                // are passed over
                if (gr > 0 && hk.n > 0) {
                    hooks_apply(parent, hk);
                    if (active) wr = uf_find_hint(parent, wr);
                    if (rt >= 0) rt = uf_find_hint(parent, rt);
                }
                const int w0 = lane_get(wr, a0);
                const int wcommon = __ballot(active && wr != w0) ? -2 : w0;
                const uint32_t len = fs >= 0 && pos < u1 && rt != wcommon ? u1 - pos : 0u;
                uint32_t incl = len;
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t y = __shfl_up(incl, d, 64);
                    if (lane >= d) incl += y;
                }
                const uint32_t T = lane_get(incl, 63);
                if (T == 0) break;
                // lane p < kGather takes particle p of the sub-cells' runs laid end
                // to end
                int tst = 13, trt = -1;
                uint32_t jt = 0;
                for (uint64_t m = __ballot(len > 0); m; m &= m - 1) {
                    const int u = (int)__builtin_ctzll(m);
                    const uint32_t stu = lane_get(incl, u) - lane_get(len, u);
                    if (stu >= (uint32_t)kGather) break;
                    if ((uint32_t)lane >= stu) {
                        tst = lane_get(st, u);
                        trt = lane_get(rt, u);
                        jt = lane_get(pos, u) + ((uint32_t)lane - stu);
                    }
                }
                // every sub-cell moves past what this round takes from it
                const uint32_t mine = incl - len;
                if (mine < (uint32_t)kGather) pos += min(len, (uint32_t)kGather - mine);
                bool cmem = false;
                float qx = 0.0f, qy = 0.0f, qz = 0.0f;
                int rc = -1;
                if ((uint32_t)lane < T && lane < kGather) {
                    const float4 lj = sloc[jt];
                    cmem = is_member(dens_s, jt, g.dl0);
                    qx = lj.x + (float)(tst % 3 - 1) * g.cellb;
                    qy = lj.y + (float)((tst / 3) % 3 - 1) * g.cellb;
                    qz = lj.z + (float)(tst / 9 - 1) * g.cellb;
                    rc = trt;
                }
                test_candidates(parent, hk, spos, g, active, li, h, wr, cmem, qx, qy, qz, jt, rc, rt);
            }
        }
    }
    hooks_apply(parent, hk);
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

// Four entries per thread (t0, t0 + kBlock, ...), their flags loaded
// together (the kernel streams the flags).
constexpr int kSparseListIlp = 4;
__global__ __launch_bounds__(kBlock) void k_fof_sparse_list(int64_t nsparse, const int32_t *__restrict__ sparse,
                                                            const uint32_t *__restrict__ flag,
                                                            const uint32_t *__restrict__ at,
                                                            int32_t *__restrict__ list) {
    const int64_t t0 = (int64_t)blockIdx.x * (kBlock * kSparseListIlp) + threadIdx.x;
    uint32_t f[kSparseListIlp];
#pragma unroll
    for (int u = 0; u < kSparseListIlp; u++) {
        const int64_t t = t0 + (int64_t)u * kBlock;
        f[u] = t < nsparse ? flag[t] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kSparseListIlp; u++) {
        const int64_t t = t0 + (int64_t)u * kBlock;
        if (f[u]) list[at[t]] = sparse[t];
    }
}

// Members of sparse cells (the compacted list, its length on the device):
// links to the later members of sparse neighbour cells (pairs with dense cells
// are found by the dense chunks).  The offsets of a stencil plane are loaded
// together, and the plane's particles are walked as one sequence.  The list fills only the first blocks of the grid, which the plain
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
#pragma unroll 1
    for (int oz = -1; oz <= 1; oz++) {
        const float gz = oz < 0 ? li.z : (oz > 0 ? g.cellb - li.z : 0.0f);
        if (gz * gz >= g.l2b_hi) continue;
        const int z = wrapc(cz + oz, nc);
        // the plane's later particles in sparse cells within reach: per cell
        // its first one and, packed three bits each, their count
        uint32_t ra[9], cnts = 0;
#pragma unroll
        for (int oy = -1; oy <= 1; oy++) {
            const uint32_t row =
                g.cell_base + ((uint32_t)z * (uint32_t)nc + (uint32_t)wrapc(cy + oy, nc)) * (uint32_t)nc;
            const uint32_t o[6] = {off[row + x0], off[row + x0 + 1], off[row + x1],
                                   off[row + x1 + 1], off[row + x2], off[row + x2 + 1]};
            const float gy = oy < 0 ? li.y : (oy > 0 ? g.cellb - li.y : 0.0f);
#pragma unroll
            for (int ox = -1; ox <= 1; ox++) {
                const int r = (oy + 1) * 3 + (ox + 1);
                uint32_t a = o[2 * (ox + 1)];
                const uint32_t b = o[2 * (ox + 1) + 1];
                const float gx = ox < 0 ? li.x : (ox > 0 ? g.cellb - li.x : 0.0f);
                const bool use = b - a < (uint32_t)kDenseMin && gx * gx + gy * gy + gz * gz < g.l2b_hi;
                if (a <= (uint32_t)i) a = (uint32_t)i + 1;
                ra[r] = a;
                cnts |= (use && b > a ? b - a : 0u) << (3 * r);
            }
        }
        // walked as one sequence (cell after cell): the wavefront waits on the
        // longest lane's count for the plane, not on the longest of each cell
        uint32_t j = 0, e = 0;
        float xs = 0.0f, ys = 0.0f, zs = 0.0f;
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
                // the lane's coordinates in this cell's frame
                xs = li.x - (float)(r % 3 - 1) * g.cellb;
                ys = li.y - (float)(r / 3 - 1) * g.cellb;
                zs = li.z - (float)oz * g.cellb;
            }
            const uint32_t jj = j++;
            const float dj = dens_s[jj];
            const float4 lj = sloc[jj];
            if (!((double)dj > g.dl0)) continue;
            const float d2f = d2_f32(lj.x - xs, lj.y - ys, lj.z - zs);
            if (d2f >= g.l2b_hi) continue;
            if (!(d2f < g.l2b_lo) && !(d2_exact(pi, spos[jj], g.L, g.half) < g.l2)) continue;
            if (uf_find_hint(parent, (int)jj) == ri) continue;
            uf_unite(parent, i, (int)jj);
            ri = uf_find_hint(parent, i);
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
    // the first members of the dense sub-cells go to the sub-cell maxima's
    // argument table (free until the candidate stage)
    hipLaunchKernelGGL(k_fof_phase_a, grid(n), dim3(kBlock), 0, s, n, bx, w.sloc, w.f_sparse, w.ssub, w.cnt,
                       w.subtab, w.dens_s, w.parent, w.subarg);
    if (w.nchunks > 0)
        // one wavefront per workgroup: chunk costs differ widely, and a
        // finished wavefront's slot is free at once
        hipLaunchKernelGGL(k_fof_dense, dim3((unsigned)w.nchunks), dim3(64), 0, s, w.nchunks, bx,
                           w.chunks, w.sloc, w.spos, w.off, w.cnt, w.subtab, w.subarg, w.dens_s, w.parent);
    if (w.nsparse > 0) {
        // sparse members: flags, positions and list in arrays that are free
        // during this stage (chunk flags of the binning, the hard-case list)
        hipLaunchKernelGGL(k_fof_sparse_flags, grid(w.nsparse), dim3(kBlock), 0, s, w.nsparse, bx, w.sparse,
                           w.dens_s, w.f_chunk);
        scan_u32(w.f_chunk, w.s_chunk, w.nsparse, w.scan_tmp, s);
        hipLaunchKernelGGL(k_fof_sparse_list, grid((w.nsparse + kSparseListIlp - 1) / kSparseListIlp), dim3(kBlock),
                           0, s, w.nsparse, w.sparse,
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
