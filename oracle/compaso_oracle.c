/*
 * CompaSO group-finding oracle.  TEST INFRASTRUCTURE: only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg load this library.
 * The product path (the HIP library) never links, includes or calls it, and the
 * two share no code.
 *
 * A plain, slow FP64 CPU implementation of the on-the-fly group finder of
 * Hadzhiyska et al., "CompaSO: A new halo finder for competitive assignment to
 * spherical overdensities":
 *   - kernel density per particle            (Sec. 2.2.1, kernel W = 1 - r^2/b^2;
 *                                             normalisation from App. B.2)
 *   - L0 friends-of-friends over dense particles (Sec. 2.2.1; FoF as in Sec. 1)
 *   - CompaSO L1 inside every L0 group, run literally as the sequential loop of
 *     Sec. 2.2.2 steps 1-4 (nucleus, R_L1 from all L0 particles, eligibility,
 *     competitive reassignment, density floor), with the flat-rotation-curve
 *     enclosed density of Sec. 2.3.2 and squared distances as in Sec. 2.3.3.
 *   - output cut at the minimum L1 halo size (end of Sec. 2.2.2, Table 1).
 *   - the threshold radius either from the sorted distances or by the radial
 *     bins of Sec. 2.3.4 (orc_radius_search; both give the same count), and
 *     the members collected into group order by the partition sweep of
 *     Sec. 2.3.5 (orc_group_sweep).
 *   - the near-threshold events through which a slightly different density
 *     field can change the labels (orc_events; used to attribute label
 *     differences against a float32 field to the density comparisons of
 *     Sec. 2.2.1 and 2.2.2).
 *
 * Neighbour search has two modes that must agree exactly: brute force over all
 * pairs (mode 0) and a cell list (mode 1) whose cells are at least the search
 * radius, so that every pair within the radius is in the 27-cell stencil.
 *
 * Canonical geometric predicate (used by every label decision):
 *   dx = (double)x_j - (double)x_i; if dx > L/2: dx -= L; else if dx < -L/2: dx += L
 *   d2 = (dx*dx + dy*dy) + dz*dz           (IEEE FP64, no fused multiply-add)
 * Enclosed-count predicates use E3(e) = (e*e)*e on squared distances and
 * II(k) = (double)k*(double)k, so that no root is ever taken:
 *   R^3 = i/K with K = (4 pi/3) Delta_L1 nbar  =>  r < R  <=>  K^2 e^3 < i^2.
 *
 * Parameter vector (doubles), shared layout with the Python wrapper only:
 *   [0] box  [1] mean_density (<=0: N/L^3)  [2] b_kernel (units of l_mean)
 *   [3] l_fof (units of l_mean)  [4] delta_l0_min  [5] delta_l1  [6] alpha_elig
 *   [7] c_roche  [8] n_new_min  [9] particle_mass  [10] n_l1_min  [11] self_count
 *   [12] delta_l2
 * Derived vector (orc_derive):
 *   [0] nbar [1] b [2] l [3] b2 [4] l2 [5] norm [6] K [7] K2 [8] floor [9] A6 [10] C3
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

enum { P_BOX, P_NBAR, P_B, P_L, P_DL0, P_DL1, P_ALPHA, P_CROCHE, P_NNEW, P_MASS,
       P_NL1MIN, P_SELF, P_DL2, P_COUNT };
enum { D_NBAR, D_B, D_L, D_B2, D_L2, D_NORM, D_K, D_K2, D_FLOOR, D_A6, D_C3, D_COUNT };

/* ---------------------------------------------------------------- constants */

/* Derived constants.
 * - l_mean = nbar^(-1/3); b and l are given in units of l_mean (Sec. 2.2.1,
 *   Table 1: DensityKernelRad 0.4, FoFLinkingLength 0.25).
 * - norm: Delta = norm * sum W, with the unit-integral kernel so that a uniform
 *   field has Delta = 1; int W d^3r = (2/5)(4 pi/3) b^3 (App. B.2).
 * - K: the enclosed density inside radius r around a nucleus with k particles
 *   inside is k / ((4 pi/3) r^3 nbar) in units of the mean, so it equals
 *   Delta_L1 when r^3 = k / K (Sec. 2.2.2 step 1).
 * - floor: kernel-smoothed central density of a singular isothermal sphere whose
 *   200x-mean radius holds N_new,min particles (Sec. 2.2.2 step 4); the SIS
 *   A/r^2 with A = (Delta_L1/3) R^2 smoothed by the unit-integral W gives 5A/b^2
 *   at its centre (App. B.2, r < b branch at r -> 0).
 * - A6 = alpha^6 (r < alpha R  <=>  K^2 e^3 < alpha^6 i^2), C3 = c_Roche^3
 *   (competition cubed: R_new^2/e_new >= c R_own^2/e_own, Sec. 2.2.2 step 3 with
 *   the flat-rotation-curve model of Sec. 2.3.2). */
int orc_derive(const double *p, int64_t n, double *d)
{
    double box = p[P_BOX];
    if (!(box > 0.0)) return 1;
    double nbar = p[P_NBAR] > 0.0 ? p[P_NBAR] : (double)n / ((box * box) * box);
    if (!(nbar > 0.0)) return 1;
    double lmean = cbrt(1.0 / nbar);
    double b = p[P_B] * lmean;
    double l = p[P_L] * lmean;
    double K = ((4.0 * ORC_PI) / 3.0) * p[P_DL1] * nbar;
    double rnew = cbrt(p[P_NNEW] / K);
    double a3 = (p[P_ALPHA] * p[P_ALPHA]) * p[P_ALPHA];
    d[D_NBAR] = nbar;
    d[D_B] = b;
    d[D_L] = l;
    d[D_B2] = b * b;
    d[D_L2] = l * l;
    d[D_NORM] = 15.0 / (((8.0 * ORC_PI) * ((b * b) * b)) * nbar);
    d[D_K] = K;
    d[D_K2] = K * K;
    d[D_FLOOR] = ((5.0 * p[P_DL1]) / 3.0) * (rnew * rnew) / (b * b);
    d[D_A6] = a3 * a3;
    d[D_C3] = (p[P_CROCHE] * p[P_CROCHE]) * p[P_CROCHE];
    return 0;
}

/* ---------------------------------------------------------------- geometry */

/* Minimum-image squared distance in FP64 (canonical predicate, see header). */
static double d2_periodic(const float *pos, int64_t i, int64_t j, double L)
{
    double half = 0.5 * L;
    double dx = (double)pos[3 * j + 0] - (double)pos[3 * i + 0];
    double dy = (double)pos[3 * j + 1] - (double)pos[3 * i + 1];
    double dz = (double)pos[3 * j + 2] - (double)pos[3 * i + 2];
    if (dx > half) dx -= L; else if (dx < -half) dx += L;
    if (dy > half) dy -= L; else if (dy < -half) dy += L;
    if (dz > half) dz -= L; else if (dz < -half) dz += L;
    double xx = dx * dx;
    double yy = dy * dy;
    double zz = dz * dz;
    double s = xx + yy;
    return s + zz;
}

static double e3(double e) { double ee = e * e; return ee * e; }
static double ii(int64_t k) { double x = (double)k; return x * x; }

/* -------------------------------------------------------------- cell list */

typedef struct {
    int nc;              /* cells per side (>= 3) */
    double cell;         /* cell side = L / nc >= search radius */
    int64_t *start;      /* [nc^3 + 1] */
    int64_t *items;      /* particle indices grouped by cell, ascending inside a cell */
} grid_t;

static int cell_coord(double x, double cell, int nc)
{
    int c = (int)floor(x / cell);
    if (c < 0) c = 0;
    if (c >= nc) c = nc - 1;
    return c;
}

/* Returns 0 on success, 1 if the box is too small for a 27-cell stencil
 * (callers then fall back to brute force), 2 on allocation failure. */
static int grid_build(grid_t *g, int64_t n, const float *pos, double L, double rmin)
{
    double ncd = floor(L / rmin);
    if (!(ncd >= 3.0)) return 1;
    if (ncd > 512.0) ncd = 512.0;           /* coarser cells stay >= rmin */
    int nc = (int)ncd;
    int64_t ncell = (int64_t)nc * nc * nc;
    g->nc = nc;
    g->cell = L / nc;
    g->start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    g->items = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *key = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!g->start || !g->items || !key) { free(g->start); free(g->items); free(key); return 2; }
    for (int64_t i = 0; i < n; i++) {
        int cx = cell_coord(pos[3 * i + 0], g->cell, nc);
        int cy = cell_coord(pos[3 * i + 1], g->cell, nc);
        int cz = cell_coord(pos[3 * i + 2], g->cell, nc);
        key[i] = ((int64_t)cz * nc + cy) * nc + cx;
        g->start[key[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; c++) g->start[c + 1] += g->start[c];
    int64_t *fill = (int64_t *)malloc((size_t)ncell * sizeof(int64_t));
    if (!fill) { free(g->start); free(g->items); free(key); return 2; }
    memcpy(fill, g->start, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) g->items[fill[key[i]]++] = i;
    free(fill);
    free(key);
    return 0;
}

static void grid_free(grid_t *g) { free(g->start); free(g->items); }

/* The 27 neighbour cells (with periodic wrap) of particle i's cell. */
static void grid_stencil(const grid_t *g, const float *pos, int64_t i, int64_t out[27])
{
    int nc = g->nc;
    int cx = cell_coord(pos[3 * i + 0], g->cell, nc);
    int cy = cell_coord(pos[3 * i + 1], g->cell, nc);
    int cz = cell_coord(pos[3 * i + 2], g->cell, nc);
    int t = 0;
    for (int oz = -1; oz <= 1; oz++)
        for (int oy = -1; oy <= 1; oy++)
            for (int ox = -1; ox <= 1; ox++) {
                int x = (cx + ox + nc) % nc, y = (cy + oy + nc) % nc, z = (cz + oz + nc) % nc;
                out[t++] = ((int64_t)z * nc + y) * nc + x;
            }
}

/* ---------------------------------------------------------------- density */

/* Kernel density of one particle: Delta_i = norm * sum_{j != i, r < b} (1 - r^2/b^2)
 * (Sec. 2.2.1; unit-integral normalisation of App. B.2).  The self pair is left
 * out unless self_count is set, in which case W(0) = 1 is added. */
static double density_one(int64_t i, int64_t n, const float *pos, double L,
                          const double *d, int self_count, const grid_t *g)
{
    double b2 = d[D_B2];
    double s = self_count ? 1.0 : 0.0;
    if (g) {
        int64_t st[27];
        grid_stencil(g, pos, i, st);
        for (int t = 0; t < 27; t++)
            for (int64_t k = g->start[st[t]]; k < g->start[st[t] + 1]; k++) {
                int64_t j = g->items[k];
                if (j == i) continue;
                double r2 = d2_periodic(pos, i, j, L);
                if (r2 < b2) s += 1.0 - r2 / b2;
            }
    } else {
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            double r2 = d2_periodic(pos, i, j, L);
            if (r2 < b2) s += 1.0 - r2 / b2;
        }
    }
    return d[D_NORM] * s;
}

/* mode 0: brute force; mode 1: cell list.  out[n] receives Delta (FP64). */
int orc_density(int64_t n, const float *pos, const double *p, int mode, double *out)
{
    double d[D_COUNT];
    if (orc_derive(p, n, d)) return 1;
    double L = p[P_BOX];
    int self_count = p[P_SELF] != 0.0;
    grid_t g;
    int use_grid = 0;
    if (mode == 1) {
        int rc = grid_build(&g, n, pos, L, d[D_B]);
        if (rc == 2) return 2;
        use_grid = rc == 0;
    }
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; i++)
        out[i] = density_one(i, n, pos, L, d, self_count, use_grid ? &g : NULL);
    if (use_grid) grid_free(&g);
    return 0;
}

/* Density of selected particles only (cell list over the whole box). */
int orc_density_sample(int64_t n, const float *pos, const double *p, int64_t m,
                       const int64_t *which, double *out)
{
    double d[D_COUNT];
    if (orc_derive(p, n, d)) return 1;
    double L = p[P_BOX];
    int self_count = p[P_SELF] != 0.0;
    grid_t g;
    int rc = grid_build(&g, n, pos, L, d[D_B]);
    if (rc == 2) return 2;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t t = 0; t < m; t++)
        out[t] = density_one(which[t], n, pos, L, d, self_count, rc == 0 ? &g : NULL);
    if (rc == 0) grid_free(&g);
    return 0;
}

/* ---------------------------------------------------------------- L0 FoF */

static int64_t uf_find(int64_t *parent, int64_t x)
{
    while (parent[x] != x) {
        parent[x] = parent[parent[x]];
        x = parent[x];
    }
    return x;
}

/* Union keeping the smaller index as the root, so a component's root is its
 * minimum original index. */
static void uf_union(int64_t *parent, int64_t a, int64_t b)
{
    int64_t ra = uf_find(parent, a), rb = uf_find(parent, b);
    if (ra == rb) return;
    if (ra < rb) parent[rb] = ra; else parent[ra] = rb;
}

/* Whether the ball of squared radius r2 around particle i can reach stencil
 * cell t (offset (t % 3 - 1, t / 3 % 3 - 1, t / 9 - 1) from i's cell): the
 * squared gap between i and that cell's slab along each axis, with a relative
 * margin of 1e-6 so that rounding never drops a pair. */
static int cell_in_reach(const grid_t *g, const float *pos, int64_t i, int t, double r2)
{
    double gap2 = 0.0;
    int off[3] = { t % 3 - 1, (t / 3) % 3 - 1, t / 9 - 1 };
    for (int a = 0; a < 3; a++) {
        if (off[a] == 0) continue;
        double x = (double)pos[3 * i + a];
        int c = cell_coord(x, g->cell, g->nc);
        double gap = off[a] < 0 ? x - (double)c * g->cell : (double)(c + 1) * g->cell - x;
        if (gap > 0.0) gap2 += gap * gap;
    }
    return gap2 < r2 * (1.0 + 1e-6);
}

typedef struct { int32_t *a; int64_t len, cap; } links_t;

static void links_push(links_t *b, int64_t i, int64_t j)
{
    if (b->len + 2 > b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1 << 16;
        b->a = (int32_t *)realloc(b->a, (size_t)b->cap * sizeof(int32_t));
    }
    b->a[b->len++] = (int32_t)i;
    b->a[b->len++] = (int32_t)j;
}

/* L0 groups: friends-of-friends with linking length l over the particles whose
 * density exceeds delta_l0_min (Sec. 2.2.1); two members are friends when their
 * separation is less than l (FoF definition, Sec. 1).  l0[i] = 1 + minimum
 * original index of i's group for members, 0 for non-members.  n_groups counts
 * groups including single-member ones.
 * The groups are the connected components of the friend pairs, which do not
 * depend on the order in which pairs are joined: in cell-list mode the pairs
 * (i, j > i) of a block of particles are listed by several threads at once and
 * then joined one by one; brute force joins them as it finds them. */
int orc_fof(int64_t n, const float *pos, const double *p, const double *dens,
            int mode, int32_t *l0, int64_t *n_groups)
{
    double d[D_COUNT];
    if (orc_derive(p, n, d)) return 1;
    double L = p[P_BOX], l2 = d[D_L2], dmin = p[P_DL0];
    int64_t *parent = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!parent) return 2;
    for (int64_t i = 0; i < n; i++) parent[i] = i;
    grid_t g;
    int use_grid = 0;
    if (mode == 1) {
        int rc = grid_build(&g, n, pos, L, d[D_L]);
        if (rc == 2) { free(parent); return 2; }
        use_grid = rc == 0;
    }
    if (use_grid) {
        int nt = 1;
#ifdef _OPENMP
        nt = omp_get_max_threads();
#endif
        links_t *buf = (links_t *)calloc((size_t)nt, sizeof(links_t));
        const int64_t block = (int64_t)1 << 16;
        for (int64_t i0 = 0; i0 < n; i0 += block) {
            int64_t i1 = i0 + block < n ? i0 + block : n;
            #pragma omp parallel for schedule(dynamic, 256)
            for (int64_t i = i0; i < i1; i++) {
                if (!(dens[i] > dmin)) continue;
                int tid = 0;
#ifdef _OPENMP
                tid = omp_get_thread_num();
#endif
                int64_t st[27];
                grid_stencil(&g, pos, i, st);
                for (int t = 0; t < 27; t++) {
                    if (!cell_in_reach(&g, pos, i, t, l2)) continue;
                    for (int64_t k = g.start[st[t]]; k < g.start[st[t] + 1]; k++) {
                        int64_t j = g.items[k];
                        if (j <= i || !(dens[j] > dmin)) continue;
                        if (d2_periodic(pos, i, j, L) < l2) links_push(&buf[tid], i, j);
                    }
                }
            }
            for (int t = 0; t < nt; t++) {
                for (int64_t k = 0; k < buf[t].len; k += 2) uf_union(parent, buf[t].a[k], buf[t].a[k + 1]);
                buf[t].len = 0;
            }
        }
        for (int t = 0; t < nt; t++) free(buf[t].a);
        free(buf);
    } else {
        for (int64_t i = 0; i < n; i++) {
            if (!(dens[i] > dmin)) continue;
            for (int64_t j = i + 1; j < n; j++) {
                if (!(dens[j] > dmin)) continue;
                if (d2_periodic(pos, i, j, L) < l2) uf_union(parent, i, j);
            }
        }
    }
    int64_t groups = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!(dens[i] > dmin)) { l0[i] = 0; continue; }
        int64_t r = uf_find(parent, i);
        if (r == i) groups++;
        l0[i] = (int32_t)(r + 1);
    }
    if (use_grid) grid_free(&g);
    free(parent);
    *n_groups = groups;
    return 0;
}

/* ---------------------------------------------------------------- CompaSO */

typedef struct { int64_t nucleus; int64_t ienc; int64_t count; } halo_t;

typedef struct {
    const float *pos;
    const double *dens;
    const int32_t *l0;
    double L;
    const double *d;
    const grid_t *g;       /* cell list with cells >= b, or NULL (brute force) */
    int64_t n;
    double rbin;           /* > 0: threshold radius by radial bins of this width (Sec. 2.3.4) */
} ctx_t;

/* "Denser" in the total order used for nuclei: higher density first, ties
 * broken by lower original index. */
static int denser(const double *dens, int64_t a, int64_t b)
{
    if (dens[a] != dens[b]) return dens[a] > dens[b];
    return a < b;
}

/* Step 2 peak condition: q is denser than every other particle of its L0 group
 * (eligible or not) within the kernel radius b. */
static int is_local_peak(const ctx_t *c, int64_t q)
{
    double b2 = c->d[D_B2];
    int32_t lab = c->l0[q];
    if (c->g) {
        int64_t st[27];
        grid_stencil(c->g, c->pos, q, st);
        for (int t = 0; t < 27; t++)
            for (int64_t k = c->g->start[st[t]]; k < c->g->start[st[t] + 1]; k++) {
                int64_t j = c->g->items[k];
                if (j == q || c->l0[j] != lab) continue;
                if (d2_periodic(c->pos, q, j, c->L) < b2 && denser(c->dens, j, q)) return 0;
            }
    } else {
        for (int64_t j = 0; j < c->n; j++) {
            if (j == q || c->l0[j] != lab) continue;
            if (d2_periodic(c->pos, q, j, c->L) < b2 && denser(c->dens, j, q)) return 0;
        }
    }
    return 1;
}

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------- threshold radius (R_L1) */

/* Enclosed count of the threshold radius from the squared distances e[0..m)
 * of the m members of a group to a nucleus (the nucleus itself included, at
 * e = 0), as defined by sorting (Sec. 2.2.2 step 1 and Sec. 2.3.3): with the
 * distances in ascending order d_0 <= d_1 <= ..., the enclosed count at sorted
 * position k is k, and the radius is the innermost d_k (k >= 1) at which the
 * enclosed density k / (K d_k^3) drops below 1 (in units of Delta_L1), i.e.
 * K^2 d_k^6 > k^2.  No such position: m (the radius is bounded by the L0
 * group).  es receives the sorted copy (scratch of m doubles). */
static int64_t radius_sorted(const double *e, int64_t m, double K2, double *es)
{
    memcpy(es, e, (size_t)m * sizeof(double));
    qsort(es, (size_t)m, sizeof(double), cmp_double);
    for (int64_t k = 1; k < m; k++)
        if (K2 * e3(es[k]) > ii(k)) return k;
    return m;
}

/* Squared outer edge of radial bin j of width w: ((j + 1) w)^2. */
static double bin_edge2(int64_t j, double w)
{
    double r = (double)(j + 1) * w;
    return r * r;
}

/* The same count by the search of Sec. 2.3.4: the members are partitioned
 * into radial bins of width w (bin j holds edge2(j-1) <= e < edge2(j)).  Let
 * C_j be the number of members inside bin j's inner edge.  If those C_j
 * members placed at the bin's outer edge still reach the density threshold
 * (K^2 edge2(j)^3 <= C_j^2), every member of the bin, being inside that edge
 * and at a sorted position >= C_j, has enclosed density above the threshold:
 * the bin is passed over.  Otherwise its members are sorted and searched in
 * order; a bin without the crossing sends the search on outwards.  The
 * innermost bin is always searched (C_0 = 0).  *searched (may be NULL)
 * receives the number of bins searched. */
static int64_t radius_bins(const double *e, int64_t m, double K2, double w, int64_t *searched)
{
    double emax = 0.0;
    for (int64_t t = 0; t < m; t++) if (e[t] > emax) emax = e[t];
    int64_t nb = (int64_t)(sqrt(emax) / w) + 1;
    while (!(emax < bin_edge2(nb - 1, w))) nb++;
    int64_t *cnt = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
    double *v = (double *)malloc((size_t)(m > 0 ? m : 1) * sizeof(double));
    int64_t found = m, nsearch = 0;
    /* bin of each member: the first j with e < edge2(j) */
    for (int64_t t = 0; t < m; t++) {
        int64_t j = (int64_t)(sqrt(e[t]) / w);
        if (j >= nb) j = nb - 1;
        while (j > 0 && e[t] < bin_edge2(j - 1, w)) j--;
        while (!(e[t] < bin_edge2(j, w))) j++;
        cnt[j]++;
    }
    int64_t C = 0;   /* members inside the current bin's inner edge */
    for (int64_t j = 0; j < nb && found == m; C += cnt[j], j++) {
        if (cnt[j] == 0) continue;
        if (K2 * e3(bin_edge2(j, w)) <= ii(C)) continue;   /* threshold not crossed in this bin */
        nsearch++;
        double lo = j > 0 ? bin_edge2(j - 1, w) : -1.0, hi = bin_edge2(j, w);
        int64_t c = 0;
        for (int64_t t = 0; t < m; t++)
            if (e[t] >= lo && e[t] < hi) v[c++] = e[t];
        qsort(v, (size_t)c, sizeof(double), cmp_double);
        for (int64_t u = 0; u < c; u++) {
            int64_t k = C + u;
            if (k >= 1 && k < m && K2 * e3(v[u]) > ii(k)) { found = k; break; }
        }
    }
    free(cnt);
    free(v);
    if (searched) *searched = nsearch;
    return found;
}

/* Exported for the tests: mode 0 the sorted definition, mode 1 the radial-bin
 * search with bin width w (searched: bins searched). */
int64_t orc_radius_search(const double *e, int64_t m, double K2, int mode, double w, int64_t *searched)
{
    if (m <= 0) return 0;
    if (mode == 1) return radius_bins(e, m, K2, w, searched);
    double *es = (double *)malloc((size_t)m * sizeof(double));
    int64_t k = radius_sorted(e, m, K2, es);
    free(es);
    if (searched) *searched = 0;
    return k;
}

typedef struct { double dens; int64_t idx; int64_t t; } rank_t;

/* Descending density, ties by ascending original index (the "denser" order). */
static int cmp_rank(const void *a, const void *b)
{
    const rank_t *x = (const rank_t *)a, *y = (const rank_t *)b;
    if (x->dens != y->dens) return x->dens > y->dens ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* One L0 group, literally as the sequential loop of Sec. 2.2.2:
 *   repeat: take the densest particle that is still eligible, at or above the
 *   nucleation floor (step 4) and a local peak within b (step 2; the densest
 *   particle of the group always is one, step 1); find R from ALL particles of
 *   the group (sorted squared distances: the enclosed count at sorted position k
 *   is k, and R_L1 is the innermost radius where the enclosed density falls
 *   below Delta_L1); assign the particles inside R if unassigned or if their
 *   model enclosed density Delta_L1 R^2/r^2 w.r.t. the new nucleus is at least
 *   c_Roche times that w.r.t. their current halo (step 3, Sec. 2.3.2); mark
 *   the particles inside alpha R ineligible (step 1).
 * mem[0..m) are the members' original indices.  Returns the halos in creation
 * order; owner[t] is the local halo index of mem[t] (-1: none). */
static int64_t compaso_group(const ctx_t *c, const int64_t *mem, int64_t m,
                             halo_t **halos_out, int64_t *owner)
{
    const double *d = c->d;
    double K2 = d[D_K2], A6 = d[D_A6], C3 = d[D_C3], floor_nuc = d[D_FLOOR];
    rank_t *order = (rank_t *)malloc((size_t)m * sizeof(rank_t));
    unsigned char *elig = (unsigned char *)malloc((size_t)m);
    signed char *peak = (signed char *)malloc((size_t)m);   /* -1 unknown, 0, 1 */
    double *e = (double *)malloc((size_t)m * sizeof(double));
    double *es = (double *)malloc((size_t)m * sizeof(double));
    double *eown = (double *)malloc((size_t)m * sizeof(double));
    int64_t *iown = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    int64_t cap = 4, nh = 0;
    halo_t *halos = (halo_t *)malloc((size_t)cap * sizeof(halo_t));
    for (int64_t t = 0; t < m; t++) {
        order[t].dens = c->dens[mem[t]];
        order[t].idx = mem[t];
        order[t].t = t;
        elig[t] = 1;
        peak[t] = -1;
        owner[t] = -1;
    }
    /* the search order of steps 1-2: descending density */
    qsort(order, (size_t)m, sizeof(rank_t), cmp_rank);
    for (;;) {
        int64_t cand = -1;
        for (int64_t r = 0; r < m; r++) {
            int64_t t = order[r].t;
            int64_t q = order[r].idx;
            if (!(order[r].dens >= floor_nuc)) break;  /* step 4: stop below the floor */
            if (!elig[t]) continue;
            if (peak[t] < 0) peak[t] = (signed char)is_local_peak(c, q);
            if (peak[t]) { cand = q; break; }
        }
        if (cand < 0) break;
        /* R from all particles of the group: sorted squared distances, or
         * the radial-bin search of Sec. 2.3.4 (the same count) */
        for (int64_t t = 0; t < m; t++) e[t] = d2_periodic(c->pos, cand, mem[t], c->L);
        int64_t ienc = c->rbin > 0.0 ? radius_bins(e, m, K2, c->rbin, NULL) : radius_sorted(e, m, K2, es);
        if (nh == cap) { cap *= 2; halos = (halo_t *)realloc(halos, (size_t)cap * sizeof(halo_t)); }
        int64_t h = nh++;
        halos[h].nucleus = cand;
        halos[h].ienc = ienc;
        halos[h].count = 0;
        double iih = ii(ienc);
        for (int64_t t = 0; t < m; t++) {
            double ee = e[t];
            if (K2 * e3(ee) < iih) {                       /* inside R */
                if (owner[t] < 0) {
                    owner[t] = h; eown[t] = ee; iown[t] = ienc;
                } else {
                    double lhs = iih * e3(eown[t]);
                    double rhs = (C3 * ii(iown[t])) * e3(ee);
                    if (lhs >= rhs) { owner[t] = h; eown[t] = ee; iown[t] = ienc; }
                }
            }
            if (K2 * e3(ee) < A6 * iih) elig[t] = 0;      /* inside alpha R */
        }
    }
    for (int64_t t = 0; t < m; t++)
        if (owner[t] >= 0) halos[owner[t]].count++;
    free(order); free(elig); free(peak);
    free(e); free(es); free(eown); free(iown);
    *halos_out = halos;
    return nh;
}

/* CompaSO L1 over all L0 groups, then the output cut (N >= n_l1_min).
 * Outputs (host arrays):
 *   halo_id[n]   1 + nucleus original index of the particle's halo if kept, else 0
 *   owner_all[n] (optional) 1 + nucleus index of the owning halo before the cut
 *   table (optional, capacity cap, ascending id): t_id, t_nucleus, t_l0, t_n, t_ienc
 *   *n_halos     number of kept halos (may exceed cap; then the table is partial)
 *   *n_found     number of halos before the cut
 *   found list (optional, capacity fcap): every halo before the cut, grouped by
 *                L0 group (ascending label) and in creation order inside a group:
 *                f_nucleus, f_ienc, f_count, f_l0
 * dens may be any density field (e.g. the GPU's values) and l0 any L0 labelling
 * with the 1 + min-index convention. */
int orc_compaso(int64_t n, const float *pos, const double *p, const double *dens,
                const int32_t *l0, int mode, int32_t *halo_id, int32_t *owner_all,
                int64_t cap, int32_t *t_id, int32_t *t_nucleus, int32_t *t_l0,
                int32_t *t_n, int32_t *t_ienc, int64_t *n_halos, int64_t *n_found,
                int64_t fcap, int32_t *f_nucleus, int32_t *f_ienc, int32_t *f_count,
                int32_t *f_l0)
{
    double d[D_COUNT];
    if (orc_derive(p, n, d)) return 1;
    int64_t nmin = (int64_t)p[P_NL1MIN];
    /* group members by label (counting sort on label-1; members ascending) */
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *mem = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!cnt || !mem) { free(cnt); free(mem); return 2; }
    for (int64_t i = 0; i < n; i++) if (l0[i] > 0) cnt[l0[i]]++;   /* l0 in 1..n */
    int64_t ngroups = 0;
    for (int64_t k = 1; k <= n; k++) if (cnt[k]) ngroups++;
    int64_t *gstart = (int64_t *)malloc((size_t)(ngroups + 1) * sizeof(int64_t));
    int64_t *glab = (int64_t *)malloc((size_t)(ngroups > 0 ? ngroups : 1) * sizeof(int64_t));
    int64_t *off = (int64_t *)calloc((size_t)n + 2, sizeof(int64_t));
    if (!gstart || !glab || !off) { free(cnt); free(mem); free(gstart); free(glab); free(off); return 2; }
    int64_t gi = 0, acc = 0;
    for (int64_t k = 1; k <= n; k++)
        if (cnt[k]) { glab[gi] = k; gstart[gi] = acc; off[k] = acc; acc += cnt[k]; gi++; }
    gstart[ngroups] = acc;
    for (int64_t i = 0; i < n; i++) if (l0[i] > 0) mem[off[l0[i]]++] = i;
    free(off);
    free(cnt);

    grid_t g;
    int use_grid = 0;
    if (mode & 1) {
        int rc = grid_build(&g, n, pos, p[P_BOX], d[D_B]);
        if (rc == 2) { free(mem); free(gstart); free(glab); return 2; }
        use_grid = rc == 0;
    }
    /* mode bit 2: R_L1 by radial bins of width max(b, l)/sqrt(3) (Sec. 2.3.4) */
    double rbin = (mode & 2) ? fmax(d[D_B], d[D_L]) / sqrt(3.0) : 0.0;
    ctx_t c = { pos, dens, l0, p[P_BOX], d, use_grid ? &g : NULL, n, rbin };

    halo_t **gh = (halo_t **)calloc((size_t)(ngroups > 0 ? ngroups : 1), sizeof(halo_t *));
    int64_t *gnh = (int64_t *)calloc((size_t)(ngroups > 0 ? ngroups : 1), sizeof(int64_t));
    int64_t *own = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n; i++) { halo_id[i] = 0; if (owner_all) owner_all[i] = 0; }

    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < ngroups; k++) {
        int64_t s = gstart[k], m = gstart[k + 1] - s;
        gnh[k] = compaso_group(&c, mem + s, m, &gh[k], own + s);
    }

    /* output cut and ids; table ascending by id via a flag sweep over indices */
    int64_t found = 0, kept = 0;
    unsigned char *keep_flag = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    int32_t *hN = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int32_t *hI = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    int32_t *hL = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    for (int64_t k = 0; k < ngroups; k++) {
        int64_t s = gstart[k], m = gstart[k + 1] - s;
        for (int64_t h = 0; h < gnh[k]; h++) {
            halo_t *H = &gh[k][h];
            if (found + h < fcap) {
                if (f_nucleus) f_nucleus[found + h] = (int32_t)H->nucleus;
                if (f_ienc) f_ienc[found + h] = (int32_t)H->ienc;
                if (f_count) f_count[found + h] = (int32_t)H->count;
                if (f_l0) f_l0[found + h] = (int32_t)glab[k];
            }
            if (H->count >= nmin) {
                keep_flag[H->nucleus] = 1;
                hN[H->nucleus] = (int32_t)H->count;
                hI[H->nucleus] = (int32_t)H->ienc;
                hL[H->nucleus] = (int32_t)glab[k];
                kept++;
            }
        }
        for (int64_t t = 0; t < m; t++) {
            int64_t q = mem[s + t];
            int64_t o = own[s + t];
            if (o < 0) continue;
            int64_t nuc = gh[k][o].nucleus;
            if (owner_all) owner_all[q] = (int32_t)(nuc + 1);
            if (gh[k][o].count >= nmin) halo_id[q] = (int32_t)(nuc + 1);
        }
        found += gnh[k];
        free(gh[k]);
    }
    int64_t w = 0;
    for (int64_t i = 0; i < n; i++) {
        if (!keep_flag[i]) continue;
        if (w < cap) {
            if (t_id) t_id[w] = (int32_t)(i + 1);
            if (t_nucleus) t_nucleus[w] = (int32_t)i;
            if (t_l0) t_l0[w] = hL[i];
            if (t_n) t_n[w] = hN[i];
            if (t_ienc) t_ienc[w] = hI[i];
        }
        w++;
    }
    *n_halos = kept;
    if (n_found) *n_found = found;
    free(keep_flag); free(hN); free(hI); free(hL);
    free(gh); free(gnh); free(own);
    if (use_grid) grid_free(&g);
    free(mem); free(gstart); free(glab);
    return 0;
}

/* ------------------------------------------------- near-threshold events */

/* Where a density field that differs from this one by at most
 * tol * max(Delta, 1) per particle (the float32 field of another
 * implementation, say) can change the labels.  Every label predicate is exact
 * given the densities, so labels can only change through a density comparison:
 *   EV_L0CUT  |Delta_i - Delta_L0,min| <= tol max(Delta_L0,min, 1): i may enter
 *             or leave the L0 members (Sec. 2.2.1);
 *   EV_FLOOR  a member with |Delta_i - floor| <= tol max(floor, 1): it may cross
 *             the nucleation floor (Sec. 2.2.2 step 4);
 *   EV_PEAK   a member at or above floor - tol max(floor, 1) whose densest other
 *             group member within b, at density M, has
 *             |Delta_i - M| <= 2 tol max(Delta_i, M, 1): the peak test of
 *             Sec. 2.2.2 step 2 may flip;
 *   EV_ORDER  a nucleus candidate (at or above the floor, denser than every
 *             other group member within b) within 2 tol max(., ., 1) of another
 *             candidate of its group: the order in which nuclei are taken
 *             (Sec. 2.2.2 step 1) may flip;
 *   EV_GROUP  a member of an L0 group that holds a member with EV_FLOOR,
 *             EV_PEAK or EV_ORDER, or that has a member within l of (or equal
 *             to) a particle with EV_L0CUT.
 * l0 is the L0 labelling of this field (1 + minimum index, 0 = not a member).
 * mode 0: brute force; mode 1: cell list.  ev[n] receives the bits. */
enum { EV_L0CUT = 1, EV_FLOOR = 2, EV_PEAK = 4, EV_ORDER = 8, EV_GROUP = 128 };

typedef struct { int32_t lab; double dens; int64_t idx; } cand_t;

static int cmp_cand(const void *a, const void *b)
{
    const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
    if (x->lab != y->lab) return x->lab < y->lab ? -1 : 1;
    if (x->dens != y->dens) return x->dens > y->dens ? -1 : 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

static double fmax3(double a, double b, double c) { return fmax(fmax(a, b), c); }

int orc_events(int64_t n, const float *pos, const double *p, const double *dens,
               const int32_t *l0, int mode, double tol, uint8_t *ev)
{
    double d[D_COUNT];
    if (orc_derive(p, n, d)) return 1;
    double L = p[P_BOX], b2 = d[D_B2], l2 = d[D_L2], dl0 = p[P_DL0], fl = d[D_FLOOR];
    double tcut = tol * fmax(dl0, 1.0), tfl = tol * fmax(fl, 1.0);
    grid_t g;
    int rc = mode == 1 ? grid_build(&g, n, pos, L, fmax(d[D_B], d[D_L])) : 1;
    if (rc == 2) return 2;
    const grid_t *gp = rc == 0 ? &g : NULL;
    unsigned char *cand = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
    unsigned char *gflag = (unsigned char *)calloc((size_t)n + 1, 1);
    if (!cand || !gflag) { free(cand); free(gflag); if (gp) grid_free(&g); return 2; }

    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; i++) {
        uint8_t e = 0;
        if (fabs(dens[i] - dl0) <= tcut) e |= EV_L0CUT;
        if (l0[i] > 0) {
            if (fabs(dens[i] - fl) <= tfl) e |= EV_FLOOR;
            if (dens[i] >= fl - tfl) {
                /* densest other member of the group within b, and whether a
                 * denser one (total order) exists */
                double M = -HUGE_VAL;
                int denser_near = 0;
                int64_t st[27];
                int nt = 1;
                if (gp) { grid_stencil(gp, pos, i, st); nt = 27; }
                for (int t = 0; t < nt; t++) {
                    int64_t k0 = gp ? gp->start[st[t]] : 0, k1 = gp ? gp->start[st[t] + 1] : n;
                    for (int64_t k = k0; k < k1; k++) {
                        int64_t j = gp ? gp->items[k] : k;
                        if (j == i || l0[j] != l0[i]) continue;
                        if (!(d2_periodic(pos, i, j, L) < b2)) continue;
                        if (dens[j] > M) M = dens[j];
                        if (dens[j] > dens[i] || (dens[j] == dens[i] && j < i)) denser_near = 1;
                    }
                }
                if (M > -HUGE_VAL && fabs(dens[i] - M) <= 2.0 * tol * fmax3(dens[i], M, 1.0)) e |= EV_PEAK;
                if (dens[i] >= fl && !denser_near) cand[i] = 1;
            }
        }
        ev[i] = e;
    }
    /* candidates of one group in descending density: neighbours in that order
     * closer than the tolerance may swap */
    int64_t nc = 0;
    for (int64_t i = 0; i < n; i++) nc += cand[i];
    cand_t *cs = (cand_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(cand_t));
    nc = 0;
    for (int64_t i = 0; i < n; i++)
        if (cand[i]) { cs[nc].lab = l0[i]; cs[nc].dens = dens[i]; cs[nc].idx = i; nc++; }
    qsort(cs, (size_t)nc, sizeof(cand_t), cmp_cand);
    for (int64_t k = 0; k + 1 < nc; k++)
        if (cs[k].lab == cs[k + 1].lab &&
            fabs(cs[k].dens - cs[k + 1].dens) <= 2.0 * tol * fmax3(cs[k].dens, cs[k + 1].dens, 1.0)) {
            ev[cs[k].idx] |= EV_ORDER;
            ev[cs[k + 1].idx] |= EV_ORDER;
        }
    free(cs);
    /* groups touched by an event */
    for (int64_t i = 0; i < n; i++)
        if (l0[i] > 0 && (ev[i] & (EV_FLOOR | EV_PEAK | EV_ORDER))) gflag[l0[i]] = 1;
    for (int64_t i = 0; i < n; i++) {
        if (!(ev[i] & EV_L0CUT)) continue;
        if (l0[i] > 0) gflag[l0[i]] = 1;
        int64_t st[27];
        int nt = 1;
        if (gp) { grid_stencil(gp, pos, i, st); nt = 27; }
        for (int t = 0; t < nt; t++) {
            int64_t k0 = gp ? gp->start[st[t]] : 0, k1 = gp ? gp->start[st[t] + 1] : n;
            for (int64_t k = k0; k < k1; k++) {
                int64_t j = gp ? gp->items[k] : k;
                if (l0[j] > 0 && d2_periodic(pos, i, j, L) < l2) gflag[l0[j]] = 1;
            }
        }
    }
    for (int64_t i = 0; i < n; i++)
        if (l0[i] > 0 && gflag[l0[i]]) ev[i] |= EV_GROUP;
    free(cand);
    free(gflag);
    if (gp) grid_free(&g);
    return 0;
}

/* ------------------------------------------------------- group order */

/* Members collected into group order by the sweep of Sec. 2.3.5: the index
 * array is partitioned in place, first for the largest halo (the most likely
 * to be the biggest set), then for the unassigned particles (halo_id 0, the
 * other big set, so that later passes do not go through them again), then for
 * each remaining halo in table order.  row_id / row_n: the halo table's ids
 * and sizes (nrows rows).  Output in table layout: row r's members in
 * members[start[r] .. start[r+1]), the unassigned ones from start[nrows] to n;
 * the order inside a run is whatever the in-place partitions leave.  Returns
 * 1 when a particle's label is neither 0 nor a table id. */
static int64_t partition_by(int64_t *idx, int64_t lo, int64_t hi, const int32_t *halo_id, int32_t id)
{
    /* in-place two-pointer partition of idx[lo, hi): label == id first */
    int64_t a = lo, b = hi - 1;
    for (;;) {
        while (a <= b && halo_id[idx[a]] == id) a++;
        while (a <= b && halo_id[idx[b]] != id) b--;
        if (a >= b) break;
        int64_t t = idx[a]; idx[a] = idx[b]; idx[b] = t;
        a++; b--;
    }
    return a;
}

int orc_group_sweep(int64_t n, const int32_t *halo_id, int64_t nrows, const int32_t *row_id,
                    const int32_t *row_n, int64_t *members, int64_t *start)
{
    int64_t *idx = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *seg = (int64_t *)malloc((size_t)(nrows + 1) * 2 * sizeof(int64_t));
    if (!idx || !seg) { free(idx); free(seg); return 2; }
    for (int64_t i = 0; i < n; i++) idx[i] = i;
    int64_t big = -1;
    for (int64_t r = 0; r < nrows; r++)
        if (big < 0 || row_n[r] > row_n[big]) big = r;
    int64_t lo = 0;
    /* seg[2r], seg[2r+1]: row r's range in idx; row nrows: the unassigned */
    if (big >= 0) { int64_t e = partition_by(idx, lo, n, halo_id, row_id[big]); seg[2 * big] = lo; seg[2 * big + 1] = e; lo = e; }
    { int64_t e = partition_by(idx, lo, n, halo_id, 0); seg[2 * nrows] = lo; seg[2 * nrows + 1] = e; lo = e; }
    for (int64_t r = 0; r < nrows; r++) {
        if (r == big) continue;
        int64_t e = partition_by(idx, lo, n, halo_id, row_id[r]);
        seg[2 * r] = lo; seg[2 * r + 1] = e; lo = e;
    }
    int rc = lo == n ? 0 : 1;   /* every particle went to some run */
    int64_t w = 0;
    for (int64_t r = 0; r <= nrows; r++) {
        start[r] = w;
        for (int64_t t = seg[2 * r]; t < seg[2 * r + 1]; t++) members[w++] = idx[t];
    }
    free(idx);
    free(seg);
    return rc;
}

/* ------------------------------------------------------ redshift scaling */

/* Thresholds at redshift z (Sec. 2.3.1) for a flat universe of matter and a
 * cosmological constant: Omega_m(z) = Om (1+z)^3 / (Om (1+z)^3 + 1 - Om).
 * The Bryan & Norman fitting function Delta_base = 18 pi^2 + 82 x - 39 x^2,
 * x = Omega_m(z) - 1, is relative to the critical density; relative to the
 * mean it is Delta_base / Omega_m(z).  The EdS thresholds are multiplied by
 * s = Delta_base / (18 pi^2 Omega_m(z)) (s = 1 for Om = 1): Delta_L1 (200 ->
 * 258.2 at z = 0.5, Om = 0.315, Table 1), Delta_L2 (800 -> 1033.0) and the L0
 * threshold (60 -> 77.5, Table 1); the FoF linking length by s^(-1/3); the
 * kernel radius b is unchanged. */
int orc_params_at_redshift(const double *pin, double om0, double z, double *pout)
{
    if (!(om0 > 0.0 && om0 <= 1.0) || !(z > -1.0)) return 1;
    for (int k = 0; k < P_COUNT; k++) pout[k] = pin[k];
    double a = 1.0 + z;
    double m = om0 * ((a * a) * a);
    double omz = m / (m + (1.0 - om0));
    double x = omz - 1.0;
    double tpi2 = 18.0 * ORC_PI * ORC_PI;
    double base = tpi2 + 82.0 * x - 39.0 * (x * x);
    double scale = base / (tpi2 * omz);
    pout[P_DL1] = pin[P_DL1] * scale;
    pout[P_DL2] = pin[P_DL2] * scale;
    pout[P_DL0] = pin[P_DL0] * scale;
    pout[P_L] = pin[P_L] / cbrt(scale);
    return 0;
}

/* -------------------------------------------- level 2 and halo statistics */

static int cmp_float(const void *a, const void *b)
{
    float x = *(const float *)a, y = *(const float *)b;
    return (x > y) - (x < y);
}

static int cmp_desc_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x < y) - (x > y);
}

/* Centre of mass of the particles mem[t] with own[t] == sel (sel < 0: all),
 * about the particle ref: each minimum-image offset is rounded to a multiple
 * of 2^-32 and the multiples are summed exactly in 64-bit integers, so the
 * mean does not depend on the order of summation; the result is wrapped into
 * [0, L). */
static void com_about(const float *pos, double L, const int64_t *mem, const int64_t *own,
                      int64_t m, int64_t sel, int64_t ref, double out[3])
{
    int64_t S[3] = {0, 0, 0};
    int64_t cnt = 0;
    for (int64_t t = 0; t < m; t++) {
        if (sel >= 0 && own[t] != sel) continue;
        int64_t j = mem[t];
        for (int a = 0; a < 3; a++) {
            double dx = (double)pos[3 * j + a] - (double)pos[3 * ref + a];
            if (dx > 0.5 * L) dx -= L;
            else if (dx < -0.5 * L) dx += L;
            S[a] += llrint(dx * 4294967296.0);
        }
        cnt++;
    }
    for (int a = 0; a < 3; a++) {
        double c = (double)S[a];
        c = c / (double)cnt;
        c = c * (1.0 / 4294967296.0);
        double x = (double)pos[3 * ref + a] + c;
        if (x < 0.0) x += L;
        else if (x >= L) x -= L;
        out[a] = x;
    }
}

static const int kPct[9] = {10, 25, 33, 50, 67, 75, 90, 95, 98};

/* Level 2 (end of Sec. 2.2.2): inside every L1 halo the competitive SO steps
 * are repeated with Delta_L2 in place of Delta_L1 everywhere (enclosed
 * density, nucleation floor), the L1 halo's members playing the part of the
 * L0 group (peak test, enclosed counts, assignment).  Then per L1 halo, in
 * ascending id (Table 1):
 *   si[5*k..]  id, N, number of L2 halos, first L2 nucleus (-1 if none), its N
 *   sf[22*k..] x_com[3] (L1 centre of mass), x_L2com[3] (centre of mass of the
 *              first L2 halo, = x_com if none), masses of the 5 largest L2
 *              halos (descending, 0 beyond their number), r_XX about x_L2com
 *              for XX = 10 25 33 50 67 75 90 95 98, vcirc_max, rvcirc_max.
 * r_XX: the k-th smallest distance, k = ceil(XX N / 100), of the L1 members
 * from x_L2com (squared distances in FP64, then rounded to float32 and sorted).
 * vcirc: with the members sorted by that distance, k of them lie within r_k;
 * the circular velocity sqrt(G m_p k / r_k) (G = 1) is largest at the first
 * position maximising k^2 / r_k^2 (members at r = 0 are skipped).
 * l2: every L2 halo (L1 id, nucleus, enclosed count, N) in L1 order and
 * creation order; l2_owner (optional): per particle 1 + the nucleus index of
 * its L2 halo, 0 if none; members/gstart: the L1 members grouped by halo
 * (ascending id, ascending index).  Returns 3 if the number of L1 halos
 * exceeds cap. */
int orc_l2_stats(int64_t n, const float *pos, const double *p, const double *dens,
                 const int32_t *halo_id, int mode, int64_t cap, int64_t *n_l1,
                 int32_t *si, double *sf, int64_t l2cap, int32_t *l2, int64_t *n_l2_total,
                 int32_t *l2_owner, int32_t *members, int64_t *gstart_out)
{
    double q[P_COUNT], d[D_COUNT];
    for (int k = 0; k < P_COUNT; k++) q[k] = p[k];
    q[P_DL1] = p[P_DL2];
    if (orc_derive(q, n, d)) return 1;
    double L = p[P_BOX];
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *mem = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!cnt || !mem) { free(cnt); free(mem); return 2; }
    for (int64_t i = 0; i < n; i++) if (halo_id[i] > 0) cnt[halo_id[i]]++;
    int64_t ng = 0;
    for (int64_t k = 1; k <= n; k++) if (cnt[k]) ng++;
    *n_l1 = ng;
    if (ng > cap) { free(cnt); free(mem); return 3; }
    int64_t *gstart = (int64_t *)malloc((size_t)(ng + 1) * sizeof(int64_t));
    int64_t *glab = (int64_t *)malloc((size_t)(ng > 0 ? ng : 1) * sizeof(int64_t));
    int64_t *off = (int64_t *)calloc((size_t)n + 2, sizeof(int64_t));
    int64_t gi = 0, acc = 0;
    for (int64_t k = 1; k <= n; k++)
        if (cnt[k]) { glab[gi] = k; gstart[gi] = acc; off[k] = acc; acc += cnt[k]; gi++; }
    gstart[ng] = acc;
    for (int64_t i = 0; i < n; i++) if (halo_id[i] > 0) mem[off[halo_id[i]]++] = i;
    free(off);
    free(cnt);
    grid_t g;
    int use_grid = 0;
    if (mode == 1) {
        int rc = grid_build(&g, n, pos, L, d[D_B]);
        if (rc == 2) { free(mem); free(gstart); free(glab); return 2; }
        use_grid = rc == 0;
    }
    ctx_t c = { pos, dens, halo_id, L, d, use_grid ? &g : NULL, n, 0.0 };
    halo_t **gh = (halo_t **)calloc((size_t)(ng > 0 ? ng : 1), sizeof(halo_t *));
    int64_t *gnh = (int64_t *)calloc((size_t)(ng > 0 ? ng : 1), sizeof(int64_t));
    int64_t *own = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));

    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < ng; k++) {
        int64_t s0 = gstart[k], m = gstart[k + 1] - s0;
        gnh[k] = compaso_group(&c, mem + s0, m, &gh[k], own + s0);
        int64_t nuc = glab[k] - 1;
        double com[3], com2[3];
        com_about(pos, L, mem + s0, own + s0, m, -1, nuc, com);
        if (gnh[k] > 0) com_about(pos, L, mem + s0, own + s0, m, 0, gh[k][0].nucleus, com2);
        else for (int a = 0; a < 3; a++) com2[a] = com[a];
        float *fd = (float *)malloc((size_t)m * sizeof(float));
        for (int64_t t = 0; t < m; t++) {
            int64_t j = mem[s0 + t];
            double dd[3];
            for (int a = 0; a < 3; a++) {
                double dx = (double)pos[3 * j + a] - com2[a];
                if (dx > 0.5 * L) dx -= L;
                else if (dx < -0.5 * L) dx += L;
                dd[a] = dx;
            }
            fd[t] = (float)((dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2]);
        }
        qsort(fd, (size_t)m, sizeof(float), cmp_float);
        int32_t *I = si + 5 * k;
        double *F = sf + 22 * k;
        I[0] = (int32_t)glab[k];
        I[1] = (int32_t)m;
        I[2] = (int32_t)gnh[k];
        I[3] = gnh[k] > 0 ? (int32_t)gh[k][0].nucleus : -1;
        I[4] = gnh[k] > 0 ? (int32_t)gh[k][0].count : 0;
        for (int a = 0; a < 3; a++) { F[a] = com[a]; F[3 + a] = com2[a]; }
        int64_t *counts = (int64_t *)malloc((size_t)(gnh[k] > 0 ? gnh[k] : 1) * sizeof(int64_t));
        for (int64_t h = 0; h < gnh[k]; h++) counts[h] = gh[k][h].count;
        qsort(counts, (size_t)gnh[k], sizeof(int64_t), cmp_desc_i64);
        for (int u = 0; u < 5; u++) F[6 + u] = u < gnh[k] ? (double)counts[u] * p[P_MASS] : 0.0;
        free(counts);
        for (int u = 0; u < 9; u++) {
            int64_t kk = ((int64_t)kPct[u] * m + 99) / 100;
            F[11 + u] = sqrt((double)fd[kk - 1]);
        }
        int64_t best = -1;
        double vbest = 0.0;
        for (int64_t t = 0; t < m; t++) {
            if (!(fd[t] > 0.0f)) continue;
            double v = ((double)(t + 1) * (double)(t + 1)) / (double)fd[t];
            if (best < 0 || v > vbest) { best = t; vbest = v; }
        }
        if (best >= 0) {
            double r = sqrt((double)fd[best]);
            F[20] = sqrt((p[P_MASS] * (double)(best + 1)) / r);
            F[21] = r;
        } else {
            F[20] = 0.0;
            F[21] = 0.0;
        }
        free(fd);
    }
    if (l2_owner) {
        for (int64_t i = 0; i < n; i++) l2_owner[i] = 0;
        for (int64_t k = 0; k < ng; k++)
            for (int64_t t = gstart[k]; t < gstart[k + 1]; t++)
                if (own[t] >= 0) l2_owner[mem[t]] = (int32_t)(gh[k][own[t]].nucleus + 1);
    }
    int64_t w = 0;
    for (int64_t k = 0; k < ng; k++) {
        for (int64_t h = 0; h < gnh[k]; h++, w++)
            if (w < l2cap) {
                l2[4 * w + 0] = (int32_t)glab[k];
                l2[4 * w + 1] = (int32_t)gh[k][h].nucleus;
                l2[4 * w + 2] = (int32_t)gh[k][h].ienc;
                l2[4 * w + 3] = (int32_t)gh[k][h].count;
            }
        free(gh[k]);
    }
    *n_l2_total = w;
    if (members) for (int64_t t = 0; t < acc; t++) members[t] = (int32_t)mem[t];
    if (gstart_out) for (int64_t k = 0; k <= ng; k++) gstart_out[k] = gstart[k];
    free(gh); free(gnh); free(own);
    if (use_grid) grid_free(&g);
    free(mem); free(gstart); free(glab);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}
