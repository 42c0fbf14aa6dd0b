// C ABI of libhf: argument checks, derived constants, the scratch arena of a
// context, and the order of the stages for each entry point.  Every pass runs
// over a set of boxes at once (a single-box call is a set of one): the boxes'
// constants go to the device as a table, particles and cells are numbered box
// after box, and each stage is one launch over all of them.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <initializer_list>
#include <mutex>
#include <string>

#include "hf_lane.h"

#define HF_PI 3.14159265358979323846

// Scratch of hf_find_noalloc: a region of device memory that every GPU the
// library runs on holds from the load of the code object to the end of the
// process, so that the entry point allocates nothing.  Host code never uses the
// array's name as an address: its device address is taken once per device with
// hipGetSymbolAddress (hf_create) and kept in scratch_addr.
static __device__ __align__(256) unsigned char scratch[hf::kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_addr[kMaxDevices] = {};

// Device address of the scratch array on `device` (current), or null.
void *scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_addr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        scratch_addr[device] = ptr;
    }
    return scratch_addr[device];
}

}  // namespace

namespace {

using hf::Geo;
using hf::Lane;
using hf::Work;

enum { D_NBAR, D_B, D_L, D_B2, D_L2, D_NORM, D_K, D_K2, D_FLOOR, D_A6, D_C3, D_COUNT };

hf_status fail(Lane *c, hf_status st, const std::string &msg) {
    if (c) c->err = msg;
    return st;
}

#define HIP_OK(ctx, expr)                                                               \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(ctx, HF_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool finite(double x) { return x == x && x != HUGE_VAL && x != -HUGE_VAL; }

// Derived constants, in the same sequence of IEEE operations as documented in
// hf.h (multiplications and divisions only, so no contraction can change them).
hf_status derive(const hf_params *p, int64_t n, double *d) {
    if (!p) return HF_ERR_INVALID;
    const double v[] = {p->box, p->mean_density, p->b_kernel, p->l_fof, p->delta_l0_min,
                        p->delta_l1, p->delta_l2, p->alpha_elig, p->c_roche, p->n_new_min,
                        p->particle_mass};
    for (double x : v)
        if (!finite(x)) return HF_ERR_INVALID;
    if (!(p->box > 0.0) || !(p->b_kernel > 0.0) || !(p->l_fof > 0.0) || !(p->delta_l1 > 0.0) ||
        !(p->delta_l2 > 0.0) ||
        p->alpha_elig < 0.0 || p->c_roche < 0.0 || !(p->n_new_min > 0.0) || n < 0)
        return HF_ERR_INVALID;
    double box = p->box;
    double nbar = p->mean_density > 0.0 ? p->mean_density : (double)n / ((box * box) * box);
    if (!(nbar > 0.0)) return HF_ERR_INVALID;
    double lmean = cbrt(1.0 / nbar);
    double b = p->b_kernel * lmean;
    double l = p->l_fof * lmean;
    double K = ((4.0 * HF_PI) / 3.0) * p->delta_l1 * nbar;
    double rnew = cbrt(p->n_new_min / K);
    double a3 = (p->alpha_elig * p->alpha_elig) * p->alpha_elig;
    d[D_NBAR] = nbar;
    d[D_B] = b;
    d[D_L] = l;
    d[D_B2] = b * b;
    d[D_L2] = l * l;
    d[D_NORM] = 15.0 / (((8.0 * HF_PI) * ((b * b) * b)) * nbar);
    d[D_K] = K;
    d[D_K2] = K * K;
    d[D_FLOOR] = ((5.0 * p->delta_l1) / 3.0) * (rnew * rnew) / (b * b);
    d[D_A6] = a3 * a3;
    d[D_C3] = (p->c_roche * p->c_roche) * p->c_roche;
    return HF_OK;
}

hf_status make_geo(Lane *c, const hf_params *p, int64_t n, Geo *g) {
    double d[D_COUNT];
    if (derive(p, n, d) != HF_OK) return fail(c, HF_ERR_INVALID, "invalid parameters");
    if (n >= (int64_t)0x7fffffff) return fail(c, HF_ERR_INVALID, "n must be below 2^31 - 1");
    double L = p->box;
    double rmin = fmax(d[D_B], d[D_L]);
    double ncd = floor(L / (rmin * (1.0 + 1e-6)));
    if (!(ncd >= 3.0))
        return fail(c, HF_ERR_INVALID, "box must be at least three cells of max(b, l) wide");
    if (ncd > 1625.0) ncd = 1625.0;  // cell ids stay below 2^32; larger cells remain valid
    g->nc = (int)ncd;
    g->L = L;
    g->half = 0.5 * L;
    g->cell = L / g->nc;
    g->inv_cell = (double)g->nc / L;
    g->inv_nc = 1.0 / (double)g->nc;
    g->inv_b = 1.0 / d[D_B];
    g->inv_b2 = 1.0 / d[D_B2];
    g->cellb = (float)(g->cell / d[D_B]);
    // sub-cells: diagonal below l (with a 0.1% margin), at most 6 per side
    double kd = floor(g->cell * sqrt(3.0) / d[D_L] * (1.0 + 1e-3)) + 1.0;
    if (kd > 6.0)
        return fail(c, HF_ERR_INVALID, "l_fof must be at least 0.29 of the cell side (about 0.29 b)");
    g->ksub = (int)kd;
    g->nsub = g->ksub * g->ksub * g->ksub;
    g->inv_sub = g->ksub / g->cell;
    g->sub2 = (g->cell / g->ksub) * (g->cell / g->ksub);
    // two face-adjacent sub-cells of side s fit in a 2s x s x s box, whose
    // diagonal is s sqrt(6); the 2 % margin covers a particle binned a
    // coordinate ulp outside its sub-cell (the cell index comes from float
    // coordinates)
    g->face_sub_in_b = (g->cell / g->ksub) * sqrt(6.0) < 0.98 * d[D_B] ? 1 : 0;
    g->rsub = (int)ceil(d[D_L] * g->ksub / g->cell);
    if (g->rsub > g->ksub) g->rsub = g->ksub;
    // FP32 prefilter margin (units of b^2): 256 ulps of the largest local
    // coordinate difference, ten times the error bound of the FP32 path.
    double M = 2.0 * g->cellb + 1.0;
    double margin = 256.0 * M * ldexp(1.0, -24);
    double l2b = d[D_L2] / d[D_B2];
    g->l2b_lo = (float)(l2b - margin);
    g->l2b_hi = (float)(l2b + margin);
    g->b2b_lo = (float)(1.0 - margin);
    g->b2b_hi = (float)(1.0 + margin);
    g->b2 = d[D_B2];
    g->l2 = d[D_L2];
    g->norm = d[D_NORM];
    g->self_count = p->self_count ? 1 : 0;
    g->dl0 = p->delta_l0_min;
    g->floor_nuc = d[D_FLOOR];
    g->K = d[D_K];
    g->K2 = d[D_K2];
    g->A6 = d[D_A6];
    g->C3 = d[D_C3];
    // radial bins of the threshold-radius search (Sec. 2.3.4): steps of the
    // cell side / sqrt(3), wider when kRadBins bins would not reach the
    // farthest minimum image, sqrt(3) L/2
    g->rbin = fmax(g->cell / sqrt(3.0), 1.0001 * sqrt(3.0) * g->half / hf::kRadBins);
    g->n_l1_min = p->n_l1_min;
    g->particle_mass = (float)p->particle_mass;
    g->cell_base = 0;
    g->orig_base = 0;
    g->n = n;
    g->halos = nullptr;
    g->halo_cap = 0;
    return HF_OK;
}

// Scratch arena: every array of the pipeline carved from one allocation.
struct Carver {
    char *base;
    size_t off = 0;
    template <class T> T *take(int64_t count) {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += (size_t)(count > 0 ? count : 1) * sizeof(T);
        return p;
    }
};


// Entries of the particle -> box table of a call over nbox boxes: a power of
// two, at least 4 per box and 4096, at most 2^20 (1 when there is one box).
int64_t box_table_len(int nbox) {
    if (nbox <= 1) return 1;
    int64_t t = 4096;
    while (t < 4 * (int64_t)nbox && t < ((int64_t)1 << 20)) t <<= 1;
    return t;
}

size_t carve(char *base, int64_t n, int64_t ncell, int nsub, int64_t rhl, int nbox, bool extra, Work *w) {
    Carver c{base};
    int64_t n1 = n + 1;
    w->cnt = c.take<uint32_t>(ncell + 1);
    w->off = c.take<uint32_t>(ncell + 1);
    // one block: the output stage stores a 16-byte record per particle there
    w->rkey[0] = c.take<uint64_t>(2 * n);
    w->rkey[1] = w->rkey[0] ? w->rkey[0] + n : nullptr;
    w->rval[0] = c.take<uint32_t>(n);
    w->rval[1] = c.take<uint32_t>(n);
    w->rhist = c.take<uint32_t>(rhl);
    w->rscan = c.take<uint32_t>(rhl);
    w->ssub = c.take<uint16_t>(n);
    w->spos = c.take<float4>(n);
    w->sloc = c.take<float4>(n);
    w->pq = c.take<float4>(n + 32);
    w->f_chunk = c.take<uint32_t>(n1);
    w->s_chunk = c.take<uint32_t>(n1);
    w->f_dcell = c.take<uint32_t>(n1);
    w->s_dcell = c.take<uint32_t>(n1);
    w->f_sparse = c.take<uint32_t>(n1);
    w->s_sparse = c.take<uint32_t>(n1);
    w->chunks = c.take<int32_t>(n1);
    w->sparse = c.take<int32_t>(n1);
    w->dcells = c.take<uint32_t>(n1);
    w->hardlist = c.take<int32_t>(n1);
    w->subtab = c.take<uint32_t>((n / hf::kDenseMin + 1) * (nsub + 1));
    w->submax = c.take<uint64_t>((n / hf::kDenseMin + 1) * (nsub + 1));
    w->subarg = c.take<int32_t>((n / hf::kDenseMin + 1) * (nsub + 1));
    w->dens_s = c.take<float>(n);
    w->parent = c.take<int32_t>(n);
    w->minorig = c.take<int32_t>(n);
    w->gkey = c.take<int32_t>(n);
    w->gid_of = c.take<int32_t>(n);
    w->owner = c.take<int32_t>(n);
    w->gcnt = c.take<uint32_t>(n1);
    w->goff = c.take<uint32_t>(n1);
    w->gidx = c.take<uint32_t>(n1);
    w->mem = c.take<int32_t>(n);
    w->g_start = c.take<int32_t>(n1);
    w->g_size = c.take<int32_t>(n1);
    w->g_label = c.take<int32_t>(n1);
    w->gccnt = c.take<uint32_t>(n1);
    w->gcoff = c.take<uint32_t>(n1);
    w->gcfill = c.take<uint32_t>(n1);
    w->gcidx = c.take<uint32_t>(n1);
    w->glist = c.take<int32_t>(n1);
    w->cand = c.take<int32_t>(n1);
    w->cand_sorted = c.take<int32_t>(n1);
    w->h_nuc = c.take<int32_t>(n1);
    w->h_ienc = c.take<int32_t>(n1);
    w->h_gid = c.take<int32_t>(n1);
    w->g_nh = c.take<int32_t>(n1);
    w->h_count = c.take<uint32_t>(n1);
    w->tflag = c.take<uint32_t>(n1);
    w->tpos = c.take<uint32_t>(n1);
    w->hist = c.take<uint32_t>(2 * n1);
    int64_t scan_len = ncell > n ? ncell : n;
    if (rhl > scan_len) scan_len = rhl;
    w->scan_tmp = c.take<uint32_t>(hf::scan_tmp_words(scan_len + 1));
    w->counters = c.take<int32_t>(16);
    w->err = c.take<int32_t>(4);
    w->geo = c.take<Geo>(nbox);
    w->geo2 = extra ? c.take<Geo>(nbox) : nullptr;
    w->base = c.take<uint32_t>(nbox + 1);
    w->btab = c.take<int32_t>(box_table_len(nbox));
    w->box_rows = c.take<int64_t>(nbox);
    w->gcom = extra ? c.take<double>(6 * n1) : nullptr;
    w->ordk = extra ? c.take<int32_t>(n1) : nullptr;
    return c.off + 256;
}

// The boxes of one call: their constants, particle ranges and cell ranges.
struct Plan {
    int nbox = 0;
    int first = 0;       // the caller's number of box 0
    bool named = false;  // error texts name the box
    int64_t n = 0;       // particles of all boxes
    int64_t ncell = 0;   // cells of all boxes
    int nsub_max = 1;
    std::vector<Geo> geo;
    std::vector<uint32_t> base;
    std::vector<int32_t> btab;  // particle -> box table (more than one box)
    int bshift = 0;
};

std::string box_prefix(const Plan *pl, int b) {
    return pl && (pl->named || pl->nbox > 1) ? "box " + std::to_string(pl->first + b) + ": " : std::string();
}

// Checks the boxes' arguments and derives their constants.  An empty box
// only has its parameters checked (with a mean density of 1 when none is
// given) and takes no cells.
hf_status plan_boxes(Lane *c, const hf::BoxSet &bs, Plan *pl) {
    if (bs.nbox < 0) return fail(c, HF_ERR_INVALID, "n_boxes is negative");
    if (bs.nbox > 0 && (!bs.offsets || !bs.params)) return fail(c, HF_ERR_INVALID, "box offsets / params is NULL");
    pl->nbox = bs.nbox;
    pl->first = bs.first;
    pl->named = bs.named;
    pl->geo.assign(bs.nbox, Geo{});
    pl->base.assign(bs.nbox + 1, 0u);
    if (bs.nbox == 0) return HF_OK;
    if (bs.offsets[0] != 0) return fail(c, HF_ERR_INVALID, "box offsets must start at 0");
    if (bs.halo_offsets && bs.halo_offsets[0] != 0) return fail(c, HF_ERR_INVALID, "halo offsets must start at 0");
    for (int b = 0; b < bs.nbox; b++) {
        const int64_t nb = bs.offsets[b + 1] - bs.offsets[b];
        if (nb < 0) return fail(c, HF_ERR_INVALID, box_prefix(pl, b) + "n is negative (offsets decrease)");
        if (bs.halo_offsets && bs.halo_offsets[b + 1] < bs.halo_offsets[b])
            return fail(c, HF_ERR_INVALID, "halo offsets must not decrease");
    }
    if (bs.offsets[bs.nbox] >= (int64_t)0x7fffffff) return fail(c, HF_ERR_INVALID, "n must be below 2^31 - 1");
    for (int b = 0; b < bs.nbox; b++) {
        const int64_t o = bs.offsets[b], nb = bs.offsets[b + 1] - o;
        Geo &g = pl->geo[b];
        if (nb == 0) {
            double d[D_COUNT];
            hf_params q = bs.params[b];
            if (!(q.mean_density > 0.0)) q.mean_density = 1.0;
            if (derive(&q, 1, d) != HF_OK) return fail(c, HF_ERR_INVALID, box_prefix(pl, b) + "invalid parameters");
            g.nsub = 1;
        } else {
            const hf_status st = make_geo(c, &bs.params[b], nb, &g);
            if (st != HF_OK) {
                c->err = box_prefix(pl, b) + c->err;
                return st;
            }
            g.cell_base = (uint32_t)pl->ncell;
            pl->ncell += (int64_t)g.nc * g.nc * g.nc;
            if (pl->ncell >= (int64_t)0xffffffff)
                return fail(c, HF_ERR_INVALID, "the boxes of one call hold more than 2^32 - 1 cells");
            if (g.nsub > pl->nsub_max) pl->nsub_max = g.nsub;
        }
        g.orig_base = (uint32_t)o;
        g.n = nb;
        if (bs.halos && bs.halo_offsets) {
            g.halos = bs.halos + bs.halo_offsets[b];
            g.halo_cap = bs.halo_offsets[b + 1] - bs.halo_offsets[b];
        }
        pl->base[b] = (uint32_t)o;
    }
    pl->n = bs.offsets[bs.nbox];
    pl->base[bs.nbox] = (uint32_t)pl->n;
    if (pl->nbox > 1) {
        // bucket k covers particles [k << shift, (k + 1) << shift); its entry
        // is the box of its first particle (the last box for buckets past n)
        const int64_t t = box_table_len(pl->nbox);
        int sh = 0;
        while ((t << sh) < pl->n) sh++;
        pl->bshift = sh;
        pl->btab.assign(t, 0);
        int b = 0;
        for (int64_t k = 0; k < t; k++) {
            const int64_t first = k << sh;
            while (b + 1 < pl->nbox && (int64_t)pl->base[b + 1] <= first) b++;
            pl->btab[k] = b;
        }
    }
    // cells with nothing to bin still end the offset grid: at least one
    if (pl->ncell == 0) pl->ncell = 1;
    return HF_OK;
}

size_t plan_arena_bytes(const Plan &pl, bool extra) {
    Work w;
    return carve(nullptr, pl.n, pl.ncell, pl.nsub_max, hf::radix_hist_len(pl.n), pl.nbox, extra, &w);
}

// Pinned staging of at least `bytes` (grown unless nothing may be allocated).
hf_status ensure_stage(Lane *c, size_t bytes, bool may_grow) {
    if (bytes <= c->stage_bytes) return HF_OK;
    if (!may_grow) return fail(c, HF_ERR_INVALID, "too many boxes for the staging of an allocation-free call");
    if (c->stage) (void)hipHostFree(c->stage);
    c->stage = nullptr;
    c->stage_bytes = 0;
    const size_t want = bytes + bytes / 2;
    if (hipHostMalloc(&c->stage, want, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        c->stage = nullptr;
        return fail(c, HF_ERR_NOMEM, "hipHostMalloc of the box tables failed");
    }
    c->stage_bytes = want;
    return HF_OK;
}

hf_status prepare(Lane *c, const Plan &pl, Work *w, bool extra, const hf::FixedArena *fx) {
    const int64_t rhl = hf::radix_hist_len(pl.n);
    size_t need = carve(nullptr, pl.n, pl.ncell, pl.nsub_max, rhl, pl.nbox, extra, w);
    HIP_OK(c, hipSetDevice(c->device));
    if (fx) {
        // a caller-given region: nothing is allocated
        if (need > fx->bytes)
            return fail(c, HF_ERR_INVALID,
                        "this box needs " + std::to_string(need) + " bytes of scratch, more than the " +
                            std::to_string(fx->bytes) + " of the static scratch");
        carve((char *)fx->base, pl.n, pl.ncell, pl.nsub_max, rhl, pl.nbox, extra, w);
    } else {
        if (need > c->arena_bytes) {
            if (c->arena) {
                // every call ends synchronized with its stream, so the old arena is idle
                HIP_OK(c, hipFree(c->arena));
                if (c->budget) c->budget->give(c->arena_bytes);
                c->arena = nullptr;
                c->arena_bytes = 0;
            }
            size_t want = need + need / 8;
            if (c->budget && !c->budget->take(want)) {
                want = need;  // no headroom for the next, larger call
                if (!c->budget->take(want))
                    return fail(c, HF_ERR_NOMEM,
                                "the scratch arena of " + std::to_string(need) +
                                    " bytes exceeds the context's HBM budget (" +
                                    std::to_string(c->budget->held.load()) + " of " +
                                    std::to_string(c->budget->limit) + " bytes held)");
            }
            if (hipMalloc(&c->arena, want) != hipSuccess) {
                (void)hipGetLastError();
                c->arena = nullptr;
                if (c->budget) c->budget->give(want);
                return fail(c, HF_ERR_NOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed");
            }
            c->arena_bytes = want;
        }
        carve((char *)c->arena, pl.n, pl.ncell, pl.nsub_max, rhl, pl.nbox, extra, w);
    }
    w->host = c->host;
    w->ncu = c->ncu;
    w->radius_bins = c->radius_bins;
    c->stats = hf_stats{};
    c->stats.n_cells = pl.ncell;
    // the box tables go up and the per-box rows come back through it
    return ensure_stage(c, pl.nbox * (2 * sizeof(Geo) + sizeof(uint32_t) + sizeof(int64_t)) +
                               pl.btab.size() * sizeof(int32_t) + 4096,
                        fx == nullptr);
}

// Device words read back in one dispatch and one wait (the lane's pinned host
// words); out[i] = *src[i].
hf_status read_dev(Lane *c, hipStream_t s, std::initializer_list<const void *> src, uint32_t *out) {
    hf::WordSrc w{};
    int k = 0;
    for (const void *p : src) w.p[k++] = static_cast<const uint32_t *>(p);
    HIP_OK(c, hf::read_words(w, k, c->host, out, s));
    return HF_OK;
}

// The error bits raised by the kernels (box: the smallest box that raised
// one, named when the call has several boxes).
hf_status err_status(Lane *c, uint32_t err, uint32_t box, const Plan *pl) {
    const std::string pre = box_prefix(pl, (int)box);
    if (err & 1) return fail(c, HF_ERR_INVALID, pre + "positions must lie in [0, box)");
    if (err & 2) return fail(c, HF_ERR_INVALID, pre + "l0_id values must lie in [0, n]");
    if (err & 16) return fail(c, HF_ERR_INVALID, pre + "densities must be non-negative numbers");
    if (err & 8)
        return fail(c, HF_ERR_INVALID,
                    pre + "an L0 group spans half the periodic box or more along an axis (minimum-image "
                          "distances would be ambiguous)");
    if (err & 4) return fail(c, HF_ERR_DEVICE, pre + "internal error: L0 group key out of range");
    return HF_OK;
}

hf_status check_pos_flags(Lane *c, const Work &w, const Plan *pl, hipStream_t s) {
    uint32_t e[2] = {0, 0};
    hf_status st = read_dev(c, s, {w.err, w.err + 1}, e);
    return st != HF_OK ? st : err_status(c, e[0], e[1], pl);
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0f;
    }
    return ms;
}

// CompaSO on the binned particles with group keys in w.gkey.  Fills halo_id,
// l0_out and dens_out (either may be null; the densities from w.dens_s), every
// box's table and its row count (n_halos, host,
// nbox entries); records events ev[3..8].  CAPACITY when a table did not fit.
// Optional output of a one-box pass: its members in group order (Sec. 2.3.5).
struct GroupOut {
    int32_t *members = nullptr;     // device [n]
    int64_t *halo_start = nullptr;  // device [halo rows + 1]
};

hf_status run_compaso(Lane *c, const Plan &pl, const hf::Boxes &bx, Work &w, int32_t *halo_id,
                      int32_t *l0_out, float *dens_out, int64_t *n_halos, hipStream_t s,
                      const GroupOut &go = GroupOut{}) {
    const int64_t n = pl.n;
    HIP_OK(c, hipEventRecord(c->ev[3], s));
    hf::launch_segment(n, w, s);
    // group and member counts, and the error flags of the steps so far (the
    // kernels before this point clamp what they index, whatever the flags)
    uint32_t r[4];
    hf_status st = read_dev(c, s, {w.gidx + n, w.goff + n, w.err, w.err + 1}, r);
    if (st == HF_OK) st = err_status(c, r[2], r[3], &pl);
    if (st != HF_OK) return st;
    int64_t G = r[0];
    c->stats.n_groups = G;
    c->stats.n_members = r[1];
    hf::launch_segment_groups(n, G, w, s);
    hf::launch_extent(G, c->stats.n_members, bx, w, s);
    HIP_OK(c, hipEventRecord(c->ev[4], s));
    hf::launch_candidates(n, bx, w, s);
    hf::scan_u32(w.gccnt, w.gcoff, G, w.scan_tmp, s);
    uint32_t NC32 = 0;
    st = read_dev(c, s, {w.gcoff + G}, &NC32);
    if (st != HF_OK) return st;
    int64_t NC = NC32;
    hf::launch_candidates_sort(n, G, NC, w, s);
    HIP_OK(c, hipEventRecord(c->ev[5], s));
    hf::launch_accept(n, G, NC, c->stats.n_members, bx, w, s);
    HIP_OK(c, hipEventRecord(c->ev[6], s));
    hf::launch_assign(n, bx, w, s);
    HIP_OK(c, hipEventRecord(c->ev[7], s));
    hf::launch_output_flags(n, NC, bx, w, s);
    hf::launch_output(n, NC, bx, w, halo_id, l0_out, dens_out, w.box_rows, s);
    HIP_OK(c, hipEventRecord(c->ev[8], s));
    // every box's rows, the nuclei accepted (counter 2) and the error flags
    int64_t *rows = reinterpret_cast<int64_t *>(c->stage);
    HIP_OK(c, hipMemcpyAsync(rows, w.box_rows, sizeof(int64_t) * pl.nbox, hipMemcpyDeviceToHost, s));
    uint32_t r2[3];
    st = read_dev(c, s, {w.counters + 2, w.err, w.err + 1}, r2);
    if (st == HF_OK) st = err_status(c, r2[1], r2[2], &pl);
    if (st != HF_OK) return st;
    c->stats.ms_segment = elapsed(c->ev[3], c->ev[4]);
    c->stats.ms_candidates = elapsed(c->ev[4], c->ev[5]);
    c->stats.ms_accept = elapsed(c->ev[5], c->ev[6]);
    c->stats.ms_assign = elapsed(c->ev[6], c->ev[7]);
    c->stats.ms_output = elapsed(c->ev[7], c->ev[8]);
    c->stats.n_candidates = NC;
    c->stats.n_dense_cells = w.ndcells;
    c->stats.n_dense_chunks = w.nchunks;
    c->stats.n_sparse = w.nsparse;
    c->stats.n_hard = w.nhard;
    c->stats.n_found = r2[0];
    int over = -1;
    int64_t total = 0;
    for (int b = 0; b < pl.nbox; b++) {
        if (n_halos) n_halos[b] = rows[b];
        total += rows[b];
        if (over < 0 && rows[b] > pl.geo[b].halo_cap) over = b;
    }
    c->stats.n_halos = total;
    if (over >= 0)
        return fail(c, HF_ERR_CAPACITY,
                    box_prefix(&pl, over) + "halos_cap is smaller than the number of halos");
    if (go.members) {
        // the rows are known and fit: members by table row (the call ends
        // synchronized with its stream, as every call does)
        hf::launch_group_order(n, total, halo_id, w, go.members, go.halo_start, s);
        HIP_OK(c, hipEventRecord(c->ev[8], s));
        HIP_OK(c, hipStreamSynchronize(s));
        c->stats.ms_output = elapsed(c->ev[7], c->ev[8]);
    }
    return HF_OK;
}

// Uploads the box tables, bins all particles and reads the work counts.
// dens: the call computes densities (binning also writes the records the
// density kernel reads); extra: halo statistics buffers.  bx receives the
// device view of the boxes.
hf_status begin(Lane *c, const Plan &pl, const float *pos, hf::Boxes *bx, Work *w, hipStream_t s, bool dens,
                bool extra = false, const hf::FixedArena *fx = nullptr) {
    if (pl.n > 0 && !pos) return fail(c, HF_ERR_INVALID, "pos is NULL");
    hf_status st = prepare(c, pl, w, extra, fx);
    if (st != HF_OK) return st;
    if (!dens) w->pq = nullptr;
    // the tables through pinned staging (the lane's previous call has ended)
    char *stg = reinterpret_cast<char *>(c->stage);
    memcpy(stg, pl.geo.data(), sizeof(Geo) * pl.nbox);
    memcpy(stg + sizeof(Geo) * pl.nbox, pl.base.data(), sizeof(uint32_t) * (pl.nbox + 1));
    HIP_OK(c, hipMemcpyAsync(w->geo, stg, sizeof(Geo) * pl.nbox, hipMemcpyHostToDevice, s));
    HIP_OK(c, hipMemcpyAsync(w->base, stg + sizeof(Geo) * pl.nbox, sizeof(uint32_t) * (pl.nbox + 1),
                             hipMemcpyHostToDevice, s));
    if (!pl.btab.empty()) {
        char *tb = stg + sizeof(Geo) * pl.nbox + sizeof(uint32_t) * (pl.nbox + 1);
        memcpy(tb, pl.btab.data(), sizeof(int32_t) * pl.btab.size());
        HIP_OK(c, hipMemcpyAsync(w->btab, tb, sizeof(int32_t) * pl.btab.size(), hipMemcpyHostToDevice, s));
    }
    *bx = hf::Boxes{w->geo, w->base, pl.nbox, pl.nsub_max, w->btab, pl.bshift};
    hf::fill_i32(w->counters, 0, 16, s);
    hf::fill_i32(w->err, 0, 1, s);
    hf::fill_i32(w->err + 1, 0x7fffffff, 1, s);
    const int64_t n = pl.n;
    HIP_OK(c, hipEventRecord(c->ev[0], s));
    hf::launch_bin(pos, n, pl.ncell, *bx, *w, s);
    // dense chunks, dense cells, sparse particles, and the range flag of the
    // positions (binning clamps cells, so nothing it wrote is out of bounds).
    // The sub-cell tables take their cell count on the device and are
    // enqueued before the host waits for these words, so the device keeps
    // working while the host reads them and enqueues the next stage.
    hf::WordSrc src{};
    src.p[0] = w->s_chunk + n;
    src.p[1] = w->s_dcell + n;
    src.p[2] = w->s_sparse + n;
    src.p[3] = reinterpret_cast<const uint32_t *>(w->err);
    src.p[4] = reinterpret_cast<const uint32_t *>(w->err + 1);
    HIP_OK(c, hf::publish_words(src, 5, c->host, s));
    HIP_OK(c, hipEventRecord(c->pub, s));
    hf::launch_subtab(n, w->s_dcell + n, *bx, *w, s);
    HIP_OK(c, hipEventSynchronize(c->pub));
    uint32_t counts[5];
    hf::collect_words(c->host, 5, counts);
    st = err_status(c, counts[3], counts[4], &pl);
    if (st != HF_OK) {
        // the sub-cell tables may still run on s: a failed call also ends
        // synchronized with its stream, so the arena is idle when it returns
        HIP_OK(c, hipStreamSynchronize(s));
        return st;
    }
    w->nchunks = counts[0];
    w->ndcells = counts[1];
    w->nsparse = counts[2];
    w->nhard = 0;
    HIP_OK(c, hipEventRecord(c->ev[1], s));
    return HF_OK;
}

// A single box as a set of one.
struct OneBox {
    int64_t offs[2];
    int64_t hoffs[2];
    hf::BoxSet set(const hf_params *p, hf_halo *halos) const {
        return hf::BoxSet{1, offs, p, halos, hoffs};
    }
};

OneBox one_box(int64_t n, int64_t cap) { return OneBox{{0, n}, {0, cap > 0 ? cap : 0}}; }

hf_status find_boxes(Lane *c, const hf::BoxSet &bs, const float *pos, float *density, int32_t *l0_id,
                     int32_t *halo_id, int64_t *n_halos, hipStream_t s, const hf::FixedArena *fx,
                     const GroupOut &go = GroupOut{}) {
    if (!c) return HF_ERR_INVALID;
    c->err.clear();
    Plan pl;
    hf_status st = plan_boxes(c, bs, &pl);
    if (st != HF_OK) return st;
    if (n_halos)
        for (int b = 0; b < pl.nbox; b++) n_halos[b] = 0;
    if (go.members && pl.nbox != 1) return fail(c, HF_ERR_INVALID, "group order is for one box");
    if (pl.n == 0) {
        if (go.halo_start) {
            // no halos and no members: halo_start[0] = 0
            hf::fill_i32(reinterpret_cast<int32_t *>(go.halo_start), 0, 2, s);
            HIP_OK(c, hipStreamSynchronize(s));
        }
        return HF_OK;
    }
    if (!halo_id) return fail(c, HF_ERR_INVALID, "halo_id is NULL");
    hf::Boxes bx;
    Work w;
    st = begin(c, pl, pos, &bx, &w, s, true, false, fx);
    if (st != HF_OK) return st;
    // with the L0 labels asked for, the three outputs leave together in the
    // output stage (one scattered record per particle costs less than three
    // scattered words); else the density kernels store the densities and the
    // output stage only the halo labels (two words cost less than a record)
    float *dens_late = l0_id ? density : nullptr;
    hf::launch_density(pl.n, bx, w, l0_id ? nullptr : density, s);
    HIP_OK(c, hipEventRecord(c->ev[2], s));
    hf::launch_fof(pl.n, bx, w, s);
    hf::launch_fof_labels(pl.n, bx, w, nullptr, s);
    HIP_OK(c, hipEventRecord(c->ev[9], s));
    st = run_compaso(c, pl, bx, w, halo_id, l0_id, dens_late, n_halos, s, go);
    c->stats.ms_bin = elapsed(c->ev[0], c->ev[1]);
    c->stats.ms_density = elapsed(c->ev[1], c->ev[2]);
    c->stats.ms_fof = elapsed(c->ev[2], c->ev[9]);
    c->stats.ms_total = elapsed(c->ev[0], c->ev[8]);
    return st;
}

}  // namespace

namespace hf {

hf_status lane_init(Lane *L, int device, bool own_stream) {
    L->device = device;
    if (hipSetDevice(device) != hipSuccess) return HF_ERR_DEVICE;
    if (hipDeviceGetAttribute(&L->ncu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        L->ncu <= 0)
        return HF_ERR_DEVICE;
    if (hipHostMalloc(reinterpret_cast<void **>(&L->host), 64 * sizeof(uint32_t), hipHostMallocCoherent) !=
        hipSuccess) {
        L->host = nullptr;
        return HF_ERR_DEVICE;
    }
    // room for the tables of a few hundred boxes; larger calls grow it
    if (hipHostMalloc(&L->stage, 64 << 10, hipHostMallocDefault) != hipSuccess) {
        L->stage = nullptr;
        return HF_ERR_DEVICE;
    }
    L->stage_bytes = 64 << 10;
    for (auto &e : L->ev)
        if (hipEventCreate(&e) != hipSuccess) return HF_ERR_DEVICE;
    if (hipEventCreateWithFlags(&L->pub, hipEventDisableTiming) != hipSuccess) return HF_ERR_DEVICE;
    if (own_stream && hipStreamCreateWithFlags(&L->stream, hipStreamNonBlocking) != hipSuccess)
        return HF_ERR_DEVICE;
    return HF_OK;
}

void lane_release(Lane *L) {
    if (L->arena) {
        (void)hipSetDevice(L->device);
        (void)hipFree(L->arena);
        if (L->budget) L->budget->give(L->arena_bytes);
    }
    L->arena = nullptr;
    L->arena_bytes = 0;
}

void lane_destroy(Lane *L) {
    lane_release(L);
    if (L->host) (void)hipHostFree(L->host);
    L->host = nullptr;
    if (L->stage) (void)hipHostFree(L->stage);
    L->stage = nullptr;
    L->stage_bytes = 0;
    for (auto &e : L->ev)
        if (e) (void)hipEventDestroy(e);
    if (L->pub) (void)hipEventDestroy(L->pub);
    L->pub = nullptr;
    if (L->stream) (void)hipStreamDestroy(L->stream);
    L->stream = nullptr;
}

size_t boxes_arena_bytes(const BoxSet &bs, int64_t *n_total, int64_t *ncell_total) {
    Lane tmp;
    Plan pl;
    if (plan_boxes(&tmp, bs, &pl) != HF_OK) return 0;
    if (n_total) *n_total = pl.n;
    if (ncell_total) *ncell_total = pl.ncell;
    const size_t need = plan_arena_bytes(pl, false);
    return need + need / 8;
}

size_t lane_arena_bytes(const hf_params *p, int64_t n) {
    if (n <= 0) return 0;
    const OneBox ob = one_box(n, 0);
    return boxes_arena_bytes(ob.set(p, nullptr), nullptr, nullptr);
}

hf_status lane_find(Lane *c, const float *pos, int64_t n, const hf_params *p, float *density,
                    int32_t *l0_id, int32_t *halo_id, hf_halo *halos, int64_t halos_cap,
                    int64_t *n_halos, hipStream_t s, const FixedArena *fx) {
    if (!c) return HF_ERR_INVALID;
    if (halos_cap < 0 || (halos_cap > 0 && !halos)) return fail(c, HF_ERR_INVALID, "bad halos / halos_cap");
    if (n < 0) return fail(c, HF_ERR_INVALID, "n is negative");
    const OneBox ob = one_box(n, halos_cap);
    int64_t nh = 0;
    const hf_status st = find_boxes(c, ob.set(p, halos), pos, density, l0_id, halo_id, &nh, s, fx);
    if (n_halos) *n_halos = nh;
    return st;
}

hf_status lane_find_boxes(Lane *L, const BoxSet &bs, const float *pos, float *density, int32_t *l0_id,
                          int32_t *halo_id, int64_t *n_halos, hipStream_t s) {
    return find_boxes(L, bs, pos, density, l0_id, halo_id, n_halos, s, nullptr);
}

}  // namespace hf

extern "C" {

void hf_default_params(hf_params *p) {
    if (!p) return;
    p->box = 1.0;
    p->mean_density = 0.0;
    p->b_kernel = 0.4;
    p->l_fof = 0.25;
    p->delta_l0_min = 60.0;
    p->delta_l1 = 200.0;
    p->delta_l2 = 800.0;
    p->alpha_elig = 0.8;
    p->c_roche = 2.0;
    p->n_new_min = 35.0;
    p->particle_mass = 1.0;
    p->n_l1_min = 35;
    p->self_count = 0;
}

hf_status hf_params_at_redshift(const hf_params *in, double omega_m0, double z, hf_params *out) {
    if (!in || !out || !(omega_m0 > 0.0 && omega_m0 <= 1.0) || !(z > -1.0)) return HF_ERR_INVALID;
    // flat matter + Lambda: Omega_m(z) = Om (1+z)^3 / (Om (1+z)^3 + 1 - Om)
    const double a = 1.0 + z;
    const double mz = omega_m0 * ((a * a) * a);
    const double omz = mz / (mz + (1.0 - omega_m0));
    const double x = omz - 1.0;
    const double c = 18.0 * HF_PI * HF_PI;
    // fitting function relative to the critical density, then to the mean
    const double factor = (c + 82.0 * x - 39.0 * (x * x)) / (c * omz);
    hf_params p = *in;
    p.delta_l1 = in->delta_l1 * factor;
    p.delta_l2 = in->delta_l2 * factor;
    p.delta_l0_min = in->delta_l0_min * factor;
    p.l_fof = in->l_fof / cbrt(factor);
    *out = p;
    return HF_OK;
}

hf_status hf_derived(const hf_params *p, int64_t n, double *out) {
    if (!out) return HF_ERR_INVALID;
    return derive(p, n, out);
}

hf_status hf_create(hf_ctx **out, int device, uint64_t hbm_budget_bytes) {
    if (!out) return HF_ERR_INVALID;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return HF_ERR_UNSUPPORTED;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return HF_ERR_DEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return HF_ERR_UNSUPPORTED;
    hf_ctx *c = new hf_ctx();
    c->budget.limit = hbm_budget_bytes;
    c->main.budget = &c->budget;
    if (hf::lane_init(&c->main, device, false) != HF_OK) {
        hf::lane_destroy(&c->main);
        delete c;
        return HF_ERR_DEVICE;
    }
    // lane_init made `device` current
    c->scratch = scratch_of(device);
    if (!c->scratch) {
        hf::lane_destroy(&c->main);
        delete c;
        return HF_ERR_DEVICE;
    }
    *out = c;
    return HF_OK;
}

void hf_destroy(hf_ctx *c) {
    if (!c) return;
    for (auto &L : c->pool) hf::lane_destroy(L.get());
    hf::lane_destroy(&c->main);
    delete c;
}

const char *hf_last_error(const hf_ctx *c) { return c ? c->main.err.c_str() : "no context"; }

hf_status hf_get_stats(const hf_ctx *c, hf_stats *out) {
    if (!c || !out) return HF_ERR_INVALID;
    *out = c->main.stats;
    return HF_OK;
}

hf_status hf_set_option(hf_ctx *ctx, int32_t option, int64_t value) {
    if (!ctx) return HF_ERR_INVALID;
    if (option != HF_OPT_RADIUS_SEARCH) return fail(&ctx->main, HF_ERR_INVALID, "unknown option");
    if (value != HF_RADIUS_HISTOGRAM && value != HF_RADIUS_BINS)
        return fail(&ctx->main, HF_ERR_INVALID, "HF_OPT_RADIUS_SEARCH takes HF_RADIUS_HISTOGRAM or HF_RADIUS_BINS");
    ctx->radius_bins = value == HF_RADIUS_BINS;
    ctx->main.radius_bins = ctx->radius_bins;
    for (auto &L : ctx->pool) L->radius_bins = ctx->radius_bins;
    return HF_OK;
}

hf_status hf_get_option(const hf_ctx *ctx, int32_t option, int64_t *value) {
    if (!ctx || !value || option != HF_OPT_RADIUS_SEARCH) return HF_ERR_INVALID;
    *value = ctx->radius_bins ? HF_RADIUS_BINS : HF_RADIUS_HISTOGRAM;
    return HF_OK;
}

hf_status hf_density(hf_ctx *ctx, const float *pos, int64_t n, const hf_params *p, float *density,
                     void *stream) {
    Lane *c = ctx ? &ctx->main : nullptr;
    if (!c) return HF_ERR_INVALID;
    c->err.clear();
    hipStream_t s = (hipStream_t)stream;
    if (n < 0) return fail(c, HF_ERR_INVALID, "n is negative");
    const OneBox ob = one_box(n, 0);
    Plan pl;
    hf_status st = plan_boxes(c, ob.set(p, nullptr), &pl);
    if (st != HF_OK || n == 0) return st;
    if (!density) return fail(c, HF_ERR_INVALID, "density is NULL");
    hf::Boxes bx;
    Work w;
    st = begin(c, pl, pos, &bx, &w, s, true);
    if (st != HF_OK) return st;
    hf::launch_density(n, bx, w, density, s);
    HIP_OK(c, hipEventRecord(c->ev[2], s));
    st = check_pos_flags(c, w, &pl, s);
    c->stats.ms_bin = elapsed(c->ev[0], c->ev[1]);
    c->stats.ms_density = elapsed(c->ev[1], c->ev[2]);
    c->stats.ms_total = elapsed(c->ev[0], c->ev[2]);
    return st;
}

hf_status hf_count_pairs(hf_ctx *ctx, const float *pos, int64_t n, const hf_params *p,
                         int64_t *pairs, void *stream) {
    Lane *c = ctx ? &ctx->main : nullptr;
    if (!c) return HF_ERR_INVALID;
    c->err.clear();
    hipStream_t s = (hipStream_t)stream;
    if (!pairs) return fail(c, HF_ERR_INVALID, "pairs is NULL");
    *pairs = 0;
    if (n < 0) return fail(c, HF_ERR_INVALID, "n is negative");
    const OneBox ob = one_box(n, 0);
    Plan pl;
    hf_status st = plan_boxes(c, ob.set(p, nullptr), &pl);
    if (st != HF_OK || n == 0) return st;
    hf::Boxes bx;
    Work w;
    st = begin(c, pl, pos, &bx, &w, s, false);
    if (st != HF_OK) return st;
    hf::fill_i32(w.counters + 4, 0, 2, s);
    hf::launch_count_pairs(n, bx, w, (unsigned long long *)(w.counters + 4), s);
    HIP_OK(c, hipMemcpyAsync(pairs, w.counters + 4, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    return check_pos_flags(c, w, &pl, s);
}

hf_status hf_l0_fof(hf_ctx *ctx, const float *pos, const float *density, int64_t n,
                    const hf_params *p, int32_t *l0_id, int64_t *n_groups, void *stream) {
    Lane *c = ctx ? &ctx->main : nullptr;
    if (!c) return HF_ERR_INVALID;
    c->err.clear();
    hipStream_t s = (hipStream_t)stream;
    if (n < 0) return fail(c, HF_ERR_INVALID, "n is negative");
    if (n > 0 && (!density || !l0_id)) return fail(c, HF_ERR_INVALID, "density / l0_id is NULL");
    const OneBox ob = one_box(n, 0);
    Plan pl;
    hf_status st = plan_boxes(c, ob.set(p, nullptr), &pl);
    if (st != HF_OK) return st;
    if (n == 0) {
        if (n_groups) *n_groups = 0;
        return HF_OK;
    }
    hf::Boxes bx;
    Work w;
    st = begin(c, pl, pos, &bx, &w, s, false);
    if (st != HF_OK) return st;
    hf::launch_gather_density(density, n, w, s);
    HIP_OK(c, hipEventRecord(c->ev[2], s));
    hf::launch_fof(n, bx, w, s);
    hf::launch_fof_labels(n, bx, w, l0_id, s);
    HIP_OK(c, hipEventRecord(c->ev[3], s));
    hf::launch_segment(n, w, s);
    uint32_t r[4] = {0, 0, 0, 0};
    st = read_dev(c, s, {w.gidx + n, w.goff + n, w.err, w.err + 1}, r);
    if (st == HF_OK) st = err_status(c, r[2], r[3], &pl);
    const uint32_t G32 = r[0], M32 = r[1];
    c->stats.ms_bin = elapsed(c->ev[0], c->ev[1]);
    c->stats.ms_fof = elapsed(c->ev[2], c->ev[3]);
    c->stats.ms_total = elapsed(c->ev[0], c->ev[3]);
    c->stats.n_members = M32;
    c->stats.n_groups = G32;
    if (n_groups) *n_groups = G32;
    return st;
}

hf_status hf_compaso(hf_ctx *ctx, const float *pos, const float *density, const int32_t *l0_id,
                     int64_t n, const hf_params *p, int32_t *halo_id, hf_halo *halos,
                     int64_t halos_cap, int64_t *n_halos, void *stream) {
    Lane *c = ctx ? &ctx->main : nullptr;
    if (!c) return HF_ERR_INVALID;
    c->err.clear();
    hipStream_t s = (hipStream_t)stream;
    if (n < 0) return fail(c, HF_ERR_INVALID, "n is negative");
    if (n > 0 && (!density || !l0_id || !halo_id))
        return fail(c, HF_ERR_INVALID, "density / l0_id / halo_id is NULL");
    if (halos_cap < 0 || (halos_cap > 0 && !halos)) return fail(c, HF_ERR_INVALID, "bad halos / halos_cap");
    const OneBox ob = one_box(n, halos_cap);
    Plan pl;
    hf_status st = plan_boxes(c, ob.set(p, halos), &pl);
    if (st != HF_OK) return st;
    if (n == 0) {
        if (n_halos) *n_halos = 0;
        return HF_OK;
    }
    hf::Boxes bx;
    Work w;
    st = begin(c, pl, pos, &bx, &w, s, false);
    if (st != HF_OK) return st;
    hf::launch_keys_from_labels(l0_id, density, n, bx, w, s);  // also gathers the densities
    HIP_OK(c, hipEventRecord(c->ev[2], s));
    int64_t nh = 0;
    st = run_compaso(c, pl, bx, w, halo_id, nullptr, nullptr, &nh, s);
    if (n_halos) *n_halos = nh;
    c->stats.ms_bin = elapsed(c->ev[0], c->ev[1]);
    c->stats.ms_total = elapsed(c->ev[0], c->ev[8]);
    return st;
}

hf_status hf_halo_stats(hf_ctx *ctx, const float *pos, const float *density, const int32_t *halo_id,
                        int64_t n, const hf_params *p, int64_t n_halos, hf_halo_summary *stats,
                        int32_t *group_start, int32_t *group_members, void *stream) {
    Lane *c = ctx ? &ctx->main : nullptr;
    if (!c) return HF_ERR_INVALID;
    c->err.clear();
    hipStream_t s = (hipStream_t)stream;
    if (n < 0) return fail(c, HF_ERR_INVALID, "n is negative");
    if (n > 0 && (!density || !halo_id)) return fail(c, HF_ERR_INVALID, "density / halo_id is NULL");
    if (n_halos < 0 || (n_halos > 0 && !stats)) return fail(c, HF_ERR_INVALID, "bad stats / n_halos");
    const OneBox ob = one_box(n, 0);
    Plan pl;
    hf_status st = plan_boxes(c, ob.set(p, nullptr), &pl);
    if (st != HF_OK) return st;
    if (n == 0) {
        if (n_halos != 0) return fail(c, HF_ERR_INVALID, "n_halos must be 0 for an empty input");
        return HF_OK;
    }
    // level 2: the same steps with delta_l2 in place of delta_l1 (the cells
    // depend on b and l only, so the geometry is the same)
    hf_params p2 = *p;
    p2.delta_l1 = p->delta_l2;
    Geo g2;
    st = make_geo(c, &p2, n, &g2);
    if (st != HF_OK) return st;
    hf::Boxes bx;
    Work w;
    st = begin(c, pl, pos, &bx, &w, s, false, true);
    if (st != HF_OK) return st;
    g2.cell_base = pl.geo[0].cell_base;
    g2.orig_base = 0;
    char *stg = reinterpret_cast<char *>(c->stage) + sizeof(Geo) * 2 + 256;
    memcpy(stg, &g2, sizeof(Geo));
    HIP_OK(c, hipMemcpyAsync(w.geo2, stg, sizeof(Geo), hipMemcpyHostToDevice, s));
    const hf::Boxes bx2{w.geo2, w.base, 1, pl.nsub_max, nullptr, 0};
    hf::launch_keys_from_labels(halo_id, density, n, bx, w, s);  // also gathers the densities
    HIP_OK(c, hipEventRecord(c->ev[2], s));
    HIP_OK(c, hipEventRecord(c->ev[3], s));
    hf::launch_segment(n, w, s);
    uint32_t r[4];
    st = read_dev(c, s, {w.gidx + n, w.goff + n, w.err, w.err + 1}, r);
    if (st == HF_OK) st = err_status(c, r[2], r[3], &pl);
    if (st != HF_OK) return st;
    const int64_t G = r[0], M = r[1];
    if (G != n_halos) return fail(c, HF_ERR_INVALID, "n_halos differs from the number of halo_id labels");
    c->stats.n_groups = G;
    c->stats.n_members = M;
    hf::launch_segment_groups(n, G, w, s);
    HIP_OK(c, hipEventRecord(c->ev[4], s));
    hf::launch_candidates(n, bx2, w, s);
    hf::scan_u32(w.gccnt, w.gcoff, G, w.scan_tmp, s);
    uint32_t NC32 = 0;
    st = read_dev(c, s, {w.gcoff + G}, &NC32);
    if (st != HF_OK) return st;
    hf::launch_candidates_sort(n, G, NC32, w, s);
    HIP_OK(c, hipEventRecord(c->ev[5], s));
    hf::launch_accept(n, G, NC32, M, bx2, w, s);
    HIP_OK(c, hipEventRecord(c->ev[6], s));
    hf::launch_assign(n, bx2, w, s);
    HIP_OK(c, hipEventRecord(c->ev[7], s));
    hf::launch_halo_stats(n, G, M, g2, p->particle_mass, pos, halo_id, w, stats, group_start, group_members, s);
    HIP_OK(c, hipEventRecord(c->ev[8], s));
    HIP_OK(c, hipStreamSynchronize(s));
    c->stats.n_candidates = NC32;
    c->stats.ms_bin = elapsed(c->ev[0], c->ev[1]);
    c->stats.ms_segment = elapsed(c->ev[3], c->ev[4]);
    c->stats.ms_candidates = elapsed(c->ev[4], c->ev[5]);
    c->stats.ms_accept = elapsed(c->ev[5], c->ev[6]);
    c->stats.ms_assign = elapsed(c->ev[6], c->ev[7]);
    c->stats.ms_output = elapsed(c->ev[7], c->ev[8]);
    c->stats.ms_total = elapsed(c->ev[0], c->ev[8]);
    return HF_OK;
}

hf_status hf_find(hf_ctx *ctx, const float *pos, int64_t n, const hf_params *p, float *density,
                  int32_t *l0_id, int32_t *halo_id, hf_halo *halos, int64_t halos_cap,
                  int64_t *n_halos, void *stream) {
    if (!ctx) return HF_ERR_INVALID;
    return hf::lane_find(&ctx->main, pos, n, p, density, l0_id, halo_id, halos, halos_cap, n_halos,
                         (hipStream_t)stream);
}

hf_status hf_find_grouped(hf_ctx *ctx, const float *pos, int64_t n, const hf_params *p, float *density,
                          int32_t *l0_id, int32_t *halo_id, hf_halo *halos, int64_t halos_cap,
                          int64_t *n_halos, int32_t *members, int64_t *halo_start, void *stream) {
    if (!ctx) return HF_ERR_INVALID;
    Lane *c = &ctx->main;
    c->err.clear();
    if (!members || !halo_start) return fail(c, HF_ERR_INVALID, "members / halo_start is NULL");
    if (halos_cap < 0 || (halos_cap > 0 && !halos)) return fail(c, HF_ERR_INVALID, "bad halos / halos_cap");
    if (n < 0) return fail(c, HF_ERR_INVALID, "n is negative");
    const OneBox ob = one_box(n, halos_cap);
    GroupOut go;
    go.members = members;
    go.halo_start = halo_start;
    int64_t nh = 0;
    const hf_status st = find_boxes(c, ob.set(p, halos), pos, density, l0_id, halo_id, &nh, (hipStream_t)stream,
                                    nullptr, go);
    if (n_halos) *n_halos = nh;
    return st;
}

hf_status hf_find_noalloc(hf_ctx *ctx, const float *pos, int64_t n, const hf_params *p, float *density,
                          int32_t *l0_id, int32_t *halo_id, hf_halo *halos, int64_t halos_cap,
                          int64_t *n_halos, void *stream) {
    if (!ctx) return HF_ERR_INVALID;
    const hf::FixedArena fx{ctx->scratch, hf::kScratchBytes};
    return hf::lane_find(&ctx->main, pos, n, p, density, l0_id, halo_id, halos, halos_cap, n_halos,
                         (hipStream_t)stream, &fx);
}

}  // extern "C"
