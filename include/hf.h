/*
 * hf.h -- C ABI of libhf, the MI355X (gfx950) CompaSO group-finding library.
 *
 * The library implements the on-the-fly group-finding pass of Hadzhiyska et al.,
 * "CompaSO: A new halo finder for competitive assignment to spherical
 * overdensities" (Sec. 2.2 and 2.3 of the paper):
 *
 *   1. kernel density of every particle, W(r) = 1 - r^2/b^2          (Sec. 2.2.1)
 *   2. L0 friends-of-friends over the particles denser than Delta_L0,min (Sec. 2.2.1)
 *   3. CompaSO L1 inside every L0 group: nuclei in descending density, the
 *      enclosed-density radius R_L1, eligibility inside alpha R_L1 and the
 *      competitive reassignment with c_Roche                          (Sec. 2.2.2)
 *   4. the output cut at the minimum L1 halo size                      (Sec. 2.2.2, Table 1)
 *
 * Conventions shared by every entry point
 *   - Array arguments named pos, density, l0_id, halo_id and halos are DEVICE
 *     pointers owned by the caller (for instance torch tensors on the GPU).  The
 *     library never frees or retains them beyond the call.
 *   - pos is float32 [n][3] (x, y, z interleaved, C-contiguous) with coordinates
 *     in [0, box).  Coordinates outside that range are rejected.
 *   - Lengths b_kernel and l_fof are given in units of the mean interparticle
 *     spacing l_mean = nbar^(-1/3) (as in Table 1); nbar is mean_density, or
 *     n / box^3 when mean_density <= 0.
 *   - Densities are in units of the mean density (a uniform field has Delta = 1).
 *   - Labels are int32: 0 means "none"; otherwise 1 + an original particle index
 *     (L0: the smallest index of the group; halo: the index of its nucleus).
 *   - Pointers named n_groups / n_halos are HOST pointers; filling them makes the
 *     call wait for the stream.  All other work is enqueued on `stream` (a
 *     hipStream_t; NULL = the default stream).
 *   - Argument errors are reported before anything is enqueued.  Device errors
 *     return HF_ERR_DEVICE and hf_last_error() gives the HIP error text.
 *   - An hf_ctx owns the scratch memory (cell lists, union-find, queues); it grows
 *     on demand with hipMalloc and is released by hf_destroy.  A context is not
 *     thread-safe: use one context per host thread / stream.
 */
#ifndef HF_H
#define HF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HF_OK = 0,
    HF_ERR_INVALID = 1,     /* bad argument (n < 0, box <= 0, NaN parameter, box too small) */
    HF_ERR_NOMEM = 2,       /* device allocation failed */
    HF_ERR_CAPACITY = 3,    /* halos_cap too small: *n_halos holds the required count */
    HF_ERR_DEVICE = 4,      /* a HIP call failed */
    HF_ERR_UNSUPPORTED = 5  /* no usable gfx950 device */
} hf_status;

/* Parameters; Table 1 names in brackets.  hf_default_params() gives the paper's
 * Einstein-de Sitter values. */
typedef struct {
    double box;            /* periodic box side L [BoxSize]                           */
    double mean_density;   /* nbar; <= 0 means n / box^3                              */
    double b_kernel;       /* kernel radius b, units of l_mean: 0.4 [DensityKernelRad]*/
    double l_fof;          /* L0 linking length, units of l_mean: 0.25 [FoFLinkingLength] */
    double delta_l0_min;   /* L0 density threshold: 60 [L0DensityThreshold]           */
    double delta_l1;       /* L1 SO threshold: 200 [SODensityL1]                      */
    double delta_l2;       /* L2 SO threshold: 800 [SODensityL2] (hf_halo_stats)      */
    double alpha_elig;     /* eligibility radius / R_L1: 0.8 [SO_alpha_eligible]      */
    double c_roche;        /* reassignment factor: 2 [SO_RocheCoeff]                  */
    double n_new_min;      /* nucleation floor from a SIS of this many particles: 35
                              [SO_NPForMinDensity]                                    */
    double particle_mass;  /* mass per particle for hf_halo.mass: 1                   */
    int32_t n_l1_min;      /* smallest L1 halo kept in the output: 35 [MinL1HaloNP]   */
    int32_t self_count;    /* 1 adds W(0) = 1 (the particle itself) to its density; 0 */
} hf_params;

/* One output halo.  Rows of the halo table are sorted by ascending id. */
typedef struct {
    int32_t id;          /* 1 + nucleus (the value written to halo_id)               */
    int32_t nucleus;     /* original index of the nucleus particle (SO_central_particle) */
    int32_t l0_id;       /* label of the L0 group holding the halo                    */
    int32_t n;           /* number of member particles N (>= n_l1_min)                */
    int32_t n_enclosed;  /* particles of the L0 group inside R_L1 (enclosed count i)  */
    float x, y, z;       /* halo centre = nucleus position                            */
    float r;             /* R_L1 = (i / ((4 pi/3) Delta_L1 nbar))^(1/3)               */
    float mass;          /* n * particle_mass                                         */
} hf_halo;

/* Level 2 summary and position statistics of one L1 halo (end of Sec. 2.2.2,
 * Table 1), from hf_halo_stats.  Distances are minimum-image. */
typedef struct {
    int32_t id;             /* L1 halo id (1 + nucleus, as in hf_halo)                 */
    int32_t n;              /* members N                                               */
    int32_t n_l2;           /* L2 halos found inside it                                */
    int32_t l2max_nucleus;  /* original index of the first L2 halo's nucleus
                               [SO_L2max_central_particle]; -1 if none                 */
    int32_t l2max_n;        /* members of the first L2 halo                            */
    float x_com[3];         /* centre of mass of the members [x_com]                   */
    float x_l2com[3];       /* centre of mass of the first L2 halo [x_L2com];
                               x_com if there is none                                  */
    float l2_mass[5];       /* masses of the 5 largest L2 halos, descending; 0 beyond  */
    float r_pct[9];         /* r_XX about x_L2com for XX = 10 25 33 50 67 75 90 95 98:
                               the k-th smallest member distance, k = ceil(XX N/100)
                               [r_XX_L2com]                                            */
    float vcirc_max;        /* max over members of sqrt(m_p k / r_k), k members within
                               r_k of x_L2com, G = 1 [vcirc_max_L2com]                 */
    float rvcirc_max;       /* the r_k where it is reached [rvcirc_max_L2com]          */
} hf_halo_summary;

/* Per-call statistics of the last call on a context (device event timings of
 * each stage on the call's stream, and work counters). */
typedef struct {
    float ms_bin, ms_density, ms_fof, ms_segment, ms_candidates, ms_accept, ms_assign,
          ms_output, ms_total;
    int64_t n_cells;          /* cells of the binning grid                      */
    int64_t n_members;        /* particles above delta_l0_min                   */
    int64_t n_groups;         /* L0 groups (including single particles)         */
    int64_t n_candidates;     /* nucleus candidates (local peaks above the floor) */
    int64_t n_found;          /* halos before the output cut                    */
    int64_t n_halos;          /* halos after the cut                            */
    int64_t n_dense_cells;    /* cells holding >= 8 particles                   */
    int64_t n_dense_chunks;   /* 64-particle wavefront chunks of dense cells    */
    int64_t n_sparse;         /* particles of the other cells                   */
    int64_t n_hard;           /* candidate tests not settled by the own sub-cell */
} hf_stats;

typedef struct hf_ctx hf_ctx;

/* Fill p with the paper's defaults (Table 1, Einstein-de Sitter thresholds). */
void hf_default_params(hf_params *p);

/* Thresholds at redshift z (Sec. 2.3.1) for a flat universe of matter (Omega_m0
 * today) and a cosmological constant: with Omega_m(z) = Om (1+z)^3 /
 * (Om (1+z)^3 + 1 - Om) and x = Omega_m(z) - 1, the fitting function
 * 18 pi^2 + 82 x - 39 x^2 (relative to the critical density) divided by
 * 18 pi^2 Omega_m(z) scales delta_l1, delta_l2 and delta_l0_min of in; l_fof is
 * divided by the cube root of that factor; b_kernel and the rest are copied.
 * Table 1 (Omega_m0 = 0.315, z = 0.5): 258.2, 1033.0, 77.5 from 200, 800, 60.
 * HF_ERR_INVALID unless 0 < omega_m0 <= 1 and z > -1.  Host only. */
hf_status hf_params_at_redshift(const hf_params *in, double omega_m0, double z, hf_params *out);

/* Derived constants for n particles under p, computed on the host exactly as the
 * kernels use them (out[11]): nbar, b, l, b^2, l^2, density normalisation
 * 15/(8 pi b^3 nbar) (App. B.2), K = (4 pi/3) Delta_L1 nbar (so that R^3 = i/K,
 * Sec. 2.2.2 step 1), K^2, the nucleation floor (smoothed centre of a SIS with
 * n_new_min particles inside its 200x-mean radius, Sec. 2.2.2 step 4 and
 * App. B.2), alpha^6 and c_Roche^3. */
hf_status hf_derived(const hf_params *p, int64_t n, double *out);

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the device
 * memory the context's scratch arenas may hold together (its single-box arena
 * and the lanes of hf_find_batch; 0 = no bound): a call whose arena would pass
 * it returns HF_ERR_NOMEM before anything is enqueued.  Fails with
 * HF_ERR_UNSUPPORTED when the device is not gfx950. */
hf_status hf_create(hf_ctx **ctx, int device, uint64_t hbm_budget_bytes);
void hf_destroy(hf_ctx *ctx);
const char *hf_last_error(const hf_ctx *ctx);
hf_status hf_get_stats(const hf_ctx *ctx, hf_stats *out);

/* Options of a context (hf_set_option / hf_get_option; they apply to the
 * calls made after the change, batches included). */
enum {
    HF_OPT_RADIUS_SEARCH = 1  /* how the enclosed count i of a nucleus (R_L1) is searched */
};
/* Values of HF_OPT_RADIUS_SEARCH.  Both give the count of the sorted
 * definition (Sec. 2.2.2 step 1, Sec. 2.3.3), so every output is the same. */
enum {
    HF_RADIUS_HISTOGRAM = 0,  /* default: one pass over the group into a histogram
                                 of the integer crossing buckets, then a prefix scan */
    HF_RADIUS_BINS = 1        /* the radial bins of Sec. 2.3.4 (width: cell side /
                                 sqrt(3)): a pass counts the members per bin, bins
                                 whose inner count placed at their outer edge still
                                 meets the threshold are passed over, and the others
                                 are searched outwards, each by one more pass */
};
/* HF_ERR_INVALID for an unknown option or value. */
hf_status hf_set_option(hf_ctx *ctx, int32_t option, int64_t value);
hf_status hf_get_option(const hf_ctx *ctx, int32_t option, int64_t *value);

/* Step 1 (Sec. 2.2.1): density[i] = norm * sum_{j != i, r_ij < b} (1 - r_ij^2/b^2)
 * over periodic minimum images; norm makes a uniform field average 1 (App. B.2).
 * density: float32 [n], original particle order. */
hf_status hf_density(hf_ctx *ctx, const float *pos, int64_t n, const hf_params *p,
                     float *density, void *stream);

/* Step 2 (Sec. 2.2.1): L0 groups = friends-of-friends with linking length l over
 * the particles with density > delta_l0_min (two members are friends when their
 * separation is less than l).  density: float32 [n] (any field, e.g. from
 * hf_density).  l0_id: int32 [n], 1 + smallest original index of the group,
 * 0 for particles below the threshold.  *n_groups (host, may be NULL): number of
 * groups including single-particle ones. */
hf_status hf_l0_fof(hf_ctx *ctx, const float *pos, const float *density, int64_t n,
                    const hf_params *p, int32_t *l0_id, int64_t *n_groups, void *stream);

/* Step 3 + 4 (Sec. 2.2.2): CompaSO L1 inside every L0 group given by l0_id (any
 * labelling with values in [0, n], 0 = outside every group, equal values = one
 * group), then the cut N >= n_l1_min.  halo_id: int32 [n], 1 + nucleus index of
 * the particle's halo, 0 if none.  halos: device array of halos_cap rows,
 * ascending id.  *n_halos (host): number of halos kept.  If it exceeds halos_cap
 * the call returns HF_ERR_CAPACITY; halo_id is still written, halos is not. */
hf_status hf_compaso(hf_ctx *ctx, const float *pos, const float *density,
                     const int32_t *l0_id, int64_t n, const hf_params *p, int32_t *halo_id,
                     hf_halo *halos, int64_t halos_cap, int64_t *n_halos, void *stream);

/* Measurement helper: number of ordered pairs (i, j), j != i, closer than b (the
 * useful pair count of step 1, P_b = sum_i #{j != i : r_ij < b}) into *pairs
 * (host).  Used to express the density kernel's work in pair-interactions. */
hf_status hf_count_pairs(hf_ctx *ctx, const float *pos, int64_t n, const hf_params *p,
                         int64_t *pairs, void *stream);

/* Level 2 and position statistics of the L1 halos (end of Sec. 2.2.2, Table 1).
 * halo_id (device int32 [n], original order): an L1 labelling such as
 * hf_find's (1 + nucleus index, 0 = none); density: the field it was found on
 * (device float32 [n]).  Inside every L1 halo the competitive SO steps are
 * repeated with delta_l2 in place of delta_l1 everywhere (nucleation floor,
 * enclosed counts, eligibility and reassignment), the halo's members taking the
 * place of the L0 group.  n_halos must equal the number of distinct non-zero
 * labels (HF_ERR_INVALID otherwise).  stats (device, n_halos rows) are in
 * ascending id.  group_start (device int32 [n_halos + 1], may be NULL) and
 * group_members (device int32 [number of labelled particles], may be NULL)
 * receive the members grouped by halo: ascending id, ascending original index
 * inside a halo (the halo-ordered particle list of Sec. 2.3.5). */
hf_status hf_halo_stats(hf_ctx *ctx, const float *pos, const float *density,
                        const int32_t *halo_id, int64_t n, const hf_params *p,
                        int64_t n_halos, hf_halo_summary *stats, int32_t *group_start,
                        int32_t *group_members, void *stream);

/* The whole pass: density, L0 FoF and CompaSO L1 with the output cut, sharing one
 * cell binning.  Outputs as in the three calls above; density and l0_id may be
 * NULL when not wanted. */
hf_status hf_find(hf_ctx *ctx, const float *pos, int64_t n, const hf_params *p,
                  float *density, int32_t *l0_id, int32_t *halo_id, hf_halo *halos,
                  int64_t halos_cap, int64_t *n_halos, void *stream);

/* hf_find for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * pass, outputs and errors as hf_find, with its scratch arena carved from a
 * static device array of 256 MiB that every GPU the library runs on holds until
 * the process ends (hf_create takes its address).  It calls no hipMalloc,
 * hipFree or allocating library routine.  A box needing more scratch than that
 * (about 6e5 particles at mean density 1 with the default parameters; the need
 * grows with n and with the cell grid box^3 / max(b, l)^3) is refused with
 * HF_ERR_INVALID before anything is enqueued.  Every context on one GPU shares
 * that array, which keeps the last call's contents: calls that overlap on one
 * GPU (several streams or threads) race and must be serialized by the caller. */
hf_status hf_find_noalloc(hf_ctx *ctx, const float *pos, int64_t n, const hf_params *p,
                          float *density, int32_t *l0_id, int32_t *halo_id, hf_halo *halos,
                          int64_t halos_cap, int64_t *n_halos, void *stream);

/* hf_find plus its members collected into group order (Sec. 2.3.5): members
 * (device int32 [n]) holds the particles of each halo of the table, rows in
 * table order and ascending original index inside a row, then the particles
 * of no halo (halo_id 0) in ascending index; halo_start (device int64
 * [halos_cap + 1]) receives in entries 0..*n_halos the first position of each
 * row's run and, last, of the rest.  On HF_ERR_CAPACITY members and
 * halo_start are not written.  The call ends synchronized with its stream. */
hf_status hf_find_grouped(hf_ctx *ctx, const float *pos, int64_t n, const hf_params *p,
                          float *density, int32_t *l0_id, int32_t *halo_id, hf_halo *halos,
                          int64_t halos_cap, int64_t *n_halos, int32_t *members,
                          int64_t *halo_start, void *stream);

/* ---- Many boxes per call ------------------------------------------------
 * hf_find on n_boxes independent periodic boxes (Sec. 2.2 applied to each box
 * on its own).  Box b holds particles [box_offsets[b], box_offsets[b+1]) of the
 * concatenated device array pos (float32 [total][3]) and is found with
 * params[b] (host array; its box side and mean density are the box's own).
 * Outputs are concatenated in the same particle order: density (may be NULL),
 * l0_id (may be NULL) and halo_id, with labels local to the box (1 + index
 * within the box).  Box b's halo table goes to rows
 * [halo_offsets[b], halo_offsets[b+1]) of halos (device); n_halos[b] (host)
 * receives its count.  box_offsets and halo_offsets are host arrays of
 * n_boxes + 1 non-decreasing values starting at 0.
 *
 * The boxes are found in fused passes: every stage is one launch over all
 * boxes of a group of consecutive boxes, whose particles and cells are numbered
 * together (the L0 groups of all its boxes form one work list for the
 * acceptance step, largest first).  The batch is cut into n_lanes groups of
 * about equal particle counts (at most 16 and n_boxes; a group also closes
 * before its cells reach 2^31), which run at once, each on its own stream and
 * scratch arena held by the context.  n_lanes <= 0 takes the count that
 * hf_tune_batch or hf_load_tuning recorded for this batch shape, else 1.
 * Every box's outputs are identical to hf_find's on that box alone.  The call
 * first waits for the caller's stream and returns when all boxes are done.
 * Returns the first failing box's error (text names the box); if only halo
 * capacities were too small, HF_ERR_CAPACITY with every n_halos[b] set to the
 * required count (tables of boxes that fit are written). */
hf_status hf_find_batch(hf_ctx *ctx, int32_t n_boxes, const int64_t *box_offsets,
                        const float *pos, const hf_params *params, float *density,
                        int32_t *l0_id, int32_t *halo_id, hf_halo *halos,
                        const int64_t *halo_offsets, int64_t *n_halos, int32_t n_lanes,
                        void *stream);

/* Autotuning of hf_find_batch (a measurement helper, no step of the method):
 * runs the batch (same arguments as hf_find_batch) with 1 .. max_groups fused
 * groups, each once untimed and then reps times, and keeps the count of the
 * fastest run (a larger count must win by more than 2 %).  The context
 * remembers it for batches with the same n_boxes and a particle total within
 * 25 %, which hf_find_batch then uses when called with n_lanes <= 0.
 * *best_groups and *best_ms (host, may be NULL) receive the choice and its
 * time in milliseconds.  table_path (may be NULL): a text file rewritten with
 * this shape's line replaced or appended, one line per shape:
 *   hf-tune v1 <arch> n_boxes=<b> total=<n> groups=<g> ms=<t>
 * The outputs hold the last run's results (identical for every count). */
hf_status hf_tune_batch(hf_ctx *ctx, int32_t n_boxes, const int64_t *box_offsets,
                        const float *pos, const hf_params *params, float *density,
                        int32_t *l0_id, int32_t *halo_id, hf_halo *halos,
                        const int64_t *halo_offsets, int64_t *n_halos, int32_t max_groups,
                        int32_t reps, const char *table_path, int32_t *best_groups,
                        float *best_ms, void *stream);

/* Load a table written by hf_tune_batch into the context: lines of the
 * context's device architecture are kept (a later line of the same shape
 * replaces an earlier one), others and lines starting with '#' are skipped.
 * *n_entries (may be NULL) receives the number of lines taken.
 * HF_ERR_INVALID when the file cannot be read. */
hf_status hf_load_tuning(hf_ctx *ctx, const char *table_path, int32_t *n_entries);

/* The group count hf_find_batch uses for a batch of n_boxes boxes and `total`
 * particles when called with n_lanes (host only, *groups receives it). */
hf_status hf_batch_groups(const hf_ctx *ctx, int32_t n_boxes, int64_t total, int32_t n_lanes,
                          int32_t *groups);

/* ---- Request loop ----------------------------------------------------------
 * A server runs halo-finding requests for boxes of different sizes as they
 * arrive.  It owns n_slots pipelines (streams, scratch arenas and device
 * buffers that stay allocated between requests) and one host thread per slot.
 * A free slot takes the oldest waiting request when the device memory of all
 * slots, with this request's need, stays within hbm_budget_bytes (idle slots
 * give their memory back when that makes it fit); requests therefore overlap
 * on the GPU while the budget allows.  When several requests of at most 4 Mi
 * particles wait, the slot takes them together (up to 16 Mi particles, 32
 * requests, and the sum of their needs within the budget) and finds them in
 * one fused pass, as hf_find_batch does; a single waiting request runs alone.
 * Each request's result is identical to hf_find on the same box alone; the
 * requests of one pass share its t_start, t_done and ms_gpu. */
typedef struct hf_server hf_server;

typedef struct {
    const float *pos;   /* host float32 [n][3]; must stay valid until waited for
                           (page-locked memory makes the copy asynchronous)   */
    int64_t n;
    hf_params params;
    float *density;     /* host float32 [n] or NULL                            */
    int32_t *l0_id;     /* host int32 [n] or NULL                              */
    int32_t *halo_id;   /* host int32 [n]                                      */
    hf_halo *halos;     /* host, halos_cap rows                                */
    int64_t halos_cap;
} hf_request;

typedef struct {
    int32_t status;     /* hf_status of the request (HF_ERR_CAPACITY: n_halos is
                           the required capacity; halo_id is still written)   */
    int32_t slot;       /* slot that ran it                                    */
    int64_t n_halos;
    double t_submit;    /* seconds on the server clock (hf_server_now)         */
    double t_start;     /* taken by a slot                                     */
    double t_done;      /* results written to the host buffers                 */
    float ms_gpu;       /* device time of its pass (first to last stage event) */
    char error[160];    /* error text when status != HF_OK                     */
} hf_result;

/* n_slots in 1..16.  HF_ERR_UNSUPPORTED when the device is not gfx950. */
hf_status hf_server_create(hf_server **srv, int device, int32_t n_slots,
                           uint64_t hbm_budget_bytes);
/* Queue a request (the struct is copied; the buffers it points to are not).
 * HF_ERR_NOMEM when the request alone needs more than the budget. */
hf_status hf_server_submit(hf_server *srv, const hf_request *req, int64_t *ticket);
/* Block until the request is done and return its result; a ticket is waited
 * for once. */
hf_status hf_server_wait(hf_server *srv, int64_t ticket, hf_result *res);
double hf_server_now(const hf_server *srv);
/* Device memory held by the slots now (arenas and request buffers). */
uint64_t hf_server_held_bytes(hf_server *srv);
const char *hf_server_last_error(const hf_server *srv);
/* Finish every queued request, then free the slots. */
void hf_server_destroy(hf_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* HF_H */
