// Many boxes per call (hf_find_batch) and a request loop (hf_server).
//
// hf_find_batch finds its boxes in fused passes: every stage is one launch over
// all boxes of a group, whose particles and cells are numbered together, so
// that small boxes that could not fill 256 CUs on their own run as one large
// problem.  A batch may be cut into a few groups that run at once on lanes
// (stream, arena and host thread each), so that one group's waits for its
// counts overlap with another's kernels.  The request loop runs one request
// per lane.  Results do not depend on the grouping or on what runs beside a
// box: the pass is deterministic and no box reads another box's data.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <fstream>
#include <condition_variable>
#include <deque>
#include <stdio.h>
#include <string.h>
#include <thread>
#include <unordered_map>

#include "hf_lane.h"

namespace {

constexpr int kDefaultBatchGroups = 1;  // fused groups of hf_find_batch when none is asked for
constexpr int kMaxLanes = 16;

void add_stats(hf_stats &a, const hf_stats &b) {
    a.ms_bin += b.ms_bin;
    a.ms_density += b.ms_density;
    a.ms_fof += b.ms_fof;
    a.ms_segment += b.ms_segment;
    a.ms_candidates += b.ms_candidates;
    a.ms_accept += b.ms_accept;
    a.ms_assign += b.ms_assign;
    a.ms_output += b.ms_output;
    a.n_cells += b.n_cells;
    a.n_members += b.n_members;
    a.n_groups += b.n_groups;
    a.n_candidates += b.n_candidates;
    a.n_found += b.n_found;
    a.n_halos += b.n_halos;
    a.n_dense_cells += b.n_dense_cells;
    a.n_dense_chunks += b.n_dense_chunks;
    a.n_sparse += b.n_sparse;
    a.n_hard += b.n_hard;
}

hf_status batch_fail(hf_ctx *c, hf_status st, const std::string &msg) {
    c->main.err = msg;
    return st;
}

// The tuned group count for a batch of n_boxes boxes and `total` particles:
// the entry with the same box count whose particle total is nearest, within
// 25 % of it; 0 when there is none.
int tuned_groups(const hf_ctx *c, int32_t n_boxes, int64_t total) {
    int best = 0;
    double best_rel = 0.25;
    for (const auto &e : c->tuning) {
        if (e.n_boxes != n_boxes || e.total <= 0) continue;
        const double rel = std::fabs((double)total - (double)e.total) / (double)e.total;
        if (rel <= best_rel) {
            best_rel = rel;
            best = e.groups;
        }
    }
    return best;
}

// Group count hf_find_batch uses for an explicit n_lanes (> 0) or, for
// n_lanes <= 0, the tuned one, else the default; at most kMaxLanes and
// n_boxes.
int batch_groups(const hf_ctx *c, int32_t n_boxes, int64_t total, int32_t n_lanes) {
    int k = n_lanes > 0 ? n_lanes : tuned_groups(c, n_boxes, total);
    if (k <= 0) k = kDefaultBatchGroups;
    return std::max(1, std::min(std::min(k, kMaxLanes), (int)n_boxes));
}

// The device's architecture name without its feature suffixes ("gfx950").
std::string arch_name(int device) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

// One line of a tuning table:
//   hf-tune v1 <arch> n_boxes=<b> total=<n> groups=<g> ms=<t>
// Lines of another architecture or format, and lines starting with '#', are
// skipped.
bool parse_tune_line(const std::string &line, const std::string &arch, hf::TuneEntry *e) {
    char a[64] = {0};
    int nb = 0, g = 0;
    long long tot = 0;
    float ms = 0.0f;
    if (line.empty() || line[0] == '#') return false;
    if (sscanf(line.c_str(), "hf-tune v1 %63s n_boxes=%d total=%lld groups=%d ms=%f", a, &nb, &tot, &g, &ms) != 5)
        return false;
    if (arch != a || nb <= 0 || tot < 0 || g <= 0 || g > kMaxLanes) return false;
    *e = hf::TuneEntry{nb, (int64_t)tot, g, ms};
    return true;
}

std::string tune_line(const std::string &arch, const hf::TuneEntry &e) {
    char buf[256];
    snprintf(buf, sizeof buf, "hf-tune v1 %s n_boxes=%d total=%lld groups=%d ms=%.3f", arch.c_str(), e.n_boxes,
             (long long)e.total, e.groups, e.ms);
    return buf;
}

// Keep e in the context's table (replacing an entry of the same shape).
void remember(hf_ctx *c, const hf::TuneEntry &e) {
    for (auto &x : c->tuning)
        if (x.n_boxes == e.n_boxes && x.total == e.total) {
            x = e;
            return;
        }
    c->tuning.push_back(e);
}

}  // namespace

extern "C" {

hf_status hf_find_batch(hf_ctx *ctx, int32_t n_boxes, const int64_t *box_offsets, const float *pos,
                        const hf_params *params, float *density, int32_t *l0_id, int32_t *halo_id,
                        hf_halo *halos, const int64_t *halo_offsets, int64_t *n_halos,
                        int32_t n_lanes, void *stream) {
    if (!ctx) return HF_ERR_INVALID;
    ctx->main.err.clear();
    ctx->main.stats = hf_stats{};
    if (n_boxes < 0) return batch_fail(ctx, HF_ERR_INVALID, "n_boxes is negative");
    if (n_boxes == 0) return HF_OK;
    if (!box_offsets || !params || !halo_offsets || !n_halos)
        return batch_fail(ctx, HF_ERR_INVALID, "box_offsets / params / halo_offsets / n_halos is NULL");
    if (box_offsets[0] != 0 || halo_offsets[0] != 0)
        return batch_fail(ctx, HF_ERR_INVALID, "box_offsets[0] and halo_offsets[0] must be 0");
    for (int32_t b = 0; b < n_boxes; b++)
        if (box_offsets[b + 1] < box_offsets[b] || halo_offsets[b + 1] < halo_offsets[b])
            return batch_fail(ctx, HF_ERR_INVALID, "box_offsets / halo_offsets must not decrease");
    const int64_t total = box_offsets[n_boxes];
    if (total >= (int64_t)0x7fffffff) return batch_fail(ctx, HF_ERR_INVALID, "too many particles");
    if (total > 0 && (!pos || !halo_id)) return batch_fail(ctx, HF_ERR_INVALID, "pos / halo_id is NULL");
    if (halo_offsets[n_boxes] > 0 && !halos) return batch_fail(ctx, HF_ERR_INVALID, "halos is NULL");

    // Groups of consecutive boxes, each found in one fused pass (every stage
    // one launch over all its boxes): k groups of about equal particle counts,
    // which run at once on k lanes so that one group's waits for its counts
    // overlap with another's kernels.  A group is also closed before its cell
    // count would pass 2^31 (cell numbers of a pass stay 32-bit).
    const int k = batch_groups(ctx, n_boxes, total, n_lanes);
    std::vector<int32_t> cut{0};
    {
        int64_t cells = 0;
        const double target = (double)total / k;
        for (int32_t b = 0; b < n_boxes; b++) {
            const int64_t nb = box_offsets[b + 1] - box_offsets[b];
            int64_t cb = 0;  // the box's cells (0 if its parameters are invalid: its pass reports it)
            if (nb > 0) {
                const int64_t o2[2] = {0, nb};
                int64_t nt = 0;
                hf::boxes_arena_bytes(hf::BoxSet{1, o2, params + b, nullptr, nullptr}, &nt, &cb);
            }
            const bool full_cells = b > cut.back() && cells + cb >= ((int64_t)1 << 31);
            const bool full_share = (int)cut.size() < k && b > cut.back() &&
                                    (double)box_offsets[b] >= target * (double)cut.size();
            if (full_cells || full_share) {
                cut.push_back(b);
                cells = 0;
            }
            cells += cb;
        }
        cut.push_back(n_boxes);
    }
    const int ngroups = (int)cut.size() - 1;
    const int lanes = std::min(k, ngroups);
    while ((int)ctx->pool.size() < lanes) {
        auto L = std::make_unique<hf::Lane>();
        L->budget = &ctx->budget;
        L->radius_bins = ctx->radius_bins;
        if (hf::lane_init(L.get(), ctx->main.device, true) != HF_OK) {
            hf::lane_destroy(L.get());
            return batch_fail(ctx, HF_ERR_DEVICE, "could not create a batch lane");
        }
        ctx->pool.push_back(std::move(L));
    }
    // work the caller queued on its stream (e.g. the copy of pos) comes first
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
        return batch_fail(ctx, HF_ERR_DEVICE, "hipStreamSynchronize of the caller's stream failed");

    std::vector<hf_status> st(ngroups, HF_OK);
    std::vector<std::string> msg(ngroups);
    std::vector<hf_stats> lane_stats(lanes, hf_stats{});
    std::atomic<int32_t> next{0};
    const auto t0 = std::chrono::steady_clock::now();
    auto work = [&](int t) {
        hf::Lane *L = ctx->pool[t].get();
        (void)hipSetDevice(L->device);
        std::vector<int64_t> offs, hoffs;
        for (;;) {
            const int32_t q = next.fetch_add(1);
            if (q >= ngroups) break;
            const int32_t b0 = cut[q], b1 = cut[q + 1], nb = b1 - b0;
            offs.resize(nb + 1);
            hoffs.resize(nb + 1);
            for (int32_t j = 0; j <= nb; j++) {
                offs[j] = box_offsets[b0 + j] - box_offsets[b0];
                hoffs[j] = halo_offsets[b0 + j] - halo_offsets[b0];
            }
            const int64_t o = box_offsets[b0];
            hf::BoxSet bs{nb, offs.data(), params + b0, halos ? halos + halo_offsets[b0] : nullptr, hoffs.data()};
            bs.first = b0;
            bs.named = true;
            st[q] = hf::lane_find_boxes(L, bs, offs[nb] ? pos + 3 * o : nullptr, density ? density + o : nullptr,
                                        l0_id ? l0_id + o : nullptr, halo_id + o, n_halos + b0, L->stream);
            if (st[q] != HF_OK) msg[q] = L->err;
            add_stats(lane_stats[t], L->stats);
        }
    };
    std::vector<std::thread> threads;
    for (int t = 1; t < lanes; t++) threads.emplace_back(work, t);
    work(0);
    for (auto &th : threads) th.join();
    const auto t1 = std::chrono::steady_clock::now();

    for (int t = 0; t < lanes; t++) add_stats(ctx->main.stats, lane_stats[t]);
    ctx->main.stats.ms_total = (float)std::chrono::duration<double, std::milli>(t1 - t0).count();
    for (int q = 0; q < ngroups; q++)
        if (st[q] != HF_OK && st[q] != HF_ERR_CAPACITY) return batch_fail(ctx, st[q], msg[q]);
    for (int q = 0; q < ngroups; q++)
        if (st[q] == HF_ERR_CAPACITY)
            return batch_fail(ctx, HF_ERR_CAPACITY, msg[q] + " (n_halos holds the required counts)");
    return HF_OK;
}

hf_status hf_batch_groups(const hf_ctx *ctx, int32_t n_boxes, int64_t total, int32_t n_lanes, int32_t *groups) {
    if (!ctx || !groups || n_boxes <= 0 || total < 0) return HF_ERR_INVALID;
    *groups = batch_groups(ctx, n_boxes, total, n_lanes);
    return HF_OK;
}

hf_status hf_tune_batch(hf_ctx *ctx, int32_t n_boxes, const int64_t *box_offsets, const float *pos,
                        const hf_params *params, float *density, int32_t *l0_id, int32_t *halo_id,
                        hf_halo *halos, const int64_t *halo_offsets, int64_t *n_halos, int32_t max_groups,
                        int32_t reps, const char *table_path, int32_t *best_groups, float *best_ms,
                        void *stream) {
    if (!ctx) return HF_ERR_INVALID;
    if (n_boxes <= 0 || !box_offsets) return batch_fail(ctx, HF_ERR_INVALID, "nothing to tune: n_boxes <= 0");
    if (max_groups <= 0 || reps <= 0) return batch_fail(ctx, HF_ERR_INVALID, "max_groups and reps must be > 0");
    const int gmax = std::min(std::min((int)max_groups, kMaxLanes), (int)n_boxes);
    const int64_t total = box_offsets[n_boxes];
    hf::TuneEntry best{n_boxes, total, 0, 0.0f};
    for (int g = 1; g <= gmax; g++) {
        // one untimed call (it also sizes the lanes' arenas), then the fastest of reps
        hf_status st = hf_find_batch(ctx, n_boxes, box_offsets, pos, params, density, l0_id, halo_id, halos,
                                     halo_offsets, n_halos, g, stream);
        if (st != HF_OK) return st;
        double ms = 0.0;
        for (int r = 0; r < reps; r++) {
            const auto t0 = std::chrono::steady_clock::now();
            st = hf_find_batch(ctx, n_boxes, box_offsets, pos, params, density, l0_id, halo_id, halos, halo_offsets,
                               n_halos, g, stream);
            const auto t1 = std::chrono::steady_clock::now();
            if (st != HF_OK) return st;
            const double t = std::chrono::duration<double, std::milli>(t1 - t0).count();
            if (r == 0 || t < ms) ms = t;
        }
        // a larger count must be faster by more than 2 % to be taken
        if (best.groups == 0 || ms < 0.98 * best.ms) {
            best.groups = g;
            best.ms = (float)ms;
        }
    }
    remember(ctx, best);
    if (best_groups) *best_groups = best.groups;
    if (best_ms) *best_ms = best.ms;
    if (table_path && table_path[0]) {
        // rewrite the table with this shape's line replaced (or appended)
        const std::string arch = arch_name(ctx->main.device);
        std::vector<std::string> lines;
        {
            std::ifstream in(table_path);
            std::string line;
            hf::TuneEntry e;
            while (std::getline(in, line)) {
                if (parse_tune_line(line, arch, &e) && e.n_boxes == best.n_boxes && e.total == best.total) continue;
                lines.push_back(line);
            }
        }
        if (lines.empty()) lines.push_back("# hf_find_batch tuning: fused group count per batch shape");
        lines.push_back(tune_line(arch, best));
        const std::string tmp = std::string(table_path) + ".tmp";
        {
            std::ofstream out(tmp, std::ios::trunc);
            for (const auto &l : lines) out << l << "\n";
            if (!out) return batch_fail(ctx, HF_ERR_INVALID, std::string("cannot write ") + tmp);
        }
        if (rename(tmp.c_str(), table_path) != 0)
            return batch_fail(ctx, HF_ERR_INVALID, std::string("cannot replace ") + table_path);
    }
    return HF_OK;
}

hf_status hf_load_tuning(hf_ctx *ctx, const char *table_path, int32_t *n_entries) {
    if (!ctx || !table_path) return HF_ERR_INVALID;
    std::ifstream in(table_path);
    if (!in) return batch_fail(ctx, HF_ERR_INVALID, std::string("cannot read ") + table_path);
    const std::string arch = arch_name(ctx->main.device);
    std::string line;
    hf::TuneEntry e;
    int32_t k = 0;
    while (std::getline(in, line))
        if (parse_tune_line(line, arch, &e)) {
            remember(ctx, e);
            k++;
        }
    if (n_entries) *n_entries = k;
    return HF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- server

namespace {

struct Pending {
    int64_t ticket;
    hf_request r;
    double t_submit;
    size_t need;
};

// Requests of at most kFuseBox particles that wait together are found in one
// fused pass (the pass of hf_find_batch), up to kFuseTotal particles and
// kFuseCount requests: small boxes alone cannot fill the GPU.  A slot that
// frees up with a single request waiting runs it alone, so at low load no
// request waits for others.
constexpr int64_t kFuseBox = (int64_t)4 << 20;
constexpr int64_t kFuseTotal = (int64_t)16 << 20;
constexpr size_t kFuseCount = 32;

struct Slot {
    hf::Lane lane;
    void *io = nullptr;  // device copies of the request's input and outputs
    size_t io_bytes = 0;
    bool busy = false;
    size_t reserved = 0;  // bytes granted at admission, counted while busy
    size_t held() const { return lane.arena_bytes + io_bytes; }
    // memory charged against the budget: a busy slot's worker may be growing its
    // buffers outside the lock, so its grant is counted instead
    size_t charged() const { return busy ? reserved : held(); }
};

size_t round256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t io_bytes_for(const hf_request &r) {
    const size_t n = (size_t)r.n;
    return round256(12 * n) + round256(4 * n) * 3 + round256(sizeof(hf_halo) * (size_t)(r.halos_cap > 0 ? r.halos_cap : 1));
}

}  // namespace

struct hf_server {
    int device = 0;
    uint64_t budget = 0;
    std::vector<std::unique_ptr<Slot>> slots;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Pending> queue;
    std::unordered_map<int64_t, hf_result> done;
    std::unordered_map<int64_t, bool> known;  // tickets submitted and not yet waited for
    int64_t next_ticket = 1;
    bool stop = false;
    std::string err;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    size_t held_total() const {
        size_t s = 0;
        for (auto &sl : slots) s += sl->charged();
        return s;
    }
    // Whether slot t may take the request at the head of the queue within the
    // memory budget; frees the memory of idle slots when that makes it fit.
    bool admit(int t) {
        const Pending &q = queue.front();
        Slot &me = *slots[t];
        auto fits = [&] { return held_total() - me.charged() + std::max(me.held(), q.need) <= budget; };
        if (fits()) return true;
        for (size_t u = 0; u < slots.size() && !fits(); u++) {
            Slot &o = *slots[u];
            if ((int)u == t || o.busy || o.held() == 0) continue;
            hf::lane_release(&o.lane);
            if (o.io) (void)hipFree(o.io);
            o.io = nullptr;
            o.io_bytes = 0;
        }
        if (fits()) return true;
        // last resort: this slot's own memory is re-allocated at the needed size
        if (held_total() - me.charged() + q.need <= budget) {
            hf::lane_release(&me.lane);
            if (me.io) (void)hipFree(me.io);
            me.io = nullptr;
            me.io_bytes = 0;
            return true;
        }
        return false;
    }
    void run(int t, const Pending &q, hf_result &res);
    void run_fused(int t, const std::vector<Pending> &qs, std::vector<hf_result> &res);
    void worker(int t);
};

void hf_server::run(int t, const Pending &q, hf_result &res) {
    Slot &sl = *slots[t];
    hf::Lane *L = &sl.lane;
    const hf_request &r = q.r;
    const hipStream_t s = L->stream;
    auto set_err = [&](hf_status stt, const std::string &m) {
        res.status = stt;
        strncpy(res.error, m.c_str(), sizeof(res.error) - 1);
    };
    const size_t iob = io_bytes_for(r);
    if (iob > sl.io_bytes) {
        if (sl.io) (void)hipFree(sl.io);
        sl.io = nullptr;
        sl.io_bytes = 0;
        if (hipMalloc(&sl.io, iob) != hipSuccess) {
            (void)hipGetLastError();
            sl.io = nullptr;
            return set_err(HF_ERR_NOMEM, "hipMalloc of the request buffers failed");
        }
        sl.io_bytes = iob;
    }
    const size_t n = (size_t)r.n;
    char *base = (char *)sl.io;
    float *pos_d = (float *)base;
    float *dens_d = (float *)(base + round256(12 * n));
    int32_t *l0_d = (int32_t *)(base + round256(12 * n) + round256(4 * n));
    int32_t *halo_d = (int32_t *)(base + round256(12 * n) + 2 * round256(4 * n));
    hf_halo *halos_d = (hf_halo *)(base + round256(12 * n) + 3 * round256(4 * n));
    if (n > 0 && hipMemcpyAsync(pos_d, r.pos, 12 * n, hipMemcpyHostToDevice, s) != hipSuccess)
        return set_err(HF_ERR_DEVICE, "copy of positions to the device failed");
    int64_t nh = 0;
    hf_status st = hf::lane_find(L, n ? pos_d : nullptr, r.n, &r.params, r.density ? dens_d : nullptr,
                                 r.l0_id ? l0_d : nullptr, halo_d, r.halos_cap > 0 ? halos_d : nullptr,
                                 r.halos_cap, &nh, s);
    res.n_halos = nh;
    res.ms_gpu = L->stats.ms_total;
    if (st != HF_OK && st != HF_ERR_CAPACITY) return set_err(st, L->err);
    bool ok = true;
    if (n > 0) {
        ok &= hipMemcpyAsync(r.halo_id, halo_d, 4 * n, hipMemcpyDeviceToHost, s) == hipSuccess;
        if (r.density) ok &= hipMemcpyAsync(r.density, dens_d, 4 * n, hipMemcpyDeviceToHost, s) == hipSuccess;
        if (r.l0_id) ok &= hipMemcpyAsync(r.l0_id, l0_d, 4 * n, hipMemcpyDeviceToHost, s) == hipSuccess;
    }
    if (st == HF_OK && nh > 0)
        ok &= hipMemcpyAsync(r.halos, halos_d, sizeof(hf_halo) * (size_t)nh, hipMemcpyDeviceToHost, s) ==
              hipSuccess;
    ok &= hipStreamSynchronize(s) == hipSuccess;
    if (!ok) return set_err(HF_ERR_DEVICE, "copy of the results to the host failed");
    if (st != HF_OK) return set_err(st, L->err);
    res.status = HF_OK;
}

// Requests qs (two or more) as one fused pass on slot t: their positions laid
// end to end in the slot's buffers, one box each, then every request's outputs
// copied back.  A box's outputs are those of hf_find on it alone; a request
// whose halo table is too small gets HF_ERR_CAPACITY (its halo_id is still
// written).  Any other failure of the pass runs the requests one by one, so
// that each gets its own status.
void hf_server::run_fused(int t, const std::vector<Pending> &qs, std::vector<hf_result> &res) {
    Slot &sl = *slots[t];
    hf::Lane *L = &sl.lane;
    const hipStream_t s = L->stream;
    const size_t nb = qs.size();
    std::vector<int64_t> offs(nb + 1, 0), hoffs(nb + 1, 0), nh(nb, 0);
    std::vector<hf_params> params(nb);
    for (size_t b = 0; b < nb; b++) {
        offs[b + 1] = offs[b] + qs[b].r.n;
        hoffs[b + 1] = hoffs[b] + (qs[b].r.halos_cap > 0 ? qs[b].r.halos_cap : 0);
        params[b] = qs[b].r.params;
    }
    const size_t n = (size_t)offs[nb];
    const size_t iob = round256(12 * n) + round256(4 * n) * 3 +
                       round256(sizeof(hf_halo) * (size_t)(hoffs[nb] > 0 ? hoffs[nb] : 1));
    auto alone = [&] {
        for (size_t b = 0; b < nb; b++) run(t, qs[b], res[b]);
    };
    if (iob > sl.io_bytes) {
        if (sl.io) (void)hipFree(sl.io);
        sl.io = nullptr;
        sl.io_bytes = 0;
        if (hipMalloc(&sl.io, iob) != hipSuccess) {
            (void)hipGetLastError();
            sl.io = nullptr;
            return alone();
        }
        sl.io_bytes = iob;
    }
    char *base = (char *)sl.io;
    float *pos_d = (float *)base;
    float *dens_d = (float *)(base + round256(12 * n));
    int32_t *l0_d = (int32_t *)(base + round256(12 * n) + round256(4 * n));
    int32_t *halo_d = (int32_t *)(base + round256(12 * n) + 2 * round256(4 * n));
    hf_halo *halos_d = (hf_halo *)(base + round256(12 * n) + 3 * round256(4 * n));
    bool ok = true;
    for (size_t b = 0; b < nb; b++)
        if (qs[b].r.n > 0)
            ok &= hipMemcpyAsync(pos_d + 3 * offs[b], qs[b].r.pos, 12 * (size_t)qs[b].r.n, hipMemcpyHostToDevice,
                                 s) == hipSuccess;
    if (!ok) return alone();
    bool want_d = false, want_l0 = false;
    for (const Pending &q : qs) {
        want_d |= q.r.density != nullptr;
        want_l0 |= q.r.l0_id != nullptr;
    }
    hf::BoxSet bs{(int32_t)nb, offs.data(), params.data(), hoffs[nb] > 0 ? halos_d : nullptr, hoffs.data()};
    bs.named = true;
    const hf_status st = hf::lane_find_boxes(L, bs, n ? pos_d : nullptr, want_d ? dens_d : nullptr,
                                             want_l0 ? l0_d : nullptr, halo_d, nh.data(), s);
    if (st != HF_OK && st != HF_ERR_CAPACITY) return alone();
    for (size_t b = 0; b < nb; b++) {
        const hf_request &r = qs[b].r;
        const size_t o = (size_t)offs[b], m = (size_t)r.n;
        res[b].n_halos = nh[b];
        res[b].ms_gpu = L->stats.ms_total;
        if (m > 0) {
            ok &= hipMemcpyAsync(r.halo_id, halo_d + o, 4 * m, hipMemcpyDeviceToHost, s) == hipSuccess;
            if (r.density)
                ok &= hipMemcpyAsync(r.density, dens_d + o, 4 * m, hipMemcpyDeviceToHost, s) == hipSuccess;
            if (r.l0_id) ok &= hipMemcpyAsync(r.l0_id, l0_d + o, 4 * m, hipMemcpyDeviceToHost, s) == hipSuccess;
        }
        const bool fits = nh[b] <= (r.halos_cap > 0 ? r.halos_cap : 0);
        if (fits && nh[b] > 0)
            ok &= hipMemcpyAsync(r.halos, halos_d + hoffs[b], sizeof(hf_halo) * (size_t)nh[b],
                                 hipMemcpyDeviceToHost, s) == hipSuccess;
        res[b].status = fits ? HF_OK : HF_ERR_CAPACITY;
        if (!fits)
            strncpy(res[b].error, "halos_cap too small: n_halos holds the required capacity",
                    sizeof(res[b].error) - 1);
    }
    ok &= hipStreamSynchronize(s) == hipSuccess;
    if (!ok)
        for (size_t b = 0; b < nb; b++) {
            res[b].status = HF_ERR_DEVICE;
            strncpy(res[b].error, "copy of the results to the host failed", sizeof(res[b].error) - 1);
        }
}

void hf_server::worker(int t) {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        while (!(stop && queue.empty()) && (queue.empty() || slots[t]->busy || !admit(t))) cv_work.wait(lk);
        if (queue.empty()) break;  // stopping and nothing left
        std::vector<Pending> qs{queue.front()};
        queue.pop_front();
        // more small requests that wait, while their sum stays within the
        // fusion limits and, with their needs added up, within the budget
        size_t need = qs[0].need;
        int64_t total = qs[0].r.n, cells = 0;
        Slot &me = *slots[t];
        auto box_cells = [](const hf_request &r) -> int64_t {
            if (r.n <= 0) return 0;
            const int64_t o2[2] = {0, r.n};
            int64_t nt = 0, cb = 0;
            hf::boxes_arena_bytes(hf::BoxSet{1, o2, &r.params, nullptr, nullptr}, &nt, &cb);
            return cb;
        };
        if (qs[0].r.n <= kFuseBox && !queue.empty()) cells = box_cells(qs[0].r);
        while (qs[0].r.n <= kFuseBox && !queue.empty() && qs.size() < kFuseCount) {
            const Pending &nx = queue.front();
            if (nx.r.n > kFuseBox || total + nx.r.n > kFuseTotal) break;
            const int64_t cb = box_cells(nx.r);
            if (cells + cb >= ((int64_t)1 << 31)) break;
            if (held_total() - me.charged() + std::max(me.held(), need + nx.need) > budget) break;
            qs.push_back(nx);
            queue.pop_front();
            need += nx.need;
            total += nx.r.n;
            cells += cb;
        }
        me.reserved = std::max(me.held(), need);
        me.busy = true;
        lk.unlock();
        std::vector<hf_result> res(qs.size());
        const double t_start = now();
        for (size_t b = 0; b < qs.size(); b++) {
            memset(&res[b], 0, sizeof(hf_result));
            res[b].slot = t;
            res[b].t_submit = qs[b].t_submit;
            res[b].t_start = t_start;
        }
        if (qs.size() == 1)
            run(t, qs[0], res[0]);
        else
            run_fused(t, qs, res);
        const double t_done = now();
        lk.lock();
        me.busy = false;
        for (size_t b = 0; b < qs.size(); b++) {
            res[b].t_done = t_done;
            done[qs[b].ticket] = res[b];
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

extern "C" {

hf_status hf_server_create(hf_server **out, int device, int32_t n_slots, uint64_t hbm_budget_bytes) {
    if (!out) return HF_ERR_INVALID;
    *out = nullptr;
    if (n_slots <= 0 || n_slots > kMaxLanes || hbm_budget_bytes == 0) return HF_ERR_INVALID;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return HF_ERR_UNSUPPORTED;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return HF_ERR_DEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return HF_ERR_UNSUPPORTED;
    hf_server *srv = new hf_server();
    srv->device = device;
    srv->budget = hbm_budget_bytes;
    for (int t = 0; t < n_slots; t++) {
        auto sl = std::make_unique<Slot>();
        if (hf::lane_init(&sl->lane, device, true) != HF_OK) {
            hf::lane_destroy(&sl->lane);
            for (auto &o : srv->slots) hf::lane_destroy(&o->lane);
            delete srv;
            return HF_ERR_DEVICE;
        }
        srv->slots.push_back(std::move(sl));
    }
    for (int t = 0; t < n_slots; t++) srv->workers.emplace_back(&hf_server::worker, srv, t);
    *out = srv;
    return HF_OK;
}

hf_status hf_server_submit(hf_server *srv, const hf_request *req, int64_t *ticket) {
    if (!srv || !req || !ticket) return HF_ERR_INVALID;
    std::lock_guard<std::mutex> lk(srv->mu);
    if (req->n < 0 || (req->n > 0 && (!req->pos || !req->halo_id)) || req->halos_cap < 0 ||
        (req->halos_cap > 0 && !req->halos)) {
        srv->err = "invalid request (n, pos, halo_id, halos / halos_cap)";
        return HF_ERR_INVALID;
    }
    size_t need = 0;
    if (req->n > 0) {
        need = hf::lane_arena_bytes(&req->params, req->n);
        if (need == 0) {
            srv->err = "invalid parameters for this request";
            return HF_ERR_INVALID;
        }
        need += io_bytes_for(*req);
    }
    if (need > srv->budget) {
        srv->err = "request needs " + std::to_string(need) + " bytes, more than the HBM budget";
        return HF_ERR_NOMEM;
    }
    const int64_t id = srv->next_ticket++;
    srv->queue.push_back(Pending{id, *req, srv->now(), need});
    srv->known[id] = true;
    *ticket = id;
    srv->cv_work.notify_all();
    return HF_OK;
}

hf_status hf_server_wait(hf_server *srv, int64_t ticket, hf_result *res) {
    if (!srv || !res) return HF_ERR_INVALID;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (!srv->known.count(ticket)) {
        srv->err = "unknown ticket";
        return HF_ERR_INVALID;
    }
    srv->cv_done.wait(lk, [&] { return srv->done.count(ticket) != 0; });
    *res = srv->done[ticket];
    srv->done.erase(ticket);
    srv->known.erase(ticket);
    return HF_OK;
}

double hf_server_now(const hf_server *srv) { return srv ? srv->now() : 0.0; }

uint64_t hf_server_held_bytes(hf_server *srv) {
    if (!srv) return 0;
    std::lock_guard<std::mutex> lk(srv->mu);
    return srv->held_total();
}

const char *hf_server_last_error(const hf_server *srv) { return srv ? srv->err.c_str() : "no server"; }

void hf_server_destroy(hf_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto &th : srv->workers) th.join();
    for (auto &sl : srv->slots) {
        hf::lane_destroy(&sl->lane);
        if (sl->io) (void)hipFree(sl->io);
    }
    delete srv;
}

}  // extern "C"
