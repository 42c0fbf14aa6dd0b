// Host-side state of one pipeline instance ("lane"): its scratch arena, the
// events that time its stages, the statistics and error text of its last call,
// and, for the lanes of the batched and serving paths, a stream of its own.
// A context owns one lane for its single-box calls and a pool of lanes for
// hf_find_batch; a server owns one lane per slot.
#pragma once

#include <atomic>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "hf_internal.h"

namespace hf {

// Device memory budget shared by the lanes of one context: arenas grow only
// while the bytes held by all of them stay within the limit (0: no limit).
struct Budget {
    uint64_t limit = 0;
    std::atomic<uint64_t> held{0};
    bool take(uint64_t b) {
        uint64_t cur = held.load();
        do {
            if (limit && cur + b > limit) return false;
        } while (!held.compare_exchange_weak(cur, cur + b));
        return true;
    }
    void give(uint64_t b) { held.fetch_sub(b); }
};

struct Lane {
    int device = 0;
    int ncu = 0;                   // compute units of the device (persistent grids)
    bool radius_bins = false;      // R_L1 by radial bins (the owning context's option)
    Budget *budget = nullptr;      // the owning context's, or null (no accounting)
    void *arena = nullptr;
    size_t arena_bytes = 0;
    hipEvent_t ev[10] = {};
    hf_stats stats = {};
    std::string err;
    hipStream_t stream = nullptr;  // owned; null for a context's main lane
    uint32_t *host = nullptr;      // pinned, coherent host words for count read-backs
    hipEvent_t pub = nullptr;      // marks a copy into host whose words are read while later work runs
    void *stage = nullptr;         // pinned staging of the box tables sent to the device, and of
    size_t stage_bytes = 0;        // the per-box results read back (grown for large calls)
};

// One call over several boxes: the boxes' particle ranges in the concatenated
// arrays, their parameters and their halo tables.
struct BoxSet {
    int32_t nbox;
    const int64_t *offsets;       // host [nbox + 1], offsets[0] = 0, non-decreasing
    const hf_params *params;      // host [nbox]
    hf_halo *halos;               // device, or null
    const int64_t *halo_offsets;  // host [nbox + 1] (rows of each box's table), or null
    int32_t first = 0;            // number of box 0 in the caller's numbering (error texts)
    bool named = false;           // name the box in error texts even when there is one
};

// Size of the static scratch region of hf_find_noalloc (per device).
constexpr size_t kScratchBytes = (size_t)256 << 20;

// A caller-given scratch region: the arena is carved from it and nothing is
// allocated (the call fails when the box needs more).
struct FixedArena {
    void *base;
    size_t bytes;
};

// Create the events, the pinned host words (and a non-blocking stream of
// default priority when own_stream).  Returns HF_ERR_DEVICE on failure.
hf_status lane_init(Lane *L, int device, bool own_stream);
// Free the arena (the lane stays usable; the next call allocates again).
void lane_release(Lane *L);
// Release, destroy events, the host words and the owned stream.
void lane_destroy(Lane *L);
// Bytes of arena a call of n particles under p needs (0 if p or n is invalid).
size_t lane_arena_bytes(const hf_params *p, int64_t n);
// The whole pass for one box on stream s (hf_find's contract).
hf_status lane_find(Lane *L, const float *pos, int64_t n, const hf_params *p, float *density,
                    int32_t *l0_id, int32_t *halo_id, hf_halo *halos, int64_t halos_cap,
                    int64_t *n_halos, hipStream_t s, const FixedArena *fx = nullptr);
// The whole pass for all boxes of bs at once on stream s (every stage one
// launch over all boxes): concatenated pos / density / l0_id / halo_id,
// n_halos[nbox] (host) per box.  Returns the first error (text naming the
// box), or HF_ERR_CAPACITY when only halo tables were too small (n_halos then
// holds the needed rows; tables that fit are written).
hf_status lane_find_boxes(Lane *L, const BoxSet &bs, const float *pos, float *density, int32_t *l0_id,
                          int32_t *halo_id, int64_t *n_halos, hipStream_t s);
// Particle and cell totals of a set of boxes and its arena size, or 0 when a
// box's parameters are invalid (for the planning of batches).
size_t boxes_arena_bytes(const BoxSet &bs, int64_t *n_total, int64_t *ncell_total);

}  // namespace hf

namespace hf {
// A tuned setting of hf_find_batch for batches of n_boxes boxes and about
// `total` particles: the number of fused groups and its measured time.
struct TuneEntry {
    int32_t n_boxes;
    int64_t total;
    int32_t groups;
    float ms;
};
}  // namespace hf

struct hf_ctx {
    hf::Budget budget;
    hf::Lane main;
    void *scratch = nullptr;  // device address of the static scratch on main.device
    std::vector<std::unique_ptr<hf::Lane>> pool;  // lanes of hf_find_batch, created on demand
    std::vector<hf::TuneEntry> tuning;            // hf_tune_batch / hf_load_tuning
    bool radius_bins = false;                     // HF_OPT_RADIUS_SEARCH = HF_RADIUS_BINS
};
