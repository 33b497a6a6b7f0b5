// Private to the library: the device workspace of a context, the cache of
// built systems, and the internal solve entry the request server uses.
#pragma once

#include <stdint.h>

#include <list>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "common.h"

namespace damas {

struct Buffer {
    void *p = nullptr;
    size_t bytes = 0;
};

// Device copies of built compressed systems (the A arena of a solve and,
// for DAMAS_PREC_BF16, its FP32 copy), keyed by everything they are a
// function of: geometry, frequencies, precision, and the kept points of
// every bin.  Entries are compared by their whole key, never by hash alone.
// Least recently used entries go first when the byte budget is exceeded.
struct PsfCache {
    struct Entry {
        std::string key;
        Buffer A, A32, Alo, cls; // systems, lo residuals and bin classes
        hipEvent_t ready = nullptr; // recorded after the copies that fill A, A32
        std::list<const std::string *>::iterator lru;
    };
    size_t budget = 0;
    size_t used = 0;
    uint64_t hits = 0, misses = 0;
    std::mutex mu;
    std::unordered_map<std::string, Entry> map;
    std::list<const std::string *> lru; // front: most recently used

    // Free entries (least recent first) until `need` more bytes fit the
    // budget; returns false if they cannot.  Caller holds mu.
    bool make_room(size_t need);
    // Free entries (least recent first) until at most `room` bytes remain
    // cached; returns whether that holds.  Caller holds mu.
    bool shrink_to(size_t room);
    void clear();
};

// Record a failure for damas_last_error() of the calling thread (and for
// damas_ctx_last_error() of the context the thread is working on, see
// CtxScope); returns `code`.
int set_error(int code, const char *fmt, ...);

// The context a thread's library calls are working on while a CtxScope
// lives: failures recorded meanwhile are also kept on that context.
damas_ctx *ctx_scope_swap(damas_ctx *ctx);
struct CtxScope {
    damas_ctx *prev;
    explicit CtxScope(damas_ctx *ctx) : prev(ctx_scope_swap(ctx)) {}
    ~CtxScope() { (void)ctx_scope_swap(prev); }
    CtxScope(const CtxScope &) = delete;
    CtxScope &operator=(const CtxScope &) = delete;
};

// One autotune choice (the cooperative schedule's knobs).
struct TuneKnobs {
    bool coop = true;
    int min_rows = 320;     // rows per rank at least
    double split = 1.25;    // bins above split x the mean work per workgroup get ranks
    double overhead = 1.3;  // cost per element of a rank relative to a bin alone
    int floor_rows = 0;     // cost model: a tile costs max(floor_rows, ld) (0: ld)
    double wide_cost = 1.7; // cost per element of a wide bin relative to a narrow one
};

} // namespace damas

struct damas_ctx {
    int device = 0;
    // Device word the context's kernels set on a device-side capacity
    // violation or a cooperative time-out; read and cleared by damas_check
    // for this context only, so concurrent contexts never see each other's
    // faults.
    int *fault = nullptr;
    damas::Buffer b, idx, st, kc, off, E, A, E16, A32;
    // per-bin precision classes: bf16 residuals of the float arena (same
    // offsets), tile sums of A, one class byte per bin
    damas::Buffer Alo, tsum, cls;
    // merged batches: per bin (map base, grid points), and its staging
    damas::Buffer mapt;
    int64_t *mapt_pinned = nullptr;
    size_t mapt_pinned_n = 0;
    uint8_t *cls_pinned = nullptr; // classes read back for the schedule
    size_t cls_pinned_n = 0;
    // keep counts last uploaded to kc (skip identical re-uploads)
    std::vector<int32_t> kc_host;
    int32_t *kc_pinned = nullptr;
    size_t kc_pinned_n = 0;
    hipEvent_t kc_done = nullptr;
    bool timing = false;
    // cooperative sweeps: workgroup budget (-1: what fits the device, 0:
    // never), exchange workspace, schedule table and its pinned staging
    int coop_budget = -1;
    int last_workgroups = 0; // of the last sweep launch (one per bin alone)
    // schedule knobs of the cooperative sweeps (set by damas_ctx_autotune)
    damas::TuneKnobs tune;
    // options (damas_ctx_create_ex): workspace budget (0: none), autotune
    // cache file and its entries (problem key -> knobs, timed sweep ms),
    // one workgroup per bin
    uint64_t hbm_budget = 0;
    std::string tune_cache;
    std::unordered_map<std::string, std::pair<damas::TuneKnobs, double>> tune_entries;
    bool deterministic = false;
    // last failure of a call made on this context (damas_ctx_last_error)
    mutable std::mutex err_mu;
    std::string err;
    // sweep gate (set by the request server for its slots): every sweep
    // launch of a context with a gate waits on the device for the previous
    // gated sweeps, so one cooperative grid at a time holds the whole chip
    hipEvent_t *sweep_gate = nullptr;
    std::mutex *sweep_gate_mu = nullptr;
    // graph capture: `capturing` marks the captured solve, which makes no
    // host synchronisation and plans no schedule: its sweeps run the
    // schedule the sizing solve before it chose, from the graph's own copy
    // of the table (cap_tab, cap_nwg workgroups, cap_gpw groups per wave),
    // or one workgroup per bin when cap_tab is null; `in_capture` refuses
    // workspace growth inside the captured solve
    bool capturing = false, in_capture = false;
    const int32_t *cap_tab = nullptr;
    int cap_nwg = 0, cap_gpw = 0;
    int graphs = 0;
    // the last sweep launch's schedule: cooperative or not, groups per wave
    bool last_coop = false;
    int last_gpw = 0;
    std::vector<int32_t> coop_tab_host; // last uploaded schedule
    damas::Buffer coop_ws, coop_tab;
    int32_t *coop_pinned = nullptr;
    size_t coop_pinned_n = 0;
    hipEvent_t coop_done = nullptr;
    // recorded (start, end) event pairs per timed phase, and spare pairs
    std::vector<std::pair<hipEvent_t, hipEvent_t>> phase_events[DAMAS_PHASES], event_pool;
};

namespace damas {

// KEEP_FRAC params in their KEEP_COUNT form (*q = &tmp), or p itself (*q =
// p) for the other modes; an invalid keep_frac fails with DAMAS_EINVAL.
int resolve_frac(const damas_params *p, int32_t N, damas_params &tmp, const damas_params **q);

// One request of a merged batch (the request server's batch former): its
// geometry (device mic), bins, device freq and csm, and params (host; the
// kept counts, KEEP_ALL or KEEP_COUNT, in keep_count or keep_count_all).
struct MergedPart {
    damas_geometry g;
    int32_t n_bins = 0;
    const double *freq = nullptr, *csm = nullptr;
    damas_params p{};
    std::vector<int32_t> keep_count;
};
// Whether two requests' sweeps can share one launch: the same precision,
// sweep counts and policy, and kept counts the host knows.
bool merge_compatible(const damas_params &a, const damas_params &b);
// The whole path for several requests on different grids at once: each
// part's DAS map, selection and system build on its own grid, then one
// sweep launch (cooperative job lists over every bin of the batch).  Part
// r's bins are bins bin0[r].. of the batch and its maps start at element
// map0[r] of x_all (n_bins x N^2 each, x of the batch's precision) and of
// st_all (device, one count per bin).  No PSF cache.  Filled bin0/map0 on
// success.
int solve_merged(damas_ctx *ctx, const std::vector<MergedPart> &parts, void *x_all,
                 int32_t *st_all, std::vector<int64_t> *bin0, std::vector<int64_t> *map0,
                 hipStream_t s);
// Host-side sizes of a merged batch: x_all elements and bins.
int merged_sizes(const std::vector<MergedPart> &parts, int64_t *map_elems, int64_t *bins);

// Device bytes a context currently holds, and release of its workspace.
size_t ctx_bytes(const damas_ctx *ctx);
int ctx_trim(damas_ctx *ctx);

// damas_solve_dev (batched) with the system build looked up in `cache`
// first: after the selection the kept sets come to the host (one stream
// synchronisation), and a hit copies the cached systems into the arena in
// place of steering and PSF launches; a miss builds them and stores a copy
// when the cache budget allows.  *hit reports which happened.
int solve_cached(damas_ctx *ctx, const damas_geometry *g, int32_t n_bins, const double *freq,
                 const double *csm, const damas_params *p, void *x_map, int32_t *s_tilde,
                 PsfCache *cache, int *hit, hipStream_t s);

} // namespace damas
