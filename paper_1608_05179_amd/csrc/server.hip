// Request server: whole-path solves submitted from host threads, run by
// worker threads (one per stream slot) in arrival order, admitted by device
// footprint against an HBM budget, with a PSF cache of built systems.
//
// Host code only (no kernels): every step of a request runs through the
// library's solve path on the slot's stream.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "ctx_internal.h"

using namespace damas;
using Clock = std::chrono::steady_clock;

namespace {

struct Req {
    uint64_t ticket = 0;
    int32_t M = 0, N = 0, n_bins = 0;
    double x0 = 0, x1 = 0, y0 = 0, y1 = 0, z0 = 0, c = 0;
    std::vector<double> mic, freq, csm;
    std::vector<int32_t> keep_count;
    damas_params params{};
    void *x_map = nullptr;
    int32_t *s_tilde = nullptr;
    uint64_t footprint = 0;
    Clock::time_point t_submit, t_start, t_end;
    int status = DAMAS_OK;
    int cache_hit = 0;
    bool done = false;
    std::string err;
};

struct Slot {
    damas_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    std::thread th;
    Buffer mic, freq, csm, x, st; // device inputs and outputs of the request
    bool busy = false;
    size_t held = 0; // device bytes: workspace + the buffers above
};

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

int grow(Buffer &b, size_t bytes)
{
    if (b.bytes >= bytes)
        return DAMAS_OK;
    if (b.p && hipFree(b.p) != hipSuccess)
        return set_error(DAMAS_EDEVICE, "hipFree of a request buffer");
    b.p = nullptr;
    b.bytes = 0;
    if (hipMalloc(&b.p, std::max(bytes, (size_t)256)) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return set_error(DAMAS_ENOMEM, "cannot allocate %zu bytes for a request", bytes);
    }
    b.bytes = std::max(bytes, (size_t)256);
    return DAMAS_OK;
}

void release(Buffer &b)
{
    if (b.p)
        (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

} // namespace

struct damas_server {
    damas_server_opts o{};
    PsfCache cache;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req *> queue;
    std::unordered_map<uint64_t, Req *> reqs;
    uint64_t next = 1;
    std::vector<Slot> slots;
    bool stop = false;
    uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, merged = 0;
    int running = 0;
    // the slots' sweep gate: their sweep launches run one after another,
    // each with the whole device's cooperative budget, while uploads,
    // system builds and downloads of other slots overlap them
    hipEvent_t sweep_gate = nullptr;
    std::mutex sweep_mu;

    size_t slot_bytes(const Slot &sl) const
    {
        size_t t = sl.ctx ? ctx_bytes(sl.ctx) : 0;
        for (const Buffer *b : {&sl.mic, &sl.freq, &sl.csm, &sl.x, &sl.st})
            t += b->bytes;
        return t;
    }
    size_t held_total() const
    {
        size_t t = 0;
        for (const Slot &sl : slots)
            t += sl.held;
        return t;
    }
    void work(int k);
    int run(Slot &sl, Req *r);
    int run_batch(Slot &sl, const std::vector<Req *> &batch);
};

// A request the batch former may merge: kept counts known on the host.
static bool mergeable(const Req *r)
{
    return r->params.select_mode == DAMAS_SEL_KEEP_ALL ||
           r->params.select_mode == DAMAS_SEL_KEEP_COUNT;
}

// Release an idle slot's device memory (caller holds mu; the slot's
// worker is waiting on it, so nothing of it is in flight).
static void trim_slot(Slot &sl)
{
    (void)ctx_trim(sl.ctx);
    for (Buffer *b : {&sl.mic, &sl.freq, &sl.csm, &sl.x, &sl.st})
        release(*b);
    sl.held = 0;
}

void damas_server::work(int k)
{
    (void)hipSetDevice(o.device);
    Slot &me = slots[k];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        if (stop)
            return;
        if (queue.empty()) {
            cv_work.wait(lk);
            continue;
        }
        // The batch: the front request and, when it can merge, later
        // compatible ones (arrival order) up to max_batch.
        std::vector<size_t> pick{0};
        size_t fp = queue.front()->footprint;
        const size_t budget = o.hbm_budget;
        // Admission: this slot reuses what it holds and the other slots
        // keep theirs; the cache gives up entries, then idle slots release
        // their workspaces, to make room.
        auto fits_fp = [&](size_t need) {
            const size_t mine = std::max(need, me.held), others = held_total() - me.held;
            if (others + mine > budget)
                return false;
            std::lock_guard<std::mutex> ck(cache.mu);
            return cache.shrink_to(budget - others - mine);
        };
        if (!fits_fp(fp)) {
            for (Slot &sl : slots)
                if (&sl != &me && !sl.busy && sl.held > 0)
                    trim_slot(sl);
            if (me.held > fp)
                trim_slot(me);
            if (!fits_fp(fp)) {
                // Wait for a running request to finish and release.
                cv_work.wait(lk);
                continue;
            }
        }
        const Req *head = queue.front();
        if (o.max_batch > 1 && mergeable(head)) {
            for (size_t i = 1; i < queue.size() && (int)pick.size() < o.max_batch; ++i) {
                const Req *q = queue[i];
                if (!mergeable(q) || !merge_compatible(head->params, q->params))
                    continue;
                const size_t more = fp + q->footprint;
                const size_t mine = std::max(more, me.held), others = held_total() - me.held;
                if (others + mine > budget)
                    break;
                fp = more;
                pick.push_back(i);
            }
            if (pick.size() > 1 && !fits_fp(fp)) {
                pick.resize(1);
                fp = head->footprint;
            }
        }
        std::vector<Req *> batch;
        for (size_t i : pick)
            batch.push_back(queue[i]);
        for (size_t j = pick.size(); j-- > 0;)
            queue.erase(queue.begin() + (std::ptrdiff_t)pick[j]);
        me.busy = true;
        running += (int)batch.size();
        me.held = std::max(me.held, fp); // reserve
        const auto t_start = Clock::now();
        for (Req *r : batch)
            r->t_start = t_start;
        lk.unlock();
        const int rc = batch.size() == 1 ? run(me, batch[0]) : run_batch(me, batch);
        const std::string err = rc ? std::string(damas_last_error()) : std::string();
        // A failed request may leave copies from its inputs or into its
        // x_map in flight; they end before it is reported done (its caller
        // may then free x_map, and damas_wait frees the inputs).
        if (rc)
            (void)hipStreamSynchronize(me.stream);
        lk.lock();
        const auto t_end = Clock::now();
        for (Req *r : batch) {
            r->t_end = t_end;
            r->status = rc;
            r->err = err;
            r->done = true;
        }
        me.busy = false;
        me.held = slot_bytes(me);
        running -= (int)batch.size();
        completed += batch.size();
        ++batches;
        if (batch.size() > 1)
            merged += batch.size();
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

// A batch of two or more requests: inputs staged side by side in the
// slot's buffers, one merged solve, each request's results copied back
// from its own slice.
int damas_server::run_batch(Slot &sl, const std::vector<Req *> &batch)
{
    CtxScope scope(sl.ctx); // failures are also the slot context's last error
    size_t n_mic = 0, n_freq = 0, n_csm = 0, n_x = 0;
    for (const Req *r : batch) {
        n_mic += r->mic.size();
        n_freq += r->freq.size();
        n_csm += r->csm.size();
        n_x += (size_t)r->n_bins * r->N * r->N;
    }
    const int prec = batch[0]->params.precision;
    const size_t xs = prec == DAMAS_PREC_FP64 ? sizeof(double) : sizeof(float);
    int rc;
    if ((rc = grow(sl.mic, sizeof(double) * n_mic)) || (rc = grow(sl.freq, sizeof(double) * n_freq)) ||
        (rc = grow(sl.csm, sizeof(double) * n_csm)) || (rc = grow(sl.x, xs * n_x)) ||
        (rc = grow(sl.st, sizeof(int32_t) * n_freq)))
        return rc;
    hipStream_t s = sl.stream;
    std::vector<MergedPart> parts(batch.size());
    size_t om = 0, of = 0, oc = 0;
    for (size_t i = 0; i < batch.size(); ++i) {
        const Req *r = batch[i];
        double *mic = (double *)sl.mic.p + om, *freq = (double *)sl.freq.p + of,
               *csm = (double *)sl.csm.p + oc;
        if (hipMemcpyAsync(mic, r->mic.data(), sizeof(double) * r->mic.size(),
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(freq, r->freq.data(), sizeof(double) * r->freq.size(),
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipMemcpyAsync(csm, r->csm.data(), sizeof(double) * r->csm.size(),
                           hipMemcpyHostToDevice, s) != hipSuccess)
            return set_error(DAMAS_EDEVICE, "upload of a batched request's inputs");
        MergedPart &q = parts[i];
        q.g.M = r->M;
        q.g.mic = mic;
        q.g.N = r->N;
        q.g.x0 = r->x0;
        q.g.x1 = r->x1;
        q.g.y0 = r->y0;
        q.g.y1 = r->y1;
        q.g.z0 = r->z0;
        q.g.c = r->c;
        q.n_bins = r->n_bins;
        q.freq = freq;
        q.csm = csm;
        q.p = r->params;
        q.keep_count = r->keep_count;
        om += r->mic.size();
        of += r->freq.size();
        oc += r->csm.size();
    }
    std::vector<int64_t> bin0, map0;
    if ((rc = solve_merged(sl.ctx, parts, sl.x.p, (int32_t *)sl.st.p, &bin0, &map0, s)))
        return rc;
    for (size_t i = 0; i < batch.size(); ++i) {
        Req *r = batch[i];
        r->cache_hit = 0;
        const size_t nx = (size_t)r->n_bins * r->N * r->N;
        if (hipMemcpyAsync(r->x_map, (char *)sl.x.p + xs * (size_t)map0[i], xs * nx,
                           hipMemcpyDeviceToHost, s) != hipSuccess ||
            (r->s_tilde &&
             hipMemcpyAsync(r->s_tilde, (int32_t *)sl.st.p + bin0[i],
                            sizeof(int32_t) * r->n_bins, hipMemcpyDeviceToHost,
                            s) != hipSuccess))
            return set_error(DAMAS_EDEVICE, "download of a batched request's results");
    }
    return damas_check(sl.ctx, s); // synchronises; reports device faults
}

int damas_server::run(Slot &sl, Req *r)
{
    CtxScope scope(sl.ctx); // failures are also the slot context's last error
    const size_t S = (size_t)r->N * r->N, nb = (size_t)r->n_bins;
    const size_t xs = r->params.precision == DAMAS_PREC_FP64 ? sizeof(double) : sizeof(float);
    int rc;
    if ((rc = grow(sl.mic, sizeof(double) * r->mic.size())) ||
        (rc = grow(sl.freq, sizeof(double) * nb)) ||
        (rc = grow(sl.csm, sizeof(double) * r->csm.size())) || (rc = grow(sl.x, xs * nb * S)) ||
        (rc = grow(sl.st, sizeof(int32_t) * nb)))
        return rc;
    hipStream_t s = sl.stream;
    if (hipMemcpyAsync(sl.mic.p, r->mic.data(), sizeof(double) * r->mic.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(sl.freq.p, r->freq.data(), sizeof(double) * nb, hipMemcpyHostToDevice,
                       s) != hipSuccess ||
        hipMemcpyAsync(sl.csm.p, r->csm.data(), sizeof(double) * r->csm.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        return set_error(DAMAS_EDEVICE, "upload of the request's inputs");
    damas_geometry g;
    g.M = r->M;
    g.mic = (const double *)sl.mic.p;
    g.N = r->N;
    g.x0 = r->x0;
    g.x1 = r->x1;
    g.y0 = r->y0;
    g.y1 = r->y1;
    g.z0 = r->z0;
    g.c = r->c;
    damas_params p = r->params;
    p.batched = 1;
    p.power = nullptr; // a request's params are host memory; its power is not kept
    p.keep_count = r->keep_count.empty() ? nullptr : r->keep_count.data();
    int hit = 0;
    rc = solve_cached(sl.ctx, &g, r->n_bins, (const double *)sl.freq.p,
                      (const double *)sl.csm.p, &p, sl.x.p, (int32_t *)sl.st.p,
                      o.cache_budget > 0 ? &cache : nullptr, &hit, s);
    if (rc)
        return rc;
    r->cache_hit = hit;
    if (hipMemcpyAsync(r->x_map, sl.x.p, xs * nb * S, hipMemcpyDeviceToHost, s) != hipSuccess ||
        (r->s_tilde && hipMemcpyAsync(r->s_tilde, sl.st.p, sizeof(int32_t) * nb,
                                      hipMemcpyDeviceToHost, s) != hipSuccess))
        return set_error(DAMAS_EDEVICE, "download of the request's results");
    return damas_check(sl.ctx, s); // synchronises; reports capacity faults
}

extern "C" int damas_server_create(const damas_server_opts *o, damas_server **out)
{
    if (!o || !out)
        return set_error(DAMAS_EINVAL, "opts and out must be non-NULL");
    if (o->slots < 1 || o->slots > 16)
        return set_error(DAMAS_EINVAL, "slots = %d outside [1, 16]", o->slots);
    if (o->max_queue < 1)
        return set_error(DAMAS_EINVAL, "max_queue must be >= 1");
    if (o->max_batch < 0 || o->max_batch > 4096)
        return set_error(DAMAS_EINVAL, "max_batch = %d outside [0, 4096]", o->max_batch);
    if (o->cache_budget > o->hbm_budget)
        return set_error(DAMAS_EINVAL, "cache_budget exceeds hbm_budget");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || o->device < 0 || o->device >= n)
        return set_error(DAMAS_EINVAL, "device %d unavailable", o->device);
    if (hipSetDevice(o->device) != hipSuccess)
        return set_error(DAMAS_EDEVICE, "hipSetDevice");
    damas_server *srv = new (std::nothrow) damas_server();
    if (!srv)
        return set_error(DAMAS_ENOMEM, "server allocation");
    srv->o = *o;
    srv->cache.budget = o->cache_budget;
    srv->slots.resize(o->slots);
    // The slots' sweeps pass a gate in turn (each waits on the device for
    // the previous ones), so every cooperative grid has the whole device.
    if (hipEventCreateWithFlags(&srv->sweep_gate, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        delete srv;
        return set_error(DAMAS_EDEVICE, "sweep gate event");
    }
    for (Slot &sl : srv->slots) {
        int rc = damas_ctx_create(o->device, &sl.ctx);
        if (rc == DAMAS_OK) {
            sl.ctx->sweep_gate = &srv->sweep_gate;
            sl.ctx->sweep_gate_mu = &srv->sweep_mu;
        }
        if (rc == DAMAS_OK && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
            rc = set_error(DAMAS_EDEVICE, "hipStreamCreate");
        if (rc) {
            for (Slot &t : srv->slots) {
                if (t.ctx)
                    damas_ctx_destroy(t.ctx);
                if (t.stream)
                    (void)hipStreamDestroy(t.stream);
            }
            (void)hipEventDestroy(srv->sweep_gate);
            delete srv;
            return rc;
        }
    }
    for (int k = 0; k < o->slots; ++k)
        srv->slots[k].th = std::thread([srv, k] { srv->work(k); });
    *out = srv;
    return DAMAS_OK;
}

extern "C" void damas_server_destroy(damas_server *srv)
{
    if (!srv)
        return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        for (Req *r : srv->queue) {
            r->status = DAMAS_EBUSY;
            r->err = "server stopped before the request ran";
            r->done = true;
        }
        srv->queue.clear();
    }
    srv->cv_work.notify_all();
    srv->cv_done.notify_all();
    for (Slot &sl : srv->slots)
        if (sl.th.joinable())
            sl.th.join();
    (void)hipSetDevice(srv->o.device);
    (void)hipDeviceSynchronize();
    for (Slot &sl : srv->slots) {
        for (Buffer *b : {&sl.mic, &sl.freq, &sl.csm, &sl.x, &sl.st})
            release(*b);
        damas_ctx_destroy(sl.ctx);
        (void)hipStreamDestroy(sl.stream);
    }
    (void)hipEventDestroy(srv->sweep_gate);
    {
        std::lock_guard<std::mutex> ck(srv->cache.mu);
        srv->cache.clear();
    }
    for (auto &kv : srv->reqs)
        delete kv.second;
    delete srv;
}

extern "C" int damas_submit(damas_server *srv, const damas_request *q, uint64_t *ticket)
{
    if (!srv || !q || !ticket)
        return set_error(DAMAS_EINVAL, "server, request and ticket must be non-NULL");
    if (q->M < 1 || q->M > 128 || q->N < 1 || q->N > 46340 || q->n_bins < 1)
        return set_error(DAMAS_EINVAL, "M, N or n_bins out of range");
    if (!q->mic || !q->freq || !q->csm || !q->x_map)
        return set_error(DAMAS_EINVAL, "mic, freq, csm and x_map must be non-NULL");
    uint64_t fp = 0;
    int rc = damas_query_footprint(q->M, q->N, q->n_bins, &q->params, &fp);
    damas_params pn;
    const damas_params *qp = &q->params;
    if (rc == DAMAS_OK)
        rc = resolve_frac(&q->params, q->N, pn, &qp);
    if (rc)
        return rc;
    if (fp > srv->o.hbm_budget) {
        std::lock_guard<std::mutex> lk(srv->mu);
        ++srv->rejected;
        return set_error(DAMAS_EADMIT, "request needs %llu bytes, the budget is %llu",
                         (unsigned long long)fp, (unsigned long long)srv->o.hbm_budget);
    }
    Req *r = new (std::nothrow) Req();
    if (!r)
        return set_error(DAMAS_ENOMEM, "request allocation");
    r->M = q->M;
    r->N = q->N;
    r->n_bins = q->n_bins;
    r->x0 = q->x0;
    r->x1 = q->x1;
    r->y0 = q->y0;
    r->y1 = q->y1;
    r->z0 = q->z0;
    r->c = q->c;
    r->mic.assign(q->mic, q->mic + 3 * (size_t)q->M);
    r->freq.assign(q->freq, q->freq + q->n_bins);
    r->csm.assign(q->csm, q->csm + (size_t)q->n_bins * q->M * q->M * 2);
    r->params = *qp;
    r->params.power = nullptr;
    if (qp->keep_count)
        r->keep_count.assign(qp->keep_count, qp->keep_count + q->n_bins);
    r->params.keep_count = nullptr;
    r->x_map = q->x_map;
    r->s_tilde = q->s_tilde;
    r->footprint = fp;
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop || (int)srv->queue.size() >= srv->o.max_queue) {
            ++srv->rejected;
            delete r;
            return set_error(DAMAS_EBUSY, "queue full (%d waiting)", (int)srv->queue.size());
        }
        r->ticket = srv->next++;
        srv->reqs[r->ticket] = r;
        srv->queue.push_back(r);
        ++srv->submitted;
        *ticket = r->ticket;
    }
    srv->cv_work.notify_one();
    return DAMAS_OK;
}

extern "C" int damas_wait(damas_server *srv, uint64_t ticket, int32_t timeout_ms,
                          damas_request_info *info)
{
    if (!srv)
        return set_error(DAMAS_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end())
        return set_error(DAMAS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    Req *r = it->second;
    if (timeout_ms < 0)
        srv->cv_done.wait(lk, [r] { return r->done; });
    else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms),
                                    [r] { return r->done; }))
        return set_error(DAMAS_ETIMEDOUT, "request %llu not finished",
                         (unsigned long long)ticket);
    if (info) {
        info->status = r->status;
        info->cache_hit = r->cache_hit;
        const bool ran = r->t_start.time_since_epoch().count() != 0;
        info->queue_ms = ran ? ms_between(r->t_submit, r->t_start) : 0.0;
        info->run_ms = ran ? ms_between(r->t_start, r->t_end) : 0.0;
        info->total_ms = ran ? ms_between(r->t_submit, r->t_end) : 0.0;
    }
    const int st = r->status;
    std::string err = r->err;
    srv->reqs.erase(it);
    delete r;
    lk.unlock();
    if (st)
        return set_error(st, "%s", err.c_str());
    return DAMAS_OK;
}

extern "C" int damas_poll(damas_server *srv, uint64_t ticket)
{
    if (!srv)
        return set_error(DAMAS_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end())
        return set_error(DAMAS_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    return it->second->done ? 1 : 0;
}

extern "C" int damas_server_get_stats(damas_server *srv, damas_server_stats *out)
{
    if (!srv || !out)
        return set_error(DAMAS_EINVAL, "server and out must be non-NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->rejected = srv->rejected;
    out->held_bytes = srv->held_total();
    out->queued = (int32_t)srv->queue.size();
    out->running = srv->running;
    std::lock_guard<std::mutex> ck(srv->cache.mu);
    out->cache_hits = srv->cache.hits;
    out->cache_misses = srv->cache.misses;
    out->cache_bytes = srv->cache.used;
    out->batches = srv->batches;
    out->merged = srv->merged;
    return DAMAS_OK;
}
