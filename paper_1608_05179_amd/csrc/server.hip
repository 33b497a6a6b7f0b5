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
    uint64_t submitted = 0, completed = 0, rejected = 0;
    int running = 0;

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
};

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
        Req *r = queue.front();
        // Admission: this slot reuses what it holds and the other slots
        // keep theirs; the cache gives up entries, then idle slots release
        // their workspaces, to make room.
        const size_t budget = o.hbm_budget, fp = r->footprint;
        auto fits = [&] {
            const size_t mine = std::max(fp, me.held), others = held_total() - me.held;
            if (others + mine > budget)
                return false;
            std::lock_guard<std::mutex> ck(cache.mu);
            return cache.shrink_to(budget - others - mine);
        };
        if (!fits()) {
            for (Slot &sl : slots)
                if (&sl != &me && !sl.busy && sl.held > 0)
                    trim_slot(sl);
            if (me.held > fp)
                trim_slot(me);
            if (!fits()) {
                // Wait for a running request to finish and release.
                cv_work.wait(lk);
                continue;
            }
        }
        queue.pop_front();
        me.busy = true;
        ++running;
        me.held = std::max(me.held, (size_t)r->footprint); // reserve
        r->t_start = Clock::now();
        lk.unlock();
        const int rc = run(me, r);
        lk.lock();
        r->t_end = Clock::now();
        r->status = rc;
        if (rc)
            r->err = damas_last_error();
        r->done = true;
        me.busy = false;
        me.held = slot_bytes(me);
        --running;
        ++completed;
        cv_done.notify_all();
        cv_work.notify_all();
    }
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
    // Cooperative sweeps of concurrent requests share the device: each slot
    // launches at most its share of the compute units, so every launched
    // workgroup can be resident at once.
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, o->device);
    for (Slot &sl : srv->slots) {
        int rc = damas_ctx_create(o->device, &sl.ctx);
        if (rc == DAMAS_OK)
            rc = damas_ctx_set_coop(sl.ctx, cus / o->slots);
        if (rc == DAMAS_OK && hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess)
            rc = set_error(DAMAS_EDEVICE, "hipStreamCreate");
        if (rc) {
            for (Slot &t : srv->slots) {
                if (t.ctx)
                    damas_ctx_destroy(t.ctx);
                if (t.stream)
                    (void)hipStreamDestroy(t.stream);
            }
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
    return DAMAS_OK;
}
