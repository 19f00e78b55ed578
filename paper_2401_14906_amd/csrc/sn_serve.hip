// Request server of libsn.so: continuous batching of contour requests.
//
// Submitted requests wait in a FIFO queue.  Each of n_streams worker threads
// owns one HIP stream; when a worker is free it admits queued requests in
// order while (a) the device bytes reserved for everything in flight stay
// within the budget and (b) fewer than max_inflight requests are in flight,
// fuses the admitted requests into one batch (one counting launch, one
// generation launch, one HIP-graph replay of the sweeps for the whole batch)
// and runs it on its stream.  Requests arriving meanwhile join the next batch
// of whichever worker frees first, so device work of different batches
// overlaps.  Finished meshes stay device-resident until claimed.
//
// Admission is in two phases, because a mesh's size is known only once its
// volume is counted (Sec. 2.3: the prefix sum sizes the outputs exactly).
//   1. A request is admitted with its exact extraction scratch plus an
//      estimate of its mesh (a running bytes-per-voxel figure of finished
//      requests, or the exact figure if it was counted before).
//   2. Between the count pass and the allocation of the outputs the batch's
//      exact mesh bytes replace the estimate.  If they do not fit the budget
//      next to what else is in flight, the batch waits for memory to be
//      released; if every other batch in flight is waiting the same way, or
//      there is no other, the batch steps back instead: its requests go back
//      to the head of the queue with their exact sizes and its reservation
//      is released, so that phase 1 admits again only what fits.
// A single request that alone exceeds the budget runs when nothing else is in
// flight; reservations otherwise never exceed the budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>

#include <atomic>
#include <unordered_map>
#include <vector>

#include "sn.h"
#include "sn_runtime.h"

using namespace sn;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t ticket = 0;
    sn_volume vol{};
    std::vector<uint32_t> selected;
    sn_smooth_params p{};
    int64_t scratch = 0;      // extraction scratch bytes (exact)
    int64_t mesh_exact = -1;  // exact mesh bytes once counted (kept if queued again)
    int64_t footprint = 0;    // bytes reserved while in flight
    hipEvent_t ready = nullptr;  // recorded on the submitter's stream: the labels are written
    Clock::time_point t_submit, t_done;
    bool done = false;
    sn_status status = SN_OK;
    std::string err;  // the worker's message when the request failed
    sn_mesh *mesh = nullptr;
};

int64_t voxels_of(const sn_volume &v) { return v.dims[0] * v.dims[1] * v.dims[2]; }

// Worker threads spin this long for new work before sleeping, and poll their
// stream for this long before blocking on it.
constexpr int64_t kSpinUs = 200;

hipError_t wait_stream(hipStream_t s)
{
    const auto until = Clock::now() + std::chrono::microseconds(kSpinUs);
    while (Clock::now() < until) {
        const hipError_t e = hipStreamQuery(s);
        if (e != hipErrorNotReady) return e;
        std::this_thread::yield();
    }
    return hipStreamSynchronize(s);
}

}  // namespace

struct sn_server {
    sn_ctx *ctx = nullptr;
    sn_serve_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done, cv_mem;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> reqs;
    uint64_t next_ticket = 1;
    int64_t reserved = 0, peak_reserved = 0;
    int32_t inflight = 0;          // requests admitted and not finished
    int32_t batches_inflight = 0;  // their batches
    int32_t mem_waiting = 0;       // batches waiting in phase 2 for memory
    bool stopping = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    // statistics
    int64_t n_submitted = 0, n_done = 0, n_rejected = 0, n_batches = 0;
    int64_t n_split = 0, n_requeued = 0;
    int64_t voxels_done = 0, point_iters_done = 0;
    std::vector<double> lat_us;
    double mesh_bpv = 16.0;  // running estimate of mesh bytes per voxel
    Clock::time_point busy_since;
    double busy_s = 0.0;
    int32_t busy_count = 0;

    std::atomic<int64_t> queued{0};  // queue length, read without the lock by spinning workers

    // phase-1 reservation of a queued request
    int64_t phase1_locked(const Request *r) const
    {
        const int64_t mesh = r->mesh_exact >= 0 ? r->mesh_exact
                                                : (int64_t)(mesh_bpv * (double)voxels_of(r->vol));
        return r->scratch + mesh;
    }
    // phase 2 for the requests b[0..n): exact mesh bytes from the totals;
    // SN_OK to go on, SN_EAGAIN when the batch steps back
    sn_status phase2(Request *const *b, int32_t n, const int64_t *totals);
    void worker(int w);
    // extract + smooth n requests as one fused batch on stream s and wait for
    // it; on failure every ms[k] is null
    sn_status run_fused(Request *const *b, const sn_volume *vols, const sn_smooth_params *ps,
                        int32_t n, hipStream_t s, sn_mesh **ms);
    void finish_locked(Request *r, sn_status st, sn_mesh *m, Clock::time_point now);
};

sn_status sn_server::phase2(Request *const *b, int32_t n, const int64_t *totals)
{
    std::vector<int64_t> exact(n);
    int64_t delta = 0;
    for (int32_t k = 0; k < n; ++k) {
        const Request *r = b[k];
        exact[k] = mesh_bytes(r->vol, totals[3 * k], totals[3 * k + 1], totals[3 * k + 2],
                              r->p.iterations > 0);
        delta += r->scratch + exact[k] - r->footprint;
    }
    std::unique_lock<std::mutex> lk(mu);
    while (true) {
        // nothing else in flight: a single request runs whatever its size;
        // a batch of several that does not fit steps back (below) and is
        // admitted again on its exact sizes, as a prefix that fits
        const bool alone = batches_inflight == 1 && n == 1;
        if (delta <= 0 || reserved + delta <= cfg.hbm_budget_bytes || alone) {
            reserved += delta;
            peak_reserved = std::max(peak_reserved, reserved);
            for (int32_t k = 0; k < n; ++k) {
                b[k]->mesh_exact = exact[k];
                b[k]->footprint = b[k]->scratch + exact[k];
            }
            if (delta < 0) cv_mem.notify_all(), cv_work.notify_all();
            return SN_OK;
        }
        if (mem_waiting + 1 >= batches_inflight) {
            // every other batch in flight waits here as well (or there is no
            // other): nothing will be released, so this one steps back
            for (int32_t k = 0; k < n; ++k) b[k]->mesh_exact = exact[k];
            return SN_EAGAIN;
        }
        ++mem_waiting;
        cv_mem.wait(lk);
        --mem_waiting;
    }
}

sn_status sn_server::run_fused(Request *const *b, const sn_volume *vols, const sn_smooth_params *ps,
                               int32_t n, hipStream_t s, sn_mesh **ms)
{
    std::fill(ms, ms + n, nullptr);
    const AdmitFn admit = [&](const int64_t *totals) { return phase2(b, n, totals); };
    sn_status st = extract_many(ctx, vols, n, s, nullptr, ms, &admit);
    if (st == SN_OK) {
        // a batch of one takes the plain path (no descriptor upload, no graph build)
        st = n == 1 ? smooth_one(ctx, ms[0], ps, s) : smooth_many(ctx, ms, ps, n, s);
        if (st == SN_OK && wait_stream(s) != hipSuccess) st = SN_EDEVICE;
        if (st != SN_OK) {
            for (int32_t k = 0; k < n; ++k) mesh_release(ms[k]);
            std::fill(ms, ms + n, nullptr);
        }
    }
    return st;
}

void sn_server::finish_locked(Request *r, sn_status st, sn_mesh *m, Clock::time_point now)
{
    r->done = true;
    r->status = st;
    r->mesh = m;
    r->t_done = now;
    if (r->ready) {
        // the worker's stream waited for it and has completed since
        (void)hipEventSynchronize(r->ready);
        ctx->sync_events.put(r->ready);
        r->ready = nullptr;
    }
    if (st == SN_OK) {
        ++n_done;
        const int64_t vox = voxels_of(r->vol);
        voxels_done += vox;
        point_iters_done += m->P * (int64_t)r->p.iterations;
        lat_us.push_back(std::chrono::duration<double, std::micro>(now - r->t_submit).count());
        const int64_t mb = mesh_bytes(r->vol, m->P, m->Q, m->S, r->p.iterations > 0);
        mesh_bpv = 0.9 * mesh_bpv + 0.1 * std::max(1.0, (double)mb / (double)std::max<int64_t>(vox, 1));
    } else {
        ++n_rejected;
    }
}

void sn_server::worker(int w)
{
    (void)hipSetDevice(ctx->device);
    hipStream_t s = streams[w];
    while (true) {
        std::vector<Request *> batch;
        // a request arriving shortly after the last one is picked up without
        // a sleep/wake round trip
        const auto spin_until = Clock::now() + std::chrono::microseconds(kSpinUs);
        while (queued.load(std::memory_order_acquire) == 0 && Clock::now() < spin_until)
            std::this_thread::yield();
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                if (stopping && queue.empty()) return true;
                if (queue.empty() || inflight >= cfg.max_inflight) return false;
                // the head must fit next to what is in flight (or run alone)
                return reserved + phase1_locked(queue.front()) <= cfg.hbm_budget_bytes || inflight == 0;
            });
            if (queue.empty() && stopping) return;
            while (!queue.empty() && (int32_t)batch.size() < cfg.max_batch &&
                   inflight < cfg.max_inflight) {
                Request *h = queue.front();
                const int64_t fp = phase1_locked(h);
                const bool fits = reserved + fp <= cfg.hbm_budget_bytes;
                if (!fits && !(batch.empty() && inflight == 0)) break;
                queue.pop_front();
                queued.fetch_sub(1, std::memory_order_release);
                h->footprint = fp;
                reserved += fp;
                ++inflight;
                batch.push_back(h);
            }
            if (batch.empty()) continue;
            peak_reserved = std::max(peak_reserved, reserved);
            if (busy_count++ == 0) busy_since = Clock::now();
            ++n_batches;
            ++batches_inflight;
        }
        const int32_t n = (int32_t)batch.size();
        std::vector<sn_volume> vols(n);
        std::vector<sn_smooth_params> ps(n);
        for (int32_t k = 0; k < n; ++k) {
            vols[k] = batch[k]->vol;
            vols[k].selected = batch[k]->selected.empty() ? nullptr : batch[k]->selected.data();
            ps[k] = batch[k]->p;
            // the labels are read only after the submitter's work on them
            if (batch[k]->ready && hipStreamWaitEvent(s, batch[k]->ready, 0) != hipSuccess) {
                (void)hipGetLastError();
                (void)hipEventSynchronize(batch[k]->ready);
            }
        }
        std::vector<sn_mesh *> ms(n, nullptr);
        std::vector<sn_status> sts(n, SN_OK);
        std::vector<std::string> errs(n);
        const sn_status st = run_fused(batch.data(), vols.data(), ps.data(), n, s, ms.data());
        bool split = false;
        if (st == SN_ENOMEM && n > 1) {
            // the fused batch did not fit in device memory next to what the
            // other streams hold: run its requests one at a time instead of
            // failing all of them
            split = true;
            for (int32_t k = 0; k < n; ++k) {
                sts[k] = run_fused(&batch[k], &vols[k], &ps[k], 1, s, &ms[k]);
                if (sts[k] != SN_OK && sts[k] != SN_EAGAIN) errs[k] = sn_last_error();
            }
        } else {
            std::fill(sts.begin(), sts.end(), st);
            if (st != SN_OK && st != SN_EAGAIN) std::fill(errs.begin(), errs.end(), sn_last_error());
        }
        const auto now = Clock::now();
        {
            std::lock_guard<std::mutex> lk(mu);
            n_split += split ? 1 : 0;
            std::vector<Request *> back;  // stepped back in phase 2: queued again
            for (int32_t k = 0; k < n; ++k) {
                Request *r = batch[k];
                reserved -= r->footprint;
                r->footprint = 0;
                --inflight;
                if (sts[k] == SN_EAGAIN) {
                    back.push_back(r);
                } else {
                    r->err = std::move(errs[k]);
                    finish_locked(r, sts[k], ms[k], now);
                }
            }
            for (auto it = back.rbegin(); it != back.rend(); ++it) queue.push_front(*it);
            queued.fetch_add((int64_t)back.size(), std::memory_order_release);
            n_requeued += (int64_t)back.size();
            --batches_inflight;
            if (--busy_count == 0)
                busy_s += std::chrono::duration<double>(now - busy_since).count();
        }
        cv_done.notify_all();
        cv_work.notify_all();
        cv_mem.notify_all();
    }
}

extern "C" sn_status sn_serve_start(sn_ctx *ctx, const sn_serve_config *cfg, sn_server **out)
{
    if (!ctx || !cfg || !out) return fail(SN_EINVAL, "sn_serve_start: NULL argument");
    if (cfg->hbm_budget_bytes <= 0 || cfg->max_inflight < 1 || cfg->n_streams < 1 ||
        cfg->max_batch < 1 || cfg->queue_capacity < 1 || cfg->n_streams > 16)
        return fail(SN_EINVAL, "sn_serve_start: bad configuration");
    HIP_TRY(hipSetDevice(ctx->device));
    sn_server *srv = new sn_server();
    srv->ctx = ctx;
    ctx_retain(ctx);
    srv->cfg = *cfg;
    for (int w = 0; w < cfg->n_streams; ++w) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (auto x : srv->streams) (void)hipStreamDestroy(x);
            delete srv;
            ctx_release(ctx);
            return fail(SN_EDEVICE, "sn_serve_start: stream creation failed");
        }
        srv->streams.push_back(s);
    }
    for (int w = 0; w < cfg->n_streams; ++w) srv->workers.emplace_back([srv, w] { srv->worker(w); });
    *out = srv;
    return SN_OK;
}

extern "C" sn_status sn_serve_submit(sn_server *srv, const sn_volume *vol, const sn_smooth_params *p,
                                     void *stream, uint64_t *ticket)
{
    if (!srv || !vol || !p || !ticket) return fail(SN_EINVAL, "sn_serve_submit: NULL argument");
    sn_status st = validate_volume(vol);
    if (st != SN_OK) return st;
    st = validate_smooth(p);
    if (st != SN_OK) return st;
    HIP_TRY(hipSetDevice(srv->ctx->device));
    Request *r = new Request();
    r->vol = *vol;
    if (vol->n_selected > 0) r->selected.assign(vol->selected, vol->selected + vol->n_selected);
    r->vol.selected = nullptr;
    r->p = *p;
    r->scratch = extract_scratch_bytes(r->vol);
    // the worker's stream waits for what the submitter's stream has enqueued
    // so far (the labels may still be being written there)
    r->ready = srv->ctx->sync_events.get();
    if (!r->ready || hipEventRecord(r->ready, static_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipGetLastError();
        srv->ctx->sync_events.put(r->ready);
        delete r;
        return fail(SN_EDEVICE, "sn_serve_submit: cannot record the submitter's stream");
    }
    r->t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stopping || (int32_t)srv->queue.size() >= srv->cfg.queue_capacity) {
            const bool stop = srv->stopping;
            (void)hipEventSynchronize(r->ready);
            srv->ctx->sync_events.put(r->ready);
            delete r;
            return stop ? fail(SN_ESHUTDOWN, "sn_serve_submit: server stopping")
                        : fail(SN_EAGAIN, "sn_serve_submit: queue full");
        }
        r->ticket = srv->next_ticket++;
        srv->reqs[r->ticket] = r;
        srv->queue.push_back(r);
        srv->queued.fetch_add(1, std::memory_order_release);
        ++srv->n_submitted;
        *ticket = r->ticket;
    }
    srv->cv_work.notify_one();
    return SN_OK;
}

static sn_status claim_locked(sn_server *srv, std::unordered_map<uint64_t, Request *>::iterator it,
                              sn_mesh **out)
{
    Request *r = it->second;
    sn_status st = r->status;
    if (st == SN_OK) {
        if (out)
            *out = r->mesh;
        else
            mesh_release(r->mesh);
    }
    const std::string err = std::move(r->err);
    srv->reqs.erase(it);
    delete r;
    return st == SN_OK ? SN_OK : fail(st, "serve: request failed: " + err);
}

extern "C" sn_status sn_serve_poll(sn_server *srv, uint64_t ticket, sn_mesh **out)
{
    if (!srv) return fail(SN_EINVAL, "sn_serve_poll: NULL server");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(SN_ENOTFOUND, "sn_serve_poll: unknown ticket");
    if (!it->second->done) return SN_EAGAIN;
    return claim_locked(srv, it, out);
}

extern "C" sn_status sn_serve_wait(sn_server *srv, uint64_t ticket, int64_t timeout_us,
                                   sn_mesh **out)
{
    if (!srv) return fail(SN_EINVAL, "sn_serve_wait: NULL server");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto ready = [&] {
        auto it = srv->reqs.find(ticket);
        return it == srv->reqs.end() || it->second->done;
    };
    if (timeout_us < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return fail(SN_ETIMEDOUT, "sn_serve_wait: timed out");
    }
    auto it = srv->reqs.find(ticket);
    if (it == srv->reqs.end()) return fail(SN_ENOTFOUND, "sn_serve_wait: unknown ticket");
    return claim_locked(srv, it, out);
}

static double percentile(std::vector<double> v, double q)
{
    if (v.empty()) return 0.0;
    std::sort(v.begin(), v.end());
    const double pos = q * (double)(v.size() - 1);
    const size_t lo = (size_t)pos;
    const size_t hi = std::min(lo + 1, v.size() - 1);
    return v[lo] + (pos - (double)lo) * (v[hi] - v[lo]);
}

extern "C" sn_status sn_serve_stats_get(sn_server *srv, sn_serve_stats *out)
{
    if (!srv || !out) return fail(SN_EINVAL, "sn_serve_stats_get: NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    sn_serve_stats s;
    std::memset(&s, 0, sizeof s);
    s.n_submitted = srv->n_submitted, s.n_done = srv->n_done, s.n_rejected = srv->n_rejected;
    s.n_batches = srv->n_batches;
    s.voxels_done = srv->voxels_done, s.point_iters_done = srv->point_iters_done;
    s.p50_us = percentile(srv->lat_us, 0.50);
    s.p99_us = percentile(srv->lat_us, 0.99);
    double sum = 0;
    for (double x : srv->lat_us) sum += x;
    s.mean_us = srv->lat_us.empty() ? 0.0 : sum / (double)srv->lat_us.size();
    s.busy_s = srv->busy_s + (srv->busy_count > 0
                                  ? std::chrono::duration<double>(Clock::now() - srv->busy_since).count()
                                  : 0.0);
    s.peak_reserved_bytes = srv->peak_reserved;
    s.n_split_batches = srv->n_split;
    s.n_requeued = srv->n_requeued;
    *out = s;
    return SN_OK;
}

extern "C" sn_status sn_serve_stop(sn_server *srv)
{
    if (!srv) return fail(SN_EINVAL, "sn_serve_stop: NULL server");
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stopping = true;
        // queued requests that never started are rejected; in-flight ones finish
        while (!srv->queue.empty()) {
            Request *r = srv->queue.front();
            srv->queue.pop_front();
            srv->queued.fetch_sub(1, std::memory_order_release);
            r->done = true;
            r->status = SN_ESHUTDOWN;
            if (r->ready) {
                (void)hipEventSynchronize(r->ready);
                srv->ctx->sync_events.put(r->ready);
                r->ready = nullptr;
            }
            ++srv->n_rejected;
        }
    }
    srv->cv_work.notify_all();
    srv->cv_done.notify_all();
    srv->cv_mem.notify_all();
    for (auto &t : srv->workers) t.join();
    (void)hipSetDevice(srv->ctx->device);
    for (auto s : srv->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (auto &kv : srv->reqs) {
        if (kv.second->mesh) mesh_release(kv.second->mesh);
        delete kv.second;
    }
    sn_ctx *ctx = srv->ctx;
    delete srv;
    ctx_release(ctx);
    return SN_OK;
}
