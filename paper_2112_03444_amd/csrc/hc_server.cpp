// hc_server.cpp -- request-serving loop with continuous batching (hc_server_*).
//
// A dispatcher thread turns pending requests into batches and a completion
// thread retires them.  Each of the server's slots owns a context (workspace)
// and a stream, so up to `max_inflight` batches are on the device at once:
// requests that arrive while others are being tracked are admitted into the
// next batch as soon as a slot and enough of the HBM budget are free, and that
// batch overlaps the ones in flight.  A batch is one hc_track_batch_device call
// (persistent work-queue tracker); every path's arithmetic is independent of
// what else is in the batch, so a request's results do not depend on the mix.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>

#include "hc_host.h"

using namespace hcx;
using clk = std::chrono::steady_clock;

namespace {

}  // namespace

// A start set kept on the device for the server's lifetime: requests that name
// it track from these points (and start parameters) without copying them.
struct hc_start_set {
    const hc_system *sys = nullptr;
    int32_t n_start = 0;
    hc_c64 *d_start = nullptr;   // [n_start][n]
    hc_c64 *d_pstart = nullptr;  // [n_params] or null
};

namespace {

struct Request {
    int64_t ticket = 0;
    const hc_system *sys = nullptr;
    const hc_start_set *set = nullptr;  // resident start points, or null (copied below)
    int n = 0, n_params = 0, n_start = 0, n_inst = 0;
    std::vector<hc_c64> start, p_start, p_target, gamma;  // copies made at submission
    hc_c64 *endpoints = nullptr;
    int32_t *status = nullptr;
    hc_track_info *info = nullptr;
    size_t bytes = 0;  // device footprint
    clk::time_point t_submit;
    // placement inside the slot's arena (offsets in bytes)
    size_t o_start = 0, o_pstart = 0, o_ptarget = 0, o_gamma = 0, o_ep = 0, o_st = 0, o_inf = 0;
};

struct Ticket {
    bool done = false;
    hc_status rc = HC_OK;
};

struct PinnedBuf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
        if (e == hipSuccess) cap = bytes;
        return e;
    }
    void release()
    {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
    }
};

struct Slot {
    hc_ctx *ctx = nullptr;
    DevBuf arena;
    PinnedBuf in, out;
    hipEvent_t done = nullptr;
    std::vector<Request *> reqs;
    size_t in_bytes = 0, out_bytes = 0, out_base = 0, bytes = 0;
    hc_status rc = HC_OK;
    bool busy = false;
};

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

struct hc_server {
    hc_ctx *ctx = nullptr;
    hc_server_opts o{};
    std::vector<Slot> slots;
    std::mutex m;
    std::condition_variable cv_dispatch, cv_complete, cv_done;
    std::deque<Request *> pending;
    std::deque<Slot *> inflight;
    std::unordered_map<int64_t, Ticket> tickets;
    int64_t next_ticket = 1;
    bool stop = false;
    size_t bytes_inflight = 0, peak_bytes = 0;
    // statistics
    int64_t submitted = 0, completed = 0, batches = 0, tracks_completed = 0;
    std::vector<double> lat_ms;
    clk::time_point t_stats;
    double busy_s = 0.0;
    std::thread dispatcher, completer;
    std::vector<hc_start_set *> start_sets;
};

namespace {

size_t footprint(const hc_system *s, int n_start, int n_inst, bool with_info, bool resident_start)
{
    const size_t total = (size_t)n_start * n_inst;
    const size_t state = total * (16 * (size_t)s->n + 28);
    const size_t tables = (size_t)(n_inst + 1) * s->n * s->T * 24;
    const size_t io = total * (16 * (size_t)s->n + 4 + (with_info ? 32 : 0)) +
                      ((size_t)n_inst + 1) * (s->n_params + 1) * 16 +
                      (resident_start ? 0 : (size_t)n_start * s->n * 16);
    return state + tables + io + 4096;
}

// Places a batch's inputs and outputs in the slot's arena, uploads the inputs,
// tracks, and downloads the outputs; all on the slot's stream.
hc_status launch_batch(hc_server *sv, Slot &sl)
{
    size_t off = 0;
    for (Request *r : sl.reqs) {
        r->o_ptarget = off;
        off += al(r->p_target.size() * sizeof(hc_c64));
        r->o_gamma = off;
        off += al(r->gamma.size() * sizeof(hc_c64));
        r->o_start = off;
        off += al(r->start.size() * sizeof(hc_c64));
        r->o_pstart = off;
        off += al(r->p_start.size() * sizeof(hc_c64));
    }
    sl.in_bytes = off;
    sl.out_base = off;
    for (Request *r : sl.reqs) {
        const size_t total = (size_t)r->n_start * r->n_inst;
        r->o_ep = off - sl.out_base;
        off += al(total * r->n * sizeof(hc_c64));
        r->o_st = off - sl.out_base;
        off += al(total * sizeof(int32_t));
        r->o_inf = off - sl.out_base;
        off += al(r->info ? total * sizeof(hc_track_info) : 0);
    }
    sl.out_bytes = off - sl.out_base;
    HIP_TRY(sl.arena.ensure(off));
    HIP_TRY(sl.in.ensure(std::max<size_t>(sl.in_bytes, 1)));
    HIP_TRY(sl.out.ensure(std::max<size_t>(sl.out_bytes, 1)));
    char *hin = static_cast<char *>(sl.in.p);
    for (Request *r : sl.reqs) {
        auto put = [&](size_t o, const std::vector<hc_c64> &v) {
            if (!v.empty()) std::memcpy(hin + o, v.data(), v.size() * sizeof(hc_c64));
        };
        put(r->o_ptarget, r->p_target);
        put(r->o_gamma, r->gamma);
        put(r->o_start, r->start);
        put(r->o_pstart, r->p_start);
    }
    hipStream_t st = sl.ctx->own_stream;
    char *dev = static_cast<char *>(sl.arena.p);
    if (sl.in_bytes) HIP_TRY(hipMemcpyAsync(dev, hin, sl.in_bytes, hipMemcpyHostToDevice, st));
    std::vector<hc_job> jobs;
    for (Request *r : sl.reqs) {
        hc_job j;
        j.sys = r->sys;
        j.start = r->set ? r->set->d_start
                         : r->start.empty() ? nullptr : reinterpret_cast<const hc_c64 *>(dev + r->o_start);
        j.n_start = r->n_start;
        j.n_inst = r->n_inst;
        j.p_start = r->set ? r->set->d_pstart
                           : r->p_start.empty() ? nullptr : reinterpret_cast<const hc_c64 *>(dev + r->o_pstart);
        j.p_target = r->p_target.empty() ? nullptr : reinterpret_cast<const hc_c64 *>(dev + r->o_ptarget);
        j.gamma = r->gamma.empty() ? nullptr : reinterpret_cast<const hc_c64 *>(dev + r->o_gamma);
        j.endpoints = reinterpret_cast<hc_c64 *>(dev + sl.out_base + r->o_ep);
        j.status = reinterpret_cast<int32_t *>(dev + sl.out_base + r->o_st);
        j.info = r->info ? reinterpret_cast<hc_track_info *>(dev + sl.out_base + r->o_inf) : nullptr;
        jobs.push_back(j);
    }
    hc_status rc = hc_track_batch_device(sl.ctx, (int32_t)jobs.size(), jobs.data(), &sv->o.opts, st);
    if (rc != HC_OK) return rc;
    if (sl.out_bytes) HIP_TRY(hipMemcpyAsync(sl.out.p, dev + sl.out_base, sl.out_bytes, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(sl.done, st));
    return HC_OK;
}

int request_class(const Request *r) { return 2 * r->sys->layout + (r->sys->kind == HC_PARAMETER ? 1 : 0); }

void dispatch_loop(hc_server *sv)
{
    (void)hipSetDevice(sv->ctx->device);
    std::unique_lock<std::mutex> lk(sv->m);
    for (;;) {
        Slot *free_slot = nullptr;
        std::vector<Request *> batch;
        size_t bytes = 0;
        sv->cv_dispatch.wait(lk, [&]() {
            if (sv->pending.empty()) return sv->stop;
            free_slot = nullptr;
            for (Slot &s : sv->slots)
                if (!s.busy) {
                    free_slot = &s;
                    break;
                }
            if (!free_slot) return false;
            // admit by device footprint: a request that does not fit waits for memory
            // to free up, unless nothing is in flight (it then runs alone)
            const Request *r = sv->pending.front();
            return sv->bytes_inflight == 0 || sv->bytes_inflight + r->bytes <= (size_t)sv->o.hbm_budget;
        });
        if (sv->pending.empty() && sv->stop) break;
        // one batch holds requests of one class (table layout x homotopy kind), so
        // it runs one tracking kernel and batches of different classes overlap on
        // the device; within the class requests go in arrival order
        const int cls = request_class(sv->pending.front());
        for (auto it = sv->pending.begin();
             it != sv->pending.end() && (int)batch.size() < sv->o.max_batch_requests;) {
            Request *r = *it;
            if (request_class(r) != cls) {
                ++it;
                continue;
            }
            if (!batch.empty() && sv->bytes_inflight + bytes + r->bytes > (size_t)sv->o.hbm_budget) break;
            batch.push_back(r);
            bytes += r->bytes;
            it = sv->pending.erase(it);
        }
        Slot &sl = *free_slot;
        sl.busy = true;
        sl.reqs = std::move(batch);
        sl.bytes = bytes;
        sv->bytes_inflight += bytes;
        sv->peak_bytes = std::max(sv->peak_bytes, sv->bytes_inflight);
        sv->batches++;
        lk.unlock();
        sl.rc = launch_batch(sv, sl);
        lk.lock();
        sv->inflight.push_back(&sl);
        sv->cv_complete.notify_one();
    }
    sv->cv_complete.notify_all();
}

void complete_loop(hc_server *sv)
{
    (void)hipSetDevice(sv->ctx->device);
    std::unique_lock<std::mutex> lk(sv->m);
    for (;;) {
        sv->cv_complete.wait(lk, [&]() {
            if (!sv->inflight.empty()) return true;
            if (!sv->stop || !sv->pending.empty()) return false;
            for (Slot &s : sv->slots)
                if (s.busy) return false;
            return true;
        });
        if (sv->inflight.empty()) break;
        // the batch the device finished first (batches of different classes take
        // different times, so completion is not in dispatch order)
        Slot *sl = nullptr;
        std::vector<Slot *> cand(sv->inflight.begin(), sv->inflight.end());
        lk.unlock();
        for (;;) {
            for (Slot *c : cand) {
                if (c->rc != HC_OK) {
                    sl = c;
                    break;
                }
                const hipError_t e = hipEventQuery(c->done);
                if (e == hipSuccess) {
                    sl = c;
                    break;
                }
                if (e != hipErrorNotReady) {
                    c->rc = fail(HC_E_DEVICE, "server: %s", hipGetErrorString(e));
                    sl = c;
                    break;
                }
            }
            if (sl) break;
            std::this_thread::sleep_for(std::chrono::microseconds(20));
            lk.lock();
            cand.assign(sv->inflight.begin(), sv->inflight.end());
            lk.unlock();
        }
        const auto t0 = clk::now();
        if (sl->rc != HC_OK) {
            // whatever the failed launch left on the stream finishes before reuse
            (void)hipStreamSynchronize(sl->ctx->own_stream);
        }
        if (sl->rc == HC_OK) {
            const char *hout = static_cast<const char *>(sl->out.p);
            for (Request *r : sl->reqs) {
                const size_t total = (size_t)r->n_start * r->n_inst;
                std::memcpy(r->endpoints, hout + r->o_ep, total * r->n * sizeof(hc_c64));
                std::memcpy(r->status, hout + r->o_st, total * sizeof(int32_t));
                if (r->info) std::memcpy(r->info, hout + r->o_inf, total * sizeof(hc_track_info));
            }
        }
        const auto t1 = clk::now();
        lk.lock();
        sv->busy_s += std::chrono::duration<double>(t1 - t0).count();
        for (Request *r : sl->reqs) {
            Ticket &tk = sv->tickets[r->ticket];
            tk.done = true;
            tk.rc = sl->rc;
            if (sl->rc == HC_OK) {
                sv->completed++;
                sv->tracks_completed += (int64_t)r->n_start * r->n_inst;
                if (r->t_submit >= sv->t_stats)
                    sv->lat_ms.push_back(std::chrono::duration<double, std::milli>(t1 - r->t_submit).count());
            }
            delete r;
        }
        sl->reqs.clear();
        sv->bytes_inflight -= sl->bytes;
        sl->busy = false;
        sv->inflight.erase(std::find(sv->inflight.begin(), sv->inflight.end(), sl));
        sv->cv_done.notify_all();
        sv->cv_dispatch.notify_all();
    }
}

}  // namespace

extern "C" {

void hc_server_default_opts(hc_server_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->max_inflight = 3;
    o->max_batch_requests = 64;
    o->hbm_budget = (int64_t)8 << 30;
    hc_default_opts(&o->opts);
    o->opts.precision = HC_MIXED;
}

hc_status hc_server_create(hc_ctx *ctx, const hc_server_opts *opts, hc_server **out)
{
    clear_error();
    if (!ctx || !out) return fail(HC_E_INVALID, "hc_server_create: NULL argument");
    hc_server_opts o;
    if (opts) o = *opts;
    else hc_server_default_opts(&o);
    if (o.max_inflight < 1 || o.max_inflight > 16 || o.max_batch_requests < 1 || o.hbm_budget <= 0)
        return fail(HC_E_INVALID, "hc_server_create: max_inflight in [1,16], max_batch_requests >= 1, hbm_budget > 0");
    if (o.opts.steps_per_launch != 0 || o.opts.lanes_per_path == 1 || o.opts.endgame != 0)
        return fail(HC_E_UNSUPPORTED, "hc_server_create: requests run on the batch tracker (steps_per_launch 0, "
                                      "no end-game)");
    hc_server *sv = new (std::nothrow) hc_server;
    if (!sv) return fail(HC_E_OOM, "hc_server_create: out of host memory");
    sv->ctx = ctx;
    sv->o = o;
    sv->slots.resize(o.max_inflight);
    for (Slot &s : sv->slots) {
        hc_status rc = hc_create(ctx->device, &s.ctx);
        hipError_t e = rc == HC_OK ? hipEventCreateWithFlags(&s.done, hipEventDisableTiming) : hipSuccess;
        if (rc != HC_OK || e != hipSuccess) {
            for (Slot &q : sv->slots) {
                if (q.done) (void)hipEventDestroy(q.done);
                if (q.ctx) hc_destroy(q.ctx);
            }
            delete sv;
            return rc != HC_OK ? rc : fail(HC_E_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    sv->t_stats = clk::now();
    sv->dispatcher = std::thread(dispatch_loop, sv);
    sv->completer = std::thread(complete_loop, sv);
    *out = sv;
    return HC_OK;
}

hc_status hc_server_submit(hc_server *sv, const hc_request *rq, int64_t *ticket)
{
    clear_error();
    if (!sv || !rq || !ticket || !rq->sys) return fail(HC_E_INVALID, "hc_server_submit: NULL argument");
    const hc_system *s = rq->sys;
    if (s->device != sv->ctx->device) return fail(HC_E_INVALID, "hc_server_submit: system on another device");
    if (s->n < 2) return fail(HC_E_UNSUPPORTED, "hc_server_submit: n = 1 is not served");
    if (rq->n_start < 0 || rq->n_inst < 0) return fail(HC_E_INVALID, "hc_server_submit: negative size");
    const bool param = s->kind == HC_PARAMETER;
    const hc_start_set *set = rq->start_set;
    if (set) {
        bool known;
        {
            std::lock_guard<std::mutex> lk(sv->m);
            known = std::find(sv->start_sets.begin(), sv->start_sets.end(), set) != sv->start_sets.end();
        }
        if (!known) return fail(HC_E_INVALID, "hc_server_submit: start_set was not added to this server");
        if (set->sys != s) return fail(HC_E_INVALID, "hc_server_submit: start_set belongs to another system");
        if (rq->start || rq->p_start || rq->n_start != set->n_start)
            return fail(HC_E_INVALID, "hc_server_submit: with start_set, start and p_start are NULL and n_start is "
                                      "the set's (%d)", set->n_start);
    }
    const size_t total = (size_t)rq->n_start * rq->n_inst;
    if (total > 0) {
        if (!rq->endpoints || !rq->status || (!rq->p_target && s->n_params > 0))
            return fail(HC_E_INVALID, "hc_server_submit: NULL buffer");
        if (!param && !rq->start && !set && rq->n_start > s->bezout)
            return fail(HC_E_INVALID, "hc_server_submit: n_start exceeds the Bezout number");
        if (param && !set && (!rq->start || (!rq->p_start && s->n_params > 0)))
            return fail(HC_E_INVALID, "hc_server_submit: a parameter homotopy needs start points and p_start");
    }
    Request *r = new (std::nothrow) Request;
    if (!r) return fail(HC_E_OOM, "hc_server_submit: out of host memory");
    r->sys = s;
    r->set = set;
    r->n = s->n;
    r->n_params = s->n_params;
    r->n_start = rq->n_start;
    r->n_inst = rq->n_inst;
    if (rq->p_target) r->p_target.assign(rq->p_target, rq->p_target + (size_t)rq->n_inst * s->n_params);
    if (rq->gamma) r->gamma.assign(rq->gamma, rq->gamma + rq->n_inst);
    if (rq->start) r->start.assign(rq->start, rq->start + (size_t)rq->n_start * s->n);
    if (rq->p_start) r->p_start.assign(rq->p_start, rq->p_start + s->n_params);
    r->endpoints = rq->endpoints;
    r->status = rq->status;
    r->info = rq->info;
    r->bytes = footprint(s, rq->n_start, rq->n_inst, rq->info != nullptr, set != nullptr);
    r->t_submit = clk::now();
    {
        std::lock_guard<std::mutex> lk(sv->m);
        if (sv->stop) {
            delete r;
            return fail(HC_E_INVALID, "hc_server_submit: server is shutting down");
        }
        r->ticket = sv->next_ticket++;
        sv->tickets[r->ticket] = Ticket{};
        *ticket = r->ticket;
        sv->submitted++;
        if (total == 0) {
            sv->tickets[r->ticket].done = true;
            sv->completed++;
            delete r;
            return HC_OK;
        }
        sv->pending.push_back(r);
    }
    sv->cv_dispatch.notify_one();
    return HC_OK;
}

hc_status hc_server_add_start_set(hc_server *sv, const hc_system *sys, const hc_c64 *start, int32_t n_start,
                                  const hc_c64 *p_start, const hc_start_set **out)
{
    clear_error();
    if (!sv || !sys || !out || !start || n_start < 1) return fail(HC_E_INVALID, "hc_server_add_start_set: bad argument");
    if (sys->device != sv->ctx->device) return fail(HC_E_INVALID, "hc_server_add_start_set: system on another device");
    if (sys->kind == HC_PARAMETER && sys->n_params > 0 && !p_start)
        return fail(HC_E_INVALID, "hc_server_add_start_set: a parameter homotopy needs p_start");
    hc_start_set *set = new (std::nothrow) hc_start_set;
    if (!set) return fail(HC_E_OOM, "hc_server_add_start_set: out of host memory");
    set->sys = sys;
    set->n_start = n_start;
    const size_t bs = (size_t)n_start * sys->n * sizeof(hc_c64);
    const size_t bp = p_start ? (size_t)sys->n_params * sizeof(hc_c64) : 0;
    hipError_t e = hipSetDevice(sv->ctx->device);
    if (e == hipSuccess) e = hipMalloc(&set->d_start, bs);
    if (e == hipSuccess) e = hipMemcpy(set->d_start, start, bs, hipMemcpyHostToDevice);
    if (e == hipSuccess && bp) e = hipMalloc(&set->d_pstart, bp);
    if (e == hipSuccess && bp) e = hipMemcpy(set->d_pstart, p_start, bp, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(set->d_start);
        (void)hipFree(set->d_pstart);
        delete set;
        return fail(e == hipErrorOutOfMemory ? HC_E_OOM : HC_E_DEVICE, "hc_server_add_start_set: %s",
                    hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> lk(sv->m);
        sv->start_sets.push_back(set);
    }
    *out = set;
    return HC_OK;
}

hc_status hc_server_poll(hc_server *sv, int64_t ticket, int32_t *done)
{
    clear_error();
    if (!sv || !done) return fail(HC_E_INVALID, "hc_server_poll: NULL argument");
    std::lock_guard<std::mutex> lk(sv->m);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(HC_E_INVALID, "hc_server_poll: unknown ticket %lld", (long long)ticket);
    *done = it->second.done ? 1 : 0;
    return it->second.done ? it->second.rc : HC_OK;
}

hc_status hc_server_wait(hc_server *sv, int64_t ticket)
{
    clear_error();
    if (!sv) return fail(HC_E_INVALID, "hc_server_wait: NULL server");
    std::unique_lock<std::mutex> lk(sv->m);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return fail(HC_E_INVALID, "hc_server_wait: unknown ticket %lld", (long long)ticket);
    sv->cv_done.wait(lk, [&]() { return sv->tickets[ticket].done; });
    const hc_status rc = sv->tickets[ticket].rc;
    sv->tickets.erase(ticket);
    if (rc != HC_OK) return fail(rc, "hc_server_wait: the batch holding ticket %lld failed", (long long)ticket);
    return HC_OK;
}

hc_status hc_server_get_stats(hc_server *sv, hc_server_stats *out)
{
    clear_error();
    if (!sv || !out) return fail(HC_E_INVALID, "hc_server_get_stats: NULL argument");
    std::lock_guard<std::mutex> lk(sv->m);
    std::memset(out, 0, sizeof *out);
    out->submitted = sv->submitted;
    out->completed = sv->completed;
    out->batches = sv->batches;
    out->tracks_completed = sv->tracks_completed;
    out->peak_bytes = (int64_t)sv->peak_bytes;
    out->wall_s = std::chrono::duration<double>(clk::now() - sv->t_stats).count();
    std::vector<double> v = sv->lat_ms;
    out->latencies = (int64_t)v.size();
    if (!v.empty()) {
        std::sort(v.begin(), v.end());
        auto q = [&](double f) { return v[std::min(v.size() - 1, (size_t)(f * (v.size() - 1) + 0.5))]; };
        double sum = 0.0;
        for (double x : v) sum += x;
        out->mean_ms = sum / v.size();
        out->p50_ms = q(0.50);
        out->p99_ms = q(0.99);
        out->max_ms = v.back();
    }
    return HC_OK;
}

hc_status hc_server_reset_stats(hc_server *sv)
{
    clear_error();
    if (!sv) return fail(HC_E_INVALID, "hc_server_reset_stats: NULL server");
    std::lock_guard<std::mutex> lk(sv->m);
    sv->submitted = sv->completed = sv->batches = sv->tracks_completed = 0;
    sv->lat_ms.clear();
    sv->peak_bytes = sv->bytes_inflight;
    sv->t_stats = clk::now();
    return HC_OK;
}

hc_status hc_server_destroy(hc_server *sv)
{
    clear_error();
    if (!sv) return HC_OK;
    {
        std::lock_guard<std::mutex> lk(sv->m);
        sv->stop = true;
    }
    sv->cv_dispatch.notify_all();
    sv->cv_complete.notify_all();
    if (sv->dispatcher.joinable()) sv->dispatcher.join();
    sv->cv_complete.notify_all();
    if (sv->completer.joinable()) sv->completer.join();
    for (Slot &s : sv->slots) {
        if (s.done) (void)hipEventDestroy(s.done);
        s.arena.release();
        s.in.release();
        s.out.release();
        if (s.ctx) hc_destroy(s.ctx);
    }
    for (hc_start_set *set : sv->start_sets) {
        (void)hipFree(set->d_start);
        (void)hipFree(set->d_pstart);
        delete set;
    }
    delete sv;
    return HC_OK;
}

}  // extern "C"
