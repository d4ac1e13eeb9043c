// libpa server: continuous hashing of a stream of requests on one GPU.
//
// Requests are admitted in arrival order as soon as a slot is free and their
// device footprint (spectra, carry state and, for host requests, the key and
// output buffers) fits in a fixed HBM budget; each admitted request runs on its
// slot's stream, so requests that arrive while others are on the GPU start at
// once and their kernels overlap on the device.  Budget memory is one
// allocation made at creation and handed out first-fit, so admission never
// calls hipMalloc.  The twiddle tables live on the device for the server's
// lifetime (its own context).  A scheduler thread drives everything; callers
// only touch a mutex-protected queue.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "arena.h"
#include "context.h"

using namespace pa;

namespace {

using Clock = std::chrono::steady_clock;

uint64_t nwords(uint64_t bits) { return (bits + 63) / 64; }

struct Request {
    uint64_t ticket = 0;
    const uint64_t* key = nullptr;
    uint64_t* out = nullptr;
    uint64_t seed_a = 0, seed_b = 0, n = 0, m = 0;
    bool device = false;          // key/out are device pointers
    hipEvent_t ready = nullptr;   // device requests: wait for it before the first kernel
    Clock::time_point submitted, finished;
    int status = -1;              // -1 pending/running, else a PA_* code
    bool done = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint64_t* in_stage = nullptr;    // pinned, for host requests
    uint64_t* out_stage = nullptr;
    Request* req = nullptr;
    uint64_t off = 0, bytes = 0;
};

double ms_between(Clock::time_point a, Clock::time_point b)
{
    return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct pa_server {
    pa_ctx* ctx = nullptr;
    pa_server_opts opts{};
    uint8_t* pool = nullptr;
    pa::Arena* arena = nullptr;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::map<uint64_t, Request*> all;   // submitted and not yet waited on
    uint64_t outstanding = 0;           // submitted and not yet done
    std::vector<double> lat_ok;         // latency of every completed request
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    // stats (guarded by mu)
    uint64_t completed = 0, failed = 0, bits = 0, admitted_peak = 0;
    Clock::time_point first_submit, last_done;
    bool any = false;
};

namespace {

uint64_t footprint(const pa_server* s, const Request& r)
{
    (void)s;
    uint64_t b = block_workspace_bytes(r.n);
    if (!r.device) b += round256(nwords(r.n) * 8) + round256(nwords(r.m) * 8);
    return b;
}

// Start request r on slot sl (scheduler thread).  Returns a PA_* code.
int start(pa_server* s, Slot& sl, Request* r, uint64_t off, uint64_t bytes)
{
    pa_ctx* ctx = s->ctx;
    sl.req = r;
    sl.off = off;
    sl.bytes = bytes;
    uint8_t* base = s->pool + off;
    BlockBufs b;
    block_layout(r->n, base, &b);
    const uint64_t* dkey = r->key;
    uint64_t* dout = r->out;
    if (!r->device) {
        uint8_t* io = base + block_workspace_bytes(r->n);
        uint64_t* kbuf = reinterpret_cast<uint64_t*>(io);
        dout = reinterpret_cast<uint64_t*>(io + round256(nwords(r->n) * 8));
        memcpy(sl.in_stage, r->key, nwords(r->n) * 8);
        if (hipMemcpyAsync(kbuf, sl.in_stage, nwords(r->n) * 8, hipMemcpyHostToDevice,
                           sl.stream) != hipSuccess)
            return PA_EDEVICE;
        dkey = kbuf;
    }
    // a device request's key (and out) may still be written by the caller's
    // work: the slot's stream waits for the event the caller gave
    if (r->ready && hipStreamWaitEvent(sl.stream, r->ready, 0) != hipSuccess) return PA_EDEVICE;
    b.key = reinterpret_cast<const uint32_t*>(dkey);
    b.seed_a = r->seed_a;
    b.seed_b = r->seed_b;
    b.n = r->n;
    b.m = r->m;
    b.out = dout;
    int rc = enqueue_block(ctx, b, sl.stream);
    if (rc) return rc;
    if (!r->device &&
        hipMemcpyAsync(sl.out_stage, dout, nwords(r->m) * 8, hipMemcpyDeviceToHost, sl.stream) !=
            hipSuccess)
        return PA_EDEVICE;
    if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return PA_EDEVICE;
    return PA_OK;
}

void finish(pa_server* s, Slot& sl, int status)
{
    Request* r = sl.req;
    if (status == PA_OK && !r->device) memcpy(r->out, sl.out_stage, nwords(r->m) * 8);
    s->arena->release(sl.off, sl.bytes);
    std::lock_guard<std::mutex> lk(s->mu);
    r->finished = Clock::now();
    r->status = status;
    r->done = true;
    --s->outstanding;
    if (status == PA_OK) {
        ++s->completed;
        s->bits += r->n;
        s->lat_ok.push_back(ms_between(r->submitted, r->finished));
    } else {
        ++s->failed;
    }
    s->last_done = r->finished;
    sl.req = nullptr;
    s->cv_done.notify_all();
}

void scheduler(pa_server* s)
{
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        bool progress = false;
        // retire finished slots
        for (auto& sl : s->slots) {
            if (!sl.req) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) {
                finish(s, sl, PA_OK);
                progress = true;
            } else if (q != hipErrorNotReady) {
                finish(s, sl, PA_EDEVICE);
                progress = true;
            }
        }
        // admit in arrival order while a slot is free and the footprint fits
        for (;;) {
            Request* r = nullptr;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                if (s->pending.empty()) break;
                r = s->pending.front();
            }
            Slot* free_slot = nullptr;
            for (auto& sl : s->slots)
                if (!sl.req) {
                    free_slot = &sl;
                    break;
                }
            if (!free_slot) break;
            const uint64_t bytes = footprint(s, *r);
            uint64_t off = 0;
            if (!s->arena->alloc(bytes, &off)) break;   // wait for memory to free up
            {
                std::lock_guard<std::mutex> lk(s->mu);
                s->pending.pop_front();
            }
            const int rc = start(s, *free_slot, r, off, bytes);
            if (rc != PA_OK) {
                (void)hipStreamSynchronize(free_slot->stream);
                finish(s, *free_slot, rc);
            }
            progress = true;
            uint64_t inflight = 0;
            for (auto& sl : s->slots) inflight += sl.req != nullptr;
            std::lock_guard<std::mutex> lk(s->mu);
            s->admitted_peak = std::max(s->admitted_peak, inflight);
        }
        bool busy = false;
        for (auto& sl : s->slots) busy |= sl.req != nullptr;
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && !busy && s->pending.empty()) return;
        if (!progress) {
            if (busy)   // kernels in flight: poll again shortly
                s->cv_work.wait_for(lk, std::chrono::microseconds(20));
            else
                s->cv_work.wait_for(lk, std::chrono::milliseconds(5),
                                    [&] { return s->stop || !s->pending.empty(); });
        }
    }
}

}  // namespace

extern "C" {

void pa_server_destroy(pa_server* s)
{
    if (!s) return;
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        s->worker.join();
    }
    if (s->ctx) {
        (void)hipSetDevice(s->ctx->device);
        for (auto& sl : s->slots) {
            if (sl.stream) (void)hipStreamSynchronize(sl.stream);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
            if (sl.in_stage) (void)hipHostFree(sl.in_stage);
            if (sl.out_stage) (void)hipHostFree(sl.out_stage);
        }
        (void)hipFree(s->pool);
        pa_destroy(s->ctx);
    }
    for (auto& kv : s->all) delete kv.second;
    delete s->arena;
    delete s;
}

int pa_server_create(int device, const pa_server_opts* opts, pa_server** out)
{
    if (!opts || !out || opts->slots <= 0 || opts->max_n == 0 || opts->max_n > PA_MAX_N)
        return PA_EINVAL;
    *out = nullptr;
    pa_server* s = new (std::nothrow) pa_server;
    if (!s) return PA_ENOMEM;
    s->opts = *opts;
    int rc = pa_init(&s->ctx, device, nullptr);
    if (rc) {
        delete s;
        return rc;
    }
    // the largest request must fit on its own
    const uint64_t need = block_workspace_bytes(opts->max_n) + round256(nwords(opts->max_n) * 8) * 2;
    if (opts->hbm_budget < need) {
        pa_server_destroy(s);
        return PA_EINVAL;
    }
    if (hipMalloc(&s->pool, opts->hbm_budget) != hipSuccess) {
        pa_server_destroy(s);
        return PA_ENOMEM;
    }
    s->arena = new (std::nothrow) pa::Arena(opts->hbm_budget);
    if (!s->arena) {
        pa_server_destroy(s);
        return PA_ENOMEM;
    }
    s->slots.resize(opts->slots);
    for (auto& sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(&sl.in_stage, nwords(opts->max_n) * 8, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&sl.out_stage, nwords(opts->max_n) * 8, hipHostMallocDefault) != hipSuccess) {
            pa_server_destroy(s);
            return PA_EDEVICE;
        }
    }
    s->worker = std::thread(scheduler, s);
    *out = s;
    return PA_OK;
}

int pa_server_submit(pa_server* s, const uint64_t* key, uint64_t seed_a, uint64_t seed_b,
                     uint64_t n, uint64_t m, uint64_t* out, int flags, uint64_t* ticket)
{
    return pa_server_submit_after(s, key, seed_a, seed_b, n, m, out, flags, nullptr, ticket);
}

int pa_server_submit_after(pa_server* s, const uint64_t* key, uint64_t seed_a, uint64_t seed_b,
                           uint64_t n, uint64_t m, uint64_t* out, int flags, void* ready,
                           uint64_t* ticket)
{
    if (!s || !key || !out || !ticket || n == 0 || m == 0 || m > n) return PA_EINVAL;
    if (n > s->opts.max_n) return PA_EINVAL;
    if (ready && !(flags & PA_SUBMIT_DEVICE)) return PA_EINVAL;
    Request* r = new (std::nothrow) Request;
    if (!r) return PA_ENOMEM;
    r->ready = (hipEvent_t)ready;
    r->key = key;
    r->out = out;
    r->seed_a = seed_a;
    r->seed_b = seed_b;
    r->n = n;
    r->m = m;
    r->device = (flags & PA_SUBMIT_DEVICE) != 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ticket = s->next_ticket++;
        r->submitted = Clock::now();
        if (!s->any) {
            s->first_submit = r->submitted;
            s->any = true;
        }
        s->all[r->ticket] = r;
        ++s->outstanding;
        s->pending.push_back(r);
    }
    s->cv_work.notify_one();
    *ticket = r->ticket;
    return PA_OK;
}

int pa_server_wait(pa_server* s, uint64_t ticket, int* status, double* latency_ms)
{
    if (!s) return PA_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return PA_EINVAL;
    Request* r = it->second;
    s->cv_done.wait(lk, [&] { return r->done; });
    if (status) *status = r->status;
    if (latency_ms) *latency_ms = ms_between(r->submitted, r->finished);
    // done: the scheduler no longer holds r (finish() let go of it under the lock)
    s->all.erase(it);
    delete r;
    return PA_OK;
}

int pa_server_drain(pa_server* s)
{
    if (!s) return PA_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
    return PA_OK;
}

int pa_server_get_stats(pa_server* s, pa_server_stats* st)
{
    if (!s || !st) return PA_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    memset(st, 0, sizeof *st);
    st->completed = s->completed;
    st->failed = s->failed;
    st->bits = s->bits;
    st->peak_inflight = s->admitted_peak;
    st->peak_bytes = s->arena ? s->arena->peak() : 0;
    std::vector<double> lat = s->lat_ok;
    if (!lat.empty()) {
        std::sort(lat.begin(), lat.end());
        auto pct = [&](double q) {
            const size_t i = (size_t)(q * (double)(lat.size() - 1) + 0.5);
            return lat[std::min(i, lat.size() - 1)];
        };
        st->lat_p50_ms = pct(0.50);
        st->lat_p99_ms = pct(0.99);
        double sum = 0;
        for (double v : lat) sum += v;
        st->lat_mean_ms = sum / (double)lat.size();
        st->wall_s = std::chrono::duration<double>(s->last_done - s->first_submit).count();
    }
    return PA_OK;
}

int pa_server_run_trace(pa_server* s, const pa_job* jobs, const double* arrival_s, size_t count,
                        int flags, double* latency_ms, int* status)
{
    if (!s || (count && (!jobs || !arrival_s))) return PA_EINVAL;
    std::vector<uint64_t> tickets(count, 0);
    std::vector<int> rcs(count, PA_OK);
    const Clock::time_point t0 = Clock::now();
    for (size_t i = 0; i < count; ++i) {
        const auto due = t0 + std::chrono::duration_cast<Clock::duration>(
                                  std::chrono::duration<double>(arrival_s[i]));
        while (Clock::now() < due) {
            const auto left = due - Clock::now();
            if (left > std::chrono::microseconds(200))
                std::this_thread::sleep_for(left - std::chrono::microseconds(100));
        }
        rcs[i] = (jobs[i].c || jobs[i].d)
                     ? PA_EINVAL
                     : pa_server_submit(s, jobs[i].key, jobs[i].seed_a, jobs[i].seed_b, jobs[i].n,
                                        jobs[i].m, jobs[i].out, flags, &tickets[i]);
    }
    for (size_t i = 0; i < count; ++i) {
        int st = rcs[i];
        double lat = -1;
        if (rcs[i] == PA_OK) pa_server_wait(s, tickets[i], &st, &lat);
        if (latency_ms) latency_ms[i] = lat;
        if (status) status[i] = st;
    }
    return PA_OK;
}

}  // extern "C"
