// libpa server: continuous hashing of a stream of requests on one GPU.
//
// Requests are admitted in arrival order as soon as a slot is free and their
// device footprint (spectra, carry state and, for host requests, the key and
// output buffers) fits in a fixed HBM budget; each admitted request runs on its
// slot's stream, so requests that arrive while others are on the GPU start at
// once and their kernels overlap on the device.  Budget memory is one
// allocation made at creation and handed out first-fit, so admission never
// calls hipMalloc.  The twiddle tables live on the device for the server's
// lifetime (its own context).  A scheduler thread admits requests, queues
// their device work and retires them; callers only touch a mutex-protected
// queue.  For host requests each slot has a copy thread that moves the key
// into the slot's pinned staging buffer and the result out of it, so that
// those copies (megabytes each) run beside each other and never hold up the
// scheduler.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
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

// Where a slot's request is (transitions under the server's mutex):
// free -> [host: staging in (copy thread) -> staged] -> running (device work
// queued) -> [host: staging out (copy thread) -> copied] -> free.
enum Phase : int { kFree, kStageIn, kStaged, kRunning, kStageOut, kCopied };

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint64_t* in_stage = nullptr;    // pinned, for host requests
    uint64_t* out_stage = nullptr;
    Request* req = nullptr;
    uint64_t off = 0, bytes = 0;
    Phase phase = kFree;
    std::condition_variable cv;      // wakes the copy thread
    std::thread copier;
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
    std::vector<std::unique_ptr<Slot>> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> pending;
    std::map<uint64_t, Request*> all;   // submitted and not yet waited on
    uint64_t outstanding = 0;           // submitted and not yet done
    std::vector<double> lat_ok;         // latency of every completed request
    uint64_t next_ticket = 1;
    bool stop = false;
    bool stop_copiers = false;
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

// Queue the device work of slot sl's request (scheduler thread): for a host
// request its key is in the slot's staging buffer.  Returns a PA_* code.
int start_gpu(pa_server* s, Slot& sl)
{
    pa_ctx* ctx = s->ctx;
    Request* r = sl.req;
    uint8_t* base = s->pool + sl.off;
    BlockBufs b;
    block_layout(r->n, base, &b);
    const uint64_t* dkey = r->key;
    uint64_t* dout = r->out;
    if (!r->device) {
        uint8_t* io = base + block_workspace_bytes(r->n);
        uint64_t* kbuf = reinterpret_cast<uint64_t*>(io);
        dout = reinterpret_cast<uint64_t*>(io + round256(nwords(r->n) * 8));
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

// A slot's copy thread: the host copies of its requests.
void copier(pa_server* s, Slot* sl)
{
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        sl->cv.wait(lk, [&] {
            return s->stop_copiers || sl->phase == kStageIn || sl->phase == kStageOut;
        });
        if (s->stop_copiers) return;
        const Request* r = sl->req;
        const bool in = sl->phase == kStageIn;
        lk.unlock();
        if (in)
            memcpy(sl->in_stage, r->key, nwords(r->n) * 8);
        else
            memcpy(r->out, sl->out_stage, nwords(r->m) * 8);
        lk.lock();
        sl->phase = in ? kStaged : kCopied;
        s->cv_work.notify_one();
    }
}

Phase phase_of(pa_server* s, const Slot& sl)
{
    std::lock_guard<std::mutex> lk(s->mu);
    return sl.phase;
}

void set_phase(pa_server* s, Slot& sl, Phase ph)
{
    {
        std::lock_guard<std::mutex> lk(s->mu);
        sl.phase = ph;
    }
    if (ph == kStageIn || ph == kStageOut) sl.cv.notify_one();
}

// Retire slot sl's request (scheduler thread); for a host request its result
// is already in the caller's buffer.
void finish(pa_server* s, Slot& sl, int status)
{
    Request* r = sl.req;
    s->arena->release(sl.off, sl.bytes);
    std::lock_guard<std::mutex> lk(s->mu);
    sl.phase = kFree;
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
    // queue the device work of a slot whose request is ready for it
    auto launch = [&](Slot& sl) {
        const int rc = start_gpu(s, sl);
        if (rc != PA_OK) {
            (void)hipStreamSynchronize(sl.stream);
            finish(s, sl, rc);
            return;
        }
        set_phase(s, sl, kRunning);
    };
    for (;;) {
        bool progress = false;
        for (auto& p : s->slots) {
            Slot& sl = *p;
            const Phase ph = phase_of(s, sl);
            if (ph == kStaged) {
                launch(sl);
                progress = true;
            } else if (ph == kRunning) {
                // retire finished device work
                const hipError_t q = hipEventQuery(sl.done);
                if (q == hipSuccess) {
                    if (sl.req->device)
                        finish(s, sl, PA_OK);
                    else
                        set_phase(s, sl, kStageOut);
                    progress = true;
                } else if (q != hipErrorNotReady) {
                    finish(s, sl, PA_EDEVICE);
                    progress = true;
                }
            } else if (ph == kCopied) {
                finish(s, sl, PA_OK);
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
            for (auto& p : s->slots)
                if (!p->req) {
                    free_slot = p.get();
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
            free_slot->req = r;
            free_slot->off = off;
            free_slot->bytes = bytes;
            if (r->device)
                launch(*free_slot);
            else
                set_phase(s, *free_slot, kStageIn);
            progress = true;
            uint64_t inflight = 0;
            for (auto& p : s->slots) inflight += p->req != nullptr;
            std::lock_guard<std::mutex> lk(s->mu);
            s->admitted_peak = std::max(s->admitted_peak, inflight);
        }
        bool busy = false;
        for (auto& p : s->slots) busy |= p->req != nullptr;
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && !busy && s->pending.empty()) return;
        if (!progress) {
            if (busy)   // kernels or copies in flight: poll again shortly
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
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop_copiers = true;
    }
    for (auto& p : s->slots) {
        p->cv.notify_all();
        if (p->copier.joinable()) p->copier.join();
    }
    if (s->ctx) {
        (void)hipSetDevice(s->ctx->device);
        for (auto& p : s->slots) {
            Slot& sl = *p;
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
    for (int i = 0; i < opts->slots; ++i) {
        s->slots.emplace_back(new (std::nothrow) Slot);
        if (!s->slots.back()) {
            s->slots.pop_back();
            pa_server_destroy(s);
            return PA_ENOMEM;
        }
        Slot& sl = *s->slots.back();
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(&sl.in_stage, nwords(opts->max_n) * 8, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&sl.out_stage, nwords(opts->max_n) * 8, hipHostMallocDefault) != hipSuccess) {
            pa_server_destroy(s);
            return PA_EDEVICE;
        }
        sl.copier = std::thread(copier, s, &sl);
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
