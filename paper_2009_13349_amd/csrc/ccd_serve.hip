// Serving loop of the CCD library: continuous batching of requests on one GPU.
//
// A request is a batch of queries in host memory.  A scheduler thread
//   1. admits queued requests in arrival order while the device pool has room
//      for their inputs and outputs, copying the inputs on a copy stream;
//   2. whenever one of the compute streams is idle, launches one pass of the
//      root finder over all admitted requests not yet started: the launch's
//      query index space is the concatenation of their queries (a request
//      table maps an index to its request), so requests of any size share one
//      set of kernels, and a request that arrives while a launch runs goes into
//      the next launch on another stream, overlapping the tail of the first;
//   3. after each launch, copies the results back on the same stream and, once
//      its completion event has fired, completes the tickets and frees the
//      pool space.
// Kernels never wait for work that is not there: each launch covers a fixed
// set of requests and ends.  Results of a request are bit-identical to those
// of the same batch run alone (the root finder is independent per query).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/ccd.h"
#include "ccd_host.h"
#include "ccd_internal.h"

using namespace ccd;

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over one device buffer.
class Pool {
  public:
    void init(size_t bytes) {
        size_ = bytes;
        free_.clear();
        free_[0] = bytes;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align256(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    std::map<size_t, size_t> free_;
    size_t size_ = 0, used_ = 0, peak_ = 0;
};

enum ReqState { kQueued = 0, kAdmitted = 1, kRunning = 2, kDone = 3 };

struct Request {
    int64_t ticket = 0;
    int64_t n = 0;
    // caller's host buffers
    const double* pos = nullptr;
    const uint8_t* kind = nullptr;
    uint8_t default_kind = 0;
    ccd_params params{};
    ccd_result_soa out{};
    // device placement
    size_t off = 0, bytes = 0;
    char* dev = nullptr;
    double* d_pos = nullptr;
    uint8_t* d_kind = nullptr;
    double *d_toi = nullptr, *d_tw = nullptr;
    uint8_t *d_hit = nullptr, *d_st = nullptr;
    uint64_t* d_nc = nullptr;
    size_t hoff = 0, hbytes = 0;   // pinned staging of the results
    char* h_stage = nullptr;
    hipEvent_t in_ready = nullptr;
    int state = kQueued;
    int rc = CCD_OK;
    double t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
};

size_t result_bytes(int64_t n) { return 3 * align256((size_t)n * 8) + 2 * align256((size_t)n); }

size_t request_bytes(int64_t n, bool kind) {
    return align256((size_t)24 * n * 8) + (kind ? align256((size_t)n) : 0) + result_bytes(n);
}

// Results laid out identically in device memory and in the pinned staging.
struct ResultLayout {
    size_t toi, tw, nc, hit, st;
    explicit ResultLayout(int64_t n) {
        toi = 0;
        tw = toi + align256((size_t)n * 8);
        nc = tw + align256((size_t)n * 8);
        hit = nc + align256((size_t)n * 8);
        st = hit + align256((size_t)n);
    }
};

struct Slot {
    ccd_context* ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t start = nullptr;  // device time of a launch: start -> done
    hipEvent_t done = nullptr;
    int64_t queries = 0;         // queries of the launch in flight
    ReqEntry* d_table = nullptr;
    ReqEntry* h_table = nullptr;  // pinned
    std::vector<Request*> reqs;
    bool busy = false;
};

}  // namespace

struct ccd_server {
    ccd_serve_config cfg{};
    char* pool_base = nullptr;
    Pool pool;
    char* pin_base = nullptr;  // pinned host staging for results
    Pool pin;
    hipStream_t copy_stream = nullptr;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;    // submitted, not admitted
    std::deque<Request*> ready;    // admitted (inputs copying), not launched
    std::map<int64_t, Request*> tickets;
    std::vector<hipEvent_t> event_pool;
    int64_t next_ticket = 1;
    double ms_per_query = 0.0;  // device time per query of recent launches (EWMA; 0: none yet)
    bool stop = false;
    bool failed = false;
    std::thread worker;
    ccd_serve_stats st{};
};

namespace {

hipEvent_t take_event(ccd_server* s) {
    if (!s->event_pool.empty()) {
        hipEvent_t e = s->event_pool.back();
        s->event_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void finish(ccd_server* s, Request* r, int rc) {
    r->rc = rc;
    r->state = kDone;
    r->t_done = now_s();
    s->pool.release(r->off, r->bytes);
    s->pin.release(r->hoff, r->hbytes);
    if (r->in_ready) s->event_pool.push_back(r->in_ready);
    r->in_ready = nullptr;
    s->st.completed += 1;
    s->st.queries_completed += (uint64_t)r->n;
}

// Admission in arrival order (head of line blocks: no overtaking, so a large
// request is never starved by small ones).  Called with the lock held.
void admit(ccd_server* s) {
    while (!s->queue.empty()) {
        Request* r = s->queue.front();
        size_t off, hoff;
        if (!s->pool.alloc(r->bytes, &off)) break;
        r->hbytes = result_bytes(r->n);
        if (!s->pin.alloc(r->hbytes, &hoff)) {
            s->pool.release(off, r->bytes);
            break;
        }
        s->queue.pop_front();
        r->off = off;
        r->hoff = hoff;
        r->h_stage = s->pin_base + hoff;
        char* p = s->pool_base + off;
        const int64_t n = r->n;
        r->d_pos = (double*)p;
        p += align256((size_t)24 * n * 8);
        if (r->kind) {
            r->d_kind = (uint8_t*)p;
            p += align256((size_t)n);
        }
        const ResultLayout L(n);
        r->d_toi = (double*)(p + L.toi);
        r->d_tw = (double*)(p + L.tw);
        r->d_nc = (uint64_t*)(p + L.nc);
        r->d_hit = (uint8_t*)(p + L.hit);
        r->d_st = (uint8_t*)(p + L.st);
        r->in_ready = take_event(s);
        bool ok = r->in_ready != nullptr &&
                  record_hip(hipMemcpyAsync(r->d_pos, r->pos, (size_t)24 * n * 8,
                                            hipMemcpyHostToDevice, s->copy_stream), "serve copy pos");
        if (ok && r->kind)
            ok = record_hip(hipMemcpyAsync(r->d_kind, r->kind, (size_t)n, hipMemcpyHostToDevice,
                                           s->copy_stream), "serve copy kind");
        if (ok) ok = record_hip(hipEventRecord(r->in_ready, s->copy_stream), "serve event");
        r->state = kAdmitted;
        r->t_admit = now_s();
        s->st.admitted += 1;
        if (!ok) {
            s->failed = true;
            finish(s, r, CCD_EDEVICE);
            continue;
        }
        s->ready.push_back(r);
    }
    s->st.pool_in_use = s->pool.used();
    s->st.pool_peak = s->pool.peak();
}

// Launch one pass over ready requests on an idle slot.  Lock held.
void launch_slot(ccd_server* s, Slot& sl) {
    std::vector<Request*> take;
    int64_t total = 0, mi_max = 1;
    // latency bound: as many queries as fill the target device time at the
    // measured cost per query (the first request always goes)
    int64_t limit = s->cfg.max_queries_per_launch;
    if (s->cfg.launch_target_us > 0 && s->ms_per_query > 0.0)
        limit = std::min<int64_t>(limit, (int64_t)(1e-3 * s->cfg.launch_target_us / s->ms_per_query) + 1);
    while (!s->ready.empty() && (int)take.size() < s->cfg.max_requests) {
        Request* r = s->ready.front();
        if (!take.empty() && total + r->n > limit) break;
        s->ready.pop_front();
        take.push_back(r);
        total += r->n;
        mi_max = std::max<int64_t>(mi_max, r->params.max_iter);
    }
    if (take.empty()) return;
    bool ok = true;
    for (size_t i = 0, base = 0; i < take.size(); ++i) {
        Request* r = take[i];
        ReqEntry& e = sl.h_table[i];
        e.base = (int64_t)base;
        e.n = r->n;
        e.pos = r->d_pos;
        e.kind = r->kind ? r->d_kind : nullptr;
        e.delta = r->params.delta;
        e.max_iter = r->params.max_iter;
        e.min_sep = r->params.min_sep;
        e.t_max = r->params.t_max;
        e.flags = r->params.flags;
        e.default_kind = r->default_kind;
        e.toi = r->d_toi;
        e.t_width = r->d_tw;
        e.hit = r->d_hit;
        e.n_checks = r->d_nc;
        e.status = r->d_st;
        base += (size_t)r->n;
        if (ok) ok = record_hip(hipStreamWaitEvent(sl.stream, r->in_ready, 0), "serve wait input");
        r->state = kRunning;
        r->t_launch = now_s();
    }
    ok = ok && record_hip(hipMemcpyAsync(sl.d_table, sl.h_table, take.size() * sizeof(ReqEntry),
                                         hipMemcpyHostToDevice, sl.stream), "serve copy table");
    ok = ok && record_hip(hipEventRecord(sl.start, sl.stream), "serve event");
    sl.queries = total;
    BatchArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = total;
    a.reqs = sl.d_table;
    a.nreq = (int64_t)take.size();
    int rc = ok ? run_args(sl.ctx, a, mi_max, sl.stream) : CCD_EDEVICE;
    for (Request* r : take) {
        if (rc != CCD_OK) break;
        // one copy of the whole result block into pinned staging
        if (!record_hip(hipMemcpyAsync(r->h_stage, (const void*)r->d_toi, r->hbytes,
                                       hipMemcpyDeviceToHost, sl.stream), "serve copy results"))
            rc = CCD_EDEVICE;
    }
    if (rc == CCD_OK && !record_hip(hipEventRecord(sl.done, sl.stream), "serve event")) rc = CCD_EDEVICE;
    s->st.launches += 1;
    if (rc != CCD_OK) {
        // the stream may hold partial work: wait for it, then fail these requests
        (void)hipStreamSynchronize(sl.stream);
        (void)hipGetLastError();
        for (Request* r : take) finish(s, r, rc);
        s->cv_done.notify_all();
        return;
    }
    sl.reqs = std::move(take);
    sl.busy = true;
}

void worker_main(ccd_server* s) {
    (void)hipSetDevice(s->cfg.device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        bool progress = false;
        // completions: results are in pinned staging once the event has fired;
        // copy them to the caller's arrays without holding the lock
        for (Slot& sl : s->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            const int rc = (q == hipSuccess) ? CCD_OK : CCD_EDEVICE;
            if (q != hipSuccess) record_hip(q, "serve launch");
            std::vector<Request*> reqs = std::move(sl.reqs);
            sl.reqs.clear();
            sl.busy = false;
            float ms = 0.0f;
            if (rc == CCD_OK && sl.queries > 0 &&
                hipEventElapsedTime(&ms, sl.start, sl.done) == hipSuccess && ms > 0.0f) {
                // (launches on two streams overlap, so this is the time a launch
                // takes next to another one: the latency it sees)
                const double c = (double)ms / (double)sl.queries;
                s->ms_per_query = s->ms_per_query > 0.0 ? 0.8 * s->ms_per_query + 0.2 * c : c;
            }
            (void)hipGetLastError();
            if (rc == CCD_OK) {
                lk.unlock();
                for (Request* r : reqs) {
                    const ResultLayout L(r->n);
                    const size_t n = (size_t)r->n;
                    std::memcpy(r->out.toi, r->h_stage + L.toi, n * 8);
                    std::memcpy(r->out.t_width, r->h_stage + L.tw, n * 8);
                    std::memcpy(r->out.n_checks, r->h_stage + L.nc, n * 8);
                    std::memcpy(r->out.hit, r->h_stage + L.hit, n);
                    std::memcpy(r->out.status, r->h_stage + L.st, n);
                }
                lk.lock();
            }
            for (Request* r : reqs) finish(s, r, rc);
            progress = true;
        }
        if (progress) s->cv_done.notify_all();
        admit(s);
        for (Slot& sl : s->slots)
            if (!sl.busy && !s->ready.empty()) {
                launch_slot(s, sl);
                progress = true;
            }
        bool idle = s->queue.empty() && s->ready.empty();
        for (Slot& sl : s->slots) idle = idle && !sl.busy;
        if (s->stop && idle) break;
        if (!progress) {
            if (idle) s->cv_work.wait(lk);  // nothing in flight: sleep until a submission
            else s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        }
    }
}

bool desc_valid_host(const ccd_batch_desc* d, const ccd_result_soa* out) {
    if (!d || !out || d->on_device || d->n <= 0 || !d->pos) return false;
    if (d->delta_q || d->max_iter_q || d->min_sep_q) return false;  // per-request scalars only
    if (d->default_kind > 1) return false;
    const ccd_params& p = d->params;
    if (!(p.t_max > 0.0 && p.t_max <= 1.0) || p.reserved || (p.flags & ~CCD_FLAG_LITERAL))
        return false;
    if (!out->toi || !out->t_width || !out->hit || !out->n_checks || !out->status) return false;
    const int64_t n = d->n;
    for (int64_t q = 0; q < n; ++q) {
        double X[24];
        for (int r = 0; r < 24; ++r) X[r] = d->pos[r * n + q];
        const int kind = d->kind ? d->kind[q] : d->default_kind;
        if (!host_valid(X, kind, p.delta, p.max_iter, p.min_sep)) return false;
    }
    return true;
}

void destroy(ccd_server* s) {
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.start) (void)hipEventDestroy(sl.start);
        if (sl.d_table) (void)hipFree(sl.d_table);
        if (sl.h_table) (void)hipHostFree(sl.h_table);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.ctx) ccd_context_destroy(sl.ctx);
    }
    if (s->copy_stream) {
        (void)hipStreamSynchronize(s->copy_stream);
        (void)hipStreamDestroy(s->copy_stream);
    }
    for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
    for (auto& kv : s->tickets) {
        if (kv.second->in_ready) (void)hipEventDestroy(kv.second->in_ready);
        delete kv.second;
    }
    if (s->pool_base) (void)hipFree(s->pool_base);
    if (s->pin_base) (void)hipHostFree(s->pin_base);
    (void)hipGetLastError();
    delete s;
}

}  // namespace

extern "C" {

void ccd_serve_config_default(ccd_serve_config* c) {
    if (!c) return;
    std::memset(c, 0, sizeof(*c));
    c->device = 0;
    c->streams = 2;
    c->max_requests = 1024;
    c->max_queries_per_launch = 4000000;
    c->launch_target_us = 5000;
    c->pool_bytes = (size_t)8 << 30;
    c->scratch_bytes = (size_t)12 << 30;
}

int ccd_serve_open(const ccd_serve_config* cfg, ccd_server** out) {
    if (!out) return CCD_EINVAL;
    ccd_serve_config c;
    ccd_serve_config_default(&c);
    if (cfg) c = *cfg;
    if (c.streams < 1 || c.streams > 4 || c.max_requests < 1 || c.max_queries_per_launch < 1 ||
        c.pool_bytes < 4096 || c.launch_target_us < 0)
        return CCD_EINVAL;
    ccd_server* s = new ccd_server();
    s->cfg = c;
    if (!record_hip(hipSetDevice(c.device), "hipSetDevice") ||
        !record_hip(hipMalloc((void**)&s->pool_base, c.pool_bytes), "serve pool") ||
        !record_hip(hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking), "serve stream")) {
        destroy(s);
        return CCD_ENOMEM;
    }
    s->pool.init(c.pool_bytes);
    // results are 26 of the ~218 bytes a query occupies in the device pool
    const size_t pin_bytes = std::max<size_t>(c.pool_bytes / 8, (size_t)1 << 20);
    if (!record_hip(hipHostMalloc((void**)&s->pin_base, pin_bytes, 0), "serve pinned staging")) {
        destroy(s);
        return CCD_ENOMEM;
    }
    s->pin.init(pin_bytes);
    s->slots.resize(c.streams);
    for (Slot& sl : s->slots) {
        int rc = ccd_context_create(c.device, c.scratch_bytes, &sl.ctx);
        if (rc != CCD_OK) {
            destroy(s);
            return rc;
        }
        ccd_context_enable_graphs(sl.ctx, 0);  // the request table changes every launch
        // a fixed 1 GiB hand-off pool: sized by what the budget leaves, the
        // pool would grow (a reallocation that stalls the device) whenever a
        // launch smaller than any before it leaves more of the budget free
        {
            ccd_tuning t;
            std::memset(&t, 0, sizeof(t));
            t.handoff_words = int64_t(1) << 27;
            rc = ccd_context_set_tuning(sl.ctx, &t);
            if (rc != CCD_OK) {
                destroy(s);
                return rc;
            }
        }
        rc = reserve(sl.ctx, c.max_queries_per_launch, 1000000);
        if (rc != CCD_OK) {
            destroy(s);
            return rc;
        }
        if (!record_hip(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking), "serve stream") ||
            !record_hip(hipEventCreate(&sl.start), "serve event") ||
            !record_hip(hipEventCreate(&sl.done), "serve event") ||
            !record_hip(hipMalloc((void**)&sl.d_table, sizeof(ReqEntry) * c.max_requests), "serve table") ||
            !record_hip(hipHostMalloc((void**)&sl.h_table, sizeof(ReqEntry) * c.max_requests, 0), "serve table")) {
            destroy(s);
            return CCD_ENOMEM;
        }
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return CCD_OK;
}

int ccd_serve_submit(ccd_server* s, const ccd_batch_desc* d, const ccd_result_soa* out, int flags,
                     int64_t* ticket) {
    if (!s || !ticket) return CCD_EINVAL;
    if (!desc_valid_host(d, out)) return CCD_EINVAL;
    const size_t bytes = request_bytes(d->n, d->kind != nullptr);
    if (bytes > s->pool.size() || result_bytes(d->n) > s->pin.size()) {
        set_last_error("request larger than the serving pool");
        return CCD_ENOMEM;
    }
    Request* r = new Request();
    r->n = d->n;
    r->pos = d->pos;
    r->kind = d->kind;
    r->default_kind = d->default_kind;
    r->params = d->params;
    r->out = *out;
    r->bytes = bytes;
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            return CCD_ECANCELED;
        }
        if ((flags & CCD_SERVE_NONBLOCKING) && !s->queue.empty()) {
            delete r;
            s->st.rejected += 1;
            return CCD_EAGAIN;
        }
        if (flags & CCD_SERVE_NONBLOCKING) {
            size_t off;
            if (!s->pool.alloc(bytes, &off)) {
                delete r;
                s->st.rejected += 1;
                return CCD_EAGAIN;
            }
            s->pool.release(off, bytes);
        }
        r->ticket = s->next_ticket++;
        s->tickets[r->ticket] = r;
        s->queue.push_back(r);
        s->st.submitted += 1;
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return CCD_OK;
}

int ccd_serve_query(ccd_server* s, int64_t ticket, ccd_serve_info* info) {
    if (!s) return CCD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return CCD_EINVAL;
    Request* r = it->second;
    if (info) {
        std::memset(info, 0, sizeof(*info));
        info->state = r->state;
        info->rc = r->rc;
        info->n = r->n;
        info->t_submit = r->t_submit;
        info->t_admit = r->t_admit;
        info->t_launch = r->t_launch;
        info->t_done = r->t_done;
    }
    return CCD_OK;
}

int ccd_serve_poll(ccd_server* s, int64_t ticket) {
    if (!s) return CCD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return CCD_EINVAL;
    if (it->second->state != kDone) return 0;
    return it->second->rc == CCD_OK ? 1 : it->second->rc;
}

int ccd_serve_wait(ccd_server* s, int64_t ticket, int timeout_ms) {
    if (!s) return CCD_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return CCD_EINVAL;
    Request* r = it->second;
    auto done = [&] { return r->state == kDone; };
    if (timeout_ms < 0) s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), done))
        return CCD_ETIMEDOUT;
    return r->rc;
}

int ccd_serve_release(ccd_server* s, int64_t ticket) {
    if (!s) return CCD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end()) return CCD_EINVAL;
    if (it->second->state != kDone) return CCD_EAGAIN;
    delete it->second;
    s->tickets.erase(it);
    return CCD_OK;
}

int ccd_serve_stats_get(ccd_server* s, ccd_serve_stats* out) {
    if (!s || !out) return CCD_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->st;
    out->queued = s->queue.size();
    out->pool_bytes = s->pool.size();
    return CCD_OK;
}

int ccd_serve_close(ccd_server* s) {
    if (!s) return CCD_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    destroy(s);
    return CCD_OK;
}

}  // extern "C"
