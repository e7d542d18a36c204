// Request-serving loop over an ldpc_engine (the ldpc_server_* entry points).
//
// Client threads submit requests (host LLRs, copied at submit: straight into
// the pinned staging arena while it has room, else into host memory).  One
// worker thread owns the engine: it admits waiting requests in arrival order
// while the device-memory budget, a completion counter and the graph's engine
// queue allow, uploads their LLRs on a copy stream that the engine waits for,
// queues their frames (each frame bumps the request's device counter when it
// finishes), runs engine steps, and when a request's counter reaches its
// frame count copies the results back and time-stamps the completion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace {

using ldpc::set_error;
using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) with coalescing; offsets aligned to 256.
class Arena {
   public:
    explicit Arena(size_t size) : size_(size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~size_t(255);
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
        bytes = (bytes + 255) & ~size_t(255);
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
    size_t size_, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Request {
    int64_t id = 0;
    int32_t graph = 0, frames = 0, n = 0;
    std::vector<float> llr;
    size_t dev_off = 0, dev_bytes = 0, stage_off = 0, stage_bytes = 0, out_off = 0, out_bytes = 0;
    bool staged = false;
    bool prestaged = false;    // LLRs copied into the pinned arena at submit
    bool ready = false;        // the submitting thread has finished copying the LLRs
    int32_t counter = -1;
    uint32_t counter_base = 0; // the counter's value when the request took it
    int64_t admit_cycle = 0;   // worker cycle of admission: counters copied by earlier replays predate it
    std::vector<uint8_t> bits, ok;
    std::vector<int32_t> iters;
    Clock::time_point t_submit, t_done;
};

// Device block of a request: [llr F*n f32][bits F*n u8][ok F u8, iters F i32], each part 256-aligned;
// the outputs (bits, ok, iters) are contiguous so one copy brings them back.
size_t req_llr_bytes(int32_t F, int32_t n) { return (size_t(F) * n * 4 + 255) & ~size_t(255); }
size_t req_out_bytes(int32_t F, int32_t n) {
    return ((size_t(F) * n + 255) & ~size_t(255)) + ((size_t(F) * 5 + 3 + 255) & ~size_t(255));
}
size_t req_dev_bytes(int32_t F, int32_t n) { return req_llr_bytes(F, n) + req_out_bytes(F, n); }

}  // namespace

struct ldpc_server {
    ldpc_engine *engine = nullptr;
    int device = -1;
    int32_t ngraphs = 0;
    std::vector<int32_t> n, queue_cap;
    hipStream_t copy = nullptr;
    char *dev = nullptr;          // device arena
    char *pinned = nullptr;       // pinned host arena
    int32_t *counters = nullptr;  // [max_requests] device completion counters
    int32_t *h_counters = nullptr;
    int32_t max_requests = 4096;
    std::unique_ptr<Arena> dev_arena, host_arena;
    std::vector<int32_t> free_counters;
    std::vector<uint32_t> counter_total;   // frames counted on each counter so far (host mirror)
    int64_t unstaged_waiting = 0;          // waiting requests whose LLRs are not in the pinned arena

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> waiting;
    std::vector<Request *> inflight, staged_uploads;
    hipStream_t engine_stream = nullptr;
    int32_t *h_cnt[2] = {nullptr, nullptr};
    hipEvent_t ev_cnt[2] = {nullptr, nullptr}, ev_out[2] = {nullptr, nullptr};
    std::unordered_map<int64_t, Request *> all;
    std::deque<int64_t> completed;
    int64_t next_id = 1, n_submitted = 0, n_admitted = 0, n_completed = 0, frames_completed = 0;
    bool stop = false;
    std::string worker_error;
    std::thread worker;
};

namespace {

void fail_worker(ldpc_server *s, const std::string &what) {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->worker_error.empty()) s->worker_error = what + ": " + ldpc_last_error();
    s->stop = true;
    s->cv_done.notify_all();
}

// Admit waiting requests in arrival order while resources allow (worker
// thread, lock held).  Frames of all admitted requests of a graph go to the
// engine in one submission that waits for the uploads on the copy stream.
bool admit_locked(ldpc_server *s, int64_t cycle) {
    std::vector<std::vector<ldpc_frame>> batch(static_cast<size_t>(s->ngraphs));
    std::vector<int64_t> queued(static_cast<size_t>(s->ngraphs), 0);
    while (!s->waiting.empty()) {
        Request *r = s->waiting.front();
        if (!r->ready || s->free_counters.empty()) break;
        int32_t cap = 0;
        if (ldpc_engine_capacity(s->engine, r->graph, &cap) != LDPC_OK) return false;
        if (cap - queued[size_t(r->graph)] < r->frames) break;
        size_t doff = 0, hoff = r->stage_off, ooff = 0;
        if (!s->dev_arena->alloc(r->dev_bytes, &doff)) break;
        if (!r->prestaged && !s->host_arena->alloc(r->stage_bytes, &hoff)) {
            s->dev_arena->release(doff, r->dev_bytes);
            break;
        }
        if (!s->host_arena->alloc(r->out_bytes, &ooff)) {
            s->dev_arena->release(doff, r->dev_bytes);
            if (!r->prestaged) s->host_arena->release(hoff, r->stage_bytes);
            break;
        }
        r->dev_off = doff;
        r->stage_off = hoff;
        r->out_off = ooff;
        r->staged = true;
        r->admit_cycle = cycle;
        r->counter = s->free_counters.back();
        r->counter_base = s->counter_total[size_t(r->counter)];
        s->free_counters.pop_back();
        s->waiting.pop_front();
        const int32_t F = r->frames, nn = r->n;
        char *base = s->dev + doff;
        float *d_llr = reinterpret_cast<float *>(base);
        uint8_t *d_bits = reinterpret_cast<uint8_t *>(base + req_llr_bytes(F, nn));
        uint8_t *d_ok = d_bits + ((size_t(F) * nn + 255) & ~size_t(255));
        int32_t *d_iters = reinterpret_cast<int32_t *>(d_ok + ((size_t(F) + 3) & ~size_t(3)));
        if (!r->prestaged) {
            std::memcpy(s->pinned + hoff, r->llr.data(), size_t(F) * nn * 4);
            std::vector<float>().swap(r->llr);
            s->unstaged_waiting--;
        }
        // the request's counter keeps counting from its previous total (no reset)
        hipError_t e = hipMemcpyAsync(d_llr, s->pinned + hoff, size_t(F) * nn * 4, hipMemcpyHostToDevice, s->copy);
        if (e != hipSuccess) {
            set_error(std::string("upload failed: ") + hipGetErrorString(e));
            return false;
        }
        std::vector<ldpc_frame> &fr = batch[size_t(r->graph)];
        for (int32_t f = 0; f < F; f++) {
            ldpc_frame x;
            x.llr = d_llr + size_t(f) * nn;
            x.bits = d_bits + size_t(f) * nn;
            x.ok = d_ok + f;
            x.iters = d_iters + f;
            x.llr_out = nullptr;
            x.done = s->counters + r->counter;
            fr.push_back(x);
        }
        queued[size_t(r->graph)] += F;
        s->inflight.push_back(r);
        s->staged_uploads.push_back(r);
        s->n_admitted++;
    }
    for (int32_t c = 0; c < s->ngraphs; c++) {
        const std::vector<ldpc_frame> &fr = batch[size_t(c)];
        if (!fr.empty() && ldpc_engine_submit(s->engine, c, fr.data(), int32_t(fr.size()), s->copy) != LDPC_OK)
            return false;
    }
    return true;
}

// Requests whose result copies have completed: hand them to the client.
void complete_requests(ldpc_server *s, std::vector<Request *> &done) {
    const auto now = Clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    for (Request *r : done) {
        const int32_t F = r->frames, nn = r->n;
        const uint8_t *h = reinterpret_cast<const uint8_t *>(s->pinned + r->out_off);
        const uint8_t *h_ok = h + ((size_t(F) * nn + 255) & ~size_t(255));
        const uint8_t *h_it = h_ok + ((size_t(F) + 3) & ~size_t(3));
        r->bits.assign(h, h + size_t(F) * nn);
        r->ok.assign(h_ok, h_ok + F);
        r->iters.resize(size_t(F));
        std::memcpy(r->iters.data(), h_it, size_t(F) * 4);
        r->t_done = now;
        s->host_arena->release(r->out_off, r->out_bytes);
        s->dev_arena->release(r->dev_off, r->dev_bytes);
        s->counter_total[size_t(r->counter)] = r->counter_base + uint32_t(F);
        s->free_counters.push_back(r->counter);
        r->counter = -1;
        s->completed.push_back(r->id);
        s->n_completed++;
        s->frames_completed += F;
    }
    if (!done.empty()) s->cv_done.notify_all();
    done.clear();
}

// Pipeline: replay k runs while the host reads the counters of replay k-1,
// queues the result copies of requests that finished by then (they run after
// replay k on the engine stream) and completes the copies queued one cycle
// earlier.
void worker_main(ldpc_server *s) {
    (void)hipSetDevice(s->device);
    std::vector<Request *> draining[2], ready, uploaded[2];
    int64_t k = 0;
    bool prev_replay = false;
    for (;;) {
        const int cur = int(k & 1), prv = cur ^ 1;
        bool launched = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (!admit_locked(s, k)) {
                lk.unlock();
                fail_worker(s, "admission");
                return;
            }
            uploaded[cur].swap(s->staged_uploads);
            s->staged_uploads.clear();
            if (s->inflight.empty() && draining[0].empty() && draining[1].empty() && !prev_replay) {
                if (s->stop && s->waiting.empty()) return;
                s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
                continue;
            }
            launched = !s->inflight.empty();
        }
        if (launched) {
            hipError_t e = hipSuccess;
            if (ldpc_engine_step(s->engine, 1) != LDPC_OK) e = hipErrorUnknown;
            if (e == hipSuccess)
                e = hipMemcpyAsync(s->h_cnt[cur], s->counters, size_t(s->max_requests) * 4, hipMemcpyDeviceToHost,
                                   s->engine_stream);
            if (e == hipSuccess) e = hipEventRecord(s->ev_cnt[cur], s->engine_stream);
            if (e != hipSuccess) {
                set_error(std::string("engine step failed: ") + hipGetErrorString(e));
                fail_worker(s, "engine");
                return;
            }
        }
        if (prev_replay) {
            if (hipEventSynchronize(s->ev_cnt[prv]) != hipSuccess) {
                set_error("event wait failed");
                fail_worker(s, "poll");
                return;
            }
            // uploads queued before replay k-1 have completed: the engine waited for them
            {
                std::lock_guard<std::mutex> lk(s->mu);
                for (Request *r : uploaded[prv]) {
                    s->host_arena->release(r->stage_off, r->stage_bytes);
                    r->staged = false;
                }
            }
            uploaded[prv].clear();
            // result copies queued one cycle earlier
            if (!draining[prv].empty()) {
                if (hipEventSynchronize(s->ev_out[prv]) != hipSuccess) {
                    set_error("event wait failed");
                    fail_worker(s, "results");
                    return;
                }
                complete_requests(s, draining[prv]);
            }
            // requests finished by replay k-1: queue their result copies.  A request
            // admitted in cycle k took its counter after replay k-1's copy was
            // queued, so only requests admitted before cycle k are checked here.
            std::vector<Request *> fin;
            {
                std::lock_guard<std::mutex> lk(s->mu);
                for (size_t i = 0; i < s->inflight.size();) {
                    Request *r = s->inflight[i];
                    const uint32_t counted = uint32_t(s->h_cnt[prv][r->counter]) - r->counter_base;
                    if (r->admit_cycle <= k - 1 && counted >= uint32_t(r->frames)) {
                        fin.push_back(r);
                        s->inflight[i] = s->inflight.back();
                        s->inflight.pop_back();
                    } else {
                        i++;
                    }
                }
            }
            for (Request *r : fin) {
                const char *src = s->dev + r->dev_off + req_llr_bytes(r->frames, r->n);
                if (hipMemcpyAsync(s->pinned + r->out_off, src, req_out_bytes(r->frames, r->n),
                                   hipMemcpyDeviceToHost, s->engine_stream) != hipSuccess) {
                    set_error("result copy failed");
                    fail_worker(s, "results");
                    return;
                }
                draining[cur].push_back(r);
            }
            if (!fin.empty() && hipEventRecord(s->ev_out[cur], s->engine_stream) != hipSuccess) {
                set_error("event record failed");
                fail_worker(s, "results");
                return;
            }
        }
        if (!launched) {
            // nothing queued behind: finish outstanding copies now
            if (hipStreamSynchronize(s->engine_stream) != hipSuccess) {
                set_error("stream wait failed");
                fail_worker(s, "results");
                return;
            }
            for (int p = 0; p < 2; p++)
                if (!draining[p].empty()) complete_requests(s, draining[p]);
        }
        prev_replay = launched;
        k++;
    }
}

}  // namespace

extern "C" ldpc_status ldpc_server_create(const ldpc_graph *const *graphs, int32_t ngraphs, const int32_t *slots,
                                          int32_t max_iter, uint32_t flags, int64_t hbm_budget, int64_t host_budget,
                                          const ldpc_server_opts *opts, ldpc_server **out) {
    if (!out || !graphs || !slots || ngraphs < 1) { set_error("ldpc_server_create: bad argument"); return LDPC_E_INVAL; }
    if (hbm_budget < (1 << 20) || host_budget < (1 << 20)) {
        set_error("ldpc_server_create: budgets must be >= 1 MiB");
        return LDPC_E_INVAL;
    }
    ldpc_engine_opts eo{};
    int32_t maxreq = 4096;
    if (opts) {
        for (int32_t r : opts->reserved)
            if (r) { set_error("ldpc_server_create: reserved options must be 0"); return LDPC_E_INVAL; }
        eo.lane_slots = opts->lane_slots;
        eo.graph_steps = opts->graph_steps;
        eo.rule = opts->rule;
        eo.rule_param = opts->rule_param;
        eo.iters_per_step = opts->iters_per_step;
        if (opts->max_requests < 0) { set_error("ldpc_server_create: max_requests < 0"); return LDPC_E_INVAL; }
        if (opts->max_requests) maxreq = opts->max_requests;
    }
    std::vector<int32_t> caps(static_cast<size_t>(ngraphs));
    for (int32_t c = 0; c < ngraphs; c++) caps[size_t(c)] = std::max<int32_t>(4096, slots[c] > 0 ? 4 * slots[c] : 1);
    ldpc_server *s = new (std::nothrow) ldpc_server;
    if (!s) { set_error("ldpc_server_create: out of host memory"); return LDPC_E_NOMEM; }
    ldpc_status st = ldpc_engine_create(graphs, ngraphs, slots, caps.data(), max_iter, flags, &eo, &s->engine);
    if (st != LDPC_OK) { delete s; return st; }
    (void)hipGetDevice(&s->device);
    s->ngraphs = ngraphs;
    for (int32_t c = 0; c < ngraphs; c++) s->n.push_back(graphs[c]->n);
    s->queue_cap = caps;
    s->max_requests = maxreq;
    hipError_t e = hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&s->dev), size_t(hbm_budget));
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&s->counters), size_t(maxreq) * 4);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&s->pinned), size_t(host_budget), 0);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&s->h_counters), size_t(maxreq) * 4, 0);
    if (e == hipSuccess) e = hipMemset(s->counters, 0, size_t(maxreq) * 4);
    for (int p = 0; p < 2 && e == hipSuccess; p++) {
        e = hipHostMalloc(reinterpret_cast<void **>(&s->h_cnt[p]), size_t(maxreq) * 4, 0);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_cnt[p], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_out[p], hipEventDisableTiming);
    }
    if (e == hipSuccess && ldpc_engine_stream(s->engine, reinterpret_cast<void **>(&s->engine_stream)) != LDPC_OK)
        e = hipErrorUnknown;
    if (e != hipSuccess) {
        set_error(std::string("ldpc_server_create: ") + hipGetErrorString(e));
        (void)hipGetLastError();
        if (s->copy) (void)hipStreamDestroy(s->copy);
        if (s->dev) (void)hipFree(s->dev);
        if (s->counters) (void)hipFree(s->counters);
        if (s->pinned) (void)hipHostFree(s->pinned);
        if (s->h_counters) (void)hipHostFree(s->h_counters);
        ldpc_engine_destroy(s->engine);
        delete s;
        return e == hipErrorOutOfMemory ? LDPC_E_NOMEM : LDPC_E_DEVICE;
    }
    s->dev_arena.reset(new Arena(size_t(hbm_budget)));
    s->host_arena.reset(new Arena(size_t(host_budget)));
    for (int32_t i = maxreq - 1; i >= 0; i--) s->free_counters.push_back(i);
    s->counter_total.assign(size_t(maxreq), 0u);
    try {
        s->worker = std::thread(worker_main, s);
    } catch (...) {
        set_error("ldpc_server_create: cannot start the worker thread");
        ldpc_engine_destroy(s->engine);
        delete s;
        return LDPC_E_NOMEM;
    }
    *out = s;
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_server_submit(ldpc_server *s, int32_t graph, const float *llr, int32_t frames,
                                          int64_t *id) {
    if (!s || !llr || !id || graph < 0 || graph >= s->ngraphs || frames < 1) {
        set_error("ldpc_server_submit: bad argument");
        return LDPC_E_INVAL;
    }
    const int32_t nn = s->n[size_t(graph)];
    Request *r = new (std::nothrow) Request;
    if (!r) { set_error("ldpc_server_submit: out of host memory"); return LDPC_E_NOMEM; }
    r->graph = graph;
    r->frames = frames;
    r->n = nn;
    r->dev_bytes = req_dev_bytes(frames, nn);
    r->stage_bytes = size_t(frames) * nn * 4;
    r->out_bytes = req_out_bytes(frames, nn);
    if (r->dev_bytes > s->dev_arena->size() || r->stage_bytes + r->out_bytes + 512 > s->host_arena->size() ||
        frames > s->queue_cap[size_t(graph)]) {
        delete r;
        set_error("ldpc_server_submit: request larger than the server's memory budgets");
        return LDPC_E_INVAL;
    }
    r->t_submit = Clock::now();
    // The LLRs go straight into the pinned staging arena when every request
    // already waiting is staged there and the arena stays at most half full;
    // otherwise into host memory (the worker stages them at admission).  The
    // decision and the queue position are taken under one lock, so a request
    // staged in host memory never has a pinned-staged request behind it, and
    // the half of the arena left free always holds the head request's outputs:
    // the queue never waits on memory that only a later request could release.
    // The copy itself runs after the lock; the worker admits a request only
    // once it is marked ready.
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) {
            delete r;
            set_error("ldpc_server_submit: server is stopping: " + s->worker_error);
            return LDPC_E_INVAL;
        }
        if (s->unstaged_waiting == 0 && s->host_arena->used() + r->stage_bytes <= s->host_arena->size() / 2)
            r->prestaged = s->host_arena->alloc(r->stage_bytes, &r->stage_off);
        if (!r->prestaged) {
            try {
                r->llr.reserve(size_t(frames) * nn);
            } catch (const std::bad_alloc &) {
                delete r;
                set_error("ldpc_server_submit: out of host memory");
                return LDPC_E_NOMEM;
            }
            s->unstaged_waiting++;
        }
        r->id = s->next_id++;
        s->all[r->id] = r;
        s->waiting.push_back(r);
        s->n_submitted++;
    }
    if (r->prestaged) std::memcpy(s->pinned + r->stage_off, llr, size_t(frames) * nn * 4);
    else r->llr.assign(llr, llr + size_t(frames) * nn);   // within the reserved capacity
    const int64_t rid = r->id;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r->ready = true;
    }
    s->cv_work.notify_one();
    *id = rid;
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_server_poll(ldpc_server *s, int64_t *ids, int32_t max_ids, int32_t *count,
                                        int32_t wait_ms) {
    if (!s || !count || max_ids < 0 || (max_ids > 0 && !ids)) { set_error("ldpc_server_poll: bad argument"); return LDPC_E_INVAL; }
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->completed.empty() && wait_ms > 0 && s->worker_error.empty())
        s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->completed.empty() || s->stop; });
    int32_t k = 0;
    while (k < max_ids && !s->completed.empty()) {
        ids[k++] = s->completed.front();
        s->completed.pop_front();
    }
    *count = k;
    if (!s->worker_error.empty()) {
        set_error("ldpc_server_poll: worker failed: " + s->worker_error);
        return LDPC_E_DEVICE;
    }
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_server_result(ldpc_server *s, int64_t id, uint8_t *bits, uint8_t *ok, int32_t *iters,
                                          double *latency_s) {
    if (!s) { set_error("ldpc_server_result: NULL server"); return LDPC_E_INVAL; }
    Request *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->all.find(id);
        if (it == s->all.end() || it->second->bits.empty()) {
            set_error("ldpc_server_result: unknown or unfinished request");
            return LDPC_E_INVAL;
        }
        r = it->second;
        s->all.erase(it);
    }
    if (bits) std::memcpy(bits, r->bits.data(), r->bits.size());
    if (ok) std::memcpy(ok, r->ok.data(), r->ok.size());
    if (iters) std::memcpy(iters, r->iters.data(), r->iters.size() * 4);
    if (latency_s) *latency_s = std::chrono::duration<double>(r->t_done - r->t_submit).count();
    delete r;
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_server_stats(ldpc_server *s, int64_t *stats) {
    if (!s || !stats) { set_error("ldpc_server_stats: bad argument"); return LDPC_E_INVAL; }
    std::lock_guard<std::mutex> lk(s->mu);
    stats[0] = s->n_submitted;
    stats[1] = s->n_admitted;
    stats[2] = s->n_completed;
    stats[3] = s->frames_completed;
    stats[4] = int64_t(s->waiting.size());
    stats[5] = int64_t(s->inflight.size());
    stats[6] = int64_t(s->dev_arena->used());
    stats[7] = int64_t(s->dev_arena->peak());
    return LDPC_OK;
}

extern "C" ldpc_status ldpc_server_destroy(ldpc_server *s) {
    if (!s) return LDPC_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    ldpc_engine_destroy(s->engine);
    (void)hipStreamSynchronize(s->copy);
    (void)hipStreamDestroy(s->copy);
    (void)hipFree(s->dev);
    (void)hipFree(s->counters);
    (void)hipHostFree(s->pinned);
    (void)hipHostFree(s->h_counters);
    for (int p = 0; p < 2; p++) {
        if (s->h_cnt[p]) (void)hipHostFree(s->h_cnt[p]);
        if (s->ev_cnt[p]) (void)hipEventDestroy(s->ev_cnt[p]);
        if (s->ev_out[p]) (void)hipEventDestroy(s->ev_out[p]);
    }
    (void)hipGetLastError();
    for (auto &kv : s->all) delete kv.second;
    delete s;
    return LDPC_OK;
}
