// pj_serve.cpp -- serving loop: continuous batching of query requests over a resident index.
//
// Threads: the caller(s) submit and wait; one scheduler thread admits queued requests into device
// batches; one worker thread per slot runs its batch on the slot's own HIP stream with its own
// device scratch, so batches on different slots overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/passjoin.h"
#include "pj_host_internal.h"

namespace pj {

struct Request {
    int64_t id = 0;
    int64_t n = 0;
    std::vector<uint8_t> bytes;
    std::vector<int32_t> offs;
    std::vector<int32_t> taus;
    int64_t footprint = 0;
    // results
    std::vector<uint64_t> pairs;   // (q << 32 | s), q local
    int status = PJ_OK;
    std::string error;
    bool done = false;
    bool waiting_noted = false;    // its current wait at the head of the queue is counted
    pj_request_info info{};
};

struct Batch {
    std::vector<std::shared_ptr<Request>> reqs;
    int64_t queries = 0;
    int64_t footprint = 0;
};

struct Slot {
    int index = 0;
    hipStream_t stream = nullptr;
    std::thread th;
    std::unique_ptr<Batch> job;     // guarded by Server::mu
    bool busy = false;
    GraphPlan* plan = nullptr;      // captured pipeline (worker thread only)
    bool plan_failed = false;
};

}  // namespace pj

struct pj_server {
    const pj_index* idx = nullptr;
    pj_server_config cfg{};
    std::string tune_cache;              // owned copy of cfg.tune_cache
    int tau_min = 0, tau_max = -1;
    std::chrono::steady_clock::time_point t0;
    std::mutex mu;
    std::condition_variable cv_sched;    // queue or slot/memory changes
    std::condition_variable cv_done;     // a request finished
    std::condition_variable cv_slot;     // a slot received a job or stop
    std::deque<std::shared_ptr<pj::Request>> queue;
    std::unordered_map<int64_t, std::shared_ptr<pj::Request>> live;
    std::vector<std::unique_ptr<pj::Slot>> slots;
    std::thread scheduler;
    int64_t next_id = 0;
    int64_t inflight_bytes = 0;
    int64_t admit_budget = 0;            // the budget less the slots' fixed buffers (0: none)
    bool stopping = false;
    bool sched_done = false;
    int device = 0;

    double now_ms() const
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
            .count();
    }
};

namespace pj {

static void run_batch(pj_server* S, Slot& slot, Batch& B)
{
    // merge the requests' queries into one set; request r owns queries [q0_r, q0_r + n_r)
    std::vector<uint8_t> bytes;
    std::vector<int32_t> offs(1, 0);
    std::vector<int32_t> taus;
    std::vector<int64_t> q0;
    for (auto& r : B.reqs) {
        q0.push_back((int64_t)taus.size());
        for (int64_t q = 0; q < r->n; ++q) {
            bytes.insert(bytes.end(), r->bytes.begin() + r->offs[q], r->bytes.begin() + r->offs[q + 1]);
            offs.push_back((int32_t)bytes.size());
            taus.push_back(r->taus[q]);
        }
    }
    pj_strings Q{(int64_t)taus.size(), bytes.empty() ? nullptr : bytes.data(), offs.data()};
    std::vector<uint64_t> pairs;
    pj_stats st{};
    int status = PJ_OK;
    std::string err;
    const char* tc = S->tune_cache.empty() ? nullptr : S->tune_cache.c_str();
    try {
        bool done = false;
        if (!S->cfg.eager) {
            if (!slot.plan && !slot.plan_failed) {
                try {
                    slot.plan = graph_plan_create(S->idx, S->cfg.max_batch_queries, slot.stream, tc);
                } catch (const Error&) {
                    slot.plan_failed = true;      // this slot runs its batches uncaptured
                }
            }
            if (slot.plan) done = graph_plan_run(slot.plan, &Q, taus.data(), pairs, st);
        }
        if (!done) {
            pairs.clear();
            st = pj_stats{};
            run_query_batch(S->idx, &Q, taus.data(), pairs, st, slot.stream, tc);
        }
    } catch (const Error& e) {
        status = e.code;
        err = e.msg;
    } catch (const std::bad_alloc&) {
        status = PJ_ENOMEM;
        err = "host allocation failed";
    }
    // split the sorted pairs by request
    size_t k = 0;
    const double t_done = S->now_ms();
    for (size_t r = 0; r < B.reqs.size(); ++r) {
        auto& R = B.reqs[r];
        const uint64_t lo = (uint64_t)q0[r], hi = lo + (uint64_t)R->n;
        while (k < pairs.size() && (pairs[k] >> 32) < lo) ++k;
        while (k < pairs.size() && (pairs[k] >> 32) < hi) {
            R->pairs.push_back(((pairs[k] >> 32) - lo) << 32 | (pairs[k] & 0xffffffffu));
            ++k;
        }
        R->status = status;
        R->error = err;
        R->info.t_done_ms = t_done;
        R->info.batch_requests = (int32_t)B.reqs.size();
        R->info.slot = slot.index;
    }
}

static void worker_main(pj_server* S, Slot* slot)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        std::unique_ptr<Batch> job;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_slot.wait(lk, [&] { return slot->job != nullptr || S->sched_done; });
            if (!slot->job) break;
            job = std::move(slot->job);
        }
        run_batch(S, *slot, *job);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (auto& r : job->reqs) r->done = true;
            S->inflight_bytes -= job->footprint;
            slot->busy = false;
        }
        S->cv_done.notify_all();
        S->cv_sched.notify_all();
    }
    if (slot->plan) {
        graph_plan_destroy(slot->plan);
        slot->plan = nullptr;
    }
    release_thread_workspace();
}

static void scheduler_main(pj_server* S)
{
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        Slot* free_slot = nullptr;
        for (auto& s : S->slots)
            if (!s->busy) {
                free_slot = s.get();
                break;
            }
        const int64_t budget = S->admit_budget;
        bool head_fits = !S->queue.empty() &&
                         (budget <= 0 || S->inflight_bytes + S->queue.front()->footprint <= budget);
        if (!S->queue.empty() && !(free_slot && head_fits) && !S->queue.front()->waiting_noted) {
            // the head of the queue has to wait: for a slot, or (a slot being free) for memory
            auto& h = S->queue.front();
            h->waiting_noted = true;
            h->info.deferrals += 1;
            if (free_slot) h->info.deferred_by_memory = 1;
        }
        if (free_slot && head_fits) {
            std::unique_ptr<Batch> B(new Batch());
            const double t_admit = S->now_ms();
            while (!S->queue.empty()) {
                auto& r = S->queue.front();
                bool fits_q = B->reqs.empty() || B->queries + r->n <= S->cfg.max_batch_queries;
                bool fits_m = budget <= 0 || S->inflight_bytes + B->footprint + r->footprint <= budget;
                if (!fits_q || !fits_m) break;
                r->info.t_admit_ms = t_admit;
                B->queries += r->n;
                B->footprint += r->footprint;
                B->reqs.push_back(r);
                S->queue.pop_front();
            }
            S->inflight_bytes += B->footprint;
            free_slot->busy = true;
            free_slot->job = std::move(B);
            S->cv_slot.notify_all();
            continue;
        }
        if (S->stopping && S->queue.empty()) break;
        S->cv_sched.wait(lk);
    }
    S->sched_done = true;
    S->cv_slot.notify_all();
}

}  // namespace pj

using namespace pj;

extern "C" {

int pj_server_start(const pj_index* idx, const pj_server_config* cfg, pj_server** out)
{
    try {
        if (!out) throw Error(PJ_EINVAL, "null output");
        *out = nullptr;
        if (!idx) throw Error(PJ_EINVAL, "null index");
        pj_server_config c{2, 256, 0, nullptr, 0};
        if (cfg) c = *cfg;
        if (c.slots < 1 || c.slots > 64) throw Error(PJ_EINVAL, "slots must be in [1, 64]");
        if (c.max_batch_queries < 1) throw Error(PJ_EINVAL, "max_batch_queries must be >= 1");
        if (c.mem_budget_bytes < 0) throw Error(PJ_EINVAL, "negative memory budget");
        std::unique_ptr<pj_server> S(new pj_server());
        S->idx = idx;
        S->cfg = c;
        if (c.tune_cache) S->tune_cache = c.tune_cache;
        S->cfg.tune_cache = nullptr;
        index_taus(idx, &S->tau_min, &S->tau_max);
        if (c.mem_budget_bytes > 0) {
            // each slot's captured pipeline holds fixed-capacity buffers for the server's
            // lifetime: they come off the budget before any request is admitted
            const int64_t fixed = c.eager ? 0 : (int64_t)c.slots *
                                                    graph_plan_device_bytes(c.max_batch_queries);
            if (fixed >= c.mem_budget_bytes)
                throw Error(PJ_ENOMEM, "memory budget %lld does not hold the %d slots' fixed "
                            "buffers (%lld bytes)", (long long)c.mem_budget_bytes, c.slots,
                            (long long)fixed);
            S->admit_budget = c.mem_budget_bytes - fixed;
        }
        S->t0 = std::chrono::steady_clock::now();
        hip_check(hipGetDevice(&S->device), "hipGetDevice");
        for (int k = 0; k < c.slots; ++k) {
            std::unique_ptr<Slot> sl(new Slot());
            sl->index = k;
            hip_check(hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking), "hipStreamCreate");
            S->slots.push_back(std::move(sl));
        }
        pj_server* raw = S.get();
        for (auto& sl : S->slots) sl->th = std::thread(worker_main, raw, sl.get());
        S->scheduler = std::thread(scheduler_main, raw);
        *out = S.release();
        t_last_error.clear();
        return PJ_OK;
    } catch (const Error& e) {
        t_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        t_last_error = "host allocation failed";
        return PJ_ENOMEM;
    }
}

int64_t pj_server_submit(pj_server* S, const pj_strings* Q, const int32_t* taus)
{
    try {
        if (!S) throw Error(PJ_EINVAL, "null server");
        validate_host_strings(Q, "Q");
        if (Q->n > 0 && !taus) throw Error(PJ_EINVAL, "null taus");
        auto r = std::make_shared<Request>();
        r->n = Q->n;
        r->offs.assign(Q->offsets, Q->offsets + Q->n + 1);
        if (Q->offsets[Q->n] > 0) r->bytes.assign(Q->bytes, Q->bytes + Q->offsets[Q->n]);
        r->taus.assign(taus, taus + Q->n);
        for (int64_t q = 0; q < Q->n; ++q) {
            if (taus[q] < S->tau_min || taus[q] > S->tau_max)
                throw Error(PJ_ERANGE, "query %lld: tau %d outside the index range [%d, %d]",
                            (long long)q, taus[q], S->tau_min, S->tau_max);
            r->footprint += query_footprint(S->idx, Q->offsets[q + 1] - Q->offsets[q], taus[q]);
        }
        if (S->admit_budget > 0 && r->footprint > S->admit_budget)
            throw Error(PJ_ENOMEM, "request footprint %lld exceeds the server budget %lld "
                        "(after the slots' fixed buffers)", (long long)r->footprint,
                        (long long)S->admit_budget);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->stopping) throw Error(PJ_EINVAL, "server is stopping");
            r->id = S->next_id++;
            r->info.t_submit_ms = S->now_ms();
            r->info.footprint_bytes = r->footprint;
            S->live[r->id] = r;
            S->queue.push_back(r);
        }
        S->cv_sched.notify_all();
        t_last_error.clear();
        return r->id;
    } catch (const Error& e) {
        t_last_error = e.msg;
        return e.code;
    } catch (const std::bad_alloc&) {
        t_last_error = "host allocation failed";
        return PJ_ENOMEM;
    }
}

int pj_server_wait(pj_server* S, int64_t request, pj_pairs* out, pj_request_info* info)
{
    if (out) {
        out->count = 0;
        out->a = out->b = nullptr;
        out->on_device = 0;
    }
    if (!S || !out) {
        t_last_error = "null argument";
        return PJ_EINVAL;
    }
    std::shared_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(S->mu);
        auto it = S->live.find(request);
        if (it == S->live.end()) {
            t_last_error = "unknown or already collected request id";
            return PJ_EINVAL;
        }
        r = it->second;
        // the wait releases the mutex: submits may rehash `live` meanwhile, so no iterator is
        // kept across it; of two waiters on one id only the first to return collects it
        S->cv_done.wait(lk, [&] { return r->done; });
        auto again = S->live.find(request);
        if (again == S->live.end() || again->second != r) {
            t_last_error = "request already collected by another waiter";
            return PJ_EINVAL;
        }
        S->live.erase(again);
    }
    if (info) *info = r->info;
    if (r->status != PJ_OK) {
        t_last_error = r->error;
        return r->status;
    }
    const size_t M = r->pairs.size();
    const size_t bytes = sizeof(int32_t) * std::max<size_t>(M, 1);
    out->a = (int32_t*)malloc(bytes);
    out->b = (int32_t*)malloc(bytes);
    if (!out->a || !out->b) {
        free(out->a);
        free(out->b);
        out->a = out->b = nullptr;
        t_last_error = "host allocation failed";
        return PJ_ENOMEM;
    }
    for (size_t k = 0; k < M; ++k) {
        out->a[k] = (int32_t)(r->pairs[k] >> 32);
        out->b[k] = (int32_t)(r->pairs[k] & 0xffffffffu);
    }
    out->count = (int64_t)M;
    t_last_error.clear();
    return PJ_OK;
}

int pj_server_stop(pj_server* S)
{
    if (!S) return PJ_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stopping = true;
    }
    S->cv_sched.notify_all();
    if (S->scheduler.joinable()) S->scheduler.join();
    S->cv_slot.notify_all();
    for (auto& sl : S->slots)
        if (sl->th.joinable()) sl->th.join();
    for (auto& sl : S->slots)
        if (sl->stream) (void)hipStreamDestroy(sl->stream);
    delete S;
    return PJ_OK;
}

}  // extern "C"
