// Batch and serving front ends of the C ABI.
//
// project_batch: every problem gets its own hierarchy (reused across calls
// from a process-wide cache keyed by shape); all batchable problems are
// solved together by the batched engine, V-cycle by V-cycle.
//
// Serving: a worker thread owns a stream and a pool of resident hierarchies.
// Requests wait in a queue; at every V-cycle boundary the worker admits as
// many queued requests as the in-flight cap and the HBM budget allow
// (resident hierarchies count against the budget; idle ones of other shapes
// are released when room is needed), sets them up, and runs the next round
// for everything in flight.  A request therefore overlaps on the device with
// requests that arrived earlier (continuous batching), and its result is the
// one mac_project gives for it alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "batch.h"
#include "mg_internal.h"
#include "runtime.h"

namespace mg {
namespace {

using ShapeKey = std::tuple<int, int, int, int, int, int, int, int, double>;

ShapeKey key_of(const mg_params& p, int device) {
    return ShapeKey(device, p.n[0], p.n[1], p.n[2], p.bc[0], p.bc[1], p.bc[2], p.precision, p.dx);
}

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Idle hierarchies kept for reuse, keyed by device and shape.
struct Pool {
    std::map<ShapeKey, std::vector<mg_hierarchy*>> idle;
    size_t idle_bytes = 0;
    size_t busy_bytes = 0;

    ~Pool() { clear(); }
    void clear() {
        for (auto& kv : idle)
            for (auto* h : kv.second) destroy(h);
        idle.clear();
        idle_bytes = 0;
    }
    bool has_idle(const mg_params& p, int dev) {
        auto it = idle.find(key_of(p, dev));
        return it != idle.end() && !it->second.empty();
    }
    int acquire(const mg_params& p, int dev, mg_hierarchy** out) {
        auto& v = idle[key_of(p, dev)];
        if (!v.empty()) {
            // oldest first: a repeated batch gets the same hierarchies in the
            // same order (and replays its captured rounds)
            *out = v.front();
            v.erase(v.begin());
            idle_bytes -= (*out)->ws_bytes;
            busy_bytes += (*out)->ws_bytes;
            (*out)->p = p;
            return MG_OK;
        }
        int rc = setup(&p, nullptr, 0, out);
        if (rc == MG_OK) busy_bytes += (*out)->ws_bytes;
        return rc;
    }
    void release(mg_hierarchy* h) {
        busy_bytes -= h->ws_bytes;
        idle_bytes += h->ws_bytes;
        idle[key_of(h->p, h->device)].push_back(h);
    }
    // free idle hierarchies (other shapes first) until idle_bytes <= target
    void trim(size_t target, const ShapeKey* keep = nullptr) {
        for (int pass = 0; pass < 2 && idle_bytes > target; ++pass)
            for (auto& kv : idle) {
                if (pass == 0 && keep && kv.first == *keep) continue;
                while (!kv.second.empty() && idle_bytes > target) {
                    idle_bytes -= kv.second.back()->ws_bytes;
                    destroy(kv.second.back());
                    kv.second.pop_back();
                }
            }
    }
};

std::mutex g_batch_mu;
Pool* g_batch_pool = nullptr;
Engine* g_batch_engine = nullptr;
constexpr size_t kBatchPoolCap = (size_t)64 << 30;   // idle bytes kept between project_batch calls
constexpr size_t kStagingBytes = (size_t)8 << 20;

int solo(mg_hierarchy* H, const mg_problem& p, mg_stats* st, hipStream_t s) {
    return project(H, p.rho, p.beta0_cc, p.beta0_edge, p.S, p.u, p.v, p.w, p.phi, st, s);
}

// ---------------------------------------------------------------------------
struct Server {
    size_t budget = 0;
    int max_inflight = 1;
    int device = 0;
    hipStream_t stream = nullptr;
    Engine engine;
    Pool pool;                                  // worker-thread only
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<Job*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next_ticket = 1;
    bool stop = false;
    double submitted = 0, completed = 0, peak = 0;
    size_t inflight_n = 0;
    size_t resident = 0;
    std::thread worker;
    int fatal = MG_OK;

    // publish a finished job: t_done (written under the lock, after every
    // other field) is what pollers test
    void finish(Job* j) {
        const double t = now_s();
        {
            std::lock_guard<std::mutex> lk(mu);
            j->st.ms_total = (t - j->t_submit) * 1e3;
            j->st.ms_other = std::max(0.0, j->st.ms_total - j->st.ms_smooth);
            j->t_done = t;
            completed += 1;
            inflight_n -= 1;
        }
        done_cv.notify_all();
    }

    void run() {
        hipSetDevice(device);
        std::vector<Job*> active;
        for (;;) {
            std::vector<Job*> fresh;
            std::deque<Job*> cand;
            {
                // under the lock only the queue: take the requests that the
                // in-flight cap allows (the pool is the worker's alone)
                std::unique_lock<std::mutex> lk(mu);
                if (active.empty() && queue.empty()) cv.wait(lk, [&] { return stop || !queue.empty(); });
                if (stop && active.empty() && queue.empty()) return;
                while (!queue.empty() && active.size() + cand.size() < (size_t)max_inflight) {
                    cand.push_back(queue.front());
                    queue.pop_front();
                }
            }
            // admission at the V-cycle boundary against the HBM budget, in
            // arrival order; hierarchies are allocated (and idle ones of other
            // shapes released) without holding the lock
            while (!cand.empty()) {
                Job* j = cand.front();
                const bool reuse = pool.has_idle(j->pr.p, device);
                const size_t need = reuse ? 0 : j->bytes;
                if (pool.busy_bytes + pool.idle_bytes + need > budget) {
                    const ShapeKey k = key_of(j->pr.p, device);
                    size_t target = budget > pool.busy_bytes + need ? budget - pool.busy_bytes - need : 0;
                    pool.trim(target, &k);
                    if (pool.busy_bytes + pool.idle_bytes + need > budget) break;   // wait for completions
                }
                cand.pop_front();
                j->t_admit = now_s();
                // reserve the hierarchy now, so the next request in this pass
                // sees the pool as it will be
                j->status = pool.acquire(j->pr.p, device, &j->H);
                fresh.push_back(j);
            }
            {
                std::lock_guard<std::mutex> lk(mu);
                for (auto it = cand.rbegin(); it != cand.rend(); ++it) queue.push_front(*it);   // not admitted yet
                inflight_n += fresh.size();
                peak = std::max(peak, (double)inflight_n);
            }
            std::vector<Job*> setup_list;
            for (Job* j : fresh) {
                if (j->status != MG_OK) {
                    j->st.status = j->status;
                    j->stage = Job::kDone;
                    j->H = nullptr;
                    finish(j);
                    continue;
                }
                if (!batchable(j->H)) {
                    // solved on its own, between rounds
                    j->status = solo(j->H, j->pr, &j->st, stream);
                    j->st.status = j->status;
                    j->stage = Job::kDone;
                    pool.release(j->H);
                    j->H = nullptr;
                    finish(j);
                    continue;
                }
                setup_list.push_back(j);
                active.push_back(j);
            }
            int rc = engine.setup_new(setup_list, stream);
            if (rc == MG_OK && !active.empty()) rc = engine.round(active, stream);
            if (rc != MG_OK) {
                // a device error: fail everything in flight, keep serving
                for (Job* j : active)
                    if (j->stage != Job::kDone) {
                        j->st.status = j->status = rc;
                        j->stage = Job::kDone;
                    }
                hipStreamSynchronize(stream);
                engine.staging.off = 0;
            }
            std::vector<Job*> still;
            for (Job* j : active) {
                if (j->stage == Job::kDone) {
                    if (j->H) {
                        pool.release(j->H);
                        j->H = nullptr;
                    }
                    finish(j);
                } else {
                    still.push_back(j);
                }
            }
            active.swap(still);
            {
                std::lock_guard<std::mutex> lk(mu);
                resident = pool.busy_bytes + pool.idle_bytes;
            }
        }
    }
};

}  // namespace
}  // namespace mg

using namespace mg;

extern "C" {

int project_batch(int32_t count, const mg_problem* probs, mg_stats* stats, void* stream) {
    if (count < 0 || (count > 0 && !probs)) {
        set_error("bad batch arguments");
        return MG_ERR_INVALID_ARG;
    }
    if (count == 0) return MG_OK;
    hipStream_t st = (hipStream_t)stream;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    try {
        if (!g_batch_pool) g_batch_pool = new Pool();
        if (!g_batch_engine) {
            g_batch_engine = new Engine();
            g_batch_engine->graph_mode = 1;      // a batch's rounds recur: capture at first sight
            if (g_batch_engine->staging.init(kStagingBytes) != MG_OK) {
                delete g_batch_engine;
                g_batch_engine = nullptr;
                set_error("staging allocation failed");
                return MG_ERR_OOM;
            }
        }
        int dev = 0;
        hipGetDevice(&dev);
        std::vector<Job> jobs((size_t)count);
        std::vector<Job*> batched;
        int worst = MG_OK;
        hipEvent_t e0, e1;
        hipEventCreate(&e0);
        hipEventCreate(&e1);
        hipEventRecord(e0, st);
        for (int i = 0; i < count; ++i) {
            Job& j = jobs[i];
            j.pr = probs[i];
            std::memset(&j.st, 0, sizeof j.st);
            int rc = validate_params(&j.pr.p);
            if (rc == MG_OK && (!j.pr.rho || !j.pr.beta0_cc || !j.pr.beta0_edge || !j.pr.S || !j.pr.u || !j.pr.v ||
                                !j.pr.w)) {
                set_error("null field pointer in a batch problem");
                rc = MG_ERR_INVALID_ARG;
            }
            if (rc == MG_OK) rc = g_batch_pool->acquire(j.pr.p, dev, &j.H);
            if (rc != MG_OK) {
                j.st.status = j.status = rc;
                j.stage = Job::kDone;
                continue;
            }
            if (!batchable(j.H)) {
                j.status = solo(j.H, j.pr, &j.st, st);
                j.st.status = j.status;
                j.stage = Job::kDone;
                continue;
            }
            batched.push_back(&j);
        }
        int rc = g_batch_engine->setup_new(batched, st);
        while (rc == MG_OK) {
            bool busy = false;
            for (Job* j : batched) busy |= j->stage == Job::kSolve || j->stage == Job::kFinish;
            if (!busy) break;
            rc = g_batch_engine->round(batched, st);
        }
        hipEventRecord(e1, st);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        g_batch_engine->staging.off = 0;
        for (int i = 0; i < count; ++i) {
            Job& j = jobs[i];
            if (rc != MG_OK && j.stage != Job::kDone) j.st.status = j.status = rc;
            j.st.ms_total = ms;
            j.st.ms_other = std::max(0.0, (double)ms - j.st.ms_smooth);
            if (stats) stats[i] = j.st;
            if (j.H) g_batch_pool->release(j.H);
            if (j.status != MG_OK && worst == MG_OK) worst = j.status;
        }
        g_batch_pool->trim(kBatchPoolCap);
        return rc != MG_OK ? rc : worst;
    } catch (...) {
        set_error("internal error in project_batch");
        return MG_ERR_HIP;
    }
}

int serve_create(size_t hbm_budget_bytes, int32_t max_inflight, void** server) {
    if (!server || max_inflight < 1) {
        set_error("bad serve_create arguments");
        return MG_ERR_INVALID_ARG;
    }
    Server* S = new (std::nothrow) Server();
    if (!S) return MG_ERR_OOM;
    S->budget = hbm_budget_bytes;
    S->max_inflight = max_inflight;
    S->engine.graph_mode = 2;                    // capture an active set once it recurs
    hipGetDevice(&S->device);
    hipError_t e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete S;
        return hip_fail(e, "hipStreamCreateWithFlags", __LINE__);
    }
    if (S->engine.staging.init(kStagingBytes) != MG_OK) {
        hipStreamDestroy(S->stream);
        delete S;
        set_error("staging allocation failed");
        return MG_ERR_OOM;
    }
    S->worker = std::thread([S] { S->run(); });
    *server = S;
    return MG_OK;
}

int serve_submit(void* server, const mg_problem* prob, uint64_t* ticket) {
    Server* S = (Server*)server;
    if (!S || !prob || !ticket) {
        set_error("bad serve_submit arguments");
        return MG_ERR_INVALID_ARG;
    }
    int rc = validate_params(&prob->p);
    if (rc) return rc;
    if (!prob->rho || !prob->beta0_cc || !prob->beta0_edge || !prob->S || !prob->u || !prob->v || !prob->w) {
        set_error("null field pointer");
        return MG_ERR_INVALID_ARG;
    }
    size_t need = workspace_bytes(&prob->p);
    if (need > S->budget) {
        set_error("request needs more device memory than the server budget");
        return MG_ERR_BUDGET;
    }
    auto j = std::make_unique<Job>();
    j->pr = *prob;
    j->bytes = need;
    j->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        j->ticket = S->next_ticket++;
        *ticket = j->ticket;
        S->queue.push_back(j.get());
        S->jobs.emplace(*ticket, std::move(j));
        S->submitted += 1;
    }
    S->cv.notify_one();
    return MG_OK;
}

int serve_poll(void* server, uint64_t ticket, mg_stats* out) {
    Server* S = (Server*)server;
    if (!S) return MG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) {
        set_error("unknown ticket");
        return MG_ERR_INVALID_ARG;
    }
    Job* j = it->second.get();
    if (j->t_done == 0.0) return MG_PENDING;
    if (out) *out = j->st;
    const int status = j->status;
    if (j->waiters == 0) S->jobs.erase(it);   // final status returned: the ticket is released
    return status;
}

int serve_wait(void* server, uint64_t ticket, mg_stats* out) {
    Server* S = (Server*)server;
    if (!S) return MG_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->jobs.find(ticket);
    if (it == S->jobs.end()) {
        set_error("unknown ticket");
        return MG_ERR_INVALID_ARG;
    }
    Job* j = it->second.get();
    j->waiters += 1;
    S->done_cv.wait(lk, [&] { return j->t_done != 0.0; });
    j->waiters -= 1;
    if (out) *out = j->st;
    const int status = j->status;
    if (j->waiters == 0) S->jobs.erase(ticket);   // final status returned: the ticket is released
    return status;
}

int serve_counters(void* server, double out[6]) {
    Server* S = (Server*)server;
    if (!S || !out) return MG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    out[0] = S->submitted;
    out[1] = S->completed;
    out[2] = (double)S->queue.size();
    out[3] = (double)S->inflight_n;
    out[4] = (double)S->resident;
    out[5] = S->peak;
    return MG_OK;
}

int serve_destroy(void* server) {
    Server* S = (Server*)server;
    if (!S) return MG_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->worker.joinable()) S->worker.join();
    hipStreamSynchronize(S->stream);
    S->pool.clear();
    S->engine.staging.release();
    hipStreamDestroy(S->stream);
    delete S;
    return MG_OK;
}

}  // extern "C"
