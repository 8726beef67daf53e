// Batch and serving front ends (first version: problems run one after the
// other on the caller's stream / the server's worker stream, each on a
// hierarchy cached by shape).
#include <hip/hip_runtime.h>

#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>

#include "mg_internal.h"
#include "runtime.h"

namespace mg {
namespace {

using ShapeKey = std::tuple<int, int, int, int, int, int, int, double>;

ShapeKey key_of(const mg_params& p) {
    return ShapeKey(p.n[0], p.n[1], p.n[2], p.bc[0], p.bc[1], p.bc[2], p.precision, p.dx);
}

// Hierarchies kept resident, keyed by shape / bc / precision / dx.
struct HierarchyCache {
    std::map<ShapeKey, std::vector<mg_hierarchy*>> free_list;
    size_t bytes = 0;
    ~HierarchyCache() { clear(); }
    void clear() {
        for (auto& kv : free_list)
            for (auto* h : kv.second) destroy(h);
        free_list.clear();
        bytes = 0;
    }
    int acquire(const mg_params& p, mg_hierarchy** out) {
        auto& v = free_list[key_of(p)];
        if (!v.empty()) {
            *out = v.back();
            v.pop_back();
            (*out)->p = p;
            return MG_OK;
        }
        int rc = setup(&p, nullptr, 0, out);
        if (rc == MG_OK) bytes += (*out)->ws_bytes;
        return rc;
    }
    void release(mg_hierarchy* h) { free_list[key_of(h->p)].push_back(h); }
};

int solve_one(HierarchyCache& cache, const mg_problem& pr, mg_stats* st, hipStream_t s) {
    mg_hierarchy* h = nullptr;
    int rc = cache.acquire(pr.p, &h);
    if (rc != MG_OK) {
        if (st) {
            std::memset(st, 0, sizeof *st);
            st->status = rc;
        }
        return rc;
    }
    rc = project(h, pr.rho, pr.beta0_cc, pr.beta0_edge, pr.S, pr.u, pr.v, pr.w, pr.phi, st, s);
    cache.release(h);
    return rc;
}

struct Server {
    size_t budget;
    int max_inflight;
    HierarchyCache cache;
    std::mutex mu;
    std::condition_variable cv, done_cv;
    std::deque<std::pair<uint64_t, mg_problem>> queue;
    std::unordered_map<uint64_t, std::pair<int, mg_stats>> results;
    uint64_t next_ticket = 1;
    bool stop = false;
    double submitted = 0, completed = 0, inflight = 0, peak = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    std::thread worker;

    void run() {
        hipSetDevice(device);
        for (;;) {
            std::pair<uint64_t, mg_problem> job;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv.wait(lk, [&] { return stop || !queue.empty(); });
                if (queue.empty() && stop) return;
                job = queue.front();
                queue.pop_front();
                inflight = 1;
                if (inflight > peak) peak = inflight;
            }
            mg_stats st;
            std::memset(&st, 0, sizeof st);
            int rc = solve_one(cache, job.second, &st, stream);
            {
                std::lock_guard<std::mutex> lk(mu);
                st.status = rc;
                results[job.first] = {rc, st};
                completed += 1;
                inflight = 0;
            }
            done_cv.notify_all();
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
    try {
        HierarchyCache cache;
        int worst = MG_OK;
        for (int i = 0; i < count; ++i) {
            int rc = solve_one(cache, probs[i], stats ? &stats[i] : nullptr, (hipStream_t)stream);
            if (rc != MG_OK && worst == MG_OK) worst = rc;
        }
        return worst;
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
    hipGetDevice(&S->device);
    hipError_t e = hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete S;
        return hip_fail(e, "hipStreamCreateWithFlags", __LINE__);
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
    size_t need = workspace_bytes(&prob->p);
    if (need > S->budget) {
        set_error("request needs more device memory than the server budget");
        return MG_ERR_BUDGET;
    }
    {
        std::lock_guard<std::mutex> lk(S->mu);
        *ticket = S->next_ticket++;
        S->queue.emplace_back(*ticket, *prob);
        S->submitted += 1;
    }
    S->cv.notify_one();
    return MG_OK;
}

int serve_poll(void* server, uint64_t ticket, mg_stats* out) {
    Server* S = (Server*)server;
    if (!S) return MG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->results.find(ticket);
    if (it == S->results.end()) return MG_PENDING;
    if (out) *out = it->second.second;
    return it->second.first;
}

int serve_wait(void* server, uint64_t ticket, mg_stats* out) {
    Server* S = (Server*)server;
    if (!S) return MG_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(S->mu);
    S->done_cv.wait(lk, [&] { return S->results.count(ticket) > 0; });
    auto& r = S->results[ticket];
    if (out) *out = r.second;
    return r.first;
}

int serve_counters(void* server, double out[6]) {
    Server* S = (Server*)server;
    if (!S || !out) return MG_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(S->mu);
    out[0] = S->submitted;
    out[1] = S->completed;
    out[2] = (double)S->queue.size();
    out[3] = S->inflight;
    out[4] = (double)S->cache.bytes;
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
    S->cache.clear();
    hipStreamDestroy(S->stream);
    delete S;
    return MG_OK;
}

}  // extern "C"
