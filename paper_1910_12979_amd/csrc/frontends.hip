// Batch and serving front ends of the C ABI.
//
// project_batch: every problem gets its own hierarchy (reused across calls
// from a process-wide cache keyed by shape); all batchable problems are
// solved together by the batched engine, V-cycle by V-cycle.
//
// Serving: a Scheduler (scheduler.h: queue, admission against the HBM budget
// and the in-flight cap at V-cycle boundaries, pool of resident hierarchies,
// continuous batching) drives a HipExecutor that owns a stream and runs the
// batched engine on it.  A request overlaps on the device with requests that
// arrived earlier, and its result is the one mac_project gives for it alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>
#include <vector>

#include "batch.h"
#include "mg_internal.h"
#include "runtime.h"
#include "scheduler.h"

namespace mg {
namespace {

// The library's executor: resident states are hierarchies on one device, the
// work runs on one stream through the batched engine.
struct HipExecutor final : Executor {
    int device = 0;
    hipStream_t stream = nullptr;
    bool owns_stream = false;
    Engine engine;

    ~HipExecutor() override {
        if (stream) hipStreamSynchronize(stream);
        engine.release();
        if (owns_stream && stream) hipStreamDestroy(stream);
    }

    void bind() override { hipSetDevice(device); }
    size_t bytes_for(const mg_params& p) override { return workspace_bytes(&p); }
    int create(const mg_params& p, void** slot, size_t* bytes) override {
        mg_hierarchy* H = nullptr;
        const int rc = setup(&p, nullptr, 0, &H);
        if (rc != MG_OK) return rc;
        *slot = H;
        *bytes = H->ws_bytes;
        return MG_OK;
    }
    void destroy(void* slot) override { mg::destroy(static_cast<mg_hierarchy*>(slot)); }
    void rebind(void* slot, const mg_params& p) override { static_cast<mg_hierarchy*>(slot)->p = p; }
    static mg_hierarchy* attach(Job* j) { return j->H = static_cast<mg_hierarchy*>(j->slot); }
    bool batchable(Job* j) override { return mg::batchable(attach(j)); }
    int solo(Job* j) override {
        const mg_problem& p = j->pr;
        return project(attach(j), p.rho, p.beta0_cc, p.beta0_edge, p.S, p.u, p.v, p.w, p.phi, &j->st, stream);
    }
    int setup_new(std::vector<Job*>& fresh) override {
        for (Job* j : fresh) attach(j);
        return engine.setup_new(fresh, stream);
    }
    int round(std::vector<Job*>& jobs) override { return engine.round(jobs, stream); }
    void recover() override {
        hipStreamSynchronize(stream);
        engine.staging.off = 0;
    }
    double now() override {
        using namespace std::chrono;
        return duration<double>(steady_clock::now().time_since_epoch()).count();
    }
};

std::mutex g_batch_mu;
HipExecutor* g_batch_ex = nullptr;   // its engine runs project_batch; its stream is the caller's
SlotPool* g_batch_pool = nullptr;
constexpr size_t kBatchPoolCap = (size_t)64 << 30;   // idle bytes kept between project_batch calls
constexpr size_t kStagingBytes = (size_t)8 << 20;

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
        if (!g_batch_ex) {
            auto* ex = new HipExecutor();
            ex->engine.graph_mode = 1;      // a batch's rounds recur: capture at first sight
            if (ex->engine.staging.init(kStagingBytes) != MG_OK) {
                delete ex;
                set_error("staging allocation failed");
                return MG_ERR_OOM;
            }
            g_batch_ex = ex;
            g_batch_pool = new SlotPool(ex);
        }
        HipExecutor& ex = *g_batch_ex;
        ex.stream = st;
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
            if (rc == MG_OK) rc = g_batch_pool->acquire(j.pr.p, dev, &j.slot);
            if (rc != MG_OK) {
                j.st.status = j.status = rc;
                j.stage = Job::kDone;
                continue;
            }
            if (!ex.batchable(&j)) {
                j.status = ex.solo(&j);
                j.st.status = j.status;
                j.stage = Job::kDone;
                continue;
            }
            batched.push_back(&j);
        }
        int rc = ex.setup_new(batched);
        while (rc == MG_OK) {
            bool busy = false;
            for (Job* j : batched) busy |= j->stage == Job::kSolve || j->stage == Job::kFinish;
            if (!busy) break;
            rc = ex.round(batched);
        }
        hipEventRecord(e1, st);
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        ex.engine.staging.off = 0;
        for (int i = 0; i < count; ++i) {
            Job& j = jobs[i];
            if (rc != MG_OK && j.stage != Job::kDone) j.st.status = j.status = rc;
            j.st.ms_total = ms;
            j.st.ms_other = std::max(0.0, (double)ms - j.st.ms_smooth);
            if (stats) stats[i] = j.st;
            if (j.slot) g_batch_pool->release(j.slot);
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
    auto* ex = new (std::nothrow) HipExecutor();
    if (!ex) return MG_ERR_OOM;
    ex->engine.graph_mode = 2;                    // capture an active set once it recurs
    ex->owns_stream = true;
    hipGetDevice(&ex->device);
    hipError_t e = hipStreamCreateWithFlags(&ex->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        ex->stream = nullptr;
        delete ex;
        return hip_fail(e, "hipStreamCreateWithFlags", __LINE__);
    }
    if (ex->engine.staging.init(kStagingBytes) != MG_OK) {
        delete ex;
        set_error("staging allocation failed");
        return MG_ERR_OOM;
    }
    auto* S = new Scheduler(ex, hbm_budget_bytes, max_inflight, ex->device);
    S->start();
    *server = S;
    return MG_OK;
}

int serve_submit(void* server, const mg_problem* prob, uint64_t* ticket) {
    auto* S = static_cast<Scheduler*>(server);
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
    rc = S->submit(*prob, ticket);
    if (rc == MG_ERR_BUDGET) set_error("request needs more device memory than the server budget");
    return rc;
}

int serve_poll(void* server, uint64_t ticket, mg_stats* out) {
    auto* S = static_cast<Scheduler*>(server);
    if (!S) return MG_ERR_INVALID_ARG;
    const int rc = S->poll(ticket, out);
    if (rc == MG_ERR_INVALID_ARG) set_error("unknown ticket");
    return rc;
}

int serve_wait(void* server, uint64_t ticket, mg_stats* out) {
    auto* S = static_cast<Scheduler*>(server);
    if (!S) return MG_ERR_INVALID_ARG;
    const int rc = S->wait(ticket, out);
    if (rc == MG_ERR_INVALID_ARG) set_error("unknown ticket");
    return rc;
}

int serve_counters(void* server, double out[6]) {
    auto* S = static_cast<Scheduler*>(server);
    if (!S || !out) return MG_ERR_INVALID_ARG;
    S->counters(out);
    return MG_OK;
}

int serve_destroy(void* server) {
    // finishes what was submitted, releases the hierarchies, then the stream
    delete static_cast<Scheduler*>(server);
    return MG_OK;
}

}  // extern "C"
