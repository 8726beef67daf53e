// Batch and serving front ends of the C ABI.
//
// project_batch: every problem gets its own hierarchy (reused across calls
// from a process-wide cache keyed by kind and shape); all batchable problems
// are solved together by the batched engine, V-cycle by V-cycle, the others
// (nodal, multi-box, small shapes) one at a time.
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

// A resident state: the hierarchy of a MAC problem (with its boxes when the
// problem asks for them) or of a nodal one.
struct Slot {
    int kind = MG_KIND_MAC;
    mg_hierarchy* H = nullptr;
    nodal_handle N = nullptr;
};

bool has_box(const mg_problem& pr) { return pr.box[0] != 0 || pr.box[1] != 0 || pr.box[2] != 0; }

// Checks a problem can pass before it is queued (the box size itself is
// checked when its hierarchy is built).
int check_problem(const mg_problem& pr) {
    int rc = validate_params(&pr.p);
    if (rc) return rc;
    if (pr.kind != MG_KIND_MAC && pr.kind != MG_KIND_NODAL) {
        set_error("unknown problem kind");
        return MG_ERR_INVALID_ARG;
    }
    if (!pr.rho || !pr.beta0_cc || !pr.S || !pr.u || !pr.v || !pr.w ||
        (pr.kind == MG_KIND_MAC && !pr.beta0_edge)) {
        set_error("null field pointer in a problem");
        return MG_ERR_INVALID_ARG;
    }
    if (pr.kind == MG_KIND_NODAL && has_box(pr)) {
        set_error("a nodal problem runs on a single box");
        return MG_ERR_INVALID_ARG;
    }
    if (has_box(pr) && (pr.box[0] <= 0 || pr.box[1] <= 0 || pr.box[2] <= 0)) {
        set_error("box sizes must all be positive, or all zero for a single box");
        return MG_ERR_INVALID_ARG;
    }
    return MG_OK;
}

// The library's executor: resident states are hierarchies on one device, the
// work runs on one stream; single-box MAC problems whose finest level takes
// the fused sweep go through the batched engine, the rest are solved alone.
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
    size_t bytes_for(const mg_problem& pr) override {
        if (pr.kind == MG_KIND_NODAL) return nodal_bytes(&pr.p);
        return workspace_bytes(&pr.p) + (has_box(pr) ? box_bytes(pr.p, pr.box) : 0);
    }
    int create(const mg_problem& pr, void** slot, size_t* bytes) override {
        auto* s = new (std::nothrow) Slot();
        if (!s) return MG_ERR_OOM;
        s->kind = pr.kind;
        int rc;
        if (pr.kind == MG_KIND_NODAL) {
            rc = nodal_setup(&pr.p, &s->N);
        } else {
            rc = setup(&pr.p, nullptr, 0, &s->H);
            if (rc == MG_OK && has_box(pr)) {
                rc = mg_set_boxes(s->H, pr.box);
                if (rc != MG_OK) mg::destroy(s->H);
            }
        }
        if (rc != MG_OK) {
            delete s;
            return rc;
        }
        *slot = s;
        *bytes = bytes_for(pr);
        return MG_OK;
    }
    void destroy(void* slot) override {
        auto* s = static_cast<Slot*>(slot);
        if (s->N) nodal_destroy(s->N);
        if (s->H) mg::destroy(s->H);
        delete s;
    }
    void rebind(void* slot, const mg_problem& pr) override {
        auto* s = static_cast<Slot*>(slot);
        if (s->N) nodal_rebind(s->N, &pr.p);
        else s->H->p = pr.p;
    }
    static mg_hierarchy* attach(Job* j) { return j->H = static_cast<Slot*>(j->slot)->H; }
    bool batchable(Job* j) override {
        mg_hierarchy* H = attach(j);
        return H && !H->boxes_on && mg::batchable(H);
    }
    int solo(Job* j) override {
        const mg_problem& p = j->pr;
        const Slot* s = static_cast<Slot*>(j->slot);
        if (s->N) return nodal_project(s->N, p.rho, p.beta0_cc, p.S, p.u, p.v, p.w, p.phi, &j->st, stream);
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
            int rc = check_problem(j.pr);
            if (rc == MG_OK) rc = g_batch_pool->acquire(j.pr, dev, &j.slot);
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
    int rc = check_problem(*prob);
    if (rc) return rc;
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
