// Request scheduling for the serving front end, independent of the device.
//
// A Scheduler owns a FIFO of requests, a pool of resident solver states (one
// per request shape, reused across requests) and one worker thread.  At every
// iteration boundary the worker admits as many queued requests, in arrival
// order, as the in-flight cap and the memory budget allow (resident states
// count against the budget; idle ones of other shapes are released when room
// is needed), sets them up, and runs the next round for everything in flight,
// so a request overlaps with requests that arrived earlier (continuous
// batching).  The device work goes through an Executor: the library's own
// runs the batched multigrid engine on a HIP stream; a host-only one with
// simulated durations lets the policy be tested without a GPU.
//
// Plain C++ (no HIP): the library compiles it with the rest, and host-only
// test programs compile it with a C++ compiler and their own executor.
#pragma once

#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "macproj.h"

namespace mg {

// One projection in flight.
struct Job {
    enum { kNew = 0, kSolve = 1, kFinish = 2, kDone = 3 };
    mg_problem pr{};
    void* slot = nullptr;     // resident solver state (the executor's)
    mg_hierarchy* H = nullptr;  // the same state, for the library's executor
    mg_stats st{};
    int status = MG_OK;
    int stage = kNew;
    int cycles = 0;
    int gslot = -1;           // row of the gathered norm block written by its last iteration
    double row[4] = {};       // that row, kept until the next round's stop test
    double fnorm = 0.0;
    double rel = 1.0;
    uint64_t ticket = 0;
    double t_submit = 0.0;
    double t_admit = 0.0;
    double t_done = 0.0;
    double t_iter0 = 0.0;     // seconds at its first iteration, and after its last
    double t_iter1 = 0.0;
    size_t bytes = 0;
    int waiters = 0;          // wait calls blocked on this ticket
    bool published = false;   // finished and its stats final (set under the scheduler's lock)
};

// What the scheduler needs from the device side.  Every call but now() and
// bytes_for() comes from the worker thread.
struct Executor {
    virtual ~Executor() = default;
    // first call on the worker thread
    virtual void bind() {}
    // resident bytes a request needs
    virtual size_t bytes_for(const mg_problem& pr) = 0;
    // a new resident state for the request's kind and shape (status, *slot, *bytes)
    virtual int create(const mg_problem& pr, void** slot, size_t* bytes) = 0;
    virtual void destroy(void* slot) = 0;
    // hand an idle state of the same key to a request (its solver controls)
    virtual void rebind(void* slot, const mg_problem& pr) = 0;
    // false: the job is solved on its own, to completion, by solo()
    virtual bool batchable(Job* j) = 0;
    virtual int solo(Job* j) = 0;
    // coefficients, right-hand side and checks of newly admitted jobs
    virtual int setup_new(std::vector<Job*>& fresh) = 0;
    // stop tests, one iteration of every job still solving, finishing of
    // the converged (stage kDone when finished)
    virtual int round(std::vector<Job*>& jobs) = 0;
    // after a failed setup or round: wait for the device, reset staging
    virtual void recover() = 0;
    // seconds on the clock request times are taken from
    virtual double now() = 0;
    // the worker has nothing queued and nothing in flight; true if the
    // executor submitted more work itself (a simulated arrival process)
    virtual bool idle() { return false; }
};

// device, kind, shape, boundaries, precision, spacing, box size
using ShapeKey = std::tuple<int, int, int, int, int, int, int, int, int, double, int, int, int>;
ShapeKey key_of(const mg_problem& pr, int device);

// Idle resident states kept for reuse, keyed by device, kind and shape.
struct SlotPool {
    Executor* ex = nullptr;
    struct Meta {
        ShapeKey key;
        size_t bytes;
    };
    std::map<ShapeKey, std::deque<void*>> idle;
    std::unordered_map<void*, Meta> meta;
    size_t idle_bytes = 0;
    size_t busy_bytes = 0;

    explicit SlotPool(Executor* e) : ex(e) {}
    ~SlotPool() { clear(); }
    void clear();
    bool has_idle(const mg_problem& pr, int dev) const;
    // the oldest idle state of the key (a repeated batch gets the same
    // states in the same order), else a new one
    int acquire(const mg_problem& pr, int dev, void** out);
    void release(void* slot);
    // free idle states (other shapes than *keep first, newest of a shape
    // first) until idle_bytes <= target
    void trim(size_t target, const ShapeKey* keep = nullptr);
};

class Scheduler {
public:
    // takes ownership of ex
    Scheduler(Executor* ex, size_t budget, int max_inflight, int device);
    ~Scheduler();   // finishes what was submitted, then stops the worker
    // start the worker thread (once)
    void start();
    // MG_ERR_BUDGET if the request can never fit the budget; t_submit < 0:
    // now() of the executor
    int submit(const mg_problem& pr, uint64_t* ticket, double t_submit = -1.0);
    // MG_PENDING while unfinished; the final status releases the ticket
    int poll(uint64_t ticket, mg_stats* out);
    int wait(uint64_t ticket, mg_stats* out);
    // submitted, completed, queued, in flight, resident bytes, peak in flight
    void counters(double out[6]);
    Executor* executor() { return ex_.get(); }

private:
    void run();
    void finish(Job* j);

    std::unique_ptr<Executor> ex_;
    size_t budget_;
    int max_inflight_;
    int device_;
    SlotPool pool_;                             // worker thread only
    std::mutex mu_;
    std::condition_variable cv_, done_cv_;
    std::deque<Job*> queue_;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs_;
    uint64_t next_ticket_ = 1;
    bool stop_ = false;
    double submitted_ = 0, completed_ = 0, peak_ = 0;
    size_t inflight_n_ = 0;
    size_t resident_ = 0;
    std::thread worker_;
};

}  // namespace mg
