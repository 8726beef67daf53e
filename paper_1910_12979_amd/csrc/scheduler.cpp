// Request scheduling for the serving front end (see scheduler.h).
#include "scheduler.h"

#include <algorithm>

namespace mg {

ShapeKey key_of(const mg_problem& pr, int device) {
    const mg_params& p = pr.p;
    return ShapeKey(device, pr.kind, p.n[0], p.n[1], p.n[2], p.bc[0], p.bc[1], p.bc[2], p.precision, p.dx,
                    pr.box[0], pr.box[1], pr.box[2]);
}

// ---------------------------------------------------------------------------
void SlotPool::clear() {
    for (auto& kv : idle)
        for (void* s : kv.second) {
            meta.erase(s);
            ex->destroy(s);
        }
    idle.clear();
    idle_bytes = 0;
}

bool SlotPool::has_idle(const mg_problem& pr, int dev) const {
    auto it = idle.find(key_of(pr, dev));
    return it != idle.end() && !it->second.empty();
}

int SlotPool::acquire(const mg_problem& pr, int dev, void** out) {
    const ShapeKey k = key_of(pr, dev);
    auto it = idle.find(k);
    if (it != idle.end() && !it->second.empty()) {
        void* s = it->second.front();
        it->second.pop_front();
        const size_t b = meta.at(s).bytes;
        idle_bytes -= b;
        busy_bytes += b;
        ex->rebind(s, pr);
        *out = s;
        return MG_OK;
    }
    void* s = nullptr;
    size_t b = 0;
    const int rc = ex->create(pr, &s, &b);
    if (rc != MG_OK) return rc;
    meta[s] = Meta{k, b};
    busy_bytes += b;
    *out = s;
    return MG_OK;
}

void SlotPool::release(void* slot) {
    const Meta& m = meta.at(slot);
    busy_bytes -= m.bytes;
    idle_bytes += m.bytes;
    idle[m.key].push_back(slot);
}

void SlotPool::trim(size_t target, const ShapeKey* keep) {
    for (int pass = 0; pass < 2 && idle_bytes > target; ++pass)
        for (auto& kv : idle) {
            if (pass == 0 && keep && kv.first == *keep) continue;
            while (!kv.second.empty() && idle_bytes > target) {
                void* s = kv.second.back();
                kv.second.pop_back();
                idle_bytes -= meta.at(s).bytes;
                meta.erase(s);
                ex->destroy(s);
            }
        }
}

// ---------------------------------------------------------------------------
Scheduler::Scheduler(Executor* ex, size_t budget, int max_inflight, int device)
    : ex_(ex), budget_(budget), max_inflight_(max_inflight), device_(device), pool_(ex) {}

void Scheduler::start() {
    if (!worker_.joinable()) worker_ = std::thread([this] { run(); });
}

Scheduler::~Scheduler() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        stop_ = true;
    }
    cv_.notify_all();
    if (worker_.joinable()) worker_.join();
    pool_.clear();
}

int Scheduler::submit(const mg_problem& pr, uint64_t* ticket, double t_submit) {
    const size_t need = ex_->bytes_for(pr);
    if (need > budget_) return MG_ERR_BUDGET;
    auto j = std::make_unique<Job>();
    j->pr = pr;
    j->bytes = need;
    j->t_submit = t_submit >= 0.0 ? t_submit : ex_->now();
    {
        std::lock_guard<std::mutex> lk(mu_);
        j->ticket = next_ticket_++;
        *ticket = j->ticket;
        queue_.push_back(j.get());
        jobs_.emplace(*ticket, std::move(j));
        submitted_ += 1;
    }
    cv_.notify_one();
    return MG_OK;
}

int Scheduler::poll(uint64_t ticket, mg_stats* out) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return MG_ERR_INVALID_ARG;
    Job* j = it->second.get();
    if (!j->published) return MG_PENDING;
    if (out) *out = j->st;
    const int status = j->status;
    if (j->waiters == 0) jobs_.erase(it);   // final status returned: the ticket is released
    return status;
}

int Scheduler::wait(uint64_t ticket, mg_stats* out) {
    std::unique_lock<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    if (it == jobs_.end()) return MG_ERR_INVALID_ARG;
    Job* j = it->second.get();
    j->waiters += 1;
    done_cv_.wait(lk, [&] { return j->published; });
    j->waiters -= 1;
    if (out) *out = j->st;
    const int status = j->status;
    if (j->waiters == 0) jobs_.erase(ticket);   // final status returned: the ticket is released
    return status;
}

void Scheduler::counters(double out[6]) {
    std::lock_guard<std::mutex> lk(mu_);
    out[0] = submitted_;
    out[1] = completed_;
    out[2] = (double)queue_.size();
    out[3] = (double)inflight_n_;
    out[4] = (double)resident_;
    out[5] = peak_;
}

// publish a finished job: `published` (written under the lock, after every
// other field) is what pollers test
void Scheduler::finish(Job* j) {
    const double t = ex_->now();
    {
        std::lock_guard<std::mutex> lk(mu_);
        j->st.ms_total = (t - j->t_submit) * 1e3;
        j->st.ms_other = std::max(0.0, j->st.ms_total - j->st.ms_smooth);
        j->t_done = t;
        j->published = true;
        completed_ += 1;
        inflight_n_ -= 1;
    }
    done_cv_.notify_all();
}

void Scheduler::run() {
    ex_->bind();
    std::vector<Job*> active;
    for (;;) {
        std::vector<Job*> fresh;
        std::deque<Job*> cand;
        {
            // under the lock only the queue: take the requests that the
            // in-flight cap allows (the pool is the worker's alone)
            std::unique_lock<std::mutex> lk(mu_);
            if (active.empty() && queue_.empty()) {
                lk.unlock();
                const bool more = ex_->idle();
                lk.lock();
                if (!more) cv_.wait(lk, [&] { return stop_ || !queue_.empty(); });
            }
            if (stop_ && active.empty() && queue_.empty()) return;
            while (!queue_.empty() && active.size() + cand.size() < (size_t)max_inflight_) {
                cand.push_back(queue_.front());
                queue_.pop_front();
            }
        }
        // admission at the iteration boundary against the budget, in arrival
        // order; states are created (and idle ones of other shapes released)
        // without holding the lock
        while (!cand.empty()) {
            Job* j = cand.front();
            const bool reuse = pool_.has_idle(j->pr, device_);
            const size_t need = reuse ? 0 : j->bytes;
            if (pool_.busy_bytes + pool_.idle_bytes + need > budget_) {
                const ShapeKey k = key_of(j->pr, device_);
                const size_t target = budget_ > pool_.busy_bytes + need ? budget_ - pool_.busy_bytes - need : 0;
                pool_.trim(target, &k);
                if (pool_.busy_bytes + pool_.idle_bytes + need > budget_) break;   // wait for completions
            }
            cand.pop_front();
            j->t_admit = ex_->now();
            // reserve the state now, so the next request in this pass sees
            // the pool as it will be
            j->status = pool_.acquire(j->pr, device_, &j->slot);
            fresh.push_back(j);
        }
        {
            std::lock_guard<std::mutex> lk(mu_);
            for (auto it = cand.rbegin(); it != cand.rend(); ++it) queue_.push_front(*it);   // not admitted yet
            inflight_n_ += fresh.size();
            peak_ = std::max(peak_, (double)inflight_n_);
        }
        std::vector<Job*> setup_list;
        for (Job* j : fresh) {
            if (j->status != MG_OK) {
                j->st.status = j->status;
                j->stage = Job::kDone;
                j->slot = nullptr;
                finish(j);
                continue;
            }
            if (!ex_->batchable(j)) {
                // solved on its own, between rounds
                j->status = ex_->solo(j);
                j->st.status = j->status;
                j->stage = Job::kDone;
                pool_.release(j->slot);
                j->slot = nullptr;
                finish(j);
                continue;
            }
            setup_list.push_back(j);
            active.push_back(j);
        }
        int rc = ex_->setup_new(setup_list);
        if (rc == MG_OK && !active.empty()) rc = ex_->round(active);
        if (rc != MG_OK) {
            // a device error: fail everything in flight, keep serving
            for (Job* j : active)
                if (j->stage != Job::kDone) {
                    j->st.status = j->status = rc;
                    j->stage = Job::kDone;
                }
            ex_->recover();
        }
        std::vector<Job*> still;
        for (Job* j : active) {
            if (j->stage == Job::kDone) {
                if (j->slot) {
                    pool_.release(j->slot);
                    j->slot = nullptr;
                }
                finish(j);
            } else {
                still.push_back(j);
            }
        }
        active.swap(still);
        {
            std::lock_guard<std::mutex> lk(mu_);
            resident_ = pool_.busy_bytes + pool_.idle_bytes;
        }
    }
}

}  // namespace mg
