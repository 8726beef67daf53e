// The serving scheduler (paper_1910_12979_amd/csrc/scheduler.cpp) driven by a
// host-only FakeExecutor, for CPU tests of its policy: admission in arrival
// order under the memory budget and the in-flight cap, reuse of resident
// states, release of idle states of other shapes, continuous batching at
// iteration boundaries, failure paths, ticket release and the latency
// bookkeeping every request's stats carry.
//
// The fake keeps a virtual clock.  Work costs bytes / bandwidth: per problem
// cell, setup_bpc bytes for the set-up, iter_bpc per iteration and
// finish_bpc for the correction; a resident state holds state_bpc bytes per
// cell.  Its "solver" halves the relative residual every iteration (2^-c after
// c iterations), and follows the stop-test order of the batched engine: the
// test on iteration c's residual comes at the start of the next round, and a
// job that stops is finished in that same round.
//
//   fake_serving replay  < scenario   arrivals replayed on the virtual clock
//   fake_serving threads T M          T client threads submitting and waiting
//
// Scenario: "budget cap bw state_bpc setup_bpc iter_bpc finish_bpc
// solo_below_nx oom_nz fail_round", then one line per request: "arrival nx ny
// nz k max_cycles" with rtol = 2^-k.  Output: one JSON object.
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "scheduler.h"

using namespace mg;

namespace {

struct Cost {
    double budget = 0, bw = 1;
    int cap = 1;
    double state_bpc = 0, setup_bpc = 0, iter_bpc = 0, finish_bpc = 0;
    int solo_below_nx = 0;   // nx below this: solved alone
    int oom_nz = -1;         // nz equal to this: creating a state fails
    int fail_round = -1;     // this round (1-based) fails as a device error would
};

struct State {
    mg_params p;
    int id;
};

// Written by the worker thread, read by the driver once the scheduler has
// been destroyed (its worker joined).
struct Report {
    int creates = 0, destroys = 0, rounds = 0, recovers = 0;
    double live = 0, max_live = 0;
    std::vector<std::vector<uint64_t>> round_jobs;   // tickets iterated or finished per round
    std::vector<uint64_t> admitted;                  // admission order
    std::vector<double> admit_t;
    std::vector<int> admit_slot;                     // state id each admitted request got
    std::unique_ptr<std::atomic<uint64_t>[]> arrival_ticket;   // ticket of each arrival once submitted
};

double cells(const mg_params& p) { return (double)p.n[0] * p.n[1] * p.n[2]; }

struct FakeExecutor final : Executor {
    Cost c;
    Report* rep;
    Scheduler* sched = nullptr;
    std::vector<std::pair<double, mg_problem>> arrivals;   // sorted by time
    size_t next = 0;
    std::atomic<double> clock{0.0};
    int next_id = 0;

    FakeExecutor(const Cost& cost, Report* r) : c(cost), rep(r) {}

    double secs(double bytes) const { return bytes / c.bw; }
    void advance(double dt) { clock.store(clock.load() + dt); }
    // submit every scheduled arrival whose time has come
    void arrive() {
        while (next < arrivals.size() && arrivals[next].first <= clock.load()) {
            uint64_t t = 0;
            const int rc = sched->submit(arrivals[next].second, &t, arrivals[next].first);
            rep->arrival_ticket[next].store(rc == MG_OK ? t : ~0ull);
            ++next;
        }
    }
    void log_admit(Job* j) {
        rep->admitted.push_back(j->ticket);
        rep->admit_t.push_back(j->t_admit);
        rep->admit_slot.push_back(j->slot ? static_cast<State*>(j->slot)->id : -1);
    }
    // iterations a job runs before its stop test passes or max_cycles ends it
    static int iterations(const mg_params& p, int* status) {
        int k = 0;
        while (std::ldexp(1.0, -k) > p.rtol && k < p.max_cycles) ++k;
        *status = std::ldexp(1.0, -k) <= p.rtol ? MG_OK : MG_ERR_NOT_CONVERGED;
        return k;
    }

    size_t bytes_for(const mg_params& p) const { return (size_t)(cells(p) * c.state_bpc); }
    size_t bytes_for(const mg_problem& pr) override { return bytes_for(pr.p); }
    int create(const mg_problem& pr, void** slot, size_t* bytes) override {
        const mg_params& p = pr.p;
        if (p.n[2] == c.oom_nz) return MG_ERR_OOM;
        auto* s = new State{p, next_id++};
        *slot = s;
        *bytes = bytes_for(p);
        rep->creates += 1;
        rep->live += (double)*bytes;
        rep->max_live = std::max(rep->max_live, rep->live);
        return MG_OK;
    }
    void destroy(void* slot) override {
        auto* s = static_cast<State*>(slot);
        rep->destroys += 1;
        rep->live -= (double)bytes_for(s->p);
        delete s;
    }
    void rebind(void* slot, const mg_problem& pr) override { static_cast<State*>(slot)->p = pr.p; }
    bool batchable(Job* j) override { return j->pr.p.n[0] >= c.solo_below_nx; }
    int solo(Job* j) override {
        log_admit(j);
        const double n = cells(j->pr.p);
        int status = MG_OK;
        const int k = iterations(j->pr.p, &status);
        std::memset(&j->st, 0, sizeof j->st);
        advance(secs(n * c.setup_bpc));
        const double t0 = clock.load();
        advance(secs(n * c.iter_bpc * k));
        j->st.ms_smooth = k > 0 ? (clock.load() - t0) * 1e3 : 0.0;
        advance(secs(n * c.finish_bpc));
        j->cycles = j->st.cycles = k;
        j->st.rel_resid = std::ldexp(1.0, -k);
        j->st.status = status;
        arrive();
        return status;
    }
    int setup_new(std::vector<Job*>& fresh) override {
        double dt = 0;
        for (Job* j : fresh) {
            log_admit(j);
            std::memset(&j->st, 0, sizeof j->st);
            j->stage = Job::kSolve;
            j->cycles = 0;
            dt += secs(cells(j->pr.p) * c.setup_bpc);
        }
        advance(dt);
        arrive();
        return MG_OK;
    }
    int round(std::vector<Job*>& jobs) override {
        rep->rounds += 1;
        if (rep->rounds == c.fail_round) return MG_ERR_HIP;
        std::vector<Job*> run, fin;
        for (Job* j : jobs) {
            if (j->stage != Job::kSolve) continue;
            if (j->cycles > 0) {
                j->rel = std::ldexp(1.0, -j->cycles);
                if (j->rel <= j->pr.p.rtol) {
                    j->status = MG_OK;
                    j->stage = Job::kFinish;
                    continue;
                }
                if (j->cycles >= j->pr.p.max_cycles) {
                    j->status = MG_ERR_NOT_CONVERGED;
                    j->stage = Job::kFinish;
                    continue;
                }
            } else if (j->pr.p.max_cycles == 0) {
                j->stage = Job::kFinish;
                continue;
            }
            run.push_back(j);
        }
        for (Job* j : jobs)
            if (j->stage == Job::kFinish) fin.push_back(j);
        std::vector<uint64_t> ids;
        double dt = 0;
        for (Job* j : run) {
            if (j->cycles == 0) j->t_iter0 = clock.load();
            dt += secs(cells(j->pr.p) * c.iter_bpc);
            ids.push_back(j->ticket);
        }
        for (Job* j : fin) {
            dt += secs(cells(j->pr.p) * c.finish_bpc);
            ids.push_back(j->ticket);
        }
        advance(dt);
        for (Job* j : run) {
            ++j->cycles;
            j->t_iter1 = clock.load();
        }
        for (Job* j : fin) {
            j->st.cycles = j->cycles;
            j->st.rel_resid = j->cycles > 0 ? j->rel : 1.0;
            j->st.ms_smooth = j->cycles > 0 ? (j->t_iter1 - j->t_iter0) * 1e3 : 0.0;
            j->st.status = j->status;
            j->stage = Job::kDone;
        }
        rep->round_jobs.push_back(ids);
        arrive();
        return MG_OK;
    }
    void recover() override { rep->recovers += 1; }
    double now() override { return clock.load(); }
    bool idle() override {
        if (next >= arrivals.size()) return false;
        if (arrivals[next].first > clock.load()) clock.store(arrivals[next].first);
        arrive();
        return true;
    }
};

mg_problem make_problem(int nx, int ny, int nz, int k, int max_cycles) {
    mg_problem pr{};
    pr.p.n[0] = nx;
    pr.p.n[1] = ny;
    pr.p.n[2] = nz;
    pr.p.dx = 1.0 / nx;
    pr.p.bc[0] = pr.p.bc[1] = MG_BC_PERIODIC;
    pr.p.bc[2] = MG_BC_WALL;
    pr.p.pre_sweeps = pr.p.post_sweeps = 2;
    pr.p.precision = MG_FP64;
    pr.p.rtol = std::ldexp(1.0, -k);
    pr.p.max_cycles = max_cycles;
    return pr;   // field pointers stay null: the fake never reads them
}

void print_list(const char* name, const std::vector<uint64_t>& v) {
    std::printf("\"%s\": [", name);
    for (size_t i = 0; i < v.size(); ++i) std::printf("%s%llu", i ? ", " : "", (unsigned long long)v[i]);
    std::printf("]");
}

int replay() {
    Cost c;
    if (std::scanf("%lf %d %lf %lf %lf %lf %lf %d %d %d", &c.budget, &c.cap, &c.bw, &c.state_bpc, &c.setup_bpc,
                   &c.iter_bpc, &c.finish_bpc, &c.solo_below_nx, &c.oom_nz, &c.fail_round) != 10) {
        std::fprintf(stderr, "bad scenario header\n");
        return 2;
    }
    Report rep;
    auto* ex = new FakeExecutor(c, &rep);
    double t;
    int nx, ny, nz, k, mc;
    while (std::scanf("%lf %d %d %d %d %d", &t, &nx, &ny, &nz, &k, &mc) == 6)
        ex->arrivals.emplace_back(t, make_problem(nx, ny, nz, k, mc));
    const size_t n = ex->arrivals.size();
    rep.arrival_ticket.reset(new std::atomic<uint64_t>[n]);
    for (size_t i = 0; i < n; ++i) rep.arrival_ticket[i].store(0);
    auto* S = new Scheduler(ex, (size_t)c.budget, c.cap, 0);
    ex->sched = S;
    S->start();
    std::vector<mg_stats> st(n);
    std::vector<int> status(n, 1);
    for (size_t i = 0; i < n; ++i) {
        for (;;) {
            // the ticket an arrival got is known once it has been submitted
            const uint64_t tk = rep.arrival_ticket[i].load();
            if (tk == ~0ull) {
                status[i] = MG_ERR_BUDGET;   // refused at submission
                break;
            }
            if (tk) {
                const int rc = S->poll(tk, &st[i]);
                if (rc != MG_PENDING) {
                    status[i] = rc;
                    break;
                }
            }
            std::this_thread::sleep_for(std::chrono::microseconds(200));
        }
    }
    double ctr[6];
    S->counters(ctr);
    delete S;
    std::printf("{");
    std::printf("\"requests\": [");
    for (size_t i = 0; i < n; ++i)
        std::printf("%s{\"ticket\": %llu, \"status\": %d, \"stat_status\": %d, \"cycles\": %d, \"ms_total\": %.17g, "
                    "\"ms_smooth\": %.17g, \"ms_other\": %.17g, \"rel_resid\": %.17g}",
                    i ? ", " : "", (unsigned long long)rep.arrival_ticket[i].load(), status[i], st[i].status, st[i].cycles,
                    st[i].ms_total, st[i].ms_smooth, st[i].ms_other, st[i].rel_resid);
    std::printf("], ");
    print_list("admitted", rep.admitted);
    std::printf(", \"admit_t\": [");
    for (size_t i = 0; i < rep.admit_t.size(); ++i) std::printf("%s%.17g", i ? ", " : "", rep.admit_t[i]);
    std::printf("], \"admit_slot\": [");
    for (size_t i = 0; i < rep.admit_slot.size(); ++i) std::printf("%s%d", i ? ", " : "", rep.admit_slot[i]);
    std::printf("], \"rounds\": [");
    for (size_t r = 0; r < rep.round_jobs.size(); ++r) {
        std::printf("%s", r ? ", " : "");
        std::printf("[");
        for (size_t q = 0; q < rep.round_jobs[r].size(); ++q)
            std::printf("%s%llu", q ? ", " : "", (unsigned long long)rep.round_jobs[r][q]);
        std::printf("]");
    }
    std::printf("], \"creates\": %d, \"destroys\": %d, \"recovers\": %d, \"max_live\": %.17g, \"live_end\": %.17g, "
                "\"counters\": [%g, %g, %g, %g, %g, %g]}\n",
                rep.creates, rep.destroys, rep.recovers, rep.max_live, rep.live, ctr[0], ctr[1], ctr[2], ctr[3],
                ctr[4], ctr[5]);
    return 0;
}

// T client threads, each submitting M requests at once (three shapes, 1..6
// iterations) and collecting them: even ones with wait, shared with a second
// waiting thread, odd ones by polling; one more thread reads the counters
// throughout.  Checks that every request finishes exactly as its own
// parameters say, that a released ticket is unknown afterwards, and the
// budget, cap and counter invariants.
int threads(int T, int M) {
    Cost c;
    c.cap = 4;
    c.bw = 1e12;
    c.state_bpc = 1.0;
    c.setup_bpc = 100;
    c.iter_bpc = 400;
    c.finish_bpc = 50;
    c.budget = 3.0 * 16 * 16 * 16;   // three states of the largest shape
    Report rep;
    auto* ex = new FakeExecutor(c, &rep);
    auto* S = new Scheduler(ex, (size_t)c.budget, c.cap, 0);
    ex->sched = S;
    S->start();
    const int shapes[3][3] = {{8, 8, 8}, {16, 8, 8}, {16, 16, 16}};
    std::atomic<int> ok{0}, bad{0}, late{0};
    std::atomic<bool> done{false};
    std::vector<std::unique_ptr<std::atomic<uint64_t>[]>> tickets(T);
    for (int i = 0; i < T; ++i) {
        tickets[i].reset(new std::atomic<uint64_t>[M]);
        for (int m = 0; m < M; ++m) tickets[i][m].store(0);
    }
    auto expect = [&](int i, int m, int rc, const mg_stats& st) {
        const int k = 1 + (i * 7 + m) % 6;
        if (rc == MG_OK && st.status == MG_OK && st.cycles == k && st.rel_resid == std::ldexp(1.0, -k) &&
            st.ms_total >= st.ms_smooth && st.ms_smooth > 0.0)
            ok += 1;
        else
            bad += 1;
    };
    std::vector<std::thread> th;
    for (int i = 0; i < T; ++i) {
        th.emplace_back([&, i] {
            for (int m = 0; m < M; ++m) {
                const int* sh = shapes[(i + m) % 3];
                uint64_t t = 0;
                if (S->submit(make_problem(sh[0], sh[1], sh[2], 1 + (i * 7 + m) % 6, 100), &t) != MG_OK) {
                    bad += 1;
                    continue;
                }
                tickets[i][m].store(t);
                mg_stats st{};
                int rc;
                if (m % 2 == 0) {
                    rc = S->wait(t, &st);
                } else {
                    while ((rc = S->poll(t, &st)) == MG_PENDING) std::this_thread::yield();
                }
                expect(i, m, rc, st);
                // released once its status was returned to every waiter (the
                // second waiter of an even request may still hold it)
                const int again = S->poll(t, &st);
                if (again != MG_ERR_INVALID_ARG && !(m % 2 == 0 && again == MG_OK)) bad += 1;
            }
        });
        th.emplace_back([&, i] {
            // second waiter on the even requests: the status, or unknown once
            // the first waiter has released the ticket
            for (int m = 0; m < M; m += 2) {
                uint64_t t;
                while ((t = tickets[i][m].load()) == 0) std::this_thread::yield();
                mg_stats st{};
                const int rc = S->wait(t, &st);
                if (rc == MG_ERR_INVALID_ARG)
                    late += 1;
                else if (rc != MG_OK || st.cycles != 1 + (i * 7 + m) % 6)
                    bad += 1;
            }
        });
    }
    double peak_seen = 0;
    std::thread spy([&] {
        double ctr[6];
        while (!done.load()) {
            S->counters(ctr);
            if (ctr[3] > c.cap || ctr[4] > c.budget || ctr[1] > ctr[0]) bad += 1;
            peak_seen = std::max(peak_seen, ctr[3]);
            std::this_thread::yield();
        }
    });
    for (auto& t : th) t.join();
    done.store(true);
    spy.join();
    int held = 0;   // tickets still known once every client has returned
    for (int i = 0; i < T; ++i)
        for (int m = 0; m < M; ++m) {
            mg_stats st{};
            if (S->poll(tickets[i][m].load(), &st) != MG_ERR_INVALID_ARG) held += 1;
        }
    double ctr[6];
    S->counters(ctr);
    delete S;
    std::printf("{\"ok\": %d, \"bad\": %d, \"late_waiters\": %d, \"held\": %d, \"counters\": [%g, %g, %g, %g, %g, %g], "
                "\"max_live\": %.17g, \"live_end\": %.17g, \"budget\": %.17g, \"cap\": %d, \"creates\": %d, "
                "\"destroys\": %d}\n",
                ok.load(), bad.load(), late.load(), held, ctr[0], ctr[1], ctr[2], ctr[3], ctr[4], ctr[5], rep.max_live,
                rep.live, c.budget, c.cap, rep.creates, rep.destroys);
    return 0;
}

}  // namespace

int main(int argc, char** argv) {
    if (argc >= 2 && std::strcmp(argv[1], "replay") == 0) return replay();
    if (argc >= 4 && std::strcmp(argv[1], "threads") == 0) return threads(std::atoi(argv[2]), std::atoi(argv[3]));
    std::fprintf(stderr, "usage: fake_serving replay < scenario | fake_serving threads T M\n");
    return 2;
}
