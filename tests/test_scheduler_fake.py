"""The serving scheduler on the CPU, against a host-only fake executor.

tests/fake_serving.cpp links the library's scheduler (csrc/scheduler.cpp, plain
C++) with a FakeExecutor whose work costs bytes / bandwidth on a virtual
clock.  Here the same scenarios run through `simulate`, an independent Python
model of the policy the scheduler documents:

* requests are taken from a FIFO at every iteration boundary while the
  in-flight count stays under the cap, and admitted in arrival order while
  the resident bytes (states in use + idle states kept for reuse) stay within
  the budget; a request that does not fit waits, with every later one, for
  completions; before giving up, idle states of other shapes are released
  (shapes in key order, newest first), then idle states of its own shape;
* an idle state of the request's shape is reused (the oldest first), else one
  is created;
* admitted requests are set up together, then every in-flight request runs
  one iteration per round (continuous batching: a request that arrives
  mid-flight joins at the next boundary); the stop test on an iteration's
  residual comes at the start of the next round, where a stopped request is
  finished;
* a request's latency is its completion time minus its arrival time.

Each scenario's admission order, admission times, per-round composition,
per-request status, iterations and latency, state creations/releases and
peak resident bytes must agree exactly with the model.  The binaries are
built with AddressSanitizer + UndefinedBehaviorSanitizer, and separately with
ThreadSanitizer for a run with many client threads submitting, waiting and
polling at once.
"""
from __future__ import annotations

import collections
import hashlib
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1910_12979_amd", "csrc")
OUT = os.path.join(ROOT, "paper_1910_12979_amd", "_build", "fake")
SRCS = [os.path.join(CSRC, "scheduler.cpp"), os.path.join(ROOT, "tests", "fake_serving.cpp")]
DEPS = SRCS + [os.path.join(CSRC, "scheduler.h"), os.path.join(ROOT, "include", "macproj.h")]

OK, NOT_CONVERGED, OOM, HIP, BUDGET = 0, -4, -6, -7, -8


def _build(variant: str) -> str:
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not installed")
    san = {"asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
           "tsan": ["-fsanitize=thread"]}[variant]
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-Werror", *san, "-I", os.path.join(ROOT, "include"),
           "-I", CSRC, *SRCS, "-o", None, "-lpthread"]
    h = hashlib.sha1(" ".join(c for c in cmd if c).encode())
    for f in DEPS:
        with open(f, "rb") as fh:
            h.update(fh.read())
    exe = os.path.join(OUT, f"fake_serving_{variant}_{h.hexdigest()[:12]}")
    if not os.path.exists(exe):
        os.makedirs(OUT, exist_ok=True)
        cmd[cmd.index(None)] = exe + ".tmp"
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"build of the fake serving driver failed:\n{r.stderr[-4000:]}")
        os.replace(exe + ".tmp", exe)
    return exe


@pytest.fixture(scope="module")
def asan_exe():
    return _build("asan")


@pytest.fixture(scope="module")
def tsan_exe():
    return _build("tsan")


SAN_ENV = dict(ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")


def run_fake(exe, cost, reqs):
    lines = [" ".join(str(x) for x in (cost["budget"], cost["cap"], cost["bw"], cost["state_bpc"], cost["setup_bpc"],
                                       cost["iter_bpc"], cost["finish_bpc"], cost["solo_below_nx"], cost["oom_nz"],
                                       cost["fail_round"]))]
    lines += [f"{r['t']!r} {r['n'][0]} {r['n'][1]} {r['n'][2]} {r['k']} {r['max_cycles']}" for r in reqs]
    r = subprocess.run([exe, "replay"], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       env={**os.environ, **SAN_ENV}, timeout=120)
    assert r.returncode == 0, r.stderr[-6000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-6000:]
    return json.loads(r.stdout)


# ---------------------------------------------------------------------------
# independent model of the policy
def simulate(c, reqs):
    cells = lambda n: float(n[0] * n[1] * n[2])
    state_bytes = lambda n: int(cells(n) * c["state_bpc"])
    secs = lambda b: b / c["bw"]
    order = sorted(range(len(reqs)), key=lambda i: reqs[i]["t"])
    assert order == list(range(len(reqs))), "scenarios list arrivals in time order"
    clock = 0.0
    nxt = 0
    ticket = 1
    jobs = {}             # ticket -> job dict
    req_ticket = [None] * len(reqs)
    queue = collections.deque()
    active = []
    idle = {}             # shape key -> list of state ids (oldest first)
    state_key, state_b = {}, {}
    busy = idle_b = 0
    live = max_live = 0
    creates = destroys = recovers = rounds = 0
    next_id = 0
    admitted, admit_t, admit_slot, round_jobs = [], [], [], []
    inflight = peak = 0

    def arrive():
        nonlocal nxt, ticket
        while nxt < len(reqs) and reqs[nxt]["t"] <= clock:
            r = reqs[nxt]
            if state_bytes(r["n"]) > c["budget"]:
                req_ticket[nxt] = "refused"
            else:
                j = dict(ticket=ticket, n=tuple(r["n"]), k=r["k"], mc=r["max_cycles"], t_submit=r["t"],
                         status=OK, stage="new", cycles=0, slot=None, smooth=0.0)
                jobs[ticket] = j
                req_ticket[nxt] = ticket
                queue.append(j)
                ticket += 1
            nxt += 1

    def destroy(s):
        nonlocal live, destroys
        live -= state_b[s]
        destroys += 1

    def trim(target, keep):
        nonlocal idle_b
        for pas in range(2):
            if idle_b <= target:
                break
            for key in sorted(idle):
                if pas == 0 and key == keep:
                    continue
                while idle[key] and idle_b > target:
                    s = idle[key].pop()
                    idle_b -= state_b[s]
                    destroy(s)

    def acquire(j):
        nonlocal busy, idle_b, next_id, live, max_live, creates
        key = j["n"]
        if idle.get(key):
            s = idle[key].pop(0)
            idle_b -= state_b[s]
            busy += state_b[s]
            return s
        if j["n"][2] == c["oom_nz"]:
            return None
        s = next_id
        next_id += 1
        state_key[s], state_b[s] = key, state_bytes(key)
        creates += 1
        live += state_b[s]
        max_live = max(max_live, live)
        busy += state_b[s]
        return s

    def release(s):
        nonlocal busy, idle_b
        busy -= state_b[s]
        idle_b += state_b[s]
        idle.setdefault(state_key[s], []).append(s)

    def finish(j):
        nonlocal inflight
        j["t_done"] = clock
        j["ms_total"] = (clock - j["t_submit"]) * 1e3
        inflight -= 1

    def log_admit(j):
        admitted.append(j["ticket"])
        admit_t.append(j["t_admit"])
        admit_slot.append(j["slot"] if j["slot"] is not None else -1)

    def iterations(j):
        k = 0
        while 2.0 ** -k > 2.0 ** -j["k"] and k < j["mc"]:
            k += 1
        return k, (OK if 2.0 ** -k <= 2.0 ** -j["k"] else NOT_CONVERGED)

    while True:
        if not active and not queue:
            if nxt < len(reqs):
                clock = max(clock, reqs[nxt]["t"])
                arrive()
            else:
                break
        cand = collections.deque()
        while queue and len(active) + len(cand) < c["cap"]:
            cand.append(queue.popleft())
        fresh = []
        while cand:
            j = cand[0]
            need = 0 if idle.get(j["n"]) else state_bytes(j["n"])
            if busy + idle_b + need > c["budget"]:
                target = c["budget"] - busy - need if c["budget"] > busy + need else 0
                trim(target, j["n"])
                if busy + idle_b + need > c["budget"]:
                    break
            cand.popleft()
            j["t_admit"] = clock
            j["slot"] = acquire(j)
            if j["slot"] is None:
                j["status"] = OOM
            fresh.append(j)
        queue.extendleft(reversed(cand))
        inflight += len(fresh)
        peak = max(peak, inflight)
        setup_list = []
        for j in fresh:
            if j["status"] != OK:
                j["stage"] = "done"
                finish(j)
                continue
            if j["n"][0] < c["solo_below_nx"]:
                log_admit(j)
                n = cells(j["n"])
                k, st = iterations(j)
                clock += secs(n * c["setup_bpc"])
                t0 = clock
                clock += secs(n * c["iter_bpc"] * k)
                j["smooth"] = (clock - t0) * 1e3 if k > 0 else 0.0
                clock += secs(n * c["finish_bpc"])
                j["cycles"], j["status"], j["stage"] = k, st, "done"
                arrive()
                release(j["slot"])
                j["slot"] = None
                finish(j)
                continue
            setup_list.append(j)
            active.append(j)
        dt = 0.0
        for j in setup_list:
            log_admit(j)
            j["stage"] = "solve"
            dt += secs(cells(j["n"]) * c["setup_bpc"])
        clock += dt
        arrive()
        failed = False
        if active:
            rounds += 1
            if rounds == c["fail_round"]:
                failed = True
            else:
                run, fin = [], []
                for j in active:
                    if j["stage"] != "solve":
                        continue
                    if j["cycles"] > 0:
                        rel = 2.0 ** -j["cycles"]
                        if rel <= 2.0 ** -j["k"]:
                            j["status"], j["stage"] = OK, "finish"
                            continue
                        if j["cycles"] >= j["mc"]:
                            j["status"], j["stage"] = NOT_CONVERGED, "finish"
                            continue
                    elif j["mc"] == 0:
                        j["stage"] = "finish"
                        continue
                    run.append(j)
                fin = [j for j in active if j["stage"] == "finish"]
                dt = 0.0
                for j in run:
                    if j["cycles"] == 0:
                        j["t_iter0"] = clock
                    dt += secs(cells(j["n"]) * c["iter_bpc"])
                for j in fin:
                    dt += secs(cells(j["n"]) * c["finish_bpc"])
                clock += dt
                for j in run:
                    j["cycles"] += 1
                    j["t_iter1"] = clock
                for j in fin:
                    j["smooth"] = (j["t_iter1"] - j["t_iter0"]) * 1e3 if j["cycles"] > 0 else 0.0
                    j["stage"] = "done"
                round_jobs.append([j["ticket"] for j in run] + [j["ticket"] for j in fin])
                arrive()
        if failed:
            for j in active:
                if j["stage"] != "done":
                    # a request failed mid-flight reports no iterations
                    j["status"], j["stage"], j["cycles"] = HIP, "done", 0
            recovers += 1
        still = []
        for j in active:
            if j["stage"] == "done":
                if j["slot"] is not None:
                    release(j["slot"])
                    j["slot"] = None
                finish(j)
            else:
                still.append(j)
        active = still
    # the pool is emptied when the scheduler is destroyed
    for key in idle:
        for s in idle[key]:
            destroy(s)
    out = []
    for i, t in enumerate(req_ticket):
        if t == "refused":
            out.append(dict(status=BUDGET))
            continue
        j = jobs[t]
        out.append(dict(ticket=t, status=j["status"], cycles=j["cycles"], ms_total=j["ms_total"],
                        ms_smooth=j["smooth"]))
    return dict(requests=out, admitted=admitted, admit_t=admit_t, admit_slot=admit_slot, rounds=round_jobs,
                creates=creates, destroys=destroys, recovers=recovers, max_live=max_live, live_end=live, peak=peak,
                n_done=len(jobs))


def check_against_model(got, want, cost):
    assert got["admitted"] == want["admitted"]
    assert np.allclose(got["admit_t"], want["admit_t"], rtol=1e-12, atol=0)
    assert got["admit_slot"] == want["admit_slot"]
    assert got["rounds"] == want["rounds"]
    for g, w in zip(got["requests"], want["requests"], strict=True):
        assert g["status"] == w["status"], (g, w)
        if w["status"] == BUDGET:
            continue
        assert g["ticket"] == w["ticket"]
        assert g["stat_status"] == w["status"]
        assert g["cycles"] == w["cycles"]
        assert np.isclose(g["ms_total"], w["ms_total"], rtol=1e-12, atol=1e-9), (g, w)
        assert np.isclose(g["ms_smooth"], w["ms_smooth"], rtol=1e-12, atol=1e-9), (g, w)
        assert np.isclose(g["ms_other"], max(0.0, w["ms_total"] - w["ms_smooth"]), rtol=1e-12, atol=1e-9)
    assert (got["creates"], got["destroys"], got["recovers"]) == (want["creates"], want["destroys"], want["recovers"])
    assert got["max_live"] == want["max_live"] <= cost["budget"]
    assert got["live_end"] == 0
    ctr = got["counters"]
    assert ctr[0] == ctr[1] == want["n_done"]          # submitted == completed
    assert ctr[2] == 0 and ctr[3] == 0                 # nothing queued or in flight at the end
    assert ctr[5] == want["peak"] <= cost["cap"]


def cost_of(**kw):
    c = dict(budget=10 ** 9, cap=64, bw=1e9, state_bpc=100.0, setup_bpc=200.0, iter_bpc=800.0, finish_bpc=100.0,
             solo_below_nx=0, oom_nz=-1, fail_round=-1)
    c.update(kw)
    return c


def req(t, n, k, max_cycles=100):
    return dict(t=float(t), n=n, k=k, max_cycles=max_cycles)


# ---------------------------------------------------------------------------
def test_budget_limits_residency_and_states_are_reused(asan_exe):
    n = (32, 32, 32)
    cost = cost_of(budget=2 * 32 ** 3 * 100, cap=8)
    reqs = [req(0, n, k) for k in (3, 5, 2, 4, 6, 1)]
    got, want = run_fake(asan_exe, cost, reqs), simulate(cost, reqs)
    check_against_model(got, want, cost)
    assert got["creates"] == 2 and got["counters"][5] == 2          # two states, reused by the other four
    assert sorted(set(got["admit_slot"])) == [0, 1]
    assert got["admitted"] == sorted(got["admitted"])              # arrival order


def test_inflight_cap_and_fifo_admission(asan_exe):
    cost = cost_of(cap=3)
    reqs = [req(0, (16, 16, 16), 1 + i % 5) for i in range(10)]
    got, want = run_fake(asan_exe, cost, reqs), simulate(cost, reqs)
    check_against_model(got, want, cost)
    assert got["counters"][5] == 3 and got["creates"] == 3
    assert got["admitted"] == list(range(1, 11))
    assert max(len(r) for r in got["rounds"]) <= 3


def test_idle_states_of_other_shapes_are_released(asan_exe):
    small, big = (16, 16, 16), (32, 32, 32)
    cost = cost_of(budget=32 ** 3 * 100 + 16 ** 3 * 100, cap=4)
    reqs = [req(0, small, 2), req(0, small, 3), req(1e-3, big, 2), req(2e-3, small, 1), req(3e-3, big, 4)]
    got, want = run_fake(asan_exe, cost, reqs), simulate(cost, reqs)
    check_against_model(got, want, cost)
    assert got["destroys"] > 0 and got["max_live"] <= cost["budget"]


def test_continuous_batching_joins_at_iteration_boundaries(asan_exe):
    cost = cost_of(cap=16)
    n = (32, 32, 16)
    round_s = 32 * 32 * 16 * cost["iter_bpc"] / cost["bw"]
    reqs = [req(0, n, 8), req(2.5 * round_s, n, 3), req(4.2 * round_s, n, 2)]
    got, want = run_fake(asan_exe, cost, reqs), simulate(cost, reqs)
    check_against_model(got, want, cost)
    # the later arrivals ran alongside the first request, not after it
    joint = [r for r in got["rounds"] if 1 in r and len(r) > 1]
    assert joint and any(2 in r for r in joint) and any(3 in r for r in joint)
    lat = [r["ms_total"] for r in got["requests"]]
    assert lat[1] < lat[0] and lat[2] < lat[0]


def test_failure_paths(asan_exe):
    cost = cost_of(cap=4, solo_below_nx=16, oom_nz=24, fail_round=3)
    reqs = [req(0, (32, 32, 16), 4), req(0, (8, 8, 8), 3), req(0, (32, 32, 24), 2), req(0, (32, 32, 16), 9, 3),
            req(0, (32, 32, 16), 5, 0), req(0, (64, 64, 64), 2), req(1.0, (32, 32, 16), 2)]
    cost["budget"] = 3 * 32 * 32 * 16 * 100 + 8 ** 3 * 100
    got, want = run_fake(asan_exe, cost, reqs), simulate(cost, reqs)
    check_against_model(got, want, cost)
    status = [r["status"] for r in got["requests"]]
    assert OOM in status                     # state creation failed
    assert BUDGET in status                  # can never fit the budget: refused at submission
    assert got["recovers"] == 1 and HIP in status   # a failed round fails what was in flight
    assert status[-1] == OK                  # and serving goes on
    assert got["requests"][1]["status"] == OK and got["requests"][1]["cycles"] == 3   # solved alone


def test_not_converged_and_zero_cycles(asan_exe):
    cost = cost_of(cap=4)
    reqs = [req(0, (16, 16, 16), 9, 3), req(0, (16, 16, 16), 4, 0), req(0, (16, 16, 16), 2)]
    got, want = run_fake(asan_exe, cost, reqs), simulate(cost, reqs)
    check_against_model(got, want, cost)
    assert [r["status"] for r in got["requests"]] == [NOT_CONVERGED, OK, OK]
    assert got["requests"][0]["status"] == NOT_CONVERGED and got["requests"][0]["cycles"] == 3
    assert got["requests"][1]["cycles"] == 0 and got["requests"][1]["ms_smooth"] == 0.0


@pytest.mark.parametrize("seed", range(12))
def test_random_open_loop_matches_model(asan_exe, seed):
    rng = np.random.default_rng(1000 + seed)
    shapes = [(16, 16, 16), (32, 16, 16), (32, 32, 16), (32, 32, 32), (8, 8, 8)]
    nreq = int(rng.integers(20, 120))
    gaps = rng.exponential(scale=float(rng.choice([1e-5, 1e-4, 1e-3])), size=nreq)
    t = np.cumsum(gaps) - gaps[0]
    reqs = [req(float(t[i]), shapes[int(rng.integers(0, len(shapes)))], int(rng.integers(1, 12)),
                int(rng.choice([100, 100, 100, 5]))) for i in range(nreq)]
    cost = cost_of(cap=int(rng.integers(1, 12)), budget=int(rng.integers(1, 6)) * 32 ** 3 * 100 + 16 ** 3 * 100,
                   solo_below_nx=int(rng.choice([0, 16])), oom_nz=int(rng.choice([-1, -1, 16])),
                   fail_round=int(rng.choice([-1, -1, int(rng.integers(1, 40))])))
    got, want = run_fake(asan_exe, cost, reqs), simulate(cost, reqs)
    check_against_model(got, want, cost)
    # latency percentiles as a serving report computes them, from the stats each request carries
    ok = [w["ms_total"] for w in want["requests"] if w["status"] == OK]
    okg = [g["ms_total"] for g in got["requests"] if g["status"] == OK]
    if ok:
        for q in (50, 99):
            assert np.isclose(np.percentile(okg, q), np.percentile(ok, q), rtol=1e-12)


def test_many_clients_under_thread_sanitizer(tsan_exe):
    r = subprocess.run([tsan_exe, "threads", "6", "60"], capture_output=True, text=True,
                       env={**os.environ, **SAN_ENV}, timeout=300)
    assert r.returncode == 0, r.stderr[-6000:]
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-6000:]
    out = json.loads(r.stdout)
    assert out["ok"] == 360 and out["bad"] == 0 and out["held"] == 0
    ctr = out["counters"]
    assert ctr[0] == ctr[1] == 360 and ctr[2] == 0 and ctr[3] == 0
    assert ctr[5] <= out["cap"] and out["max_live"] <= out["budget"]
    assert out["live_end"] == 0 and out["creates"] == out["destroys"]


def test_many_clients_under_address_sanitizer(asan_exe):
    r = subprocess.run([asan_exe, "threads", "4", "80"], capture_output=True, text=True,
                       env={**os.environ, **SAN_ENV}, timeout=300)
    assert r.returncode == 0, r.stderr[-6000:]
    out = json.loads(r.stdout)
    assert out["ok"] == 320 and out["bad"] == 0 and out["held"] == 0
