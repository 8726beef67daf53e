#!/usr/bin/env python3
"""Benchmark: variable-coefficient MAC-projection solves/s on one MI355X.

Headline workload: the 256^3 steeply stratified box (periodic x,y, solid
walls in z, beta0 = exp(-z/0.1), rho = beta0 (1 + 0.01 N(0,1)), S = 0.1 N(0,1)
with its beta0-weighted mean removed, U ~ N(0,1)), FP64, V(2,2) red-black GS
cycles to a 1e-10 relative residual.  One step = one whole projection
(coefficients, right-hand side, V-cycles, velocity correction) of the same
input.  The projection corrects its velocity in place, so every timed step
gets its own device copy of the input velocity, made before the timed region
(up to STAGE_CAP_BYTES of copies; beyond that the velocity is restored from
one device copy before each step, inside the timed region, and the line says
so); the other legs below time their solves and batches the same way, except
the server, whose requests restore their inputs as they are submitted.
Inputs are resident in HBM before timing.

Also reported on the same JSON line:
  * roofline: the finest-level fused sweep (the dominant kernel), its launch
    duration measured with HIP events on the stream it runs on, against the
    8 TB/s HBM peak; `traffic` is the counter-measured HBM bytes per launch
    when they were taken on the current sweep source, else null;
  * mixed: the same box in mixed precision (FP32 cycles with FP64 iterative
    refinement) and its phi difference from the FP64 GPU solve;
  * batch: 64 independent boxes with edges from {32,48,64,96,128} solved by
    project_batch, against the same problems solved one by one;
  * n512: the 512^3 box (H = 0.15, 5% density noise) in mixed precision and
    in FP64, with every solve's phi error against the FP64 oracle's exact
    discrete solution (definition mode, computed once on the host);
  * serve: Poisson request streams of {32,64,128,256}^3 boxes through the
    continuous-batching server at 50 to 2000 req/s (2000 requests per rate
    after 200 warm-up), solves/s with p50/p99 latency per rate, in FP64 and
    at two rates in mixed precision;
  * full_rhs: the box with its base state given as p0 and Gamma1 (beta0
    computed on the device each step, dp0/dt term in the right-hand side);
  * cpu_baseline: the FP64 CPU oracle timed on the host cores on whole
    solves of the headline box (about 10 s of CPU work).

Prints one JSON line.  `--gpus` above 1 is refused: this path runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
import types

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of one red-black Gauss-Seidel sweep per cell: phi, f and
# the three face coefficients read once, phi written once (8 + 8 + 24 + 8).
SWEEP_BYTES_PER_CELL = 48.0
# What this library's finest-level sweep moves instead: phi_in, f and rho in,
# phi_out out (the face coefficients are recomputed from rho and beta0).
SWEEP_KERNEL_BYTES_PER_CELL = 32.0

# HBM bytes per finest-level sweep launch at 256^3, from two rocprofv3 --pmc
# passes over this script (FETCH_SIZE, then WRITE_SIZE), each scaled by what
# the same counter reads for a plain device copy of known size.  Valid only
# for the sweep source it was taken on (SHA-1 of the files below) and tile.
SWEEP_SOURCES = ("paper_1910_12979_amd/csrc/sweep.hip", "paper_1910_12979_amd/csrc/sweep.h",
                 "paper_1910_12979_amd/csrc/devmath.h")
SWEEP_TRAFFIC = {"sha1": "697055d832cfe875ca2e3ca7e2e498b4a726d5d6", "tile": [64, 16, 64], "n": 256,
                 "read": 435405979, "write": 133695495}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sweep_source_sha1():
    h = hashlib.sha1()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


class Restorable:
    """A device problem plus copies of its input velocity."""

    def __init__(self, macproj, prob, dev):
        self.prob = prob
        self.d = macproj.to_device(prob, dev)
        self.u0, self.v0, self.w0 = self.d.u.clone(), self.d.v.clone(), self.d.w.clone()

    def restore(self):
        self.d.u.copy_(self.u0)
        self.d.v.copy_(self.v0)
        self.d.w.copy_(self.w0)

    def stage(self, k):
        """k device copies of the input velocity, one per timed step, or None
        when they would take more than STAGE_CAP_BYTES."""
        per = sum(t.numel() * t.element_size() for t in (self.u0, self.v0, self.w0))
        if k * per > STAGE_CAP_BYTES:
            return None
        return [(self.u0.clone(), self.v0.clone(), self.w0.clone()) for _ in range(k)]


# device copies of the input velocity staged for the timed steps (bytes)
STAGE_CAP_BYTES = 48 << 30


def stage_problems(rs, k):
    """k sets of the problems' device inputs (namespaces like Restorable.d),
    each with its own copies of the input velocities, made before a timed
    region; None when they would take more than STAGE_CAP_BYTES."""
    per = sum(t.numel() * t.element_size() for r in rs for t in (r.u0, r.v0, r.w0))
    if k * per > STAGE_CAP_BYTES:
        return None
    sets = []
    for _ in range(k):
        ds = []
        for r in rs:
            d = types.SimpleNamespace(**vars(r.d))
            d.u, d.v, d.w = r.u0.clone(), r.v0.clone(), r.w0.clone()
            ds.append(d)
        sets.append(ds)
    return sets


class CellVelocities(Restorable):
    """The cell-centred velocity of a nodal problem, restorable and stageable
    like a face velocity (u, v, w stand for uc, vc, wc)."""

    def __init__(self, d):
        self.prob = None
        self.d = types.SimpleNamespace(u=d.uc, v=d.vc, w=d.wc)
        self.u0, self.v0, self.w0 = d.uc.clone(), d.vc.clone(), d.wc.clone()


def timed_steps(torch, R, solve, k):
    """k timed projections of R's input by solve(u, v, w): each on its own
    staged copy of the input velocity when they fit, else on R's velocity
    restored before each step.  Returns (seconds, per-step latencies in ms,
    per-step stats, the last step's corrected u, whether copies were staged)."""
    sets = R.stage(k)
    torch.cuda.synchronize()
    lat, stats = [], []
    t0 = time.perf_counter()
    for i in range(k):
        ts = time.perf_counter()
        if sets is None:
            R.restore()
            u, v, w = R.d.u, R.d.v, R.d.w
        else:
            u, v, w = sets[i]
        stats.append(solve(u, v, w))  # returns after the solve's final status is on the host
        lat.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for st in stats:
        assert st["status_name"] == "OK" and st["rel_resid"] <= 1e-10, st
    return elapsed, lat, stats, u, sets is not None


def fp64_leg(args, torch, macproj, R):
    d = R.d
    H = macproj.Hierarchy(macproj.params_of(R.prob))

    def solve(u, v, w):
        return H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, u, v, w, d.phi)

    log(f"{args.n}^3 FP64 warmup {args.warmup}")
    for _ in range(args.warmup):
        R.restore()
        solve(d.u, d.v, d.w)
    log(f"timing {args.steps} steps")
    elapsed, lat, stats, u_last, staged = timed_steps(torch, R, solve, args.steps)
    return H, elapsed, lat, stats, u_last, staged


def smoother_leg(args, torch, H, R):
    """Finest-level fused sweep: HIP events on the stream it is launched on."""
    d = R.d
    stream = torch.cuda.current_stream()
    N = args.n ** 3
    tile = H.sweep_config(0)
    H.set_coefficients(d.rho, d.beta0_cc, d.beta0_edge)    # finest level reads rho, as in the solve
    # steady clocks before timing: at least 0.25 s of back-to-back launches
    # (a GPU left idle, e.g. by host-only work, takes a while to come back up)
    t0, launched = time.perf_counter(), 0
    while launched < 50 or time.perf_counter() - t0 < 0.25:
        for _ in range(25):
            H.level_step(0, "smooth", 1)
        torch.cuda.synchronize()
        launched += 25
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    batches = []
    for _ in range(5):                                       # median of 5 batches of back-to-back launches
        e0.record(stream)
        for _ in range(args.kernel_reps):
            H.level_step(0, "smooth", 1)                     # one launch = one red+black sweep
        e1.record(stream)
        e1.synchronize()
        batches.append(e0.elapsed_time(e1) / args.kernel_reps)
    launch_ms = sorted(batches)[2]
    launch_bytes = SWEEP_BYTES_PER_CELL * N
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9

    # a plain device copy of the same field size on the same stream: the
    # practical HBM ceiling for a read+write stream, and the counter
    # calibration kernel for the traffic figures
    a = torch.empty(N, dtype=torch.float64, device=d.rho.device).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.kernel_reps):
        b.copy_(a)
    e1.record(stream)
    e1.synchronize()
    copy_ms = e0.elapsed_time(e1) / args.kernel_reps
    # three reads and one write over 4 arrays of the same size (more than the
    # 256 MB last-level cache holds): the stream pattern of the sweep itself
    c = torch.empty_like(a).fill_(2.0)
    o = torch.empty_like(a)
    torch.addcmul(a, b, c, out=o)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.kernel_reps):
        torch.addcmul(a, b, c, out=o)
    e1.record(stream)
    e1.synchronize()
    stream_ms = e0.elapsed_time(e1) / args.kernel_reps
    del a, b, c, o

    traffic = None
    sha = sweep_source_sha1()
    if (SWEEP_TRAFFIC and SWEEP_TRAFFIC["sha1"] == sha and tile is not None
            and list(SWEEP_TRAFFIC["tile"]) == list(tile[:3]) and SWEEP_TRAFFIC["n"] == args.n):
        traffic = SWEEP_TRAFFIC["read"] + SWEEP_TRAFFIC["write"]
    # the HBM bytes the counters saw, over the same launch time: what the
    # memory system actually moved (the sweep recomputes its coefficients
    # from rho, so it moves fewer bytes than the algorithmic figure)
    counter_gbs = traffic / (launch_ms * 1e-3) / 1e9 if traffic else None
    tx, ty, tz = tile[:3] if tile else (0, 0, 0)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "achieved_counter_GBs": counter_gbs,
            "frac_counter": counter_gbs / HBM_PEAK_GBS if counter_gbs else None,
            "kernel": f"mg::k_sweep<double, {tx}, {ty}, true, 1, 0, false> (finest level, coefficients from rho, "
                      f"one red+black sweep per launch, {tx}x{ty}-cell tiles, {tz}-plane z-chunks)",
            "launch_ms": launch_ms, "launch_ms_batches": batches, "bytes_per_launch": launch_bytes,
            "bytes_per_cell": SWEEP_BYTES_PER_CELL,
            "kernel_bytes_per_cell": SWEEP_KERNEL_BYTES_PER_CELL,
            "achieved_at_kernel_bytes": SWEEP_KERNEL_BYTES_PER_CELL * N / (launch_ms * 1e-3) / 1e9,
            "copy_GBs": 2 * 8 * N / (copy_ms * 1e-3) / 1e9,
            "stream_3r1w_GBs": 4 * 8 * N / (stream_ms * 1e-3) / 1e9,
            "sweep_source_sha1": sha}


def mixed_leg(args, torch, macproj, R, phi64):
    """The same box in mixed precision; returns the leg's figures and the
    last solve's phi (its error against the oracle is added by the caller)."""
    d = R.d
    Hm = macproj.Hierarchy(macproj.params_of(R.prob, precision="mixed", inner_cycles=args.inner_cycles))

    def solve(u, v, w):
        return Hm.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, u, v, w, d.phi)

    log(f"mixed precision {args.mixed_steps} steps")
    R.restore()
    solve(d.u, d.v, d.w)
    tm, lat, mst, _, staged = timed_steps(torch, R, solve, args.mixed_steps)
    diff = float(torch.linalg.norm(d.phi - phi64) / torch.linalg.norm(phi64))
    phi_mixed = d.phi.clone()
    Hm.close()
    return {"value": args.mixed_steps / tm, "unit": "solves/s", "ms_per_step": tm * 1e3 / args.mixed_steps,
            "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
            "refinement_steps": mst[-1]["cycles"], "rel_resid": mst[-1]["rel_resid"],
            "ms_smooth": mst[-1]["ms_smooth"], "ms_other": mst[-1]["ms_other"],
            "input_copies_staged": staged,
            "phi_rel_diff_vs_fp64_gpu": diff, "phi_rel_err_vs_fp64_oracle": None}, phi_mixed


# finest-level tile configurations the batched sweep takes (32x8, 64x8, 64x16 tiles)
BATCH_TILE_CFGS = (0, 1, 2, 6, 7, 8, 9, 11)


def batch_autotune(args, torch, macproj, rs, specs):
    """Tile choice for the batch as a whole: every problem of a shape sweeps
    its finest level with the same configuration, which the process-wide
    tuning table holds, so a problem solved alone afterwards takes the same
    tiles and the batched results stay bit-identical to one-by-one solves.
    Timed on whole project_batch calls (inputs restored before each): first
    one configuration for every shape, then each shape's own, largest
    shapes first, kept when it is faster by more than 1%.  FP64 entries on
    the FP64 batch, then the FP32 entries on the mixed-precision batch."""
    edges = sorted({e for e, _, _ in specs}, reverse=True)
    macproj.tune_cache_clear()
    choice = {}

    cfg_tile = {0: [32, 8, 32], 1: [32, 8, 64], 2: [64, 8, 32], 6: [32, 8, 16], 7: [32, 8, 8], 8: [64, 8, 64],
                9: [64, 16, 32], 11: [64, 16, 64]}

    def fits(e, c):
        return cfg_tile[c][0] <= e and cfg_tile[c][1] <= e

    def record(fp64):
        for e in edges:
            macproj.tune_record((e, e, e), choice[(e, fp64)], rho=True, fp64=fp64, coarse=False)

    def timed(prec):
        params = [macproj.params_of(r.prob, precision=prec) for r in rs]
        best = None
        for _ in range(3):
            for r in rs:
                r.restore()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            code, _ = macproj.project_batch(params, [r.d for r in rs])
            torch.cuda.synchronize()
            assert code == 0, code
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best

    for fp64, prec in ((True, "fp64"), (False, "mixed")):
        log(f"batch autotune ({prec}): {len(BATCH_TILE_CFGS)} uniform choices, then per shape")
        results = {}
        for c in BATCH_TILE_CFGS:
            for e in edges:
                choice[(e, fp64)] = c if fits(e, c) else 0
            record(fp64)
            results[c] = timed(prec)
        cur = min(results, key=results.get)
        for e in edges:
            choice[(e, fp64)] = cur if fits(e, cur) else 0
        record(fp64)
        t_cur = results[cur]
        for e in edges:
            for c in BATCH_TILE_CFGS:
                if c == choice[(e, fp64)] or not fits(e, c):
                    continue
                old = choice[(e, fp64)]
                choice[(e, fp64)] = c
                record(fp64)
                t = timed(prec)
                if t < 0.99 * t_cur:
                    t_cur = t
                else:
                    choice[(e, fp64)] = old
                    record(fp64)
    return [{"edge": e, "fp64_level0_tile": cfg_tile[choice[(e, True)]],
             "fp32_level0_tile": cfg_tile[choice[(e, False)]]} for e in sorted(edges)]


def batch_leg(args, torch, macproj, inputs, dev):
    """64 independent uneven boxes: one project_batch call against one
    mac_project call per problem (hierarchies kept, as the batch keeps them),
    in mixed precision (FP32 cycles, FP64 refinement) and in FP64."""
    specs = inputs.mixed_batch_specs(64)
    log("batch: generating 64 problems")
    rs = [Restorable(macproj, inputs.make_problem(e, H=H, rho_noise=0.01, seed=s), dev) for e, H, s in specs]
    cells = sum(r.prob.ncells for r in rs)
    tuned = batch_autotune(args, torch, macproj, rs, specs) if args.autotune else []
    out = {"problems": 64, "cells": cells, "autotuned": tuned}
    for prec in ("mixed", "fp64"):
        params = [macproj.params_of(r.prob, precision=prec) for r in rs]

        def run_batch(ds=None):
            if ds is None:                      # restored in place (untimed, or past the staging cap)
                for r in rs:
                    r.restore()
                ds = [r.d for r in rs]
            code, st = macproj.project_batch(params, ds)
            assert code == 0 and all(s["status_name"] == "OK" and s["rel_resid"] <= 1e-10 for s in st), code
            return st

        log(f"batch ({prec}): {args.batch_reps} x project_batch(64)")
        run_batch()
        sets = stage_problems(rs, args.batch_reps)   # each timed call projects its own input copies
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.batch_reps):
            st = run_batch(sets[i] if sets else None)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / args.batch_reps
        staged = sets is not None
        del sets
        phis = [r.d.phi.clone() for r in rs]

        log(f"batch ({prec}): the same 64 problems one by one")
        hs = [macproj.Hierarchy(p) for p in params]

        def run_solo(ds=None):
            if ds is None:
                for r in rs:
                    r.restore()
                ds = [r.d for r in rs]
            return [h.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi)
                    for h, d in zip(hs, ds)]

        run_solo()
        sets = stage_problems(rs, args.batch_reps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.batch_reps):
            so = run_solo(sets[i] if sets else None)
        torch.cuda.synchronize()
        ts = (time.perf_counter() - t0) / args.batch_reps
        del sets
        identical = all(torch.equal(p, r.d.phi) for p, r in zip(phis, rs))
        for h in hs:
            h.close()
        del phis
        out[prec] = {"value": 64 / tb, "unit": "solves/s", "ms_per_batch": tb * 1e3,
                     "one_by_one": {"value": 64 / ts, "ms_per_batch": ts * 1e3},
                     "speedup_vs_one_by_one": ts / tb,
                     "cycles_total": sum(s["cycles"] for s in st), "cycles_one_by_one": sum(s["cycles"] for s in so),
                     "phi_identical_to_one_by_one": identical, "input_copies_staged": staged}
    del rs
    return out


def serve_leg(args, torch, macproj, inputs, dev):
    """Open-loop Poisson arrivals through the continuous-batching server.
    Each size has a few buffer sets (distinct problems); a request takes a
    free set of its size, has its velocity restored and is submitted at its
    arrival time.  Latency = (submission delay past the arrival time) +
    the server's submit-to-done time."""
    pools = {32: 32, 64: 24, 128: 12, 256: 8}
    log("serve: generating buffer sets")
    sets = {}
    for e, m in pools.items():
        sets[e] = [Restorable(macproj, inputs.make_problem(e, H=0.08 + 0.42 * (k + 0.5) / m, rho_noise=0.01,
                                                             seed=50000 + 100 * e + k), dev) for k in range(m)]
    torch.cuda.synchronize()
    out = []
    runs = [(r, "fp64") for r in args.serve_rates] + [(r, "mixed") for r in args.serve_mixed_rates]
    for rate, prec in runs:
        reqs = inputs.serving_requests(args.serve_warmup + args.serve_requests, rate)
        S = macproj.Server(hbm_budget_bytes=200 << 30, max_inflight=64)
        busy = {e: [None] * len(v) for e, v in sets.items()}   # ticket holding each set
        done = {}

        def finish(t):
            if t not in done:
                done[t] = S.wait(t)

        def free_set(e):
            for k, t in enumerate(busy[e]):
                if t is None:
                    return k
                if t in done:
                    return k
                r = S.poll(t)
                if r is not None:
                    done[t] = r
                    return k
            k = min(range(len(busy[e])), key=lambda i: busy[e][i])   # oldest ticket of this size
            finish(busy[e][k])
            return k

        log(f"serve ({prec}): {len(reqs)} requests at {rate} req/s ({args.serve_warmup} warm-up)")
        tickets = []
        t0 = time.perf_counter()
        t_meas = None
        for q, (ta, e, H, tol, _seed) in enumerate(reqs):
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            if q == args.serve_warmup:
                t_meas = time.perf_counter() - t0
            k = free_set(e)
            r = sets[e][k]
            r.restore()
            p = macproj.params_of(r.prob, rtol=tol, precision=prec)
            delay = max(0.0, time.perf_counter() - t0 - ta)
            t = S.submit(p, r.d)
            busy[e][k] = t
            tickets.append((t, delay, e, tol, q >= args.serve_warmup))
        for t, _, _, _, _ in tickets:
            finish(t)
        t_end = time.perf_counter() - t0
        c = S.counters()
        S.close()
        lat = []
        for t, delay, e, tol, measured in tickets:
            st = done[t]
            assert st["status_name"] == "OK" and st["rel_resid"] <= tol, (e, st)
            if measured:
                lat.append(delay * 1e3 + st["ms_total"])
        meas = [x for x in tickets if x[4]]
        mix = {e: sum(1 for x in meas if x[2] == e) for e in pools}
        t_meas = t_meas if t_meas is not None else 0.0
        out.append({"rate": rate, "precision": prec, "requests": len(meas), "warmup": args.serve_warmup,
                    "solves_per_s": len(meas) / max(t_end - t_meas, 1e-9),
                    "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
                    "peak_inflight": c["peak_inflight"], "mix": mix})
        log(f"serve ({prec}) {rate} req/s: {out[-1]['solves_per_s']:.1f} solves/s, "
            f"p50 {out[-1]['p50_ms']:.2f} ms, p99 {out[-1]['p99_ms']:.2f} ms")
    del sets
    return {"budget_bytes": 200 << 30, "max_inflight": 64,
            "workload": "open-loop Poisson arrivals; sizes 32/64/128/256^3 with weights 0.4/0.3/0.2/0.1, "
                        "H ~ U(0.08, 0.5), rtol 1e-8 or 1e-10 per request; latency = submission delay past the "
                        "arrival time + submit-to-done; solves/s over the measured requests",
            "rates": out}


def full_leg(args, torch, macproj, inputs, dev):
    """The same box size with the base state given as p0 and Gamma1: each step
    computes beta0 on the device and projects with the dp0/dt term in the
    right-hand side (FP64)."""
    log(f"full right-hand side: {args.full_steps} steps")
    prob = inputs.make_full_problem(args.n, seed=5)
    R = Restorable(macproj, prob, dev)
    d = R.d
    H = macproj.Hierarchy(macproj.params_of(prob))

    def solve(u, v, w):
        b0c, b0e = macproj.mg_beta0_from_p0(prob.rho0_base, d.p0_edge, d.p0_cc, d.gamma1_cc)
        return H.mac_project_full(d.rho, b0c, b0e, d.S, d.p0_cc, d.gamma1_cc, d.dp0dt_cc, u, v, w, d.phi)

    R.restore()
    solve(d.u, d.v, d.w)
    tf, _, stats, _, staged = timed_steps(torch, R, solve, args.full_steps)
    H.close()
    return {"value": args.full_steps / tf, "unit": "solves/s", "ms_per_step": tf * 1e3 / args.full_steps,
            "cycles": stats[-1]["cycles"], "input_copies_staged": staged,
            "workload": f"{args.n}^3, p0 = exp(-z/0.25), Gamma1 1.67 -> 1.3, "
                        "beta0 computed on the device each step, dp0/dt term in f"}


def star_leg(args, torch, macproj, inputs, dev):
    """A star-like box of the same size: beta0 a function of the radius from
    the box centre (radial profile, mapped onto faces and cells on the
    device), every side an outflow side (phi = 0), FP64 and mixed precision."""
    prob = inputs.make_star_problem(args.n, Hr=0.1, rho_noise=0.01, seed=6)
    R = Restorable(macproj, prob, dev)
    d = R.d
    out = {"workload": f"{args.n}^3, beta0 = exp(-r/0.1) on a radial profile of {len(prob.beta0_r)} points "
                       f"(dr = dx/2) about the box centre, outflow on all six sides, rtol 1e-10"}
    for prec in ("fp64", "mixed"):
        log(f"star box ({prec}): {args.star_steps} steps")
        H = macproj.Hierarchy(macproj.params_of(prob, precision=prec))

        def solve(u, v, w):
            return H.mac_project_radial(d.rho, d.beta0_r, prob.dr_base, prob.centre, d.S, u, v, w, d.phi)

        R.restore()
        solve(d.u, d.v, d.w)
        ts, _, stats, _, staged = timed_steps(torch, R, solve, args.star_steps)
        H.close()
        out[prec] = {"value": args.star_steps / ts, "unit": "solves/s", "ms_per_step": ts * 1e3 / args.star_steps,
                     "cycles": stats[-1]["cycles"], "rel_resid": stats[-1]["rel_resid"],
                     "input_copies_staged": staged}
    return out


def nodal_leg(args, torch, macproj, inputs, dev):
    """The nodal (cell-velocity) projection of the same box size: phi on the
    nodes, cell-centred velocities, FP64 and mixed precision."""
    prob = inputs.make_nodal_problem(args.n, H=0.1, rho_noise=0.01, seed=7)
    d = macproj.nodal_to_device(prob, dev)
    R = CellVelocities(d)
    H = macproj.NodalHierarchy(macproj.make_params(prob.n, prob.dx, prob.periodic))
    log(f"nodal projection: {args.nodal_steps} steps")

    def solve(u, v, w):
        return H.project(d.rho, d.beta0_cc, d.S, u, v, w, d.phi)

    R.restore()
    solve(d.uc, d.vc, d.wc)
    tn, _, stats, _, staged = timed_steps(torch, R, solve, args.nodal_steps)
    st = stats[-1]
    # one four-colour Gauss-Seidel sweep of the finest level (one fused launch)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    H.level_step(0, "smooth", 1)
    e0.record()
    H.level_step(0, "smooth", args.kernel_reps)
    e1.record()
    torch.cuda.synchronize()
    sweep_ms = e0.elapsed_time(e1) / args.kernel_reps
    H.close()
    phi64 = d.phi.clone()
    # the same problem in mixed precision (FP32 V-cycles, FP64 refinement)
    Hm = macproj.NodalHierarchy(macproj.make_params(prob.n, prob.dx, prob.periodic, precision="mixed"))
    log(f"nodal projection, mixed precision: {args.nodal_steps} steps")

    def solve_m(u, v, w):
        return Hm.project(d.rho, d.beta0_cc, d.S, u, v, w, d.phi)

    R.restore()
    solve_m(d.uc, d.vc, d.wc)
    tm, _, stats_m, _, _ = timed_steps(torch, R, solve_m, args.nodal_steps)
    stm = stats_m[-1]
    diff = float(torch.linalg.vector_norm(d.phi - phi64) / torch.linalg.vector_norm(phi64))
    Hm.close()
    nodes = (args.n ** 2) * (args.n + 1)
    return {"value": args.nodal_steps / tn, "unit": "solves/s", "ms_per_step": tn * 1e3 / args.nodal_steps,
            "cycles": st["cycles"], "rel_resid": st["rel_resid"], "input_copies_staged": staged,
            "fine_sweep_ms": sweep_ms,
            "fine_sweep_GBs_at_24B_per_node": 24.0 * nodes / (sweep_ms * 1e-3) / 1e9,
            "mixed": {"value": args.nodal_steps / tm, "unit": "solves/s", "ms_per_step": tm * 1e3 / args.nodal_steps,
                      "refinement_steps": stm["cycles"], "rel_resid": stm["rel_resid"],
                      "phi_rel_diff_vs_fp64_gpu": diff},
            "workload": f"{args.n}^3 cells ({nodes} nodes), beta0 = exp(-z/0.1), periodic x,y, walls z, rtol 1e-10"}


def boxes_leg(args, torch, macproj, R):
    """The same 256^3 box with its finest level split into boxes (one ghost
    layer each, a halo-exchange kernel after every colour), FP64."""
    d = R.d
    out = {"workload": f"{args.n}^3 steep-stratification box, finest level as boxes with halo exchange, FP64, "
                       f"rtol 1e-10"}
    for b in (args.n // 4, args.n // 2):
        log(f"multi-box finest level, boxes of {b}^3: {args.boxes_steps} steps")
        H = macproj.Hierarchy(macproj.params_of(R.prob))
        H.set_boxes((b, b, b))

        def solve(u, v, w):
            return H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, u, v, w, d.phi)

        R.restore()
        solve(d.u, d.v, d.w)
        tb, _, stats, _, staged = timed_steps(torch, R, solve, args.boxes_steps)
        H.close()
        out[f"{b}^3 x {(args.n // b) ** 3}"] = {"value": args.boxes_steps / tb, "unit": "solves/s",
                                               "ms_per_step": tb * 1e3 / args.boxes_steps,
                                               "cycles": stats[-1]["cycles"], "input_copies_staged": staged}
    return out


def n512_leg(args, torch, macproj, inputs, dev):
    """The 512^3 box (H = 0.15, 5% density noise): mixed precision (FP32
    cycles, FP64 refinement) against FP64, every solve's phi compared with the
    FP64 oracle's exact discrete solution (definition mode)."""
    from oracle import oracle as orc
    prob = inputs.MIXED_512()
    log("512^3: FP64 oracle, definition mode (host)")
    tc = time.perf_counter()
    ref = orc.mac_project(prob, mode="definition")
    t_oracle = time.perf_counter() - tc
    assert ref["status"] == 0
    R = Restorable(macproj, prob, dev)
    d = R.d
    phi_ref = torch.from_numpy(ref["phi"]).to(dev)
    nref = float(torch.linalg.norm(phi_ref))
    del ref
    out = {"workload": "512^3 box, beta0 = exp(-z/0.15), rho = beta0 (1 + 0.05 N(0,1)), S = 0.1 N(0,1) "
                       "weighted-mean-removed, periodic x,y, walls z, rtol 1e-10",
           "oracle_definition_s": t_oracle}
    for prec in ("mixed", "fp64"):
        H = macproj.Hierarchy(macproj.params_of(prob, precision=prec))

        def solve(u, v, w):
            return H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, u, v, w, d.phi)

        log(f"512^3 {prec}: {args.n512_steps} solves")
        R.restore()
        solve(d.u, d.v, d.w)
        sets = R.stage(args.n512_steps)            # one input copy per timed solve, made untimed
        torch.cuda.synchronize()
        errs, lat = [], []
        tt = 0.0
        for i in range(args.n512_steps):
            if sets is None:
                R.restore()
                torch.cuda.synchronize()
                u, v, w = d.u, d.v, d.w
            else:
                u, v, w = sets[i]
            ts = time.perf_counter()
            st = solve(u, v, w)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - ts) * 1e3)
            tt += lat[-1] * 1e-3
            assert st["status_name"] == "OK" and st["rel_resid"] <= 1e-10, st
            errs.append(float(torch.linalg.norm(d.phi - phi_ref)) / nref)
        H.close()
        del sets
        out[prec] = {"value": args.n512_steps / tt, "unit": "solves/s", "ms_per_step": tt * 1e3 / args.n512_steps,
                     "cycles": st["cycles"], "rel_resid": st["rel_resid"],
                     "phi_rel_err_vs_fp64_oracle": errs, "ms_smooth": st["ms_smooth"]}
    out["mixed_speedup_vs_fp64"] = out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"]
    del R, phi_ref
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_leg(args, prob):
    log("CPU oracle baseline")
    from oracle import oracle as orc
    solves = 0
    tc0 = time.perf_counter()
    while True:                       # whole solves until ~10 s of CPU work (at most 8)
        ref = orc.mac_project(prob)
        assert ref["status"] == 0
        solves += 1
        tc = time.perf_counter() - tc0
        if tc >= 10.0 or solves >= 8:
            break
    return {"value": solves / tc, "unit": "solves/s", "cores": orc.max_threads(), "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": f"{solves} full {args.n}^3 FP64 projections of the same box (algorithm mode, "
                      f"{ref['cycles']} V-cycles each), {tc:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="box edge (default 256)")
    ap.add_argument("--mixed-steps", type=int, default=5)
    ap.add_argument("--inner-cycles", type=int, default=0,
                    help="FP32 V-cycles per refinement step of the single-box mixed solves (0: one)")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--batch-reps", type=int, default=3, help="0 skips the batch leg")
    ap.add_argument("--autotune", type=int, default=1, help="tune the batch's tile choices on the batch first")
    ap.add_argument("--serve-rates", type=float, nargs="*", default=[50.0, 100.0, 200.0, 500.0, 1000.0, 1500.0,
                                                                     2000.0])
    ap.add_argument("--serve-mixed-rates", type=float, nargs="*", default=[200.0, 1000.0],
                    help="rates served in mixed precision")
    ap.add_argument("--serve-requests", type=int, default=2000, help="measured requests per rate")
    ap.add_argument("--serve-warmup", type=int, default=200, help="requests before the measured ones")
    ap.add_argument("--n512-steps", type=int, default=3, help="0 skips the 512^3 leg")
    ap.add_argument("--full-steps", type=int, default=5, help="0 skips the p0/Gamma1 base-state leg")
    ap.add_argument("--star-steps", type=int, default=5, help="0 skips the radial-base-state outflow leg")
    ap.add_argument("--nodal-steps", type=int, default=3, help="0 skips the nodal-projection leg")
    ap.add_argument("--boxes-steps", type=int, default=3, help="0 skips the multi-box finest-level leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--oracle-check", type=int, default=1,
                    help="compare the headline phi with the FP64 oracle's exact solution (host)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs the projection on one GPU only; "
              "--gpus N with N > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1910_12979_amd import inputs, macproj

    if not os.path.exists(macproj.LIB_PATH):
        from paper_1910_12979_amd import build as hip_build
        hip_build.build()
    torch.cuda.set_device(0)
    dev = "cuda:0"
    n = args.n
    prob = inputs.STEEP_256(n=n)
    R = Restorable(macproj, prob, dev)

    H, elapsed, lat, stats, u_last, staged = fp64_leg(args, torch, macproj, R)
    value = args.steps / elapsed
    cycles = stats[-1]["cycles"]
    phi64 = R.d.phi.clone()
    # GPU timings first (the host-only oracle below leaves the GPU idle, and
    # its clocks take a while to come back)
    log("smoother kernel timing")
    roofline = smoother_leg(args, torch, H, R)
    H.close()
    mixed, phi_mixed = mixed_leg(args, torch, macproj, R, phi64) if args.mixed_steps > 0 else (None, None)

    parity = None
    if args.oracle_check:
        # every timed solve projects the same input: the last one's phi
        # against the FP64 oracle's exact discrete solution (definition mode)
        from oracle import oracle as orc
        log(f"{n}^3: FP64 oracle, definition mode (host)")
        tc = time.perf_counter()
        ref = orc.mac_project(prob, mode="definition")
        assert ref["status"] == 0
        phi_ref = torch.from_numpy(ref["phi"]).to(dev)
        nref = torch.linalg.norm(phi_ref)
        parity = {"phi_rel_err_vs_fp64_oracle": float(torch.linalg.norm(phi64 - phi_ref) / nref),
                  "u_rel_err_vs_fp64_oracle": float(np.linalg.norm(u_last.cpu().numpy() - ref["u"])
                                                    / np.linalg.norm(ref["u"])),
                  "oracle_definition_s": time.perf_counter() - tc,
                  "ms_smooth": stats[-1]["ms_smooth"], "ms_other": stats[-1]["ms_other"]}
        if mixed is not None:
            mixed["phi_rel_err_vs_fp64_oracle"] = float(torch.linalg.norm(phi_mixed - phi_ref) / nref)
        del ref, phi_ref
    del phi64, phi_mixed
    batch = batch_leg(args, torch, macproj, inputs, dev) if args.batch_reps > 0 else None
    serve = serve_leg(args, torch, macproj, inputs, dev) if (args.serve_rates or args.serve_mixed_rates) else None
    n512 = n512_leg(args, torch, macproj, inputs, dev) if args.n512_steps > 0 else None
    full = full_leg(args, torch, macproj, inputs, dev) if args.full_steps > 0 else None
    star = star_leg(args, torch, macproj, inputs, dev) if args.star_steps > 0 else None
    nodal = nodal_leg(args, torch, macproj, inputs, dev) if args.nodal_steps > 0 else None
    boxes = boxes_leg(args, torch, macproj, R) if args.boxes_steps > 0 else None
    cpu = None if args.no_cpu_baseline else cpu_leg(args, prob)

    model_bytes = n ** 3 * (156.0 + cycles * 326.0)
    out = {
        "metric": "MAC-projection solves/s at 256^3 to 1e-10 resid, mixed vs FP64; p99 latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 steep-stratification box (H=0.1, periodic x,y, walls z), "
                               f"FP64 V(2,2) red-black GS multigrid to 1e-10",
                   "n": n, "rtol": 1e-10, "precision": "fp64", "cycles": cycles,
                   "input_copies_staged": staged},
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
        "parity": parity,
        "roofline": roofline,
        "model_roofline_frac": value * model_bytes / (HBM_PEAK_GBS * 1e9),
        "mixed": mixed,
        "batch": batch,
        "serve": serve,
        "n512": n512,
        "full_rhs": full,
        "star_outflow": star,
        "nodal": nodal,
        "multi_box": boxes,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
