#!/usr/bin/env python3
"""Benchmark: variable-coefficient MAC-projection solves/s on one MI355X.

Workload: the 256^3 steeply stratified box (periodic x,y, solid walls in z,
beta0 = exp(-z/0.1), rho = beta0 (1 + 0.01 N(0,1)), S = 0.1 N(0,1) with its
beta0-weighted mean removed, U ~ N(0,1)), FP64, V(2,2) red-black GS cycles
to a 1e-10 relative residual.  One step = one whole projection (coefficients,
right-hand side, V-cycles, velocity correction) of the same input; the input
velocity is restored from a device copy before each step (a device-to-device
copy inside the timed region).  Inputs are resident in HBM before timing.

Also reported: the same box in mixed precision (FP32 cycles with FP64
iterative refinement), the smoother's roofline figure measured with HIP
events, per-step latency percentiles, and the FP64 CPU oracle timed on the
host cores on whole solves of the same box (about 10 s of CPU work).

Prints one JSON line.  `--gpus` above 1 is refused: this path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# One fused FP64 sweep on the finest level reads phi_in, f and rho and writes
# phi_out once: 32 bytes per cell (the face coefficients are recomputed from
# rho).  A stored-coefficient sweep would read 24 bytes of coefficients
# instead of rho's 8 (48 bytes per cell); that figure is reported beside it.
SWEEP_BYTES_PER_CELL = 32.0
SWEEP_BYTES_STORED_COEFF = 48.0


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256, help="box edge (default 256)")
    ap.add_argument("--mixed-steps", type=int, default=5)
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs the projection on one GPU only; "
              "--gpus N with N > 1 is not supported", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1910_12979_amd import inputs, macproj

    if not os.path.exists(macproj.LIB_PATH):
        from paper_1910_12979_amd import build as hip_build
        hip_build.build()
    torch.cuda.set_device(0)
    dev = "cuda:0"
    n = args.n
    prob = inputs.STEEP_256(n=n)
    d = macproj.to_device(prob, dev)
    u0, v0, w0 = d.u.clone(), d.v.clone(), d.w.clone()
    H = macproj.Hierarchy(macproj.params_of(prob))
    stream = torch.cuda.current_stream()

    def step(h):
        d.u.copy_(u0)
        d.v.copy_(v0)
        d.w.copy_(w0)
        return h.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi)

    print(f"[bench] {n}^3 FP64 warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step(H)
    torch.cuda.synchronize()
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    lat = []
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        st = step(H)
        lat.append((time.perf_counter() - ts) * 1e3)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    for st in stats:
        assert st["status_name"] == "OK" and st["rel_resid"] <= 1e-10, st
    value = args.steps / elapsed
    cycles = stats[-1]["cycles"]
    phi64 = d.phi.clone()

    # --- smoother roofline: HIP events around level-0 sweeps on this stream
    print("[bench] smoother kernel timing", file=sys.stderr, flush=True)
    N = n ** 3
    H.set_coefficients(d.rho, d.beta0_cc, d.beta0_edge)    # finest level reads rho, as in the solve
    H.level_step(0, "smooth", 1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.kernel_reps):
        H.level_step(0, "smooth", 1)
    e1.record(stream)
    e1.synchronize()
    launch_ms = e0.elapsed_time(e1) / args.kernel_reps   # one launch = one whole sweep
    launch_bytes = SWEEP_BYTES_PER_CELL * N
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    achieved_stored = SWEEP_BYTES_STORED_COEFF * N / (launch_ms * 1e-3) / 1e9
    H.close()

    # --- mixed precision on the same box
    mixed = None
    if args.mixed_steps > 0:
        print(f"[bench] mixed precision {args.mixed_steps} steps", file=sys.stderr, flush=True)
        Hm = macproj.Hierarchy(macproj.params_of(prob, precision="mixed"))
        step(Hm)
        torch.cuda.synchronize()
        tm0 = time.perf_counter()
        mst = []
        for _ in range(args.mixed_steps):
            mst.append(step(Hm))
        torch.cuda.synchronize()
        tm1 = time.perf_counter()
        for st in mst:
            assert st["status_name"] == "OK" and st["rel_resid"] <= 1e-10, st
        diff = float(torch.linalg.norm(d.phi - phi64) / torch.linalg.norm(phi64))
        mixed = {"value": args.mixed_steps / (tm1 - tm0), "unit": "solves/s",
                 "ms_per_step": (tm1 - tm0) * 1e3 / args.mixed_steps,
                 "refinement_steps": mst[-1]["cycles"], "rel_resid": mst[-1]["rel_resid"],
                 "phi_rel_diff_vs_fp64_gpu": diff}
        Hm.close()

    # --- CPU oracle on the host cores: one FP64 solve of the same box
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
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
        cpu = {"value": solves / tc, "unit": "solves/s", "cores": orc.max_threads(), "kind": "oracle",
               "sample": f"{solves} full {n}^3 FP64 projections of the same box (algorithm mode, "
                         f"{ref['cycles']} V-cycles each), {tc:.1f} s wall"}

    model_bytes = N * (156.0 + cycles * 326.0)
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
                   "n": n, "rtol": 1e-10, "precision": "fp64", "cycles": cycles},
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_sweep<double, 32, 8, true, 1> (finest level, one red+black sweep per launch)",
                     "launch_ms": launch_ms, "bytes_per_launch": launch_bytes,
                     "achieved_at_48B_per_cell": achieved_stored},
        "model_roofline_frac": value * model_bytes / (HBM_PEAK_GBS * 1e9),
        "mixed": mixed,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
