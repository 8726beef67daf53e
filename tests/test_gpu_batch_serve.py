"""Batched and served projections (GPU): each result must be the one the
single-problem path gives for that problem alone, bit for bit (same kernels,
same per-problem tiles and reduction order), and the single-problem path is
itself checked against the oracle elsewhere; a few problems are re-checked
against the oracle here too."""
import time

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1910_12979_amd import inputs as I

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def solo(mp, prob, precision="fp64", inner_cycles=0):
    H = mp.Hierarchy(mp.params_of(prob, precision=precision, inner_cycles=inner_cycles))
    d = mp.to_device(prob)
    st = H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi,
                       allow=(0, -1, -3, -4, -5))
    torch.cuda.synchronize()
    H.close()
    return st, {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("phi", "u", "v", "w"))


def mixed_problems(count, seed=3, edges=(32, 48, 64, 96, 128)):
    return [I.make_problem(e, H=H, rho_noise=0.01, seed=s)
            for e, H, s in I.mixed_batch_specs(count, seed=seed, edges=edges)]


def test_batch_matches_single_problem_bitwise(mp):
    probs = [I.make_problem(32, seed=1), I.make_problem(48, H=0.2, seed=2),
             I.make_problem((40, 24, 56), seed=3, dx=1 / 40), I.make_problem(64, H=0.1, seed=4),
             I.make_problem((64, 32, 32), seed=5, periodic=(False, True, False), dx=1 / 64),
             I.make_problem(16, seed=6),                        # not batchable: solved alone inside
             I.make_problem(64, seed=7, rtol=1e-8)]
    ref = [solo(mp, p) for p in probs]
    devs = [mp.to_device(p) for p in probs]
    code, stats = mp.project_batch([mp.params_of(p) for p in probs], devs)
    torch.cuda.synchronize()
    assert code == 0
    for p, (st0, out0), st, d in zip(probs, ref, stats, devs):
        out = {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}
        assert st["status_name"] == "OK"
        assert st["cycles"] == st0["cycles"] and st["rel_resid"] == st0["rel_resid"]
        assert same(out, out0), p.n


def test_batch_mixed_precision_matches_single_problem_bitwise(mp):
    """Mixed-precision problems in a batch (FP32 cycles and FP64 refinements
    in shared launches, mixed with FP64 problems) equal their single-problem
    mixed solves bit for bit; shapes the batched FP32 cycle does not cover
    (a 24^3 level too large for the bottom solver in FP64 would be fine in
    FP32; 40x24x56 has a non-fused level above the bottom) are solved alone
    inside the call."""
    probs = [(I.make_problem(32, seed=21), "mixed"), (I.make_problem(64, H=0.1, seed=22), "mixed"),
             (I.make_problem((128, 64, 32), seed=23, dx=1 / 128), "mixed"),
             (I.make_problem(48, H=0.2, seed=24), "mixed"),
             (I.make_problem((40, 24, 56), seed=25, dx=1 / 40), "mixed"),
             (I.make_problem(64, seed=26, rtol=1e-8), "mixed"),
             (I.make_problem(64, seed=27), "fp64")]
    ref = [solo(mp, p, prec) for p, prec in probs]
    devs = [mp.to_device(p) for p, _ in probs]
    code, stats = mp.project_batch([mp.params_of(p, precision=prec) for p, prec in probs], devs)
    torch.cuda.synchronize()
    assert code == 0
    for (p, prec), (st0, out0), st, d in zip(probs, ref, stats, devs):
        out = {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}
        assert st["status_name"] == "OK" and st["rel_resid"] <= p.rtol
        assert st["cycles"] == st0["cycles"] and st["rel_resid"] == st0["rel_resid"], (p.n, prec)
        assert same(out, out0), (p.n, prec)


def test_batch_mixed_inner_cycles_match_single_problem_bitwise(mp):
    """Mixed-precision problems with 1, 2 (the default) and 3 FP32 V-cycles
    per refinement step in one batch: the batch runs each problem's extra
    V-cycles on the subset that has them, and every problem equals its
    single-problem solve bit for bit."""
    probs = [(I.make_problem(64, H=0.1, seed=31), 1), (I.make_problem(64, H=0.1, seed=31), 0),
             (I.make_problem(48, H=0.2, seed=32), 3), (I.make_problem(32, seed=33), 1),
             (I.make_problem((128, 64, 32), seed=34, dx=1 / 128), 2)]
    ref = [solo(mp, p, "mixed", inner_cycles=k) for p, k in probs]
    devs = [mp.to_device(p) for p, _ in probs]
    code, stats = mp.project_batch([mp.params_of(p, precision="mixed", inner_cycles=k) for p, k in probs], devs)
    torch.cuda.synchronize()
    assert code == 0
    for (p, k), (st0, out0), st, d in zip(probs, ref, stats, devs):
        out = {name: getattr(d, name).cpu().numpy() for name in ("phi", "u", "v", "w")}
        assert st["status_name"] == "OK" and st["rel_resid"] <= p.rtol
        assert st["cycles"] == st0["cycles"] and st["rel_resid"] == st0["rel_resid"], (p.n, k)
        assert same(out, out0), (p.n, k)
    # more V-cycles per step, fewer refinement steps
    assert stats[0]["cycles"] >= stats[1]["cycles"]


def test_batch_reuses_pooled_states_with_other_inner_cycles(mp):
    """Back-to-back batches of the same shapes reuse the pooled states and
    their captured rounds; a batch that asks for another number of FP32
    V-cycles per refinement step must run that number, not replay the
    previous batch's rounds."""
    probs = [I.make_problem(64, H=0.1, seed=41), I.make_problem(64, H=0.2, seed=42)]
    for k in (1, 3, 1):
        ref = [solo(mp, p, "mixed", inner_cycles=k) for p in probs]
        devs = [mp.to_device(p) for p in probs]
        code, stats = mp.project_batch([mp.params_of(p, precision="mixed", inner_cycles=k) for p in probs], devs)
        torch.cuda.synchronize()
        assert code == 0
        for p, (st0, out0), st, d in zip(probs, ref, stats, devs):
            out = {name: getattr(d, name).cpu().numpy() for name in ("phi", "u", "v", "w")}
            assert st["status_name"] == "OK"
            assert st["cycles"] == st0["cycles"] and st["rel_resid"] == st0["rel_resid"], k
            assert same(out, out0), k


def test_batch_isolates_failing_problems(mp):
    good = I.make_problem(32, seed=11)
    bad_rhs = I.make_problem(32, seed=12); bad_rhs.w[0, 3, 3] = 1.0
    bad_nan = I.make_problem(48, seed=13); bad_nan.S[1, 1, 1] = np.nan
    short = I.make_problem(64, seed=14, max_cycles=2)
    probs = [good, bad_rhs, bad_nan, short]
    ref = [solo(mp, p) for p in probs]
    devs = [mp.to_device(p) for p in probs]
    code, stats = mp.project_batch([mp.params_of(p) for p in probs], devs)
    torch.cuda.synchronize()
    assert [s["status_name"] for s in stats] == ["OK", "INCOMPATIBLE_RHS", "NONFINITE", "NOT_CONVERGED"]
    assert code != 0
    for i in (0, 3):
        out = {k: getattr(devs[i], k).cpu().numpy() for k in ("phi", "u", "v", "w")}
        assert same(out, ref[i][1])
    assert stats[3]["cycles"] == 2


def test_batch_of_64_uneven_boxes_full_size(mp):
    """The 64-problem batch (edges 32..128): every problem bitwise equal to
    its single-problem solve; four of them checked against the oracle."""
    probs = mixed_problems(64)
    devs = [mp.to_device(p) for p in probs]
    code, stats = mp.project_batch([mp.params_of(p) for p in probs], devs)
    torch.cuda.synchronize()
    assert code == 0 and all(s["status_name"] == "OK" and s["rel_resid"] <= 1e-10 for s in stats)
    outs = [{k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")} for d in devs]
    del devs
    for i in range(0, 64, 4):
        st0, out0 = solo(mp, probs[i])
        assert same(outs[i], out0), (i, probs[i].n)
        assert stats[i]["cycles"] == st0["cycles"]
    for i in (0, 1, 2, 3):
        ref = O.mac_project(probs[i], mode="definition")
        assert rel(outs[i]["phi"], ref["phi"]) <= 1e-9


def test_server_results_equal_single_problem(mp):
    """Requests of mixed sizes, tolerances and precisions submitted while
    others run: each served result equals the single-problem solve of the
    same request bit for bit, and three of them are checked against the
    oracle's exact discrete solution (definition mode): an FP64 and a
    mixed-precision request at rtol 1e-10 within 1e-9, and a request at rtol
    1e-8 within the bar its tolerance allows (3 x the oracle's own
    deviation when it stops at 1e-8), its residual evaluated by the oracle."""
    sizes = (32, 64, 32, 48, 64, 32, 96, 32)
    probs = [I.make_problem(e, H=0.1 + 0.05 * k, seed=100 + k, rtol=(1e-8 if k % 2 else 1e-10))
             for k, e in enumerate(sizes)]
    precs = ["mixed" if k in (2, 3, 6) else "fp64" for k in range(len(probs))]
    ref = [solo(mp, p, prec) for p, prec in zip(probs, precs)]
    S = mp.Server(hbm_budget_bytes=8 << 30, max_inflight=16)
    devs = [mp.to_device(p) for p in probs]
    tickets = []
    for k, (p, d, prec) in enumerate(zip(probs, devs, precs)):
        tickets.append(S.submit(mp.params_of(p, precision=prec), d))
        if k == 3:
            time.sleep(0.002)               # later requests arrive while the first are running
    res = [S.wait(t) for t in tickets]
    c = S.counters()
    S.close()
    assert c["completed"] == len(probs) and c["peak_inflight"] >= 2
    outs = []
    for p, d, r, (st0, out0), prec in zip(probs, devs, res, ref, precs):
        assert r["status_name"] == "OK" and r["rel_resid"] <= p.rtol and r["cycles"] == st0["cycles"]
        out = {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}
        assert same(out, out0), (p.n, prec)
        outs.append(out)
    # served results against the oracle
    for k in (0, 2):                        # rtol 1e-10: FP64 (k = 0) and mixed (k = 2)
        assert probs[k].rtol == 1e-10
        d = O.mac_project(probs[k], mode="definition")
        assert d["status"] == 0
        assert rel(outs[k]["phi"], d["phi"]) <= 1e-9, (k, precs[k])
    k = 1                                   # rtol 1e-8, FP64
    p = probs[k]
    d = O.mac_project(p, mode="definition")
    a = O.mac_project(p)                    # the oracle's own iterate at the same 1e-8 stop
    e_alg = rel(a["phi"], d["phi"])
    assert rel(outs[k]["phi"], d["phi"]) <= max(1e-9, 3 * e_alg), (rel(outs[k]["phi"], d["phi"]), e_alg)
    cf = O.face_coeffs(p.n, p.periodic, p.rho, p.beta0_cc, p.beta0_edge)
    f = O.rhs(p.n, p.periodic, p.dx, p.beta0_cc, p.beta0_edge, p.u, p.v, p.w, p.S)
    f -= f.mean()
    r = O.residual(p.n, p.periodic, p.dx, cf, outs[k]["phi"], f)
    assert np.linalg.norm(r) <= 1.05e-8 * np.linalg.norm(f)


def test_server_budget_and_failures(mp):
    small = I.make_problem(32, seed=201)
    big = I.make_problem(64, seed=202)
    budget = mp.mg_workspace_bytes(mp.params_of(small)) + 1024     # room for one 32^3 at a time
    S = mp.Server(hbm_budget_bytes=budget, max_inflight=8)
    with pytest.raises(mp.MGError) as e:
        S.submit(mp.params_of(big), mp.to_device(big))
    assert e.value.name == "BUDGET"
    bad = I.make_problem(32, seed=203); bad.w[0, 1, 1] = 2.0
    probs = [small, bad, I.make_problem(32, seed=204)]
    ref = [solo(mp, p) for p in probs]
    devs = [mp.to_device(p) for p in probs]
    ts = [S.submit(mp.params_of(p), d) for p, d in zip(probs, devs)]
    res = [S.wait(t) for t in ts]
    c = S.counters()
    S.close()
    assert [r["status_name"] for r in res] == ["OK", "INCOMPATIBLE_RHS", "OK"]
    assert c["peak_inflight"] == 1 and c["resident_bytes"] <= budget
    for i in (0, 2):
        out = {k: getattr(devs[i], k).cpu().numpy() for k in ("phi", "u", "v", "w")}
        assert same(out, ref[i][1])


# ---------------------------------------------------------------- other problem kinds
def solo_boxes(mp, prob, box):
    H = mp.Hierarchy(mp.params_of(prob))
    H.set_boxes(box)
    d = mp.to_device(prob)
    st = H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi)
    torch.cuda.synchronize()
    H.close()
    return st, {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}


def nodal_params(mp, prob, precision="fp64"):
    return mp.make_params(prob.n, prob.dx, prob.periodic, rtol=prob.rtol, precision=precision)


def solo_nodal(mp, prob, precision="fp64"):
    H = mp.NodalHierarchy(nodal_params(mp, prob, precision))
    d = mp.nodal_to_device(prob)
    st = H.project(d.rho, d.beta0_cc, d.S, d.uc, d.vc, d.wc, d.phi)
    torch.cuda.synchronize()
    H.close()
    return st, nodal_out(d)


def nodal_out(d):
    return {"phi": d.phi.cpu().numpy(), "u": d.uc.cpu().numpy(), "v": d.vc.cpu().numpy(), "w": d.wc.cpu().numpy()}


def mac_out(d):
    return {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}


def check_mac_oracle(prob, out):
    ref = O.mac_project(prob, mode="definition")
    alg = O.mac_project(prob)
    assert ref["status"] == 0 and alg["status"] == 0
    for k in ("phi", "u", "v", "w"):
        assert rel(out[k], ref[k]) <= max(1e-9, 3 * rel(alg[k], ref[k])), k


def check_nodal_oracle(prob, out):
    ref = O.nodal_project(prob, mode="definition")
    alg = O.nodal_project(prob)
    assert ref["status"] == 0 and alg["status"] == 0
    for k in ("phi", "u", "v", "w"):
        assert rel(out[k], ref[k]) <= max(1e-9, 3 * rel(alg[k], ref[k])), k


def kinds_mix():
    """Single-box MAC problems (batched), multi-box ones with even and uneven
    boxes, and nodal projections."""
    mac = [I.make_problem(32, H=0.15, seed=301), I.make_problem(64, H=0.1, seed=302)]
    boxed = [(I.make_problem((40, 24, 56), H=0.15, rho_noise=0.05, seed=303, dx=1 / 40), (16, 16, 24)),
             (I.make_problem((96, 64, 64), H=0.15, rho_noise=0.05, seed=304, periodic=(True, True, True),
                             dx=1 / 96), (64, 48, 40)),
             (I.make_problem(32, H=0.2, rho_noise=0.05, seed=305), (16, 16, 16))]
    nodal = [I.make_nodal_problem((32, 32, 32), seed=306, periodic=(True, True, False)),
             I.make_nodal_problem((24, 16, 32), seed=307, periodic=(False, False, False))]
    return mac, boxed, nodal


def test_batch_of_mixed_kinds_matches_solo_and_oracle(mp):
    """One project_batch call holding single-box, multi-box (uneven boxes
    included) and nodal problems: every result equals its own entry point's
    solo result bit for bit, and is within the oracle bar of its kind."""
    mac, boxed, nodal = kinds_mix()
    ref_mac = [solo(mp, p) for p in mac]
    ref_box = [solo_boxes(mp, p, b) for p, b in boxed]
    ref_nod = [solo_nodal(mp, p) for p in nodal]
    d_mac = [mp.to_device(p) for p in mac]
    d_box = [mp.to_device(p) for p, _ in boxed]
    d_nod = [mp.nodal_to_device(p) for p in nodal]
    probs = ([mp.problem_struct(mp.params_of(p), d) for p, d in zip(mac, d_mac)]
             + [mp.problem_struct(mp.params_of(p), d, b) for (p, b), d in zip(boxed, d_box)]
             + [mp.nodal_problem_struct(nodal_params(mp, p), d) for p, d in zip(nodal, d_nod)])
    # interleave the kinds
    order = [0, 2, 5, 1, 3, 6, 4]
    code, stats = mp.project_batch_problems([probs[i] for i in order])
    torch.cuda.synchronize()
    assert code == 0, stats
    st = [None] * len(order)
    for pos, i in enumerate(order):
        st[i] = stats[pos]
    refs = ref_mac + ref_box + ref_nod
    outs = [mac_out(d) for d in d_mac] + [mac_out(d) for d in d_box] + [nodal_out(d) for d in d_nod]
    for i, ((st0, out0), s, out) in enumerate(zip(refs, st, outs)):
        assert s["status_name"] == "OK", (i, s)
        assert s["cycles"] == st0["cycles"] and s["rel_resid"] == st0["rel_resid"], i
        assert same(out, out0), i
    check_mac_oracle(boxed[1][0], outs[3])
    check_mac_oracle(boxed[0][0], outs[2])
    check_nodal_oracle(nodal[0], outs[5])
    check_nodal_oracle(nodal[1], outs[6])


def test_server_of_mixed_kinds_matches_solo_and_oracle(mp):
    """The same mixture served (arrivals while others run): each result equals
    the solo one bit for bit; one uneven-box and one nodal result against the
    oracle; a nodal request with boxes is refused at submission, a mixed-
    precision request with boxes fails at admission."""
    mac, boxed, nodal = kinds_mix()
    ref_mac = [solo(mp, p) for p in mac]
    ref_box = [solo_boxes(mp, p, b) for p, b in boxed]
    ref_nod = [solo_nodal(mp, p) for p in nodal]
    S = mp.Server(hbm_budget_bytes=8 << 30, max_inflight=8)
    d_mac = [mp.to_device(p) for p in mac]
    d_box = [mp.to_device(p) for p, _ in boxed]
    d_nod = [mp.nodal_to_device(p) for p in nodal]
    t = []
    t.append(S.submit(mp.params_of(mac[0]), d_mac[0]))
    t.append(S.submit_nodal(nodal_params(mp, nodal[0]), d_nod[0]))
    t.append(S.submit(mp.params_of(boxed[1][0]), d_box[1], box=boxed[1][1]))
    time.sleep(0.002)
    t.append(S.submit(mp.params_of(mac[1]), d_mac[1]))
    t.append(S.submit(mp.params_of(boxed[0][0]), d_box[0], box=boxed[0][1]))
    t.append(S.submit_nodal(nodal_params(mp, nodal[1]), d_nod[1]))
    t.append(S.submit(mp.params_of(boxed[2][0]), d_box[2], box=boxed[2][1]))
    bad_n = I.make_nodal_problem((16, 16, 16), seed=308, periodic=(True, True, False))
    pr = mp.nodal_problem_struct(nodal_params(mp, bad_n), mp.nodal_to_device(bad_n))
    pr.box[0] = pr.box[1] = pr.box[2] = 8
    with pytest.raises(mp.MGError):
        S.submit_problem(pr, None)
    bad_m = I.make_problem(32, seed=309)
    d_bad = mp.to_device(bad_m)
    t_bad = S.submit(mp.params_of(bad_m, precision="mixed"), d_bad, box=(16, 16, 16))
    res = [S.wait(x) for x in t]
    r_bad = S.wait(t_bad)
    c = S.counters()
    S.close()
    assert r_bad["status_name"] == "INVALID_ARG"
    assert c["completed"] == len(t) + 1
    got = {0: (res[0], mac_out(d_mac[0]), ref_mac[0]), 1: (res[1], nodal_out(d_nod[0]), ref_nod[0]),
           2: (res[2], mac_out(d_box[1]), ref_box[1]), 3: (res[3], mac_out(d_mac[1]), ref_mac[1]),
           4: (res[4], mac_out(d_box[0]), ref_box[0]), 5: (res[5], nodal_out(d_nod[1]), ref_nod[1]),
           6: (res[6], mac_out(d_box[2]), ref_box[2])}
    for i, (r, out, (st0, out0)) in got.items():
        assert r["status_name"] == "OK", (i, r)
        assert r["cycles"] == st0["cycles"], i
        assert same(out, out0), i
    check_mac_oracle(boxed[1][0], got[2][1])
    check_nodal_oracle(nodal[1], got[5][1])


def test_batch_nodal_mixed_precision_matches_solo_and_oracle(mp):
    """Nodal problems in FP64 and in mixed precision in one batch: each equals
    its solo solve bit for bit and meets the oracle bar."""
    probs = [I.make_nodal_problem((32, 32, 32), seed=311, periodic=(True, True, False)),
             I.make_nodal_problem((24, 16, 32), seed=312, periodic=(False, False, False)),
             I.make_nodal_problem((32, 32, 32), seed=313, periodic=(True, False, True))]
    precs = ["mixed", "mixed", "fp64"]
    refs = [solo_nodal(mp, p, pr) for p, pr in zip(probs, precs)]
    devs = [mp.nodal_to_device(p) for p in probs]
    code, stats = mp.project_batch_problems([mp.nodal_problem_struct(nodal_params(mp, p, pr), d)
                                             for p, pr, d in zip(probs, precs, devs)])
    torch.cuda.synchronize()
    assert code == 0, stats
    for p, (st0, out0), s, d in zip(probs, refs, stats, devs):
        out = nodal_out(d)
        assert s["status_name"] == "OK" and s["cycles"] == st0["cycles"]
        assert same(out, out0)
        check_nodal_oracle(p, out)


def test_batch_boxes_mixed_precision_matches_solo_and_oracle(mp):
    """A multi-box problem in mixed precision (fused boxes, uneven) inside a
    batch with a single-box one: each equals its solo solve bit for bit, the
    boxed one meets the oracle bar."""
    pb = I.make_problem((96, 48, 40), H=0.15, rho_noise=0.05, seed=321, periodic=(False, False, False), dx=1 / 96)
    ps = I.make_problem(32, H=0.2, seed=322)
    H = mp.Hierarchy(mp.params_of(pb, precision="mixed"))
    H.set_boxes((64, 32, 16))
    d = mp.to_device(pb)
    st0 = H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi)
    torch.cuda.synchronize()
    H.close()
    out0 = mac_out(d)
    ref_s = solo(mp, ps, "mixed")
    db, ds = mp.to_device(pb), mp.to_device(ps)
    code, stats = mp.project_batch_problems([mp.problem_struct(mp.params_of(pb, precision="mixed"), db, (64, 32, 16)),
                                             mp.problem_struct(mp.params_of(ps, precision="mixed"), ds)])
    torch.cuda.synchronize()
    assert code == 0, stats
    assert stats[0]["cycles"] == st0["cycles"] and same(mac_out(db), out0)
    assert stats[1]["cycles"] == ref_s[0]["cycles"] and same(mac_out(ds), ref_s[1])
    check_mac_oracle(pb, mac_out(db))


def test_batch_with_64x16_tiles_matches_solo(mp):
    """A shape whose finest level is tuned to 64x16-cell tiles (the batched
    sweep's widest form) in FP64 and in mixed precision: batched results equal
    the solo ones bit for bit."""
    n = (128, 64, 64)
    try:
        mp.tune_record(n, 9, rho=True, fp64=True, coarse=False)
        mp.tune_record(n, 11, rho=True, fp64=False, coarse=False)
        probs = [I.make_problem(n, H=0.15, seed=331, dx=1 / 128), I.make_problem(n, H=0.2, seed=332, dx=1 / 128),
                 I.make_problem(64, H=0.1, seed=333)]
        precs = ["fp64", "mixed", "fp64"]
        refs = [solo(mp, p, pr) for p, pr in zip(probs, precs)]
        devs = [mp.to_device(p) for p in probs]
        code, stats = mp.project_batch([mp.params_of(p, precision=pr) for p, pr in zip(probs, precs)], devs)
        torch.cuda.synchronize()
        assert code == 0, stats
        for (st0, out0), s, d in zip(refs, stats, devs):
            assert s["status_name"] == "OK" and s["cycles"] == st0["cycles"] and s["rel_resid"] == st0["rel_resid"]
            assert same(mac_out(d), out0)
        H = mp.Hierarchy(mp.params_of(probs[0]))
        assert H.sweep_config(0)[:2] == (64, 16)
        H.close()
    finally:
        mp.tune_cache_clear()
