"""GPU parity of the multi-box finest level (the domain tiled by boxes with a
halo exchange between them) against the FP64 CPU oracle and against the
single-box GPU solve.

Boxes of 32 x 8 x 4 cells and more run the fused sweep on each box interior
(two-cell ghost shells), smaller ones one launch per colour.  Uneven boxes:
a box size that does not divide the domain leaves a smaller last box in that
direction (its tiles partly empty on the fused path, its neighbours across a
periodic side of another size).

Bar at rtol 1e-10: phi and U within max(1e-9, 3 x the oracle's own
algorithm-mode deviation) of the oracle's exact discrete solution, with the
GPU residual <= rtol (evaluated by the oracle's operator) and the correction
exact (<= 1e-12) given the GPU's phi; solved to rtol 1e-12, phi and U within
1e-9 of the exact solution outright.  Against the single-box GPU solve: the
same cycle count and phi, U within 1e-12 (the per-cell arithmetic is the
same; only the summation order of the residual norm and of the finest-level
restriction can differ, so the two iterates agree to rounding).
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1910_12979_amd import inputs as I

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_gpu(mp, prob, box=None, allow=(0,), H=None, precision="fp64", inner_cycles=0):
    own = H is None
    if own:
        H = mp.Hierarchy(mp.params_of(prob, precision=precision, inner_cycles=inner_cycles))
        if box is not None:
            H.set_boxes(box)
    d = mp.to_device(prob)
    if prob.beta0_r is not None:
        st = H.mac_project_radial(d.rho, d.beta0_r, prob.dr_base, prob.centre, d.S, d.u, d.v, d.w, d.phi,
                                  allow=allow)
    else:
        st = H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi, allow=allow)
    torch.cuda.synchronize()
    out = {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}
    if own:
        H.close()
    return st, out


def check_oracle(prob, st, out, vcycles_per_step=1):
    """The oracle bar; vcycles_per_step: V-cycles behind one of the solve's
    cycles (a mixed-precision refinement step runs inner_cycles of them, 2 by
    default), so that the V-cycle counts compare."""
    ref = O.mac_project(prob, mode="definition")
    alg = O.mac_project(prob)
    assert ref["status"] == 0 and alg["status"] == 0
    assert st["status_name"] == "OK", st
    assert st["rel_resid"] <= prob.rtol
    e_alg_phi = rel(alg["phi"], ref["phi"])
    assert rel(out["phi"], ref["phi"]) <= max(1e-9, 3 * e_alg_phi)
    sides = O.side_codes(prob.periodic, prob.outflow)
    rad = O.prob_radial(prob)
    coeffs = O.face_coeffs_gen(prob.n, sides, prob.dx, prob.rho, prob.beta0_cc, prob.beta0_edge, rad)
    f = O.rhs_gen(prob.n, sides, prob.dx, prob.u, prob.v, prob.w, prob.S, prob.beta0_cc, prob.beta0_edge, rad)
    f -= f.mean()
    u_c = O.correct_gen(prob.n, sides, prob.dx, prob.rho, out["phi"], prob.u, prob.v, prob.w) \
        if rad is not None else \
        O.correct(prob.n, prob.periodic, prob.dx, prob.beta0_cc, prob.beta0_edge,
                  O.face_coeffs(prob.n, prob.periodic, prob.rho, prob.beta0_cc, prob.beta0_edge),
                  out["phi"], prob.u, prob.v, prob.w)
    for name, exact in zip(("u", "v", "w"), u_c):
        assert rel(out[name], exact) <= 1e-12, name
        assert rel(out[name], ref[name]) <= max(1e-9, 3 * rel(alg[name], ref[name])), name
    r = f - O.apply_gen(prob.n, sides, prob.dx, coeffs, out["phi"])
    assert np.linalg.norm(r) <= 1.05 * prob.rtol * np.linalg.norm(f)
    k = vcycles_per_step
    assert abs(st["cycles"] * k - alg["cycles"]) <= max(1, k), (st["cycles"], k, alg["cycles"])


def check_single(mp, prob, st, out):
    st1, out1 = run_gpu(mp, prob)
    assert st1["status_name"] == "OK"
    assert st["cycles"] == st1["cycles"]
    assert abs(st["rel_resid"] - st1["rel_resid"]) <= 1e-6 * st1["rel_resid"]
    for k in ("phi", "u", "v", "w"):
        assert rel(out[k], out1[k]) <= 1e-12, k


CASES = [
    ((32, 32, 32), (True, True, False), (16, 16, 16), 1),     # 8 boxes, walls in z
    ((40, 24, 56), (True, True, False), (20, 12, 28), 2),     # ragged boxes, 8 of them
    ((32, 32, 32), (False, False, False), (8, 16, 32), 3),    # walls everywhere, boxes span z
    ((32, 16, 32), (True, True, True), (16, 16, 16), 4),      # fully periodic, one box in y
    ((32, 32, 32), (True, False, True), (32, 32, 32), 5),     # one box: it exchanges with itself
    ((16, 16, 16), (True, True, False), (2, 4, 8), 6),        # 256 tiny boxes
    ((6, 10, 14), (True, True, False), (2, 10, 14), 7),       # two levels, 105-cell coarsest
    ((64, 64, 64), (False, True, False), (32, 16, 64), 8),     # fused sweeps inside the boxes
    ((64, 32, 32), (True, True, True), (32, 16, 16), 9),       # fused, fully periodic
    ((96, 48, 40), (False, False, False), (32, 8, 4), 10),     # fused, walls, the smallest fused box
    ((128, 64, 32), (True, False, False), (64, 32, 16), 11),   # fused with 64-wide tiles
    # uneven boxes: the last box of a direction holds the remainder
    ((40, 24, 56), (True, True, False), (16, 16, 24), 12),     # 16+16+8, 16+8, 24+24+8: per colour
    ((96, 48, 40), (False, False, False), (64, 32, 16), 13),   # fused: 64+32, 32+16, 16+16+8
    ((96, 64, 64), (True, True, True), (64, 48, 40), 14),      # fused, periodic across unequal boxes
    ((32, 32, 32), (True, False, True), (30, 32, 18), 15),     # 30+2 and 18+14: two-cell boxes
]


@pytest.mark.parametrize("n,per,box,seed", CASES)
def test_boxes_match_oracle_and_single_box(mp, n, per, box, seed):
    prob = I.make_problem(n, H=0.15, rho_noise=0.05, seed=seed, periodic=per, dx=1.0 / n[0])
    st, out = run_gpu(mp, prob, box=box)
    check_oracle(prob, st, out)
    check_single(mp, prob, st, out)


@pytest.mark.parametrize("n,per,box,seed", [
    ((32, 32, 32), (True, True, False), (16, 16, 16), 51),
    ((64, 64, 64), (False, True, False), (32, 16, 64), 52),    # fused sweeps inside the boxes
    ((40, 24, 56), (True, True, False), (20, 12, 28), 53),     # ragged boxes
    ((96, 64, 64), (True, True, True), (64, 48, 40), 54),      # uneven, fused
    ((40, 24, 56), (False, True, False), (16, 16, 24), 55),    # uneven, per colour
])
def test_boxes_strict_at_rtol_1e12(mp, n, per, box, seed):
    """Solved to rtol 1e-12, the multi-box phi and U are within 1e-9 of the
    oracle's exact discrete solution outright."""
    prob = I.make_problem(n, H=0.15, rho_noise=0.05, seed=seed, periodic=per, dx=1.0 / n[0], rtol=1e-12)
    st, out = run_gpu(mp, prob, box=box)
    assert st["status_name"] == "OK" and st["rel_resid"] <= 1e-12
    ref = O.mac_project(prob, mode="definition")
    assert ref["status"] == 0
    for k in ("phi", "u", "v", "w"):
        assert rel(out[k], ref[k]) <= 1e-9, (k, rel(out[k], ref[k]))


def _radial_walls(n, seed):
    """A radial base state inside solid walls, S shifted so that the
    right-hand side is compatible (sum of beta0 S over the cells = 0)."""
    prob = I.make_star_problem(n, Hr=0.2, rho_noise=0.02, seed=seed, outflow=(False,) * 6)
    b0 = O.map_radial(prob.n, prob.dx, prob.beta0_r, prob.dr_base, prob.centre)
    prob.S = np.ascontiguousarray(prob.S - np.sum(b0 * prob.S) / np.sum(b0))
    return prob


@pytest.mark.parametrize("n,box", [((32, 32, 48), (16, 16, 16)), ((64, 32, 48), (32, 16, 24))])
def test_boxes_radial_base_state(mp, n, box):
    prob = _radial_walls(n, 11)
    st, out = run_gpu(mp, prob, box=box)
    check_oracle(prob, st, out)
    check_single(mp, prob, st, out)


def test_boxes_set_and_reset(mp):
    """Switching boxes on, changing their size and switching them off on one
    hierarchy: each solve equals a fresh hierarchy's."""
    prob = I.make_problem((32, 32, 32), H=0.2, rho_noise=0.05, seed=21)
    H = mp.Hierarchy(mp.params_of(prob))
    try:
        st0, out0 = run_gpu(mp, prob, H=H)
        for box in ((16, 16, 16), (8, 32, 16)):
            H.set_boxes(box)
            st, out = run_gpu(mp, prob, H=H)
            stf, outf = run_gpu(mp, prob, box=box)
            assert st["cycles"] == stf["cycles"]
            for k in out:
                assert np.array_equal(out[k], outf[k]), k
                assert rel(out[k], out0[k]) <= 1e-12, k
        H.set_boxes(None)
        st, out = run_gpu(mp, prob, H=H)
        assert st["cycles"] == st0["cycles"]
        for k in out:
            assert np.array_equal(out[k], out0[k]), k
    finally:
        H.close()


def test_boxes_errors(mp):
    prob = I.make_problem((32, 32, 32), H=0.2, seed=22)
    H = mp.Hierarchy(mp.params_of(prob))
    try:
        for bad in ((3, 16, 16), (34, 16, 16), (0, 16, 16), (64, 16, 16), (16, -2, 16), (16, 16, 15)):
            with pytest.raises(mp.MGError):
                H.set_boxes(bad)
    finally:
        H.close()
    H = mp.Hierarchy(mp.params_of(prob, precision="mixed"))
    try:
        with pytest.raises(mp.MGError):
            H.set_boxes((16, 16, 16))
    finally:
        H.close()
    out = I.make_problem((32, 32, 32), H=0.2, seed=22, outflow=(False,) * 5 + (True,))
    H = mp.Hierarchy(mp.params_of(out))
    try:
        with pytest.raises(mp.MGError):
            H.set_boxes((16, 16, 16))
    finally:
        H.close()
    # an incompatible right-hand side is still caught before the box solve
    q = prob.copy()
    q.S = q.S + 0.5
    st, _ = run_gpu(mp, q, box=(16, 16, 16), allow=(-3,))
    assert st["status_name"] == "INCOMPATIBLE_RHS"


@pytest.mark.parametrize("box", [(64, 64, 64), (96, 96, 96)])
def test_boxes_256_full_size(mp, box):
    """The 256^3 steep-stratification box split into 64 boxes of 64^3, or
    into 27 uneven ones (96 + 96 + 64 per direction): the single-box solve's
    cycles and result, and the discrete system satisfied to rtol (the
    oracle's operator in FP64)."""
    prob = I.STEEP_256()
    st, out = run_gpu(mp, prob, box=box)
    assert st["status_name"] == "OK" and st["rel_resid"] <= 1e-10
    check_single(mp, prob, st, out)
    c = O.face_coeffs(prob.n, prob.periodic, prob.rho, prob.beta0_cc, prob.beta0_edge)
    f = O.rhs(prob.n, prob.periodic, prob.dx, prob.beta0_cc, prob.beta0_edge, prob.u, prob.v, prob.w, prob.S)
    f -= f.mean()
    r = O.residual(prob.n, prob.periodic, prob.dx, c, out["phi"], f)
    assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(f)


@pytest.mark.parametrize("pre,post", [(1, 1), (3, 1), (0, 2)])
def test_boxes_other_sweep_counts(mp, pre, post):
    """Odd and zero sweep counts: the box smoother's colour exchanges keep
    every ghost current for the residual that follows."""
    prob = I.make_problem((32, 48, 32), H=0.2, rho_noise=0.05, seed=30 + pre, periodic=(True, False, False),
                          dx=1.0 / 32)
    prob.pre_sweeps, prob.post_sweeps = pre, post
    st, out = run_gpu(mp, prob, box=(16, 16, 8))
    assert st["status_name"] == "OK"
    check_single(mp, prob, st, out)


def test_boxes_cycle_cap(mp):
    """max_cycles reached: the same not-converged iterate as the single box."""
    prob = I.make_problem((32, 32, 32), H=0.15, rho_noise=0.05, seed=33)
    prob.max_cycles = 2
    st, out = run_gpu(mp, prob, box=(8, 8, 8), allow=(0, -4))
    st1, out1 = run_gpu(mp, prob, allow=(0, -4))
    assert st["status_name"] == "NOT_CONVERGED" and st1["status_name"] == "NOT_CONVERGED"
    assert st["cycles"] == st1["cycles"] == 2
    for k in out:
        assert rel(out[k], out1[k]) <= 1e-12, k



MIXED_CASES = [
    ((64, 64, 64), (False, True, False), (32, 16, 64), 61),    # fused, 32x8 tiles
    ((128, 64, 32), (True, False, False), (64, 32, 16), 62),   # fused, 64-wide tiles
    ((96, 48, 40), (False, False, False), (64, 32, 16), 63),   # uneven: 64+32, 32+16, 16+16+8
    ((96, 64, 64), (True, True, True), (64, 48, 40), 64),      # uneven, periodic across unequal boxes
]


@pytest.mark.parametrize("n,per,box,seed", MIXED_CASES)
def test_boxes_mixed_precision_matches_oracle(mp, n, per, box, seed):
    """Mixed precision on boxes (FP32 box sweeps and FP64 refinement over the
    boxes): the oracle bar of the single-box solve, and within 1e-9 of the
    single-box mixed solve."""
    prob = I.make_problem(n, H=0.15, rho_noise=0.05, seed=seed, periodic=per, dx=1.0 / n[0])
    st, out = run_gpu(mp, prob, box=box, precision="mixed")
    check_oracle(prob, st, out, vcycles_per_step=2)
    H1 = mp.Hierarchy(mp.params_of(prob, precision="mixed"))
    st1, out1 = run_gpu(mp, prob, H=H1)
    H1.close()
    assert abs(st["cycles"] - st1["cycles"]) <= 1
    for k in ("phi", "u", "v", "w"):
        assert rel(out[k], out1[k]) <= 1e-9, k


def test_boxes_mixed_precision_strict_and_radial(mp):
    """Solved to rtol 1e-12 in mixed precision on uneven boxes: within 1e-9 of
    the exact solution outright; and a radial base state inside walls (the
    FP32 stored-coefficient box sweep) at the oracle bar."""
    prob = I.make_problem((96, 64, 64), H=0.15, rho_noise=0.05, seed=65, periodic=(True, True, True), dx=1 / 96,
                          rtol=1e-12)
    st, out = run_gpu(mp, prob, box=(64, 48, 40), precision="mixed")
    assert st["status_name"] == "OK" and st["rel_resid"] <= 1e-12
    ref = O.mac_project(prob, mode="definition")
    assert ref["status"] == 0
    for k in ("phi", "u", "v", "w"):
        assert rel(out[k], ref[k]) <= 1e-9, (k, rel(out[k], ref[k]))
    rad = _radial_walls((64, 32, 48), 66)
    st, out = run_gpu(mp, rad, box=(32, 16, 24), precision="mixed")
    check_oracle(rad, st, out, vcycles_per_step=2)


def test_boxes_mixed_inner_cycles(mp):
    """Mixed precision on boxes with one FP32 V-cycle per refinement step
    and with three (the default is two): each at the oracle bar, and more
    V-cycles per step need no more refinement steps."""
    prob = I.make_problem((64, 48, 48), H=0.2, rho_noise=0.05, seed=67, dx=1 / 64)
    res = {}
    for k in (1, 3):
        st, out = run_gpu(mp, prob, box=(32, 24, 24), precision="mixed", inner_cycles=k)
        check_oracle(prob, st, out, vcycles_per_step=k)
        res[k] = st["cycles"]
    assert res[3] <= res[1]


def test_boxes_mixed_256_full_size(mp):
    """The 256^3 steep box in 64 boxes of 64^3, mixed precision: converged in
    FP64 terms by the oracle's operator, and within 1e-9 of the single-box
    mixed solve."""
    prob = I.STEEP_256()
    st, out = run_gpu(mp, prob, box=(64, 64, 64), precision="mixed")
    assert st["status_name"] == "OK" and st["rel_resid"] <= 1e-10
    H1 = mp.Hierarchy(mp.params_of(prob, precision="mixed"))
    st1, out1 = run_gpu(mp, prob, H=H1)
    H1.close()
    assert rel(out["phi"], out1["phi"]) <= 1e-9
    c = O.face_coeffs(prob.n, prob.periodic, prob.rho, prob.beta0_cc, prob.beta0_edge)
    f = O.rhs(prob.n, prob.periodic, prob.dx, prob.beta0_cc, prob.beta0_edge, prob.u, prob.v, prob.w, prob.S)
    f -= f.mean()
    r = O.residual(prob.n, prob.periodic, prob.dx, c, out["phi"], f)
    assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(f)
