"""GPU parity of the HIP MAC projection against the FP64 CPU oracle.

Every test calls the library through the C ABI (ctypes binding) on seeded
inputs from paper_1910_12979_amd.inputs and compares with the oracle on the
same host arrays.  Tolerances:
  * phi: relative L2 <= 1e-9 against the oracle's definition-mode (exact
    discrete) solution, with the GPU relative residual <= 1e-10;
  * U: the correction step exact (<= 1e-12) given the GPU's phi, and U within
    max(1e-9, 3x the oracle's own algorithm-mode deviation) of the exact
    projection;
  * single steps (coefficients, one sweep, residual/restriction,
    prolongation, coarse solve, one V-cycle): relative <= 1e-13 against the
    oracle's same step on the same input (both sides evaluate the same
    per-cell expression order without FMA contraction).
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


def run_gpu(mp, prob, precision="fp64", rtol=None, max_cycles=None, allow=(0,), inner_cycles=0):
    params = mp.params_of(prob, precision=precision, rtol=rtol, max_cycles=max_cycles, inner_cycles=inner_cycles)
    H = mp.Hierarchy(params)
    d = mp.to_device(prob)
    st = H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi, allow=allow)
    torch.cuda.synchronize()
    out = {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}
    H.close()
    return st, out


def check_against_definition(prob, st, out, tol_phi=1e-9):
    """phi within tol_phi of the exact discrete solution; U checked twice:
    (a) the correction step is exact given the GPU's phi (oracle correction of
    that phi, <= 1e-12), and (b) U is within max(1e-9, 3 e_alg) of the exact
    projection, e_alg being the oracle's own deviation when it runs the same
    cycle with the same 1e-10 stopping rule (U inherits phi's smooth residual
    error through grad phi, so its relative error can exceed phi's)."""
    ref = O.mac_project(prob, mode="definition")
    alg = O.mac_project(prob)
    assert ref["status"] == 0 and alg["status"] == 0
    assert st["status_name"] == "OK", st
    assert st["rel_resid"] <= prob.rtol
    assert abs(np.mean(out["phi"])) <= 1e-12 * np.max(np.abs(out["phi"])) + 1e-300
    e_phi = rel(out["phi"], ref["phi"])
    assert e_phi <= tol_phi, e_phi
    c = O.face_coeffs(prob.n, prob.periodic, prob.rho, prob.beta0_cc, prob.beta0_edge)
    u_c = O.correct(prob.n, prob.periodic, prob.dx, prob.beta0_cc, prob.beta0_edge, c, out["phi"],
                    prob.u, prob.v, prob.w)
    for name, exact in zip(("u", "v", "w"), u_c):
        assert rel(out[name], exact) <= 1e-12, (name, rel(out[name], exact))
        e_alg = rel(alg[name], ref[name])
        e = rel(out[name], ref[name])
        assert e <= max(1e-9, 3 * e_alg), (name, e, e_alg)
    # the GPU's own residual, recomputed by the oracle in FP64
    f = O.rhs(prob.n, prob.periodic, prob.dx, prob.beta0_cc, prob.beta0_edge, prob.u, prob.v, prob.w, prob.S)
    f -= f.mean()
    r = O.residual(prob.n, prob.periodic, prob.dx, c, out["phi"], f)
    assert np.linalg.norm(r) <= 1.05 * prob.rtol * np.linalg.norm(f)
    return e_phi, ref


# ------------------------------------------------------------ end to end
def test_small_box_fp64(mp):
    prob = I.SMALL_BOX(0)
    st, out = run_gpu(mp, prob)
    check_against_definition(prob, st, out)
    alg = O.mac_project(prob)
    assert abs(st["cycles"] - alg["cycles"]) <= 1
    n = min(len(st["hist"]), len(alg["hist"])) - 1
    np.testing.assert_allclose(st["hist"][:n], alg["hist"][:n], rtol=1e-6)


@pytest.mark.parametrize("shape,per,seed", [
    ((40, 24, 56), (True, True, False), 5),      # non-cubic, ragged against every tile width
    ((48, 48, 48), (True, True, False), 6),      # coarsest level 3^3
    ((32, 32, 32), (False, False, False), 7),    # solid walls everywhere
    ((32, 16, 32), (True, True, True), 8),       # fully periodic
    ((64, 64, 32), (False, True, False), 9),
    ((6, 10, 14), (True, True, False), 10),      # two levels, 105-cell coarsest
])
def test_shapes_and_boundaries(mp, shape, per, seed):
    prob = I.make_problem(shape, H=0.15, rho_noise=0.05, seed=seed, periodic=per, dx=1.0 / shape[0])
    st, out = run_gpu(mp, prob)
    check_against_definition(prob, st, out)


@pytest.mark.parametrize("n", [4, 2])
def test_direct_solve_only(mp, n):
    """Boxes small enough to be solved by the coarsest-level direct solve alone."""
    prob = I.make_problem(n, H=0.3, seed=3)
    st, out = run_gpu(mp, prob)
    check_against_definition(prob, st, out)
    assert st["cycles"] == 1


def test_zero_right_hand_side(mp):
    prob = I.make_problem(16, S_kind="zero", vel_scale=0.0, seed=1)
    st, out = run_gpu(mp, prob)
    assert st["status_name"] == "OK" and st["cycles"] == 0
    assert np.all(out["phi"] == 0.0) and np.all(out["u"] == 0.0)


def test_error_paths(mp):
    prob = I.make_problem(16, seed=2)
    q = prob.copy(); q.w[0, 1, 1] = 0.5                # flux through a wall
    st, _ = run_gpu(mp, q, allow=(-3,))
    assert st["status_name"] == "INCOMPATIBLE_RHS"
    q = prob.copy(); q.S[2, 2, 2] = np.inf
    st, _ = run_gpu(mp, q, allow=(-5,))
    assert st["status_name"] == "NONFINITE"
    q = prob.copy(); q.rho[3, 3, 3] = 0.0
    st, _ = run_gpu(mp, q, allow=(-1,))
    assert st["status_name"] == "INVALID_ARG"
    st, out = run_gpu(mp, prob, max_cycles=1, allow=(-4,))
    assert st["status_name"] == "NOT_CONVERGED" and st["cycles"] == 1
    ref = O.mac_project(prob, max_cycles=1)
    assert ref["status_name"] == "NOT_CONVERGED"
    assert rel(out["phi"], ref["phi"]) < 1e-12
    with pytest.raises(mp.MGError) as e:
        mp.Hierarchy(mp.make_params((37, 37, 37), 1 / 37))
    assert e.value.name == "BAD_SIZE"


# ------------------------------------------------------------ single steps
def _step_setup(mp, prob):
    params = mp.params_of(prob)
    H = mp.Hierarchy(params)
    d = mp.to_device(prob)
    H.set_coefficients(d.rho, d.beta0_cc, d.beta0_edge)
    c = O.face_coeffs(prob.n, prob.periodic, prob.rho, prob.beta0_cc, prob.beta0_edge)
    OH = O.Hierarchy(prob.n, prob.periodic, prob.dx, c)
    return H, OH


def _get(H, l, name):
    (nx, ny, nz), _ = H.level_info(l)
    t = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    H.level_copy(l, name, t, to_hierarchy=False)
    return t.cpu().numpy()


def _put(H, l, name, a):
    H.level_copy(l, name, torch.from_numpy(np.ascontiguousarray(a)).cuda(), to_hierarchy=True)


@pytest.mark.parametrize("shape,per", [
    ((32, 16, 24), (True, True, False)),
    ((24, 32, 16), (False, True, True)),
])
def test_rho_recomputed_coefficients_equal_stored(mp, shape, per):
    """The first coarse averaging recomputes the level-0 face coefficients
    from rho: it must use exactly the values the coefficient kernel stores.
    Level 1 equals the stored level 0 averaged over the 2 x 2 fine faces of
    each coarse face (in the kernel's order), and the corrected U equals
    U - (b / beta0) grad(phi) formed from the stored coefficients and the
    returned phi, bit for bit."""
    prob = I.make_problem(shape, H=0.1, rho_noise=0.2, seed=21, periodic=per)
    H = mp.Hierarchy(mp.params_of(prob))
    d = mp.to_device(prob)
    st = H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi)
    torch.cuda.synchronize()
    assert st["status_name"] == "OK"
    bx, by, bz = (_get(H, 0, n) for n in ("bx", "by", "bz"))
    cbx, cby, cbz = (_get(H, 1, n) for n in ("bx", "by", "bz"))
    H.close()
    q = 0.25
    assert np.array_equal(cbx, q * (bx[0::2, 0::2, 0::2] + bx[0::2, 1::2, 0::2] + bx[1::2, 0::2, 0::2]
                                    + bx[1::2, 1::2, 0::2]))
    assert np.array_equal(cby, q * (by[0::2, 0::2, 0::2] + by[0::2, 0::2, 1::2] + by[1::2, 0::2, 0::2]
                                    + by[1::2, 0::2, 1::2]))
    assert np.array_equal(cbz, q * (bz[0::2, 0::2, 0::2] + bz[0::2, 0::2, 1::2] + bz[0::2, 1::2, 0::2]
                                    + bz[0::2, 1::2, 1::2]))
    P = d.phi.cpu().numpy()                       # phi minus its mean, as the correction uses it
    h = prob.dx
    nx, ny, nz = prob.n
    b0c = prob.beta0_cc[:, None, None]
    b0e = prob.beta0_edge[:nz, None, None]
    u, v, w = prob.u.copy(), prob.v.copy(), prob.w.copy()
    lo = 0 if per[0] else 1
    g = (P - np.roll(P, 1, axis=2)) / h
    u[:, :, lo:nx] = u[:, :, lo:nx] - (bx / b0c)[:, :, lo:] * g[:, :, lo:]
    if per[0]:
        u[:, :, nx] = u[:, :, 0]
    lo = 0 if per[1] else 1
    g = (P - np.roll(P, 1, axis=1)) / h
    v[:, lo:ny, :] = v[:, lo:ny, :] - (by / b0c)[:, lo:, :] * g[:, lo:, :]
    if per[1]:
        v[:, ny, :] = v[:, 0, :]
    lo = 0 if per[2] else 1
    g = (P - np.roll(P, 1, axis=0)) / h
    w[lo:nz] = w[lo:nz] - (bz / b0e)[lo:] * g[lo:]
    if per[2]:
        w[nz] = w[0]
    assert np.array_equal(d.u.cpu().numpy(), u)
    assert np.array_equal(d.v.cpu().numpy(), v)
    assert np.array_equal(d.w.cpu().numpy(), w)


def test_step_coefficients_all_levels(mp):
    prob = I.make_problem((32, 16, 24), H=0.1, rho_noise=0.2, seed=4, dx=1 / 32)
    H, OH = _step_setup(mp, prob)
    assert H.nlevels == OH.nlevels
    for l in range(H.nlevels):
        gx, gy, gz = _get(H, l, "bx"), _get(H, l, "by"), _get(H, l, "bz")
        # the GPU stores the low face of each cell; face n of a direction is face 0
        assert rel(gx, OH.get(l, "bx")[:, :, :-1]) <= 1e-15
        assert rel(gy, OH.get(l, "by")[:, :-1, :]) <= 1e-15
        assert rel(gz, OH.get(l, "bz")[:-1]) <= 1e-15


@pytest.mark.parametrize("shape,per", [
    ((32, 16, 24), (True, True, False)),
    ((32, 16, 24), (False, False, False)),
    ((32, 16, 24), (True, True, True)),
    ((64, 32, 48), (True, True, False)),     # fused sweeps on levels 0 (rho) and 1 (stored)
    ((72, 40, 48), (False, True, False)),    # ragged fused tiles in x, y and z
])
def test_step_smooth_restrict_prolong_coarse(mp, shape, per):
    prob = I.make_problem(shape, H=0.2, rho_noise=0.1, seed=12, periodic=per, dx=1 / shape[0])
    H, OH = _step_setup(mp, prob)
    rng = np.random.default_rng(7)
    nx0, ny0, nz0 = shape
    for l in (0, 1):
        (nx, ny, nz), _ = H.level_info(l)
        phi_l = rng.standard_normal((nz, ny, nx))
        f_l = rng.standard_normal((nz, ny, nx))
        _put(H, l, "phi", phi_l); _put(H, l, "f", f_l)
        OH.set(l, "phi", phi_l); OH.set(l, "f", f_l)
        H.level_step(l, "smooth", 2)
        OH.smooth(l, 2)
        g, o = _get(H, l, "phi"), OH.get(l, "phi")
        assert rel(g, o) <= 1e-13, (l, rel(g, o), np.max(np.abs(g - o)))
        H.level_step(l, "resid_restrict")
        OH.resid_restrict(l)
        assert rel(_get(H, l + 1, "f"), OH.get(l + 1, "f")) <= 1e-13
        assert np.all(_get(H, l + 1, "phi") == 0.0)
        e = rng.standard_normal(OH.get(l + 1, "phi").shape)
        _put(H, l + 1, "phi", e); OH.set(l + 1, "phi", e)
        H.level_step(l, "prolong")
        OH.prolong(l)
        assert rel(_get(H, l, "phi"), OH.get(l, "phi")) <= 1e-14
        H.level_step(l, "up", 1)
        OH.prolong(l); OH.smooth(l, 1)
        assert rel(_get(H, l, "phi"), OH.get(l, "phi")) <= 1e-13
    Lc = H.nlevels - 1
    (nx, ny, nz), _ = H.level_info(Lc)
    fc = rng.standard_normal((nz, ny, nx))
    _put(H, Lc, "f", fc); OH.set(Lc, "f", fc)
    H.level_step(Lc, "coarse")
    OH.coarse()
    assert rel(_get(H, Lc, "phi"), OH.get(Lc, "phi")) <= 1e-13


def test_step_fused_down_up_match_separate(mp):
    prob = I.make_problem((64, 32, 48), H=0.2, rho_noise=0.1, seed=13, dx=1 / 64)
    H, OH = _step_setup(mp, prob)
    rng = np.random.default_rng(8)
    phi0 = rng.standard_normal((48, 32, 64))
    f0 = rng.standard_normal((48, 32, 64))
    f0 -= f0.mean()
    _put(H, 0, "phi", phi0); _put(H, 0, "f", f0)
    OH.set(0, "phi", phi0); OH.set(0, "f", f0)
    H.level_step(0, "down", 2)
    OH.smooth(0, 2); OH.resid_restrict(0)
    assert rel(_get(H, 0, "phi"), OH.get(0, "phi")) <= 1e-13
    assert rel(_get(H, 1, "f"), OH.get(1, "f")) <= 1e-13
    e = rng.standard_normal((24, 16, 32))
    _put(H, 1, "phi", e); OH.set(1, "phi", e)
    H.level_step(0, "up", 2)
    OH.prolong(0); OH.smooth(0, 2)
    assert rel(_get(H, 0, "phi"), OH.get(0, "phi")) <= 1e-13


def test_every_tile_config_gives_the_same_sweep(mp):
    """Each fused-sweep tile configuration (forced through mg_tune_sweep) must
    give the default configuration's sweeps and residual+restriction bit for
    bit (the update of a cell does not depend on the tiling), on a shape with
    ragged tiles in x, y and z, on the rho level and a stored-coefficient one;
    the default result itself is checked against the oracle."""
    prob = I.make_problem((96, 40, 48), H=0.2, rho_noise=0.1, seed=15, dx=1 / 96)
    H, OH = _step_setup(mp, prob)
    rng = np.random.default_rng(10)
    phi0 = rng.standard_normal((48, 40, 96))
    f0 = rng.standard_normal((48, 40, 96))
    f0 -= f0.mean()
    e1 = rng.standard_normal((24, 20, 48))

    def run():
        _put(H, 0, "phi", phi0); _put(H, 0, "f", f0)
        H.level_step(0, "down", 2)
        out = [_get(H, 0, "phi"), _get(H, 1, "f")]
        _put(H, 1, "phi", e1)
        H.level_step(1, "smooth", 3)
        out.append(_get(H, 1, "phi"))
        return out

    base = run()
    OH.set(0, "phi", phi0); OH.set(0, "f", f0)
    OH.smooth(0, 2); OH.resid_restrict(0)
    assert rel(base[0], OH.get(0, "phi")) <= 1e-13
    assert rel(base[1], OH.get(1, "f")) <= 1e-13
    try:
        for cfg in range(14):
            mp.mg_tune_sweep(cfg)
            got = run()
            for a, b in zip(got, base):
                assert np.array_equal(a, b), cfg
    finally:
        mp.mg_tune_sweep(-1)


def test_graph_replays_match_eager(mp):
    """Solves whose later cycles replay a captured hipGraph give the eager
    solve's results bit for bit: over several solves in a row (replays across
    solves, with eager work in between), for a second problem (new buffers:
    a new capture), with V(2,1) (odd sweep count: no capture) and with a
    forced tile configuration (a new capture)."""
    probs = [I.make_problem((64, 48, 32), H=0.15, seed=41),
             I.make_problem((64, 48, 32), H=0.3, seed=42, rtol=1e-9)]
    He = mp.Hierarchy(mp.params_of(probs[0]))
    He.set_graphs(False)
    Hg = mp.Hierarchy(mp.params_of(probs[0]))

    def solve(H, prob):
        d = mp.to_device(prob)
        st = H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi)
        torch.cuda.synchronize()
        return st, {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}

    def check(prob):
        st0, out0 = solve(He, prob)
        for _ in range(3):
            st1, out1 = solve(Hg, prob)
            assert st1["cycles"] == st0["cycles"] and st1["rel_resid"] == st0["rel_resid"]
            assert st1["hist"] == st0["hist"]
            assert same_out(out1, out0)
        return st0

    try:
        st = check(probs[0])
        assert st["cycles"] >= 4 and st["status_name"] == "OK"
        check(probs[1])
        for H in (He, Hg):
            H.set_params(mp.make_params((64, 48, 32), 1 / 64, post_sweeps=1))
        check(probs[0])
        for H in (He, Hg):
            H.set_params(mp.params_of(probs[0]))
        mp.mg_tune_sweep(0)
        check(probs[0])
    finally:
        mp.mg_tune_sweep(-1)
        He.close()
        Hg.close()


def test_graph_replays_match_eager_mixed(mp):
    """Mixed precision: iterations replayed from the two captured graphs (the
    finest FP64 phi alternates buffers) equal the eager solve bit for bit,
    over several solves in a row."""
    prob = I.make_problem((64, 64, 32), H=0.12, rho_noise=0.05, seed=44)
    He = mp.Hierarchy(mp.params_of(prob, precision="mixed"))
    He.set_graphs(False)
    Hg = mp.Hierarchy(mp.params_of(prob, precision="mixed"))

    def solve(H):
        d = mp.to_device(prob)
        st = H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi)
        torch.cuda.synchronize()
        return st, {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}

    try:
        st0, out0 = solve(He)
        assert st0["status_name"] == "OK" and st0["cycles"] >= 4
        for _ in range(3):
            st1, out1 = solve(Hg)
            assert st1["cycles"] == st0["cycles"] and st1["hist"] == st0["hist"]
            assert same_out(out1, out0)
    finally:
        He.close()
        Hg.close()


@pytest.mark.parametrize("shape,per,prec", [
    ((32, 32, 32), (True, True, False), "fp64"),
    ((64, 32, 48), (False, False, False), "fp64"),
    ((64, 64, 64), (True, True, True), "mixed"),
    ((128, 64, 32), (True, True, False), "mixed"),
    ((64, 32, 32), (True, False, True), "mixed"),
    ((48, 48, 48), (True, True, False), "fp64"),
    ((96, 48, 48), (False, True, False), "fp64"),
])
def test_bottom_solver_matches_per_level_launches(mp, shape, per, prec):
    """The one-workgroup bottom of the V-cycle gives the per-level launches'
    solve bit for bit (same cycles, residual history, phi and U).  The
    (64, 32, 32) mixed case has a 32 x 16 x 16 first bottom level in FP32
    (4096 cells per colour); in the two FP64 cases with 48-cell sides the
    first level the fused sweep cannot take (24-cell sides) does not fit in
    the bottom's LDS, which then starts one level lower."""
    prob = I.make_problem(shape, H=0.2, rho_noise=0.05, seed=43, periodic=per)
    res = []
    for on in (False, True):
        H = mp.Hierarchy(mp.params_of(prob, precision=prec))
        H.set_bottom(on)
        d = mp.to_device(prob)
        st = H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi)
        torch.cuda.synchronize()
        res.append((st, {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}))
        H.close()
    (s0, o0), (s1, o1) = res
    assert s0["status_name"] == "OK" and s1["cycles"] == s0["cycles"] and s1["hist"] == s0["hist"]
    assert same_out(o1, o0)


def same_out(a, b):
    return all(np.array_equal(a[k], b[k]) for k in ("phi", "u", "v", "w"))


def test_step_vcycle(mp):
    prob = I.make_problem(32, H=0.1, seed=14)
    H, OH = _step_setup(mp, prob)
    rng = np.random.default_rng(9)
    f = rng.standard_normal((32, 32, 32))
    f -= f.mean()
    phi = torch.zeros((32, 32, 32), dtype=torch.float64, device="cuda")
    ft = torch.from_numpy(f).cuda()
    OH.set(0, "phi", np.zeros_like(f)); OH.set(0, "f", f)
    for cyc in range(3):
        rel_gpu = H.mg_vcycle(phi, ft)
        OH.vcycle(0)
        assert rel(phi.cpu().numpy(), OH.get(0, "phi")) <= 1e-12
    r = O.residual(prob.n, prob.periodic, prob.dx,
                   O.face_coeffs(prob.n, prob.periodic, prob.rho, prob.beta0_cc, prob.beta0_edge),
                   OH.get(0, "phi"), f)
    assert abs(rel_gpu - np.linalg.norm(r) / np.linalg.norm(f)) <= 1e-6 * rel_gpu


# ------------------------------------------------------------ full sizes
def test_steep_256_fp64_full_size(mp):
    """The 256^3 steep-stratification box at full size, as the benchmark runs
    it (rtol 1e-10): phi within 1e-9 of the oracle's exact discrete solution
    (definition mode) and U within 1e-9 of the exact projection; the GPU
    iterate equal to the oracle's same-cycle iterate to 1e-11; the correction
    exact given the GPU's phi; the post-projection constraint met to the
    final residual."""
    prob = I.STEEP_256()
    st, out = run_gpu(mp, prob)
    assert st["status_name"] == "OK" and st["rel_resid"] <= 1e-10
    ref = O.mac_project(prob, mode="definition")
    assert ref["status"] == 0
    e_phi = rel(out["phi"], ref["phi"])
    e_u = {k: rel(out[k], ref[k]) for k in ("u", "v", "w")}
    print(f"256^3 FP64: cycles={st['cycles']} e_phi={e_phi:.3e} e_u={e_u}")
    assert e_phi <= 1e-9, e_phi
    for k, e in e_u.items():
        assert e <= 1e-9, (k, e)
    del ref
    alg = O.mac_project(prob)             # oracle, same algorithm, same inputs
    assert alg["status"] == 0
    assert abs(st["cycles"] - alg["cycles"]) <= 1
    if st["cycles"] == alg["cycles"]:
        assert rel(out["phi"], alg["phi"]) <= 1e-11
    del alg
    c = O.face_coeffs(prob.n, prob.periodic, prob.rho, prob.beta0_cc, prob.beta0_edge)
    u_c = O.correct(prob.n, prob.periodic, prob.dx, prob.beta0_cc, prob.beta0_edge, c,
                    out["phi"], prob.u, prob.v, prob.w)
    for name, exact in zip(("u", "v", "w"), u_c):
        assert rel(out[name], exact) <= 1e-12
    del u_c
    # post-projection constraint, evaluated by the oracle on the GPU output
    f = O.rhs(prob.n, prob.periodic, prob.dx, prob.beta0_cc, prob.beta0_edge, prob.u, prob.v, prob.w, prob.S)
    f0 = f - f.mean()
    div_new = O.rhs(prob.n, prob.periodic, prob.dx, prob.beta0_cc, prob.beta0_edge,
                    out["u"], out["v"], out["w"], prob.S)
    r = O.residual(prob.n, prob.periodic, prob.dx, c, out["phi"], f0)
    assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(f0)
    assert np.max(np.abs(div_new - f.mean() - r)) <= 1e-12 * np.max(np.abs(f0))


def test_mixed_precision_64(mp):
    prob = I.make_problem(64, H=0.15, rho_noise=0.05, seed=22)
    st, out = run_gpu(mp, prob, precision="mixed")
    check_against_definition(prob, st, out)


@pytest.mark.parametrize("shape,per", [
    ((40, 24, 56), (True, True, False)),     # ragged tiles in x, y and z
    ((64, 32, 48), (False, False, False)),   # walls everywhere
    ((32, 16, 32), (True, True, True)),      # fully periodic
    ((6, 10, 14), (True, True, False)),      # below the fused sweep's minimum tile
])
def test_mixed_precision_shapes(mp, shape, per):
    """Mixed precision (FP32 cycles, FP64 refinement) against the exact
    discrete solution, and its iteration count against the FP64 cycles."""
    prob = I.make_problem(shape, H=0.2, rho_noise=0.05, seed=31, periodic=per)
    st, out = run_gpu(mp, prob, precision="mixed")
    check_against_definition(prob, st, out)
    st64, _ = run_gpu(mp, prob)
    assert st["cycles"] <= st64["cycles"] + 2, (st["cycles"], st64["cycles"])


@pytest.mark.parametrize("inner", [1, 3])
def test_mixed_precision_inner_cycles(mp, inner):
    """Mixed precision with 1 and 3 FP32 V-cycles per refinement step (the
    default is 2) against the exact discrete solution; more V-cycles per
    step need no more refinement steps."""
    prob = I.make_problem((64, 32, 48), H=0.2, rho_noise=0.05, seed=37)
    st, out = run_gpu(mp, prob, precision="mixed", inner_cycles=inner)
    check_against_definition(prob, st, out)
    st2, _ = run_gpu(mp, prob, precision="mixed")
    assert (st["cycles"] >= st2["cycles"]) if inner == 1 else (st["cycles"] <= st2["cycles"])


def test_mixed_inner_cycles_changed_on_a_live_hierarchy(mp):
    """mg_set_params changing the FP32 V-cycles per refinement step between
    solves: the captured iteration graph is not reused, and each solve
    equals a fresh hierarchy's with the same count bit for bit."""
    prob = I.make_problem(64, H=0.15, rho_noise=0.05, seed=38)

    def solve(H):
        d = mp.to_device(prob)
        st = H.mac_project(d.rho, d.beta0_cc, d.beta0_edge, d.S, d.u, d.v, d.w, d.phi)
        torch.cuda.synchronize()
        return st, {k: getattr(d, k).cpu().numpy() for k in ("phi", "u", "v", "w")}

    live = mp.Hierarchy(mp.params_of(prob, precision="mixed"))
    try:
        for k in (0, 1, 3, 0):
            live.set_params(mp.params_of(prob, precision="mixed", inner_cycles=k))
            for _ in range(2):                    # the second solve replays the captured iteration
                st, out = solve(live)
                fresh = mp.Hierarchy(mp.params_of(prob, precision="mixed", inner_cycles=k))
                st0, out0 = solve(fresh)
                fresh.close()
                assert st["cycles"] == st0["cycles"] and st["rel_resid"] == st0["rel_resid"], k
                assert same_out(out, out0), k
    finally:
        live.close()


def test_mixed_precision_512_full_size(mp):
    """The 512^3 mixed-precision box (FP32 cycles, FP64 refinement): phi
    within 1e-9 of the FP64 oracle's exact discrete solution (definition
    mode), the residual and the correction checked by the oracle."""
    prob = I.MIXED_512()
    st, out = run_gpu(mp, prob, precision="mixed")
    assert st["status_name"] == "OK" and st["rel_resid"] <= 1e-10
    ref = O.mac_project(prob, mode="definition")
    assert ref["status"] == 0
    e_phi = rel(out["phi"], ref["phi"])
    e_u = {k: rel(out[k], ref[k]) for k in ("u", "v", "w")}
    print(f"512^3 mixed: refinement steps={st['cycles']} e_phi={e_phi:.3e} e_u={e_u}")
    assert e_phi <= 1e-9, e_phi
    for k, e in e_u.items():
        assert e <= 1e-9, (k, e)
    del ref
    c = O.face_coeffs(prob.n, prob.periodic, prob.rho, prob.beta0_cc, prob.beta0_edge)
    f = O.rhs(prob.n, prob.periodic, prob.dx, prob.beta0_cc, prob.beta0_edge, prob.u, prob.v, prob.w, prob.S)
    f -= f.mean()
    r = O.residual(prob.n, prob.periodic, prob.dx, c, out["phi"], f)
    assert np.linalg.norm(r) <= 1.05e-10 * np.linalg.norm(f)
    del r, f
    u_c = O.correct(prob.n, prob.periodic, prob.dx, prob.beta0_cc, prob.beta0_edge, c,
                    out["phi"], prob.u, prob.v, prob.w)
    for name, exact in zip(("u", "v", "w"), u_c):
        assert rel(out[name], exact) <= 1e-12, name
