"""FP64 CPU oracle for the MAC projection: Python side.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library; it is fed by the seeded input generators and nothing else.

Wraps ``mg_oracle.c`` (plain C, FP64, built with gcc) through ctypes.  The
arithmetic and the discretisation are documented in that file's header: the
projection enforcing the divergence constraint of the paper (Sec. 2) with
multigrid (Sec. 3).

Two ways to run the solver:

* ``mode="algorithm"``: the V(nu1, nu2) red-black Gauss-Seidel cycle step by
  step, stopping at the first cycle whose relative residual is <= rtol;
* ``mode="definition"``: the same cycles iterated to stagnation, i.e. the
  exact discrete solution up to round-off.  This is the reference for phi and
  U parity.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
_SRC_NODAL = os.path.join(_HERE, "nodal_oracle.c")
_LIB = os.path.join(_HERE, "libmgoracle.so")

STATUS = {0: "OK", -1: "INVALID_ARG", -2: "BAD_SIZE", -3: "INCOMPATIBLE_RHS",
          -4: "NOT_CONVERGED", -5: "NONFINITE", -6: "OOM"}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unknown-pragmas",
               _SRC, _SRC_NODAL, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                      os.path.getmtime(_SRC_NODAL)):
            build()
        L = ctypes.CDLL(_LIB)
        i, d = ctypes.c_int, ctypes.c_double
        L.orc_face_coeffs.argtypes = [i, i, i, i, i, i, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_rhs.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_rhs_w0.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_beta0_from_p0.argtypes = [i, d, _dp, _dp, _dp, _dp, _dp]
        L.orc_dp0_term.argtypes = [i, _dp, _dp, _dp, _dp]
        L.orc_mac_project_w0.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                         d, i, i, i, i, _dp, i, _dp]
        L.orc_apply.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _dp, _dp]
        L.orc_residual.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_rbgs.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _dp, _dp, i]
        L.orc_num_levels.argtypes = [i, i, i]
        L.orc_mg_create.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _ip]
        L.orc_mg_create.restype = ctypes.c_void_p
        L.orc_mg_destroy.argtypes = [ctypes.c_void_p]
        L.orc_mg_nlevels.argtypes = [ctypes.c_void_p]
        L.orc_mg_level_info.argtypes = [ctypes.c_void_p, i, _ip, _dp]
        L.orc_mg_io.argtypes = [ctypes.c_void_p, i, i, _dp, i]
        L.orc_mg_smooth.argtypes = [ctypes.c_void_p, i, i]
        L.orc_mg_resid_restrict.argtypes = [ctypes.c_void_p, i]
        L.orc_mg_prolong.argtypes = [ctypes.c_void_p, i]
        L.orc_mg_coarse.argtypes = [ctypes.c_void_p]
        L.orc_mg_vcycle.argtypes = [ctypes.c_void_p, i, i, i]
        L.orc_mg_solve.argtypes = [ctypes.c_void_p, _dp, _dp, d, i, i, i, i, _dp, i, _ip]
        L.orc_correct.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_mac_project.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                      d, i, i, i, i, _dp, i, _dp]
        L.orc_max_threads.argtypes = []
        ip6 = ctypes.POINTER(ctypes.c_int)
        L.orc_map_radial.argtypes = [i, i, i, d, i, d, _dp, _dp, _dp]
        L.orc_face_coeffs_gen.argtypes = [i, i, i, ip6, d, _dp, _dp, _dp, i, d, _dp, _dp, _dp, _dp, _dp]
        L.orc_rhs_gen.argtypes = [i, i, i, ip6, d, _dp, _dp, i, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_apply_gen.argtypes = [i, i, i, ip6, d, _dp, _dp, _dp, _dp, _dp]
        L.orc_rbgs_gen.argtypes = [i, i, i, ip6, d, _dp, _dp, _dp, _dp, _dp, i]
        L.orc_correct_gen.argtypes = [i, i, i, ip6, d, _dp, _dp, _dp, _dp, _dp]
        L.orc_mg_create_gen.argtypes = [i, i, i, ip6, d, _dp, _dp, _dp, _ip]
        L.orc_mg_create_gen.restype = ctypes.c_void_p
        L.nod_num_levels.argtypes = [i, i, i, i, i, i]
        L.nod_sigma.argtypes = [i, i, i, _dp, _dp, _dp]
        L.nod_apply.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp]
        L.nod_gs.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, i]
        L.nod_rhs.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _dp, _dp, _dp]
        L.nod_correct.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _dp, _dp]
        L.nod_project.argtypes = [i, i, i, i, i, i, d, _dp, _dp, _dp, _dp, _dp, _dp, _dp, d, i, i, i, i, _dp, i,
                                  _dp]
        L.nod_mg_create.argtypes = [i, i, i, i, i, i, d, _dp, _ip]
        L.nod_mg_create.restype = ctypes.c_void_p
        L.nod_mg_destroy.argtypes = [ctypes.c_void_p]
        L.nod_mg_nlevels.argtypes = [ctypes.c_void_p]
        L.nod_mg_level_info.argtypes = [ctypes.c_void_p, i, _ip]
        L.nod_mg_io.argtypes = [ctypes.c_void_p, i, i, _dp, i]
        L.nod_mg_smooth.argtypes = [ctypes.c_void_p, i, i]
        L.nod_mg_resid_restrict.argtypes = [ctypes.c_void_p, i]
        L.nod_mg_prolong.argtypes = [ctypes.c_void_p, i]
        L.nod_mg_coarse.argtypes = [ctypes.c_void_p]
        L.nod_mg_solve.argtypes = [ctypes.c_void_p, _dp, _dp, d, i, i, i, i, _dp, i, _ip]
        L.orc_mac_project_gen.argtypes = [i, i, i, ip6, d, _dp, _dp, _dp, i, d, _dp, _dp, _dp, _dp, _dp, _dp,
                                          _dp, _dp, d, i, i, i, i, _dp, i, _dp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _shape_args(n, periodic):
    nx, ny, nz = n
    px, py, pz = (1 if p else 0 for p in periodic)
    return nx, ny, nz, px, py, pz


SIDE_PERIODIC, SIDE_WALL, SIDE_OUTFLOW = 0, 1, 2


def side_codes(periodic, outflow=None):
    """Per-side codes (x low, x high, y low, y high, z low, z high): 0
    periodic, 1 solid wall, 2 outflow (phi = 0).  ``outflow`` is None or six
    booleans; a periodic direction ignores it."""
    outflow = (False,) * 6 if outflow is None else tuple(bool(o) for o in outflow)
    codes = []
    for d in range(3):
        for e in range(2):
            if periodic[d]:
                codes.append(SIDE_PERIODIC)
            else:
                codes.append(SIDE_OUTFLOW if outflow[2 * d + e] else SIDE_WALL)
    return (ctypes.c_int * 6)(*codes)


def _opt(a):
    return None if a is None else _p(np.ascontiguousarray(a, dtype=np.float64))


def _radial_args(radial):
    """(nr, dr, profile, centre) for a radial beta0 given as (profile, dr,
    centre); zeros / None for a plane-parallel one."""
    if radial is None:
        return 0, 0.0, None, None
    prof, dr, centre = radial
    prof = np.ascontiguousarray(prof, dtype=np.float64)
    return len(prof), float(dr), _p(prof), _p(np.ascontiguousarray(centre, dtype=np.float64))


def map_radial(n, h, prof, dr, centre):
    """beta0 of a radial profile at the cell centres (nz, ny, nx)."""
    nx, ny, nz = n
    out = np.empty((nz, ny, nx))
    prof = np.ascontiguousarray(prof, dtype=np.float64)
    lib().orc_map_radial(nx, ny, nz, h, len(prof), float(dr), _p(prof),
                         _p(np.ascontiguousarray(centre, dtype=np.float64)), _p(out))
    return out


def face_coeffs_gen(n, sides, h, rho, b0c=None, b0e=None, radial=None):
    """Full face arrays with per-side boundaries (``sides`` from side_codes)
    and a plane-parallel (b0c, b0e) or radial (profile, dr, centre) beta0."""
    nx, ny, nz = n
    bx = np.empty((nz, ny, nx + 1))
    by = np.empty((nz, ny + 1, nx))
    bz = np.empty((nz + 1, ny, nx))
    st = lib().orc_face_coeffs_gen(nx, ny, nz, sides, h, _p(rho), _opt(b0c), _opt(b0e), *_radial_args(radial),
                                   _p(bx), _p(by), _p(bz))
    assert st == 0
    return bx, by, bz


def rhs_gen(n, sides, h, u, v, w, S, b0c=None, b0e=None, radial=None, w0=None):
    """f = D(beta0 U) - beta0 (S - w0) with each face velocity weighted by its
    own face's beta0."""
    nx, ny, nz = n
    f = np.empty((nz, ny, nx))
    st = lib().orc_rhs_gen(nx, ny, nz, sides, h, _opt(b0c), _opt(b0e), *_radial_args(radial), _p(u), _p(v),
                           _p(w), _p(S), _opt(w0), _p(f))
    assert st == 0
    return f


def apply_gen(n, sides, h, coeffs, phi):
    bx, by, bz = coeffs
    out = np.empty_like(phi)
    lib().orc_apply_gen(*n, sides, h, _p(bx), _p(by), _p(bz), _p(phi), _p(out))
    return out


def rbgs_gen(n, sides, h, coeffs, phi, f, nsweeps=1):
    bx, by, bz = coeffs
    out = np.ascontiguousarray(phi, dtype=np.float64).copy()
    lib().orc_rbgs_gen(*n, sides, h, _p(bx), _p(by), _p(bz), _p(out), _p(f), nsweeps)
    return out


def correct_gen(n, sides, h, rho, phi, u, v, w):
    u, v, w = u.copy(), v.copy(), w.copy()
    lib().orc_correct_gen(*n, sides, h, _p(rho), _p(phi), _p(u), _p(v), _p(w))
    return u, v, w


def num_levels(n) -> int:
    return lib().orc_num_levels(*n)


def max_threads() -> int:
    return lib().orc_max_threads()


def face_coeffs(n, periodic, rho, b0c, b0e):
    """Full face arrays bx (nz,ny,nx+1), by (nz,ny+1,nx), bz (nz+1,ny,nx)."""
    nx, ny, nz = n
    bx = np.empty((nz, ny, nx + 1))
    by = np.empty((nz, ny + 1, nx))
    bz = np.empty((nz + 1, ny, nx))
    lib().orc_face_coeffs(*_shape_args(n, periodic), _p(rho), _p(b0c), _p(b0e), _p(bx), _p(by), _p(bz))
    return bx, by, bz


def rhs(n, periodic, h, b0c, b0e, u, v, w, S, w0=None):
    """f = D(beta0 U) - beta0 (S - w0[k]) (before mean removal); w0 = None
    leaves the dp0/dt term folded into S."""
    nx, ny, nz = n
    f = np.empty((nz, ny, nx))
    if w0 is None:
        lib().orc_rhs(*_shape_args(n, periodic), h, _p(b0c), _p(b0e), _p(u), _p(v), _p(w), _p(S), _p(f))
    else:
        w0 = np.ascontiguousarray(w0, dtype=np.float64)
        lib().orc_rhs_w0(*_shape_args(n, periodic), h, _p(b0c), _p(b0e), _p(u), _p(v), _p(w), _p(S), _p(w0),
                         _p(f))
    return f


def beta0_from_p0(rho0_base, p0_edge, p0_cc, gamma1_cc):
    """beta0 at layer centres and z faces from p0 (faces and centres) and the
    layer Gamma1 (Sec. 2, definition of beta0; see mg_oracle.c)."""
    nz = len(p0_cc)
    b0c = np.empty(nz)
    b0e = np.empty(nz + 1)
    st = lib().orc_beta0_from_p0(nz, float(rho0_base), _p(np.ascontiguousarray(p0_edge, dtype=np.float64)),
                                 _p(np.ascontiguousarray(p0_cc, dtype=np.float64)),
                                 _p(np.ascontiguousarray(gamma1_cc, dtype=np.float64)), _p(b0c), _p(b0e))
    if st != 0:
        raise ValueError(f"orc_beta0_from_p0: {STATUS.get(st, st)}")
    return b0c, b0e


def dp0_term(p0_cc, gamma1_cc, dp0dt_cc):
    """w0[k] = dp0dt[k] / (Gamma1[k] p0[k]), the dp0/dt term of the constraint per layer."""
    nz = len(p0_cc)
    w0 = np.empty(nz)
    st = lib().orc_dp0_term(nz, _p(np.ascontiguousarray(p0_cc, dtype=np.float64)),
                            _p(np.ascontiguousarray(gamma1_cc, dtype=np.float64)),
                            _p(np.ascontiguousarray(dp0dt_cc, dtype=np.float64)), _p(w0))
    if st != 0:
        raise ValueError(f"orc_dp0_term: {STATUS.get(st, st)}")
    return w0


def apply(n, periodic, h, coeffs, phi):
    """L phi."""
    bx, by, bz = coeffs
    out = np.empty_like(phi)
    lib().orc_apply(*_shape_args(n, periodic), h, _p(bx), _p(by), _p(bz), _p(phi), _p(out))
    return out


def residual(n, periodic, h, coeffs, phi, f):
    bx, by, bz = coeffs
    r = np.empty_like(phi)
    lib().orc_residual(*_shape_args(n, periodic), h, _p(bx), _p(by), _p(bz), _p(phi), _p(f), _p(r))
    return r


def rbgs(n, periodic, h, coeffs, phi, f, nsweeps=1):
    """Red-black Gauss-Seidel sweeps, returns a new array."""
    bx, by, bz = coeffs
    out = np.ascontiguousarray(phi, dtype=np.float64).copy()
    lib().orc_rbgs(*_shape_args(n, periodic), h, _p(bx), _p(by), _p(bz), _p(out), _p(f), nsweeps)
    return out


def correct(n, periodic, h, b0c, b0e, coeffs, phi, u, v, w):
    """Corrected copies of u, v, w."""
    bx, by, bz = coeffs
    u, v, w = u.copy(), v.copy(), w.copy()
    lib().orc_correct(*_shape_args(n, periodic), h, _p(b0c), _p(b0e), _p(bx), _p(by), _p(bz),
                      _p(phi), _p(u), _p(v), _p(w))
    return u, v, w


class Hierarchy:
    """The oracle's multigrid hierarchy, exposing every step of the V-cycle."""

    def __init__(self, n, periodic, h, coeffs, outflow=None):
        self.n = tuple(n)
        self.periodic = tuple(periodic)
        bx, by, bz = (np.ascontiguousarray(c) for c in coeffs)
        st = ctypes.c_int(0)
        self._h = lib().orc_mg_create_gen(*self.n, side_codes(periodic, outflow), h, _p(bx), _p(by), _p(bz),
                                          ctypes.byref(st))
        if not self._h:
            raise RuntimeError(f"oracle hierarchy: {STATUS.get(st.value, st.value)}")
        self.nlevels = lib().orc_mg_nlevels(self._h)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_mg_destroy(self._h)
            self._h = None

    def level(self, l):
        dims = (ctypes.c_int * 3)()
        h = ctypes.c_double()
        lib().orc_mg_level_info(self._h, l, dims, ctypes.byref(h))
        return (dims[0], dims[1], dims[2]), h.value

    _WHICH = {"phi": 0, "f": 1, "r": 2, "bx": 3, "by": 4, "bz": 5}

    def _shape(self, l, which):
        (nx, ny, nz), _ = self.level(l)
        return {"phi": (nz, ny, nx), "f": (nz, ny, nx), "r": (nz, ny, nx),
                "bx": (nz, ny, nx + 1), "by": (nz, ny + 1, nx), "bz": (nz + 1, ny, nx)}[which]

    def get(self, l, which):
        out = np.empty(self._shape(l, which))
        st = lib().orc_mg_io(self._h, l, self._WHICH[which], _p(out), 0)
        assert st == 0
        return out

    def set(self, l, which, arr):
        arr = np.ascontiguousarray(arr, dtype=np.float64)
        assert arr.shape == self._shape(l, which)
        st = lib().orc_mg_io(self._h, l, self._WHICH[which], _p(arr), 1)
        assert st == 0

    def smooth(self, l, nsweeps):
        lib().orc_mg_smooth(self._h, l, nsweeps)

    def resid_restrict(self, l):
        lib().orc_mg_resid_restrict(self._h, l)

    def prolong(self, l):
        lib().orc_mg_prolong(self._h, l)

    def coarse(self):
        lib().orc_mg_coarse(self._h)

    def vcycle(self, l=0, nu1=2, nu2=2):
        lib().orc_mg_vcycle(self._h, l, nu1, nu2)

    def solve(self, f, rtol=1e-10, max_cycles=100, nu1=2, nu2=2, mode="algorithm"):
        """Solve L phi = f (f must already have zero mean).  Returns (status, phi, hist)."""
        f = np.ascontiguousarray(f, dtype=np.float64)
        phi = np.empty_like(f)
        hist = np.full(max_cycles + 1, np.nan)
        cyc = ctypes.c_int(0)
        st = lib().orc_mg_solve(self._h, _p(f), _p(phi), rtol, max_cycles, nu1, nu2,
                                1 if mode == "definition" else 0, _p(hist), len(hist), ctypes.byref(cyc))
        return st, phi, hist[: cyc.value + 1]


def mac_project_full(prob, mode="algorithm", rtol=None, max_cycles=None):
    """The projection of a problem whose base state is given as p0 and
    Gamma1 (inputs.make_full_problem): beta0 from p0, the dp0/dt term of the
    constraint, then the projection with the full right-hand side.  Returns
    mac_project's dict plus beta0_cc, beta0_edge and w0."""
    b0c, b0e = beta0_from_p0(prob.rho0_base, prob.p0_edge, prob.p0_cc, prob.gamma1_cc)
    w0 = dp0_term(prob.p0_cc, prob.gamma1_cc, prob.dp0dt_cc)
    out = _project(prob, b0c, b0e, w0, mode, rtol, max_cycles, None, None)
    out.update(beta0_cc=b0c, beta0_edge=b0e, w0=w0)
    return out


def mac_project(prob, mode="algorithm", rtol=None, max_cycles=None, nu1=None, nu2=None):
    """The whole projection on host copies of ``prob`` (an inputs.Problem).

    Returns a dict with status, phi (zero mean unless a side is an outflow),
    corrected u/v/w, the residual history and the RHS statistics.  Problems
    with outflow sides or a radial beta0 take the general-boundary path.
    """
    if is_general(prob):
        return _project_gen(prob, mode, rtol, max_cycles, nu1, nu2)
    return _project(prob, prob.beta0_cc, prob.beta0_edge, None, mode, rtol, max_cycles, nu1, nu2)


def is_general(prob):
    return any(getattr(prob, "outflow", None) or ()) or getattr(prob, "beta0_r", None) is not None


def prob_radial(prob):
    if getattr(prob, "beta0_r", None) is None:
        return None
    return prob.beta0_r, prob.dr_base, prob.centre


def _project_gen(prob, mode, rtol, max_cycles, nu1, nu2, w0=None):
    n = prob.n
    rtol = prob.rtol if rtol is None else rtol
    max_cycles = (prob.max_cycles if mode == "algorithm" else 200) if max_cycles is None else max_cycles
    nu1 = prob.pre_sweeps if nu1 is None else nu1
    nu2 = prob.post_sweeps if nu2 is None else nu2
    u, v, w = prob.u.copy(), prob.v.copy(), prob.w.copy()
    nx, ny, nz = n
    phi = np.zeros((nz, ny, nx))
    hist = np.full(max_cycles + 1, np.nan)
    stats = np.zeros(8)
    st = lib().orc_mac_project_gen(nx, ny, nz, side_codes(prob.periodic, prob.outflow), prob.dx, _p(prob.rho),
                                   _opt(prob.beta0_cc), _opt(prob.beta0_edge), *_radial_args(prob_radial(prob)),
                                   _p(prob.S), _opt(w0), _p(u), _p(v), _p(w), _p(phi), rtol, max_cycles, nu1,
                                   nu2, 1 if mode == "definition" else 0, _p(hist), len(hist), _p(stats))
    cycles = int(stats[0])
    return {"status": st, "status_name": STATUS.get(st, str(st)), "phi": phi, "u": u, "v": v, "w": w,
            "cycles": cycles, "hist": hist[: cycles + 1], "rel_resid": stats[1],
            "mean_removed": stats[2], "sum_f": stats[3], "sum_abs_f": stats[4], "norm_f": stats[5]}


def _project(prob, b0c, b0e, w0, mode, rtol, max_cycles, nu1, nu2):
    n, per = prob.n, prob.periodic
    rtol = prob.rtol if rtol is None else rtol
    max_cycles = (prob.max_cycles if mode == "algorithm" else 200) if max_cycles is None else max_cycles
    nu1 = prob.pre_sweeps if nu1 is None else nu1
    nu2 = prob.post_sweeps if nu2 is None else nu2
    u, v, w = prob.u.copy(), prob.v.copy(), prob.w.copy()
    nx, ny, nz = n
    phi = np.zeros((nz, ny, nx))
    hist = np.full(max_cycles + 1, np.nan)
    stats = np.zeros(8)
    w0p = _p(np.ascontiguousarray(w0, dtype=np.float64)) if w0 is not None else None
    st = lib().orc_mac_project_w0(*_shape_args(n, per), prob.dx, _p(prob.rho), _p(b0c), _p(b0e), _p(prob.S),
                                  w0p, _p(u), _p(v), _p(w), _p(phi),
                                  rtol, max_cycles, nu1, nu2, 1 if mode == "definition" else 0,
                                  _p(hist), len(hist), _p(stats))
    cycles = int(stats[0])
    return {"status": st, "status_name": STATUS.get(st, str(st)), "phi": phi, "u": u, "v": v, "w": w,
            "cycles": cycles, "hist": hist[: cycles + 1], "rel_resid": stats[1],
            "mean_removed": stats[2], "sum_f": stats[3], "sum_abs_f": stats[4], "norm_f": stats[5]}


# ---------------------------------------------------------------- nodal
# The nodal (cell-velocity) projection: phi on the cell corners, cell-centred
# velocities (see nodal_oracle.c for the discretisation).

def node_dims(n, periodic):
    """Node counts (Nx, Ny, Nz): n in a periodic direction, n + 1 otherwise."""
    return tuple(int(n[d]) + (0 if periodic[d] else 1) for d in range(3))


def nodal_num_levels(n, periodic):
    return lib().nod_num_levels(*_shape_args(n, periodic))


def nodal_sigma(rho, b0c):
    nz, ny, nx = rho.shape
    sig = np.empty_like(rho)
    lib().nod_sigma(nx, ny, nz, _p(rho), _p(np.ascontiguousarray(b0c, dtype=np.float64)), _p(sig))
    return sig


def nodal_apply(n, periodic, h, sig, phi):
    Nx, Ny, Nz = node_dims(n, periodic)
    out = np.empty((Nz, Ny, Nx))
    lib().nod_apply(*_shape_args(n, periodic), h, _p(sig), _p(np.ascontiguousarray(phi, dtype=np.float64)), _p(out))
    return out


def nodal_gs(n, periodic, h, sig, phi, f, nsweeps=1):
    out = np.ascontiguousarray(phi, dtype=np.float64).copy()
    lib().nod_gs(*_shape_args(n, periodic), h, _p(sig), _p(out), _p(np.ascontiguousarray(f, dtype=np.float64)),
                 nsweeps)
    return out


def nodal_rhs(n, periodic, h, b0c, uc, vc, wc, S):
    Nx, Ny, Nz = node_dims(n, periodic)
    f = np.empty((Nz, Ny, Nx))
    lib().nod_rhs(*_shape_args(n, periodic), h, _p(np.ascontiguousarray(b0c, dtype=np.float64)), _p(uc), _p(vc),
                  _p(wc), _p(S), _p(f))
    return f


def nodal_correct(n, periodic, h, rho, phi, uc, vc, wc):
    uc, vc, wc = uc.copy(), vc.copy(), wc.copy()
    lib().nod_correct(*_shape_args(n, periodic), h, _p(rho), _p(np.ascontiguousarray(phi, dtype=np.float64)),
                      _p(uc), _p(vc), _p(wc))
    return uc, vc, wc


class NodalHierarchy:
    """The oracle's nodal multigrid hierarchy, exposing every step."""

    def __init__(self, n, periodic, h, sig):
        self.n = tuple(n)
        self.periodic = tuple(periodic)
        st = ctypes.c_int(0)
        self._h = lib().nod_mg_create(*_shape_args(n, periodic), h, _p(np.ascontiguousarray(sig)),
                                      ctypes.byref(st))
        if not self._h:
            raise RuntimeError(f"nodal oracle hierarchy: {STATUS.get(st.value, st.value)}")
        self.nlevels = lib().nod_mg_nlevels(self._h)

    def __del__(self):
        if getattr(self, "_h", None):
            lib().nod_mg_destroy(self._h)
            self._h = None

    def dims(self, l):
        d = (ctypes.c_int * 6)()
        lib().nod_mg_level_info(self._h, l, d)
        return (d[0], d[1], d[2]), (d[3], d[4], d[5])

    _WHICH = {"phi": 0, "f": 1, "r": 2, "sigma": 3}

    def _shape(self, l, which):
        (Nx, Ny, Nz), (nx, ny, nz) = self.dims(l)
        return (nz, ny, nx) if which == "sigma" else (Nz, Ny, Nx)

    def get(self, l, which):
        out = np.empty(self._shape(l, which))
        assert lib().nod_mg_io(self._h, l, self._WHICH[which], _p(out), 0) == 0
        return out

    def set(self, l, which, arr):
        arr = np.ascontiguousarray(arr, dtype=np.float64)
        assert arr.shape == self._shape(l, which)
        assert lib().nod_mg_io(self._h, l, self._WHICH[which], _p(arr), 1) == 0

    def smooth(self, l, nsweeps):
        lib().nod_mg_smooth(self._h, l, nsweeps)

    def resid_restrict(self, l):
        lib().nod_mg_resid_restrict(self._h, l)

    def prolong(self, l):
        lib().nod_mg_prolong(self._h, l)

    def coarse(self):
        lib().nod_mg_coarse(self._h)

    def solve(self, f, rtol=1e-10, max_cycles=100, nu1=2, nu2=2, mode="algorithm"):
        f = np.ascontiguousarray(f, dtype=np.float64)
        phi = np.empty_like(f)
        hist = np.full(max_cycles + 1, np.nan)
        cyc = ctypes.c_int(0)
        st = lib().nod_mg_solve(self._h, _p(f), _p(phi), rtol, max_cycles, nu1, nu2,
                                1 if mode == "definition" else 0, _p(hist), len(hist), ctypes.byref(cyc))
        return st, phi, hist[: cyc.value + 1]


def nodal_project(prob, mode="algorithm", rtol=None, max_cycles=None, nu1=None, nu2=None):
    """The nodal projection of an inputs.NodalProblem (host copies)."""
    n, per = prob.n, prob.periodic
    rtol = prob.rtol if rtol is None else rtol
    max_cycles = (prob.max_cycles if mode == "algorithm" else 200) if max_cycles is None else max_cycles
    nu1 = prob.pre_sweeps if nu1 is None else nu1
    nu2 = prob.post_sweeps if nu2 is None else nu2
    uc, vc, wc = prob.uc.copy(), prob.vc.copy(), prob.wc.copy()
    Nx, Ny, Nz = node_dims(n, per)
    phi = np.zeros((Nz, Ny, Nx))
    hist = np.full(max_cycles + 1, np.nan)
    stats = np.zeros(8)
    st = lib().nod_project(*_shape_args(n, per), prob.dx, _p(prob.rho), _p(prob.beta0_cc), _p(prob.S), _p(uc),
                           _p(vc), _p(wc), _p(phi), rtol, max_cycles, nu1, nu2, 1 if mode == "definition" else 0,
                           _p(hist), len(hist), _p(stats))
    cycles = int(stats[0])
    return {"status": st, "status_name": STATUS.get(st, str(st)), "phi": phi, "u": uc, "v": vc, "w": wc,
            "cycles": cycles, "hist": hist[: cycles + 1], "rel_resid": stats[1], "mean_removed": stats[2],
            "sum_f": stats[3], "sum_abs_f": stats[4], "norm_f": stats[5]}
