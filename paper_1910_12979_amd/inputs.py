"""Seeded synthetic inputs for the variable-coefficient MAC projection.

This module only draws and lays out input fields; it holds none of the
projection's arithmetic, so both the HIP path and the CPU oracle can be fed
from it.  Every field is float64, C-ordered ``[k][j][i]`` (i fastest):

* cell fields (rho, S): shape ``(nz, ny, nx)``
* x-face velocity u: ``(nz, ny, nx+1)``, face i sits between cells i-1 and i
* y-face velocity v: ``(nz, ny+1, nx)``
* z-face velocity w: ``(nz+1, ny, nx)``
* base state beta0 at cell centres ``(nz,)`` and at z-faces ``(nz+1,)``

The stratified base state follows the plane-parallel reading of the paper's
1-D base state beta0(r) (Sec. 2, definition of beta0) with r taken as the
height z and an exponential profile exp(-z/H).  The expansion term S is an
input field (Sec. 2, constraint and expansion-term equations); where it is
random its beta0-weighted mean is removed so that the divergence constraint is
solvable with periodic / solid-wall boundaries.

Draw order for a problem (one ``numpy.random.default_rng(seed)`` stream):
rho noise (nz,ny,nx); S noise (nz,ny,nx) only when S is random; u faces
0..nx-1; v faces 0..ny-1; w faces 1..nz-1 (all standard normal).  Periodic
duplicate faces (face n) are then copied from face 0; wall faces are zero.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "Problem", "make_problem", "stratified_base_state",
    "make_full_problem", "make_star_problem", "mixed_batch_specs", "serving_requests",
    "NodalProblem", "make_nodal_problem",
    "SMALL_BOX", "STEEP_256", "MIXED_512",
]


@dataclasses.dataclass
class Problem:
    """One projection problem: inputs and solver parameters (host arrays)."""
    n: tuple            # (nx, ny, nz) cells
    dx: float
    periodic: tuple     # (px, py, pz) booleans; False means solid walls on both sides
    rho: np.ndarray
    beta0_cc: np.ndarray
    beta0_edge: np.ndarray
    S: np.ndarray
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    rtol: float = 1e-10
    max_cycles: int = 100
    pre_sweeps: int = 2
    post_sweeps: int = 2
    seed: int = 0
    H: float = 0.3
    # base state given as p0 and Gamma1 instead of beta0 (make_full_problem):
    # beta0 and the dp0/dt term of the constraint are then computed by the
    # method; beta0_cc / beta0_edge are None
    rho0_base: float | None = None
    p0_cc: np.ndarray | None = None       # (nz,)
    p0_edge: np.ndarray | None = None     # (nz+1,)
    gamma1_cc: np.ndarray | None = None   # (nz,)
    dp0dt_cc: np.ndarray | None = None    # (nz,)
    # outflow sides (phi = 0 on the boundary faces): x low, x high, y low,
    # y high, z low, z high; only for non-periodic directions
    outflow: tuple = (False, False, False, False, False, False)
    # radial base state (make_star_problem): beta0_r[m] at r = (m + 1/2)
    # dr_base from centre; beta0_cc / beta0_edge are then None
    beta0_r: np.ndarray | None = None
    dr_base: float | None = None
    centre: tuple | None = None

    @property
    def ncells(self) -> int:
        nx, ny, nz = self.n
        return nx * ny * nz

    def copy(self) -> "Problem":
        out = dataclasses.replace(self)
        for name in ("rho", "beta0_cc", "beta0_edge", "S", "u", "v", "w",
                     "p0_cc", "p0_edge", "gamma1_cc", "dp0dt_cc", "beta0_r"):
            a = getattr(self, name)
            setattr(out, name, None if a is None else a.copy())
        return out


def stratified_base_state(nz: int, dx: float, H: float):
    """beta0 = exp(-z/H) at cell centres z=(k+1/2)dx and at z-faces z=k dx."""
    zc = (np.arange(nz, dtype=np.float64) + 0.5) * dx
    ze = np.arange(nz + 1, dtype=np.float64) * dx
    return np.exp(-zc / H), np.exp(-ze / H)


def _fill_faces(u, v, w, periodic):
    px, py, pz = periodic
    if px:
        u[:, :, -1] = u[:, :, 0]
    else:
        u[:, :, 0] = 0.0
        u[:, :, -1] = 0.0
    if py:
        v[:, -1, :] = v[:, 0, :]
    else:
        v[:, 0, :] = 0.0
        v[:, -1, :] = 0.0
    if pz:
        w[-1] = w[0]
    else:
        w[0] = 0.0
        w[-1] = 0.0


def _draw_outflow_faces(rng, u, v, w, periodic, outflow, vel_scale):
    """Normal velocities of the outflow boundary faces (drawn after every
    other field, side by side in the order x low, x high, ..., z high)."""
    for q in range(6):
        d, hi = divmod(q, 2)
        if periodic[d] or not outflow[q]:
            continue
        if d == 0:
            u[:, :, -1 if hi else 0] = vel_scale * rng.standard_normal(u.shape[:2])
        elif d == 1:
            v[:, -1 if hi else 0, :] = vel_scale * rng.standard_normal((v.shape[0], v.shape[2]))
        else:
            w[-1 if hi else 0] = vel_scale * rng.standard_normal(w.shape[1:])


def make_problem(n, *, H=0.3, rho_noise=0.01, S_kind="random", S_amp=0.1,
                 seed=0, dx=None, periodic=(True, True, False), rtol=1e-10,
                 max_cycles=100, vel_scale=1.0, outflow=None) -> Problem:
    """Draw one seeded problem.

    ``n`` is an int (cubic box) or an ``(nx, ny, nz)`` tuple.  ``dx`` defaults
    to ``1/nx`` (the unit box for cubic grids).  ``S_kind`` is ``"random"``
    (S_amp * N(0,1) with the beta0-weighted mean removed), ``"sine"``
    (sin(2 pi x) sin(2 pi y) cos(pi z) at cell centres) or ``"zero"``.
    ``outflow``: six booleans (x low, x high, ..., z high) marking sides of
    non-periodic directions as outflow (phi = 0) instead of solid walls; their
    boundary-face velocities are drawn last, so the other fields are those of
    the same seed without outflow sides.
    """
    if isinstance(n, int):
        n = (n, n, n)
    nx, ny, nz = (int(a) for a in n)
    if dx is None:
        dx = 1.0 / nx
    periodic = tuple(bool(p) for p in periodic)
    rng = np.random.default_rng(seed)
    b0c, b0e = stratified_base_state(nz, dx, H)
    xi_rho = rng.standard_normal((nz, ny, nx))
    rho = b0c[:, None, None] * (1.0 + rho_noise * xi_rho)
    if S_kind == "random":
        S = S_amp * rng.standard_normal((nz, ny, nx))
        wts = np.broadcast_to(b0c[:, None, None], S.shape)
        S -= float(np.sum(wts * S) / np.sum(wts))
    elif S_kind == "sine":
        x = (np.arange(nx) + 0.5) * dx
        y = (np.arange(ny) + 0.5) * dx
        z = (np.arange(nz) + 0.5) * dx
        S = (np.cos(np.pi * z)[:, None, None] * np.sin(2 * np.pi * y)[None, :, None]
             * np.sin(2 * np.pi * x)[None, None, :])
    elif S_kind == "zero":
        S = np.zeros((nz, ny, nx))
    else:
        raise ValueError(f"unknown S_kind {S_kind!r}")
    u = np.zeros((nz, ny, nx + 1))
    v = np.zeros((nz, ny + 1, nx))
    w = np.zeros((nz + 1, ny, nx))
    u[:, :, :nx] = vel_scale * rng.standard_normal((nz, ny, nx))
    v[:, :ny, :] = vel_scale * rng.standard_normal((nz, ny, nx))
    if nz > 1:
        w[1:nz] = vel_scale * rng.standard_normal((nz - 1, ny, nx))
    if periodic[2]:
        # periodic z: face 0 is a real face, drawn after the interior faces
        w[0] = vel_scale * rng.standard_normal((ny, nx))
    _fill_faces(u, v, w, periodic)
    outflow = (False,) * 6 if outflow is None else tuple(bool(o) for o in outflow)
    _draw_outflow_faces(rng, u, v, w, periodic, outflow, vel_scale)
    return Problem(n=(nx, ny, nz), dx=float(dx), periodic=periodic, rho=rho,
                   beta0_cc=b0c, beta0_edge=b0e, S=np.ascontiguousarray(S),
                   u=u, v=v, w=w, rtol=rtol, max_cycles=max_cycles, seed=seed, H=H,
                   outflow=outflow)


def make_full_problem(n, *, Hp=0.25, gamma1=(5.0 / 3.0, 1.3), rho0_base=1.0, rho_noise=0.01, S_amp=0.1,
                      q_amp=0.05, seed=0, dx=None, periodic=(True, True, False), rtol=1e-10,
                      max_cycles=100) -> Problem:
    """A problem whose base state is given the way the method carries it:
    p0 and the layer Gamma1, from which beta0 follows (Sec. 2, definition of
    beta0), plus dp0/dt, which enters the constraint's right-hand side.

    p0 = exp(-z/Hp) at the z faces and layer centres; Gamma1 varies linearly
    over the layers from gamma1[0] at the bottom to gamma1[1] at the top;
    rho = exp(-z/(Gm Hp)) (1 + rho_noise N(0,1)) with Gm the mean of the two
    Gamma1 values.  S = S' + q_k: S' = S_amp N(0,1) with each layer's mean
    removed, q_k = q_amp cos(pi z_k) a layer-mean expansion, and dp0/dt_k =
    q_k Gamma1_k p0_k, so that the dp0/dt term takes up the layer-mean
    expansion (as the base state's pressure change does in the method) and the
    constraint is solvable whatever beta0 the base state gives.  Draw order as
    make_problem: rho noise, S' noise, u, v, w.
    """
    if isinstance(n, int):
        n = (n, n, n)
    nx, ny, nz = (int(a) for a in n)
    if dx is None:
        dx = 1.0 / nx
    periodic = tuple(bool(p) for p in periodic)
    rng = np.random.default_rng(seed)
    zc = (np.arange(nz, dtype=np.float64) + 0.5) * dx
    ze = np.arange(nz + 1, dtype=np.float64) * dx
    p0c, p0e = np.exp(-zc / Hp), np.exp(-ze / Hp)
    frac = (np.arange(nz, dtype=np.float64) + 0.5) / nz
    g1 = gamma1[0] + (gamma1[1] - gamma1[0]) * frac
    gm = 0.5 * (gamma1[0] + gamma1[1])
    xi_rho = rng.standard_normal((nz, ny, nx))
    rho = rho0_base * np.exp(-zc / (gm * Hp))[:, None, None] * (1.0 + rho_noise * xi_rho)
    Sp = S_amp * rng.standard_normal((nz, ny, nx))
    Sp -= Sp.mean(axis=(1, 2), keepdims=True)
    q = q_amp * np.cos(np.pi * zc)
    S = Sp + q[:, None, None]
    dp0dt = q * g1 * p0c
    u = np.zeros((nz, ny, nx + 1))
    v = np.zeros((nz, ny + 1, nx))
    w = np.zeros((nz + 1, ny, nx))
    u[:, :, :nx] = rng.standard_normal((nz, ny, nx))
    v[:, :ny, :] = rng.standard_normal((nz, ny, nx))
    if nz > 1:
        w[1:nz] = rng.standard_normal((nz - 1, ny, nx))
    if periodic[2]:
        w[0] = rng.standard_normal((ny, nx))
    _fill_faces(u, v, w, periodic)
    return Problem(n=(nx, ny, nz), dx=float(dx), periodic=periodic, rho=rho,
                   beta0_cc=None, beta0_edge=None, S=np.ascontiguousarray(S),
                   u=u, v=v, w=w, rtol=rtol, max_cycles=max_cycles, seed=seed, H=Hp,
                   rho0_base=float(rho0_base), p0_cc=p0c, p0_edge=p0e, gamma1_cc=g1, dp0dt_cc=dp0dt)


def make_star_problem(n, *, Hr=0.15, rho_noise=0.01, S_amp=0.1, seed=0, dx=None, centre=None,
                      dr_per_dx=0.5, outflow=(True,) * 6, rtol=1e-10, max_cycles=100) -> Problem:
    """A star-like box: the base state is a function of the radius from a
    centre (spherical base state), the domain boundaries are outflow sides.

    beta0_r[m] = exp(-r_m/Hr) at r_m = (m + 1/2) dr, dr = dr_per_dx * dx,
    with enough points to reach every corner of the box; rho =
    exp(-r_c/Hr) (1 + rho_noise N(0,1)) with r_c the distance of each cell
    centre from ``centre`` (default: the middle of the box); S = S_amp N(0,1);
    every face velocity N(0,1), then zero on wall sides.  Draw order: rho
    noise, S noise, u (all nx+1 faces), v, w.
    """
    if isinstance(n, int):
        n = (n, n, n)
    nx, ny, nz = (int(a) for a in n)
    if dx is None:
        dx = 1.0 / nx
    outflow = tuple(bool(o) for o in outflow)
    rng = np.random.default_rng(seed)
    ext = np.array([nx, ny, nz], dtype=np.float64) * dx
    c = 0.5 * ext if centre is None else np.asarray(centre, dtype=np.float64)
    dr = dr_per_dx * dx
    rmax = float(np.sqrt(np.sum(np.maximum(c, ext - c) ** 2)))
    nr = int(np.ceil(rmax / dr)) + 2
    rr = (np.arange(nr, dtype=np.float64) + 0.5) * dr
    prof = np.exp(-rr / Hr)
    x, y, z = domain_centres((nx, ny, nz), dx)
    rc = np.sqrt((z[:, None, None] - c[2]) ** 2 + (y[None, :, None] - c[1]) ** 2 + (x[None, None, :] - c[0]) ** 2)
    rho = np.exp(-rc / Hr) * (1.0 + rho_noise * rng.standard_normal((nz, ny, nx)))
    S = S_amp * rng.standard_normal((nz, ny, nx))
    u = rng.standard_normal((nz, ny, nx + 1))
    v = rng.standard_normal((nz, ny + 1, nx))
    w = rng.standard_normal((nz + 1, ny, nx))
    for q in range(6):
        if outflow[q]:
            continue
        d, hi = divmod(q, 2)
        if d == 0:
            u[:, :, -1 if hi else 0] = 0.0
        elif d == 1:
            v[:, -1 if hi else 0, :] = 0.0
        else:
            w[-1 if hi else 0] = 0.0
    return Problem(n=(nx, ny, nz), dx=float(dx), periodic=(False, False, False), rho=rho,
                   beta0_cc=None, beta0_edge=None, S=np.ascontiguousarray(S), u=u, v=v, w=w,
                   rtol=rtol, max_cycles=max_cycles, seed=seed, H=Hr, outflow=outflow,
                   beta0_r=prof, dr_base=float(dr), centre=tuple(float(a) for a in c))


@dataclasses.dataclass
class NodalProblem:
    """One nodal (cell-velocity) projection problem: cell-centred rho, S and
    velocity components uc, vc, wc, all (nz, ny, nx); beta0 at the layer
    centres (nz,).  phi lives on the nodes."""
    n: tuple
    dx: float
    periodic: tuple
    rho: np.ndarray
    beta0_cc: np.ndarray
    S: np.ndarray
    uc: np.ndarray
    vc: np.ndarray
    wc: np.ndarray
    rtol: float = 1e-10
    max_cycles: int = 100
    pre_sweeps: int = 2
    post_sweeps: int = 2
    seed: int = 0
    H: float = 0.3

    def copy(self) -> "NodalProblem":
        out = dataclasses.replace(self)
        for name in ("rho", "beta0_cc", "S", "uc", "vc", "wc"):
            setattr(out, name, getattr(self, name).copy())
        return out


def make_nodal_problem(n, *, H=0.3, rho_noise=0.01, S_amp=0.1, seed=0, dx=None, periodic=(True, True, False),
                       rtol=1e-10, max_cycles=100, vel_scale=1.0) -> NodalProblem:
    """Draw one seeded nodal-projection problem: beta0 = exp(-z/H) at the
    layer centres, rho = beta0 (1 + rho_noise N(0,1)), S = S_amp N(0,1) with
    its beta0-weighted mean removed, uc, vc, wc ~ vel_scale N(0,1).  Draw
    order: rho noise, S noise, uc, vc, wc."""
    if isinstance(n, int):
        n = (n, n, n)
    nx, ny, nz = (int(a) for a in n)
    if dx is None:
        dx = 1.0 / nx
    periodic = tuple(bool(p) for p in periodic)
    rng = np.random.default_rng(seed)
    b0c, _ = stratified_base_state(nz, dx, H)
    rho = b0c[:, None, None] * (1.0 + rho_noise * rng.standard_normal((nz, ny, nx)))
    S = S_amp * rng.standard_normal((nz, ny, nx))
    wts = np.broadcast_to(b0c[:, None, None], S.shape)
    S -= float(np.sum(wts * S) / np.sum(wts))
    uc = vel_scale * rng.standard_normal((nz, ny, nx))
    vc = vel_scale * rng.standard_normal((nz, ny, nx))
    wc = vel_scale * rng.standard_normal((nz, ny, nx))
    return NodalProblem(n=(nx, ny, nz), dx=float(dx), periodic=periodic, rho=rho, beta0_cc=b0c,
                        S=np.ascontiguousarray(S), uc=uc, vc=vc, wc=wc, rtol=rtol, max_cycles=max_cycles,
                        seed=seed, H=H)


# Named workloads (unit box, periodic in x and y, solid walls in z).
def SMALL_BOX(seed=0):
    """32^3, H=0.3, 1% density noise, S = sin(2 pi x) sin(2 pi y) cos(pi z)."""
    return make_problem(32, H=0.3, rho_noise=0.01, S_kind="sine", seed=seed)


def STEEP_256(seed=1, n=256):
    """256^3 steeply stratified box, H=0.1 (density contrast ~2e4), S=0.1 N(0,1)."""
    return make_problem(n, H=0.1, rho_noise=0.01, S_kind="random", seed=seed)


def MIXED_512(seed=2, n=512):
    """512^3 box, H=0.15, 5% density noise, S=0.1 N(0,1); solved in mixed precision."""
    return make_problem(n, H=0.15, rho_noise=0.05, S_kind="random", seed=seed)


def mixed_batch_specs(count=64, seed=3, edges=(32, 48, 64, 96, 128), hmin=0.08, hmax=0.5):
    """(edge, H, problem_seed) for a batch of independent cubic problems."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(count):
        e = int(rng.choice(np.asarray(edges)))
        H = float(rng.uniform(hmin, hmax))
        out.append((e, H, seed * 1000 + p))
    return out


def serving_requests(count, rate, seed=4, edges=(32, 64, 128, 256),
                     weights=(0.4, 0.3, 0.2, 0.1), rtols=(1e-8, 1e-10),
                     hmin=0.08, hmax=0.5):
    """Open-loop Poisson arrivals: list of (t_arrival_s, edge, H, rtol, seed)."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(count):
        t += float(rng.exponential(1.0 / rate))
        e = int(rng.choice(np.asarray(edges), p=np.asarray(weights)))
        H = float(rng.uniform(hmin, hmax))
        tol = float(rtols[int(rng.integers(0, len(rtols)))])
        out.append((t, e, H, tol, seed * 10000 + r))
    return out


def domain_centres(n, dx):
    """Cell-centre coordinates (x, y, z) along each axis."""
    nx, ny, nz = n
    return ((np.arange(nx) + 0.5) * dx, (np.arange(ny) + 0.5) * dx,
            (np.arange(nz) + 0.5) * dx)

