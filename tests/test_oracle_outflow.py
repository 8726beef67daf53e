"""Pins of the oracle's general-boundary path: outflow sides (phi = 0 on the
boundary faces) and a radial (spherical) base state.

Each test checks the oracle against something other than itself: closed-form
eigenpairs of the discrete operator, a sparse direct solve of a system
assembled here from a face list, exact interpolation of linear profiles, the
projected velocity's constraint, second-order convergence to an analytic
solution.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import oracle as O
from paper_1910_12979_amd import inputs as I


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _unit_coeffs(n, periodic, outflow):
    """Full face arrays of b = 1 on every face that carries flux."""
    nx, ny, nz = n
    sides = O.side_codes(periodic, outflow)
    rho = np.ones((nz, ny, nx))
    return sides, O.face_coeffs_gen(n, sides, 1.0 / nx, rho, np.ones(nz), np.ones(nz + 1))


def _mode(n_d, m, kind):
    """1-D eigenvector of the cell-centred second difference and its eigenvalue
    (times h^2): outflow sin(pi m (i+1/2)/n), wall cos(pi m (i+1/2)/n),
    periodic sin(2 pi m (i+1/2)/n)."""
    x = np.arange(n_d) + 0.5
    if kind == "outflow":
        return np.sin(np.pi * m * x / n_d), -4.0 * np.sin(np.pi * m / (2 * n_d)) ** 2
    if kind == "wall":
        return np.cos(np.pi * m * x / n_d), -4.0 * np.sin(np.pi * m / (2 * n_d)) ** 2
    return np.sin(2 * np.pi * m * x / n_d), -4.0 * np.sin(np.pi * m / n_d) ** 2


@pytest.mark.parametrize("kinds,n,modes", [
    (("outflow", "outflow", "outflow"), (12, 10, 8), (1, 3, 2)),
    (("periodic", "wall", "outflow"), (16, 12, 10), (2, 1, 3)),
    (("outflow", "periodic", "wall"), (10, 8, 14), (4, 1, 2)),
])
def test_dirichlet_eigenmodes(kinds, n, modes):
    """phi = product of 1-D modes is an eigenvector of L with eigenvalue the
    sum of the 1-D ones / h^2 (separable operator with b = 1)."""
    periodic = tuple(k == "periodic" for k in kinds)
    outflow = tuple(k == "outflow" for k in kinds for _ in range(2))
    sides, coeffs = _unit_coeffs(n, periodic, outflow)
    h = 1.0 / n[0]
    (ex, lx), (ey, ly), (ez, lz) = (_mode(n[d], modes[d], kinds[d]) for d in range(3))
    phi = ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
    Lphi = O.apply_gen(n, sides, h, coeffs, np.ascontiguousarray(phi))
    lam = (lx + ly + lz) / h**2
    assert rel(Lphi, lam * phi) < 1e-12


def _assemble(n, periodic, outflow, h, rho, beta_face):
    """Sparse -A (SPD) from the face list: interior/periodic faces couple two
    cells with b = beta_face / mean rho; an outflow face adds 2 b to its cell's
    diagonal with b = beta_face / rho_cell (phi = 0 half a cell away)."""
    nx, ny, nz = n
    idx = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []

    def couple(a, b, coef):
        rows.extend([a, b, a, b]); cols.extend([a, b, b, a]); vals.extend([coef, coef, -coef, -coef])

    for d, nd in enumerate((nx, ny, nz)):
        ax = 2 - d                                      # numpy axis of direction d
        for f in range(nd + 1):
            lo, hi = f - 1, f
            if 0 < f < nd or periodic[d]:
                if f == nd:
                    continue                              # periodic: face n is face 0
                lo = lo % nd
                ca = np.take(idx, lo, axis=ax).ravel()
                cb = np.take(idx, hi, axis=ax).ravel()
                ra = np.take(rho, lo, axis=ax).ravel()
                rb = np.take(rho, hi, axis=ax).ravel()
                bf = beta_face(d, f).ravel() / (0.5 * (ra + rb))
                for a, b, c in zip(ca, cb, bf):
                    couple(a, b, c)
            elif outflow[2 * d + (1 if f == nd else 0)]:
                cell = 0 if f == 0 else nd - 1
                cc = np.take(idx, cell, axis=ax).ravel()
                rc = np.take(rho, cell, axis=ax).ravel()
                bf = beta_face(d, f).ravel() / rc
                rows.extend(cc); cols.extend(cc); vals.extend(2.0 * bf)
    N = nx * ny * nz
    return sp.csc_matrix((np.asarray(vals) / h**2, (rows, cols)), shape=(N, N))


def _plane_beta_face(n, b0c, b0e):
    nx, ny, nz = n

    def beta_face(d, f):
        if d == 2:
            return np.full((ny, nx), b0e[f])
        shape = (nz, nx) if d == 1 else (nz, ny)
        return np.broadcast_to(b0c[:, None], shape)
    return beta_face


def _radial_beta_face(n, h, prof, dr, centre):
    nx, ny, nz = n
    rr = (np.arange(len(prof)) + 0.5) * dr
    xc, yc, zc = ((np.arange(m) + 0.5) * h for m in (nx, ny, nz))

    def at(x, y, z):
        r = np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)
        return np.interp(r, rr, prof)          # linear, held constant beyond the ends

    def beta_face(d, f):
        if d == 0:
            return at(f * h, yc[None, :], zc[:, None])            # (nz, ny)
        if d == 1:
            return at(xc[None, :], f * h, zc[:, None])            # (nz, nx)
        return at(xc[None, :], yc[:, None], f * h)                # (ny, nx)
    return beta_face, at(xc[None, None, :], yc[None, :, None], zc[:, None, None])


def _divergence(n, periodic, h, u, v, w, beta_face, beta_cell, S):
    """D(beta0 U) - beta0 S with each face's own beta0 (numpy, face by face)."""
    nx, ny, nz = n
    bu = np.stack([beta_face(0, f) for f in range(nx + 1)], axis=-1) * u
    bv = np.stack([beta_face(1, f) for f in range(ny + 1)], axis=1) * v
    bw = np.stack([beta_face(2, f) for f in range(nz + 1)], axis=0) * w
    if periodic[0]:
        bu[:, :, nx] = bu[:, :, 0]
    if periodic[1]:
        bv[:, ny, :] = bv[:, 0, :]
    if periodic[2]:
        bw[nz] = bw[0]
    div = (bu[:, :, 1:] - bu[:, :, :-1]) + (bv[:, 1:, :] - bv[:, :-1, :]) + (bw[1:] - bw[:-1])
    return div / h - beta_cell * S


CASES = [
    ("plane", (16, 16, 16), (True, True, False), (False, False, False, False, False, True)),
    ("plane", (12, 8, 20), (False, True, False), (True, False, False, False, True, True)),
    ("radial", (16, 16, 16), (False, False, False), (True,) * 6),
    ("radial", (12, 16, 8), (False, False, True), (True, False, False, True, False, False)),
]


def _case_problem(kind, n, periodic, outflow, seed):
    if kind == "plane":
        return I.make_problem(n, H=0.2, rho_noise=0.05, seed=seed, periodic=periodic, outflow=outflow)
    p = I.make_star_problem(n, Hr=0.2, rho_noise=0.05, seed=seed, outflow=outflow)
    if any(periodic):
        # a periodic direction: same fields, periodic duplicate faces refreshed
        p.periodic = periodic
        for d, a in ((0, p.u), (1, p.v), (2, p.w)):
            if periodic[d]:
                sl_last = [slice(None)] * 3
                sl_first = [slice(None)] * 3
                sl_last[2 - d], sl_first[2 - d] = -1, 0
                a[tuple(sl_last)] = a[tuple(sl_first)]
    return p


@pytest.mark.parametrize("kind,n,periodic,outflow", CASES)
def test_general_projection_vs_sparse_direct_solve(kind, n, periodic, outflow):
    """The oracle's exact discrete solution (definition mode) equals a sparse
    LU solve of the system assembled from the face list, with the right-hand
    side computed face by face in numpy; the corrected U then satisfies the
    constraint D(beta0 U) = beta0 S."""
    p = _case_problem(kind, n, periodic, outflow, seed=5)
    h = p.dx
    if kind == "plane":
        beta_face = _plane_beta_face(n, p.beta0_cc, p.beta0_edge)
        beta_cell = p.beta0_cc[:, None, None]
    else:
        beta_face, beta_cell = _radial_beta_face(n, h, p.beta0_r, p.dr_base, p.centre)
    f = _divergence(n, periodic, h, p.u, p.v, p.w, beta_face, beta_cell, p.S)
    A = _assemble(n, periodic, outflow, h, p.rho, beta_face)
    phi_lu = spla.splu(A).solve(-f.ravel()).reshape(f.shape)        # A = -L
    res = O.mac_project(p, mode="definition")
    assert res["status_name"] == "OK"
    assert rel(res["phi"], phi_lu) < 1e-11
    after = _divergence(n, periodic, h, res["u"], res["v"], res["w"], beta_face, beta_cell, p.S)
    assert np.linalg.norm(after) <= 1e-10 * np.linalg.norm(f)


def test_radial_mapping_is_linear_interpolation():
    """A profile linear in r is reproduced exactly inside [r_0, r_last] and
    held at its end values outside; a centred profile gives a field with the
    box's mirror symmetries bit for bit."""
    n, h = (10, 12, 14), 0.1
    dr, nr = 0.2, 5
    rr = (np.arange(nr) + 0.5) * dr
    prof = 2.0 - 1.5 * rr
    centre = (0.5, 0.6, 0.7)
    out = O.map_radial(n, h, prof, dr, centre)
    xc, yc, zc = ((np.arange(m) + 0.5) * h for m in n)
    r = np.sqrt((xc[None, None, :] - 0.5) ** 2 + (yc[None, :, None] - 0.6) ** 2 + (zc[:, None, None] - 0.7) ** 2)
    want = 2.0 - 1.5 * np.clip(r, rr[0], rr[-1])
    assert np.max(np.abs(out - want)) < 1e-14
    assert np.any(r > rr[-1]) and np.any(r < rr[0])      # both clamps are exercised
    sym = O.map_radial((8, 8, 8), 0.125, np.exp(-rr), 0.07, (0.5, 0.5, 0.5))
    assert np.array_equal(sym, sym[::-1]) and np.array_equal(sym, sym[:, ::-1]) and np.array_equal(sym, sym[:, :, ::-1])


def test_outflow_second_order_convergence():
    """L phi = f with f = -3 pi^2 sin(pi x) sin(pi y) sin(pi z) (b = 1) and
    phi = 0 on every side: the discrete solution converges to the analytic
    sin(pi x) sin(pi y) sin(pi z) at second order."""
    errs = []
    for n in (8, 16, 32):
        sides, coeffs = _unit_coeffs((n, n, n), (False,) * 3, (True,) * 6)
        x = (np.arange(n) + 0.5) / n
        exact = np.sin(np.pi * x)[:, None, None] * np.sin(np.pi * x)[None, :, None] * np.sin(np.pi * x)[None, None, :]
        H = O.Hierarchy((n, n, n), (False,) * 3, 1.0 / n, coeffs, outflow=(True,) * 6)
        st, phi, hist = H.solve(np.ascontiguousarray(-3 * np.pi**2 * exact), rtol=1e-12, mode="definition")
        assert st == 0
        errs.append(np.max(np.abs(phi - exact)))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.5 < q < 4.5 for q in ratios), ratios


def test_outflow_accepts_a_net_source_that_walls_reject():
    """With walls the constraint needs sum(beta0 S) = 0; with an outflow side
    any S is admissible (the boundary carries the net flux)."""
    p = I.make_problem(16, H=0.3, seed=3)
    p.S = p.S + 0.5
    assert O.mac_project(p)["status_name"] == "INCOMPATIBLE_RHS"
    q = I.make_problem(16, H=0.3, seed=3, outflow=(False, False, False, False, False, True))
    q.S = q.S + 0.5
    res = O.mac_project(q)
    assert res["status_name"] == "OK" and res["mean_removed"] == 0.0
    assert abs(res["phi"].mean()) > 1e-6          # phi is not shifted to zero mean


def test_general_path_equals_the_wall_path_without_outflow():
    """Side codes periodic/wall and a plane-parallel beta0 through the general
    functions give the same projection as the original path (the two differ
    only in rounding order)."""
    p = I.make_problem((16, 12, 20), H=0.25, seed=8, periodic=(True, False, False))
    a = O._project(p, p.beta0_cc, p.beta0_edge, None, "definition", None, None, None, None)
    b = O._project_gen(p, "definition", None, None, None, None)
    assert a["status_name"] == b["status_name"] == "OK"
    assert rel(b["phi"], a["phi"]) < 1e-12
    for k in ("u", "v", "w"):
        assert rel(b[k], a[k]) < 1e-12


def test_outflow_projection_is_idempotent():
    p = I.make_star_problem(16, Hr=0.2, seed=6)
    r1 = O.mac_project(p, mode="definition")
    q = p.copy()
    q.u, q.v, q.w = r1["u"], r1["v"], r1["w"]
    r2 = O.mac_project(q, mode="definition")
    scale = np.linalg.norm(r1["phi"])
    assert np.linalg.norm(r2["phi"]) <= 1e-10 * scale
    assert rel(r2["u"], r1["u"]) < 1e-12
