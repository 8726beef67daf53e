"""Pins of the oracle's nodal (cell-velocity) projection.

The oracle hand-codes the trilinear-element stencils (weights 1/3, 0, -1/12,
the 1/(4h) divergence, the mean-gradient correction).  These tests assemble
the same discrete operators here from element integrals evaluated by Gauss
quadrature of the trilinear shape functions (nothing taken from the oracle)
and check the oracle against them, against a sparse direct solve, against a
closed-form solution at second order, and for the colour order of its
Gauss-Seidel sweep.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import oracle as O
from paper_1910_12979_amd import inputs as I

G1 = 0.5 - 0.5 / np.sqrt(3.0)
G2 = 0.5 + 0.5 / np.sqrt(3.0)
GP = [(x, y, z) for x in (G1, G2) for y in (G1, G2) for z in (G1, G2)]      # weights 1/8 each
CORNERS = list(itertools.product((0, 1), repeat=3))                         # (a, b, c) = x, y, z offsets


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def _shape(p, a):
    """Trilinear shape function of corner a and its reference gradient at p."""
    l = [(1 - p[d]) if a[d] == 0 else p[d] for d in range(3)]
    dl = [-1.0 if a[d] == 0 else 1.0 for d in range(3)]
    return l[0] * l[1] * l[2], np.array([dl[0] * l[1] * l[2], l[0] * dl[1] * l[2], l[0] * l[1] * dl[2]])


def _element_integrals():
    """K[p, q] = int grad N_p . grad N_q, g[p] = int grad N_p, m[p] = int N_p
    over the unit cube (2-point Gauss rule, exact for these polynomials)."""
    K = np.zeros((8, 8)); g = np.zeros((8, 3)); m = np.zeros(8)
    for pt in GP:
        vals = [_shape(pt, a) for a in CORNERS]
        for p, (Np, dNp) in enumerate(vals):
            g[p] += dNp / 8
            m[p] += Np / 8
            for q, (_, dNq) in enumerate(vals):
                K[p, q] += dNp @ dNq / 8
    return K, g, m


KE, GE, ME = _element_integrals()


def _node_index(n, periodic):
    N = O.node_dims(n, periodic)

    def idx(I, J, K):
        X = [I, J, K]
        for d in range(3):
            if periodic[d]:
                X[d] %= N[d]
        return (X[2] * N[1] + X[1]) * N[0] + X[0]
    return N, idx


def assemble(n, periodic, h, sig):
    """-A (A = the nodal operator) as a sparse matrix: h^-3 sum_e sigma_e h K_e."""
    nx, ny, nz = n
    N, idx = _node_index(n, periodic)
    rows, cols, vals = [], [], []
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        nodes = [idx(i + a[0], j + a[1], k + a[2]) for a in CORNERS]
        for p in range(8):
            for q in range(8):
                rows.append(nodes[p]); cols.append(nodes[q]); vals.append(sig[k, j, i] * KE[p, q] / h**2)
    M = int(np.prod(N))
    return sp.csc_matrix((vals, (rows, cols)), shape=(M, M))


def rhs_fe(n, periodic, h, b0c, uc, vc, wc, S):
    """f_n = -h^-3 int beta0 U . grad N_n - h^-3 int beta0 S N_n."""
    nx, ny, nz = n
    N, idx = _node_index(n, periodic)
    f = np.zeros(int(np.prod(N)))
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        U = np.array([uc[k, j, i], vc[k, j, i], wc[k, j, i]]) * b0c[k]
        for p, a in enumerate(CORNERS):
            n_ = idx(i + a[0], j + a[1], k + a[2])
            f[n_] += -(GE[p] @ U) / h - b0c[k] * S[k, j, i] * ME[p]
    return f.reshape(N[::-1])


def grad_fe(n, periodic, h, phi):
    """Mean gradient of the trilinear interpolant of phi over every cell."""
    nx, ny, nz = n
    N, idx = _node_index(n, periodic)
    ph = phi.ravel()
    G = np.zeros((3, nz, ny, nx))
    for k, j, i in itertools.product(range(nz), range(ny), range(nx)):
        for p, a in enumerate(CORNERS):
            G[:, k, j, i] += ph[idx(i + a[0], j + a[1], k + a[2])] * GE[p] / h
    return G


SHAPES = [((6, 4, 5), (False, False, False)), ((4, 6, 4), (True, True, False)), ((4, 4, 6), (True, False, True))]


@pytest.mark.parametrize("n,per", SHAPES)
def test_operator_equals_assembled_trilinear_stiffness(n, per):
    rng = np.random.default_rng(1)
    nx, ny, nz = n
    sig = np.exp(rng.standard_normal((nz, ny, nx)))
    N = O.node_dims(n, per)
    phi = rng.standard_normal(N[::-1])
    h = 0.3
    A = assemble(n, per, h, sig)
    want = -(A @ phi.ravel()).reshape(phi.shape)
    assert rel(O.nodal_apply(n, per, h, sig, phi), want) < 1e-13


@pytest.mark.parametrize("n,per", SHAPES)
def test_rhs_and_correction_equal_element_integrals(n, per):
    p = I.make_nodal_problem(n, seed=3, periodic=per, H=0.4)
    f = O.nodal_rhs(n, per, p.dx, p.beta0_cc, p.uc, p.vc, p.wc, p.S)
    assert rel(f, rhs_fe(n, per, p.dx, p.beta0_cc, p.uc, p.vc, p.wc, p.S)) < 1e-13
    rng = np.random.default_rng(4)
    phi = rng.standard_normal(O.node_dims(n, per)[::-1])
    u, v, w = O.nodal_correct(n, per, p.dx, p.rho, phi, p.uc, p.vc, p.wc)
    G = grad_fe(n, per, p.dx, phi)
    for got, u0, g in zip((u, v, w), (p.uc, p.vc, p.wc), G):
        assert rel(got, u0 - g / p.rho) < 1e-13


@pytest.mark.parametrize("n,per", [((8, 8, 8), (True, True, False)), ((16, 8, 12), (False, False, False)),
                                   ((8, 16, 8), (True, False, True))])
def test_nodal_projection_vs_sparse_direct_solve(n, per):
    """The oracle's exact discrete phi equals the bordered sparse LU solution
    of -A phi = -f, sum phi = 0 (A assembled from element integrals)."""
    p = I.make_nodal_problem(n, seed=5, periodic=per, H=0.25, rho_noise=0.1)
    res = O.nodal_project(p, mode="definition")
    assert res["status_name"] == "OK"
    sig = p.beta0_cc[:, None, None] / p.rho
    A = assemble(n, per, p.dx, sig)
    f = rhs_fe(n, per, p.dx, p.beta0_cc, p.uc, p.vc, p.wc, p.S).ravel()
    assert abs(f.sum()) < 1e-10 * np.abs(f).sum()
    f = f - f.mean()
    M = f.size
    ones = sp.csc_matrix(np.ones((M, 1)))
    B = sp.bmat([[A, ones], [ones.T, None]], format="csc")
    x = spla.splu(B).solve(np.concatenate([-f, [0.0]]))[:M]
    assert rel(res["phi"].ravel(), x) < 1e-11
    G = grad_fe(n, per, p.dx, res["phi"])
    for got, u0, g in zip((res["u"], res["v"], res["w"]), (p.uc, p.vc, p.wc), G):
        assert rel(got, u0 - g / p.rho) < 1e-12


def test_second_order_convergence_to_a_closed_form_solution():
    """sigma = 1, periodic x, y and walls in z: phi = cos(2 pi x) cos(2 pi y)
    cos(pi z) solves div grad phi = -9 pi^2 phi with zero normal gradient at
    the walls; the nodal solution with f = that value at the nodes converges
    at second order."""
    errs = []
    for n in (8, 16, 32):
        per = (True, True, False)
        N = O.node_dims((n, n, n), per)
        x = np.arange(N[0]) / n
        z = np.arange(N[2]) / n
        ex = (np.cos(np.pi * z)[:, None, None] * np.cos(2 * np.pi * x)[None, :, None]
              * np.cos(2 * np.pi * x)[None, None, :])
        H = O.NodalHierarchy((n, n, n), per, 1.0 / n, np.ones((n, n, n)))
        f = -9 * np.pi**2 * ex
        # the wall nodes carry half a control volume: the load of f there is f/2
        f[0] *= 0.5
        f[-1] *= 0.5
        st, phi, _ = H.solve(f - f.mean(), rtol=1e-12, mode="definition")
        assert st == 0
        errs.append(np.max(np.abs((phi - phi.mean()) - (ex - ex.mean()))))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(3.5 < q < 4.5 for q in ratios), (errs, ratios)


def test_gauss_seidel_colour_order():
    """One sweep visits the colours (J mod 2) + 2 (K mod 2) in order 0..3: afterwards
    the residual vanishes on the last colour (its neighbours all belong to
    other colours, updated before it) and not on the first; and no two
    coupled nodes share a colour (checked on the assembled operator)."""
    n, per = (8, 6, 10), (True, True, False)
    rng = np.random.default_rng(6)
    sig = np.exp(0.3 * rng.standard_normal(n[::-1]))
    N = O.node_dims(n, per)
    phi = rng.standard_normal(N[::-1])
    f = rng.standard_normal(N[::-1])
    out = O.nodal_gs(n, per, 0.1, sig, phi, f)
    r = f - O.nodal_apply(n, per, 0.1, sig, out)
    K, J, Ii = np.meshgrid(np.arange(N[2]), np.arange(N[1]), np.arange(N[0]), indexing="ij")
    cls = (J & 1) + 2 * (K & 1)
    assert np.max(np.abs(r[cls == 3])) < 1e-10 * np.max(np.abs(f))
    assert np.max(np.abs(r[cls == 0])) > 1e-3
    A = assemble(n, per, 0.1, sig).tocoo()
    c = cls.ravel()
    # couplings (edge neighbours have weight 0, up to the quadrature's rounding)
    off = (A.row != A.col) & (np.abs(A.data) > 1e-12 * np.abs(A.data).max())
    assert np.all(c[A.row[off]] != c[A.col[off]])


def test_restriction_is_an_eighth_of_the_prolongation_transpose():
    n, per = (8, 4, 8), (True, False, False)
    sig = np.ones(n[::-1])
    H = O.NodalHierarchy(n, per, 0.125, sig)
    (Nf, _), (Nc, _) = H.dims(0), H.dims(1)
    rng = np.random.default_rng(7)
    r = rng.standard_normal(Nf[::-1])
    e = rng.standard_normal(Nc[::-1])
    # R r: set phi = 0 and f = r on level 0, so the level-0 residual is r
    H.set(0, "phi", np.zeros(Nf[::-1])); H.set(0, "f", r)
    H.resid_restrict(0)
    Rr = H.get(1, "f")
    # P e: prolongation adds P e to a zero phi
    H.set(0, "phi", np.zeros(Nf[::-1])); H.set(1, "phi", e)
    H.prolong(0)
    Pe = H.get(0, "phi")
    assert abs(8 * np.sum(Rr * e) - np.sum(r * Pe)) < 1e-12 * np.sum(np.abs(r * Pe))
    # constants are prolongated exactly
    H.set(0, "phi", np.zeros(Nf[::-1])); H.set(1, "phi", np.full(Nc[::-1], 2.5))
    H.prolong(0)
    assert np.allclose(H.get(0, "phi"), 2.5, rtol=0, atol=1e-15)


def test_nodal_compatibility_and_errors():
    p = I.make_nodal_problem(8, seed=9)
    q = p.copy(); q.S = q.S + 0.3
    assert O.nodal_project(q)["status_name"] == "INCOMPATIBLE_RHS"
    q = p.copy(); q.rho[1, 1, 1] = -1.0
    assert O.nodal_project(q)["status_name"] == "INVALID_ARG"
    q = p.copy(); q.uc[0, 0, 0] = np.nan
    assert O.nodal_project(q)["status_name"] == "NONFINITE"
