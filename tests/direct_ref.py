"""Independent references used to pin the oracle (test helper, CPU only).

Nothing here calls the oracle's stencil code.  The operator is assembled as a
sparse matrix from an explicit list of faces (each face couples its two
cells), the divergence and gradient are written per face, and solutions come
from library direct solvers (dense LU, sparse LU) or from closed forms.  A
mistake in the oracle's stencil, coefficient, sign or indexing therefore shows
up as a disagreement with these.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def cell_index(n):
    nx, ny, nz = n
    return np.arange(nx * ny * nz).reshape(nz, ny, nx)


def faces(n, periodic):
    """Per axis: list of (face_key, left_cell_index, right_cell_index).

    face_key is the index tuple (k, j, i) of the face in the full face array of
    that axis.  Wall faces are not listed (they carry no flux).
    """
    nx, ny, nz = n
    C = cell_index(n)
    out = {0: [], 1: [], 2: []}
    for k in range(nz):
        for j in range(ny):
            for i in range(nx + 1):
                if i == 0 or i == nx:
                    if not periodic[0] or i == nx:
                        continue          # wall, or the periodic duplicate of face 0
                    out[0].append(((k, j, 0), C[k, j, nx - 1], C[k, j, 0]))
                else:
                    out[0].append(((k, j, i), C[k, j, i - 1], C[k, j, i]))
    for k in range(nz):
        for j in range(ny + 1):
            for i in range(nx):
                if j == 0 or j == ny:
                    if not periodic[1] or j == ny:
                        continue
                    out[1].append(((k, 0, i), C[k, ny - 1, i], C[k, 0, i]))
                else:
                    out[1].append(((k, j, i), C[k, j - 1, i], C[k, j, i]))
    for k in range(nz + 1):
        for j in range(ny):
            for i in range(nx):
                if k == 0 or k == nz:
                    if not periodic[2] or k == nz:
                        continue
                    out[2].append(((0, j, i), C[nz - 1, j, i], C[0, j, i]))
                else:
                    out[2].append(((k, j, i), C[k - 1, j, i], C[k, j, i]))
    return out


def face_beta0(axis, key, b0c, b0e):
    k = key[0]
    return b0c[k] if axis < 2 else b0e[k]


def face_coefficient(axis, key, left, right, rho_flat, b0c, b0e):
    """beta0 at the face over the mean density of its two cells."""
    return face_beta0(axis, key, b0c, b0e) / (0.5 * (rho_flat[left] + rho_flat[right]))


def assemble(n, periodic, h, rho, b0c, b0e):
    """Sparse matrix of L phi = h^-2 sum_f b_f (phi_nb - phi_c), from the face list."""
    N = int(np.prod(n))
    rf = rho.ravel()
    rows, cols, vals = [], [], []
    for axis, lst in faces(n, periodic).items():
        for key, L, R in lst:
            b = face_coefficient(axis, key, L, R, rf, b0c, b0e) / (h * h)
            rows += [L, L, R, R]
            cols += [R, L, L, R]
            vals += [b, -b, b, -b]
    return sp.csr_matrix((vals, (rows, cols)), shape=(N, N))


def divergence(n, periodic, h, b0c, b0e, u, v, w):
    """MAC divergence of beta0 U, accumulated face by face (wall faces included)."""
    nx, ny, nz = n
    C = cell_index(n)
    div = np.zeros(nx * ny * nz)
    arrays = (u, v, w)
    for axis in range(3):
        U = arrays[axis]
        for key in np.ndindex(U.shape):
            k, j, i = key
            idx = (i, j, k)[axis]
            nmax = (nx, ny, nz)[axis]
            if periodic[axis] and idx == nmax:
                continue                  # duplicate of face 0
            flux = face_beta0(axis, key, b0c, b0e) * U[key] / h
            lo = list(key)
            hi = list(key)
            # the cell on the low side of face idx is idx-1, the high side is idx
            lo[2 - axis] = idx - 1
            if idx - 1 >= 0:
                div[C[tuple(lo)]] += flux
            elif periodic[axis]:
                lo[2 - axis] = nmax - 1
                div[C[tuple(lo)]] += flux
            if idx < nmax:
                div[C[tuple(hi)]] -= flux
    return div.reshape(nz, ny, nx)


def gradient_update(n, periodic, h, rho, b0c, b0e, phi, u, v, w):
    """U - (1/rho_f) grad phi on every non-wall face, with 1/rho_f = b_f / beta0_f."""
    u, v, w = u.copy(), v.copy(), w.copy()
    arrays = [u, v, w]
    rf, pf = rho.ravel(), phi.ravel()
    for axis, lst in faces(n, periodic).items():
        U = arrays[axis]
        for key, L, R in lst:
            b = face_coefficient(axis, key, L, R, rf, b0c, b0e)
            beta = face_beta0(axis, key, b0c, b0e)
            U[key] -= (b / beta) * (pf[R] - pf[L]) / h
    nx, ny, nz = n
    if periodic[0]:
        u[:, :, nx] = u[:, :, 0]
    if periodic[1]:
        v[:, ny, :] = v[:, 0, :]
    if periodic[2]:
        w[nz] = w[0]
    return u, v, w


def solve_bordered_dense(A, f):
    """[A 1; 1^T 0][phi; lam] = [f; 0] by dense LU: the zero-mean solution."""
    A = A.toarray() if sp.issparse(A) else A
    N = A.shape[0]
    M = np.zeros((N + 1, N + 1))
    M[:N, :N] = A
    M[:N, N] = 1.0
    M[N, :N] = 1.0
    rhs = np.concatenate([f.ravel(), [0.0]])
    x = np.linalg.solve(M, rhs)
    return x[:N]


def solve_pinned_sparse(A, f):
    """Sparse LU with phi_0 fixed at 0 (drops row/column 0), then mean removal."""
    A = sp.csc_matrix(A)
    fr = f.ravel()
    lu = spla.splu(A[1:, 1:].tocsc())
    x = np.zeros_like(fr)
    x[1:] = lu.solve(fr[1:])
    return x - x.mean()


def column_solve_1d(h, bz_faces, f_col):
    """Exact solution of the 1-D wall-bounded problem by flux integration.

    (1/h^2)[b_{k+1}(phi_{k+1}-phi_k) - b_k(phi_k-phi_{k-1})] = f_k with
    b_0 = b_nz = 0: the flux through face k+1 is h^2 sum_{m<=k} f_m, and
    phi_k - phi_{k-1} = flux_k / b_k.  Returns the zero-mean solution.
    """
    nz = len(f_col)
    flux = np.zeros(nz + 1)
    for k in range(nz):
        flux[k + 1] = flux[k] + h * h * f_col[k]
    phi = np.zeros(nz)
    for k in range(1, nz):
        phi[k] = phi[k - 1] + flux[k] / bz_faces[k]
    return phi - phi.mean()
