/*
 * FP64 CPU oracle for the variable-coefficient MAC projection.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference against
 * which the HIP path is checked.  It shares no code, header, table or helper
 * with the HIP library; only tests, the smoke check and the benchmark's CPU
 * baseline may load it.
 *
 * What it computes (arXiv:1910.12979, Sec. 2 and Sec. 3):
 *   the divergence constraint  div(beta0 U) = beta0 S   (Sec. 2, constraint
 *   equation, with the d p0/dt term folded into the caller's S, or given per
 *   layer as w0 = dp0/dt / (Gamma1 p0): orc_rhs_w0, orc_mac_project_w0) is
 *   enforced by a projection: solve
 *       div((beta0/rho) grad phi) = div(beta0 U) - beta0 S          (1)
 *   by geometric multigrid (Sec. 3: multigrid solvers for the projections) and
 *   correct U -= (1/rho) grad phi on every non-wall face, which is the
 *   gradient form (beta0/rho) grad(.) of the momentum equation (Sec. 2) with
 *   the potential absorbing beta0.
 *
 * Discretisation (the paper gives none; these readings are stated once here):
 *   cell-centred finite volume on a uniform grid of spacing h, phi/rho/S at
 *   cell centres, U on faces (MAC).  Face coefficient
 *       b = beta0_face / (0.5*(rho_left + rho_right)),
 *   beta0_face = beta0 at the cell centre of the layer for x/y faces and the
 *   caller's z-face beta0 for z faces.  Solid-wall faces carry no flux.  In a
 *   periodic direction face n is face 0.
 *       (L phi)_c = h^-2 sum_faces b_f (phi_nb - phi_c),  L phi = f.
 *   The solution is unique up to a constant; the oracle returns the zero-mean
 *   one.
 *
 * Outflow boundaries (the *_gen functions): a side may instead carry
 *   phi = 0 on its faces (Dirichlet).  The boundary face's coefficient is
 *   beta0_face / rho of the one adjacent cell, and the face enters the operator
 *   through the ghost value -phi_c (phi is zero half a cell away), i.e. as
 *   b (-phi_c - phi_c).  With any outflow side the operator is non-singular:
 *   no compatibility condition, no mean removal of f or phi, and the coarsest
 *   level is solved with -A itself.  Outflow faces are corrected like interior
 *   faces, U -= (phi_c - phi_ghost)/h / rho_face with rho_face = rho of the
 *   adjacent cell (interior faces: the mean of the two cells).
 *
 * beta0 on a radial profile (the *_gen functions, spherical base state):
 *   the profile gives beta0 at radii r_m = (m + 1/2) dr, m = 0..nr-1, about a
 *   centre c; beta0 at any point x is the linear interpolation in r = |x - c|
 *   between the two nearest profile radii, held constant below r_0 and above
 *   r_{nr-1}.  Face coefficients use beta0 at the face centre, beta0 S uses it
 *   at the cell centre, and the divergence weights every face velocity with
 *   its own face value:
 *       f = ((bxh uh - bxl ul) + (byh vh - byl vl) + (bzh wh - bzl wl)) / h
 *           - beta0_c S.
 *
 * beta0 from the base-state pressure (Sec. 2, definition of beta0):
 *   orc_beta0_from_p0 integrates (1/(Gamma1 p0)) dp0/dr layer by layer with
 *   Gamma1 constant in a layer, exactly ln(p0(b)/p0(a))/Gamma1 over [a, b].
 *
 * Multigrid (V-cycle, as the algorithm is stated for this reference):
 *   nu1 red-black Gauss-Seidel sweeps (red = (i+j+k) even, updated first),
 *   residual, 8-cell-average restriction, coarse correction started from zero,
 *   piecewise-constant prolongation, nu2 sweeps.  Coarse face coefficient = the
 *   mean of the 4 coincident fine faces, coarse spacing 2h.  Coarsening goes on
 *   while every dimension is even and the level has more than 64 cells; the
 *   coarsest level (at most 512 cells) is solved exactly: f <- f - mean(f),
 *   dense Cholesky of (-A + c 1 1^T) with c the mean diagonal of -A, then
 *   x <- x - mean(x).
 *
 * Built with gcc, no fast-math, no FMA contraction.  OpenMP is used only on
 * loops whose iterations are independent (one colour of a sweep, cell-wise
 * maps); every reduction is a serial loop in index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_ERR_INVALID (-1)
#define ORC_ERR_SIZE (-2)
#define ORC_ERR_INCOMPATIBLE (-3)
#define ORC_ERR_NOT_CONVERGED (-4)
#define ORC_ERR_NONFINITE (-5)
#define ORC_ERR_OOM (-6)

#define MAXLEV 32
#define COARSE_MAX 512

typedef struct {
    int nx, ny, nz;
    int px, py, pz;      /* 1 = periodic, 0 = solid walls on both sides */
    int dir[6];          /* outflow (phi = 0) sides: x low, x high, y low, y high, z low, z high */
    double h;
    double *bx, *by, *bz; /* full face arrays: (nz,ny,nx+1), (nz,ny+1,nx), (nz+1,ny,nx) */
    double *phi, *f, *r;  /* cell arrays (nz,ny,nx) */
} olev;

typedef struct {
    int nlev;
    olev lev[MAXLEV];
    double *chol;        /* coarsest-level Cholesky factor (lower, row-major) */
    int ncoarse;
    int singular;        /* no outflow side: solution defined up to a constant */
} omg;

static inline size_t CI(const olev* L, int i, int j, int k) {
    return ((size_t)k * L->ny + j) * L->nx + i;
}
static inline size_t FXI(const olev* L, int i, int j, int k) {
    return ((size_t)k * L->ny + j) * (L->nx + 1) + i;
}
static inline size_t FYI(const olev* L, int i, int j, int k) {
    return ((size_t)k * (L->ny + 1) + j) * L->nx + i;
}
static inline size_t FZI(const olev* L, int i, int j, int k) {
    return ((size_t)k * L->ny + j) * L->nx + i;
}
static inline size_t ncell(const olev* L) { return (size_t)L->nx * L->ny * L->nz; }

/*
 * The faces of cell (i,j,k) that carry flux, in the fixed order x-low, x-high,
 * y-low, y-high, z-low, z-high: coefficient b[], neighbour cell index nb[] and
 * ghost[] = 1 for an outflow boundary face (its neighbour value is -phi_c).
 * A wall face is left out.  Returns the number of faces listed.
 */
static int cell_faces(const olev* L, int i, int j, int k, double b[6], size_t nb[6], int ghost[6]) {
    int m = 0;
    size_t c = CI(L, i, j, k);
#define FACE(bv, nbv, g) do { b[m] = (bv); nb[m] = (nbv); ghost[m] = (g); ++m; } while (0)
    /* x-low: face i */
    if (i > 0) FACE(L->bx[FXI(L, i, j, k)], CI(L, i - 1, j, k), 0);
    else if (L->px) FACE(L->bx[FXI(L, 0, j, k)], CI(L, L->nx - 1, j, k), 0);
    else if (L->dir[0]) FACE(L->bx[FXI(L, 0, j, k)], c, 1);
    /* x-high: face i+1 */
    if (i < L->nx - 1) FACE(L->bx[FXI(L, i + 1, j, k)], CI(L, i + 1, j, k), 0);
    else if (L->px) FACE(L->bx[FXI(L, L->nx, j, k)], CI(L, 0, j, k), 0);
    else if (L->dir[1]) FACE(L->bx[FXI(L, L->nx, j, k)], c, 1);
    /* y-low */
    if (j > 0) FACE(L->by[FYI(L, i, j, k)], CI(L, i, j - 1, k), 0);
    else if (L->py) FACE(L->by[FYI(L, i, 0, k)], CI(L, i, L->ny - 1, k), 0);
    else if (L->dir[2]) FACE(L->by[FYI(L, i, 0, k)], c, 1);
    /* y-high */
    if (j < L->ny - 1) FACE(L->by[FYI(L, i, j + 1, k)], CI(L, i, j + 1, k), 0);
    else if (L->py) FACE(L->by[FYI(L, i, L->ny, k)], CI(L, i, 0, k), 0);
    else if (L->dir[3]) FACE(L->by[FYI(L, i, L->ny, k)], c, 1);
    /* z-low */
    if (k > 0) FACE(L->bz[FZI(L, i, j, k)], CI(L, i, j, k - 1), 0);
    else if (L->pz) FACE(L->bz[FZI(L, i, j, 0)], CI(L, i, j, L->nz - 1), 0);
    else if (L->dir[4]) FACE(L->bz[FZI(L, i, j, 0)], c, 1);
    /* z-high */
    if (k < L->nz - 1) FACE(L->bz[FZI(L, i, j, k + 1)], CI(L, i, j, k + 1), 0);
    else if (L->pz) FACE(L->bz[FZI(L, i, j, L->nz)], CI(L, i, j, 0), 0);
    else if (L->dir[5]) FACE(L->bz[FZI(L, i, j, L->nz)], c, 1);
#undef FACE
    return m;
}

/* (L phi) at one cell. */
static double apply_cell(const olev* L, const double* phi, int i, int j, int k) {
    double b[6];
    size_t nb[6];
    int ghost[6];
    int m = cell_faces(L, i, j, k, b, nb, ghost);
    double pc = phi[CI(L, i, j, k)];
    double s = 0.0;
    for (int q = 0; q < m; ++q) {
        double pn = ghost[q] ? -pc : phi[nb[q]];
        s += b[q] * (pn - pc);
    }
    return s / (L->h * L->h);
}

static void wrap_level(olev* L, int nx, int ny, int nz, int px, int py, int pz, double h,
                       double* bx, double* by, double* bz) {
    memset(L, 0, sizeof(*L));
    L->nx = nx; L->ny = ny; L->nz = nz;
    L->px = px; L->py = py; L->pz = pz;
    L->h = h;
    L->bx = bx; L->by = by; L->bz = bz;
}

/* Side codes of the *_gen functions, per side (x low, x high, y low, y high,
 * z low, z high): 0 periodic, 1 solid wall, 2 outflow.  A periodic direction
 * has code 0 on both sides. */
#define SIDE_PERIODIC 0
#define SIDE_WALL 1
#define SIDE_OUTFLOW 2

static int sides_valid(const int* side) {
    for (int d = 0; d < 3; ++d) {
        int lo = side[2 * d], hi = side[2 * d + 1];
        if (lo < 0 || lo > 2 || hi < 0 || hi > 2) return 0;
        if ((lo == SIDE_PERIODIC) != (hi == SIDE_PERIODIC)) return 0;
    }
    return 1;
}

static void wrap_level_gen(olev* L, int nx, int ny, int nz, const int* side, double h,
                           double* bx, double* by, double* bz) {
    wrap_level(L, nx, ny, nz, side[0] == SIDE_PERIODIC, side[2] == SIDE_PERIODIC, side[4] == SIDE_PERIODIC, h,
               bx, by, bz);
    for (int q = 0; q < 6; ++q) L->dir[q] = side[q] == SIDE_OUTFLOW;
}

static int any_outflow(const int* side) {
    for (int q = 0; q < 6; ++q)
        if (side[q] == SIDE_OUTFLOW) return 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Face coefficients b = beta0_face / (0.5 (rho_L + rho_R)).           */
/* ------------------------------------------------------------------ */
int orc_face_coeffs(int nx, int ny, int nz, int px, int py, int pz,
                    const double* rho, const double* b0c, const double* b0e,
                    double* bx, double* by, double* bz) {
    olev L;
    wrap_level(&L, nx, ny, nz, px, py, pz, 1.0, bx, by, bz);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double b;
                if (i == 0 || i == nx) {
                    b = px ? b0c[k] / (0.5 * (rho[CI(&L, nx - 1, j, k)] + rho[CI(&L, 0, j, k)])) : 0.0;
                } else {
                    b = b0c[k] / (0.5 * (rho[CI(&L, i - 1, j, k)] + rho[CI(&L, i, j, k)]));
                }
                bx[FXI(&L, i, j, k)] = b;
            }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double b;
                if (j == 0 || j == ny) {
                    b = py ? b0c[k] / (0.5 * (rho[CI(&L, i, ny - 1, k)] + rho[CI(&L, i, 0, k)])) : 0.0;
                } else {
                    b = b0c[k] / (0.5 * (rho[CI(&L, i, j - 1, k)] + rho[CI(&L, i, j, k)]));
                }
                by[FYI(&L, i, j, k)] = b;
            }
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double b;
                if (k == 0 || k == nz) {
                    /* periodic: face nz is face 0 and uses face 0's beta0 */
                    b = pz ? b0e[0] / (0.5 * (rho[CI(&L, i, j, nz - 1)] + rho[CI(&L, i, j, 0)])) : 0.0;
                } else {
                    b = b0e[k] / (0.5 * (rho[CI(&L, i, j, k - 1)] + rho[CI(&L, i, j, k)]));
                }
                bz[FZI(&L, i, j, k)] = b;
            }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Right-hand side f = D(beta0 U) - beta0 S  (MAC divergence).          */
/* In a periodic direction the high face of the last cell is face 0.  */
/* ------------------------------------------------------------------ */
/* Full right-hand side of the constraint (Sec. 2, constraint equation):
 *   f = D(beta0 U) - beta0 (S - w0[k]),  w0[k] = (1/(Gamma1 p0)) dp0/dt of
 * layer k (orc_dp0_term).  w0 == NULL: the dp0/dt term is folded into S. */
int orc_rhs_w0(int nx, int ny, int nz, int px, int py, int pz, double h,
               const double* b0c, const double* b0e,
               const double* u, const double* v, const double* w, const double* S, const double* w0,
               double* f) {
    olev L;
    wrap_level(&L, nx, ny, nz, px, py, pz, h, NULL, NULL, NULL);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double ul = u[FXI(&L, i, j, k)];
                double uh = (i == nx - 1 && px) ? u[FXI(&L, 0, j, k)] : u[FXI(&L, i + 1, j, k)];
                double vl = v[FYI(&L, i, j, k)];
                double vh = (j == ny - 1 && py) ? v[FYI(&L, i, 0, k)] : v[FYI(&L, i, j + 1, k)];
                double wl = w[FZI(&L, i, j, k)];
                double bl = b0e[k];
                double wh, bh;
                if (k == nz - 1 && pz) { wh = w[FZI(&L, i, j, 0)]; bh = b0e[0]; }
                else { wh = w[FZI(&L, i, j, k + 1)]; bh = b0e[k + 1]; }
                if (k == 0 && pz) bl = b0e[0];
                double div = (b0c[k] * (uh - ul) + b0c[k] * (vh - vl) + (bh * wh - bl * wl)) / h;
                double src = S[CI(&L, i, j, k)];
                if (w0) src = src - w0[k];
                f[CI(&L, i, j, k)] = div - b0c[k] * src;
            }
    return ORC_OK;
}

int orc_rhs(int nx, int ny, int nz, int px, int py, int pz, double h,
            const double* b0c, const double* b0e,
            const double* u, const double* v, const double* w, const double* S, double* f) {
    return orc_rhs_w0(nx, ny, nz, px, py, pz, h, b0c, b0e, u, v, w, S, NULL, f);
}

/* ------------------------------------------------------------------ */
/* Base state (Sec. 2, definition of beta0): with r the height z,      */
/*   beta0(r) = rho0(0) exp( int_0^r (1/(Gamma1 p0)) dp0/dr' dr' ).    */
/* Reading: Gamma1 is constant within a layer, so over any part [a,b]  */
/* of layer k the integral is exactly ln(p0(b)/p0(a)) / Gamma1[k].     */
/* p0e: p0 at the nz+1 z faces (face 0 is r = 0), p0c: at the layer    */
/* centres.  beta0 at faces and centres follows by summing the layer   */
/* integrals from the bottom.                                          */
/* ------------------------------------------------------------------ */
int orc_beta0_from_p0(int nz, double rho0_base, const double* p0e, const double* p0c, const double* g1c,
                      double* b0c, double* b0e) {
    if (nz < 1 || !(rho0_base > 0.0)) return ORC_ERR_INVALID;
    for (int k = 0; k <= nz; ++k)
        if (!(p0e[k] > 0.0) || !isfinite(p0e[k])) return ORC_ERR_INVALID;
    for (int k = 0; k < nz; ++k)
        if (!(p0c[k] > 0.0) || !(g1c[k] > 0.0) || !isfinite(p0c[k]) || !isfinite(g1c[k])) return ORC_ERR_INVALID;
    double acc = 0.0;            /* integral from r = 0 to face k */
    for (int k = 0; k < nz; ++k) {
        b0e[k] = rho0_base * exp(acc);
        b0c[k] = rho0_base * exp(acc + log(p0c[k] / p0e[k]) / g1c[k]);
        acc += log(p0e[k + 1] / p0e[k]) / g1c[k];
    }
    b0e[nz] = rho0_base * exp(acc);
    return ORC_OK;
}

/* The dp0/dt term of the constraint per layer: w0[k] = dp0dt[k] / (Gamma1[k] p0[k]). */
int orc_dp0_term(int nz, const double* p0c, const double* g1c, const double* dp0dt, double* w0) {
    for (int k = 0; k < nz; ++k) {
        if (!(p0c[k] > 0.0) || !(g1c[k] > 0.0)) return ORC_ERR_INVALID;
        w0[k] = dp0dt[k] / (g1c[k] * p0c[k]);
    }
    return ORC_OK;
}

/* out = L phi on a single level described by full face arrays. */
void orc_apply(int nx, int ny, int nz, int px, int py, int pz, double h,
               const double* bx, const double* by, const double* bz,
               const double* phi, double* out) {
    olev L;
    wrap_level(&L, nx, ny, nz, px, py, pz, h, (double*)bx, (double*)by, (double*)bz);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) out[CI(&L, i, j, k)] = apply_cell(&L, phi, i, j, k);
}

static void residual_level(const olev* L, const double* phi, const double* f, double* r) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < L->nz; ++k)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) {
                size_t c = CI(L, i, j, k);
                r[c] = f[c] - apply_cell(L, phi, i, j, k);
            }
}

void orc_residual(int nx, int ny, int nz, int px, int py, int pz, double h,
                  const double* bx, const double* by, const double* bz,
                  const double* phi, const double* f, double* r) {
    olev L;
    wrap_level(&L, nx, ny, nz, px, py, pz, h, (double*)bx, (double*)by, (double*)bz);
    residual_level(&L, phi, f, r);
}

/* One red-black Gauss-Seidel sweep: red ((i+j+k) even) cells, then black. */
static void rbgs_level(const olev* L, double* phi, const double* f, int nsweeps) {
    double h2 = L->h * L->h;
    for (int s = 0; s < nsweeps; ++s) {
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
            for (int k = 0; k < L->nz; ++k)
                for (int j = 0; j < L->ny; ++j)
                    for (int i = 0; i < L->nx; ++i) {
                        if (((i + j + k) & 1) != colour) continue;
                        double b[6];
                        size_t nb[6];
                        int ghost[6];
                        int m = cell_faces(L, i, j, k, b, nb, ghost);
                        double num = 0.0, den = 0.0;
                        for (int q = 0; q < m; ++q) {
                            if (ghost[q]) {
                                /* b (-phi - phi): the face moves 2b to the diagonal */
                                den += 2.0 * b[q];
                            } else {
                                num += b[q] * phi[nb[q]];
                                den += b[q];
                            }
                        }
                        size_t c = CI(L, i, j, k);
                        phi[c] = (num - h2 * f[c]) / den;
                    }
        }
    }
}

void orc_rbgs(int nx, int ny, int nz, int px, int py, int pz, double h,
              const double* bx, const double* by, const double* bz,
              double* phi, const double* f, int nsweeps) {
    olev L;
    wrap_level(&L, nx, ny, nz, px, py, pz, h, (double*)bx, (double*)by, (double*)bz);
    rbgs_level(&L, phi, f, nsweeps);
}

/* Coarse cell value = average of its 8 children. */
static void restrict_level(const olev* F, const olev* C, const double* r, double* fc) {
#pragma omp parallel for schedule(static)
    for (int K = 0; K < C->nz; ++K)
        for (int J = 0; J < C->ny; ++J)
            for (int I = 0; I < C->nx; ++I) {
                double s = 0.0;
                for (int dk = 0; dk < 2; ++dk)
                    for (int dj = 0; dj < 2; ++dj)
                        for (int di = 0; di < 2; ++di)
                            s += r[CI(F, 2 * I + di, 2 * J + dj, 2 * K + dk)];
                fc[CI(C, I, J, K)] = 0.125 * s;
            }
}

/* Fine cell += value of its parent (piecewise-constant prolongation). */
static void prolong_level(const olev* F, const olev* C, const double* phic, double* phi) {
#pragma omp parallel for schedule(static)
    for (int k = 0; k < F->nz; ++k)
        for (int j = 0; j < F->ny; ++j)
            for (int i = 0; i < F->nx; ++i)
                phi[CI(F, i, j, k)] += phic[CI(C, i / 2, j / 2, k / 2)];
}

/* Coarse face coefficient = mean of the 4 coincident fine faces. */
static void coarsen_coeffs(const olev* F, olev* C) {
    for (int K = 0; K < C->nz; ++K)
        for (int J = 0; J < C->ny; ++J)
            for (int I = 0; I <= C->nx; ++I) {
                int i = 2 * I;
                C->bx[FXI(C, I, J, K)] = 0.25 * (F->bx[FXI(F, i, 2 * J, 2 * K)] + F->bx[FXI(F, i, 2 * J + 1, 2 * K)] +
                                                 F->bx[FXI(F, i, 2 * J, 2 * K + 1)] + F->bx[FXI(F, i, 2 * J + 1, 2 * K + 1)]);
            }
    for (int K = 0; K < C->nz; ++K)
        for (int J = 0; J <= C->ny; ++J)
            for (int I = 0; I < C->nx; ++I) {
                int j = 2 * J;
                C->by[FYI(C, I, J, K)] = 0.25 * (F->by[FYI(F, 2 * I, j, 2 * K)] + F->by[FYI(F, 2 * I + 1, j, 2 * K)] +
                                                 F->by[FYI(F, 2 * I, j, 2 * K + 1)] + F->by[FYI(F, 2 * I + 1, j, 2 * K + 1)]);
            }
    for (int K = 0; K <= C->nz; ++K)
        for (int J = 0; J < C->ny; ++J)
            for (int I = 0; I < C->nx; ++I) {
                int k = 2 * K;
                C->bz[FZI(C, I, J, K)] = 0.25 * (F->bz[FZI(F, 2 * I, 2 * J, k)] + F->bz[FZI(F, 2 * I + 1, 2 * J, k)] +
                                                 F->bz[FZI(F, 2 * I, 2 * J + 1, k)] + F->bz[FZI(F, 2 * I + 1, 2 * J + 1, k)]);
            }
}

/* ------------------------------------------------------------------ */
/* Coarsest level: dense Cholesky of M = -A + c 1 1^T.                 */
/* ------------------------------------------------------------------ */
static int coarse_factor(const olev* L, int singular, double** out) {
    int n = (int)ncell(L);
    double* M = (double*)calloc((size_t)n * n, sizeof(double));
    if (!M) return ORC_ERR_OOM;
    double ih2 = 1.0 / (L->h * L->h);
    for (int k = 0; k < L->nz; ++k)
        for (int j = 0; j < L->ny; ++j)
            for (int i = 0; i < L->nx; ++i) {
                double b[6];
                size_t nb[6];
                int ghost[6];
                int m = cell_faces(L, i, j, k, b, nb, ghost);
                size_t c = CI(L, i, j, k);
                for (int q = 0; q < m; ++q) {
                    if (ghost[q]) {
                        M[c * n + c] += 2.0 * b[q] * ih2;
                    } else {
                        M[c * n + c] += b[q] * ih2;
                        M[c * n + nb[q]] -= b[q] * ih2;
                    }
                }
            }
    if (singular) {
        double dsum = 0.0;
        for (int c = 0; c < n; ++c) dsum += M[(size_t)c * n + c];
        double shift = dsum / n;
        for (size_t e = 0; e < (size_t)n * n; ++e) M[e] += shift;
    }
    /* in-place Cholesky, lower triangle: M = G G^T */
    for (int j = 0; j < n; ++j) {
        double d = M[(size_t)j * n + j];
        for (int p = 0; p < j; ++p) d -= M[(size_t)j * n + p] * M[(size_t)j * n + p];
        if (!(d > 0.0)) { free(M); return ORC_ERR_INVALID; }
        double g = sqrt(d);
        M[(size_t)j * n + j] = g;
        for (int i = j + 1; i < n; ++i) {
            double s = M[(size_t)i * n + j];
            for (int p = 0; p < j; ++p) s -= M[(size_t)i * n + p] * M[(size_t)j * n + p];
            M[(size_t)i * n + j] = s / g;
        }
    }
    *out = M;
    return ORC_OK;
}

static void coarse_solve(const double* G, int n, int singular, const double* f, double* x) {
    double mf = 0.0;
    if (singular) {
        for (int c = 0; c < n; ++c) mf += f[c];
        mf /= n;
    }
    /* forward: G y = -(f - mean f) */
    for (int i = 0; i < n; ++i) {
        double s = -(f[i] - mf);
        for (int p = 0; p < i; ++p) s -= G[(size_t)i * n + p] * x[p];
        x[i] = s / G[(size_t)i * n + i];
    }
    /* backward: G^T x = y */
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int p = i + 1; p < n; ++p) s -= G[(size_t)p * n + i] * x[p];
        x[i] = s / G[(size_t)i * n + i];
    }
    if (singular) {
        double mx = 0.0;
        for (int c = 0; c < n; ++c) mx += x[c];
        mx /= n;
        for (int c = 0; c < n; ++c) x[c] -= mx;
    }
}

/* ------------------------------------------------------------------ */
/* Hierarchy                                                           */
/* ------------------------------------------------------------------ */
static int alloc_level(olev* L) {
    size_t N = ncell(L);
    L->bx = (double*)calloc((size_t)L->nz * L->ny * (L->nx + 1), sizeof(double));
    L->by = (double*)calloc((size_t)L->nz * (L->ny + 1) * L->nx, sizeof(double));
    L->bz = (double*)calloc((size_t)(L->nz + 1) * L->ny * L->nx, sizeof(double));
    L->phi = (double*)calloc(N, sizeof(double));
    L->f = (double*)calloc(N, sizeof(double));
    L->r = (double*)calloc(N, sizeof(double));
    return (L->bx && L->by && L->bz && L->phi && L->f && L->r) ? ORC_OK : ORC_ERR_OOM;
}

void orc_mg_destroy(void* hv) {
    omg* M = (omg*)hv;
    if (!M) return;
    for (int l = 0; l < M->nlev; ++l) {
        free(M->lev[l].bx); free(M->lev[l].by); free(M->lev[l].bz);
        free(M->lev[l].phi); free(M->lev[l].f); free(M->lev[l].r);
    }
    free(M->chol);
    free(M);
}

/* Number of levels for a shape (coarsening rule above); 0 if the coarsest
 * level would exceed COARSE_MAX cells. */
int orc_num_levels(int nx, int ny, int nz) {
    int n = 1;
    while ((nx % 2 == 0) && (ny % 2 == 0) && (nz % 2 == 0) && (long)nx * ny * nz > 64 && n < MAXLEV) {
        nx /= 2; ny /= 2; nz /= 2; ++n;
    }
    if ((long)nx * ny * nz > COARSE_MAX) return 0;
    return n;
}

/* Build the hierarchy from level-0 full face arrays (copied); side codes as
 * for the *_gen functions. */
void* orc_mg_create_gen(int nx, int ny, int nz, const int* side, double h,
                        const double* bx, const double* by, const double* bz, int* status) {
    if (!sides_valid(side)) { *status = ORC_ERR_INVALID; return NULL; }
    int nl = orc_num_levels(nx, ny, nz);
    if (nl == 0) { *status = ORC_ERR_SIZE; return NULL; }
    omg* M = (omg*)calloc(1, sizeof(omg));
    if (!M) { *status = ORC_ERR_OOM; return NULL; }
    M->nlev = nl;
    M->singular = !any_outflow(side);
    for (int l = 0; l < nl; ++l) {
        olev* L = &M->lev[l];
        wrap_level_gen(L, nx >> l, ny >> l, nz >> l, side, h * (double)(1 << l), NULL, NULL, NULL);
        if (alloc_level(L) != ORC_OK) { orc_mg_destroy(M); *status = ORC_ERR_OOM; return NULL; }
    }
    olev* L0 = &M->lev[0];
    memcpy(L0->bx, bx, sizeof(double) * (size_t)nz * ny * (nx + 1));
    memcpy(L0->by, by, sizeof(double) * (size_t)nz * (ny + 1) * nx);
    memcpy(L0->bz, bz, sizeof(double) * (size_t)(nz + 1) * ny * nx);
    for (int l = 0; l + 1 < nl; ++l) coarsen_coeffs(&M->lev[l], &M->lev[l + 1]);
    M->ncoarse = (int)ncell(&M->lev[nl - 1]);
    int st = coarse_factor(&M->lev[nl - 1], M->singular, &M->chol);
    if (st != ORC_OK) { orc_mg_destroy(M); *status = st; return NULL; }
    *status = ORC_OK;
    return M;
}

static void sides_of(int px, int py, int pz, int side[6]) {
    int p[3] = {px, py, pz};
    for (int d = 0; d < 3; ++d) side[2 * d] = side[2 * d + 1] = p[d] ? SIDE_PERIODIC : SIDE_WALL;
}

/* Build the hierarchy from level-0 full face arrays (copied). */
void* orc_mg_create(int nx, int ny, int nz, int px, int py, int pz, double h,
                    const double* bx, const double* by, const double* bz, int* status) {
    int side[6];
    sides_of(px, py, pz, side);
    return orc_mg_create_gen(nx, ny, nz, side, h, bx, by, bz, status);
}

int orc_mg_nlevels(void* hv) { return ((omg*)hv)->nlev; }

void orc_mg_level_info(void* hv, int l, int* dims, double* h) {
    olev* L = &((omg*)hv)->lev[l];
    dims[0] = L->nx; dims[1] = L->ny; dims[2] = L->nz;
    *h = L->h;
}

/* which: 0 phi, 1 f, 2 r, 3 bx, 4 by, 5 bz.  dir 0: copy out, 1: copy in. */
int orc_mg_io(void* hv, int l, int which, double* buf, int dir) {
    omg* M = (omg*)hv;
    if (l < 0 || l >= M->nlev) return ORC_ERR_INVALID;
    olev* L = &M->lev[l];
    double* p;
    size_t n;
    switch (which) {
        case 0: p = L->phi; n = ncell(L); break;
        case 1: p = L->f; n = ncell(L); break;
        case 2: p = L->r; n = ncell(L); break;
        case 3: p = L->bx; n = (size_t)L->nz * L->ny * (L->nx + 1); break;
        case 4: p = L->by; n = (size_t)L->nz * (L->ny + 1) * L->nx; break;
        case 5: p = L->bz; n = (size_t)(L->nz + 1) * L->ny * L->nx; break;
        default: return ORC_ERR_INVALID;
    }
    if (dir == 0) memcpy(buf, p, n * sizeof(double));
    else memcpy(p, buf, n * sizeof(double));
    return ORC_OK;
}

void orc_mg_smooth(void* hv, int l, int nsweeps) {
    omg* M = (omg*)hv;
    rbgs_level(&M->lev[l], M->lev[l].phi, M->lev[l].f, nsweeps);
}

/* r_l = f_l - L phi_l;  f_{l+1} = R r_l;  phi_{l+1} = 0. */
void orc_mg_resid_restrict(void* hv, int l) {
    omg* M = (omg*)hv;
    olev* F = &M->lev[l];
    olev* C = &M->lev[l + 1];
    residual_level(F, F->phi, F->f, F->r);
    restrict_level(F, C, F->r, C->f);
    memset(C->phi, 0, ncell(C) * sizeof(double));
}

void orc_mg_prolong(void* hv, int l) {
    omg* M = (omg*)hv;
    prolong_level(&M->lev[l], &M->lev[l + 1], M->lev[l + 1].phi, M->lev[l].phi);
}

void orc_mg_coarse(void* hv) {
    omg* M = (omg*)hv;
    olev* L = &M->lev[M->nlev - 1];
    coarse_solve(M->chol, M->ncoarse, M->singular, L->f, L->phi);
}

static void vcycle(omg* M, int l, int nu1, int nu2) {
    if (l == M->nlev - 1) { orc_mg_coarse(M); return; }
    olev* F = &M->lev[l];
    rbgs_level(F, F->phi, F->f, nu1);
    orc_mg_resid_restrict(M, l);
    vcycle(M, l + 1, nu1, nu2);
    orc_mg_prolong(M, l);
    rbgs_level(F, F->phi, F->f, nu2);
}

void orc_mg_vcycle(void* hv, int l, int nu1, int nu2) { vcycle((omg*)hv, l, nu1, nu2); }

static double norm2(const double* a, size_t n) {
    double s = 0.0;
    for (size_t c = 0; c < n; ++c) s += a[c] * a[c];
    return sqrt(s);
}

/*
 * Multigrid solve of L phi = f on level 0 (f taken as given: the caller has
 * already removed its mean).  phi starts at 0.
 *   mode 0 ("algorithm"): stop after the first V-cycle with
 *          ||f - L phi||_2 / ||f||_2 <= rtol.
 *   mode 1 ("definition"): iterate to stagnation (relative residual <= 1e-13
 *          or no new minimum over 3 cycles); returns the best iterate.
 * hist[c] = relative residual after c cycles (hist[0] = 1).  On exit phi has
 * zero mean (singular operator) or is returned as computed (outflow sides).  Returns ORC_OK, ORC_ERR_NOT_CONVERGED or ORC_ERR_NONFINITE.
 */
int orc_mg_solve(void* hv, const double* f0, double* phi_out, double rtol, int max_cycles,
                 int nu1, int nu2, int mode, double* hist, int hist_len, int* cycles_out) {
    omg* M = (omg*)hv;
    olev* L0 = &M->lev[0];
    size_t N = ncell(L0);
    memcpy(L0->f, f0, N * sizeof(double));
    memset(L0->phi, 0, N * sizeof(double));
    double fn = norm2(L0->f, N);
    int status = ORC_OK;
    int c = 0;
    if (hist_len > 0) hist[0] = (fn > 0.0) ? 1.0 : 0.0;
    if (fn > 0.0) {
        double best = INFINITY;
        double* best_phi = (mode == 1) ? (double*)malloc(N * sizeof(double)) : NULL;
        int since_best = 0;
        status = ORC_ERR_NOT_CONVERGED;
        while (c < max_cycles) {
            vcycle(M, 0, nu1, nu2);
            ++c;
            residual_level(L0, L0->phi, L0->f, L0->r);
            double rel = norm2(L0->r, N) / fn;
            if (c < hist_len) hist[c] = rel;
            if (!isfinite(rel)) { status = ORC_ERR_NONFINITE; break; }
            if (mode == 0) {
                if (rel <= rtol) { status = ORC_OK; break; }
            } else {
                if (rel < best) {
                    best = rel; since_best = 0;
                    memcpy(best_phi, L0->phi, N * sizeof(double));
                } else if (++since_best >= 3) { status = ORC_OK; break; }
                if (rel <= 1e-13) { status = ORC_OK; break; }
            }
        }
        if (mode == 1 && best_phi) {
            if (status == ORC_ERR_NOT_CONVERGED && best <= rtol) status = ORC_OK;
            memcpy(L0->phi, best_phi, N * sizeof(double));
            free(best_phi);
        }
    }
    double m = 0.0;
    if (M->singular) {
        for (size_t e = 0; e < N; ++e) m += L0->phi[e];
        m /= (double)N;
    }
    for (size_t e = 0; e < N; ++e) phi_out[e] = L0->phi[e] - m;
    *cycles_out = c;
    return status;
}

/* ------------------------------------------------------------------ */
/* Velocity correction U -= (b/beta0)_f grad phi on non-wall faces.     */
/* ------------------------------------------------------------------ */
void orc_correct(int nx, int ny, int nz, int px, int py, int pz, double h,
                 const double* b0c, const double* b0e,
                 const double* bx, const double* by, const double* bz,
                 const double* phi, double* u, double* v, double* w) {
    olev L;
    wrap_level(&L, nx, ny, nz, px, py, pz, h, (double*)bx, (double*)by, (double*)bz);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                if (i == 0 && !px) continue;
                int im = (i == 0) ? nx - 1 : i - 1;
                double g = (phi[CI(&L, i, j, k)] - phi[CI(&L, im, j, k)]) / h;
                u[FXI(&L, i, j, k)] -= (bx[FXI(&L, i, j, k)] / b0c[k]) * g;
            }
    if (px)
        for (int k = 0; k < nz; ++k)
            for (int j = 0; j < ny; ++j) u[FXI(&L, nx, j, k)] = u[FXI(&L, 0, j, k)];
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                if (j == 0 && !py) continue;
                int jm = (j == 0) ? ny - 1 : j - 1;
                double g = (phi[CI(&L, i, j, k)] - phi[CI(&L, i, jm, k)]) / h;
                v[FYI(&L, i, j, k)] -= (by[FYI(&L, i, j, k)] / b0c[k]) * g;
            }
    if (py)
        for (int k = 0; k < nz; ++k)
            for (int i = 0; i < nx; ++i) v[FYI(&L, i, ny, k)] = v[FYI(&L, i, 0, k)];
    for (int k = 0; k < nz; ++k) {
        if (k == 0 && !pz) continue;
        int km = (k == 0) ? nz - 1 : k - 1;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double g = (phi[CI(&L, i, j, k)] - phi[CI(&L, i, j, km)]) / h;
                w[FZI(&L, i, j, k)] -= (bz[FZI(&L, i, j, k)] / b0e[k]) * g;
            }
    }
    if (pz)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) w[FZI(&L, i, j, nz)] = w[FZI(&L, i, j, 0)];
}

/* ------------------------------------------------------------------ */
/* The whole projection, end to end.                                   */
/* stats: [0] cycles, [1] rel residual, [2] mean removed from f,       */
/*        [3] sum f, [4] sum |f|, [5] ||f||_2 (after mean removal)     */
/* ------------------------------------------------------------------ */
int orc_mac_project_w0(int nx, int ny, int nz, int px, int py, int pz, double h,
                       const double* rho, const double* b0c, const double* b0e, const double* S,
                       const double* w0, double* u, double* v, double* w, double* phi_out,
                       double rtol, int max_cycles, int nu1, int nu2, int mode,
                       double* hist, int hist_len, double* stats) {
    size_t N = (size_t)nx * ny * nz;
    for (size_t c = 0; c < N; ++c)
        if (!isfinite(rho[c]) || !isfinite(S[c])) return ORC_ERR_NONFINITE;
    for (size_t c = 0; c < N; ++c)
        if (!(rho[c] > 0.0)) return ORC_ERR_INVALID;
    size_t nbx = (size_t)nz * ny * (nx + 1), nby = (size_t)nz * (ny + 1) * nx, nbz = (size_t)(nz + 1) * ny * nx;
    for (size_t e = 0; e < nbx; ++e) if (!isfinite(u[e])) return ORC_ERR_NONFINITE;
    for (size_t e = 0; e < nby; ++e) if (!isfinite(v[e])) return ORC_ERR_NONFINITE;
    for (size_t e = 0; e < nbz; ++e) if (!isfinite(w[e])) return ORC_ERR_NONFINITE;
    double* bx = (double*)malloc(nbx * sizeof(double));
    double* by = (double*)malloc(nby * sizeof(double));
    double* bz = (double*)malloc(nbz * sizeof(double));
    double* f = (double*)malloc(N * sizeof(double));
    if (!bx || !by || !bz || !f) { free(bx); free(by); free(bz); free(f); return ORC_ERR_OOM; }
    orc_face_coeffs(nx, ny, nz, px, py, pz, rho, b0c, b0e, bx, by, bz);
    orc_rhs_w0(nx, ny, nz, px, py, pz, h, b0c, b0e, u, v, w, S, w0, f);
    double sf = 0.0, saf = 0.0;
    for (size_t c = 0; c < N; ++c) { sf += f[c]; saf += fabs(f[c]); }
    stats[3] = sf; stats[4] = saf;
    int status;
    if (fabs(sf) > 1e-8 * saf) {
        status = ORC_ERR_INCOMPATIBLE;
        goto done;
    }
    double mean = sf / (double)N;
    for (size_t c = 0; c < N; ++c) f[c] -= mean;
    stats[2] = mean;
    stats[5] = norm2(f, N);
    {
        int st = 0;
        void* M = orc_mg_create(nx, ny, nz, px, py, pz, h, bx, by, bz, &st);
        if (!M) { status = st; goto done; }
        int cyc = 0;
        status = orc_mg_solve(M, f, phi_out, rtol, max_cycles, nu1, nu2, mode, hist, hist_len, &cyc);
        stats[0] = cyc;
        stats[1] = (cyc < hist_len) ? hist[cyc] : NAN;
        orc_mg_destroy(M);
    }
    if (status == ORC_OK || status == ORC_ERR_NOT_CONVERGED)
        orc_correct(nx, ny, nz, px, py, pz, h, b0c, b0e, bx, by, bz, phi_out, u, v, w);
done:
    free(bx); free(by); free(bz); free(f);
    return status;
}

int orc_mac_project(int nx, int ny, int nz, int px, int py, int pz, double h,
                    const double* rho, const double* b0c, const double* b0e, const double* S,
                    double* u, double* v, double* w, double* phi_out,
                    double rtol, int max_cycles, int nu1, int nu2, int mode,
                    double* hist, int hist_len, double* stats) {
    return orc_mac_project_w0(nx, ny, nz, px, py, pz, h, rho, b0c, b0e, S, NULL, u, v, w, phi_out, rtol,
                              max_cycles, nu1, nu2, mode, hist, hist_len, stats);
}

/* ------------------------------------------------------------------ */
/* General boundaries and base states (outflow sides, radial beta0).   */
/* ------------------------------------------------------------------ */
typedef struct {
    const double* b0c;       /* plane-parallel: beta0 at layer centres (nz) */
    const double* b0e;       /*                 and at z faces (nz+1) */
    int nr;                  /* radial: profile of nr values at r = (m + 1/2) dr */
    double dr;
    const double* prof;      /* NULL: plane-parallel */
    double c[3];             /* centre of the radial profile */
    double h;
} obeta;

static void obeta_init(obeta* B, const double* b0c, const double* b0e, int nr, double dr, const double* prof,
                       const double* centre, double h) {
    B->b0c = b0c; B->b0e = b0e; B->nr = nr; B->dr = dr; B->prof = prof; B->h = h;
    B->c[0] = centre ? centre[0] : 0.0;
    B->c[1] = centre ? centre[1] : 0.0;
    B->c[2] = centre ? centre[2] : 0.0;
}

/* beta0 at distance r from the centre: linear in r between the two nearest
 * profile radii, constant below the first and above the last. */
static double radial_beta0(const obeta* B, double r) {
    double s = r / B->dr - 0.5;
    if (!(s > 0.0)) return B->prof[0];
    if (s >= (double)(B->nr - 1)) return B->prof[B->nr - 1];
    int m = (int)s;
    double t = s - (double)m;
    return B->prof[m] + t * (B->prof[m + 1] - B->prof[m]);
}

static double radial_at(const obeta* B, double x, double y, double z) {
    double dx = x - B->c[0], dy = y - B->c[1], dz = z - B->c[2];
    return radial_beta0(B, sqrt(dx * dx + dy * dy + dz * dz));
}

/* beta0 at the centre of cell (i,j,k). */
static double beta0_cell(const obeta* B, int i, int j, int k) {
    if (!B->prof) return B->b0c[k];
    return radial_at(B, (i + 0.5) * B->h, (j + 0.5) * B->h, (k + 0.5) * B->h);
}

/* beta0 at face f of direction d (0 x, 1 y, 2 z) in row/column (a, b): the
 * face at coordinate f h along d, the cell centres of (a, b) across it
 * (x faces: a = j, b = k; y faces: a = i, b = k; z faces: a = i, b = j). */
static double beta0_face(const obeta* B, int d, int f, int a, int b) {
    if (!B->prof) return d == 2 ? B->b0e[f] : B->b0c[b];
    double h = B->h;
    if (d == 0) return radial_at(B, f * h, (a + 0.5) * h, (b + 0.5) * h);
    if (d == 1) return radial_at(B, (a + 0.5) * h, f * h, (b + 0.5) * h);
    return radial_at(B, (a + 0.5) * h, (b + 0.5) * h, f * h);
}

/* beta0 at cell centres (the radial mapping alone). */
void orc_map_radial(int nx, int ny, int nz, double h, int nr, double dr, const double* prof,
                    const double* centre, double* out) {
    obeta B;
    obeta_init(&B, NULL, NULL, nr, dr, prof, centre, h);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) out[((size_t)k * ny + j) * nx + i] = beta0_cell(&B, i, j, k);
}

/* Face coefficients with per-side boundaries: interior and periodic faces
 * beta0_face / (0.5 (rho_L + rho_R)) (in a periodic direction face n is face
 * 0), outflow faces beta0_face / rho of the adjacent cell, walls 0. */
static void face_coeffs_gen(int nx, int ny, int nz, const int* side, const obeta* B, const double* rho,
                            double* bx, double* by, double* bz) {
    olev L;
    wrap_level_gen(&L, nx, ny, nz, side, B->h, bx, by, bz);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                double b;
                if (i > 0 && i < nx) {
                    b = beta0_face(B, 0, i, j, k) / (0.5 * (rho[CI(&L, i - 1, j, k)] + rho[CI(&L, i, j, k)]));
                } else if (L.px) {
                    b = beta0_face(B, 0, 0, j, k) / (0.5 * (rho[CI(&L, nx - 1, j, k)] + rho[CI(&L, 0, j, k)]));
                } else if (i == 0 && side[0] == SIDE_OUTFLOW) {
                    b = beta0_face(B, 0, 0, j, k) / rho[CI(&L, 0, j, k)];
                } else if (i == nx && side[1] == SIDE_OUTFLOW) {
                    b = beta0_face(B, 0, nx, j, k) / rho[CI(&L, nx - 1, j, k)];
                } else {
                    b = 0.0;
                }
                bx[FXI(&L, i, j, k)] = b;
            }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double b;
                if (j > 0 && j < ny) {
                    b = beta0_face(B, 1, j, i, k) / (0.5 * (rho[CI(&L, i, j - 1, k)] + rho[CI(&L, i, j, k)]));
                } else if (L.py) {
                    b = beta0_face(B, 1, 0, i, k) / (0.5 * (rho[CI(&L, i, ny - 1, k)] + rho[CI(&L, i, 0, k)]));
                } else if (j == 0 && side[2] == SIDE_OUTFLOW) {
                    b = beta0_face(B, 1, 0, i, k) / rho[CI(&L, i, 0, k)];
                } else if (j == ny && side[3] == SIDE_OUTFLOW) {
                    b = beta0_face(B, 1, ny, i, k) / rho[CI(&L, i, ny - 1, k)];
                } else {
                    b = 0.0;
                }
                by[FYI(&L, i, j, k)] = b;
            }
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double b;
                if (k > 0 && k < nz) {
                    b = beta0_face(B, 2, k, i, j) / (0.5 * (rho[CI(&L, i, j, k - 1)] + rho[CI(&L, i, j, k)]));
                } else if (L.pz) {
                    b = beta0_face(B, 2, 0, i, j) / (0.5 * (rho[CI(&L, i, j, nz - 1)] + rho[CI(&L, i, j, 0)]));
                } else if (k == 0 && side[4] == SIDE_OUTFLOW) {
                    b = beta0_face(B, 2, 0, i, j) / rho[CI(&L, i, j, 0)];
                } else if (k == nz && side[5] == SIDE_OUTFLOW) {
                    b = beta0_face(B, 2, nz, i, j) / rho[CI(&L, i, j, nz - 1)];
                } else {
                    b = 0.0;
                }
                bz[FZI(&L, i, j, k)] = b;
            }
}

int orc_face_coeffs_gen(int nx, int ny, int nz, const int* side, double h, const double* rho,
                        const double* b0c, const double* b0e, int nr, double dr, const double* prof,
                        const double* centre, double* bx, double* by, double* bz) {
    if (!sides_valid(side)) return ORC_ERR_INVALID;
    obeta B;
    obeta_init(&B, b0c, b0e, nr, dr, prof, centre, h);
    face_coeffs_gen(nx, ny, nz, side, &B, rho, bx, by, bz);
    return ORC_OK;
}

/* f = D(beta0 U) - beta0_c (S - w0[k]) with every face velocity weighted by
 * its own face's beta0 (in a periodic direction face n is face 0). */
static void rhs_gen(int nx, int ny, int nz, const int* side, const obeta* B, const double* u, const double* v,
                    const double* w, const double* S, const double* w0, double* f) {
    olev L;
    wrap_level_gen(&L, nx, ny, nz, side, B->h, NULL, NULL, NULL);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                int ih = (i == nx - 1 && L.px) ? 0 : i + 1;
                int jh = (j == ny - 1 && L.py) ? 0 : j + 1;
                int kh = (k == nz - 1 && L.pz) ? 0 : k + 1;
                double fx = beta0_face(B, 0, ih, j, k) * u[FXI(&L, ih, j, k)] - beta0_face(B, 0, i, j, k) * u[FXI(&L, i, j, k)];
                double fy = beta0_face(B, 1, jh, i, k) * v[FYI(&L, i, jh, k)] - beta0_face(B, 1, j, i, k) * v[FYI(&L, i, j, k)];
                double fz = beta0_face(B, 2, kh, i, j) * w[FZI(&L, i, j, kh)] - beta0_face(B, 2, k, i, j) * w[FZI(&L, i, j, k)];
                double src = S[CI(&L, i, j, k)];
                if (w0) src = src - w0[k];
                f[CI(&L, i, j, k)] = (fx + fy + fz) / B->h - beta0_cell(B, i, j, k) * src;
            }
}

int orc_rhs_gen(int nx, int ny, int nz, const int* side, double h, const double* b0c, const double* b0e, int nr,
                double dr, const double* prof, const double* centre, const double* u, const double* v,
                const double* w, const double* S, const double* w0, double* f) {
    if (!sides_valid(side)) return ORC_ERR_INVALID;
    obeta B;
    obeta_init(&B, b0c, b0e, nr, dr, prof, centre, h);
    rhs_gen(nx, ny, nz, side, &B, u, v, w, S, w0, f);
    return ORC_OK;
}

/* Single-level operator, residual and sweeps with per-side boundaries on full
 * face arrays (outflow faces hold their coefficient, walls anything). */
void orc_apply_gen(int nx, int ny, int nz, const int* side, double h, const double* bx, const double* by,
                   const double* bz, const double* phi, double* out) {
    olev L;
    wrap_level_gen(&L, nx, ny, nz, side, h, (double*)bx, (double*)by, (double*)bz);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) out[CI(&L, i, j, k)] = apply_cell(&L, phi, i, j, k);
}

void orc_rbgs_gen(int nx, int ny, int nz, const int* side, double h, const double* bx, const double* by,
                  const double* bz, double* phi, const double* f, int nsweeps) {
    olev L;
    wrap_level_gen(&L, nx, ny, nz, side, h, (double*)bx, (double*)by, (double*)bz);
    rbgs_level(&L, phi, f, nsweeps);
}

/* U -= (phi_c - phi_nb) / h / rho_face on every face that is not a wall:
 * interior and periodic faces with rho_face = 0.5 (rho_L + rho_R), outflow
 * faces with the ghost value -phi_c and rho_face = rho of the adjacent cell.
 * Periodic duplicate faces (face n) are refreshed from face 0. */
static void correct_gen(int nx, int ny, int nz, const int* side, double h, const double* rho, const double* phi,
                        double* u, double* v, double* w) {
    olev L;
    wrap_level_gen(&L, nx, ny, nz, side, h, NULL, NULL, NULL);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                double pc = phi[CI(&L, i, j, k)];
                if (i > 0 || L.px) {
                    int im = i > 0 ? i - 1 : nx - 1;
                    double g = (pc - phi[CI(&L, im, j, k)]) / h;
                    u[FXI(&L, i, j, k)] -= g / (0.5 * (rho[CI(&L, im, j, k)] + rho[CI(&L, i, j, k)]));
                } else if (side[0] == SIDE_OUTFLOW) {
                    double g = (pc - (-pc)) / h;
                    u[FXI(&L, 0, j, k)] -= g / rho[CI(&L, 0, j, k)];
                }
            }
            if (L.px) u[FXI(&L, nx, j, k)] = u[FXI(&L, 0, j, k)];
            else if (side[1] == SIDE_OUTFLOW) {
                double pc = phi[CI(&L, nx - 1, j, k)];
                double g = ((-pc) - pc) / h;
                u[FXI(&L, nx, j, k)] -= g / rho[CI(&L, nx - 1, j, k)];
            }
        }
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) {
            for (int j = 0; j < ny; ++j) {
                double pc = phi[CI(&L, i, j, k)];
                if (j > 0 || L.py) {
                    int jm = j > 0 ? j - 1 : ny - 1;
                    double g = (pc - phi[CI(&L, i, jm, k)]) / h;
                    v[FYI(&L, i, j, k)] -= g / (0.5 * (rho[CI(&L, i, jm, k)] + rho[CI(&L, i, j, k)]));
                } else if (side[2] == SIDE_OUTFLOW) {
                    double g = (pc - (-pc)) / h;
                    v[FYI(&L, i, 0, k)] -= g / rho[CI(&L, i, 0, k)];
                }
            }
            if (L.py) v[FYI(&L, i, ny, k)] = v[FYI(&L, i, 0, k)];
            else if (side[3] == SIDE_OUTFLOW) {
                double pc = phi[CI(&L, i, ny - 1, k)];
                double g = ((-pc) - pc) / h;
                v[FYI(&L, i, ny, k)] -= g / rho[CI(&L, i, ny - 1, k)];
            }
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            for (int k = 0; k < nz; ++k) {
                double pc = phi[CI(&L, i, j, k)];
                if (k > 0 || L.pz) {
                    int km = k > 0 ? k - 1 : nz - 1;
                    double g = (pc - phi[CI(&L, i, j, km)]) / h;
                    w[FZI(&L, i, j, k)] -= g / (0.5 * (rho[CI(&L, i, j, km)] + rho[CI(&L, i, j, k)]));
                } else if (side[4] == SIDE_OUTFLOW) {
                    double g = (pc - (-pc)) / h;
                    w[FZI(&L, i, j, 0)] -= g / rho[CI(&L, i, j, 0)];
                }
            }
            if (L.pz) w[FZI(&L, i, j, nz)] = w[FZI(&L, i, j, 0)];
            else if (side[5] == SIDE_OUTFLOW) {
                double pc = phi[CI(&L, i, j, nz - 1)];
                double g = ((-pc) - pc) / h;
                w[FZI(&L, i, j, nz)] -= g / rho[CI(&L, i, j, nz - 1)];
            }
        }
}

void orc_correct_gen(int nx, int ny, int nz, const int* side, double h, const double* rho, const double* phi,
                     double* u, double* v, double* w) {
    correct_gen(nx, ny, nz, side, h, rho, phi, u, v, w);
}

/* The whole projection with per-side boundaries and a plane-parallel
 * (b0c, b0e) or radial (prof != NULL) beta0.  Statuses, stats and modes as
 * orc_mac_project_w0; with an outflow side there is no compatibility check
 * and neither f nor phi has its mean removed (stats[2] = 0). */
int orc_mac_project_gen(int nx, int ny, int nz, const int* side, double h, const double* rho,
                        const double* b0c, const double* b0e, int nr, double dr, const double* prof,
                        const double* centre, const double* S, const double* w0, double* u, double* v,
                        double* w, double* phi_out, double rtol, int max_cycles, int nu1, int nu2, int mode,
                        double* hist, int hist_len, double* stats) {
    if (!sides_valid(side)) return ORC_ERR_INVALID;
    size_t N = (size_t)nx * ny * nz;
    for (size_t c = 0; c < N; ++c)
        if (!isfinite(rho[c]) || !isfinite(S[c])) return ORC_ERR_NONFINITE;
    for (size_t c = 0; c < N; ++c)
        if (!(rho[c] > 0.0)) return ORC_ERR_INVALID;
    if (prof) {
        if (nr < 1 || !(dr > 0.0)) return ORC_ERR_INVALID;
        for (int m = 0; m < nr; ++m) {
            if (!isfinite(prof[m])) return ORC_ERR_NONFINITE;
            if (!(prof[m] > 0.0)) return ORC_ERR_INVALID;
        }
    }
    size_t nbx = (size_t)nz * ny * (nx + 1), nby = (size_t)nz * (ny + 1) * nx, nbz = (size_t)(nz + 1) * ny * nx;
    for (size_t e = 0; e < nbx; ++e) if (!isfinite(u[e])) return ORC_ERR_NONFINITE;
    for (size_t e = 0; e < nby; ++e) if (!isfinite(v[e])) return ORC_ERR_NONFINITE;
    for (size_t e = 0; e < nbz; ++e) if (!isfinite(w[e])) return ORC_ERR_NONFINITE;
    obeta B;
    obeta_init(&B, b0c, b0e, nr, dr, prof, centre, h);
    double* bx = (double*)malloc(nbx * sizeof(double));
    double* by = (double*)malloc(nby * sizeof(double));
    double* bz = (double*)malloc(nbz * sizeof(double));
    double* f = (double*)malloc(N * sizeof(double));
    if (!bx || !by || !bz || !f) { free(bx); free(by); free(bz); free(f); return ORC_ERR_OOM; }
    face_coeffs_gen(nx, ny, nz, side, &B, rho, bx, by, bz);
    rhs_gen(nx, ny, nz, side, &B, u, v, w, S, w0, f);
    double sf = 0.0, saf = 0.0;
    for (size_t c = 0; c < N; ++c) { sf += f[c]; saf += fabs(f[c]); }
    stats[3] = sf; stats[4] = saf;
    stats[2] = 0.0;
    int status;
    if (!any_outflow(side)) {
        if (fabs(sf) > 1e-8 * saf) {
            status = ORC_ERR_INCOMPATIBLE;
            goto done;
        }
        double mean = sf / (double)N;
        for (size_t c = 0; c < N; ++c) f[c] -= mean;
        stats[2] = mean;
    }
    stats[5] = norm2(f, N);
    {
        int st = 0;
        void* M = orc_mg_create_gen(nx, ny, nz, side, h, bx, by, bz, &st);
        if (!M) { status = st; goto done; }
        int cyc = 0;
        status = orc_mg_solve(M, f, phi_out, rtol, max_cycles, nu1, nu2, mode, hist, hist_len, &cyc);
        stats[0] = cyc;
        stats[1] = (cyc < hist_len) ? hist[cyc] : NAN;
        orc_mg_destroy(M);
    }
    if (status == ORC_OK || status == ORC_ERR_NOT_CONVERGED)
        correct_gen(nx, ny, nz, side, h, rho, phi_out, u, v, w);
done:
    free(bx); free(by); free(bz); free(f);
    return status;
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
