/*
 * FP64 CPU oracle for the nodal (cell-velocity) projection.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow reference for the HIP path's nodal
 * projection; it shares no code, header, table or helper with the HIP
 * library, and only tests, the smoke check and the benchmark's CPU baseline
 * may load it.
 *
 * What it computes (arXiv:1910.12979, Sec. 3: the second-order projection
 * method projects both the face velocities (the MAC projection, mg_oracle.c)
 * and the cell-centred velocities; this file is the latter).  The constraint
 * is the same as for the MAC projection (Sec. 2, div(beta0 U) = beta0 S); the
 * potential phi lives on the nodes (cell corners) and the cell velocities are
 * corrected by U -= (1/rho) G phi.
 *
 * Discretisation (the paper gives none; this is the reading, stated once):
 *   trilinear (Q1) finite elements on the nodes with a cell-constant
 *   coefficient sigma_c = beta0_c / rho_c.  The element stiffness of a cube
 *   couples two corners with weight 1/3 h (same corner), 0 (corners joined by
 *   an edge), -1/12 h (across a face or the body diagonal).  Dividing the weak
 *   form by the node's volume h^3:
 *     (L phi)_n = 1/(12 h^2) sum_{cells c at n} sigma_c
 *                 [ sum_{the 4 corners m of c across a face or the diagonal
 *                   from n} phi_m  -  4 phi_n ]
 *     f_n = D_n(beta0 U) - (beta0 S)_n,
 *     D_n(beta0 U) = 1/(4h) sum_c beta0_c (+-u_c +- v_c +- w_c)  (+ for a cell
 *                    on the high side of n in that direction, - on the low side)
 *     (beta0 S)_n  = 1/8 sum_c beta0_c S_c
 *   and L phi = f.  Only the cells that exist contribute (a solid wall is a
 *   natural boundary: its nodes are unknowns, no flux leaves).  In a periodic
 *   direction node n is node 0.  G phi of a cell is its mean gradient, e.g.
 *   (G phi)_x = 1/(4h) sum over its 4 x-edges of (phi_high - phi_low).
 *   L differs from D sigma G (the projection is approximate, the velocity it
 *   returns satisfies the constraint to truncation error, not to round-off).
 *
 * Multigrid (V-cycle): four-colour Gauss-Seidel, colour c = (J mod 2) +
 *   2 (K mod 2) visited in the order 0, 1, 2, 3.  Two nodes are coupled only
 *   when they differ by one in at least two coordinates (the edge weight is
 *   zero), so at least one of J, K differs by one and the colours differ (for
 *   even node counts also across a periodic wrap): each colour is a Jacobi
 *   step of a true Gauss-Seidel sweep, and every x-row has one colour;
 *   residual
 *   restricted by full weighting f_C = 1/8 sum_d prod_i (1 - |d_i|/2)
 *   r_{2C+d} (d in {-1,0,1}^3, existing fine nodes only), coarse phi = 0;
 *   trilinear prolongation; coarse sigma = mean of the 8 fine cells, spacing
 *   2h; coarsening while every cell dimension is even and the level has more
 *   than 64 cells; coarsest level (at most 512 nodes) solved exactly: f <-
 *   f - mean(f), dense Cholesky of (-A + c 1 1^T), c the mean diagonal of -A,
 *   x <- x - mean(x).
 *
 * Built with gcc, no fast-math, no FMA contraction; every reduction is a
 * serial loop in index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NOD_OK 0
#define NOD_ERR_INVALID (-1)
#define NOD_ERR_SIZE (-2)
#define NOD_ERR_INCOMPATIBLE (-3)
#define NOD_ERR_NOT_CONVERGED (-4)
#define NOD_ERR_NONFINITE (-5)
#define NOD_ERR_OOM (-6)

#define NOD_MAXLEV 32
#define NOD_COARSE_MAX 512

typedef struct {
    int nx, ny, nz;          /* cells */
    int p[3];                /* periodic flags */
    int Nx, Ny, Nz;          /* nodes: n (periodic) or n + 1 */
    double h;
    double *sig;             /* (nz, ny, nx) cell coefficients */
    double *phi, *f, *r;     /* (Nz, Ny, Nx) node arrays */
} nlev;

typedef struct {
    int nlev;
    nlev lev[NOD_MAXLEV];
    double* chol;
    int ncoarse;
} nmg;

static void nlev_init(nlev* L, int nx, int ny, int nz, const int* per, double h) {
    memset(L, 0, sizeof(*L));
    L->nx = nx; L->ny = ny; L->nz = nz;
    for (int d = 0; d < 3; ++d) L->p[d] = per[d];
    L->Nx = nx + (per[0] ? 0 : 1);
    L->Ny = ny + (per[1] ? 0 : 1);
    L->Nz = nz + (per[2] ? 0 : 1);
    L->h = h;
}

static size_t NI(const nlev* L, int I, int J, int K) { return ((size_t)K * L->Ny + J) * L->Nx + I; }
static size_t CIc(const nlev* L, int i, int j, int k) { return ((size_t)k * L->ny + j) * L->nx + i; }
static size_t nnodes(const nlev* L) { return (size_t)L->Nx * L->Ny * L->Nz; }
static size_t ncells(const nlev* L) { return (size_t)L->nx * L->ny * L->nz; }

/* Cell index along one direction of the cell on side s (0: low, 1: high) of
 * node coordinate I; -1 if it does not exist (wall). */
static int cell_of(int I, int s, int n, int per) {
    int c = s ? I : I - 1;
    if (per) return (c + n) % n;
    return (c >= 0 && c < n) ? c : -1;
}

/* Node index along one direction, I + o (o in {-1, 0, 1}); -1 if outside. */
static int node_of(int I, int o, int N, int per) {
    int m = I + o;
    if (per) return (m + N) % N;
    return (m >= 0 && m < N) ? m : -1;
}

/* (L phi)_n */
static double apply_node(const nlev* L, const double* phi, int I, int J, int K) {
    const int Nn[3] = {L->Nx, L->Ny, L->Nz}, nc[3] = {L->nx, L->ny, L->nz};
    const int X[3] = {I, J, K};
    const double pn = phi[NI(L, I, J, K)];
    double s = 0.0;
    for (int sz = 0; sz < 2; ++sz)
        for (int sy = 0; sy < 2; ++sy)
            for (int sx = 0; sx < 2; ++sx) {
                int S[3] = {sx, sy, sz}, c[3];
                int ok = 1;
                for (int d = 0; d < 3; ++d) {
                    c[d] = cell_of(X[d], S[d], nc[d], L->p[d]);
                    if (c[d] < 0) ok = 0;
                }
                if (!ok) continue;
                double sig = L->sig[CIc(L, c[0], c[1], c[2])];
                /* the cell's corners are X + o with o_d in {0, +1} (high side) or {-1, 0} */
                double acc = 0.0;
                for (int mz = 0; mz < 2; ++mz)
                    for (int my = 0; my < 2; ++my)
                        for (int mx = 0; mx < 2; ++mx) {
                            int moved = mx + my + mz;
                            if (moved < 2) continue;
                            int M[3] = {mx, my, mz}, m[3];
                            for (int d = 0; d < 3; ++d) {
                                int o = M[d] ? (S[d] ? 1 : -1) : 0;
                                m[d] = node_of(X[d], o, Nn[d], L->p[d]);
                            }
                            acc += phi[NI(L, m[0], m[1], m[2])];
                        }
                s += sig * (acc - 4.0 * pn);
            }
    return s / (12.0 * L->h * L->h);
}

/* One Gauss-Seidel sweep: the 4 colours (J mod 2) + 2 (K mod 2) in order. */
static void gs_level(const nlev* L, double* phi, const double* f, int nsweeps) {
    const int Nn[3] = {L->Nx, L->Ny, L->Nz}, nc[3] = {L->nx, L->ny, L->nz};
    const double h2 = L->h * L->h;
    for (int sw = 0; sw < nsweeps; ++sw)
        for (int col = 0; col < 4; ++col)
            for (int K = 0; K < L->Nz; ++K)
                for (int J = 0; J < L->Ny; ++J)
                    for (int I = 0; I < L->Nx; ++I) {
                        if ((J & 1) + 2 * (K & 1) != col) continue;
                        const int X[3] = {I, J, K};
                        double num = 0.0, den = 0.0;
                        for (int sz = 0; sz < 2; ++sz)
                            for (int sy = 0; sy < 2; ++sy)
                                for (int sx = 0; sx < 2; ++sx) {
                                    int S[3] = {sx, sy, sz}, c[3];
                                    int ok = 1;
                                    for (int d = 0; d < 3; ++d) {
                                        c[d] = cell_of(X[d], S[d], nc[d], L->p[d]);
                                        if (c[d] < 0) ok = 0;
                                    }
                                    if (!ok) continue;
                                    double sig = L->sig[CIc(L, c[0], c[1], c[2])];
                                    double acc = 0.0;
                                    for (int mz = 0; mz < 2; ++mz)
                                        for (int my = 0; my < 2; ++my)
                                            for (int mx = 0; mx < 2; ++mx) {
                                                if (mx + my + mz < 2) continue;
                                                int M[3] = {mx, my, mz}, m[3];
                                                for (int d = 0; d < 3; ++d) {
                                                    int o = M[d] ? (S[d] ? 1 : -1) : 0;
                                                    m[d] = node_of(X[d], o, Nn[d], L->p[d]);
                                                }
                                                acc += phi[NI(L, m[0], m[1], m[2])];
                                            }
                                    num += sig * acc;
                                    den += 4.0 * sig;
                                }
                        /* (num - den phi) / (12 h^2) = f  =>  phi = (num - 12 h^2 f) / den */
                        size_t n = NI(L, I, J, K);
                        phi[n] = (num - 12.0 * h2 * f[n]) / den;
                    }
}

static void resid_level(const nlev* L, const double* phi, const double* f, double* r) {
    for (int K = 0; K < L->Nz; ++K)
        for (int J = 0; J < L->Ny; ++J)
            for (int I = 0; I < L->Nx; ++I) {
                size_t n = NI(L, I, J, K);
                r[n] = f[n] - apply_node(L, phi, I, J, K);
            }
}

/* f_C = 1/8 sum_d w(d) r_{2C+d} over existing fine nodes. */
static void restrict_level(const nlev* F, const nlev* C, const double* r, double* fc) {
    const int Nn[3] = {F->Nx, F->Ny, F->Nz};
    for (int K = 0; K < C->Nz; ++K)
        for (int J = 0; J < C->Ny; ++J)
            for (int I = 0; I < C->Nx; ++I) {
                const int X[3] = {2 * I, 2 * J, 2 * K};
                double s = 0.0;
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int D[3] = {dx, dy, dz}, m[3], ok = 1;
                            double w = 1.0;
                            for (int d = 0; d < 3; ++d) {
                                m[d] = node_of(X[d], D[d], Nn[d], F->p[d]);
                                if (m[d] < 0) ok = 0;
                                if (D[d] != 0) w *= 0.5;
                            }
                            if (ok) s += w * r[NI(F, m[0], m[1], m[2])];
                        }
                fc[NI(C, I, J, K)] = 0.125 * s;
            }
}

/* phi_fine += trilinear interpolation of phi_coarse. */
static void prolong_level(const nlev* F, const nlev* C, const double* pc, double* pf) {
    const int Nc[3] = {C->Nx, C->Ny, C->Nz};
    for (int K = 0; K < F->Nz; ++K)
        for (int J = 0; J < F->Ny; ++J)
            for (int I = 0; I < F->Nx; ++I) {
                const int X[3] = {I, J, K};
                double v = 0.0;
                /* each direction: even -> coarse node X/2 (weight 1); odd -> nodes (X-1)/2 and (X+1)/2 (1/2 each) */
                for (int bz = 0; bz < 2; ++bz)
                    for (int by = 0; by < 2; ++by)
                        for (int bx = 0; bx < 2; ++bx) {
                            int B[3] = {bx, by, bz}, m[3], ok = 1;
                            double w = 1.0;
                            for (int d = 0; d < 3; ++d) {
                                if (X[d] % 2 == 0) {
                                    if (B[d]) { ok = 0; break; }
                                    m[d] = X[d] / 2;
                                } else {
                                    m[d] = B[d] ? (X[d] + 1) / 2 : (X[d] - 1) / 2;
                                    if (C->p[d]) m[d] %= Nc[d];
                                    w *= 0.5;
                                }
                            }
                            if (ok) v += w * pc[NI(C, m[0], m[1], m[2])];
                        }
                pf[NI(F, I, J, K)] += v;
            }
}

static void coarsen_sigma(const nlev* F, nlev* C) {
    for (int k = 0; k < C->nz; ++k)
        for (int j = 0; j < C->ny; ++j)
            for (int i = 0; i < C->nx; ++i) {
                double s = 0.0;
                for (int dk = 0; dk < 2; ++dk)
                    for (int dj = 0; dj < 2; ++dj)
                        for (int di = 0; di < 2; ++di) s += F->sig[CIc(F, 2 * i + di, 2 * j + dj, 2 * k + dk)];
                C->sig[CIc(C, i, j, k)] = 0.125 * s;
            }
}

static int coarse_factor(const nlev* L, double** out) {
    int n = (int)nnodes(L);
    double* M = (double*)calloc((size_t)n * n, sizeof(double));
    double* e = (double*)calloc((size_t)n, sizeof(double));
    if (!M || !e) { free(M); free(e); return NOD_ERR_OOM; }
    /* column q of -A = -L e_q */
    for (int q = 0; q < n; ++q) {
        e[q] = 1.0;
        for (int K = 0; K < L->Nz; ++K)
            for (int J = 0; J < L->Ny; ++J)
                for (int I = 0; I < L->Nx; ++I) {
                    size_t r = NI(L, I, J, K);
                    M[r * n + q] = -apply_node(L, e, I, J, K);
                }
        e[q] = 0.0;
    }
    free(e);
    double dsum = 0.0;
    for (int c = 0; c < n; ++c) dsum += M[(size_t)c * n + c];
    double shift = dsum / n;
    for (size_t k = 0; k < (size_t)n * n; ++k) M[k] += shift;
    for (int j = 0; j < n; ++j) {
        double d = M[(size_t)j * n + j];
        for (int p = 0; p < j; ++p) d -= M[(size_t)j * n + p] * M[(size_t)j * n + p];
        if (!(d > 0.0)) { free(M); return NOD_ERR_INVALID; }
        double g = sqrt(d);
        M[(size_t)j * n + j] = g;
        for (int i = j + 1; i < n; ++i) {
            double s = M[(size_t)i * n + j];
            for (int p = 0; p < j; ++p) s -= M[(size_t)i * n + p] * M[(size_t)j * n + p];
            M[(size_t)i * n + j] = s / g;
        }
    }
    *out = M;
    return NOD_OK;
}

static void coarse_solve(const double* G, int n, const double* f, double* x) {
    double mf = 0.0;
    for (int c = 0; c < n; ++c) mf += f[c];
    mf /= n;
    for (int i = 0; i < n; ++i) {
        double s = -(f[i] - mf);
        for (int p = 0; p < i; ++p) s -= G[(size_t)i * n + p] * x[p];
        x[i] = s / G[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int p = i + 1; p < n; ++p) s -= G[(size_t)p * n + i] * x[p];
        x[i] = s / G[(size_t)i * n + i];
    }
    double mx = 0.0;
    for (int c = 0; c < n; ++c) mx += x[c];
    mx /= n;
    for (int c = 0; c < n; ++c) x[c] -= mx;
}

/* ------------------------------------------------------------------ */
int nod_num_levels(int nx, int ny, int nz, int px, int py, int pz) {
    int n = 1;
    while (nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0 && (long)nx * ny * nz > 64 && n < NOD_MAXLEV) {
        nx /= 2; ny /= 2; nz /= 2; ++n;
    }
    long nodes = (long)(nx + (px ? 0 : 1)) * (ny + (py ? 0 : 1)) * (nz + (pz ? 0 : 1));
    if (nodes > NOD_COARSE_MAX) return 0;
    return n;
}

void nod_mg_destroy(void* hv) {
    nmg* M = (nmg*)hv;
    if (!M) return;
    for (int l = 0; l < M->nlev; ++l) {
        free(M->lev[l].sig); free(M->lev[l].phi); free(M->lev[l].f); free(M->lev[l].r);
    }
    free(M->chol);
    free(M);
}

/* Hierarchy from the level-0 cell coefficients sigma (copied). */
void* nod_mg_create(int nx, int ny, int nz, int px, int py, int pz, double h, const double* sig, int* status) {
    int nl = nod_num_levels(nx, ny, nz, px, py, pz);
    if (nl == 0) { *status = NOD_ERR_SIZE; return NULL; }
    nmg* M = (nmg*)calloc(1, sizeof(nmg));
    if (!M) { *status = NOD_ERR_OOM; return NULL; }
    M->nlev = nl;
    const int per[3] = {px, py, pz};
    for (int l = 0; l < nl; ++l) {
        nlev* L = &M->lev[l];
        nlev_init(L, nx >> l, ny >> l, nz >> l, per, h * (double)(1 << l));
        L->sig = (double*)calloc(ncells(L), sizeof(double));
        L->phi = (double*)calloc(nnodes(L), sizeof(double));
        L->f = (double*)calloc(nnodes(L), sizeof(double));
        L->r = (double*)calloc(nnodes(L), sizeof(double));
        if (!L->sig || !L->phi || !L->f || !L->r) { nod_mg_destroy(M); *status = NOD_ERR_OOM; return NULL; }
    }
    memcpy(M->lev[0].sig, sig, ncells(&M->lev[0]) * sizeof(double));
    for (int l = 0; l + 1 < nl; ++l) coarsen_sigma(&M->lev[l], &M->lev[l + 1]);
    M->ncoarse = (int)nnodes(&M->lev[nl - 1]);
    int st = coarse_factor(&M->lev[nl - 1], &M->chol);
    if (st != NOD_OK) { nod_mg_destroy(M); *status = st; return NULL; }
    *status = NOD_OK;
    return M;
}

int nod_mg_nlevels(void* hv) { return ((nmg*)hv)->nlev; }

void nod_mg_level_info(void* hv, int l, int* dims) {
    nlev* L = &((nmg*)hv)->lev[l];
    dims[0] = L->Nx; dims[1] = L->Ny; dims[2] = L->Nz;
    dims[3] = L->nx; dims[4] = L->ny; dims[5] = L->nz;
}

/* which: 0 phi, 1 f, 2 r (nodes), 3 sigma (cells).  dir 0: out, 1: in. */
int nod_mg_io(void* hv, int l, int which, double* buf, int dir) {
    nmg* M = (nmg*)hv;
    if (l < 0 || l >= M->nlev) return NOD_ERR_INVALID;
    nlev* L = &M->lev[l];
    double* p;
    size_t n;
    switch (which) {
        case 0: p = L->phi; n = nnodes(L); break;
        case 1: p = L->f; n = nnodes(L); break;
        case 2: p = L->r; n = nnodes(L); break;
        case 3: p = L->sig; n = ncells(L); break;
        default: return NOD_ERR_INVALID;
    }
    if (dir == 0) memcpy(buf, p, n * sizeof(double));
    else memcpy(p, buf, n * sizeof(double));
    return NOD_OK;
}

void nod_mg_smooth(void* hv, int l, int nsweeps) {
    nmg* M = (nmg*)hv;
    gs_level(&M->lev[l], M->lev[l].phi, M->lev[l].f, nsweeps);
}

void nod_mg_resid_restrict(void* hv, int l) {
    nmg* M = (nmg*)hv;
    nlev* F = &M->lev[l];
    nlev* C = &M->lev[l + 1];
    resid_level(F, F->phi, F->f, F->r);
    restrict_level(F, C, F->r, C->f);
    memset(C->phi, 0, nnodes(C) * sizeof(double));
}

void nod_mg_prolong(void* hv, int l) {
    nmg* M = (nmg*)hv;
    prolong_level(&M->lev[l], &M->lev[l + 1], M->lev[l + 1].phi, M->lev[l].phi);
}

void nod_mg_coarse(void* hv) {
    nmg* M = (nmg*)hv;
    nlev* L = &M->lev[M->nlev - 1];
    coarse_solve(M->chol, M->ncoarse, L->f, L->phi);
}

static void vcycle(nmg* M, int l, int nu1, int nu2) {
    if (l == M->nlev - 1) { nod_mg_coarse(M); return; }
    nlev* F = &M->lev[l];
    gs_level(F, F->phi, F->f, nu1);
    nod_mg_resid_restrict(M, l);
    vcycle(M, l + 1, nu1, nu2);
    nod_mg_prolong(M, l);
    gs_level(F, F->phi, F->f, nu2);
}

static double norm2(const double* a, size_t n) {
    double s = 0.0;
    for (size_t c = 0; c < n; ++c) s += a[c] * a[c];
    return sqrt(s);
}

/* L phi = f0 from phi = 0, modes as the MAC oracle (0 algorithm: stop at
 * the first cycle with ||f - L phi|| / ||f|| <= rtol; 1 definition: iterate
 * to stagnation).  phi returned with zero mean. */
int nod_mg_solve(void* hv, const double* f0, double* phi_out, double rtol, int max_cycles, int nu1, int nu2,
                 int mode, double* hist, int hist_len, int* cycles_out) {
    nmg* M = (nmg*)hv;
    nlev* L0 = &M->lev[0];
    size_t N = nnodes(L0);
    memcpy(L0->f, f0, N * sizeof(double));
    memset(L0->phi, 0, N * sizeof(double));
    double fn = norm2(L0->f, N);
    int status = NOD_OK, c = 0;
    if (hist_len > 0) hist[0] = fn > 0.0 ? 1.0 : 0.0;
    if (fn > 0.0) {
        double best = INFINITY;
        double* best_phi = mode == 1 ? (double*)malloc(N * sizeof(double)) : NULL;
        int since = 0;
        status = NOD_ERR_NOT_CONVERGED;
        while (c < max_cycles) {
            vcycle(M, 0, nu1, nu2);
            ++c;
            resid_level(L0, L0->phi, L0->f, L0->r);
            double rel = norm2(L0->r, N) / fn;
            if (c < hist_len) hist[c] = rel;
            if (!isfinite(rel)) { status = NOD_ERR_NONFINITE; break; }
            if (mode == 0) {
                if (rel <= rtol) { status = NOD_OK; break; }
            } else {
                if (rel < best) { best = rel; since = 0; memcpy(best_phi, L0->phi, N * sizeof(double)); }
                else if (++since >= 3) { status = NOD_OK; break; }
                if (rel <= 1e-13) { status = NOD_OK; break; }
            }
        }
        if (mode == 1 && best_phi) {
            if (status == NOD_ERR_NOT_CONVERGED && best <= rtol) status = NOD_OK;
            memcpy(L0->phi, best_phi, N * sizeof(double));
            free(best_phi);
        }
    }
    double m = 0.0;
    for (size_t e = 0; e < N; ++e) m += L0->phi[e];
    m /= (double)N;
    for (size_t e = 0; e < N; ++e) phi_out[e] = L0->phi[e] - m;
    *cycles_out = c;
    return status;
}

/* ------------------------------------------------------------------ */
/* Level-0 pieces on their own.                                        */
/* ------------------------------------------------------------------ */
void nod_sigma(int nx, int ny, int nz, const double* rho, const double* b0c, double* sig) {
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = ((size_t)k * ny + j) * nx + i;
                sig[c] = b0c[k] / rho[c];
            }
}

void nod_apply(int nx, int ny, int nz, int px, int py, int pz, double h, const double* sig, const double* phi,
               double* out) {
    nlev L;
    const int per[3] = {px, py, pz};
    nlev_init(&L, nx, ny, nz, per, h);
    L.sig = (double*)sig;
    for (int K = 0; K < L.Nz; ++K)
        for (int J = 0; J < L.Ny; ++J)
            for (int I = 0; I < L.Nx; ++I) out[NI(&L, I, J, K)] = apply_node(&L, phi, I, J, K);
}

void nod_gs(int nx, int ny, int nz, int px, int py, int pz, double h, const double* sig, double* phi,
            const double* f, int nsweeps) {
    nlev L;
    const int per[3] = {px, py, pz};
    nlev_init(&L, nx, ny, nz, per, h);
    L.sig = (double*)sig;
    gs_level(&L, phi, f, nsweeps);
}

/* f_n = D_n(beta0 U) - (beta0 S)_n for cell-centred u, v, w, S (nz,ny,nx). */
void nod_rhs(int nx, int ny, int nz, int px, int py, int pz, double h, const double* b0c, const double* u,
             const double* v, const double* w, const double* S, double* f) {
    nlev L;
    const int per[3] = {px, py, pz};
    nlev_init(&L, nx, ny, nz, per, h);
    const int nc[3] = {nx, ny, nz};
    for (int K = 0; K < L.Nz; ++K)
        for (int J = 0; J < L.Ny; ++J)
            for (int I = 0; I < L.Nx; ++I) {
                const int X[3] = {I, J, K};
                double div = 0.0, src = 0.0;
                for (int sz = 0; sz < 2; ++sz)
                    for (int sy = 0; sy < 2; ++sy)
                        for (int sx = 0; sx < 2; ++sx) {
                            int S3[3] = {sx, sy, sz}, c[3], ok = 1;
                            for (int d = 0; d < 3; ++d) {
                                c[d] = cell_of(X[d], S3[d], nc[d], per[d]);
                                if (c[d] < 0) ok = 0;
                            }
                            if (!ok) continue;
                            size_t cc = CIc(&L, c[0], c[1], c[2]);
                            double b = b0c[c[2]];
                            /* + for a cell on the high side of the node (s = 1) */
                            div += b * ((sx ? u[cc] : -u[cc]) + (sy ? v[cc] : -v[cc]) + (sz ? w[cc] : -w[cc]));
                            src += b * S[cc];
                        }
                f[NI(&L, I, J, K)] = div / (4.0 * h) - 0.125 * src;
            }
}

/* U_c -= (1/rho_c) (G phi)_c, the cell's mean gradient of the nodal phi. */
void nod_correct(int nx, int ny, int nz, int px, int py, int pz, double h, const double* rho, const double* phi,
                 double* u, double* v, double* w) {
    nlev L;
    const int per[3] = {px, py, pz};
    nlev_init(&L, nx, ny, nz, per, h);
    const int Nn[3] = {L.Nx, L.Ny, L.Nz};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int lo[3] = {i, j, k};
                int hi[3];
                for (int d = 0; d < 3; ++d) hi[d] = node_of(lo[d], 1, Nn[d], per[d]);
                double g[3] = {0.0, 0.0, 0.0};
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        /* x-edge at (y, z) corner (a, b) */
                        int y = a ? hi[1] : lo[1], z = b ? hi[2] : lo[2];
                        g[0] += phi[NI(&L, hi[0], y, z)] - phi[NI(&L, lo[0], y, z)];
                        int x = a ? hi[0] : lo[0];
                        g[1] += phi[NI(&L, x, hi[1], z)] - phi[NI(&L, x, lo[1], z)];
                        int yy = b ? hi[1] : lo[1];
                        g[2] += phi[NI(&L, x, yy, hi[2])] - phi[NI(&L, x, yy, lo[2])];
                    }
                size_t c = CIc(&L, i, j, k);
                u[c] -= (g[0] / (4.0 * h)) / rho[c];
                v[c] -= (g[1] / (4.0 * h)) / rho[c];
                w[c] -= (g[2] / (4.0 * h)) / rho[c];
            }
}

/* The whole nodal projection.  stats: [0] cycles, [1] rel resid, [2] mean
 * removed from f, [3] sum f, [4] sum |f|, [5] ||f|| after mean removal. */
int nod_project(int nx, int ny, int nz, int px, int py, int pz, double h, const double* rho, const double* b0c,
                const double* S, double* u, double* v, double* w, double* phi_out, double rtol, int max_cycles,
                int nu1, int nu2, int mode, double* hist, int hist_len, double* stats) {
    size_t N = (size_t)nx * ny * nz;
    for (size_t c = 0; c < N; ++c) {
        if (!isfinite(rho[c]) || !isfinite(S[c]) || !isfinite(u[c]) || !isfinite(v[c]) || !isfinite(w[c]))
            return NOD_ERR_NONFINITE;
        if (!(rho[c] > 0.0)) return NOD_ERR_INVALID;
    }
    for (int k = 0; k < nz; ++k)
        if (!(b0c[k] > 0.0)) return NOD_ERR_INVALID;
    nlev L;
    const int per[3] = {px, py, pz};
    nlev_init(&L, nx, ny, nz, per, h);
    size_t NN = nnodes(&L);
    double* sig = (double*)malloc(N * sizeof(double));
    double* f = (double*)malloc(NN * sizeof(double));
    if (!sig || !f) { free(sig); free(f); return NOD_ERR_OOM; }
    nod_sigma(nx, ny, nz, rho, b0c, sig);
    nod_rhs(nx, ny, nz, px, py, pz, h, b0c, u, v, w, S, f);
    double sf = 0.0, saf = 0.0;
    for (size_t n = 0; n < NN; ++n) { sf += f[n]; saf += fabs(f[n]); }
    stats[3] = sf; stats[4] = saf;
    int status;
    if (fabs(sf) > 1e-8 * saf) { status = NOD_ERR_INCOMPATIBLE; goto done; }
    {
        double mean = sf / (double)NN;
        for (size_t n = 0; n < NN; ++n) f[n] -= mean;
        stats[2] = mean;
        stats[5] = norm2(f, NN);
        int st = 0;
        void* M = nod_mg_create(nx, ny, nz, px, py, pz, h, sig, &st);
        if (!M) { status = st; goto done; }
        int cyc = 0;
        status = nod_mg_solve(M, f, phi_out, rtol, max_cycles, nu1, nu2, mode, hist, hist_len, &cyc);
        stats[0] = cyc;
        stats[1] = cyc < hist_len ? hist[cyc] : NAN;
        nod_mg_destroy(M);
    }
    if (status == NOD_OK || status == NOD_ERR_NOT_CONVERGED) nod_correct(nx, ny, nz, px, py, pz, h, rho, phi_out, u, v, w);
done:
    free(sig); free(f);
    return status;
}
