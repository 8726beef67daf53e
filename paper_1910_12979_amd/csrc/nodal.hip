// Nodal (cell-velocity) projection for gfx950: phi on the cell corners,
// cell-centred velocities, the same divergence constraint as the MAC
// projection (arXiv:1910.12979, Sec. 2), solved by multigrid (Sec. 3).
//
// Discretisation: trilinear elements on the nodes with a cell-constant
// coefficient sigma = beta0 / rho.  Divided by the node volume h^3,
//   (L phi)_n = 1/(12 h^2) sum_{cells c at n} sigma_c
//               [ sum of phi over the 4 corners of c across a face or the body
//                 diagonal from n  -  4 phi_n ]
// (corners joined to n by an edge have weight 0 in the element stiffness),
//   f_n = 1/(4h) sum_c beta0_c (+-u_c +- v_c +- w_c) - 1/8 sum_c beta0_c S_c
// (+ for a cell on the high side of n in that direction), and the cells'
// velocities are corrected by their mean gradient of phi over rho.  A solid
// wall is a natural boundary (its nodes are unknowns, only existing cells
// contribute); in a periodic direction node n is node 0.
//
// Multigrid: four-colour Gauss-Seidel, colour (J mod 2) + 2 (K mod 2) in the
// order 0..3 (one launch per colour: coupled nodes differ by one in at least
// two coordinates, so in J or K, and their colours differ; each x-row has one
// colour, so a launch reads and writes whole rows); residual, full-weighting
// restriction 1/8 sum_d prod(1 - |d_i|/2) r_{2C+d}; trilinear prolongation;
// coarse sigma the mean of the 8 fine cells; exact coarsest solve (at most
// 512 nodes) by the dense inverse of -A + c 1 1^T.  Every per-node
// expression is evaluated in one fixed order, without FMA contraction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "dense.h"
#include "mg_internal.h"
#include "runtime.h"

namespace mg {
namespace {

constexpr int kNodBlock = 256;
constexpr int kNodSetupThreads = 1024;

// One level of the nodal hierarchy: cells (nx, ny, nz), nodes (Nx, Ny, Nz).
struct NodLevel {
    int nx, ny, nz;
    int Nx, Ny, Nz;
    int px, py, pz;
    double h;
    double* sig;        // cells
    double* phi;        // nodes
    double* f;
    double* r;
    __host__ __device__ size_t nodes() const { return (size_t)Nx * Ny * Nz; }
    __host__ __device__ size_t cells() const { return (size_t)nx * ny * nz; }
};

__device__ inline int nod_cell(int I, int s, int n, int per) {
    int c = s ? I : I - 1;
    if (per) return c < 0 ? c + n : (c >= n ? c - n : c);
    return (c >= 0 && c < n) ? c : -1;
}

__device__ inline int nod_node(int I, int o, int N, int per) {
    int m = I + o;
    if (per) return m < 0 ? m + N : (m >= N ? m - N : m);
    return (m >= 0 && m < N) ? m : -1;
}

__device__ inline size_t nidx(const NodLevel& L, int I, int J, int K) {
    return ((size_t)K * L.Ny + J) * L.Nx + I;
}

__device__ inline size_t cidx3(const NodLevel& L, int i, int j, int k) {
    return ((size_t)k * L.ny + j) * L.nx + i;
}

// Neighbour and cell indices of node coordinate X along one direction:
// nodes X-1 / X+1 (m[0], m[1]) and the cells on its low / high side (c[0],
// c[1], e[s] = whether that cell exists).
struct NodAxis {
    int m[2], c[2];
    bool e[2];
};

__device__ inline NodAxis nod_axis(int X, int N, int n, int per) {
    NodAxis a;
    if (per) {
        a.m[0] = X > 0 ? X - 1 : N - 1;
        a.m[1] = X + 1 < N ? X + 1 : 0;
        a.c[0] = X > 0 ? X - 1 : n - 1;
        a.c[1] = X;
        a.e[0] = a.e[1] = true;
    } else {
        a.m[0] = X - 1;
        a.m[1] = X + 1;
        a.c[0] = X - 1;
        a.c[1] = X;
        a.e[0] = X >= 1;
        a.e[1] = X < n;
    }
    return a;
}

// The 20 neighbours of node (I, J, K) that the stencil couples (moved in at
// least two directions), each loaded once: v[dz+1][dy+1][dx+1]; entries
// whose node does not exist (beyond a wall) are never used and stay 0.
struct NodNbr {
    double v[3][3][3];
};

__device__ inline void nod_load_nbrs(const NodLevel& L, const double* __restrict__ phi, int I, const NodAxis& ax,
                                     const NodAxis& ay, const NodAxis& az, int J, int K, NodNbr& N) {
    const long long Nx = L.Nx, NxNy = (long long)L.Nx * L.Ny;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
            for (int dx = -1; dx <= 1; ++dx) {
                if ((dx != 0) + (dy != 0) + (dz != 0) < 2) continue;
                const bool ok = (dx == 0 || ax.e[dx > 0]) && (dy == 0 || ay.e[dy > 0]) && (dz == 0 || az.e[dz > 0]);
                const long long xi = dx == 0 ? I : ax.m[dx > 0];
                const long long yi = dy == 0 ? J : ay.m[dy > 0];
                const long long zi = dz == 0 ? K : az.m[dz > 0];
                N.v[dz + 1][dy + 1][dx + 1] = ok ? phi[zi * NxNy + yi * Nx + xi] : 0.0;
            }
}

// num = sum_c sigma_c sum_{4 far corners} phi, den = 4 sum_c sigma_c over
// the existing cells at node (I, J, K), in the oracle's order (cells sz, sy,
// sx; far corners of the cell on side (sx, sy, sz): x+y, x+z, y+z, x+y+z
// moved), with per-axis index tables and each neighbour loaded once.
__device__ inline void nod_stencil_fast(const NodLevel& L, const double* __restrict__ phi, int I, int J, int K,
                                        double& num, double& den) {
    const NodAxis ax = nod_axis(I, L.Nx, L.nx, L.px);
    const NodAxis ay = nod_axis(J, L.Ny, L.ny, L.py);
    const NodAxis az = nod_axis(K, L.Nz, L.nz, L.pz);
    NodNbr N;
    nod_load_nbrs(L, phi, I, ax, ay, az, J, K, N);
    const long long nx = L.nx, nxny = (long long)L.nx * L.ny;
    num = 0.0;
    den = 0.0;
#pragma unroll
    for (int sz = 0; sz < 2; ++sz) {
        if (!az.e[sz]) continue;
        const int oz = sz ? 2 : 0;
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
            if (!ay.e[sy]) continue;
            const int oy = sy ? 2 : 0;
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
                if (!ax.e[sx]) continue;
                const int ox = sx ? 2 : 0;
                const double sig = L.sig[az.c[sz] * nxny + ay.c[sy] * nx + ax.c[sx]];
                double acc = 0.0;
                acc += N.v[1][oy][ox];
                acc += N.v[oz][1][ox];
                acc += N.v[oz][oy][1];
                acc += N.v[oz][oy][ox];
                num += sig * acc;
                den += 4.0 * sig;
            }
        }
    }
}

__device__ inline void block_row(double v0, double v1, double v2, double v3, double* out) {
    __shared__ double sh[4][kNodBlock];
    const int t = threadIdx.y * blockDim.x + threadIdx.x;
    sh[0][t] = v0;
    sh[1][t] = v1;
    sh[2][t] = v2;
    sh[3][t] = v3;
    __syncthreads();
    for (int s = kNodBlock / 2; s > 0; s >>= 1) {
        if (t < s) {
            sh[0][t] = sh[0][t] + sh[0][t + s];
            sh[1][t] = sh[1][t] + sh[1][t + s];
            sh[2][t] = fmax(sh[2][t], sh[2][t + s]);
            sh[3][t] = sh[3][t] + sh[3][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = sh[0][0];
        out[1] = sh[1][0];
        out[2] = sh[2][0];
        out[3] = sh[3][0];
    }
}

// Point loops of the reductions: 64 x 4 threads per workgroup over (x, y),
// the workgroups of a launch striding over x, y and the planes; no
// per-thread index division.  The partial row of a workgroup is its flat
// index.
constexpr int kPtX = 64, kPtY = 4;
__device__ inline int part_row() { return (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x; }

// sigma = beta0 / rho per cell; partial rows {0, 0, bad, #non-finite} of
// rho, beta0, S and the three velocity components.
__global__ __launch_bounds__(kNodBlock) void k_nod_sigma(NodLevel L, const double* __restrict__ rho,
                                                         const double* __restrict__ b0c,
                                                         const double* __restrict__ S, const double* __restrict__ u,
                                                         const double* __restrict__ v, const double* __restrict__ w,
                                                         double* __restrict__ partials) {
    double bad = 0.0, nonfin = 0.0;
    for (int k = blockIdx.z; k < L.nz; k += gridDim.z)
    for (int j = blockIdx.y * kPtY + threadIdx.y; j < L.ny; j += gridDim.y * kPtY)
    for (int i = blockIdx.x * kPtX + threadIdx.x; i < L.nx; i += gridDim.x * kPtX) {
        const size_t c = cidx3(L, i, j, k);
        const double r = rho[c], b = b0c[k];
        if (!isfinite(r) || !isfinite(b)) nonfin += 1.0;
        if (S && (!isfinite(S[c]) || !isfinite(u[c]) || !isfinite(v[c]) || !isfinite(w[c]))) nonfin += 1.0;
        if (!(r > 0.0) || !(b > 0.0)) bad = 1.0;
        L.sig[c] = b / r;
    }
    block_row(0.0, 0.0, bad, nonfin, partials + (size_t)part_row() * kReduceWidth);
}

// f_n and partial rows {sum f, sum |f|, 0, 0}.
__global__ __launch_bounds__(kNodBlock) void k_nod_rhs(NodLevel L, const double* __restrict__ b0c,
                                                       const double* __restrict__ u, const double* __restrict__ v,
                                                       const double* __restrict__ w, const double* __restrict__ S,
                                                       double* __restrict__ partials) {
    const int nc[3] = {L.nx, L.ny, L.nz}, per[3] = {L.px, L.py, L.pz};
    double sf = 0.0, saf = 0.0;
    for (int K = blockIdx.z; K < L.Nz; K += gridDim.z)
    for (int J = blockIdx.y * kPtY + threadIdx.y; J < L.Ny; J += gridDim.y * kPtY)
    for (int I = blockIdx.x * kPtX + threadIdx.x; I < L.Nx; I += gridDim.x * kPtX) {
        const size_t n = nidx(L, I, J, K);
        const int X[3] = {I, J, K};
        double div = 0.0, src = 0.0;
        for (int sz = 0; sz < 2; ++sz)
            for (int sy = 0; sy < 2; ++sy)
                for (int sx = 0; sx < 2; ++sx) {
                    const int S3[3] = {sx, sy, sz};
                    int c[3];
                    bool ok = true;
                    for (int d = 0; d < 3; ++d) {
                        c[d] = nod_cell(X[d], S3[d], nc[d], per[d]);
                        if (c[d] < 0) ok = false;
                    }
                    if (!ok) continue;
                    const size_t cc = cidx3(L, c[0], c[1], c[2]);
                    const double b = b0c[c[2]];
                    div += b * ((sx ? u[cc] : -u[cc]) + (sy ? v[cc] : -v[cc]) + (sz ? w[cc] : -w[cc]));
                    src += b * S[cc];
                }
        const double fn = div / (4.0 * L.h) - 0.125 * src;
        L.f[n] = fn;
        sf += fn;
        saf += fabs(fn);
    }
    block_row(sf, saf, 0.0, 0.0, partials + (size_t)part_row() * kReduceWidth);
}

// One colour of the Gauss-Seidel sweep; thread (I, tj, tk) owns node
// (I, 2 tj + (col & 1), 2 tk + (col >> 1)).
__global__ void k_nod_gs(NodLevel L, int col) {
    const int I = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int J = 2 * (int)(blockIdx.y * blockDim.y + threadIdx.y) + (col & 1);
    const int K = 2 * (int)(blockIdx.z * blockDim.z + threadIdx.z) + (col >> 1);
    if (I >= L.Nx || J >= L.Ny || K >= L.Nz) return;
    double num, den;
    nod_stencil_fast(L, L.phi, I, J, K, num, den);
    const size_t n = nidx(L, I, J, K);
    L.phi[n] = (num - 12.0 * (L.h * L.h) * L.f[n]) / den;
}

// (L phi)_n = 1/(12 h^2) sum_c sigma_c (far corners - 4 phi_n), per cell in
// the oracle's order.
__device__ inline double nod_apply(const NodLevel& L, const double* __restrict__ phi, int I, int J, int K) {
    const NodAxis ax = nod_axis(I, L.Nx, L.nx, L.px);
    const NodAxis ay = nod_axis(J, L.Ny, L.ny, L.py);
    const NodAxis az = nod_axis(K, L.Nz, L.nz, L.pz);
    NodNbr N;
    nod_load_nbrs(L, phi, I, ax, ay, az, J, K, N);
    const long long nx = L.nx, nxny = (long long)L.nx * L.ny;
    const double pn = phi[((long long)K * L.Ny + J) * L.Nx + I];
    double s = 0.0;
#pragma unroll
    for (int sz = 0; sz < 2; ++sz) {
        if (!az.e[sz]) continue;
        const int oz = sz ? 2 : 0;
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
            if (!ay.e[sy]) continue;
            const int oy = sy ? 2 : 0;
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
                if (!ax.e[sx]) continue;
                const int ox = sx ? 2 : 0;
                const double sig = L.sig[az.c[sz] * nxny + ay.c[sy] * nx + ax.c[sx]];
                double acc = 0.0;
                acc += N.v[1][oy][ox];
                acc += N.v[oz][1][ox];
                acc += N.v[oz][oy][1];
                acc += N.v[oz][oy][ox];
                s += sig * (acc - 4.0 * pn);
            }
        }
    }
    return s / (12.0 * L.h * L.h);
}

// r = f - L phi into L.r; partial rows {sum r^2, 0, max |r|, #non-finite}
// when partials != null.
__global__ __launch_bounds__(kNodBlock) void k_nod_resid(NodLevel L, double* __restrict__ partials) {
    double s = 0.0, mx = 0.0, nonfin = 0.0;
    for (int K = blockIdx.z; K < L.Nz; K += gridDim.z)
    for (int J = blockIdx.y * kPtY + threadIdx.y; J < L.Ny; J += gridDim.y * kPtY)
    for (int I = blockIdx.x * kPtX + threadIdx.x; I < L.Nx; I += gridDim.x * kPtX) {
        const size_t n = nidx(L, I, J, K);
        const double r = L.f[n] - nod_apply(L, L.phi, I, J, K);
        L.r[n] = r;
        if (!isfinite(r)) nonfin += 1.0;
        s += r * r;
        mx = fmax(mx, fabs(r));
    }
    if (partials) block_row(s, 0.0, mx, nonfin, partials + (size_t)part_row() * kReduceWidth);
}

// coarse f = 1/8 sum_d w(d) r_{2C+d} (existing fine nodes), coarse phi = 0.
__global__ void k_nod_restrict(NodLevel F, NodLevel C) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= C.Nx || J >= C.Ny || K >= C.Nz) return;
    const int X[3] = {2 * I, 2 * J, 2 * K};
    const int Nn[3] = {F.Nx, F.Ny, F.Nz}, per[3] = {F.px, F.py, F.pz};
    double s = 0.0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int D[3] = {dx, dy, dz};
                int m[3];
                bool ok = true;
                double w = 1.0;
                for (int d = 0; d < 3; ++d) {
                    m[d] = nod_node(X[d], D[d], Nn[d], per[d]);
                    if (m[d] < 0) ok = false;
                    if (D[d] != 0) w *= 0.5;
                }
                if (ok) s += w * F.r[nidx(F, m[0], m[1], m[2])];
            }
    const size_t c = nidx(C, I, J, K);
    C.f[c] = 0.125 * s;
    C.phi[c] = 0.0;
}

// fine phi += trilinear interpolation of the coarse phi.
__global__ void k_nod_prolong(NodLevel F, NodLevel C) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= F.Nx || J >= F.Ny || K >= F.Nz) return;
    const int X[3] = {I, J, K};
    const int Nc[3] = {C.Nx, C.Ny, C.Nz}, per[3] = {C.px, C.py, C.pz};
    double v = 0.0;
    for (int bz = 0; bz < 2; ++bz)
        for (int by = 0; by < 2; ++by)
            for (int bx = 0; bx < 2; ++bx) {
                const int B[3] = {bx, by, bz};
                int m[3];
                bool ok = true;
                double w = 1.0;
                for (int d = 0; d < 3; ++d) {
                    if ((X[d] & 1) == 0) {
                        if (B[d]) {
                            ok = false;
                            break;
                        }
                        m[d] = X[d] >> 1;
                    } else {
                        m[d] = B[d] ? (X[d] + 1) >> 1 : (X[d] - 1) >> 1;
                        if (per[d] && m[d] >= Nc[d]) m[d] -= Nc[d];
                        w *= 0.5;
                    }
                }
                if (ok) v += w * C.phi[nidx(C, m[0], m[1], m[2])];
            }
    const size_t n = nidx(F, I, J, K);
    F.phi[n] = F.phi[n] + v;
}

__global__ void k_nod_avg_sigma(NodLevel F, NodLevel C) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= C.nx || j >= C.ny || k >= C.nz) return;
    double s = 0.0;
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) s += F.sig[cidx3(F, 2 * i + di, 2 * j + dj, 2 * k + dk)];
    C.sig[cidx3(C, i, j, k)] = 0.125 * s;
}

// Coarsest level: M = -A + c 1 1^T (c the mean diagonal), inverted in place.
// Row n of -A: -(1/(12 h^2)) sum_c sigma_c (far corners - 4 e_n).
__global__ __launch_bounds__(kNodSetupThreads) void k_nod_coarse_setup(NodLevel L, double* __restrict__ M) {
    __shared__ double fac[kCoarseMax], prow[kCoarseMax];
    __shared__ double shift;
    const int n = (int)L.nodes();
    const int tid = threadIdx.x, nt = blockDim.x;
    const double s12 = 1.0 / (12.0 * L.h * L.h);
    for (int e = tid; e < n * n; e += nt) M[e] = 0.0;
    __syncthreads();
    for (int r = tid; r < n; r += nt) {
        const int I = r % L.Nx, J = (r / L.Nx) % L.Ny, K = r / (L.Nx * L.Ny);
        const int X[3] = {I, J, K};
        const int Nn[3] = {L.Nx, L.Ny, L.Nz}, nc[3] = {L.nx, L.ny, L.nz}, per[3] = {L.px, L.py, L.pz};
        double* row = M + (size_t)r * n;
        for (int sz = 0; sz < 2; ++sz)
            for (int sy = 0; sy < 2; ++sy)
                for (int sx = 0; sx < 2; ++sx) {
                    const int S[3] = {sx, sy, sz};
                    int c[3];
                    bool ok = true;
                    for (int d = 0; d < 3; ++d) {
                        c[d] = nod_cell(X[d], S[d], nc[d], per[d]);
                        if (c[d] < 0) ok = false;
                    }
                    if (!ok) continue;
                    const double sig = L.sig[cidx3(L, c[0], c[1], c[2])];
                    row[r] += 4.0 * sig * s12;
                    for (int mz = 0; mz < 2; ++mz)
                        for (int my = 0; my < 2; ++my)
                            for (int mx = 0; mx < 2; ++mx) {
                                if (mx + my + mz < 2) continue;
                                const int Mo[3] = {mx, my, mz};
                                int m[3];
                                for (int d = 0; d < 3; ++d)
                                    m[d] = nod_node(X[d], Mo[d] ? (S[d] ? 1 : -1) : 0, Nn[d], per[d]);
                                row[nidx(L, m[0], m[1], m[2])] -= sig * s12;
                            }
                }
    }
    __syncthreads();
    if (tid == 0) {
        double d = 0.0;
        for (int c = 0; c < n; ++c) d += M[(size_t)c * n + c];
        shift = d / n;
    }
    __syncthreads();
    for (int e = tid; e < n * n; e += nt) M[e] += shift;
    gj_invert(M, n, fac, prow);
}

// U_c -= (G phi)_c / rho_c with phi - mean (mean = *phi_sum / nodes); phi_out
// (nullable) = phi - mean at the nodes (written by the threads of the first
// nodes).
__global__ void k_nod_correct(NodLevel L, const double* __restrict__ rho, const double* __restrict__ phi_sum,
                              double* __restrict__ u, double* __restrict__ v, double* __restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= L.nx || j >= L.ny || k >= L.nz) return;
    const double m = phi_sum[0] / (double)L.nodes();
    const int lo[3] = {i, j, k};
    const int Nn[3] = {L.Nx, L.Ny, L.Nz}, per[3] = {L.px, L.py, L.pz};
    int hi[3];
    for (int d = 0; d < 3; ++d) hi[d] = nod_node(lo[d], 1, Nn[d], per[d]);
    auto P = [&](int x, int y, int z) { return L.phi[nidx(L, x, y, z)] - m; };
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int y = a ? hi[1] : lo[1], z = b ? hi[2] : lo[2];
            g0 += P(hi[0], y, z) - P(lo[0], y, z);
            const int x = a ? hi[0] : lo[0];
            g1 += P(x, hi[1], z) - P(x, lo[1], z);
            const int yy = b ? hi[1] : lo[1];
            g2 += P(x, yy, hi[2]) - P(x, yy, lo[2]);
        }
    const size_t c = cidx3(L, i, j, k);
    const double h4 = 4.0 * L.h;
    u[c] = u[c] - (g0 / h4) / rho[c];
    v[c] = v[c] - (g1 / h4) / rho[c];
    w[c] = w[c] - (g2 / h4) / rho[c];
}

__global__ void k_nod_shift_out(size_t n, const double* __restrict__ phi, const double* __restrict__ phi_sum,
                                double* __restrict__ out) {
    const double m = phi_sum[0] / (double)n;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        out[e] = phi[e] - m;
}

// Grid of a point loop over an X x Y x Z box: at most 2048 workgroups (the
// partial rows), the planes shared out among them.
inline dim3 point_grid(int X, int Y, int Z) {
    const int gx = std::min((X + kPtX - 1) / kPtX, 2048);
    const int gy = std::max(1, std::min((Y + kPtY - 1) / kPtY, 2048 / gx));
    const int gz = std::max(1, std::min(Z, 2048 / (gx * gy)));
    return dim3(gx, gy, gz);
}
inline int grid_blocks(dim3 g) { return (int)(g.x * g.y * g.z); }

inline int nod_partial_blocks(size_t N) {
    size_t b = (N + kNodBlock - 1) / kNodBlock;
    return (int)std::min<size_t>(b, 2048);
}

inline dim3 grid3(int x, int y, int z, dim3 block) {
    return dim3((x + block.x - 1) / block.x, (y + block.y - 1) / block.y, (z + block.z - 1) / block.z);
}

}  // namespace
}  // namespace mg

// ============================================================================
// host side: hierarchy and C ABI
// ============================================================================
using namespace mg;

struct nodal_hierarchy {
    mg_params p{};
    int nlev = 0;
    NodLevel lev[kMaxLevels];
    void* ws = nullptr;
    double* minv = nullptr;
    double* partials = nullptr;
    double* scal = nullptr;
    double* host = nullptr;
    bool coeffs_valid = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // One V-cycle plus the finest residual norm (copied to host) as a
    // replayable hipGraph on the hierarchy's own stream; every buffer is
    // fixed, so one capture serves every cycle of every solve with the same
    // sweep counts.
    bool graphs_on = true;
    hipStream_t gstream = nullptr;
    hipEvent_t gev = nullptr;
    hipGraphExec_t cycle_exec = nullptr;
    int cycle_pre = -1, cycle_post = -1;
};

namespace {

int nod_count_levels(const mg_params* p) {
    int nx = p->n[0], ny = p->n[1], nz = p->n[2];
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    int n = 1;
    while (nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0 && (long long)nx * ny * nz > kCoarsenMin && n < kMaxLevels) {
        nx /= 2;
        ny /= 2;
        nz /= 2;
        ++n;
    }
    const long long nodes = (long long)(nx + (p->bc[0] == MG_BC_PERIODIC ? 0 : 1)) *
                            (ny + (p->bc[1] == MG_BC_PERIODIC ? 0 : 1)) * (nz + (p->bc[2] == MG_BC_PERIODIC ? 0 : 1));
    return nodes <= kCoarseMax ? n : 0;
}

#define NHIP(expr)                                                        \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr, __LINE__);       \
    } while (0)

int nod_reduce(nodal_hierarchy* H, int nparts, int slot, hipStream_t st) {
    NHIP(launch_reduce(H->partials, nparts, H->scal + slot * kReduceWidth, st));
    NHIP(hipMemcpyAsync(H->host + slot * kReduceWidth, H->scal + slot * kReduceWidth, kReduceWidth * sizeof(double),
                        hipMemcpyDeviceToHost, st));
    NHIP(hipStreamSynchronize(st));
    return MG_OK;
}

int nod_smooth(nodal_hierarchy* H, int l, int nsweeps, hipStream_t st) {
    const NodLevel& L = H->lev[l];
    const dim3 block(64, 2, 2);
    const dim3 grid = grid3(L.Nx, (L.Ny + 1) / 2, (L.Nz + 1) / 2, block);
    for (int s = 0; s < nsweeps; ++s)
        for (int col = 0; col < 4; ++col) hipLaunchKernelGGL(k_nod_gs, grid, block, 0, st, L, col);
    NHIP(hipGetLastError());
    return MG_OK;
}

int nod_resid_restrict(nodal_hierarchy* H, int l, hipStream_t st) {
    const NodLevel& F = H->lev[l];
    const NodLevel& C = H->lev[l + 1];
    hipLaunchKernelGGL(k_nod_resid, point_grid(F.Nx, F.Ny, F.Nz), dim3(kPtX, kPtY), 0, st, F, (double*)nullptr);
    const dim3 block(32, 4, 2);
    hipLaunchKernelGGL(k_nod_restrict, grid3(C.Nx, C.Ny, C.Nz, block), block, 0, st, F, C);
    NHIP(hipGetLastError());
    return MG_OK;
}

int nod_prolong(nodal_hierarchy* H, int l, hipStream_t st) {
    const NodLevel& F = H->lev[l];
    const NodLevel& C = H->lev[l + 1];
    const dim3 block(32, 4, 2);
    hipLaunchKernelGGL(k_nod_prolong, grid3(F.Nx, F.Ny, F.Nz, block), block, 0, st, F, C);
    NHIP(hipGetLastError());
    return MG_OK;
}

int nod_vcycle(nodal_hierarchy* H, int l, hipStream_t st) {
    if (l == H->nlev - 1) {
        const NodLevel& L = H->lev[l];
        NHIP(launch_coarse_solve((int)L.nodes(), H->minv, L.f, L.phi, st, 1));
        return MG_OK;
    }
    int rc = nod_smooth(H, l, H->p.pre_sweeps, st);
    if (rc) return rc;
    rc = nod_resid_restrict(H, l, st);
    if (rc) return rc;
    rc = nod_vcycle(H, l + 1, st);
    if (rc) return rc;
    rc = nod_prolong(H, l, st);
    if (rc) return rc;
    return nod_smooth(H, l, H->p.post_sweeps, st);
}

// sigma on every level from rho and beta0, coarsest inverse; partial rows
// of the input checks reduced into slot kSlotRhs (bad, #non-finite).
int nod_coefficients(nodal_hierarchy* H, const double* rho, const double* b0c, const double* S, const double* u,
                     const double* v, const double* w, hipStream_t st) {
    const NodLevel& L0 = H->lev[0];
    const dim3 sg = point_grid(L0.nx, L0.ny, L0.nz);
    const int nb = grid_blocks(sg);
    hipLaunchKernelGGL(k_nod_sigma, sg, dim3(kPtX, kPtY), 0, st, L0, rho, b0c, S, u, v, w, H->partials);
    NHIP(hipGetLastError());
    int rc = nod_reduce(H, nb, kSlotRhs, st);
    if (rc) return rc;
    const dim3 block(32, 4, 2);
    for (int l = 0; l + 1 < H->nlev; ++l) {
        const NodLevel& C = H->lev[l + 1];
        hipLaunchKernelGGL(k_nod_avg_sigma, grid3(C.nx, C.ny, C.nz, block), block, 0, st, H->lev[l], C);
    }
    hipLaunchKernelGGL(k_nod_coarse_setup, dim3(1), dim3(kNodSetupThreads), 0, st, H->lev[H->nlev - 1], H->minv);
    NHIP(hipGetLastError());
    const double* q = H->host + kSlotRhs * kReduceWidth;
    if (q[3] > 0.0) {
        set_error("non-finite value in rho, beta0, U or S");
        return MG_ERR_NONFINITE;
    }
    if (q[2] > 0.0) {
        set_error("rho and beta0 must be positive");
        return MG_ERR_INVALID_ARG;
    }
    H->coeffs_valid = true;
    return MG_OK;
}

int nod_project(nodal_hierarchy* H, const double* rho, const double* b0c, const double* S, double* u, double* v,
                double* w, double* phi_out, mg_stats* S_, hipStream_t st) {
    std::memset(S_, 0, sizeof *S_);
    S_->nlevels = H->nlev;
    NHIP(hipEventRecord(H->ev0, st));
    int rc = nod_coefficients(H, rho, b0c, S, u, v, w, st);
    if (rc) return S_->status = rc;
    NodLevel& L0 = H->lev[0];
    const size_t NN = L0.nodes();
    const dim3 ng = point_grid(L0.Nx, L0.Ny, L0.Nz);
    const int nb = grid_blocks(ng);
    hipLaunchKernelGGL(k_nod_rhs, ng, dim3(kPtX, kPtY), 0, st, L0, b0c, u, v, w, S, H->partials);
    NHIP(hipGetLastError());
    rc = nod_reduce(H, nb, kSlotNorm, st);
    if (rc) return S_->status = rc;
    const double sf = H->host[kSlotNorm * kReduceWidth], saf = H->host[kSlotNorm * kReduceWidth + 1];
    S_->sum_f = sf;
    S_->sum_abs_f = saf;
    if (!std::isfinite(sf) || !std::isfinite(saf)) {
        set_error("non-finite right-hand side");
        return S_->status = MG_ERR_NONFINITE;
    }
    if (std::fabs(sf) > 1e-8 * saf) {
        set_error("incompatible right-hand side: |sum f| > 1e-8 sum |f|");
        return S_->status = MG_ERR_INCOMPATIBLE_RHS;
    }
    const double mean = sf / (double)NN;
    S_->mean_removed = mean;
    int np = 0;
    NHIP(launch_shift_norm(Shape{L0.Nx, L0.Ny, L0.Nz}, L0.f, mean, H->partials, &np, st));
    rc = nod_reduce(H, np, kSlotNorm, st);
    if (rc) return S_->status = rc;
    const double fnorm = std::sqrt(H->host[kSlotNorm * kReduceWidth]);
    S_->norm_f = fnorm;
    NHIP(launch_fill<double>(L0.phi, NN, 0.0, st));
    int status = MG_OK, cycles = 0;
    double rel = 0.0;
    S_->resid_hist[0] = fnorm > 0.0 ? 1.0 : 0.0;
    S_->rel_resid0 = S_->resid_hist[0];
    S_->hist_len = 1;
    // every cycle ends with a host synchronisation: the loop's wall time is
    // the device time of the cycles
    const auto t_s0 = std::chrono::steady_clock::now();
    if (fnorm > 0.0 && H->p.rtol < 1.0) {
        status = MG_ERR_NOT_CONVERGED;
        bool on_graph = false;
        auto cycle = [&](hipStream_t s) -> int {
            int r2 = nod_vcycle(H, 0, s);
            if (r2) return r2;
            hipLaunchKernelGGL(k_nod_resid, ng, dim3(kPtX, kPtY), 0, s, L0, H->partials);
            NHIP(hipGetLastError());
            NHIP(launch_reduce(H->partials, nb, H->scal + kSlotRes * kReduceWidth, s));
            NHIP(hipMemcpyAsync(H->host + kSlotRes * kReduceWidth, H->scal + kSlotRes * kReduceWidth,
                                kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, s));
            return MG_OK;
        };
        while (cycles < H->p.max_cycles) {
            if (H->graphs_on) {
                if (!H->gstream) {
                    NHIP(hipStreamCreateWithFlags(&H->gstream, hipStreamNonBlocking));
                    NHIP(hipEventCreateWithFlags(&H->gev, hipEventDisableTiming));
                }
                if (!on_graph) {                    // after the caller's earlier work
                    NHIP(hipEventRecord(H->gev, st));
                    NHIP(hipStreamWaitEvent(H->gstream, H->gev, 0));
                    on_graph = true;
                }
                if (!H->cycle_exec || H->cycle_pre != H->p.pre_sweeps || H->cycle_post != H->p.post_sweeps) {
                    if (H->cycle_exec) {
                        hipGraphExecDestroy(H->cycle_exec);
                        H->cycle_exec = nullptr;
                    }
                    NHIP(hipStreamBeginCapture(H->gstream, hipStreamCaptureModeRelaxed));
                    int r2 = cycle(H->gstream);
                    hipGraph_t g = nullptr;
                    hipError_t e = hipStreamEndCapture(H->gstream, &g);
                    if (r2) {
                        if (g) hipGraphDestroy(g);
                        return S_->status = r2;
                    }
                    if (e != hipSuccess) return S_->status = hip_fail(e, "hipStreamEndCapture", __LINE__);
                    e = hipGraphInstantiate(&H->cycle_exec, g, nullptr, nullptr, 0);
                    hipGraphDestroy(g);
                    if (e != hipSuccess) {
                        H->cycle_exec = nullptr;
                        return S_->status = hip_fail(e, "hipGraphInstantiate", __LINE__);
                    }
                    H->cycle_pre = H->p.pre_sweeps;
                    H->cycle_post = H->p.post_sweeps;
                }
                NHIP(hipGraphLaunch(H->cycle_exec, H->gstream));
                NHIP(hipStreamSynchronize(H->gstream));
            } else {
                rc = cycle(st);
                if (rc) return S_->status = rc;
                NHIP(hipStreamSynchronize(st));
            }
            ++cycles;
            const double* r = H->host + kSlotRes * kReduceWidth;
            rel = std::sqrt(r[0]) / fnorm;
            if (cycles < MG_HIST_MAX) {
                S_->resid_hist[cycles] = rel;
                S_->hist_len = cycles + 1;
            }
            if (r[3] > 0.0 || !std::isfinite(rel)) {
                set_error("non-finite residual during the solve");
                status = MG_ERR_NONFINITE;
                break;
            }
            if (rel <= H->p.rtol) {
                status = MG_OK;
                break;
            }
        }
    }
    if (H->gstream) {                       // the caller's stream continues after the graph work
        NHIP(hipEventRecord(H->gev, H->gstream));
        NHIP(hipStreamWaitEvent(st, H->gev, 0));
    }
    S_->ms_smooth = cycles > 0 ? std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_s0).count()
                               : 0.0;
    S_->cycles = cycles;
    S_->rel_resid = rel;
    if (status != MG_OK && status != MG_ERR_NOT_CONVERGED) return S_->status = status;
    NHIP(launch_sum(Shape{L0.Nx, L0.Ny, L0.Nz}, L0.phi, H->partials, &np, st));
    NHIP(launch_reduce(H->partials, np, H->scal + kSlotPhi * kReduceWidth, st));
    const double* psum = H->scal + kSlotPhi * kReduceWidth;
    const dim3 block(32, 4, 2);
    hipLaunchKernelGGL(k_nod_correct, grid3(L0.nx, L0.ny, L0.nz, block), block, 0, st, L0, rho, psum, u, v, w);
    if (phi_out)
        hipLaunchKernelGGL(k_nod_shift_out, dim3(nod_partial_blocks(NN)), dim3(kNodBlock), 0, st, NN, L0.phi, psum,
                           phi_out);
    NHIP(hipGetLastError());
    NHIP(hipEventRecord(H->ev1, st));
    NHIP(hipMemcpyAsync(H->host + kSlotPhi * kReduceWidth, psum, sizeof(double), hipMemcpyDeviceToHost, st));
    NHIP(hipStreamSynchronize(st));
    S_->phi_mean = H->host[kSlotPhi * kReduceWidth] / (double)NN;
    float ms = 0.f;
    hipEventElapsedTime(&ms, H->ev0, H->ev1);
    S_->ms_total = ms;
    S_->ms_other = std::max(0.0, S_->ms_total - S_->ms_smooth);
    S_->status = status;
    if (status == MG_ERR_NOT_CONVERGED) set_error("maximum number of cycles reached");
    return status;
}

}  // namespace

extern "C" {

int32_t nodal_num_levels_for(const mg_params* p) {
    if (!p) return 0;
    for (int d = 0; d < 3; ++d)
        if (p->bc[d] != MG_BC_PERIODIC && p->bc[d] != MG_BC_WALL) return 0;
    return nod_count_levels(p);
}

int nodal_setup(const mg_params* p, nodal_handle* out) {
    if (!out || !p) {
        set_error("null argument to nodal_setup");
        return MG_ERR_INVALID_ARG;
    }
    *out = nullptr;
    int st = validate_params(p);
    if (st != MG_OK) return st;
    for (int d = 0; d < 3; ++d)
        if (p->bc[d] != MG_BC_PERIODIC && p->bc[d] != MG_BC_WALL) {
            set_error("the nodal projection takes periodic or wall boundaries");
            return MG_ERR_INVALID_ARG;
        }
    if (p->precision != MG_FP64) {
        set_error("the nodal projection runs in FP64");
        return MG_ERR_INVALID_ARG;
    }
    const int nl = nod_count_levels(p);
    if (nl == 0) {
        set_error("shape not solvable: the coarsest nodal level would exceed 512 nodes");
        return MG_ERR_BAD_SIZE;
    }
    nodal_hierarchy* H = new (std::nothrow) nodal_hierarchy();
    if (!H) return MG_ERR_OOM;
    H->p = *p;
    H->nlev = nl;
    size_t bytes = 0;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    for (int l = 0; l < nl; ++l) {
        NodLevel& L = H->lev[l];
        L.nx = p->n[0] >> l;
        L.ny = p->n[1] >> l;
        L.nz = p->n[2] >> l;
        L.px = p->bc[0] == MG_BC_PERIODIC;
        L.py = p->bc[1] == MG_BC_PERIODIC;
        L.pz = p->bc[2] == MG_BC_PERIODIC;
        L.Nx = L.nx + (L.px ? 0 : 1);
        L.Ny = L.ny + (L.py ? 0 : 1);
        L.Nz = L.nz + (L.pz ? 0 : 1);
        L.h = p->dx * (double)(1 << l);
        bytes += al(L.cells() * 8) + 3 * al(L.nodes() * 8);
    }
    const size_t nc = H->lev[nl - 1].nodes();
    bytes += al(nc * nc * 8) + al(2048 * kReduceWidth * 8) + al(64 * 8);
    if (hipMalloc(&H->ws, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete H;
        set_error("hipMalloc of the nodal hierarchy failed");
        return MG_ERR_OOM;
    }
    char* b = (char*)H->ws;
    auto take = [&](size_t n) {
        char* q = b;
        b += al(n);
        return (double*)q;
    };
    for (int l = 0; l < nl; ++l) {
        NodLevel& L = H->lev[l];
        L.sig = take(L.cells() * 8);
        L.phi = take(L.nodes() * 8);
        L.f = take(L.nodes() * 8);
        L.r = take(L.nodes() * 8);
    }
    H->minv = take(nc * nc * 8);
    H->partials = take(2048 * kReduceWidth * 8);
    H->scal = take(64 * 8);
    if (hipHostMalloc((void**)&H->host, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
        hipFree(H->ws);
        delete H;
        set_error("hipHostMalloc failed");
        return MG_ERR_HIP;
    }
    hipEventCreate(&H->ev0);
    hipEventCreate(&H->ev1);
    *out = H;
    return MG_OK;
}

int nodal_destroy(nodal_handle h) {
    if (!h) return MG_OK;
    if (h->cycle_exec) hipGraphExecDestroy(h->cycle_exec);
    if (h->gstream) hipStreamDestroy(h->gstream);
    if (h->gev) hipEventDestroy(h->gev);
    if (h->ws) hipFree(h->ws);
    if (h->host) hipHostFree(h->host);
    hipEventDestroy(h->ev0);
    hipEventDestroy(h->ev1);
    delete h;
    return MG_OK;
}

int nodal_project(nodal_handle h, const double* rho, const double* beta0_cc, const double* S, double* uc,
                  double* vc, double* wc, double* phi, mg_stats* stats, void* stream) {
    if (!h || !rho || !beta0_cc || !S || !uc || !vc || !wc) {
        set_error("null argument to nodal_project");
        return MG_ERR_INVALID_ARG;
    }
    mg_stats local;
    try {
        return nod_project(h, rho, beta0_cc, S, uc, vc, wc, phi, stats ? stats : &local, (hipStream_t)stream);
    } catch (...) {
        set_error("internal error in nodal_project");
        return MG_ERR_HIP;
    }
}

int nodal_set_coefficients(nodal_handle h, const double* rho, const double* beta0_cc, void* stream) {
    if (!h || !rho || !beta0_cc) {
        set_error("null argument to nodal_set_coefficients");
        return MG_ERR_INVALID_ARG;
    }
    return nod_coefficients(h, rho, beta0_cc, nullptr, nullptr, nullptr, nullptr, (hipStream_t)stream);
}

int nodal_set_graphs(nodal_handle h, int32_t enable) {
    if (!h) {
        set_error("null handle");
        return MG_ERR_INVALID_ARG;
    }
    h->graphs_on = enable != 0;
    return MG_OK;
}

int nodal_level_info(nodal_handle h, int32_t level, int32_t dims[6], double* dx) {
    if (!h || level < 0 || level >= h->nlev || !dims) {
        set_error("bad nodal_level_info arguments");
        return MG_ERR_INVALID_ARG;
    }
    const NodLevel& L = h->lev[level];
    dims[0] = L.Nx;
    dims[1] = L.Ny;
    dims[2] = L.Nz;
    dims[3] = L.nx;
    dims[4] = L.ny;
    dims[5] = L.nz;
    if (dx) *dx = L.h;
    return MG_OK;
}

int nodal_level_copy(nodal_handle h, int32_t level, int32_t array, void* buffer, int32_t to_hierarchy,
                     void* stream) {
    if (!h || level < 0 || level >= h->nlev || !buffer) {
        set_error("bad nodal_level_copy arguments");
        return MG_ERR_INVALID_ARG;
    }
    const NodLevel& L = h->lev[level];
    double* a;
    size_t n;
    switch (array) {
        case MG_NOD_PHI: a = L.phi; n = L.nodes(); break;
        case MG_NOD_F: a = L.f; n = L.nodes(); break;
        case MG_NOD_SIGMA: a = L.sig; n = L.cells(); break;
        default: set_error("bad nodal array id"); return MG_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = to_hierarchy ? launch_copy(a, (const double*)buffer, n, st)
                                : launch_copy((double*)buffer, a, n, st);
    if (e != hipSuccess) return hip_fail(e, "nodal_level_copy", __LINE__);
    return MG_OK;
}

int nodal_level_step(nodal_handle h, int32_t level, int32_t step, int32_t arg, void* stream) {
    if (!h || level < 0 || level >= h->nlev) {
        set_error("bad level");
        return MG_ERR_INVALID_ARG;
    }
    if (!h->coeffs_valid) {
        set_error("nodal_level_step before nodal_set_coefficients / nodal_project");
        return MG_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    const bool has_coarse = level + 1 < h->nlev;
    switch (step) {
        case MG_STEP_SMOOTH: return nod_smooth(h, level, arg, st);
        case MG_STEP_RESID_RESTRICT:
            if (!has_coarse) break;
            return nod_resid_restrict(h, level, st);
        case MG_STEP_PROLONG:
            if (!has_coarse) break;
            return nod_prolong(h, level, st);
        case MG_STEP_COARSE: {
            if (has_coarse) break;
            const NodLevel& L = h->lev[level];
            hipLaunchKernelGGL(k_nod_coarse_setup, dim3(1), dim3(kNodSetupThreads), 0, st, L, h->minv);
            NHIP(hipGetLastError());
            NHIP(launch_coarse_solve((int)L.nodes(), h->minv, L.f, L.phi, st, 1));
            return MG_OK;
        }
        default: break;
    }
    set_error("step not available on this level");
    return MG_ERR_INVALID_ARG;
}

}  // extern "C"
