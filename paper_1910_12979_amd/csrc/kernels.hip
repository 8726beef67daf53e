// gfx950 kernels of the MAC projection: coefficients and right-hand side,
// red-black Gauss-Seidel, residual + restriction, prolongation, residual norm,
// coarsest-level direct solve and velocity correction.
//
// The operator is the cell-centred discretisation of div((beta0/rho) grad phi)
// whose right-hand side is div(beta0 U) - beta0 S (arXiv:1910.12979, Sec. 2,
// divergence constraint), solved by multigrid as the paper's projections are
// (Sec. 3).  Every kernel here is HBM-bandwidth bound: plain coalesced sweeps,
// one thread per cell, fixed-order reductions so results are reproducible.
//
// Arithmetic order inside each cell update follows the face order x-low,
// x-high, y-low, y-high, z-low, z-high; the library is compiled without FMA
// contraction so the per-cell results do not depend on which kernel variant
// (single problem, batched) evaluates them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "dense.h"
#include "devmath.h"
#include "mg_internal.h"

namespace mg {
namespace {

constexpr int kBlock = 256;          // threads per block for cell kernels
constexpr int kMaxPartialBlocks = 2048;

struct Launch3 {
    dim3 grid, block;
};

inline int pow2_at_least(int v, int cap) {
    int p = 1;
    while (p < v && p < cap) p <<= 1;
    return p;
}

// Block shape: up to 64 threads along x (one wavefront per row), the rest
// along y then z; grid covers the box.
inline Launch3 cell_launch(int nx, int ny, int nz) {
    int bx = pow2_at_least(nx, 64);
    int by = pow2_at_least(ny, kBlock / bx);
    int bz = pow2_at_least(nz, kBlock / (bx * by));
    Launch3 L;
    L.block = dim3(bx, by, bz);
    L.grid = dim3((nx + bx - 1) / bx, (ny + by - 1) / by, (nz + bz - 1) / bz);
    return L;
}

inline int partial_blocks(size_t N) {
    size_t b = (N + kBlock - 1) / kBlock;
    return (int)(b < (size_t)kMaxPartialBlocks ? b : (size_t)kMaxPartialBlocks);
}

__device__ inline size_t cidx(int i, int j, int k, int nx, int ny) {
    return ((size_t)k * ny + j) * nx + i;
}

// Reduce a row of 4 values over a 1-D block of kBlock threads: [0],[1],[3]
// summed, [2] max.  Fixed tree order.  Thread 0 writes the row.
__device__ void block_reduce_row(double v0, double v1, double v2, double v3, double* out) {
    __shared__ double sh[4][kBlock];
    int t = threadIdx.y * blockDim.x + threadIdx.x;      // kBlock threads, 1-D or 2-D
    sh[0][t] = v0;
    sh[1][t] = v1;
    sh[2][t] = v2;
    sh[3][t] = v3;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
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

__device__ inline bool finite_d(double x) { return isfinite(x); }

// ---------------------------------------------------------------------------
// Level-0 face coefficients (+ optional right-hand side).  64 x 4 threads per
// workgroup over (x, y); the workgroups stride over x, y and the planes so
// the number of partial rows stays small, with no per-cell index division.
// ---------------------------------------------------------------------------
constexpr int kPtX = 64, kPtY = 4;
// Workgroup (bx, by, bz) of a (gx, gy, gz) grid over problem a.
template <bool kRhs>
__device__ void coeff_rhs_body(const CoeffDesc& a, int bxi, int byi, int bzi) {
    const int nx = a.nx, ny = a.ny, nz = a.nz, px = a.px, py = a.py, pz = a.pz;
    const double h = a.h;
    const double* __restrict__ rho = a.rho;
    const double* __restrict__ b0c = a.b0c;
    const double* __restrict__ b0e = a.b0e;
    const double* __restrict__ S = a.S;
    const double* __restrict__ u = a.u;
    const double* __restrict__ v = a.v;
    const double* __restrict__ w = a.w;
    const double* __restrict__ w0 = a.w0;
    double* __restrict__ bx = a.bx;
    double* __restrict__ by = a.by;
    double* __restrict__ bz = a.bz;
    double* __restrict__ f = a.f;
    float* __restrict__ rho32 = a.rho32;
    double sf = 0.0, saf = 0.0, bad = 0.0, nonfin = 0.0;
    for (int k = bzi; k < nz; k += a.gz)
    for (int j = byi * kPtY + threadIdx.y; j < ny; j += a.gy * kPtY)
    for (int i = bxi * kPtX + threadIdx.x; i < nx; i += a.gx * kPtX) {
        const size_t c = cidx(i, j, k, nx, ny);
        double rc = rho[c];
        if (rho32) rho32[c] = (float)rc;
        double bk = b0c[k];
        double bek = b0e[k];
        if (!finite_d(rc) || !finite_d(bk) || !finite_d(bek)) nonfin += 1.0;
        if (!(rc > 0.0) || !(bk > 0.0) || !(bek > 0.0)) bad = 1.0;
        // x-low face i
        double cx;
        if (i > 0) cx = qdiv(bk, 0.5 * (rho[c - 1] + rc));
        else cx = px ? qdiv(bk, 0.5 * (rho[c + (nx - 1)] + rc)) : 0.0;
        // y-low face j
        double cy;
        if (j > 0) cy = qdiv(bk, 0.5 * (rho[c - nx] + rc));
        else cy = py ? qdiv(bk, 0.5 * (rho[c + (size_t)(ny - 1) * nx] + rc)) : 0.0;
        // z-low face k (periodic: face 0 uses beta0_edge[0])
        double cz;
        size_t plane = (size_t)nx * ny;
        if (k > 0) cz = qdiv(bek, 0.5 * (rho[c - plane] + rc));
        else cz = pz ? qdiv(b0e[0], 0.5 * (rho[c + (size_t)(nz - 1) * plane] + rc)) : 0.0;
        bx[c] = cx;
        by[c] = cy;
        bz[c] = cz;
        if (kRhs) {
            size_t ub = ((size_t)k * ny + j) * (nx + 1);
            double ul = u[ub + i];
            double uh = (i == nx - 1 && px) ? u[ub] : u[ub + i + 1];
            size_t vb = (size_t)k * (ny + 1) * nx + i;
            double vl = v[vb + (size_t)j * nx];
            double vh = (j == ny - 1 && py) ? v[vb] : v[vb + (size_t)(j + 1) * nx];
            size_t wc = (size_t)j * nx + i;
            double wl = w[(size_t)k * plane + wc];
            double bl = b0e[k];
            double wh, bh;
            if (k == nz - 1 && pz) {
                wh = w[wc];
                bh = b0e[0];
            } else {
                wh = w[(size_t)(k + 1) * plane + wc];
                bh = b0e[k + 1];
            }
            if (k == 0 && pz) bl = b0e[0];
            double sc = S[c];
            if (w0) sc = sc - w0[k];         // the dp0/dt term of the constraint, per layer
            if (!finite_d(ul) || !finite_d(uh) || !finite_d(vl) || !finite_d(vh) ||
                !finite_d(wl) || !finite_d(wh) || !finite_d(sc))
                nonfin += 1.0;
            double div = (bk * (uh - ul) + bk * (vh - vl) + (bh * wh - bl * wl)) / h;
            double fc = div - bk * sc;
            f[c] = fc;
            sf += fc;
            saf += fabs(fc);
        }
    }
    const int row = (bzi * a.gy + byi) * a.gx + bxi;
    block_reduce_row(sf, saf, bad, nonfin, a.partials + (size_t)row * kReduceWidth);
}

template <bool kRhs>
__global__ __launch_bounds__(kBlock) void k_coeff_rhs(CoeffDesc a) {
    coeff_rhs_body<kRhs>(a, blockIdx.x, blockIdx.y, blockIdx.z);
}

__device__ void next_scale(const double* res, double* scales, double n);

// Sum of the partial rows into out; with scales, also the next power-of-two
// scale of the FP32 residual from out[0] (next_scale), in the same launch.
__global__ __launch_bounds__(kBlock) void k_reduce(const double* __restrict__ partials, int nparts,
                                                   double* __restrict__ out, double* __restrict__ scales,
                                                   double n) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int r = threadIdx.x; r < nparts; r += kBlock) {
        const double* p = partials + (size_t)r * kReduceWidth;
        a0 += p[0];
        a1 += p[1];
        a2 = fmax(a2, p[2]);
        a3 += p[3];
    }
    block_reduce_row(a0, a1, a2, a3, out);
    if (scales && threadIdx.x == 0 && threadIdx.y == 0) next_scale(out, scales, n);   // out written by this thread
}

// Workgroup b of nb: f -= shift over its strided cells, partial row {sum f^2}.
__device__ void shift_norm_body(size_t N, double* __restrict__ f, double shift, double* __restrict__ partials,
                                int b, int nb) {
    double s = 0.0;
    for (size_t c = (size_t)b * kBlock + threadIdx.x; c < N; c += (size_t)nb * kBlock) {
        double x = f[c] - shift;
        f[c] = x;
        s += x * x;
    }
    block_reduce_row(s, 0.0, 0.0, 0.0, partials + (size_t)b * kReduceWidth);
}

__device__ void sum_body(size_t N, const double* __restrict__ a, double* __restrict__ partials, int b, int nb) {
    double s = 0.0;
    for (size_t c = (size_t)b * kBlock + threadIdx.x; c < N; c += (size_t)nb * kBlock)
        s += a[c];
    block_reduce_row(s, 0.0, 0.0, 0.0, partials + (size_t)b * kReduceWidth);
}

__global__ __launch_bounds__(kBlock) void k_shift_norm(size_t N, double* __restrict__ f, double shift,
                                                       double* __restrict__ partials) {
    shift_norm_body(N, f, shift, partials, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kBlock) void k_sum(size_t N, const double* __restrict__ a,
                                                double* __restrict__ partials) {
    sum_body(N, a, partials, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// Coarse coefficients: coarse face I <- fine face 2I, averaged over the 2x2
// fine faces it covers (orders as in the reference definition).
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void avg_coeff_cell(int nx, int ny, int I, int J, int K, int cx, int cy, const T* __restrict__ bx,
                                      const T* __restrict__ by, const T* __restrict__ bz, T* __restrict__ cbx,
                                      T* __restrict__ cby, T* __restrict__ cbz) {
    int i = 2 * I, j = 2 * J, k = 2 * K;
    size_t C = cidx(I, J, K, cx, cy);
    const T q = T(0.25);
    cbx[C] = q * (bx[cidx(i, j, k, nx, ny)] + bx[cidx(i, j + 1, k, nx, ny)] +
                  bx[cidx(i, j, k + 1, nx, ny)] + bx[cidx(i, j + 1, k + 1, nx, ny)]);
    cby[C] = q * (by[cidx(i, j, k, nx, ny)] + by[cidx(i + 1, j, k, nx, ny)] +
                  by[cidx(i, j, k + 1, nx, ny)] + by[cidx(i + 1, j, k + 1, nx, ny)]);
    cbz[C] = q * (bz[cidx(i, j, k, nx, ny)] + bz[cidx(i + 1, j, k, nx, ny)] +
                  bz[cidx(i, j + 1, k, nx, ny)] + bz[cidx(i + 1, j + 1, k, nx, ny)]);
}

// With mx non-null, also the FP32 mirrors of the coarse coefficients (the
// conversion the separate mirror pass makes).
template <typename T>
__global__ void k_avg_coeff(int nx, int ny, int nz, const T* __restrict__ bx, const T* __restrict__ by,
                            const T* __restrict__ bz, T* __restrict__ cbx, T* __restrict__ cby,
                            T* __restrict__ cbz, float* __restrict__ mx, float* __restrict__ my,
                            float* __restrict__ mz) {
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    int J = blockIdx.y * blockDim.y + threadIdx.y;
    int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= cx || J >= cy || K >= cz) return;
    avg_coeff_cell<T>(nx, ny, I, J, K, cx, cy, bx, by, bz, cbx, cby, cbz);
    if (mx) {
        const size_t C = cidx(I, J, K, cx, cy);
        mx[C] = (float)cbx[C];
        my[C] = (float)cby[C];
        mz[C] = (float)cbz[C];
    }
}

// ---------------------------------------------------------------------------
// Red-black Gauss-Seidel: one colour per launch, one thread per cell of that
// colour.  phi_c <- (sum_f b_f phi_nb - h^2 f_c) / sum_f b_f.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_rbgs_colour(int nx, int ny, int nz, T h2, T* __restrict__ phi, const T* __restrict__ f,
                              const T* __restrict__ bx, const T* __restrict__ by,
                              const T* __restrict__ bz, int colour, Bnd<T> bnd, int has_bnd) {
    int ih = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (2 * ih >= nx || j >= ny || k >= nz) return;
    int i = 2 * ih + ((j + k + colour) & 1);
    if (i >= nx) return;
    int im = i > 0 ? i - 1 : nx - 1, ip = i < nx - 1 ? i + 1 : 0;
    int jm = j > 0 ? j - 1 : ny - 1, jp = j < ny - 1 ? j + 1 : 0;
    int km = k > 0 ? k - 1 : nz - 1, kp = k < nz - 1 ? k + 1 : 0;
    size_t c = cidx(i, j, k, nx, ny);
    T bxl = bx[c], bxh = bx[cidx(ip, j, k, nx, ny)];
    T byl = by[c], byh = by[cidx(i, jp, k, nx, ny)];
    T bzl = bz[c], bzh = bz[cidx(i, j, kp, nx, ny)];
    T num = bxl * phi[cidx(im, j, k, nx, ny)];
    num = num + bxh * phi[cidx(ip, j, k, nx, ny)];
    num = num + byl * phi[cidx(i, jm, k, nx, ny)];
    num = num + byh * phi[cidx(i, jp, k, nx, ny)];
    num = num + bzl * phi[cidx(i, j, km, nx, ny)];
    num = num + bzh * phi[cidx(i, j, kp, nx, ny)];
    T den = bxl + bxh;
    den = den + byl;
    den = den + byh;
    den = den + bzl;
    den = den + bzh;
    if (has_bnd) den = den + bnd_diag(bnd, i, j, k, nx, ny, nz);
    phi[c] = qdiv(num - h2 * f[c], den);
}

// Face coefficients of a cell: stored per-cell low-face arrays (any level).
template <typename T>
struct StoredCoeff {
    const T* bx;
    const T* by;
    const T* bz;
    Bnd<T> bnd;          // outflow boundary faces (has_bnd != 0)
    int has_bnd;
    __device__ inline void get(size_t c, size_t cxp, size_t cyp, size_t czp, int, int, int, int, int, int,
                               T b[6]) const {
        b[0] = bx[c];
        b[1] = bx[cxp];
        b[2] = by[c];
        b[3] = by[cyp];
        b[4] = bz[c];
        b[5] = bz[czp];
    }
};

// Finest level: b = beta0_face / (0.5 (rho_L + rho_R)) recomputed from rho and
// beta0 with the same expression the coefficient kernel stores.
struct RhoCoeff {
    const double* rho;
    const double* b0c;
    const double* b0e;
    int nx, ny, nz, px, py, pz;
    Bnd<double> bnd;     // outflow boundary faces (has_bnd != 0)
    int has_bnd;
    // low face of the cell at flat index c (coordinates i, j, k) in direction d
    __device__ inline double low(int d, size_t c, int i, int j, int k) const {
        const size_t plane = (size_t)nx * ny;
        const double rc = rho[c];
        if (d == 0) {
            if (i > 0) return qdiv(b0c[k], 0.5 * (rho[c - 1] + rc));
            return px ? qdiv(b0c[k], 0.5 * (rho[c + (nx - 1)] + rc)) : 0.0;
        }
        if (d == 1) {
            if (j > 0) return qdiv(b0c[k], 0.5 * (rho[c - nx] + rc));
            return py ? qdiv(b0c[k], 0.5 * (rho[c + (size_t)(ny - 1) * nx] + rc)) : 0.0;
        }
        if (k > 0) return qdiv(b0e[k], 0.5 * (rho[c - plane] + rc));
        return pz ? qdiv(b0e[0], 0.5 * (rho[c + (size_t)(nz - 1) * plane] + rc)) : 0.0;
    }
    __device__ inline void get(size_t c, size_t cxp, size_t cyp, size_t czp, int i, int j, int k, int ip,
                               int jp, int kp, double b[6]) const {
        b[0] = low(0, c, i, j, k);
        b[1] = low(0, cxp, ip, j, k);
        b[2] = low(1, c, i, j, k);
        b[3] = low(1, cyp, i, jp, k);
        b[4] = low(2, c, i, j, k);
        b[5] = low(2, czp, i, j, kp);
    }
};

// The first coarse level's coefficients averaged (as k_avg_coeff does) from
// level 0's recomputed from rho: one array read instead of the three stored
// ones, which hold the same values.  With mx non-null, also the FP32 mirrors.
__global__ void k_avg_coeff_rho(RhoCoeff co, double* __restrict__ cbx, double* __restrict__ cby,
                                double* __restrict__ cbz, float* __restrict__ mx, float* __restrict__ my,
                                float* __restrict__ mz) {
    const int nx = co.nx, ny = co.ny;
    const int cx = nx / 2, cy = ny / 2, cz = co.nz / 2;
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= cx || J >= cy || K >= cz) return;
    const int i = 2 * I, j = 2 * J, k = 2 * K;
    auto b = [&](int d, int ii, int jj, int kk) { return co.low(d, cidx(ii, jj, kk, nx, ny), ii, jj, kk); };
    const size_t C = cidx(I, J, K, cx, cy);
    const double q = 0.25;
    const double vx = q * (b(0, i, j, k) + b(0, i, j + 1, k) + b(0, i, j, k + 1) + b(0, i, j + 1, k + 1));
    const double vy = q * (b(1, i, j, k) + b(1, i + 1, j, k) + b(1, i, j, k + 1) + b(1, i + 1, j, k + 1));
    const double vz = q * (b(2, i, j, k) + b(2, i + 1, j, k) + b(2, i, j + 1, k) + b(2, i + 1, j + 1, k));
    cbx[C] = vx;
    cby[C] = vy;
    cbz[C] = vz;
    if (mx) {
        mx[C] = (float)vx;
        my[C] = (float)vy;
        mz[C] = (float)vz;
    }
}

// (L phi)_c = (sum_f b_f (phi_nb - phi_c)) / h^2, faces in the fixed order.
template <typename T, typename C>
__device__ inline T apply_cell(int i, int j, int k, int nx, int ny, int nz, T h2, const T* __restrict__ phi,
                               const C& coef) {
    int im = i > 0 ? i - 1 : nx - 1, ip = i < nx - 1 ? i + 1 : 0;
    int jm = j > 0 ? j - 1 : ny - 1, jp = j < ny - 1 ? j + 1 : 0;
    int km = k > 0 ? k - 1 : nz - 1, kp = k < nz - 1 ? k + 1 : 0;
    size_t c = cidx(i, j, k, nx, ny);
    size_t cxp = cidx(ip, j, k, nx, ny), cyp = cidx(i, jp, k, nx, ny), czp = cidx(i, j, kp, nx, ny);
    T b[6];
    coef.get(c, cxp, cyp, czp, i, j, k, ip, jp, kp, b);
    T pc = phi[c];
    T s = b[0] * (phi[cidx(im, j, k, nx, ny)] - pc);
    s = s + b[1] * (phi[cxp] - pc);
    s = s + b[2] * (phi[cidx(i, jm, k, nx, ny)] - pc);
    s = s + b[3] * (phi[cyp] - pc);
    s = s + b[4] * (phi[cidx(i, j, km, nx, ny)] - pc);
    s = s + b[5] * (phi[czp] - pc);
    if (coef.has_bnd) s = s - bnd_diag(coef.bnd, i, j, k, nx, ny, nz) * pc;
    return s * (T(1) / h2);
}

template <typename T, typename Coef>
__global__ void k_resid_restrict(int nx, int ny, int nz, T h2, const T* __restrict__ phi,
                                 const T* __restrict__ f, Coef coef, T* __restrict__ fc, T* __restrict__ phic) {
    int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    int J = blockIdx.y * blockDim.y + threadIdx.y;
    int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= cx || J >= cy || K >= cz) return;
    T s = T(0);
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                T r = f[cidx(i, j, k, nx, ny)] - apply_cell<T>(i, j, k, nx, ny, nz, h2, phi, coef);
                s = s + r;
            }
    size_t C = cidx(I, J, K, cx, cy);
    fc[C] = T(0.125) * s;
    phic[C] = T(0);
}

template <typename T>
__global__ void k_prolong(int nx, int ny, int nz, T* __restrict__ phi, const T* __restrict__ phic) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= nx || j >= ny || k >= nz) return;
    size_t c = cidx(i, j, k, nx, ny);
    phi[c] = phi[c] + phic[cidx(i / 2, j / 2, k / 2, nx / 2, ny / 2)];
}

template <typename T, typename Coef>
__global__ __launch_bounds__(kBlock) void k_resid_norm(int nx, int ny, int nz, T h2, const T* __restrict__ phi,
                                                       const T* __restrict__ f, Coef coef,
                                                       double* __restrict__ r_out, double* __restrict__ partials) {
    const size_t N = (size_t)nx * ny * nz;
    double s = 0.0, mx = 0.0, nonfin = 0.0;
    for (size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x; c < N; c += (size_t)gridDim.x * kBlock) {
        int i = (int)(c % nx);
        int j = (int)((c / nx) % ny);
        int k = (int)(c / ((size_t)nx * ny));
        double r = (double)(f[c] - apply_cell<T>(i, j, k, nx, ny, nz, h2, phi, coef));
        if (r_out) r_out[c] = r;
        if (!finite_d(r)) nonfin += 1.0;
        s += r * r;
        mx = fmax(mx, fabs(r));
    }
    block_reduce_row(s, 0.0, mx, nonfin, partials + (size_t)blockIdx.x * kReduceWidth);
}

// ---------------------------------------------------------------------------
// Coarsest level.  One workgroup builds M = -A + c 1 1^T (c = mean diagonal
// of -A) and inverts it in place by Gauss-Jordan elimination (M is SPD, so
// no pivoting is needed).  The per-cycle solve is then a mat-vec.
// ---------------------------------------------------------------------------
constexpr int kSetupThreads = 1024;
constexpr int kSetupLdsN = 128;      // matrices up to this order are inverted in LDS

// The workgroup's build and inversion of one problem's coarsest matrix; Ms
// (order-kSetupLdsN LDS matrix, used when kLds), fac, prow (kCoarseMax
// each) and shift are LDS scratch of the calling kernel.
template <bool kLds>
__device__ void coarse_setup_body(int nx, int ny, int nz, double h, const double* __restrict__ bx,
                                  const double* __restrict__ by, const double* __restrict__ bz,
                                  double* __restrict__ Mg, const Bnd<double>& bnd, int has_bnd, int singular,
                                  double* Ms, double* fac, double* prow, double& shift) {
    const int n = nx * ny * nz;
    const int tid = threadIdx.x, nt = blockDim.x;
    double* M = kLds ? Ms : Mg;
    const double ih2 = 1.0 / (h * h);
    for (int e = tid; e < n * n; e += nt) M[e] = 0.0;
    __syncthreads();
    for (int c = tid; c < n; c += nt) {
        int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        int im = i > 0 ? i - 1 : nx - 1, ip = i < nx - 1 ? i + 1 : 0;
        int jm = j > 0 ? j - 1 : ny - 1, jp = j < ny - 1 ? j + 1 : 0;
        int km = k > 0 ? k - 1 : nz - 1, kp = k < nz - 1 ? k + 1 : 0;
        double b[6] = {bx[c], bx[cidx(ip, j, k, nx, ny)], by[c], by[cidx(i, jp, k, nx, ny)],
                       bz[c], bz[cidx(i, j, kp, nx, ny)]};
        int nb[6] = {(int)cidx(im, j, k, nx, ny), (int)cidx(ip, j, k, nx, ny), (int)cidx(i, jm, k, nx, ny),
                     (int)cidx(i, jp, k, nx, ny), (int)cidx(i, j, km, nx, ny), (int)cidx(i, j, kp, nx, ny)};
        double* row = M + c * n;
        for (int q = 0; q < 6; ++q) {
            if (b[q] == 0.0) continue;      // wall face: no coupling
            row[c] += b[q] * ih2;
            row[nb[q]] -= b[q] * ih2;
        }
        if (has_bnd) row[c] += bnd_diag(bnd, i, j, k, nx, ny, nz) * ih2;   // outflow faces
    }
    __syncthreads();
    if (singular) {      // constant null space: M = -A + c 1 1^T, c the mean diagonal
        if (tid == 0) {
            double d = 0.0;
            for (int c = 0; c < n; ++c) d += M[c * n + c];
            shift = d / n;
        }
        __syncthreads();
        for (int e = tid; e < n * n; e += nt) M[e] += shift;
    }
    gj_invert(M, n, fac, prow);
    if (kLds)
        for (int e = tid; e < n * n; e += nt) Mg[e] = Ms[e];
}

template <bool kLds>
__global__ __launch_bounds__(kSetupThreads) void k_coarse_setup(int nx, int ny, int nz, double h,
                                                                const double* __restrict__ bx,
                                                                const double* __restrict__ by,
                                                                const double* __restrict__ bz,
                                                                double* __restrict__ Mg, Bnd<double> bnd,
                                                                int has_bnd, int singular) {
    __shared__ double Ms[kLds ? kSetupLdsN * kSetupLdsN : 1];
    __shared__ double fac[kCoarseMax];      // column p before the elimination step
    __shared__ double prow[kCoarseMax];     // row p before the elimination step
    __shared__ double shift;
    coarse_setup_body<kLds>(nx, ny, nz, h, bx, by, bz, Mg, bnd, has_bnd, singular, Ms, fac, prow, shift);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_solve(int n, const double* __restrict__ Minv,
                                                         const T* __restrict__ f, T* __restrict__ phi,
                                                         int singular) {
    __shared__ double rhs[kCoarseMax];
    __shared__ double x[kCoarseMax];
    __shared__ double mean;
    for (int c = threadIdx.x; c < n; c += kBlock) rhs[c] = (double)f[c];
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        if (singular)
            for (int c = 0; c < n; ++c) s += rhs[c];
        mean = singular ? s / n : 0.0;
    }
    __syncthreads();
    double m = mean;
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += kBlock) rhs[c] = -(rhs[c] - m);
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += kBlock) {
        const double* row = Minv + (size_t)r * n;
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += row[c] * rhs[c];
        x[r] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        if (singular)
            for (int c = 0; c < n; ++c) s += x[c];
        mean = singular ? s / n : 0.0;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += kBlock) phi[c] = (T)(x[c] - mean);
}

// ---------------------------------------------------------------------------
// Velocity correction: U <- U - (b/beta0)_f (phi_c - phi_nb)/h on every
// non-wall face (low faces of each cell), periodic duplicate faces refreshed.
// ---------------------------------------------------------------------------
__device__ inline void correct_cell(int i, int j, int k, int nx, int ny, int nz, int px, int py, int pz, double h,
                                    const double* __restrict__ b0c, const double* __restrict__ b0e,
                                    const double* __restrict__ bx, const double* __restrict__ by,
                                    const double* __restrict__ bz, const double* __restrict__ phi,
                                    const double* __restrict__ phi_sum, double* __restrict__ u,
                                    double* __restrict__ v, double* __restrict__ w, double* __restrict__ phi_out) {
    const size_t N = (size_t)nx * ny * nz;
    const double m = phi_sum[0] / (double)N;
    size_t c = cidx(i, j, k, nx, ny);
    double pc = phi[c] - m;
    if (phi_out) phi_out[c] = pc;
    size_t plane = (size_t)nx * ny;
    if (px || i > 0) {
        int im = i > 0 ? i - 1 : nx - 1;
        double g = (pc - (phi[cidx(im, j, k, nx, ny)] - m)) / h;
        size_t e = ((size_t)k * ny + j) * (nx + 1) + i;
        double un = u[e] - (bx[c] / b0c[k]) * g;
        u[e] = un;
        if (px && i == 0) u[e + nx] = un;
    }
    if (py || j > 0) {
        int jm = j > 0 ? j - 1 : ny - 1;
        double g = (pc - (phi[cidx(i, jm, k, nx, ny)] - m)) / h;
        size_t e = ((size_t)k * (ny + 1) + j) * nx + i;
        double vn = v[e] - (by[c] / b0c[k]) * g;
        v[e] = vn;
        if (py && j == 0) v[e + (size_t)ny * nx] = vn;
    }
    if (pz || k > 0) {
        int km = k > 0 ? k - 1 : nz - 1;
        double g = (pc - (phi[cidx(i, j, km, nx, ny)] - m)) / h;
        size_t e = (size_t)k * plane + (size_t)j * nx + i;
        double wn = w[e] - (bz[c] / b0e[k]) * g;
        w[e] = wn;
        if (pz && k == 0) w[e + (size_t)nz * plane] = wn;
    }
}

__global__ void k_correct(int nx, int ny, int nz, int px, int py, int pz, double h,
                          const double* __restrict__ b0c, const double* __restrict__ b0e,
                          const double* __restrict__ bx, const double* __restrict__ by,
                          const double* __restrict__ bz, const double* __restrict__ phi,
                          const double* __restrict__ phi_sum, double* __restrict__ u,
                          double* __restrict__ v, double* __restrict__ w, double* __restrict__ phi_out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int j = blockIdx.y * blockDim.y + threadIdx.y;
    int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= nx || j >= ny || k >= nz) return;
    correct_cell(i, j, k, nx, ny, nz, px, py, pz, h, b0c, b0e, bx, by, bz, phi, phi_sum, u, v, w, phi_out);
}

// ---------------------------------------------------------------------------
// General boundaries and base states: outflow sides (phi = 0 on the boundary
// faces) and a radial beta0.
// ---------------------------------------------------------------------------
enum { kSidePeriodic = 0, kSideWall = 1, kSideOutflow = 2 };

// beta0 at a point: plane-parallel layers or the radial profile (linear in r
// between the profile radii (m + 1/2) dr, constant beyond the ends).
struct Beta0At {
    const GenArgs& a;
    __device__ double radial(double x, double y, double z) const {
        const double dx = x - a.cx, dy = y - a.cy, dz = z - a.cz;
        const double r = sqrt(dx * dx + dy * dy + dz * dz);
        const double s = r / a.dr - 0.5;
        if (!(s > 0.0)) return a.prof[0];
        if (s >= (double)(a.nr - 1)) return a.prof[a.nr - 1];
        const int m = (int)s;
        const double t = s - (double)m;
        return a.prof[m] + t * (a.prof[m + 1] - a.prof[m]);
    }
    __device__ double cell(int i, int j, int k) const {
        if (!a.prof) return a.b0c[k];
        return radial((i + 0.5) * a.h, (j + 0.5) * a.h, (k + 0.5) * a.h);
    }
    // face f of direction x / y / z with the cell centres of the other two indices
    __device__ double fx(int f, int j, int k) const {
        if (!a.prof) return a.b0c[k];
        return radial(f * a.h, (j + 0.5) * a.h, (k + 0.5) * a.h);
    }
    __device__ double fy(int f, int i, int k) const {
        if (!a.prof) return a.b0c[k];
        return radial((i + 0.5) * a.h, f * a.h, (k + 0.5) * a.h);
    }
    __device__ double fz(int f, int i, int j) const {
        if (!a.prof) return a.b0e[f];
        return radial((i + 0.5) * a.h, (j + 0.5) * a.h, f * a.h);
    }
};

template <bool kRhs>
__global__ __launch_bounds__(kBlock) void k_coeff_rhs_gen(GenArgs a) {
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const double* __restrict__ rho = a.rho;
    const size_t N = (size_t)nx * ny * nz;
    const size_t plane = (size_t)nx * ny;
    const Beta0At B{a};
    const bool px = a.side[0] == kSidePeriodic, py = a.side[2] == kSidePeriodic, pz = a.side[4] == kSidePeriodic;
    double sf = 0.0, saf = 0.0, bad = 0.0, nonfin = 0.0;
    const size_t tid = (size_t)blockIdx.x * kBlock + threadIdx.x, stride = (size_t)gridDim.x * kBlock;
    if (a.prof)                                  // the whole profile must be usable
        for (size_t m = tid; m < (size_t)a.nr; m += stride) {
            if (!finite_d(a.prof[m])) nonfin += 1.0;
            if (!(a.prof[m] > 0.0)) bad = 1.0;
        }
    for (size_t c = tid; c < N; c += stride) {
        const int i = (int)(c % nx);
        const int j = (int)((c / nx) % ny);
        const int k = (int)(c / plane);
        const double rc = rho[c];
        const double bc = B.cell(i, j, k);
        if (!finite_d(rc) || !finite_d(bc)) nonfin += 1.0;
        if (!(rc > 0.0) || !(bc > 0.0)) bad = 1.0;
        const double bxl = B.fx(i, j, k), byl = B.fy(j, i, k), bzl = B.fz(k, i, j);
        // low faces: interior, periodic wrap, or 0 (wall / outflow side)
        double cx = 0.0, cy = 0.0, cz = 0.0;
        if (i > 0) cx = qdiv(bxl, 0.5 * (rho[c - 1] + rc));
        else if (px) cx = qdiv(bxl, 0.5 * (rho[c + (nx - 1)] + rc));
        if (j > 0) cy = qdiv(byl, 0.5 * (rho[c - nx] + rc));
        else if (py) cy = qdiv(byl, 0.5 * (rho[c + (size_t)(ny - 1) * nx] + rc));
        if (k > 0) cz = qdiv(bzl, 0.5 * (rho[c - plane] + rc));
        else if (pz) cz = qdiv(bzl, 0.5 * (rho[c + (size_t)(nz - 1) * plane] + rc));
        a.bx[c] = cx;
        a.by[c] = cy;
        a.bz[c] = cz;
        // outflow boundary faces: beta0_face / rho of this cell
        if (i == 0 && a.bnd[0]) a.bnd[0][(size_t)k * ny + j] = qdiv(bxl, rc);
        if (i == nx - 1 && a.bnd[1]) a.bnd[1][(size_t)k * ny + j] = qdiv(B.fx(nx, j, k), rc);
        if (j == 0 && a.bnd[2]) a.bnd[2][(size_t)k * nx + i] = qdiv(byl, rc);
        if (j == ny - 1 && a.bnd[3]) a.bnd[3][(size_t)k * nx + i] = qdiv(B.fy(ny, i, k), rc);
        if (k == 0 && a.bnd[4]) a.bnd[4][(size_t)j * nx + i] = qdiv(bzl, rc);
        if (k == nz - 1 && a.bnd[5]) a.bnd[5][(size_t)j * nx + i] = qdiv(B.fz(nz, i, j), rc);
        if (kRhs) {
            // high faces (periodic: face n is face 0)
            const int ih = (i == nx - 1 && px) ? 0 : i + 1;
            const int jh = (j == ny - 1 && py) ? 0 : j + 1;
            const int kh = (k == nz - 1 && pz) ? 0 : k + 1;
            const size_t ub = ((size_t)k * ny + j) * (nx + 1);
            const double ul = a.u[ub + i], uh = a.u[ub + ih];
            const size_t vb = (size_t)k * (ny + 1) * nx + i;
            const double vl = a.v[vb + (size_t)j * nx], vh = a.v[vb + (size_t)jh * nx];
            const size_t wc = (size_t)j * nx + i;
            const double wl = a.w[(size_t)k * plane + wc], wh = a.w[(size_t)kh * plane + wc];
            double sc = a.S[c];
            if (a.w0) sc = sc - a.w0[k];         // the dp0/dt term of the constraint, per layer
            if (!finite_d(ul) || !finite_d(uh) || !finite_d(vl) || !finite_d(vh) || !finite_d(wl) ||
                !finite_d(wh) || !finite_d(sc))
                nonfin += 1.0;
            const double fxs = B.fx(ih, j, k) * uh - bxl * ul;
            const double fys = B.fy(jh, i, k) * vh - byl * vl;
            const double fzs = B.fz(kh, i, j) * wh - bzl * wl;
            const double fc = (fxs + fys + fzs) / a.h - bc * sc;
            a.f[c] = fc;
            sf += fc;
            saf += fabs(fc);
        }
    }
    block_reduce_row(sf, saf, bad, nonfin, a.partials + (size_t)blockIdx.x * kReduceWidth);
}

__global__ __launch_bounds__(kBlock) void k_map_radial(GenArgs a, double* __restrict__ out) {
    const size_t N = (size_t)a.nx * a.ny * a.nz;
    const Beta0At B{a};
    for (size_t c = (size_t)blockIdx.x * kBlock + threadIdx.x; c < N; c += (size_t)gridDim.x * kBlock) {
        const int i = (int)(c % a.nx);
        const int j = (int)((c / a.nx) % a.ny);
        const int k = (int)(c / ((size_t)a.nx * a.ny));
        out[c] = B.cell(i, j, k);
    }
}

// One thread per cell: its low faces, and its high faces on outflow sides.
__global__ void k_correct_gen(GenArgs a, const double* __restrict__ phi, const double* __restrict__ phi_sum,
                              double* __restrict__ u, double* __restrict__ v, double* __restrict__ w,
                              double* __restrict__ phi_out) {
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= nx || j >= ny || k >= nz) return;
    const size_t N = (size_t)nx * ny * nz;
    const double m = phi_sum ? phi_sum[0] / (double)N : 0.0;
    const size_t c = cidx(i, j, k, nx, ny);
    const size_t plane = (size_t)nx * ny;
    const double pc = phi[c] - m;
    const double rc = a.rho[c];
    const double h = a.h;
    if (phi_out) phi_out[c] = pc;
    const bool px = a.side[0] == kSidePeriodic, py = a.side[2] == kSidePeriodic, pz = a.side[4] == kSidePeriodic;
    {   // x faces
        const size_t e = ((size_t)k * ny + j) * (nx + 1) + i;
        if (i > 0 || px) {
            const size_t cm = cidx(i > 0 ? i - 1 : nx - 1, j, k, nx, ny);
            const double g = (pc - (phi[cm] - m)) / h;
            const double un = u[e] - g / (0.5 * (a.rho[cm] + rc));
            u[e] = un;
            if (px && i == 0) u[e + nx] = un;
        } else if (a.side[0] == kSideOutflow) {
            u[e] = u[e] - ((pc - (-pc)) / h) / rc;
        }
        if (i == nx - 1 && a.side[1] == kSideOutflow) u[e + 1] = u[e + 1] - (((-pc) - pc) / h) / rc;
    }
    {   // y faces
        const size_t e = ((size_t)k * (ny + 1) + j) * nx + i;
        if (j > 0 || py) {
            const size_t cm = cidx(i, j > 0 ? j - 1 : ny - 1, k, nx, ny);
            const double g = (pc - (phi[cm] - m)) / h;
            const double vn = v[e] - g / (0.5 * (a.rho[cm] + rc));
            v[e] = vn;
            if (py && j == 0) v[e + (size_t)ny * nx] = vn;
        } else if (a.side[2] == kSideOutflow) {
            v[e] = v[e] - ((pc - (-pc)) / h) / rc;
        }
        if (j == ny - 1 && a.side[3] == kSideOutflow) v[e + nx] = v[e + nx] - (((-pc) - pc) / h) / rc;
    }
    {   // z faces
        const size_t e = (size_t)k * plane + (size_t)j * nx + i;
        if (k > 0 || pz) {
            const size_t cm = cidx(i, j, k > 0 ? k - 1 : nz - 1, nx, ny);
            const double g = (pc - (phi[cm] - m)) / h;
            const double wn = w[e] - g / (0.5 * (a.rho[cm] + rc));
            w[e] = wn;
            if (pz && k == 0) w[e + (size_t)nz * plane] = wn;
        } else if (a.side[4] == kSideOutflow) {
            w[e] = w[e] - ((pc - (-pc)) / h) / rc;
        }
        if (k == nz - 1 && a.side[5] == kSideOutflow) w[e + plane] = w[e + plane] - (((-pc) - pc) / h) / rc;
    }
}

// Per-cell boundary diagonal of a level (bnd_diag of every cell, zero away
// from the outflow sides), read by the fused sweeps.
template <typename T>
__global__ void k_bnd_diag3(int nx, int ny, int nz, Bnd<T> bnd, T* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y * blockDim.y + threadIdx.y;
    const int k = blockIdx.z * blockDim.z + threadIdx.z;
    if (i >= nx || j >= ny || k >= nz) return;
    out[cidx(i, j, k, nx, ny)] = bnd_diag(bnd, i, j, k, nx, ny, nz);
}

// Coarse boundary faces of one side: cf[A + B*ca] = mean of the fine faces
// (2A, 2B), (2A+1, 2B), (2A, 2B+1), (2A+1, 2B+1) (first index fastest).
template <typename T>
__global__ void k_avg_bnd(int fa, int fb, const T* __restrict__ ff, T* __restrict__ cf) {
    const int ca = fa / 2, cb = fb / 2;
    const int A = blockIdx.x * blockDim.x + threadIdx.x;
    const int Bq = blockIdx.y * blockDim.y + threadIdx.y;
    if (A >= ca || Bq >= cb) return;
    const size_t r0 = (size_t)(2 * Bq) * fa, r1 = r0 + fa;
    cf[(size_t)Bq * ca + A] = T(0.25) * (ff[r0 + 2 * A] + ff[r0 + 2 * A + 1] + ff[r1 + 2 * A] + ff[r1 + 2 * A + 1]);
}

template <typename T>
__global__ void k_fill(T* __restrict__ a, size_t n, T value) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        a[e] = value;
}

__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        dst[e] = src[e];
}

// Mixed precision helpers ---------------------------------------------------
__global__ void k_to_f32(const double* __restrict__ r, float* __restrict__ r32, size_t n,
                         const double* __restrict__ scale_inv) {
    const double s = 1.0 / scale_inv[0];
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        r32[e] = (float)(r[e] * s);
}

__global__ void k_accumulate(double* __restrict__ phi, const float* __restrict__ e32, size_t n,
                             const double* __restrict__ scale_inv) {
    const double s = scale_inv[0];
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        phi[e] = phi[e] + (double)e32[e] * s;
}

// Mixed precision, after the residual of iteration k is reduced into
// res[0] = sum r^2: scales[0] <- scales[1] (the scale the FP32 residual now
// holds), scales[1] <- the power of two nearest 1/rms(r) (1 for a zero or
// non-finite residual), the scale for the next FP32 residual.
// ---------------------------------------------------------------------------
// Base state (Sec. 2, definition of beta0): with r the height z, beta0 is
// rho0(0) exp of the integral of (1/(Gamma1 p0)) dp0/dr from the bottom.
// Gamma1 is constant in a layer, so the integral over any part [a, b] of
// layer k is ln(p0(b)/p0(a)) / Gamma1[k].  One workgroup: the per-layer
// logarithms in parallel (into the outputs), one thread sums them from the
// bottom in order, then the exponentials in parallel.  Non-positive or
// non-finite p0 / Gamma1 give non-finite beta0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_beta0_from_p0(int nz, double rho0, const double* __restrict__ p0e,
                                                        const double* __restrict__ p0c,
                                                        const double* __restrict__ g1c, double* __restrict__ b0c,
                                                        double* __restrict__ b0e) {
    for (int k = threadIdx.x; k < nz; k += blockDim.x) {
        const double g = g1c[k];
        const double ok = (p0e[k] > 0.0 && p0e[k + 1] > 0.0 && p0c[k] > 0.0 && g > 0.0) ? 1.0 : NAN;
        b0e[k] = ok * (log(p0e[k + 1] / p0e[k]) / g);     // layer integral
        b0c[k] = ok * (log(p0c[k] / p0e[k]) / g);         // bottom face to the centre
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;                                  // integral from r = 0 to face k
        for (int k = 0; k < nz; ++k) {
            const double layer = b0e[k];
            b0e[k] = acc;
            acc += layer;
        }
        b0e[nz] = acc;
    }
    __syncthreads();
    for (int k = threadIdx.x; k <= nz; k += blockDim.x) {
        const double below = b0e[k];
        if (k < nz) b0c[k] = rho0 * exp(below + b0c[k]);
        b0e[k] = rho0 * exp(below);
    }
}

// w0[k] = dp0dt[k] / (Gamma1[k] p0[k]), the dp0/dt term of the constraint per layer
__global__ void k_dp0_term(int nz, const double* __restrict__ p0c, const double* __restrict__ g1c,
                           const double* __restrict__ dp0dt, double* __restrict__ w0) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nz) w0[k] = dp0dt[k] / (g1c[k] * p0c[k]);
}

__device__ void next_scale(const double* res, double* scales, double n) {
    const double rms = sqrt(res[0] / n);
    double s = 1.0;
    if (rms > 0.0 && isfinite(rms)) s = ldexp(1.0, -ilogb(rms));
    scales[0] = scales[1];
    scales[1] = s;
}

__global__ void k_next_scale(const double* __restrict__ res, double* __restrict__ scales, double n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) next_scale(res, scales, n);
}

// Batched form: one thread per problem.
__global__ void k_next_scale_multi(const ScaleDesc* __restrict__ d, int nprob) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) next_scale(d[p].res, d[p].scales, d[p].n);
}

__global__ void k_scale_to_f32(const double* __restrict__ a, float* __restrict__ b, size_t n, double s) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        b[e] = (float)(a[e] * s);
}

__global__ void k_d2f(const double* __restrict__ a, float* __restrict__ b, size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        b[e] = (float)a[e];
}

inline int stream_blocks(size_t n) {
    size_t b = (n + kBlock - 1) / kBlock;
    return (int)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

}  // namespace

// ============================================================================
// launchers
// ============================================================================
int num_blocks_for_partials(const Shape& s) { return partial_blocks(s.N()); }

// Grid of a point loop over a level: at most kMaxPartialBlocks workgroups.
static dim3 point_grid(const Shape& s) {
    const int gx = std::min((s.nx + kPtX - 1) / kPtX, kMaxPartialBlocks);
    const int gy = std::max(1, std::min((s.ny + kPtY - 1) / kPtY, kMaxPartialBlocks / gx));
    const int gz = std::max(1, std::min(s.nz, kMaxPartialBlocks / (gx * gy)));
    return dim3(gx, gy, gz);
}

int coeff_grid(const Shape& s, int g[3]) {
    const dim3 d = point_grid(s);
    g[0] = (int)d.x;
    g[1] = (int)d.y;
    g[2] = (int)d.z;
    return g[0] * g[1] * g[2];
}

hipError_t launch_coeff_rhs(const Shape& s, int px, int py, int pz, double h, const double* rho,
                            const double* b0c, const double* b0e, const double* S, const double* u,
                            const double* v, const double* w, double* bx, double* by, double* bz,
                            double* f, double* partials, int* nparts, hipStream_t st, const double* w0,
                            float* rho32) {
    const dim3 g = point_grid(s);
    const CoeffDesc a{s.nx, s.ny, s.nz, px, py, pz, h, rho, b0c, b0e, S, u, v, w, w0, bx, by, bz, f, partials,
                      (int)g.x, (int)g.y, (int)g.z, 0, rho32};
    hipLaunchKernelGGL(k_coeff_rhs<true>, g, dim3(kPtX, kPtY), 0, st, a);
    *nparts = (int)(g.x * g.y * g.z);
    return hipGetLastError();
}

hipError_t launch_coeff(const Shape& s, int px, int py, int pz, const double* rho, const double* b0c,
                        const double* b0e, double* bx, double* by, double* bz, double* partials,
                        int* nparts, hipStream_t st) {
    const dim3 g = point_grid(s);
    const CoeffDesc a{s.nx, s.ny, s.nz, px, py, pz, 1.0, rho, b0c, b0e, nullptr, nullptr, nullptr, nullptr, nullptr,
                      bx, by, bz, nullptr, partials, (int)g.x, (int)g.y, (int)g.z, 0};
    hipLaunchKernelGGL(k_coeff_rhs<false>, g, dim3(kPtX, kPtY), 0, st, a);
    *nparts = (int)(g.x * g.y * g.z);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nparts, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, st, partials, nparts, out, (double*)nullptr, 0.0);
    return hipGetLastError();
}

hipError_t launch_reduce_scale(const double* partials, int nparts, double* out, double* scales, size_t n,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kBlock), 0, st, partials, nparts, out, scales, (double)n);
    return hipGetLastError();
}

hipError_t launch_shift_norm(const Shape& s, double* f, double shift, double* partials, int* nparts,
                             hipStream_t st) {
    int nb = partial_blocks(s.N());
    hipLaunchKernelGGL(k_shift_norm, dim3(nb), dim3(kBlock), 0, st, s.N(), f, shift, partials);
    *nparts = nb;
    return hipGetLastError();
}

hipError_t launch_sum(const Shape& s, const double* a, double* partials, int* nparts, hipStream_t st) {
    int nb = partial_blocks(s.N());
    hipLaunchKernelGGL(k_sum, dim3(nb), dim3(kBlock), 0, st, s.N(), a, partials);
    *nparts = nb;
    return hipGetLastError();
}

hipError_t launch_avg_coeff_rho(const Shape& fine, int px, int py, int pz, const double* rho, const double* b0c,
                                const double* b0e, double* cbx, double* cby, double* cbz, float* const* m32,
                                hipStream_t st) {
    Launch3 L = cell_launch(fine.nx / 2, fine.ny / 2, fine.nz / 2);
    RhoCoeff co{rho, b0c, b0e, fine.nx, fine.ny, fine.nz, px, py, pz, Bnd<double>{}, 0};
    hipLaunchKernelGGL(k_avg_coeff_rho, L.grid, L.block, 0, st, co, cbx, cby, cbz, m32 ? m32[0] : nullptr,
                       m32 ? m32[1] : nullptr, m32 ? m32[2] : nullptr);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_avg_coeff(const Shape& fine, const T* bx, const T* by, const T* bz, T* cbx, T* cby,
                            T* cbz, hipStream_t st, float* const* m32) {
    Launch3 L = cell_launch(fine.nx / 2, fine.ny / 2, fine.nz / 2);
    hipLaunchKernelGGL(k_avg_coeff<T>, L.grid, L.block, 0, st, fine.nx, fine.ny, fine.nz, bx, by, bz, cbx,
                       cby, cbz, m32 ? m32[0] : nullptr, m32 ? m32[1] : nullptr, m32 ? m32[2] : nullptr);
    return hipGetLastError();
}

template <typename T>
inline void set_bnd(Bnd<T>& dst, int& has, const Bnd<T>* src) {
    has = 0;
    for (int q = 0; q < 6; ++q) {
        dst.s[q] = src ? src->s[q] : nullptr;
        if (dst.s[q]) has = 1;
    }
}

template <typename T>
hipError_t launch_rbgs(const Shape& s, double h, T* phi, const T* f, const T* bx, const T* by,
                       const T* bz, int nsweeps, hipStream_t st, const Bnd<T>* bnd) {
    Launch3 L = cell_launch((s.nx + 1) / 2, s.ny, s.nz);
    T h2 = (T)(h * h);
    Bnd<T> b;
    int has = 0;
    set_bnd(b, has, bnd);
    for (int sw = 0; sw < nsweeps; ++sw)
        for (int colour = 0; colour < 2; ++colour)
            hipLaunchKernelGGL(k_rbgs_colour<T>, L.grid, L.block, 0, st, s.nx, s.ny, s.nz, h2, phi, f, bx, by,
                               bz, colour, b, has);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_resid_restrict(const Shape& fine, double h, const T* phi, const T* f, const T* bx,
                                 const T* by, const T* bz, T* fc, T* phic, hipStream_t st, const Bnd<T>* bnd) {
    Launch3 L = cell_launch(fine.nx / 2, fine.ny / 2, fine.nz / 2);
    StoredCoeff<T> coef{bx, by, bz};
    set_bnd(coef.bnd, coef.has_bnd, bnd);
    hipLaunchKernelGGL((k_resid_restrict<T, StoredCoeff<T>>), L.grid, L.block, 0, st, fine.nx, fine.ny, fine.nz,
                       (T)(h * h), phi, f, coef, fc, phic);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const Shape& fine, T* phi, const T* phic, hipStream_t st) {
    Launch3 L = cell_launch(fine.nx, fine.ny, fine.nz);
    hipLaunchKernelGGL(k_prolong<T>, L.grid, L.block, 0, st, fine.nx, fine.ny, fine.nz, phi, phic);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_resid_norm(const Shape& s, double h, const T* phi, const T* f, const T* bx, const T* by,
                             const T* bz, double* partials, int* nparts, hipStream_t st, const Bnd<T>* bnd) {
    int nb = partial_blocks(s.N());
    StoredCoeff<T> coef{bx, by, bz};
    set_bnd(coef.bnd, coef.has_bnd, bnd);
    hipLaunchKernelGGL((k_resid_norm<T, StoredCoeff<T>>), dim3(nb), dim3(kBlock), 0, st, s.nx, s.ny, s.nz,
                       (T)(h * h), phi, f, coef, (double*)nullptr, partials);
    *nparts = nb;
    return hipGetLastError();
}

hipError_t launch_resid_store(const Shape& s, double h, const double* phi, const double* f,
                              const double* bx, const double* by, const double* bz, double* r,
                              double* partials, int* nparts, hipStream_t st, const Bnd<double>* bnd) {
    int nb = partial_blocks(s.N());
    StoredCoeff<double> coef{bx, by, bz};
    set_bnd(coef.bnd, coef.has_bnd, bnd);
    hipLaunchKernelGGL((k_resid_norm<double, StoredCoeff<double>>), dim3(nb), dim3(kBlock), 0, st, s.nx, s.ny,
                       s.nz, h * h, phi, f, coef, r, partials);
    *nparts = nb;
    return hipGetLastError();
}

hipError_t launch_resid_norm_rho(const Shape& s, double h, const RhoArgs& ra, const double* phi,
                                 const double* f, double* r_out, double* partials, int* nparts,
                                 hipStream_t st, const Bnd<double>* bnd) {
    int nb = partial_blocks(s.N());
    RhoCoeff coef{ra.rho, ra.b0c, ra.b0e, s.nx, s.ny, s.nz, ra.px, ra.py, ra.pz};
    set_bnd(coef.bnd, coef.has_bnd, bnd);
    hipLaunchKernelGGL((k_resid_norm<double, RhoCoeff>), dim3(nb), dim3(kBlock), 0, st, s.nx, s.ny, s.nz,
                       h * h, phi, f, coef, r_out, partials);
    *nparts = nb;
    return hipGetLastError();
}

hipError_t launch_resid_restrict_rho(const Shape& fine, double h, const RhoArgs& ra, const double* phi,
                                     const double* f, double* fc, double* phic, hipStream_t st,
                                     const Bnd<double>* bnd) {
    Launch3 L = cell_launch(fine.nx / 2, fine.ny / 2, fine.nz / 2);
    RhoCoeff coef{ra.rho, ra.b0c, ra.b0e, fine.nx, fine.ny, fine.nz, ra.px, ra.py, ra.pz};
    set_bnd(coef.bnd, coef.has_bnd, bnd);
    hipLaunchKernelGGL((k_resid_restrict<double, RhoCoeff>), L.grid, L.block, 0, st, fine.nx, fine.ny, fine.nz,
                       h * h, phi, f, coef, fc, phic);
    return hipGetLastError();
}

hipError_t launch_coarse_setup(const Shape& s, double h, const double* bx, const double* by,
                               const double* bz, double* minv, hipStream_t st, const Bnd<double>* bnd,
                               int singular) {
    if (s.N() > (size_t)kCoarseMax) return hipErrorInvalidValue;
    Bnd<double> b;
    int has = 0;
    set_bnd(b, has, bnd);
    if (s.N() <= (size_t)kSetupLdsN)
        hipLaunchKernelGGL(k_coarse_setup<true>, dim3(1), dim3(kSetupThreads), 0, st, s.nx, s.ny, s.nz, h, bx, by, bz,
                           minv, b, has, singular);
    else
        hipLaunchKernelGGL(k_coarse_setup<false>, dim3(1), dim3(kSetupThreads), 0, st, s.nx, s.ny, s.nz, h, bx, by,
                           bz, minv, b, has, singular);
    return hipGetLastError();
}

hipError_t launch_coarse_solve(int N, const double* minv, const double* f, double* phi, hipStream_t st,
                               int singular) {
    hipLaunchKernelGGL(k_coarse_solve<double>, dim3(1), dim3(kBlock), 0, st, N, minv, f, phi, singular);
    return hipGetLastError();
}

hipError_t launch_coarse_solve_f32(int N, const double* minv, const float* f, float* phi, hipStream_t st,
                                   int singular) {
    hipLaunchKernelGGL(k_coarse_solve<float>, dim3(1), dim3(kBlock), 0, st, N, minv, f, phi, singular);
    return hipGetLastError();
}

hipError_t launch_coeff_rhs_gen(const GenArgs& a, int* nparts, hipStream_t st) {
    const Shape s{a.nx, a.ny, a.nz};
    int nb = partial_blocks(s.N());
    if (a.S) hipLaunchKernelGGL(k_coeff_rhs_gen<true>, dim3(nb), dim3(kBlock), 0, st, a);
    else hipLaunchKernelGGL(k_coeff_rhs_gen<false>, dim3(nb), dim3(kBlock), 0, st, a);
    *nparts = nb;
    return hipGetLastError();
}

hipError_t launch_map_radial(const GenArgs& a, double* out, hipStream_t st) {
    const size_t N = (size_t)a.nx * a.ny * a.nz;
    hipLaunchKernelGGL(k_map_radial, dim3(stream_blocks(N)), dim3(kBlock), 0, st, a, out);
    return hipGetLastError();
}

hipError_t launch_correct_gen(const GenArgs& a, const double* phi, const double* phi_sum, double* u, double* v,
                              double* w, double* phi_out, hipStream_t st) {
    Launch3 L = cell_launch(a.nx, a.ny, a.nz);
    hipLaunchKernelGGL(k_correct_gen, L.grid, L.block, 0, st, a, phi, phi_sum, u, v, w, phi_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bnd_diag3(const Shape& s, const Bnd<T>& bnd, T* out, hipStream_t st) {
    Launch3 L = cell_launch(s.nx, s.ny, s.nz);
    hipLaunchKernelGGL(k_bnd_diag3<T>, L.grid, L.block, 0, st, s.nx, s.ny, s.nz, bnd, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_avg_bnd(const Shape& fine, const Bnd<T>& fb, T* const cb[6], hipStream_t st) {
    for (int q = 0; q < 6; ++q) {
        if (!fb.s[q] || !cb[q]) continue;
        const int fa = q < 2 ? fine.ny : fine.nx;        // first (fastest) index of the side array
        const int fbn = q < 4 ? fine.nz : fine.ny;       // second index
        dim3 block(32, 8);
        dim3 grid((fa / 2 + 31) / 32, (fbn / 2 + 7) / 8);
        hipLaunchKernelGGL(k_avg_bnd<T>, grid, block, 0, st, fa, fbn, fb.s[q], cb[q]);
    }
    return hipGetLastError();
}

hipError_t launch_correct(const Shape& s, int px, int py, int pz, double h, const double* b0c,
                          const double* b0e, const double* bx, const double* by, const double* bz,
                          const double* phi, const double* phi_sum, double* u, double* v, double* w,
                          double* phi_out, hipStream_t st) {
    Launch3 L = cell_launch(s.nx, s.ny, s.nz);
    hipLaunchKernelGGL(k_correct, L.grid, L.block, 0, st, s.nx, s.ny, s.nz, px, py, pz, h, b0c, b0e, bx, by, bz,
                       phi, phi_sum, u, v, w, phi_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* a, size_t n, T value, hipStream_t st) {
    hipLaunchKernelGGL(k_fill<T>, dim3(stream_blocks(n)), dim3(kBlock), 0, st, a, n, value);
    return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_copy, dim3(stream_blocks(n)), dim3(kBlock), 0, st, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_to_f32(const double* r, float* r32, size_t n, const double* scale_inv, hipStream_t st) {
    hipLaunchKernelGGL(k_to_f32, dim3(stream_blocks(n)), dim3(kBlock), 0, st, r, r32, n, scale_inv);
    return hipGetLastError();
}

hipError_t launch_accumulate(double* phi, const float* e32, size_t n, const double* scale_inv,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_accumulate, dim3(stream_blocks(n)), dim3(kBlock), 0, st, phi, e32, n, scale_inv);
    return hipGetLastError();
}

hipError_t launch_beta0_from_p0(int nz, double rho0, const double* p0e, const double* p0c, const double* g1c,
                                double* b0c, double* b0e, hipStream_t st) {
    hipLaunchKernelGGL(k_beta0_from_p0, dim3(1), dim3(1024), 0, st, nz, rho0, p0e, p0c, g1c, b0c, b0e);
    return hipGetLastError();
}

hipError_t launch_dp0_term(int nz, const double* p0c, const double* g1c, const double* dp0dt, double* w0,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_dp0_term, dim3((nz + 255) / 256), dim3(256), 0, st, nz, p0c, g1c, dp0dt, w0);
    return hipGetLastError();
}

hipError_t launch_next_scale_multi(const ScaleDesc* d, int nprob, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_next_scale_multi, dim3((nprob + 63) / 64), dim3(64), 0, st, d, nprob);
    return hipGetLastError();
}

hipError_t launch_next_scale(const double* res, double* scales, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_next_scale, dim3(1), dim3(64), 0, st, res, scales, (double)n);
    return hipGetLastError();
}

hipError_t launch_scale_to_f32(const double* a, float* b, size_t n, double s, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_to_f32, dim3(stream_blocks(n)), dim3(kBlock), 0, st, a, b, n, s);
    return hipGetLastError();
}

hipError_t launch_coeff_to_f32(const double* a, float* b, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_d2f, dim3(stream_blocks(n)), dim3(kBlock), 0, st, a, b, n);
    return hipGetLastError();
}

// explicit instantiations
#define MG_INST(T)                                                                                      \
    template hipError_t launch_avg_coeff<T>(const Shape&, const T*, const T*, const T*, T*, T*, T*,      \
                                            hipStream_t, float* const*);                                 \
    template hipError_t launch_rbgs<T>(const Shape&, double, T*, const T*, const T*, const T*, const T*, \
                                       int, hipStream_t, const Bnd<T>*);                                 \
    template hipError_t launch_resid_restrict<T>(const Shape&, double, const T*, const T*, const T*,     \
                                                 const T*, const T*, T*, T*, hipStream_t, const Bnd<T>*); \
    template hipError_t launch_prolong<T>(const Shape&, T*, const T*, hipStream_t);                      \
    template hipError_t launch_resid_norm<T>(const Shape&, double, const T*, const T*, const T*,         \
                                             const T*, const T*, double*, int*, hipStream_t,             \
                                             const Bnd<T>*);                                             \
    template hipError_t launch_avg_bnd<T>(const Shape&, const Bnd<T>&, T* const*, hipStream_t);         \
    template hipError_t launch_bnd_diag3<T>(const Shape&, const Bnd<T>&, T*, hipStream_t);              \
    template hipError_t launch_fill<T>(T*, size_t, T, hipStream_t);
MG_INST(double)
MG_INST(float)
#undef MG_INST

}  // namespace mg

// ============================================================================
// Batched (multi-problem) forms of the small-level kernels.  Problem p owns
// blocks [d[p].block0, d[p+1].block0) of a launch; each thread evaluates the
// same per-cell expression as the single-problem kernel, so a problem's
// values do not depend on what it was launched with.
// ============================================================================
namespace mg {
namespace {

template <typename D>
__device__ inline int find_problem(const D* __restrict__ d, int nprob, int b) {
    int lo = 0, hi = nprob;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (d[mid].block0 <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

// one colour of a red-black sweep; threads cover (nx/2) x ny x nz
__global__ __launch_bounds__(256) void k_rbgs_colour_multi(const CellDesc* __restrict__ d, int nprob, int colour) {
    const int p = find_problem(d, nprob, blockIdx.x);
    const CellDesc c = d[p];
    const long long t = (long long)(blockIdx.x - c.block0) * 256 + threadIdx.x;
    const int hx = c.nx / 2;
    if (t >= (long long)hx * c.ny * c.nz) return;
    const int ih = (int)(t % hx);
    const int j = (int)((t / hx) % c.ny);
    const int k = (int)(t / ((long long)hx * c.ny));
    const int nx = c.nx, ny = c.ny, nz = c.nz;
    const int i = 2 * ih + ((j + k + colour) & 1);
    if (i >= nx) return;
    int im = i > 0 ? i - 1 : nx - 1, ip = i < nx - 1 ? i + 1 : 0;
    int jm = j > 0 ? j - 1 : ny - 1, jp = j < ny - 1 ? j + 1 : 0;
    int km = k > 0 ? k - 1 : nz - 1, kp = k < nz - 1 ? k + 1 : 0;
    double* phi = c.phi;
    const size_t cc = cidx(i, j, k, nx, ny);
    const double bxl = c.bx[cc], bxh = c.bx[cidx(ip, j, k, nx, ny)];
    const double byl = c.by[cc], byh = c.by[cidx(i, jp, k, nx, ny)];
    const double bzl = c.bz[cc], bzh = c.bz[cidx(i, j, kp, nx, ny)];
    double num = bxl * phi[cidx(im, j, k, nx, ny)];
    num = num + bxh * phi[cidx(ip, j, k, nx, ny)];
    num = num + byl * phi[cidx(i, jm, k, nx, ny)];
    num = num + byh * phi[cidx(i, jp, k, nx, ny)];
    num = num + bzl * phi[cidx(i, j, km, nx, ny)];
    num = num + bzh * phi[cidx(i, j, kp, nx, ny)];
    double den = bxl + bxh;
    den = den + byl;
    den = den + byh;
    den = den + bzl;
    den = den + bzh;
    phi[cc] = qdiv(num - c.h2 * c.f[cc], den);
}

// f_c = R (f - L phi), phi_c = 0 with stored coefficients; threads cover coarse cells
__global__ __launch_bounds__(256) void k_resid_restrict_multi(const CellDesc* __restrict__ d, int nprob) {
    const int p = find_problem(d, nprob, blockIdx.x);
    const CellDesc c = d[p];
    const int cx = c.nx / 2, cy = c.ny / 2, cz = c.nz / 2;
    const long long t = (long long)(blockIdx.x - c.block0) * 256 + threadIdx.x;
    if (t >= (long long)cx * cy * cz) return;
    const int I = (int)(t % cx), J = (int)((t / cx) % cy), K = (int)(t / ((long long)cx * cy));
    StoredCoeff<double> coef{c.bx, c.by, c.bz};
    double s = 0.0;
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                const double r = c.f[cidx(i, j, k, c.nx, c.ny)] -
                                 apply_cell<double>(i, j, k, c.nx, c.ny, c.nz, c.h2, c.phi, coef);
                s = s + r;
            }
    const size_t C = cidx(I, J, K, cx, cy);
    c.fc[C] = 0.125 * s;
    c.phic[C] = 0.0;
}

// phi += P phic; threads cover fine cells
__global__ __launch_bounds__(256) void k_prolong_multi(const CellDesc* __restrict__ d, int nprob) {
    const int p = find_problem(d, nprob, blockIdx.x);
    const CellDesc c = d[p];
    const long long t = (long long)(blockIdx.x - c.block0) * 256 + threadIdx.x;
    if (t >= (long long)c.nx * c.ny * c.nz) return;
    const int i = (int)(t % c.nx), j = (int)((t / c.nx) % c.ny), k = (int)(t / ((long long)c.nx * c.ny));
    const size_t cc = cidx(i, j, k, c.nx, c.ny);
    c.phi[cc] = c.phi[cc] + c.phic[cidx(i / 2, j / 2, k / 2, c.nx / 2, c.ny / 2)];
}

// one block per problem: coarsest solve, same code as the single-problem kernel
__global__ __launch_bounds__(kBlock) void k_coarse_solve_multi(const CellDesc* __restrict__ d) {
    const CellDesc c = d[blockIdx.x];
    __shared__ double rhs[kCoarseMax];
    __shared__ double x[kCoarseMax];
    __shared__ double mean;
    const int n = c.nx * c.ny * c.nz;
    for (int q = threadIdx.x; q < n; q += kBlock) rhs[q] = c.f[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < n; ++q) s += rhs[q];
        mean = s / n;
    }
    __syncthreads();
    const double m = mean;
    __syncthreads();
    for (int q = threadIdx.x; q < n; q += kBlock) rhs[q] = -(rhs[q] - m);
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += kBlock) {
        const double* row = c.minv + (size_t)r * n;
        double s = 0.0;
        for (int q = 0; q < n; ++q) s += row[q] * rhs[q];
        x[r] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int q = 0; q < n; ++q) s += x[q];
        mean = s / n;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < n; q += kBlock) c.phi[q] = x[q] - mean;
}

// one block per problem: the single-problem k_reduce on each problem's rows
__global__ __launch_bounds__(kBlock) void k_reduce_multi(const ReduceDesc* __restrict__ d) {
    const ReduceDesc r = d[blockIdx.x];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int q = threadIdx.x; q < r.nparts; q += kBlock) {
        const double* p = r.partials + (size_t)q * kReduceWidth;
        a0 += p[0];
        a1 += p[1];
        a2 = fmax(a2, p[2]);
        a3 += p[3];
    }
    block_reduce_row(a0, a1, a2, a3, r.out);
    if (threadIdx.x == 0 && r.copy)
        for (int q = 0; q < kReduceWidth; ++q) r.copy[q] = r.out[q];
}

// ---- batched set-up and finishing kernels ----------------------------------
__global__ __launch_bounds__(kBlock) void k_coeff_rhs_multi(const CoeffDesc* __restrict__ d, int nprob) {
    const int p = find_problem(d, nprob, blockIdx.x);
    const CoeffDesc a = d[p];
    const int b = blockIdx.x - a.block0;
    const int bxi = b % a.gx, byi = (b / a.gx) % a.gy, bzi = b / (a.gx * a.gy);
    if (a.S) coeff_rhs_body<true>(a, bxi, byi, bzi);
    else coeff_rhs_body<false>(a, bxi, byi, bzi);
}

__global__ __launch_bounds__(kBlock) void k_shift_norm_multi(const RowDesc* __restrict__ d, int nprob) {
    const int p = find_problem(d, nprob, blockIdx.x);
    const RowDesc r = d[p];
    shift_norm_body(r.N, r.a, r.shift, r.partials, blockIdx.x - r.block0, r.nb);
}

__global__ __launch_bounds__(kBlock) void k_sum_multi(const RowDesc* __restrict__ d, int nprob) {
    const int p = find_problem(d, nprob, blockIdx.x);
    const RowDesc r = d[p];
    sum_body(r.N, r.a, r.partials, blockIdx.x - r.block0, r.nb);
}

// threads cover the coarse cells of each problem's level
__global__ __launch_bounds__(256) void k_avg_coeff_multi(const AvgDesc* __restrict__ d, int nprob) {
    const int p = find_problem(d, nprob, blockIdx.x);
    const AvgDesc a = d[p];
    const int cx = a.nx / 2, cy = a.ny / 2, cz = a.nz / 2;
    const long long t = (long long)(blockIdx.x - a.block0) * 256 + threadIdx.x;
    if (t >= (long long)cx * cy * cz) return;
    const int I = (int)(t % cx), J = (int)((t / cx) % cy), K = (int)(t / ((long long)cx * cy));
    avg_coeff_cell<double>(a.nx, a.ny, I, J, K, cx, cy, a.bx, a.by, a.bz, a.cbx, a.cby, a.cbz);
}

// one workgroup per problem
template <bool kLds>
__global__ __launch_bounds__(kSetupThreads) void k_coarse_setup_multi(const CoarseDesc* __restrict__ d) {
    __shared__ double Ms[kLds ? kSetupLdsN * kSetupLdsN : 1];
    __shared__ double fac[kCoarseMax];
    __shared__ double prow[kCoarseMax];
    __shared__ double shift;
    const CoarseDesc c = d[blockIdx.x];
    const Bnd<double> none{};
    coarse_setup_body<kLds>(c.nx, c.ny, c.nz, c.h, c.bx, c.by, c.bz, c.minv, none, 0, c.singular, Ms, fac, prow,
                            shift);
}

__global__ __launch_bounds__(256) void k_elt_multi(const EltDesc* __restrict__ d, int nprob) {
    const int p = find_problem(d, nprob, blockIdx.x);
    const EltDesc c = d[p];
    const size_t e = (size_t)(blockIdx.x - c.block0) * 256 + threadIdx.x;
    if (e >= c.n) return;
    switch (c.op) {
        case kEltFill: ((double*)c.dst)[e] = c.s; break;
        case kEltToF32: ((float*)c.dst)[e] = (float)c.src[e]; break;
        default: ((float*)c.dst)[e] = (float)(c.src[e] * c.s); break;
    }
}

__global__ __launch_bounds__(256) void k_correct_multi(const CorrectDesc* __restrict__ d, int nprob) {
    const int p = find_problem(d, nprob, blockIdx.x);
    const CorrectDesc c = d[p];
    const long long t = (long long)(blockIdx.x - c.block0) * 256 + threadIdx.x;
    if (t >= (long long)c.nx * c.ny * c.nz) return;
    const int i = (int)(t % c.nx), j = (int)((t / c.nx) % c.ny), k = (int)(t / ((long long)c.nx * c.ny));
    correct_cell(i, j, k, c.nx, c.ny, c.nz, c.px, c.py, c.pz, c.h, c.b0c, c.b0e, c.bx, c.by, c.bz, c.phi, c.phi_sum,
                 c.u, c.v, c.w, c.phi_out);
}

}  // namespace

int row_blocks(size_t n) { return partial_blocks(n); }
int elt_blocks(size_t n) { return (int)((n + 255) / 256); }
int cell_blocks(size_t n) { return (int)((n + 255) / 256); }
bool coarse_setup_in_lds(size_t n) { return n <= (size_t)kSetupLdsN; }

hipError_t launch_coeff_rhs_multi(const CoeffDesc* d, int nprob, int blocks, hipStream_t st) {
    if (nprob <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_coeff_rhs_multi, dim3(blocks), dim3(kPtX, kPtY), 0, st, d, nprob);
    return hipGetLastError();
}

hipError_t launch_shift_norm_multi(const RowDesc* d, int nprob, int blocks, hipStream_t st) {
    if (nprob <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_shift_norm_multi, dim3(blocks), dim3(kBlock), 0, st, d, nprob);
    return hipGetLastError();
}

hipError_t launch_sum_multi(const RowDesc* d, int nprob, int blocks, hipStream_t st) {
    if (nprob <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_multi, dim3(blocks), dim3(kBlock), 0, st, d, nprob);
    return hipGetLastError();
}

hipError_t launch_avg_coeff_multi(const AvgDesc* d, int nprob, int blocks, hipStream_t st) {
    if (nprob <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_avg_coeff_multi, dim3(blocks), dim3(256), 0, st, d, nprob);
    return hipGetLastError();
}

hipError_t launch_coarse_setup_multi(const CoarseDesc* d, int nprob, bool lds, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    if (lds) hipLaunchKernelGGL(k_coarse_setup_multi<true>, dim3(nprob), dim3(kSetupThreads), 0, st, d);
    else hipLaunchKernelGGL(k_coarse_setup_multi<false>, dim3(nprob), dim3(kSetupThreads), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_elt_multi(const EltDesc* d, int nprob, int blocks, hipStream_t st) {
    if (nprob <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_elt_multi, dim3(blocks), dim3(256), 0, st, d, nprob);
    return hipGetLastError();
}

hipError_t launch_correct_multi(const CorrectDesc* d, int nprob, int blocks, hipStream_t st) {
    if (nprob <= 0 || blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_correct_multi, dim3(blocks), dim3(256), 0, st, d, nprob);
    return hipGetLastError();
}

hipError_t launch_rbgs_multi(const CellDesc* d, int nprob, int blocks, int colour, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rbgs_colour_multi, dim3(blocks), dim3(256), 0, st, d, nprob, colour);
    return hipGetLastError();
}

hipError_t launch_resid_restrict_multi(const CellDesc* d, int nprob, int blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_resid_restrict_multi, dim3(blocks), dim3(256), 0, st, d, nprob);
    return hipGetLastError();
}

hipError_t launch_prolong_multi(const CellDesc* d, int nprob, int blocks, hipStream_t st) {
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_prolong_multi, dim3(blocks), dim3(256), 0, st, d, nprob);
    return hipGetLastError();
}

hipError_t launch_coarse_solve_multi(const CellDesc* d, int nprob, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_coarse_solve_multi, dim3(nprob), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_reduce_multi(const ReduceDesc* d, int nprob, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_multi, dim3(nprob), dim3(kBlock), 0, st, d);
    return hipGetLastError();
}

}  // namespace mg
