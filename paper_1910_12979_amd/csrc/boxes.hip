// Multi-box finest level for gfx950: the domain is tiled by a grid of equal
// boxes, each holding its own phi (with one ghost layer on its faces), f and
// face coefficients.  Smoothing, residual + restriction, prolongation and
// the residual norm of the finest level run box by box (all boxes in one
// launch) with a halo exchange that refills every ghost face from the
// neighbouring box (or the periodic image, or 0 beyond a wall, where the
// face coefficient is 0) after each colour.  Levels 1 and coarser are the
// hierarchy's single-box levels.  This is the layout of a domain whose boxes
// are spread over several devices (the exchange then becomes a message),
// kept on one GPU.
//
// Per cell the arithmetic follows the single-box kernels (face order
// x-low, x-high, y-low, y-high, z-low, z-high; the same division; the same
// restriction order); only the order in which the residual norm is summed
// differs.
//
// Launch shape: every cell kernel runs 256-thread workgroups over 2-D
// (x, y) patches of one plane of one box; the flat workgroup index is split
// into (patch x, patch y, plane, box) with uniform 32-bit arithmetic, so no
// per-thread 64-bit division is needed.
#include <hip/hip_runtime.h>

#include "boxes.h"
#include "devmath.h"
#include "mg_internal.h"

namespace mg {
namespace {

constexpr int kBoxBlock = 256;
constexpr int kCellTX = 64, kCellTY = 4;     // cell kernels: 64 x 4 cells
constexpr int kGsTX = 32, kGsTY = 8;         // one colour: 32 x 8 cells of that colour (64 x 8 cells)
constexpr int kRrTX = 32, kRrTY = 4;         // residual + restriction: 32 x 4 x 2 fine cells
constexpr int kMaxNormBlocks = 2048;         // partial rows available for the norm

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

struct Patch {
    int x0, y0, k, b;
};

// Workgroup t of a launch over gx x gy patches per plane, nz planes per box.
__device__ inline Patch patch_of(unsigned t, int gx, int gy, int nz, int tx, int ty) {
    Patch p;
    const unsigned px = t % (unsigned)gx;
    t /= (unsigned)gx;
    const unsigned py = t % (unsigned)gy;
    t /= (unsigned)gy;
    p.k = (int)(t % (unsigned)nz);
    p.b = (int)(t / (unsigned)nz);
    p.x0 = (int)px * tx;
    p.y0 = (int)py * ty;
    return p;
}

__device__ inline void box_coords(const BoxSet& B, int b, int c[3]) {
    c[0] = b % B.nb[0];
    c[1] = (b / B.nb[0]) % B.nb[1];
    c[2] = b / (B.nb[0] * B.nb[1]);
}

__device__ inline size_t gidx(int i, int j, int k, int nx, int ny) { return ((size_t)k * ny + j) * nx + i; }

// Per-box views (32-bit offsets inside a box).
struct BoxView {
    double* phi;          // ghosted, (B0+2)(B1+2)(B2+2), origin at local (-1, -1, -1)
    const double* f;
    const double* cx;
    const double* cy;
    const double* cz;
    int gx, gxy;          // ghosted row and plane strides
    int B0, B1;
    __device__ inline int p(int i, int j, int k) const { return (k + 1) * gxy + (j + 1) * gx + (i + 1); }
    __device__ inline int c(int i, int j, int k) const { return (k * B1 + j) * B0 + i; }
    __device__ inline int fx(int f, int j, int k) const { return (k * B1 + j) * (B0 + 1) + f; }
    __device__ inline int fy(int i, int f, int k) const { return (k * (B1 + 1) + f) * B0 + i; }
    __device__ inline int fz(int i, int j, int f) const { return (f * B1 + j) * B0 + i; }
};

__device__ inline BoxView view(const BoxSet& B, int b) {
    BoxView v;
    v.phi = B.phi + (size_t)b * B.phi_stride;
    v.f = B.f + (size_t)b * B.f_stride;
    v.cx = B.cx + (size_t)b * B.cx_stride;
    v.cy = B.cy + (size_t)b * B.cy_stride;
    v.cz = B.cz + (size_t)b * B.cz_stride;
    v.gx = B.B[0] + 2;
    v.gxy = (B.B[0] + 2) * (B.B[1] + 2);
    v.B0 = B.B[0];
    v.B1 = B.B[1];
    return v;
}

// The six stored face coefficients of local cell (i, j, k) (x-low, x-high,
// y-low, y-high, z-low, z-high).
__device__ inline void coef6(const BoxView& v, int i, int j, int k, double b[6]) {
    b[0] = v.cx[v.fx(i, j, k)];
    b[1] = v.cx[v.fx(i + 1, j, k)];
    b[2] = v.cy[v.fy(i, j, k)];
    b[3] = v.cy[v.fy(i, j + 1, k)];
    b[4] = v.cz[v.fz(i, j, k)];
    b[5] = v.cz[v.fz(i, j, k + 1)];
}

// (L phi) at local cell (i, j, k), faces in the fixed order.
__device__ inline double box_apply(const BoxView& v, int i, int j, int k, double h2) {
    double b[6];
    coef6(v, i, j, k, b);
    const int c = v.p(i, j, k);
    const double pc = v.phi[c];
    double s = b[0] * (v.phi[c - 1] - pc);
    s = s + b[1] * (v.phi[c + 1] - pc);
    s = s + b[2] * (v.phi[c - v.gx] - pc);
    s = s + b[3] * (v.phi[c + v.gx] - pc);
    s = s + b[4] * (v.phi[c - v.gxy] - pc);
    s = s + b[5] * (v.phi[c + v.gxy] - pc);
    return s * (1.0 / h2);
}

// phi = 0 everywhere, ghosts included.
__global__ __launch_bounds__(kBoxBlock) void k_box_zero(BoxSet B) {
    const size_t n = B.phi_stride * B.nbox;
    for (size_t e = (size_t)blockIdx.x * kBoxBlock + threadIdx.x; e < n; e += (size_t)gridDim.x * kBoxBlock)
        B.phi[e] = 0.0;
}

// f and the face coefficients of every box from the global level-0 arrays
// (cell-aligned low faces; face n of a direction is face 0).
__global__ __launch_bounds__(kBoxBlock) void k_box_scatter(BoxSet B, const double* __restrict__ f,
                                                           const double* __restrict__ bx,
                                                           const double* __restrict__ by,
                                                           const double* __restrict__ bz, int gx, int gy) {
    const Patch q = patch_of(blockIdx.x, gx, gy, B.B[2], kCellTX, kCellTY);
    const int i = q.x0 + (int)threadIdx.x, j = q.y0 + (int)threadIdx.y, k = q.k;
    if (i >= B.B[0] || j >= B.B[1]) return;
    int bc[3];
    box_coords(B, q.b, bc);
    const int gi = bc[0] * B.B[0] + i, gj = bc[1] * B.B[1] + j, gk = bc[2] * B.B[2] + k;
    const int nx = B.n[0], ny = B.n[1], nz = B.n[2];
    BoxView v = view(B, q.b);
    const size_t g = gidx(gi, gj, gk, nx, ny);
    B.f[(size_t)q.b * B.f_stride + v.c(i, j, k)] = f[g];
    double* cx = B.cx + (size_t)q.b * B.cx_stride;
    double* cy = B.cy + (size_t)q.b * B.cy_stride;
    double* cz = B.cz + (size_t)q.b * B.cz_stride;
    cx[v.fx(i, j, k)] = bx[g];
    cy[v.fy(i, j, k)] = by[g];
    cz[v.fz(i, j, k)] = bz[g];
    if (i == B.B[0] - 1) cx[v.fx(i + 1, j, k)] = bx[gidx(gi + 1 < nx ? gi + 1 : 0, gj, gk, nx, ny)];
    if (j == B.B[1] - 1) cy[v.fy(i, j + 1, k)] = by[gidx(gi, gj + 1 < ny ? gj + 1 : 0, gk, nx, ny)];
    if (k == B.B[2] - 1) cz[v.fz(i, j, k + 1)] = bz[gidx(gi, gj, gk + 1 < nz ? gk + 1 : 0, nx, ny)];
}

// Halo exchange: every ghost face cell of every box from the neighbouring
// box's boundary cell (the periodic image at the domain edge, 0 beyond a
// wall).  Workgroup = (chunk of a face, side, box); side 0/1 x low/high,
// 2/3 y, 4/5 z; the face's cells run over its two other directions, first
// fastest.  colour 0 / 1: only the ghosts of that colour (the cells the
// last red or black update changed; a ghost has its source cell's global
// parity); -1: all.
__global__ __launch_bounds__(kBoxBlock) void k_box_exchange(BoxSet B, int chunks, int colour) {
    unsigned t = blockIdx.x;
    const int chunk = (int)(t % (unsigned)chunks);
    t /= (unsigned)chunks;
    const int side = (int)(t % 6u);
    const int b = (int)(t / 6u);
    const int d = side >> 1, hi = side & 1;
    const int a1 = d == 0 ? 1 : 0, a2 = d == 2 ? 1 : 2;     // the face's two directions
    const int nu = B.B[a1], nv = B.B[a2];
    const int q = chunk * kBoxBlock + (int)threadIdx.x;
    if (q >= nu * nv) return;
    int L[3];
    L[a1] = q % nu;
    L[a2] = q / nu;
    L[d] = hi ? B.B[d] : -1;                               // the ghost cell
    if (colour >= 0 && ((L[0] + L[1] + L[2]) & 1) != colour) return;
    int c[3];
    box_coords(B, b, c);
    c[d] += hi ? 1 : -1;                                   // the neighbouring box
    bool wall = false;
    if (c[d] < 0 || c[d] >= B.nb[d]) {
        if (B.per[d]) c[d] = c[d] < 0 ? B.nb[d] - 1 : 0;
        else wall = true;
    }
    const BoxView v = view(B, b);
    double val = 0.0;
    if (!wall) {
        const int sb = (c[2] * B.nb[1] + c[1]) * B.nb[0] + c[0];
        int S[3] = {L[0], L[1], L[2]};
        S[d] = hi ? 0 : B.B[d] - 1;                        // its boundary cell
        val = B.phi[(size_t)sb * B.phi_stride + v.p(S[0], S[1], S[2])];
    }
    v.phi[v.p(L[0], L[1], L[2])] = val;
}

// One colour of red-black Gauss-Seidel in every box; red = (i + j + k)
// even (boxes start at even global coordinates, so the local parity is the
// global one).
__global__ __launch_bounds__(kBoxBlock) void k_box_rbgs(BoxSet B, double h2, int colour, int gx, int gy) {
    const Patch q = patch_of(blockIdx.x, gx, gy, B.B[2], kGsTX, kGsTY);
    const int ih = q.x0 + (int)threadIdx.x, j = q.y0 + (int)threadIdx.y, k = q.k;
    if (2 * ih >= B.B[0] || j >= B.B[1]) return;
    const int i = 2 * ih + ((j + k + colour) & 1);
    const BoxView v = view(B, q.b);
    double b[6];
    coef6(v, i, j, k, b);
    const int c = v.p(i, j, k);
    double num = b[0] * v.phi[c - 1];
    num = num + b[1] * v.phi[c + 1];
    num = num + b[2] * v.phi[c - v.gx];
    num = num + b[3] * v.phi[c + v.gx];
    num = num + b[4] * v.phi[c - v.gxy];
    num = num + b[5] * v.phi[c + v.gxy];
    double den = b[0] + b[1];
    den = den + b[2];
    den = den + b[3];
    den = den + b[4];
    den = den + b[5];
    v.phi[c] = qdiv(num - h2 * v.f[v.c(i, j, k)], den);
}

// Coarse (single-box level 1) f = 1/8 sum of the 8 children's residuals
// (x fastest, then y, then z), coarse phi = 0.  Each thread forms one fine
// residual; the 2 x 2 x 2 sums come from LDS.
__global__ __launch_bounds__(kBoxBlock) void k_box_resid_restrict(BoxSet B, double h2, double* __restrict__ fc,
                                                                  double* __restrict__ phic, int gx, int gy) {
    __shared__ double r[2][kRrTY][kRrTX];
    const Patch q = patch_of(blockIdx.x, gx, gy, B.B[2] / 2, kRrTX, kRrTY);
    const int tx = threadIdx.x, ty = threadIdx.y, tz = threadIdx.z;
    const int i = q.x0 + tx, j = q.y0 + ty, k = 2 * q.k + tz;
    int o[3];
    box_coords(B, q.b, o);
    o[0] *= B.B[0];
    o[1] *= B.B[1];
    o[2] *= B.B[2];
    const BoxView v = view(B, q.b);
    double rv = 0.0;
    if (i < B.B[0] && j < B.B[1]) rv = v.f[v.c(i, j, k)] - box_apply(v, i, j, k, h2);
    r[tz][ty][tx] = rv;
    __syncthreads();
    const int flat = (tz * kRrTY + ty) * kRrTX + tx;
    if (flat >= (kRrTX / 2) * (kRrTY / 2)) return;
    const int cxl = flat % (kRrTX / 2), cyl = flat / (kRrTX / 2);
    if (q.x0 + 2 * cxl >= B.B[0] || q.y0 + 2 * cyl >= B.B[1]) return;
    double s = 0.0;
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) s = s + r[dk][2 * cyl + dj][2 * cxl + di];
    const int Cx = B.n[0] / 2, Cy = B.n[1] / 2;
    const size_t C = gidx((o[0] + q.x0) / 2 + cxl, (o[1] + q.y0) / 2 + cyl, o[2] / 2 + q.k, Cx, Cy);
    fc[C] = 0.125 * s;
    phic[C] = 0.0;
}

// phi += phi_coarse of the parent cell (piecewise constant).
__global__ __launch_bounds__(kBoxBlock) void k_box_prolong(BoxSet B, const double* __restrict__ phic, int gx, int gy) {
    const Patch q = patch_of(blockIdx.x, gx, gy, B.B[2], kCellTX, kCellTY);
    const int i = q.x0 + (int)threadIdx.x, j = q.y0 + (int)threadIdx.y, k = q.k;
    if (i >= B.B[0] || j >= B.B[1]) return;
    int o[3];
    box_coords(B, q.b, o);
    const BoxView v = view(B, q.b);
    const int c = v.p(i, j, k);
    v.phi[c] = v.phi[c] + phic[gidx((o[0] * B.B[0] + i) >> 1, (o[1] * B.B[1] + j) >> 1, (o[2] * B.B[2] + k) >> 1,
                                    B.n[0] >> 1, B.n[1] >> 1)];
}

// Partial rows {sum r^2, 0, max |r|, #non-finite} of r = f - L phi; the
// launch's workgroups stride over the cell patches.
__global__ __launch_bounds__(kBoxBlock) void k_box_resid_norm(BoxSet B, double h2, double* __restrict__ partials,
                                                              int gx, int gy, unsigned npatch) {
    double s = 0.0, mx = 0.0, nonfin = 0.0;
    for (unsigned t = blockIdx.x; t < npatch; t += gridDim.x) {
        const Patch q = patch_of(t, gx, gy, B.B[2], kCellTX, kCellTY);
        const int i = q.x0 + (int)threadIdx.x, j = q.y0 + (int)threadIdx.y;
        if (i >= B.B[0] || j >= B.B[1]) continue;
        const BoxView v = view(B, q.b);
        const double r = v.f[v.c(i, j, q.k)] - box_apply(v, i, j, q.k, h2);
        if (!isfinite(r)) nonfin += 1.0;
        s += r * r;
        mx = fmax(mx, fabs(r));
    }
    __shared__ double sh[3][kBoxBlock];
    const int t = threadIdx.y * kCellTX + threadIdx.x;
    sh[0][t] = s;
    sh[1][t] = mx;
    sh[2][t] = nonfin;
    __syncthreads();
    for (int w = kBoxBlock / 2; w > 0; w >>= 1) {
        if (t < w) {
            sh[0][t] = sh[0][t] + sh[0][t + w];
            sh[1][t] = fmax(sh[1][t], sh[1][t + w]);
            sh[2][t] = sh[2][t] + sh[2][t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        double* row = partials + (size_t)blockIdx.x * kReduceWidth;
        row[0] = sh[0][0];
        row[1] = 0.0;
        row[2] = sh[1][0];
        row[3] = sh[2][0];
    }
}

// Global phi from the boxes' interiors.
__global__ __launch_bounds__(kBoxBlock) void k_box_gather(BoxSet B, double* __restrict__ phi, int gx, int gy) {
    const Patch q = patch_of(blockIdx.x, gx, gy, B.B[2], kCellTX, kCellTY);
    const int i = q.x0 + (int)threadIdx.x, j = q.y0 + (int)threadIdx.y, k = q.k;
    if (i >= B.B[0] || j >= B.B[1]) return;
    int o[3];
    box_coords(B, q.b, o);
    const BoxView v = view(B, q.b);
    phi[gidx(o[0] * B.B[0] + i, o[1] * B.B[1] + j, o[2] * B.B[2] + k, B.n[0], B.n[1])] = v.phi[v.p(i, j, k)];
}

// Workgroups of a cell launch (64 x 4 patches, B2 planes per box).
inline void cell_grid(const BoxSet& B, int& gx, int& gy, unsigned& blocks) {
    gx = cdiv(B.B[0], kCellTX);
    gy = cdiv(B.B[1], kCellTY);
    blocks = (unsigned)gx * gy * B.B[2] * B.nbox;
}

hipError_t exchange(const BoxSet& B, int colour, hipStream_t st) {
    const int chunks = cdiv(B.face_max, kBoxBlock);
    hipLaunchKernelGGL(k_box_exchange, dim3((unsigned)chunks * 6 * B.nbox), dim3(kBoxBlock), 0, st, B, chunks,
                       colour);
    return hipGetLastError();
}

}  // namespace

size_t boxset_cells(const BoxSet& B) { return (size_t)B.B[0] * B.B[1] * B.B[2] * B.nbox; }

hipError_t launch_box_scatter(const BoxSet& B, const double* f, const double* bx, const double* by, const double* bz,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_box_zero, dim3(2048), dim3(kBoxBlock), 0, st, B);
    int gx, gy;
    unsigned blocks;
    cell_grid(B, gx, gy, blocks);
    hipLaunchKernelGGL(k_box_scatter, dim3(blocks), dim3(kCellTX, kCellTY), 0, st, B, f, bx, by, bz, gx, gy);
    return hipGetLastError();
}

hipError_t launch_box_exchange(const BoxSet& B, hipStream_t st) { return exchange(B, -1, st); }

hipError_t launch_box_smooth(const BoxSet& B, double h, int nsweeps, hipStream_t st) {
    const int gx = cdiv(B.B[0] / 2, kGsTX), gy = cdiv(B.B[1], kGsTY);
    const unsigned blocks = (unsigned)gx * gy * B.B[2] * B.nbox;
    for (int s = 0; s < nsweeps; ++s)
        for (int colour = 0; colour < 2; ++colour) {
            hipLaunchKernelGGL(k_box_rbgs, dim3(blocks), dim3(kGsTX, kGsTY), 0, st, B, h * h, colour, gx, gy);
            hipError_t e = exchange(B, colour, st);
            if (e != hipSuccess) return e;
        }
    return hipGetLastError();
}

hipError_t launch_box_resid_restrict(const BoxSet& B, double h, double* fc, double* phic, hipStream_t st) {
    const int gx = cdiv(B.B[0], kRrTX), gy = cdiv(B.B[1], kRrTY);
    const unsigned blocks = (unsigned)gx * gy * (B.B[2] / 2) * B.nbox;
    hipLaunchKernelGGL(k_box_resid_restrict, dim3(blocks), dim3(kRrTX, kRrTY, 2), 0, st, B, h * h, fc, phic, gx, gy);
    return hipGetLastError();
}

hipError_t launch_box_prolong(const BoxSet& B, const double* phic, hipStream_t st) {
    int gx, gy;
    unsigned blocks;
    cell_grid(B, gx, gy, blocks);
    hipLaunchKernelGGL(k_box_prolong, dim3(blocks), dim3(kCellTX, kCellTY), 0, st, B, phic, gx, gy);
    return exchange(B, -1, st);
}

hipError_t launch_box_resid_norm(const BoxSet& B, double h, double* partials, int* nparts, hipStream_t st) {
    int gx, gy;
    unsigned npatch;
    cell_grid(B, gx, gy, npatch);
    const unsigned nb = npatch < (unsigned)kMaxNormBlocks ? npatch : (unsigned)kMaxNormBlocks;
    hipLaunchKernelGGL(k_box_resid_norm, dim3(nb), dim3(kCellTX, kCellTY), 0, st, B, h * h, partials, gx, gy,
                       npatch);
    *nparts = (int)nb;
    return hipGetLastError();
}

hipError_t launch_box_gather(const BoxSet& B, double* phi, hipStream_t st) {
    int gx, gy;
    unsigned blocks;
    cell_grid(B, gx, gy, blocks);
    hipLaunchKernelGGL(k_box_gather, dim3(blocks), dim3(kCellTX, kCellTY), 0, st, B, phi, gx, gy);
    return hipGetLastError();
}

}  // namespace mg
