// Multi-box finest level for gfx950: the domain is tiled by a grid of boxes
// (equal, except that the last box of a direction the box size does not
// divide holds the remainder), each holding its own phi (two buffers), f, rho and face
// coefficients with a two-cell ghost shell.  Smoothing, residual +
// restriction, prolongation and the residual norm of the finest level run
// box by box (all boxes in one launch); a halo exchange refills every ghost
// cell from the box that owns it (or the periodic image, or 0 beyond a
// wall) after each sweep and after an explicit prolongation.  Levels 1 and
// coarser are the hierarchy's single-box levels.  This is the layout of a
// domain whose boxes are spread over several devices (the exchange then
// becomes a message), kept on one GPU.
//
// Boxes of at least 32 x 8 x 4 cells run the single-box finest-level
// kernels on each box interior: the fused out-of-place sweep (its red update
// on a ring around each tile reads the ghost shell, which is why the shell
// is two cells deep and holds f, rho and the coefficients too), with the
// coefficients recomputed from rho for a plane-parallel beta0, the residual
// norm folded into a speculative sweep, the prolongation folded into the
// first post-sweep's load, and the tiled residual + restriction.  Smaller
// boxes use the per-cell kernels below, one launch per colour with an
// exchange of that colour in between.  Either way every cell update is the
// single-box expression, so only the order in which the residual norm and
// the restriction are summed can differ from the single-box solve.
//
// Launch shape of the cell kernels: 256-thread workgroups over 2-D (x, y)
// patches of one plane of one box; the flat workgroup index is split into
// (patch x, patch y, plane, box) with uniform 32-bit arithmetic.
#include <hip/hip_runtime.h>

#include "boxes.h"
#include "devmath.h"
#include "mg_internal.h"
#include "sweep.h"

namespace mg {
namespace {

constexpr int kBoxBlock = 256;
constexpr int kCellTX = 64, kCellTY = 4;     // cell kernels: 64 x 4 cells
constexpr int kGsTX = 32, kGsTY = 8;         // one colour: 32 x 8 cells of that colour (64 x 8 cells)
constexpr int kRrTX = 32, kRrTY = 4;         // residual + restriction: 32 x 4 x 2 fine cells
constexpr int kMaxNormBlocks = 2048;         // partial rows available for the norm
constexpr int kG = kBoxGhost;

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

// Box coordinates and cells of box b.
__device__ inline void box_shape(const BoxSet& B, int b, int c[3], int E[3]) {
    box_coords(B, b, c);
    for (int d = 0; d < 3; ++d) E[d] = box_ext(B, d, c[d]);
}

__device__ inline size_t gidx(int i, int j, int k, int nx, int ny) { return ((size_t)k * ny + j) * nx + i; }

// Per-box view (32-bit offsets inside a box); local cells -kG .. B + kG - 1.
struct BoxView {
    double* phi;
    const double* f;
    const double* cx;
    const double* cy;
    const double* cz;
    int gx, gxy;          // ghosted row and plane strides
    __device__ inline int p(int i, int j, int k) const { return (k + kG) * gxy + (j + kG) * gx + (i + kG); }
};

__device__ inline BoxView view(const BoxSet& B, int b) {
    const size_t o = (size_t)b * B.stride;
    BoxView v;
    v.phi = B.phi + o;
    v.f = B.f + o;
    v.cx = B.cx + o;
    v.cy = B.cy + o;
    v.cz = B.cz + o;
    v.gx = B.G[0];
    v.gxy = B.G[0] * B.G[1];
    return v;
}

// (L phi) at the cell with ghosted index c, faces in the fixed order
// (x-low, x-high, y-low, y-high, z-low, z-high).
__device__ inline double box_apply(const BoxView& v, int c, double h2) {
    const double pc = v.phi[c];
    double s = v.cx[c] * (v.phi[c - 1] - pc);
    s = s + v.cx[c + 1] * (v.phi[c + 1] - pc);
    s = s + v.cy[c] * (v.phi[c - v.gx] - pc);
    s = s + v.cy[c + v.gx] * (v.phi[c + v.gx] - pc);
    s = s + v.cz[c] * (v.phi[c - v.gxy] - pc);
    s = s + v.cz[c + v.gxy] * (v.phi[c + v.gxy] - pc);
    return s * (1.0 / h2);
}

// Global cell of local coordinate L of a box at origin o along direction d:
// wrapped on a periodic direction; -1 beyond a wall.
__device__ inline int box_global(const BoxSet& B, int d, int o, int L) {
    int g = o + L;
    if (g >= 0 && g < B.n[d]) return g;
    if (!B.per[d]) return -1;
    return g < 0 ? g + B.n[d] : g - B.n[d];
}

// phi = phi2 = 0; f and the face arrays of every ghosted cell.  One thread
// per ghosted cell, patches over the ghosted planes.
__global__ __launch_bounds__(kBoxBlock) void k_box_scatter(BoxSet B, const double* __restrict__ f,
                                                           const double* __restrict__ bx,
                                                           const double* __restrict__ by,
                                                           const double* __restrict__ bz,
                                                           const double* __restrict__ rho, int coeffs, int gx,
                                                           int gy) {
    const Patch q = patch_of(blockIdx.x, gx, gy, B.G[2], kCellTX, kCellTY);
    const int i = q.x0 + (int)threadIdx.x, j = q.y0 + (int)threadIdx.y;
    if (i >= B.G[0] || j >= B.G[1]) return;
    const size_t e = (size_t)q.b * B.stride + ((size_t)q.k * B.G[1] + j) * B.G[0] + i;
    int c[3];
    box_coords(B, q.b, c);
    const int L[3] = {i - kG, j - kG, q.k - kG};
    int g[3];
    int out = 0, wall_d = -1;                 // directions beyond a wall; the one at a high wall face
    for (int d = 0; d < 3; ++d) {
        g[d] = box_global(B, d, c[d] * B.B[d], L[d]);
        if (g[d] < 0) {
            ++out;
            if (c[d] * B.B[d] + L[d] == B.n[d]) wall_d = d;
        }
    }
    B.phi[e] = 0.0;
    B.phi2[e] = 0.0;     // cells past a smaller box's shell are read by the tile windows, never written
    double fv = 0.0, cv[3] = {1.0, 1.0, 1.0}, rv = 1.0;
    if (out == 0) {
        const size_t gi = gidx(g[0], g[1], g[2], B.n[0], B.n[1]);
        fv = f[gi];
        if (rho) rv = rho[gi];
        cv[0] = bx[gi];
        cv[1] = by[gi];
        cv[2] = bz[gi];
    } else if (out == 1 && wall_d >= 0) {
        cv[wall_d] = 0.0;                     // the first cell past a high wall: its low face is the wall
    }
    B.f[e] = fv;
    if (rho) B.rho[e] = rv;
    if (!coeffs) return;
    B.cx[e] = cv[0];
    B.cy[e] = cv[1];
    B.cz[e] = cv[2];
}

// beta0 at the centre and low face of every ghosted plane of every box: the
// global layer (periodic image; beyond a wall the nearest layer or face).
__global__ void k_box_beta0(BoxSet B, const double* __restrict__ b0c, const double* __restrict__ b0e) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B.nbox * B.G[2]) return;
    const int b = e / B.G[2], t = e % B.G[2];
    const int kb = b / (B.nb[0] * B.nb[1]);
    int z = kb * B.B[2] + t - kG;
    const int nz = B.n[2];
    int zc, ze;
    if (B.per[2]) {
        zc = z < 0 ? z + nz : (z >= nz ? z - nz : z);
        ze = zc;
    } else {
        zc = z < 0 ? 0 : (z >= nz ? nz - 1 : z);
        ze = z < 0 ? 0 : (z > nz ? nz : z);
    }
    B.b0c[e] = b0c[zc];
    B.b0e[e] = b0e[ze];
}

// Halo exchange over the ghost shell of every box: workgroup (chunk,
// plane, box) treats up to kExChunk shell cells of one ghosted plane (all of
// a ghost plane, the two-cell border of an interior plane).  colour 0 / 1:
// only that colour's ghosts (a ghost has the global parity of its cell);
// -1: all.
constexpr int kExChunk = 4 * kBoxBlock;
template <typename T>
__global__ __launch_bounds__(kBoxBlock) void k_box_exchange(BoxSet B, T* __restrict__ arr, int colour, int chunks) {
    const int G2 = B.G[2];
    const int chunk = (int)(blockIdx.x % (unsigned)chunks);
    const int kp = (int)((blockIdx.x / (unsigned)chunks) % (unsigned)G2);
    const int b = (int)(blockIdx.x / ((unsigned)chunks * G2));
    const int k = kp - kG;
    int c[3], E[3];
    box_shape(B, b, c, E);
    if (k >= E[2] + kG) return;               // past this box's ghost shell
    const int W0 = E[0] + 2 * kG, W1 = E[1] + 2 * kG;
    const bool ghost_plane = k < 0 || k >= E[2];
    const int ncell = ghost_plane ? W0 * W1 : 2 * kG * W0 + 2 * kG * E[1];
    const int gx = B.G[0], gxy = B.G[0] * B.G[1];
    auto p = [&](int i, int j, int k) { return (k + kG) * gxy + (j + kG) * gx + (i + kG); };
    T* own = arr + (size_t)b * B.stride;
    const int e_end = min(ncell, (chunk + 1) * kExChunk);
    for (int e = chunk * kExChunk + threadIdx.x; e < e_end; e += kBoxBlock) {
        int i, j;
        if (ghost_plane) {
            i = e % W0 - kG;
            j = e / W0 - kG;
        } else if (e < 2 * kG * W0) {         // the ghost rows, whole
            const int r = e / W0;
            j = r < kG ? r - kG : E[1] + r - kG;
            i = e % W0 - kG;
        } else {                              // the ghost columns of the interior rows
            const int e2 = e - 2 * kG * W0;
            j = e2 / (2 * kG);
            const int r = e2 % (2 * kG);
            i = r < kG ? r - kG : E[0] + r - kG;
        }
        if (colour >= 0 && ((i + j + k) & 1) != colour) continue;
        // the owner is the adjacent box in each direction the ghost leaves
        // (a ghost at most two cells out, boxes at least two cells wide);
        // past the high side its local coordinate starts at 0, below the low
        // side it counts back from the owner's last cell
        const int L[3] = {i, j, k};
        int S[3], o[3];
        bool wall = false;
        for (int d = 0; d < 3; ++d) {
            const int step = L[d] < 0 ? -1 : (L[d] >= E[d] ? 1 : 0);
            o[d] = c[d] + step;
            if (o[d] < 0 || o[d] >= B.nb[d]) {
                if (B.per[d]) o[d] = o[d] < 0 ? B.nb[d] - 1 : 0;
                else wall = true;
            }
            S[d] = step > 0 ? L[d] - E[d] : (step < 0 ? L[d] + box_ext(B, d, wall ? 0 : o[d]) : L[d]);
        }
        T val = T(0);
        if (!wall) {
            const int sb = (o[2] * B.nb[1] + o[1]) * B.nb[0] + o[0];
            val = arr[(size_t)sb * B.stride + p(S[0], S[1], S[2])];
        }
        own[p(i, j, k)] = val;
    }
}

// One colour of red-black Gauss-Seidel in every box (boxes too small for
// the fused sweep); red = (i + j + k) even (boxes start at even global
// coordinates, so the local parity is the global one).
__global__ __launch_bounds__(kBoxBlock) void k_box_rbgs(BoxSet B, double h2, int colour, int gx, int gy) {
    const Patch q = patch_of(blockIdx.x, gx, gy, B.B[2], kGsTX, kGsTY);
    const int ih = q.x0 + (int)threadIdx.x, j = q.y0 + (int)threadIdx.y, k = q.k;
    int c3[3], E[3];
    box_shape(B, q.b, c3, E);
    if (2 * ih >= E[0] || j >= E[1] || k >= E[2]) return;
    const int i = 2 * ih + ((j + k + colour) & 1);
    const BoxView v = view(B, q.b);
    const int c = v.p(i, j, k);
    const double bxl = v.cx[c], bxh = v.cx[c + 1];
    const double byl = v.cy[c], byh = v.cy[c + v.gx];
    const double bzl = v.cz[c], bzh = v.cz[c + v.gxy];
    double num = bxl * v.phi[c - 1];
    num = num + bxh * v.phi[c + 1];
    num = num + byl * v.phi[c - v.gx];
    num = num + byh * v.phi[c + v.gx];
    num = num + bzl * v.phi[c - v.gxy];
    num = num + bzh * v.phi[c + v.gxy];
    double den = bxl + bxh;
    den = den + byl;
    den = den + byh;
    den = den + bzl;
    den = den + bzh;
    v.phi[c] = qdiv(num - h2 * v.f[c], den);
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
    int o[3], E[3];
    box_shape(B, q.b, o, E);
    o[0] *= B.B[0];
    o[1] *= B.B[1];
    o[2] *= B.B[2];
    const BoxView v = view(B, q.b);
    double rv = 0.0;
    if (i < E[0] && j < E[1] && k < E[2]) {
        const int c = v.p(i, j, k);
        rv = v.f[c] - box_apply(v, c, h2);
    }
    r[tz][ty][tx] = rv;
    __syncthreads();
    const int flat = (tz * kRrTY + ty) * kRrTX + tx;
    if (flat >= (kRrTX / 2) * (kRrTY / 2)) return;
    const int cxl = flat % (kRrTX / 2), cyl = flat / (kRrTX / 2);
    if (q.x0 + 2 * cxl >= E[0] || q.y0 + 2 * cyl >= E[1] || 2 * q.k >= E[2]) return;
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
    int o[3], E[3];
    box_shape(B, q.b, o, E);
    if (i >= E[0] || j >= E[1] || k >= E[2]) return;
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
        int c3[3], E[3];
        box_shape(B, q.b, c3, E);
        if (i >= E[0] || j >= E[1] || q.k >= E[2]) continue;
        const BoxView v = view(B, q.b);
        const int c = v.p(i, j, q.k);
        const double r = v.f[c] - box_apply(v, c, h2);
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
    int o[3], E[3];
    box_shape(B, q.b, o, E);
    if (i >= E[0] || j >= E[1] || k >= E[2]) return;
    const BoxView v = view(B, q.b);
    phi[gidx(o[0] * B.B[0] + i, o[1] * B.B[1] + j, o[2] * B.B[2] + k, B.n[0], B.n[1])] = v.phi[v.p(i, j, k)];
}

// Workgroups of a cell launch over the box interiors (64 x 4 patches).
inline void cell_grid(const BoxSet& B, int& gx, int& gy, unsigned& blocks) {
    gx = cdiv(B.B[0], kCellTX);
    gy = cdiv(B.B[1], kCellTY);
    blocks = (unsigned)gx * gy * B.B[2] * B.nbox;
}

template <typename T>
hipError_t exchange_arr(const BoxSet& B, T* arr, int colour, hipStream_t st) {
    const int chunks = cdiv(B.G[0] * B.G[1], kExChunk);
    hipLaunchKernelGGL(k_box_exchange<T>, dim3((unsigned)chunks * B.G[2] * B.nbox), dim3(kBoxBlock), 0, st, B, arr,
                       colour, chunks);
    return hipGetLastError();
}

hipError_t exchange(const BoxSet& B, int colour, hipStream_t st) { return exchange_arr<double>(B, B.phi, colour, st); }

// f32 = s f (s a power of two) and the plain FP32 copies, over whole arrays.
__global__ void k_box_f32(size_t n, const double* __restrict__ a, float* __restrict__ b, double s) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        b[i] = (float)(s * a[i]);
}

}  // namespace

size_t boxset_cells(const BoxSet& B) { return (size_t)B.n[0] * B.n[1] * B.n[2]; }

hipError_t launch_box_scatter(const BoxSet& B, const double* f, const double* bx, const double* by, const double* bz,
                              const double* rho, const double* b0c, const double* b0e, bool coeffs, hipStream_t st) {
    const int gx = cdiv(B.G[0], kCellTX), gy = cdiv(B.G[1], kCellTY);
    const unsigned blocks = (unsigned)gx * gy * B.G[2] * B.nbox;
    hipLaunchKernelGGL(k_box_scatter, dim3(blocks), dim3(kCellTX, kCellTY), 0, st, B, f, bx, by, bz, rho,
                       coeffs ? 1 : 0, gx, gy);
    if (rho)
        hipLaunchKernelGGL(k_box_beta0, dim3(cdiv(B.nbox * B.G[2], kBoxBlock)), dim3(kBoxBlock), 0, st, B, b0c, b0e);
    return hipGetLastError();
}

hipError_t launch_box_exchange(const BoxSet& B, int colour, hipStream_t st) { return exchange(B, colour, st); }

// Arguments of the fused sweep over every box interior (FP64 arrays; the
// FP32 ones by box_sweep_args32).
SweepArgs<double> box_sweep_args(const BoxSet& B, double h) {
    SweepArgs<double> a{};
    a.nx = B.G[0];
    a.ny = B.G[1];
    a.nz = B.G[2];
    a.px = a.py = a.pz = 1;
    a.ox = a.oy = a.oz = kG;
    a.ex = B.B[0];
    a.ey = B.B[1];
    a.ez = B.B[2];
    a.h2 = h * h;
    a.f = B.f;
    a.bx = B.cx;
    a.by = B.cy;
    a.bz = B.cz;
    if (B.rho_on) {
        a.rho = B.rho;
        a.b0c = B.b0c;
        a.b0e = B.b0e;
    }
    return a;
}

SweepArgs<float> box_sweep_args32(const BoxSet& B, double h) {
    SweepArgs<float> a{};
    a.nx = B.G[0];
    a.ny = B.G[1];
    a.nz = B.G[2];
    a.px = a.py = a.pz = 1;
    a.ox = a.oy = a.oz = kG;
    a.ex = B.B[0];
    a.ey = B.B[1];
    a.ez = B.B[2];
    a.h2 = (float)(h * h);
    a.f = B.f32;
    a.bx = B.cx32;
    a.by = B.cy32;
    a.bz = B.cz32;
    if (B.rho_on) {
        a.rho = B.rho32;
        a.b0c = B.b0c;
        a.b0e = B.b0e;
    }
    return a;
}

BoxGeom box_geom(const BoxSet& B) {
    BoxGeom g;
    for (int d = 0; d < 3; ++d) {
        g.nb[d] = B.nb[d];
        g.per[d] = B.per[d];
    }
    g.b0stride = B.G[2];
    for (int d = 0; d < 3; ++d) {
        g.box[d] = B.B[d];
        g.n[d] = B.n[d];
    }
    return g;
}

hipError_t launch_box_smooth(BoxSet& B, double h, int nsweeps, hipStream_t st, const double* phic) {
    if (phic && !(B.fused && nsweeps >= 1)) {
        hipError_t e = launch_box_prolong(B, phic, st);
        if (e != hipSuccess) return e;
        phic = nullptr;
    }
    if (B.fused) {
        SweepArgs<double> a = box_sweep_args(B, h);
        a.phic = phic;
        for (int s = 0; s < nsweeps; ++s) {
            a.phi_in = B.phi;
            a.phi_out = B.phi2;
            hipError_t e = launch_sweep_boxes(a, box_geom(B), B.nbox, B.stride, nullptr, st, s == 0 && phic);
            if (e != hipSuccess) return e;
            std::swap(B.phi, B.phi2);
            e = exchange(B, -1, st);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
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

bool box_norm_sweep_fits(const BoxSet& B) {
    return B.fused && (long long)sweep_boxes_tiles(B.B[0], B.B[1], B.B[2]) * B.nbox <= kMaxPartialRows;
}

hipError_t launch_box_sweep_norm(const BoxSet& B, double h, double* partials, int* nparts, hipStream_t st) {
    if (!box_norm_sweep_fits(B)) return hipErrorInvalidValue;
    SweepArgs<double> a = box_sweep_args(B, h);
    a.phi_in = B.phi;
    a.phi_out = B.phi2;
    a.partials = partials;
    return launch_sweep_boxes(a, box_geom(B), B.nbox, B.stride, nparts, st);
}

hipError_t launch_box_resid_restrict(const BoxSet& B, double h, double* fc, double* phic, hipStream_t st) {
    if (B.fused) {                            // the fused sweep's tiles, no sweep
        SweepArgs<double> a = box_sweep_args(B, h);
        a.phi_in = B.phi;
        a.fc = fc;
        a.phic_out = phic;
        return launch_sweep_boxes(a, box_geom(B), B.nbox, B.stride, nullptr, st, false, true);
    }
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

// ---- mixed precision ------------------------------------------------------
hipError_t launch_box_to_f32(const BoxSet& B, double s, hipStream_t st) {
    const size_t n = B.stride * B.nbox;
    const unsigned blocks = (unsigned)std::min<size_t>((n + kBoxBlock - 1) / kBoxBlock, 4096);
    hipLaunchKernelGGL(k_box_f32, dim3(blocks), dim3(kBoxBlock), 0, st, n, B.f, B.f32, s);
    if (B.rho_on) {
        hipLaunchKernelGGL(k_box_f32, dim3(blocks), dim3(kBoxBlock), 0, st, n, B.rho, B.rho32, 1.0);
    } else {
        hipLaunchKernelGGL(k_box_f32, dim3(blocks), dim3(kBoxBlock), 0, st, n, B.cx, B.cx32, 1.0);
        hipLaunchKernelGGL(k_box_f32, dim3(blocks), dim3(kBoxBlock), 0, st, n, B.cy, B.cy32, 1.0);
        hipLaunchKernelGGL(k_box_f32, dim3(blocks), dim3(kBoxBlock), 0, st, n, B.cz, B.cz32, 1.0);
    }
    return hipGetLastError();
}

hipError_t launch_box_smooth32(BoxSet& B, double h, int nsweeps, bool zero_first, const float* phic,
                               hipStream_t st) {
    if (!B.fused || !B.phi32) return hipErrorInvalidValue;
    SweepArgs<float> a = box_sweep_args32(B, h);
    a.phic = phic;
    for (int s = 0; s < nsweeps; ++s) {
        a.phi_in = B.phi32;
        a.phi_out = B.phi2_32;
        const int mode = s > 0 ? kBoxSweep : (zero_first ? kBoxSweepZero : (phic ? kBoxSweepProlong : kBoxSweep));
        hipError_t e = launch_sweep_boxes_mode<float>(a, box_geom(B), B.nbox, B.stride, mode, nullptr, st);
        if (e != hipSuccess) return e;
        std::swap(B.phi32, B.phi2_32);
        e = exchange_arr<float>(B, B.phi32, -1, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_box_resid_restrict32(const BoxSet& B, double h, float* fc, float* phic, hipStream_t st) {
    if (!B.fused || !B.phi32) return hipErrorInvalidValue;
    SweepArgs<float> a = box_sweep_args32(B, h);
    a.phi_in = B.phi32;
    a.fc = fc;
    a.phic_out = phic;
    return launch_sweep_boxes_mode<float>(a, box_geom(B), B.nbox, B.stride, kBoxResidRestrict, nullptr, st);
}

hipError_t launch_box_refine(BoxSet& B, double h, const double* scales, double* partials, int* nparts,
                             hipStream_t st) {
    if (!B.fused || !B.phi32) return hipErrorInvalidValue;
    SweepArgs<double> a = box_sweep_args(B, h);
    a.phi_in = B.phi;
    a.phi_out = B.phi2;
    a.corr = B.phi32;
    a.r32 = B.f32;
    a.scales = scales;
    a.partials = partials;
    hipError_t e = launch_sweep_boxes_mode<double>(a, box_geom(B), B.nbox, B.stride, kBoxRefine, nparts, st);
    if (e != hipSuccess) return e;
    std::swap(B.phi, B.phi2);
    e = exchange_arr<double>(B, B.phi, -1, st);
    if (e != hipSuccess) return e;
    return exchange_arr<float>(B, B.f32, -1, st);
}

}  // namespace mg
