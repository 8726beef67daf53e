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
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <utility>
#include <vector>
#include <new>
#include <string>

#include "dense.h"
#include "devmath.h"
#include "mg_internal.h"
#include "runtime.h"

namespace mg {
namespace {

constexpr int kNodBlock = 256;
constexpr int kNodSetupThreads = 1024;

// One level of the nodal hierarchy: cells (nx, ny, nz), nodes (Nx, Ny, Nz);
// arrays in T (FP64, or FP32 for the inner cycle of a mixed-precision solve).
template <typename T>
struct NodLevelT {
    int nx, ny, nz;
    int Nx, Ny, Nz;
    int px, py, pz;
    double h;
    T* sig;             // cells
    T* phi;             // nodes
    T* f;
    T* r;
    T* phi2;            // nodes: the other buffer of the out-of-place fused sweep
    __host__ __device__ size_t nodes() const { return (size_t)Nx * Ny * Nz; }
    __host__ __device__ size_t cells() const { return (size_t)nx * ny * nz; }
};
using NodLevel = NodLevelT<double>;

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

template <typename T>
__device__ inline size_t nidx(const NodLevelT<T>& L, int I, int J, int K) {
    return ((size_t)K * L.Ny + J) * L.Nx + I;
}

template <typename T>
__device__ inline size_t cidx3(const NodLevelT<T>& L, int i, int j, int k) {
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
template <typename T>
struct NodNbr {
    T v[3][3][3];
};

template <typename T>
__device__ inline void nod_load_nbrs(const NodLevelT<T>& L, const T* __restrict__ phi, int I, const NodAxis& ax,
                                     const NodAxis& ay, const NodAxis& az, int J, int K, NodNbr<T>& N) {
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
                N.v[dz + 1][dy + 1][dx + 1] = ok ? phi[zi * NxNy + yi * Nx + xi] : T(0);
            }
}

// num = sum_c sigma_c sum_{4 far corners} phi, den = 4 sum_c sigma_c over
// the existing cells at node (I, J, K), in the oracle's order (cells sz, sy,
// sx; far corners of the cell on side (sx, sy, sz): x+y, x+z, y+z, x+y+z
// moved), with per-axis index tables and each neighbour loaded once.
template <typename T>
__device__ inline void nod_stencil_fast(const NodLevelT<T>& L, const T* __restrict__ phi, int I, int J, int K,
                                        T& num, T& den) {
    const NodAxis ax = nod_axis(I, L.Nx, L.nx, L.px);
    const NodAxis ay = nod_axis(J, L.Ny, L.ny, L.py);
    const NodAxis az = nod_axis(K, L.Nz, L.nz, L.pz);
    NodNbr<T> N;
    nod_load_nbrs(L, phi, I, ax, ay, az, J, K, N);
    const long long nx = L.nx, nxny = (long long)L.nx * L.ny;
    num = T(0);
    den = T(0);
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
                const T sig = L.sig[az.c[sz] * nxny + ay.c[sy] * nx + ax.c[sx]];
                T acc = T(0);
                acc += N.v[1][oy][ox];
                acc += N.v[oz][1][ox];
                acc += N.v[oz][oy][1];
                acc += N.v[oz][oy][ox];
                num += sig * acc;
                den += T(4) * sig;
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
template <typename T>
__global__ void k_nod_gs(NodLevelT<T> L, int col) {
    const int I = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    const int J = 2 * (int)(blockIdx.y * blockDim.y + threadIdx.y) + (col & 1);
    const int K = 2 * (int)(blockIdx.z * blockDim.z + threadIdx.z) + (col >> 1);
    if (I >= L.Nx || J >= L.Ny || K >= L.Nz) return;
    T num, den;
    nod_stencil_fast(L, L.phi, I, J, K, num, den);
    const size_t n = nidx(L, I, J, K);
    const T c12 = (T)(12.0 * (L.h * L.h));
    L.phi[n] = pdiv(num - c12 * L.f[n], den);
}

// ---------------------------------------------------------------------------
// Fused out-of-place sweep: out = the four-colour Gauss-Seidel sweep of
// L.phi (colours 0..3 in order), one launch.
//
// Colour c of node (I, J, K) is (J mod 2) + 2 (K mod 2); every row of nodes
// along x has one colour.  Coupled nodes differ in at least two coordinates,
// so in an even plane colour 0 reads only old values and colour 1 the new
// colour-0 values of its four in-plane diagonal neighbours (old values
// above and below); in an odd plane colour 2 reads the new values of the
// even planes above and below, colour 3 those and the new colour-2 values of
// its in-plane diagonal neighbours.
//
// A workgroup owns a TX x TY tile of nodes and a chunk of planes and marches
// up through it, one even plane and the odd plane below it per step:
// colour 0 of the even plane on the tile plus a ring of 3, colour 1 on ring
// 2, then colour 2 of the odd plane on ring 1 and colour 3 on the tile, so
// every value a later colour reads was computed by the workgroup itself;
// loads cover the tile plus a ring of 4.  New values overwrite old ones in
// place in the LDS plane buffers (a colour reads only rows of the other
// colour of its plane), so a plane needs one buffer: four rolling node
// planes (even plane below, the odd plane, the even plane, the odd plane
// above) and three rolling cell layers.  The even plane at the top of a
// chunk is computed again by the next chunk (it reads only old values).
// Cells beyond a wall carry sigma = 0 and nodes beyond it the value 0, so
// their terms add exact zeros.  The per-node sums are the per-colour
// kernel's, term by term, with the sigma products accumulated by fused
// multiply-adds (the two kernels agree to rounding).
//
// Each thread owns one column x of the window and a pair of rows (even J,
// odd J): one node per colour stage.
// ---------------------------------------------------------------------------
__device__ inline int nod_wrapi(int g, int n) {
    g %= n;
    return g < 0 ? g + n : g;
}
__device__ inline int nod_m3(int k) {
    k %= 3;
    return k < 0 ? k + 3 : k;
}

template <typename T, int TX, int TY>
__global__ __launch_bounds__((TX + 8) * (TY + 8) / 2) void k_nod_sweep(NodLevelT<T> L, T* __restrict__ out, int tz,
                                                                      int ntx, int nty, int etop) {
    constexpr int WX = TX + 8, WY = TY + 8, WP = WY / 2;
    __shared__ T sp[4][WY][WX];             // node planes, by plane & 3
    __shared__ T ss[3][WY - 1][WX];         // cell layers, by layer mod 3; [jw][wx]: the cell whose low corner is
                                            // node (wx, jw) (the window's last row of cells is never read)
    const int tile = blockIdx.x;
    const int tx = tile % ntx, ty = (tile / ntx) % nty, tc = tile / (ntx * nty);
    const int ks = tc * tz;
    const int ke = min(ks + tz, etop);
    const int wx = threadIdx.x % WX, p = threadIdx.x / WX;
    const int je = 2 * p, jo = 2 * p + 1;                  // window rows of the pair
    const int gI = tx * TX - 4 + wx;                       // global node / low-corner cell coordinates
    const int gJe = ty * TY - 4 + je, gJo = gJe + 1;
    // existence along x and y (nodes and the cells whose low corner they are)
    const bool xn = L.px || (gI >= 0 && gI < L.Nx), xc = L.px || (gI >= 0 && gI < L.nx);
    const bool yne = L.py || (gJe >= 0 && gJe < L.Ny), yce = L.py || (gJe >= 0 && gJe < L.ny);
    const bool yno = L.py || (gJo >= 0 && gJo < L.Ny), yco = L.py || (gJo >= 0 && gJo < L.ny);
    const int Iw = L.px ? nod_wrapi(gI, L.Nx) : min(max(gI, 0), L.Nx - 1);
    const int Jwe = L.py ? nod_wrapi(gJe, L.Ny) : min(max(gJe, 0), L.Ny - 1);
    const int Jwo = L.py ? nod_wrapi(gJo, L.Ny) : min(max(gJo, 0), L.Ny - 1);
    const int iw = L.px ? nod_wrapi(gI, L.nx) : min(max(gI, 0), L.nx - 1);
    const int jwe = L.py ? nod_wrapi(gJe, L.ny) : min(max(gJe, 0), L.ny - 1);
    const int jwo = L.py ? nod_wrapi(gJo, L.ny) : min(max(gJo, 0), L.ny - 1);
    const size_t NxNy = (size_t)L.Nx * L.Ny, nxny = (size_t)L.nx * L.ny;
    const size_t ne = (size_t)Jwe * L.Nx + Iw, no = (size_t)Jwo * L.Nx + Iw;
    const size_t ce = (size_t)jwe * L.nx + iw, co = (size_t)jwo * L.nx + iw;
    const T c12 = (T)(12.0 * (L.h * L.h));

    auto plane_ok = [&](int K) { return L.pz || (K >= 0 && K < L.Nz); };
    auto layer_ok = [&](int k) { return L.pz || (k >= 0 && k < L.nz); };
    auto pw = [&](int K) { return L.pz ? nod_wrapi(K, L.Nz) : min(max(K, 0), L.Nz - 1); };
    auto lw = [&](int k) { return L.pz ? nod_wrapi(k, L.nz) : min(max(k, 0), L.nz - 1); };
    // Loads are always issued from valid (wrapped or clamped) addresses, so
    // a set of them is plain load results the compiler never has to wait for
    // early; the values of nodes and cells beyond a wall are replaced by 0
    // when they are stored into LDS.
    auto ld_phi = [&](int K, T& a, T& b) {
        const size_t o = (size_t)pw(K) * NxNy;
        a = L.phi[o + ne];
        b = L.phi[o + no];
    };
    auto ld_sig = [&](int k, T& a, T& b) {
        const size_t o = (size_t)lw(k) * nxny;
        a = L.sig[o + ce];
        b = L.sig[o + co];
    };
    auto ld_f = [&](int K, T& a, T& b) {
        const size_t o = (size_t)pw(K) * NxNy;
        a = L.f[o + ne];
        b = L.f[o + no];
    };
    auto st_phi = [&](int K, T a, T b) {
        const bool ok = plane_ok(K) && xn;
        sp[K & 3][je][wx] = (ok && yne) ? a : T(0);
        sp[K & 3][jo][wx] = (ok && yno) ? b : T(0);
    };
    auto st_sig = [&](int k, T a, T b) {
        const bool ok = layer_ok(k) && xc;
        ss[nod_m3(k)][je][wx] = (ok && yce) ? a : T(0);
        if (jo < WY - 1) ss[nod_m3(k)][jo][wx] = (ok && yco) ? b : T(0);
    };
    // the update of window node (x, y) of plane slot pc with planes below
    // (pm) and above (pp) and cell layers below (sm) and above (sq): the 20
    // coupled neighbours and 8 cell coefficients are read from LDS first (all
    // loads independent), then combined in the per-colour kernel's order:
    // cells sz, sy, sx; far corners x+y, x+z, y+z, x+y+z
    auto update = [&](int x, int y, int pm, int pc, int pp, int sm, int sq, T fv) -> T {
        T v[3][3][3];
        T sg[2][2][2];
#pragma unroll
        for (int dz = 0; dz < 3; ++dz) {
            const int pl = dz == 0 ? pm : (dz == 1 ? pc : pp);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
                    v[dz][dy][dx] = ((dx != 1) + (dy != 1) + (dz != 1) >= 2) ? sp[pl][y - 1 + dy][x - 1 + dx] : T(0);
        }
#pragma unroll
        for (int sz = 0; sz < 2; ++sz)
#pragma unroll
            for (int sy = 0; sy < 2; ++sy)
#pragma unroll
                for (int sx = 0; sx < 2; ++sx) sg[sz][sy][sx] = ss[sz ? sq : sm][y - 1 + sy][x - 1 + sx];
        T num = T(0), den = T(0);
#pragma unroll
        for (int sz = 0; sz < 2; ++sz) {
            const int oz = sz ? 2 : 0;
#pragma unroll
            for (int sy = 0; sy < 2; ++sy) {
                const int oy = sy ? 2 : 0;
#pragma unroll
                for (int sx = 0; sx < 2; ++sx) {
                    const int ox = sx ? 2 : 0;
                    const T sig = sg[sz][sy][sx];
                    T acc = v[1][oy][ox];
                    acc += v[oz][1][ox];
                    acc += v[oz][oy][1];
                    acc += v[oz][oy][ox];
                    num = fma(sig, acc, num);
                    den = fma(T(4), sig, den);
                }
            }
        }
        return pdiv(num - c12 * fv, den);
    };

    // rings (window rows / columns) of the four colour stages
    const bool colx3 = wx >= 1 && wx < WX - 1, colx2 = wx >= 2 && wx < WX - 2;
    const bool colx1 = wx >= 3 && wx < WX - 3, colx0 = wx >= 4 && wx < WX - 4;
    const bool st0 = colx3 && p >= 1 && p <= WP - 1 && xn && yne;        // colour 0 / 2 row: even
    const bool st1 = colx2 && p >= 1 && p <= WP - 2 && xn && yno;        // colour 1 / 3 row: odd
    const bool st2 = colx1 && p >= 2 && p <= WP - 2 && xn && yne;
    const bool st3 = colx0 && p >= 2 && p <= WP - 3 && xn && yno;
    const bool tile_pair = colx0 && p >= 2 && p <= WP - 3 && gI < L.Nx;   // output nodes (unwrapped inside the box)
    const bool oute = tile_pair && gJe < L.Ny, outo = tile_pair && gJo < L.Ny;

    // prologue: planes ks-1, ks, ks+1, layers ks-1, ks, f of plane ks
    {
        T a0, b0, a1, b1, a2, b2, a3, b3, a4, b4;
        ld_phi(ks - 1, a0, b0);
        ld_phi(ks, a1, b1);
        ld_phi(ks + 1, a2, b2);
        ld_sig(ks - 1, a3, b3);
        ld_sig(ks, a4, b4);
        st_phi(ks - 1, a0, b0);
        st_phi(ks, a1, b1);
        st_phi(ks + 1, a2, b2);
        st_sig(ks - 1, a3, b3);
        st_sig(ks, a4, b4);
    }
    T fe0, fo0, fe1 = T(0), fo1 = T(0);         // f of the even plane (e/o rows), of the odd plane below
    ld_f(ks, fe0, fo0);
    __syncthreads();

    for (int E = ks; E <= ke; E += 2) {
        // next step's loads in flight: planes E+2, E+3, layers E+1, E+2, f of planes E+2, E+1
        const bool more = E + 2 <= ke;
        T q0, q1, q2, q3, s0, s1, s2, s3, nfe, nfo, nfe1, nfo1;
        ld_phi(E + 2, q0, q1);
        ld_phi(E + 3, q2, q3);
        ld_sig(E + 1, s0, s1);
        ld_sig(E + 2, s2, s3);
        ld_f(E + 2, nfe, nfo);
        ld_f(E + 1, nfe1, nfo1);
        const int pm = (E - 1) & 3, pc = E & 3, pp = (E + 1) & 3, pmm = (E - 2) & 3;
        const int sm = nod_m3(E - 1), sq = nod_m3(E), smm = nod_m3(E - 2);
        const bool even_ok = plane_ok(E);
        // A: colour 0 of plane E (ring 3)
        T ve = T(0), vo = T(0);
        if (st0 && even_ok) {
            ve = update(wx, je, pm, pc, pp, sm, sq, fe0);
            sp[pc][je][wx] = ve;
        }
        __syncthreads();
        // B: colour 1 of plane E (ring 2); plane E written where this chunk owns it
        if (st1 && even_ok) {
            vo = update(wx, jo, pm, pc, pp, sm, sq, fo0);
            sp[pc][jo][wx] = vo;
        }
        const bool own_e = even_ok && (E < ke || (E == ke && !L.pz && ke == etop));
        if (own_e) {
            const size_t o = (size_t)pw(E) * NxNy;
            if (oute) out[o + ne] = ve;
            if (outo) out[o + no] = vo;
        }
        __syncthreads();
        if (E > ks) {
            // C: colour 2 of plane E-1 (ring 1)
            T ve2 = T(0), vo2 = T(0);
            if (st2) {
                ve2 = update(wx, je, pmm, pm, pc, smm, sm, fe1);
                sp[pm][je][wx] = ve2;
            }
            __syncthreads();
            // D: colour 3 of plane E-1 (tile); plane E-1 written
            if (st3) vo2 = update(wx, jo, pmm, pm, pc, smm, sm, fo1);
            const size_t o = (size_t)pw(E - 1) * NxNy;
            if (oute) out[o + ne] = ve2;
            if (outo) out[o + no] = vo2;
        }
        if (!more) break;
        __syncthreads();                 // every read of planes E-2, E-1 and layers E-2, E-1 done
        st_phi(E + 2, q0, q1);
        st_phi(E + 3, q2, q3);
        st_sig(E + 1, s0, s1);
        st_sig(E + 2, s2, s3);
        fe0 = nfe;
        fo0 = nfo;
        fe1 = nfe1;
        fo1 = nfo1;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Residual on tiles staged in LDS: a workgroup owns RTX x RTY x RTZ nodes,
// loads phi on the tile plus one node around it and sigma on the cells
// touching the tile once (instead of each node gathering its 20 neighbours
// and 8 cells from the caches), then evaluates r = f - L phi per node with
// (L phi)_n = 1/(12 h^2) sum_c sigma_c (far corners - 4 phi_n), cells in the
// order sz, sy, sx and far corners x+y, x+z, y+z, x+y+z.  Nodes beyond a wall read 0 and cells beyond it
// sigma = 0 (their terms add exact zeros).  kStore: r written to L.r; kNorm:
// the workgroup's partial row {sum r^2, 0, max |r|, #non-finite} at row
// blockIdx.x.
// ---------------------------------------------------------------------------
constexpr int kRTX = 32, kRTY = 8, kRTZ = 8;
constexpr int kRWX = kRTX + 2, kRWY = kRTY + 2, kRWZ = kRTZ + 2;      // node window
constexpr int kRCX = kRTX + 1, kRCY = kRTY + 1, kRCZ = kRTZ + 1;      // cell window

template <typename T>
inline int nod_resid_tiles(const NodLevelT<T>& L) {
    return ((L.Nx + kRTX - 1) / kRTX) * ((L.Ny + kRTY - 1) / kRTY) * ((L.Nz + kRTZ - 1) / kRTZ);
}

// The refinement step of a mixed-precision solve in the same pass (kRefine):
// the window's phi is phi + corr / s (corr the FP32 V-cycle's correction,
// s = scales[0] the scale its residual carried, a power of two), written out
// of place for the tile's own nodes (neighbouring tiles read the old phi of
// their halos), and the residual of the updated phi is written in FP32 times
// scales[1] (the scale of the previous residual: lagged by one step, as the
// reduction advances the scales afterwards).
struct NodRefine {
    const float* corr;
    const double* scales;
    double* phi_out;
    float* r32;
};

template <typename T, bool kStore, bool kNorm, bool kRefine = false>
__global__ __launch_bounds__(kRTX * kRTY) void k_nod_resid_tile(NodLevelT<T> L, double* __restrict__ partials,
                                                                NodRefine ra = NodRefine{}) {
    __shared__ __align__(16) T sphi[kRWZ][kRWY][kRWX];
    __shared__ T ssig[kRCZ][kRCY][kRCX];
    const int ntx = (L.Nx + kRTX - 1) / kRTX, nty = (L.Ny + kRTY - 1) / kRTY;
    const int b = blockIdx.x;
    const int I0 = (b % ntx) * kRTX, J0 = ((b / ntx) % nty) * kRTY, K0 = (b / (ntx * nty)) * kRTZ;
    const int tid = threadIdx.x;
    const size_t NxNy = (size_t)L.Nx * L.Ny, nxny = (size_t)L.nx * L.ny;
    // A window index g one beyond either end of [0, n): the periodic image
    // (one wrap; a ragged tile's positions beyond n + 1 are clamped, their
    // values are never read) or, beyond a wall, absent.
    auto at = [](int g, int n, int per, bool& ok) {
        if (per) {
            if (g < 0) g += n;
            else if (g >= n) g -= n;
            return min(g, n - 1);
        }
        ok = ok && g >= 0 && g < n;
        return min(max(g, 0), n - 1);
    };
    // node window (nodes I0-1 .. I0+RTX, etc.) and cell window (cells I0-1
    // .. I0+RTX-1: those around the tile's nodes), x fastest across the
    // threads: every load of the thread is issued before any is stored, so
    // they are all in flight together
    constexpr int kNT = kRTX * kRTY;
    constexpr int kPN = (kRWX * kRWY * kRWZ + kNT - 1) / kNT, kPC = (kRCX * kRCY * kRCZ + kNT - 1) / kNT;
    T vp[kPN], vs[kPC];
    const double inv_s = kRefine ? 1.0 / ra.scales[0] : 0.0;     // exact: a power of two
    const double r_s = kRefine ? ra.scales[1] : 0.0;
#pragma unroll
    for (int q = 0; q < kPN; ++q) {
        const int e = min(tid + q * kNT, kRWX * kRWY * kRWZ - 1);
        const int x = e % kRWX, yz = e / kRWX, y = yz % kRWY, z = yz / kRWY;
        bool ok = true;
        const int I = at(I0 - 1 + x, L.Nx, L.px, ok), J = at(J0 - 1 + y, L.Ny, L.py, ok);
        const int K = at(K0 - 1 + z, L.Nz, L.pz, ok);
        const size_t n = (size_t)K * NxNy + (size_t)J * L.Nx + I;
        vp[q] = L.phi[n];
        if (kRefine) vp[q] = vp[q] + (double)ra.corr[n] * inv_s;   // the correction add's expression
        if (!ok) vp[q] = T(0);
    }
#pragma unroll
    for (int q = 0; q < kPC; ++q) {
        const int e = min(tid + q * kNT, kRCX * kRCY * kRCZ - 1);
        const int x = e % kRCX, yz = e / kRCX, y = yz % kRCY, z = yz / kRCY;
        bool ok = true;
        const int i = at(I0 - 1 + x, L.nx, L.px, ok), j = at(J0 - 1 + y, L.ny, L.py, ok);
        const int k = at(K0 - 1 + z, L.nz, L.pz, ok);
        vs[q] = L.sig[(size_t)k * nxny + (size_t)j * L.nx + i];
        if (!ok) vs[q] = T(0);
    }
#pragma unroll
    for (int q = 0; q < kPN; ++q) {
        const int e = tid + q * kNT;
        if (e < kRWX * kRWY * kRWZ) (&sphi[0][0][0])[e] = vp[q];
    }
#pragma unroll
    for (int q = 0; q < kPC; ++q) {
        const int e = tid + q * kNT;
        if (e < kRCX * kRCY * kRCZ) (&ssig[0][0][0])[e] = vs[q];
    }
    __syncthreads();
    const int tx = tid % kRTX, ty = tid / kRTX;
    const int I = I0 + tx, J = J0 + ty;
    const T ih = (T)(12.0 * L.h * L.h);
    double s2 = 0.0, mx = 0.0, nonfin = 0.0;
    if (I < L.Nx && J < L.Ny) {
        for (int tz = 0; tz < kRTZ; ++tz) {
            const int K = K0 + tz;
            if (K >= L.Nz) break;
            const int x = tx + 1, y = ty + 1, z = tz + 1;        // the node in the windows
            const T pn = sphi[z][y][x];
            T sum = T(0);
#pragma unroll
            for (int sz = 0; sz < 2; ++sz) {
                const int zo = sz ? z + 1 : z - 1;
#pragma unroll
                for (int sy = 0; sy < 2; ++sy) {
                    const int yo = sy ? y + 1 : y - 1;
#pragma unroll
                    for (int sx = 0; sx < 2; ++sx) {
                        const int xo = sx ? x + 1 : x - 1;
                        // the cell on side (sx, sy, sz) of the node: cell window index node - 1 + s
                        const T sig = ssig[z - 1 + sz][y - 1 + sy][x - 1 + sx];
                        T acc = T(0);
                        acc += sphi[z][yo][xo];
                        acc += sphi[zo][y][xo];
                        acc += sphi[zo][yo][x];
                        acc += sphi[zo][yo][xo];
                        sum += sig * (acc - T(4) * pn);
                    }
                }
            }
            const size_t n = (size_t)K * NxNy + (size_t)J * L.Nx + I;
            const T r = L.f[n] - pdiv(sum, ih);
            if (kStore) L.r[n] = r;
            if (kRefine) {
                ra.phi_out[n] = pn;
                ra.r32[n] = (float)(r * r_s);
            }
            if (kNorm) {
                const double rd = (double)r;
                if (!isfinite(rd)) nonfin += 1.0;
                s2 += rd * rd;
                mx = fmax(mx, fabs(rd));
            }
        }
    }
    if (kNorm) {
        // fixed-order tree over the workgroup, in the (now free) phi window
        static_assert(sizeof(sphi) >= 3 * kRTX * kRTY * sizeof(double), "reduction buffer");
        double* red = reinterpret_cast<double*>(&sphi[0][0][0]);
        constexpr int nt = kRTX * kRTY;
        __syncthreads();
        red[tid] = s2;
        red[nt + tid] = mx;
        red[2 * nt + tid] = nonfin;
        __syncthreads();
        for (int w = nt / 2; w > 0; w >>= 1) {
            if (tid < w) {
                red[tid] = red[tid] + red[tid + w];
                red[nt + tid] = fmax(red[nt + tid], red[nt + tid + w]);
                red[2 * nt + tid] = red[2 * nt + tid] + red[2 * nt + tid + w];
            }
            __syncthreads();
        }
        if (tid == 0) {
            double* row = partials + (size_t)b * kReduceWidth;
            row[0] = red[0];
            row[1] = 0.0;
            row[2] = red[nt];
            row[3] = red[2 * nt];
        }
    }
}

// coarse f = 1/8 sum_d w(d) r_{2C+d} (existing fine nodes), coarse phi = 0.
template <typename T>
__global__ void k_nod_restrict(NodLevelT<T> F, NodLevelT<T> C) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= C.Nx || J >= C.Ny || K >= C.Nz) return;
    const int X[3] = {2 * I, 2 * J, 2 * K};
    const int Nn[3] = {F.Nx, F.Ny, F.Nz}, per[3] = {F.px, F.py, F.pz};
    T s = T(0);
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int D[3] = {dx, dy, dz};
                int m[3];
                bool ok = true;
                T w = T(1);
                for (int d = 0; d < 3; ++d) {
                    m[d] = nod_node(X[d], D[d], Nn[d], per[d]);
                    if (m[d] < 0) ok = false;
                    if (D[d] != 0) w *= T(0.5);
                }
                if (ok) s += w * F.r[nidx(F, m[0], m[1], m[2])];
            }
    const size_t c = nidx(C, I, J, K);
    C.f[c] = T(0.125) * s;
    C.phi[c] = T(0);
}

// fine phi += trilinear interpolation of the coarse phi.  One thread per
// coarse node (I, J, K) updates the up to 8 fine nodes (2I + dx, 2J + dy,
// 2K + dz), dx, dy, dz in {0, 1}, from the 8 coarse values around it,
// loaded once; per fine node the parents are summed in the order (z, y, x)
// with the weight 1 or 1/2 per direction.
template <typename T>
__global__ void k_nod_prolong(NodLevelT<T> F, NodLevelT<T> C) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x;
    const int J = blockIdx.y * blockDim.y + threadIdx.y;
    const int K = blockIdx.z * blockDim.z + threadIdx.z;
    if (I >= C.Nx || J >= C.Ny || K >= C.Nz) return;
    // coarse node + 1 in each direction (the periodic image; beyond a wall
    // the node itself, whose value is never used: no fine node lies there)
    const int I1 = I + 1 < C.Nx ? I + 1 : (C.px ? 0 : I);
    const int J1 = J + 1 < C.Ny ? J + 1 : (C.py ? 0 : J);
    const int K1 = K + 1 < C.Nz ? K + 1 : (C.pz ? 0 : K);
    T c[2][2][2];
    c[0][0][0] = C.phi[nidx(C, I, J, K)];
    c[0][0][1] = C.phi[nidx(C, I1, J, K)];
    c[0][1][0] = C.phi[nidx(C, I, J1, K)];
    c[0][1][1] = C.phi[nidx(C, I1, J1, K)];
    c[1][0][0] = C.phi[nidx(C, I, J, K1)];
    c[1][0][1] = C.phi[nidx(C, I1, J, K1)];
    c[1][1][0] = C.phi[nidx(C, I, J1, K1)];
    c[1][1][1] = C.phi[nidx(C, I1, J1, K1)];
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int X = 2 * I + dx, Y = 2 * J + dy, Z = 2 * K + dz;
                if (X >= F.Nx || Y >= F.Ny || Z >= F.Nz) continue;
                const int D[3] = {dx, dy, dz};
                T v = T(0);
#pragma unroll
                for (int bz = 0; bz < 2; ++bz)
#pragma unroll
                    for (int by = 0; by < 2; ++by)
#pragma unroll
                        for (int bx = 0; bx < 2; ++bx) {
                            const int B[3] = {bx, by, bz};
                            bool ok = true;
                            T w = T(1);
#pragma unroll
                            for (int d = 0; d < 3; ++d) {
                                if (D[d] == 0) {
                                    if (B[d]) ok = false;    // an even fine index has one parent
                                } else {
                                    w *= T(0.5);
                                }
                            }
                            if (ok) v += w * c[bz][by][bx];
                        }
                const size_t n = nidx(F, X, Y, Z);
                F.phi[n] = F.phi[n] + v;
            }
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

// ---------------------------------------------------------------------------
// Bottom of the nodal V-cycle in one workgroup: from the first level whose
// phi, f and r (with every coarser level's) fit in LDS down to the coarsest
// solve and back, with barriers between dependent steps instead of one
// launch of a few microseconds per colour, residual, restriction and
// prolongation.  Per node the arithmetic is that of the per-level kernels
// (the same stencil routine for the colours, the same sums in the same
// order for the residual, restriction, prolongation and coarsest solve), so
// a bottom launch gives the same bits as the launches it replaces.  sigma
// stays in global memory.
// ---------------------------------------------------------------------------
constexpr int kNodBottomThreads = 1024;
constexpr size_t kNodBottomLds = 136 * 1024;     // phi, f, r of every bottom level
constexpr int kNodBottomMax = 8;

template <typename T>
struct NodBottomArgs {
    int nlev;
    NodLevelT<T> lev[kNodBottomMax];    // sig global; phi, f of lev[0] global (in and out)
    int off[kNodBottomMax];             // element offsets of each level's phi, f, r in LDS
    const double* minv;
    int pre, post;
};

// (L phi) at node (I, J, K) as the residual kernel forms it: cells sz, sy,
// sx, each sigma times (far corners - 4 phi_n), nodes beyond a wall 0 and
// cells beyond it skipped (their sigma is 0 there).
template <typename T>
__device__ inline T nb_apply(const NodLevelT<T>& L, const T* P, int I, int J, int K) {
    const NodAxis ax = nod_axis(I, L.Nx, L.nx, L.px);
    const NodAxis ay = nod_axis(J, L.Ny, L.ny, L.py);
    const NodAxis az = nod_axis(K, L.Nz, L.nz, L.pz);
    NodNbr<T> N;
    nod_load_nbrs(L, P, I, ax, ay, az, J, K, N);
    const T pn = P[((size_t)K * L.Ny + J) * L.Nx + I];
    const long long nx = L.nx, nxny = (long long)L.nx * L.ny;
    T sum = T(0);
#pragma unroll
    for (int sz = 0; sz < 2; ++sz) {
        const int oz = sz ? 2 : 0;
#pragma unroll
        for (int sy = 0; sy < 2; ++sy) {
            const int oy = sy ? 2 : 0;
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
                const int ox = sx ? 2 : 0;
                T sig = T(0);
                if (az.e[sz] && ay.e[sy] && ax.e[sx]) sig = L.sig[az.c[sz] * nxny + ay.c[sy] * nx + ax.c[sx]];
                T acc = T(0);
                acc += N.v[1][oy][ox];
                acc += N.v[oz][1][ox];
                acc += N.v[oz][oy][1];
                acc += N.v[oz][oy][ox];
                sum += sig * (acc - T(4) * pn);
            }
        }
    }
    return sum;
}

template <typename T>
__device__ void nb_colour(const NodLevelT<T>& L, T* P, const T* F, int col) {
    const int hy = (L.Ny + 1 - (col & 1)) >> 1, hz = (L.Nz + 1 - (col >> 1)) >> 1;
    const int items = L.Nx * hy * hz;
    const T c12 = (T)(12.0 * (L.h * L.h));
    for (int e = threadIdx.x; e < items; e += blockDim.x) {
        int I, r, jh, kh;
        small_divmod(e, L.Nx, r, I);
        small_divmod(r, hy, kh, jh);
        const int J = 2 * jh + (col & 1), K = 2 * kh + (col >> 1);
        T num, den;
        nod_stencil_fast(L, P, I, J, K, num, den);
        const size_t n = ((size_t)K * L.Ny + J) * L.Nx + I;
        P[n] = pdiv(num - c12 * F[n], den);
    }
    __syncthreads();
}

template <typename T>
__device__ void nb_resid(const NodLevelT<T>& L, const T* P, const T* F, T* R) {
    const int items = L.Nx * L.Ny * L.Nz;
    const T ih = (T)(12.0 * L.h * L.h);
    for (int e = threadIdx.x; e < items; e += blockDim.x) {
        int I, J, K, r;
        small_divmod(e, L.Nx, r, I);
        small_divmod(r, L.Ny, K, J);
        R[e] = F[e] - pdiv(nb_apply(L, P, I, J, K), ih);
    }
    __syncthreads();
}

template <typename T>
__device__ void nb_restrict(const NodLevelT<T>& Fl, const T* R, const NodLevelT<T>& Cl, T* cP, T* cF) {
    const int items = Cl.Nx * Cl.Ny * Cl.Nz;
    const int Nn[3] = {Fl.Nx, Fl.Ny, Fl.Nz}, per[3] = {Fl.px, Fl.py, Fl.pz};
    for (int e = threadIdx.x; e < items; e += blockDim.x) {
        int I, J, K, r;
        small_divmod(e, Cl.Nx, r, I);
        small_divmod(r, Cl.Ny, K, J);
        const int X[3] = {2 * I, 2 * J, 2 * K};
        T s = T(0);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int D[3] = {dx, dy, dz};
                    int m[3];
                    bool ok = true;
                    T w = T(1);
                    for (int d = 0; d < 3; ++d) {
                        m[d] = nod_node(X[d], D[d], Nn[d], per[d]);
                        if (m[d] < 0) ok = false;
                        if (D[d] != 0) w *= T(0.5);
                    }
                    if (ok) s += w * R[((size_t)m[2] * Fl.Ny + m[1]) * Fl.Nx + m[0]];
                }
        cF[e] = T(0.125) * s;
        cP[e] = T(0);
    }
    __syncthreads();
}

template <typename T>
__device__ void nb_prolong(const NodLevelT<T>& Fl, T* P, const NodLevelT<T>& Cl, const T* cP) {
    const int items = Fl.Nx * Fl.Ny * Fl.Nz;
    const int Nc[3] = {Cl.Nx, Cl.Ny, Cl.Nz}, per[3] = {Cl.px, Cl.py, Cl.pz};
    for (int e = threadIdx.x; e < items; e += blockDim.x) {
        int X[3], r;
        small_divmod(e, Fl.Nx, r, X[0]);
        small_divmod(r, Fl.Ny, X[2], X[1]);
        T v = T(0);
        for (int bz = 0; bz < 2; ++bz)
            for (int by = 0; by < 2; ++by)
                for (int bx = 0; bx < 2; ++bx) {
                    const int B[3] = {bx, by, bz};
                    int m[3];
                    bool ok = true;
                    T w = T(1);
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
                            w *= T(0.5);
                        }
                    }
                    if (ok) v += w * cP[((size_t)m[2] * Cl.Ny + m[1]) * Cl.Nx + m[0]];
                }
        P[e] = P[e] + v;
    }
    __syncthreads();
}

// Coarsest level as the coarse-solve kernel does it: remove mean(f), x =
// Minv (-f'), remove mean(x), serial sums and row dot products in its order.
template <typename T>
__device__ void nb_coarse(int n, const double* __restrict__ minv, const T* F, T* P, double* rhs, double* x,
                          double* mean) {
    for (int c = threadIdx.x; c < n; c += blockDim.x) rhs[c] = (double)F[c];
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += rhs[c];
        *mean = s / n;
    }
    __syncthreads();
    const double m = *mean;
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) rhs[c] = -(rhs[c] - m);
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        const double* row = minv + (size_t)r * n;
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += row[c] * rhs[c];
        x[r] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += x[c];
        *mean = s / n;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) P[c] = (T)(x[c] - *mean);
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kNodBottomThreads) void k_nod_bottom(NodBottomArgs<T> A) {
    __shared__ double lds_raw[kNodBottomLds / sizeof(double)];
    __shared__ double rhs[kCoarseMax], x[kCoarseMax];
    __shared__ double mean;
    T* lds = reinterpret_cast<T*>(lds_raw);
    const int nb = A.nlev;
    auto nodes = [&](int b) { return (int)A.lev[b].nodes(); };
    auto Pof = [&](int b) { return lds + A.off[b]; };
    auto Fof = [&](int b) { return lds + A.off[b] + nodes(b); };
    auto Rof = [&](int b) { return lds + A.off[b] + 2 * nodes(b); };
    {   // first bottom level: f from the restriction above, phi = 0
        const int n0 = nodes(0);
        for (int e = threadIdx.x; e < n0; e += blockDim.x) {
            Fof(0)[e] = A.lev[0].f[e];
            Pof(0)[e] = T(0);
        }
        __syncthreads();
    }
    for (int b = 0; b + 1 < nb; ++b) {
        for (int s = 0; s < A.pre; ++s)
            for (int col = 0; col < 4; ++col) nb_colour(A.lev[b], Pof(b), Fof(b), col);
        nb_resid(A.lev[b], Pof(b), Fof(b), Rof(b));
        nb_restrict(A.lev[b], Rof(b), A.lev[b + 1], Pof(b + 1), Fof(b + 1));
    }
    nb_coarse(nodes(nb - 1), A.minv, Fof(nb - 1), Pof(nb - 1), rhs, x, &mean);
    for (int b = nb - 2; b >= 0; --b) {
        nb_prolong(A.lev[b], Pof(b), A.lev[b + 1], Pof(b + 1));
        for (int s = 0; s < A.post; ++s)
            for (int col = 0; col < 4; ++col) nb_colour(A.lev[b], Pof(b), Fof(b), col);
    }
    const int n0 = nodes(0);
    for (int e = threadIdx.x; e < n0; e += blockDim.x) A.lev[0].phi[e] = Pof(0)[e];
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
    // mixed precision: FP32 mirrors of every level (sigma, phi, f, r, phi2),
    // the inner V-cycle's arrays
    bool mixed = false;
    NodLevelT<float> lev32[kMaxLevels];
    void* ws = nullptr;
    double* minv = nullptr;
    double* partials = nullptr;
    double* scal = nullptr;
    double* host = nullptr;
    bool coeffs_valid = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // One V-cycle plus the finest residual norm (copied to host) as a
    // replayable hipGraph on the hierarchy's own stream, keyed by the sweep
    // counts and every level's phi buffers at the start of the cycle (the
    // fused sweeps swap them; with an even number of sweeps a cycle they
    // come back, so one capture serves every cycle of every solve).
    bool graphs_on = true;
    bool bottom_on = true;      // the coarse levels that fit in LDS run in one workgroup (k_nod_bottom)
    hipStream_t gstream = nullptr;
    hipEvent_t gev = nullptr;
    hipGraphExec_t cycle_exec = nullptr;
    int cycle_pre = -1, cycle_post = -1;
    std::vector<void*> cycle_bufs;
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

// Partial-sum rows of the finest level's residual norm.
size_t nod_partial_rows(const NodLevel& L0) { return std::max<size_t>(2048, (size_t)nod_resid_tiles(L0)); }

// Level shapes of a hierarchy of nl levels for p (into lev), and the device
// bytes it needs: per level sigma on cells and phi, f, r, phi2 on nodes (in
// mixed precision also FP32 copies of all five); the coarsest level's dense
// inverse, the partial rows and the scalar block.
size_t nod_layout(const mg_params* p, int nl, NodLevel* lev) {
    size_t bytes = 0;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    for (int l = 0; l < nl; ++l) {
        NodLevel& L = lev[l];
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
        bytes += al(L.cells() * 8) + 4 * al(L.nodes() * 8);
        if (p->precision == MG_MIXED) bytes += al(L.cells() * 4) + 4 * al(L.nodes() * 4);
    }
    const size_t nc = lev[nl - 1].nodes();
    bytes += al(nc * nc * 8) + al(nod_partial_rows(lev[0]) * kReduceWidth * 8) + al(64 * 8);
    return bytes;
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

// The fused sweep takes levels whose colouring is consistent across periodic
// wraps (even node counts there), an even number of node planes to march
// (the top plane of a walled z is even) and at least one 32 x 8 tile.
template <typename T>
bool nod_sweep_fits(const NodLevelT<T>& L) {
    if (L.Nx < 32 || L.Ny < 16) return false;
    if (L.py && L.Ny % 2 != 0) return false;
    if (L.pz ? (L.Nz % 2 != 0) : (L.nz % 2 != 0)) return false;
    return (L.pz ? L.Nz : L.Nz - 1) >= 2;
}

template <typename T, int TX, int TY>
hipError_t launch_nod_sweep_t(const NodLevelT<T>& L, T* out, int tz, hipStream_t st) {
    const int etop = L.pz ? L.Nz : L.Nz - 1;
    const int ntx = (L.Nx + TX - 1) / TX, nty = (L.Ny + TY - 1) / TY, nch = (etop + tz - 1) / tz;
    hipLaunchKernelGGL((k_nod_sweep<T, TX, TY>), dim3(ntx * nty * nch), dim3((TX + 8) * (TY + 8) / 2), 0, st, L,
                       out, tz, ntx, nty, etop);
    return hipGetLastError();
}

// Fused-sweep tiles (TX x TY nodes, tz planes per chunk).
struct NodSweepCfg {
    int tx, ty, tz;
};
constexpr int kNumNodSweepCfg = 8;
constexpr NodSweepCfg kNodSweepCfgs[kNumNodSweepCfg] = {{64, 8, 32}, {32, 8, 32}, {32, 16, 32}, {64, 16, 32},
                                                       {64, 8, 64}, {32, 8, 16}, {32, 16, 64}, {64, 8, 16}};
std::atomic<int> g_nod_cfg{-1};                  // forced configuration (-1: the default below)

template <typename T>
hipError_t launch_nod_sweep(const NodLevelT<T>& L, T* out, int cfg, hipStream_t st) {
    const NodSweepCfg& c = kNodSweepCfgs[cfg];
    if (c.tx == 64 && c.ty == 8) return launch_nod_sweep_t<T, 64, 8>(L, out, c.tz, st);
    if (c.tx == 32 && c.ty == 8) return launch_nod_sweep_t<T, 32, 8>(L, out, c.tz, st);
    if (c.tx == 32 && c.ty == 16) return launch_nod_sweep_t<T, 32, 16>(L, out, c.tz, st);
    return launch_nod_sweep_t<T, 64, 16>(L, out, c.tz, st);
}

// The levels a V-cycle in T runs on: the FP64 hierarchy, or its FP32 mirrors.
template <typename T>
NodLevelT<T>* nod_levels(nodal_hierarchy* H);
template <>
NodLevelT<double>* nod_levels<double>(nodal_hierarchy* H) { return H->lev; }
template <>
NodLevelT<float>* nod_levels<float>(nodal_hierarchy* H) { return H->lev32; }

// Sweeps on level l: the fused out-of-place sweep where it fits (the level's
// two phi buffers swap), else one in-place launch per colour.
template <typename T = double>
int nod_smooth(nodal_hierarchy* H, int l, int nsweeps, hipStream_t st) {
    NodLevelT<T>& L = nod_levels<T>(H)[l];
    // default: the fused sweep on levels of 4M nodes or more, 32 x 16 tiles
    // of 32-plane chunks (measured on MI355X: 215 us per 256^3 sweep against
    // 346 us for four colour launches; on a 128^3 level the colour launches
    // are faster); a forced configuration applies wherever it fits
    int cfg = g_nod_cfg.load();
    if (cfg >= 0 && (L.Nx < kNodSweepCfgs[cfg].tx || L.Ny < kNodSweepCfgs[cfg].ty)) cfg = -1;
    const bool fused = nod_sweep_fits(L) && (cfg >= 0 || L.nodes() >= ((size_t)4 << 20));
    if (fused) {
        if (cfg < 0) cfg = 2;
        for (int s = 0; s < nsweeps; ++s) {
            NHIP(launch_nod_sweep(L, L.phi2, cfg, st));
            std::swap(L.phi, L.phi2);
        }
        return MG_OK;
    }
    const dim3 block(64, 2, 2);
    const dim3 grid = grid3(L.Nx, (L.Ny + 1) / 2, (L.Nz + 1) / 2, block);
    for (int s = 0; s < nsweeps; ++s)
        for (int col = 0; col < 4; ++col) hipLaunchKernelGGL(k_nod_gs<T>, grid, block, 0, st, L, col);
    NHIP(hipGetLastError());
    return MG_OK;
}

template <typename T = double>
int nod_resid_restrict(nodal_hierarchy* H, int l, hipStream_t st) {
    const NodLevelT<T>& F = nod_levels<T>(H)[l];
    const NodLevelT<T>& C = nod_levels<T>(H)[l + 1];
    hipLaunchKernelGGL((k_nod_resid_tile<T, true, false>), dim3(nod_resid_tiles(F)), dim3(kRTX * kRTY), 0, st, F,
                       (double*)nullptr);
    const dim3 block(32, 4, 2);
    hipLaunchKernelGGL(k_nod_restrict<T>, grid3(C.Nx, C.Ny, C.Nz, block), block, 0, st, F, C);
    NHIP(hipGetLastError());
    return MG_OK;
}

template <typename T = double>
int nod_prolong(nodal_hierarchy* H, int l, hipStream_t st) {
    const NodLevelT<T>& F = nod_levels<T>(H)[l];
    const NodLevelT<T>& C = nod_levels<T>(H)[l + 1];
    const dim3 block(32, 4, 2);
    hipLaunchKernelGGL(k_nod_prolong<T>, grid3(C.Nx, C.Ny, C.Nz, block), block, 0, st, F, C);
    NHIP(hipGetLastError());
    return MG_OK;
}

hipError_t nod_coarse_solve(int n, const double* minv, const double* f, double* phi, hipStream_t st) {
    return launch_coarse_solve(n, minv, f, phi, st, 1);
}
hipError_t nod_coarse_solve(int n, const double* minv, const float* f, float* phi, hipStream_t st) {
    return launch_coarse_solve_f32(n, minv, f, phi, st, 1);
}

// First level (>= 1) from which every level's phi, f and r fit in the
// bottom kernel's LDS, or -1 (no level above the coarsest qualifies).
template <typename T>
int nod_bottom_start(const nodal_hierarchy* H) {
    const NodLevelT<T>* lev = nod_levels<T>(const_cast<nodal_hierarchy*>(H));
    size_t bytes = 0;
    int start = -1;
    for (int l = H->nlev - 1; l >= 1; --l) {
        bytes += 3 * lev[l].nodes() * sizeof(T);
        if (bytes > kNodBottomLds || H->nlev - l > kNodBottomMax) break;
        start = l;
    }
    return start < H->nlev - 1 ? start : -1;
}

// V-cycle from level l in T (the coarsest solve applies the FP64 inverse).
template <typename T = double>
int nod_vcycle(nodal_hierarchy* H, int l, hipStream_t st) {
    if (H->bottom_on && l > 0 && l == nod_bottom_start<T>(H)) {
        NodBottomArgs<T> a{};
        a.nlev = H->nlev - l;
        size_t off = 0;
        for (int b = 0; b < a.nlev; ++b) {
            a.lev[b] = nod_levels<T>(H)[l + b];
            a.off[b] = (int)off;
            off += 3 * a.lev[b].nodes();
        }
        a.minv = H->minv;
        a.pre = H->p.pre_sweeps;
        a.post = H->p.post_sweeps;
        hipLaunchKernelGGL(k_nod_bottom<T>, dim3(1), dim3(kNodBottomThreads), 0, st, a);
        NHIP(hipGetLastError());
        return MG_OK;
    }
    if (l == H->nlev - 1) {
        const NodLevelT<T>& L = nod_levels<T>(H)[l];
        NHIP(nod_coarse_solve((int)L.nodes(), H->minv, L.f, L.phi, st));
        return MG_OK;
    }
    int rc = nod_smooth<T>(H, l, H->p.pre_sweeps, st);
    if (rc) return rc;
    rc = nod_resid_restrict<T>(H, l, st);
    if (rc) return rc;
    rc = nod_vcycle<T>(H, l + 1, st);
    if (rc) return rc;
    rc = nod_prolong<T>(H, l, st);
    if (rc) return rc;
    return nod_smooth<T>(H, l, H->p.post_sweeps, st);
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

// Mixed-precision solve (iterative refinement with the multigrid of Sec. 3
// as its inner solver): each iteration runs one FP32 V-cycle from zero on the
// FP64 residual scaled by the power of two nearest 1/rms(r), adds the FP32
// correction divided by that power of two (exact) to the FP64 phi, and
// recomputes r = f - L phi and its norm in FP64; the stop test is the FP64
// solve's.  Returns MG_OK or a launch error; *status is the solve's.
int nod_solve_mixed(nodal_hierarchy* H, double fnorm, mg_stats* S_, int* status_out, int* cycles_out,
                    double* rel_out, hipStream_t st) {
    NodLevel& L0 = H->lev[0];
    NodLevelT<float>& M0 = H->lev32[0];
    const size_t NN = L0.nodes();
    for (int l = 0; l < H->nlev; ++l)
        NHIP(launch_coeff_to_f32(H->lev[l].sig, H->lev32[l].sig, H->lev[l].cells(), st));
    const double s0 = residual_scale(fnorm, NN);
    NHIP(launch_scale_to_f32(L0.f, M0.f, NN, s0, st));       // the residual of phi = 0 is f
    double* scales = H->scal + kSlotScale * kReduceWidth;      // {scale of the FP32 residual, scale for the next}
    H->host[kSlotScale * kReduceWidth] = s0;
    H->host[kSlotScale * kReduceWidth + 1] = s0;
    NHIP(hipMemcpyAsync(scales, H->host + kSlotScale * kReduceWidth, 2 * sizeof(double), hipMemcpyHostToDevice, st));
    const int nt = nod_resid_tiles(L0);
    int status = MG_ERR_NOT_CONVERGED, cycles = 0;
    double rel = 1.0;
    // nodal default one: its FP32 V-cycle costs several refinement passes
    // (256^3: two per step took 8.90 ms against 8.19 with one)
    const int inner = H->p.inner_cycles > 0 ? H->p.inner_cycles : 1;
    while (cycles < H->p.max_cycles) {
        NHIP(launch_fill<float>(M0.phi, NN, 0.0f, st));
        for (int c = 0; c < inner; ++c) {                 // the FP32 correction: V-cycles from zero
            int rc = nod_vcycle<float>(H, 0, st);
            if (rc) return rc;
        }
        // phi += corr / s, r = f - L phi with its norm rows, FP32 r for the
        // next cycle, in one pass (phi out of place); the reduction then
        // advances the scales
        const NodRefine ra{M0.phi, scales, L0.phi2, M0.f};
        hipLaunchKernelGGL((k_nod_resid_tile<double, false, true, true>), dim3(nt), dim3(kRTX * kRTY), 0, st, L0,
                           H->partials, ra);
        NHIP(hipGetLastError());
        std::swap(L0.phi, L0.phi2);
        NHIP(launch_reduce_scale(H->partials, nt, H->scal + kSlotRes * kReduceWidth, scales, NN, st));
        NHIP(hipMemcpyAsync(H->host + kSlotRes * kReduceWidth, H->scal + kSlotRes * kReduceWidth,
                            kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, st));
        NHIP(hipStreamSynchronize(st));
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
        if (cycles >= H->p.max_cycles) break;
    }
    *status_out = status;
    *cycles_out = cycles;
    *rel_out = rel;
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
    if (fnorm > 0.0 && H->p.rtol < 1.0 && H->mixed) {
        rc = nod_solve_mixed(H, fnorm, S_, &status, &cycles, &rel, st);
        if (rc) return S_->status = rc;
    } else if (fnorm > 0.0 && H->p.rtol < 1.0) {
        status = MG_ERR_NOT_CONVERGED;
        bool on_graph = false;
        auto cycle = [&](hipStream_t s) -> int {
            int r2 = nod_vcycle(H, 0, s);
            if (r2) return r2;
            hipLaunchKernelGGL((k_nod_resid_tile<double, false, true>), dim3(nod_resid_tiles(L0)),
                               dim3(kRTX * kRTY), 0, s, L0, H->partials);
            NHIP(hipGetLastError());
            NHIP(launch_reduce(H->partials, nod_resid_tiles(L0), H->scal + kSlotRes * kReduceWidth, s));
            NHIP(hipMemcpyAsync(H->host + kSlotRes * kReduceWidth, H->scal + kSlotRes * kReduceWidth,
                                kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, s));
            return MG_OK;
        };
        // a captured cycle bakes in the levels' phi buffers: replayable when
        // every level's buffers come back (an even number of sweeps a cycle)
        const bool graphs = H->graphs_on && (H->p.pre_sweeps + H->p.post_sweeps) % 2 == 0;
        while (cycles < H->p.max_cycles) {
            if (graphs) {
                if (!H->gstream) {
                    NHIP(hipStreamCreateWithFlags(&H->gstream, hipStreamNonBlocking));
                    NHIP(hipEventCreateWithFlags(&H->gev, hipEventDisableTiming));
                }
                if (!on_graph) {                    // after the caller's earlier work
                    NHIP(hipEventRecord(H->gev, st));
                    NHIP(hipStreamWaitEvent(H->gstream, H->gev, 0));
                    on_graph = true;
                }
                std::vector<void*> bufs;
                for (int l = 0; l < H->nlev; ++l) {
                    bufs.push_back(H->lev[l].phi);
                    bufs.push_back(H->lev[l].phi2);
                }
                bufs.push_back((void*)(intptr_t)g_nod_cfg.load());      // the tiles the capture baked in
                if (!H->cycle_exec || H->cycle_pre != H->p.pre_sweeps || H->cycle_post != H->p.post_sweeps ||
                    H->cycle_bufs != bufs) {
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
                    H->cycle_bufs = bufs;
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

namespace mg {

size_t nodal_bytes(const mg_params* p) {
    if (!p || validate_params(p) != MG_OK) return 0;
    for (int d = 0; d < 3; ++d)
        if (p->bc[d] != MG_BC_PERIODIC && p->bc[d] != MG_BC_WALL) return 0;
    const int nl = nod_count_levels(p);
    if (nl == 0) return 0;
    NodLevel lev[kMaxLevels];
    return nod_layout(p, nl, lev);
}

void nodal_rebind(nodal_handle h, const mg_params* p) { h->p = *p; }

}  // namespace mg

extern "C" {

int nodal_tune_sweep(int32_t cfg) {
    if (cfg < -1 || cfg >= kNumNodSweepCfg) {
        set_error("nodal sweep configuration out of range");
        return MG_ERR_INVALID_ARG;
    }
    g_nod_cfg.store(cfg);
    return MG_OK;
}

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
    if (p->precision != MG_FP64 && p->precision != MG_MIXED) {
        set_error("unknown precision");
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
    const size_t bytes = nod_layout(p, nl, H->lev);
    if (hipMalloc(&H->ws, bytes) != hipSuccess) {
        (void)hipGetLastError();
        delete H;
        set_error("hipMalloc of the nodal hierarchy failed");
        return MG_ERR_OOM;
    }
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t nc = H->lev[nl - 1].nodes();
    const size_t prow = nod_partial_rows(H->lev[0]);
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
        L.phi2 = take(L.nodes() * 8);
    }
    H->mixed = p->precision == MG_MIXED;
    if (H->mixed) {
        auto take32 = [&](size_t n) { return reinterpret_cast<float*>(take(n * 4)); };
        for (int l = 0; l < nl; ++l) {
            const NodLevel& L = H->lev[l];
            NodLevelT<float>& M = H->lev32[l];
            M.nx = L.nx; M.ny = L.ny; M.nz = L.nz;
            M.Nx = L.Nx; M.Ny = L.Ny; M.Nz = L.Nz;
            M.px = L.px; M.py = L.py; M.pz = L.pz;
            M.h = L.h;
            M.sig = take32(L.cells());
            M.phi = take32(L.nodes());
            M.f = take32(L.nodes());
            M.r = take32(L.nodes());
            M.phi2 = take32(L.nodes());
        }
    }
    H->minv = take(nc * nc * 8);
    H->partials = take(prow * kReduceWidth * 8);
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

int nodal_set_bottom(nodal_handle h, int32_t enable) {
    if (!h) {
        set_error("null handle");
        return MG_ERR_INVALID_ARG;
    }
    h->bottom_on = enable != 0;
    if (h->cycle_exec) {                 // a captured cycle baked in the other choice
        hipGraphExecDestroy(h->cycle_exec);
        h->cycle_exec = nullptr;
    }
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
