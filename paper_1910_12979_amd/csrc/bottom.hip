// Bottom of the V-cycle in one workgroup (gfx950).
//
// Below the levels the fused sweep covers, a level has at most a few
// thousand cells and the per-colour kernels, residual+restriction, coarsest
// solve and prolongation are each a launch of a few microseconds that keeps
// a handful of CUs busy.  Here one 1024-thread workgroup runs the whole
// V-cycle from the first such level down to the coarsest and back, with phi
// and f of every bottom level in LDS (coefficients stay in global memory,
// read through the caches) and a barrier between dependent steps.
//
// Per cell the arithmetic is exactly that of the per-level kernels (same
// expressions, same face order, same summation order in the restriction and
// the coarsest solve), so a bottom launch gives the same bits as the
// launches it replaces.  The batched form runs one workgroup per problem.
#include <hip/hip_runtime.h>

#include "devmath.h"
#include "mg_internal.h"

namespace mg {
namespace {

constexpr int kBottomThreads = 1024;

__device__ inline int bidx(int i, int j, int k, int nx, int ny) { return (k * ny + j) * nx + i; }

// One colour of red-black Gauss-Seidel on a bottom level (phi, f in LDS).
template <typename T>
__device__ void b_colour(const BottomLevel<T>& lv, T* P, const T* F, int colour) {
    const int nx = lv.nx, ny = lv.ny, nz = lv.nz;
    const int hx = (nx + 1) >> 1;
    const int items = hx * ny * nz;
    const T h2 = lv.h2;
    for (int e = threadIdx.x; e < items; e += blockDim.x) {
        int ih, r, j, k;
        small_divmod(e, hx, r, ih);
        small_divmod(r, ny, k, j);
        const int i = 2 * ih + ((j + k + colour) & 1);
        if (i >= nx) continue;
        const int im = i > 0 ? i - 1 : nx - 1, ip = i < nx - 1 ? i + 1 : 0;
        const int jm = j > 0 ? j - 1 : ny - 1, jp = j < ny - 1 ? j + 1 : 0;
        const int km = k > 0 ? k - 1 : nz - 1, kp = k < nz - 1 ? k + 1 : 0;
        const int c = bidx(i, j, k, nx, ny);
        const T bxl = lv.bx[c], bxh = lv.bx[bidx(ip, j, k, nx, ny)];
        const T byl = lv.by[c], byh = lv.by[bidx(i, jp, k, nx, ny)];
        const T bzl = lv.bz[c], bzh = lv.bz[bidx(i, j, kp, nx, ny)];
        T num = bxl * P[bidx(im, j, k, nx, ny)];
        num = num + bxh * P[bidx(ip, j, k, nx, ny)];
        num = num + byl * P[bidx(i, jm, k, nx, ny)];
        num = num + byh * P[bidx(i, jp, k, nx, ny)];
        num = num + bzl * P[bidx(i, j, km, nx, ny)];
        num = num + bzh * P[bidx(i, j, kp, nx, ny)];
        T den = bxl + bxh;
        den = den + byl;
        den = den + byh;
        den = den + bzl;
        den = den + bzh;
        if (lv.has_bnd) den = den + bnd_diag(lv.bnd, i, j, k, nx, ny, nz);
        P[c] = qdiv(num - h2 * F[c], den);
    }
    __syncthreads();
}

// (L phi)_c on a bottom level: faces in the fixed order, then times 1/h^2.
template <typename T>
__device__ inline T b_apply(const BottomLevel<T>& lv, const T* P, int i, int j, int k) {
    const int nx = lv.nx, ny = lv.ny, nz = lv.nz;
    const int im = i > 0 ? i - 1 : nx - 1, ip = i < nx - 1 ? i + 1 : 0;
    const int jm = j > 0 ? j - 1 : ny - 1, jp = j < ny - 1 ? j + 1 : 0;
    const int km = k > 0 ? k - 1 : nz - 1, kp = k < nz - 1 ? k + 1 : 0;
    const int c = bidx(i, j, k, nx, ny);
    const int cxp = bidx(ip, j, k, nx, ny), cyp = bidx(i, jp, k, nx, ny), czp = bidx(i, j, kp, nx, ny);
    const T pc = P[c];
    T s = lv.bx[c] * (P[bidx(im, j, k, nx, ny)] - pc);
    s = s + lv.bx[cxp] * (P[cxp] - pc);
    s = s + lv.by[c] * (P[bidx(i, jm, k, nx, ny)] - pc);
    s = s + lv.by[cyp] * (P[cyp] - pc);
    s = s + lv.bz[c] * (P[bidx(i, j, km, nx, ny)] - pc);
    s = s + lv.bz[czp] * (P[czp] - pc);
    if (lv.has_bnd) s = s - bnd_diag(lv.bnd, i, j, k, nx, ny, nz) * pc;
    return s * (T(1) / lv.h2);
}

// f_c = (1/8) sum over the 8 children of (f - L phi), children x fastest,
// then y, then z; phi_c = 0.
template <typename T>
__device__ void b_resid_restrict(const BottomLevel<T>& lv, const T* P, const T* F, T* cP, T* cF) {
    const int cx = lv.nx >> 1, cy = lv.ny >> 1, cz = lv.nz >> 1;
    const int items = cx * cy * cz;
    for (int e = threadIdx.x; e < items; e += blockDim.x) {
        int I, J, K, r;
        small_divmod(e, cx, r, I);
        small_divmod(r, cy, K, J);
        T s = T(0);
        for (int dk = 0; dk < 2; ++dk)
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di) {
                    const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                    const T r = F[bidx(i, j, k, lv.nx, lv.ny)] - b_apply(lv, P, i, j, k);
                    s = s + r;
                }
        cF[e] = T(0.125) * s;
        cP[e] = T(0);
    }
    __syncthreads();
}

// phi += P phi_coarse (piecewise constant).
template <typename T>
__device__ void b_prolong(const BottomLevel<T>& lv, T* P, const T* cP) {
    const int nx = lv.nx, ny = lv.ny, nz = lv.nz;
    const int items = nx * ny * nz;
    for (int e = threadIdx.x; e < items; e += blockDim.x) {
        int i, j, k, r;
        small_divmod(e, nx, r, i);
        small_divmod(r, ny, k, j);
        P[e] = P[e] + cP[bidx(i >> 1, j >> 1, k >> 1, nx >> 1, ny >> 1)];
    }
    __syncthreads();
}

// Coarsest level: remove mean(f), x = Minv (-f'), remove mean(x) (without
// the mean removals when an outflow side makes the operator non-singular).
// Serial sums and row dot products in the same order as the coarse-solve
// kernel.
template <typename T>
__device__ void b_coarse(int n, int singular, const double* __restrict__ minv, const T* F, T* P, double* rhs,
                         double* x, double* mean) {
    for (int c = threadIdx.x; c < n; c += blockDim.x) rhs[c] = (double)F[c];
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        if (singular)
            for (int c = 0; c < n; ++c) s += rhs[c];
        *mean = singular ? s / n : 0.0;
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
        if (singular)
            for (int c = 0; c < n; ++c) s += x[c];
        *mean = singular ? s / n : 0.0;
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) P[c] = (T)(x[c] - *mean);
    __syncthreads();
}

template <typename T>
__device__ void bottom_body(const BottomArgs<T>& A) {
    __shared__ double lds_raw[kBottomLdsBytes / sizeof(double)];
    __shared__ double rhs[kCoarseMax], x[kCoarseMax];
    __shared__ double mean;
    T* lds = reinterpret_cast<T*>(lds_raw);
    const int nb = A.nlev;
    auto Pof = [&](int b) { return lds + A.lev[b].off; };
    auto Fof = [&](int b) { return lds + A.lev[b].off + A.lev[b].nx * A.lev[b].ny * A.lev[b].nz; };

    {   // first bottom level: f from the level above's restriction, phi = 0
        const int n0 = A.lev[0].nx * A.lev[0].ny * A.lev[0].nz;
        T* P = Pof(0);
        T* F = Fof(0);
        for (int e = threadIdx.x; e < n0; e += blockDim.x) {
            F[e] = A.f[e];
            P[e] = T(0);
        }
        __syncthreads();
    }
    for (int b = 0; b + 1 < nb; ++b) {
        for (int s = 0; s < A.pre; ++s) {
            b_colour(A.lev[b], Pof(b), Fof(b), 0);
            b_colour(A.lev[b], Pof(b), Fof(b), 1);
        }
        b_resid_restrict(A.lev[b], Pof(b), Fof(b), Pof(b + 1), Fof(b + 1));
    }
    {
        const BottomLevel<T>& c = A.lev[nb - 1];
        b_coarse(c.nx * c.ny * c.nz, A.singular, A.minv, Fof(nb - 1), Pof(nb - 1), rhs, x, &mean);
    }
    for (int b = nb - 2; b >= 0; --b) {
        b_prolong(A.lev[b], Pof(b), Pof(b + 1));
        for (int s = 0; s < A.post; ++s) {
            b_colour(A.lev[b], Pof(b), Fof(b), 0);
            b_colour(A.lev[b], Pof(b), Fof(b), 1);
        }
    }
    const int n0 = A.lev[0].nx * A.lev[0].ny * A.lev[0].nz;
    const T* P = Pof(0);
    for (int e = threadIdx.x; e < n0; e += blockDim.x) A.phi[e] = P[e];
}

template <typename T>
__global__ __launch_bounds__(kBottomThreads) void k_bottom(BottomArgs<T> a) {
    bottom_body<T>(a);
}

template <typename T>
__global__ __launch_bounds__(kBottomThreads) void k_bottom_multi(const BottomArgs<T>* __restrict__ descs) {
    bottom_body<T>(descs[blockIdx.x]);
}

}  // namespace

template <typename T>
hipError_t launch_bottom(const BottomArgs<T>& a, hipStream_t st) {
    hipLaunchKernelGGL(k_bottom<T>, dim3(1), dim3(kBottomThreads), 0, st, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_bottom_multi(const BottomArgs<T>* d, int nprob, hipStream_t st) {
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bottom_multi<T>, dim3(nprob), dim3(kBottomThreads), 0, st, d);
    return hipGetLastError();
}

template hipError_t launch_bottom<double>(const BottomArgs<double>&, hipStream_t);
template hipError_t launch_bottom<float>(const BottomArgs<float>&, hipStream_t);
template hipError_t launch_bottom_multi<double>(const BottomArgs<double>*, int, hipStream_t);
template hipError_t launch_bottom_multi<float>(const BottomArgs<float>*, int, hipStream_t);

}  // namespace mg
