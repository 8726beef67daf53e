// Dense coarsest-level inversion shared by the cell-centred and the nodal
// multigrid (one workgroup).
#pragma once

#include <hip/hip_runtime.h>

namespace mg {

// In-place Gauss-Jordan inversion of the SPD n x n row-major matrix M (no
// pivoting) by the calling workgroup; fac and prow are n-element scratch
// arrays in LDS.  Thread tid owns column jj = tid % n of rows tid / n,
// tid / n + nt / n, ... (n <= nt); per pivot p: row p becomes row p / M_pp
// (with 1 / M_pp in column p), every other row i subtracts M_ip times the new
// row p (column p: -M_ip / M_pp).  Ends with a barrier.
__device__ inline void gj_invert(double* M, int n, double* fac, double* prow) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int jj = tid % n;
    const int rstep = nt / n;
    const int r0 = tid / n;
    for (int p = 0; p < n; ++p) {
        __syncthreads();                     // previous step complete
        for (int e = tid; e < n; e += nt) {
            fac[e] = M[e * n + p];
            prow[e] = M[p * n + e];
        }
        __syncthreads();
        const double inv = 1.0 / fac[p];
        const double np = jj == p ? inv : prow[jj] * inv;     // new row p, column jj
        if (r0 < rstep) {
            for (int ii = r0; ii < n; ii += rstep) {
                if (ii == p) {
                    M[p * n + jj] = np;
                } else {
                    const double old = jj == p ? 0.0 : M[ii * n + jj];
                    M[ii * n + jj] = old - fac[ii] * np;
                }
            }
        }
    }
    __syncthreads();
}

}  // namespace mg
