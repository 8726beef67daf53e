// Device arithmetic shared by every kernel that forms face coefficients or
// Gauss-Seidel updates, so that a quantity computed by different kernels
// (stored coefficient arrays, coefficients recomputed inside a sweep, single
// or batched launches) is always the same bit pattern.
#pragma once

#include <hip/hip_runtime.h>

namespace mg {

// x / y for y > 0 finite: hardware reciprocal, one Newton step, one residual
// correction (Markstein's form).  Within one ulp of the IEEE quotient and far
// cheaper than the correctly rounded division sequence, which dominated the
// FP64 sweeps.
__device__ __forceinline__ double qdiv(double x, double y) {
    double r = __builtin_amdgcn_rcp(y);
    const double e = fma(-y, r, 1.0);
    r = fma(r, e, r);
    const double q = x * r;
    const double rem = fma(-y, q, x);
    return fma(r, rem, q);
}

__device__ __forceinline__ float qdiv(float x, float y) { return x / y; }

}  // namespace mg
