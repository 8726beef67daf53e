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

// FP32 (the inner cycle of the mixed-precision solve, whose error the FP64
// refinement removes): hardware reciprocal with one Newton step, then one
// multiply; a few ulp at most instead of the correctly rounded sequence.
__device__ __forceinline__ float qdiv(float x, float y) {
    float r = __builtin_amdgcn_rcpf(y);
    const float e = __builtin_fmaf(-y, r, 1.0f);
    r = __builtin_fmaf(r, e, r);
    return x * r;
}

// Divisions of the fused sweep: qdiv in FP64; in FP32 (the sweeps of the
// inner cycle of a mixed-precision solve, a preconditioner whose error the
// FP64 refinement removes) the hardware reciprocal times x, within 2 ulp,
// two instructions fewer per division in a kernel bound by instruction issue.
__device__ __forceinline__ double pdiv(double x, double y) { return qdiv(x, y); }
__device__ __forceinline__ float pdiv(float x, float y) { return x * __builtin_amdgcn_rcpf(y); }

}  // namespace mg
