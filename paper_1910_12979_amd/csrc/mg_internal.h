// Internal declarations shared by the HIP kernels and the host runtime of
// the MAC-projection library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/macproj.h"

namespace mg {

constexpr int kMaxLevels = 24;
constexpr int kCoarseMax = 512;     // cells on the coarsest (directly solved) level
constexpr int kCoarsenMin = 64;     // keep coarsening while a level has more cells than this
constexpr int kReduceWidth = 4;     // doubles per block in a partial-sum row

// One multigrid level.  Coefficient arrays are cell-aligned: b?[c] is the
// coefficient of the LOW face of cell c in that direction; face n of a
// direction is face 0 (walls hold 0 there, periodic faces wrap).
template <typename T>
struct LevelArrays {
    T* phi = nullptr;
    T* f = nullptr;
    T* bx = nullptr;
    T* by = nullptr;
    T* bz = nullptr;
};

struct Level {
    int nx = 0, ny = 0, nz = 0;
    size_t N = 0;
    double h = 0.0;
    LevelArrays<double> d;   // FP64 arrays
    LevelArrays<float> s;    // FP32 mirrors (mixed precision only)
    double* phi2_d = nullptr;  // second phi buffer (out-of-place sweeps swap with d.phi)
    float* phi2_s = nullptr;
};

struct Shape {
    int nx, ny, nz;
    size_t N() const { return (size_t)nx * ny * nz; }
};

// Finest-level coefficient source: rho, beta0 and the periodic flags.
struct RhoArgs {
    const double* rho;
    const double* b0c;
    const double* b0e;
    int px, py, pz;
};

// ---- bottom of the V-cycle in one workgroup (bottom.hip) -------------------
// Levels below the fused-sweep ones, from the first such level (phi = 0, f
// given) down to the coarsest and back, with phi and f of every bottom level
// in LDS.  Same per-cell arithmetic as the per-level kernels.
constexpr int kMaxBottomLevels = 8;
constexpr size_t kBottomLdsBytes = 136 * 1024;  // phi and f of every bottom level

template <typename T>
struct BottomLevel {
    int nx, ny, nz;
    int off;            // LDS offset (elements): phi at off, f at off + nx*ny*nz
    T h2;
    const T* bx;        // stored low-face coefficients (global)
    const T* by;
    const T* bz;
};

template <typename T>
struct BottomArgs {
    int nlev;           // bottom levels; the last one is solved directly
    int pre, post;      // sweeps before / after the coarse correction
    const double* minv; // inverse of the coarsest-level matrix
    const T* f;         // right-hand side of the first bottom level (global)
    T* phi;             // its phi (global), written
    BottomLevel<T> lev[kMaxBottomLevels];
};

template <typename T>
hipError_t launch_bottom(const BottomArgs<T>& a, hipStream_t st);
// One workgroup per problem; d is device memory.
template <typename T>
hipError_t launch_bottom_multi(const BottomArgs<T>* d, int nprob, hipStream_t st);

// ---- kernel launchers (kernels.hip) ---------------------------------------
// All launch on `stream` and return hipGetLastError().

// Level-0 coefficients and right-hand side, plus per-block partial sums
// {sum f, sum |f|, #non-finite inputs, #non-positive rho/beta0}.
hipError_t launch_coeff_rhs(const Shape& s, int px, int py, int pz, double h,
                            const double* rho, const double* b0c, const double* b0e,
                            const double* S, const double* u, const double* v, const double* w,
                            double* bx, double* by, double* bz, double* f,
                            double* partials, int* nparts, hipStream_t st, const double* w0 = nullptr);
// beta0 at layer centres and z faces from p0 (faces, centres) and the layer
// Gamma1 (one workgroup); w0[k] = dp0dt[k] / (Gamma1[k] p0[k]).
hipError_t launch_beta0_from_p0(int nz, double rho0, const double* p0e, const double* p0c, const double* g1c,
                                double* b0c, double* b0e, hipStream_t st);
hipError_t launch_dp0_term(int nz, const double* p0c, const double* g1c, const double* dp0dt, double* w0,
                           hipStream_t st);
// Coefficients only (no right-hand side).  Partials as above (sum f = 0).
hipError_t launch_coeff(const Shape& s, int px, int py, int pz, const double* rho,
                        const double* b0c, const double* b0e, double* bx, double* by,
                        double* bz, double* partials, int* nparts, hipStream_t st);
// Fixed-order reduction of nparts rows of kReduceWidth doubles into out[0..3].
hipError_t launch_reduce(const double* partials, int nparts, double* out, hipStream_t st);
// f -= shift; partial row = {sum f^2 (after), 0, 0, 0}.
hipError_t launch_shift_norm(const Shape& s, double* f, double shift, double* partials,
                             int* nparts, hipStream_t st);
// Coarse coefficients = mean of the 4 coincident fine faces.
template <typename T>
hipError_t launch_avg_coeff(const Shape& fine, const T* bx, const T* by, const T* bz,
                            T* cbx, T* cby, T* cbz, hipStream_t st);
// One red-black GS sweep (red then black), in place.
template <typename T>
hipError_t launch_rbgs(const Shape& s, double h, T* phi, const T* f, const T* bx,
                       const T* by, const T* bz, int nsweeps, hipStream_t st);
// f_c = R (f - L phi); phi_c = 0.
template <typename T>
hipError_t launch_resid_restrict(const Shape& fine, double h, const T* phi, const T* f,
                                 const T* bx, const T* by, const T* bz, T* fc, T* phic,
                                 hipStream_t st);
// phi += P phic.
template <typename T>
hipError_t launch_prolong(const Shape& fine, T* phi, const T* phic, hipStream_t st);
// Partial rows {sum r^2, max |r|, #non-finite, 0} of r = f - L phi.
template <typename T>
hipError_t launch_resid_norm(const Shape& s, double h, const T* phi, const T* f, const T* bx,
                             const T* by, const T* bz, double* partials, int* nparts,
                             hipStream_t st);
// Finest level, coefficients recomputed from rho: residual partial rows (r
// stored when r_out != nullptr) and fused residual + restriction.
hipError_t launch_resid_norm_rho(const Shape& s, double h, const RhoArgs& ra, const double* phi,
                                 const double* f, double* r_out, double* partials, int* nparts,
                                 hipStream_t st);
hipError_t launch_resid_restrict_rho(const Shape& fine, double h, const RhoArgs& ra, const double* phi,
                                     const double* f, double* fc, double* phic, hipStream_t st);
// Coarsest level: build M = -A + c 1 1^T from the coefficients and invert it
// in place (one workgroup).  minv holds N*N doubles.
hipError_t launch_coarse_setup(const Shape& s, double h, const double* bx, const double* by,
                               const double* bz, double* minv, hipStream_t st);
// Coarsest level: phi = zero-mean solution of L phi = f (f's mean removed first).
hipError_t launch_coarse_solve(int N, const double* minv, const double* f, double* phi,
                               hipStream_t st);
// Partial rows {sum phi, 0, 0, 0}.
hipError_t launch_sum(const Shape& s, const double* a, double* partials, int* nparts,
                      hipStream_t st);
// Velocity correction on non-wall faces with the zero-mean potential
// phi - (*phi_sum)/N; writes phi_out (nullable) = phi - mean.
hipError_t launch_correct(const Shape& s, int px, int py, int pz, double h, const double* b0c,
                          const double* b0e, const double* bx, const double* by,
                          const double* bz, const double* phi, const double* phi_sum,
                          double* u, double* v, double* w, double* phi_out, hipStream_t st);
// Fills and copies (graph-safe replacements for memset / memcpy).
template <typename T>
hipError_t launch_fill(T* a, size_t n, T value, hipStream_t st);
hipError_t launch_copy(double* dst, const double* src, size_t n, hipStream_t st);

// Mixed precision helpers.
// r = f - L phi (FP64), partial rows {sum r^2, max|r|, #nonfinite, 0}; r stored.
hipError_t launch_resid_store(const Shape& s, double h, const double* phi, const double* f,
                              const double* bx, const double* by, const double* bz, double* r,
                              double* partials, int* nparts, hipStream_t st);
// r32 = (float)(r / *rmax), rmax = max |r| (a device scalar).
hipError_t launch_to_f32(const double* r, float* r32, size_t n, const double* rmax,
                         hipStream_t st);
// phi += (double)e32 * (*rmax).
hipError_t launch_accumulate(double* phi, const float* e32, size_t n, const double* rmax,
                             hipStream_t st);
// FP32 copies of the coefficients.
hipError_t launch_coeff_to_f32(const double* a, float* b, size_t n, hipStream_t st);
// scales[0] <- scales[1]; scales[1] <- power of two nearest 1/rms (res[0] = sum r^2 over n)
hipError_t launch_next_scale(const double* res, double* scales, size_t n, hipStream_t st);
// b = (float)(s * a)
hipError_t launch_scale_to_f32(const double* a, float* b, size_t n, double s, hipStream_t st);
// Coarsest level in FP32 cycles: phi32 = (float) solve((double) f32).
hipError_t launch_coarse_solve_f32(int N, const double* minv, const float* f, float* phi,
                                   hipStream_t st);

int num_blocks_for_partials(const Shape& s);

// ---- batched forms (one launch, many problems) ------------------------------
// One problem at one level for the batched small-level kernels; block0 is the
// problem's first block in the launch (ascending over the table).
struct CellDesc {
    int nx, ny, nz;
    int block0;
    double h2;
    double* phi;
    const double* f;
    const double* bx;
    const double* by;
    const double* bz;
    double* fc;              // restriction: coarse f
    double* phic;            // restriction: coarse phi (zeroed) / prolongation source
    const double* minv;      // coarsest solve
};
struct ReduceDesc {
    const double* partials;
    int nparts;
    double* out;             // 4 doubles
};
hipError_t launch_rbgs_multi(const CellDesc* d, int nprob, int blocks, int colour, hipStream_t st);
hipError_t launch_resid_restrict_multi(const CellDesc* d, int nprob, int blocks, hipStream_t st);
hipError_t launch_prolong_multi(const CellDesc* d, int nprob, int blocks, hipStream_t st);
hipError_t launch_coarse_solve_multi(const CellDesc* d, int nprob, hipStream_t st);
hipError_t launch_reduce_multi(const ReduceDesc* d, int nprob, hipStream_t st);
// Mixed precision: the scale update of launch_next_scale for many problems.
struct ScaleDesc {
    const double* res;       // reduced residual row (sum r^2 first)
    double* scales;          // {scale of the FP32 residual, scale for the next}
    double n;                // cells
};
hipError_t launch_next_scale_multi(const ScaleDesc* d, int nprob, hipStream_t st);

}  // namespace mg
