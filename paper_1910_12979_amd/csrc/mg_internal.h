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

// q = a / d, r = a % d for 0 <= a < 2^20 and 1 <= d < 2^11 with d the same
// across the workgroup (a level size), as the one-workgroup bottom solvers
// decode their item indices: those run issue-bound on one CU, and an integer
// division by a run-time value takes about twenty instructions.  A power of
// two is a shift and a mask; otherwise the FP32 quotient a * rcp(d) (a exact
// in FP32, relative error below 2^-22, so within 1/4 of a / d) truncated and
// corrected once by the exact integer remainder.
__device__ __forceinline__ void small_divmod(int a, int d, int& q, int& r) {
    if ((d & (d - 1)) == 0) {
        const int s = __ffs(d) - 1;
        q = a >> s;
        r = a & (d - 1);
        return;
    }
    int t = (int)((float)a * __builtin_amdgcn_rcpf((float)d));
    int m = a - t * d;
    if (m < 0) {
        t -= 1;
        m += d;
    } else if (m >= d) {
        t += 1;
        m -= d;
    }
    q = t;
    r = m;
}

// FP32 V-cycles per refinement step of a mixed-precision MAC solve (0 in
// the parameters: the default, two; the nodal solve's default is one).
inline int inner_cycles_of(const mg_params& p) { return p.inner_cycles > 0 ? p.inner_cycles : 2; }

// Outflow sides of a level (phi = 0 on their boundary faces): for each side
// (x low, x high, y low, y high, z low, z high) the coefficient of the
// boundary face of every cell on that side, or null for a periodic or wall
// side.  x sides are indexed [k][j], y sides [k][i], z sides [j][i].
template <typename T>
struct Bnd {
    const T* s[6];
};

// Extra diagonal of cell (i,j,k) from its outflow boundary faces.  The face
// lies half a cell from the centre and its ghost value is -phi_c, so each
// contributes b (-phi_c - phi_c): 2 b on the diagonal, nothing to the
// neighbour sum.  Sides summed in the fixed order above, then doubled.
template <typename T>
__device__ inline T bnd_diag(const Bnd<T>& B, int i, int j, int k, int nx, int ny, int nz) {
    T d = T(0);
    if (i == 0 && B.s[0]) d = d + B.s[0][(size_t)k * ny + j];
    if (i == nx - 1 && B.s[1]) d = d + B.s[1][(size_t)k * ny + j];
    if (j == 0 && B.s[2]) d = d + B.s[2][(size_t)k * nx + i];
    if (j == ny - 1 && B.s[3]) d = d + B.s[3][(size_t)k * nx + i];
    if (k == 0 && B.s[4]) d = d + B.s[4][(size_t)j * nx + i];
    if (k == nz - 1 && B.s[5]) d = d + B.s[5][(size_t)j * nx + i];
    return d + d;
}

// Cells on side q of an nx x ny x nz level (the size of its boundary array).
inline size_t bnd_count(int q, int nx, int ny, int nz) {
    return q < 2 ? (size_t)ny * nz : q < 4 ? (size_t)nx * nz : (size_t)nx * ny;
}

struct Level {
    int nx = 0, ny = 0, nz = 0;
    size_t N = 0;
    double h = 0.0;
    LevelArrays<double> d;   // FP64 arrays
    LevelArrays<float> s;    // FP32 mirrors (mixed precision only)
    double* phi2_d = nullptr;  // second phi buffer (out-of-place sweeps swap with d.phi)
    float* phi2_s = nullptr;
    double* phi_home_d[2] = {};  // the two phi buffers as laid out (d.phi, phi2_d at set-up)
    float* phi_home_s[2] = {};
    double* bnd_d[6] = {};   // outflow boundary-face coefficients (null: not an outflow side)
    float* bnd_s[6] = {};    // FP32 mirrors (mixed precision only)
    double* dg_d = nullptr;  // per-cell boundary diagonal (outflow sides), FP64
    float* dg_s = nullptr;   // and from the FP32 boundary faces (mixed precision)
    bool has_bnd = false;
    Bnd<double> bnd64() const { return Bnd<double>{{bnd_d[0], bnd_d[1], bnd_d[2], bnd_d[3], bnd_d[4], bnd_d[5]}}; }
    Bnd<float> bnd32() const { return Bnd<float>{{bnd_s[0], bnd_s[1], bnd_s[2], bnd_s[3], bnd_s[4], bnd_s[5]}}; }
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
    int has_bnd;        // outflow sides present
    Bnd<T> bnd;
};

template <typename T>
struct BottomArgs {
    int nlev;           // bottom levels; the last one is solved directly
    int pre, post;      // sweeps before / after the coarse correction
    int singular;       // no outflow side: coarsest solve with mean removals
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

// General boundaries and base states (outflow sides, radial beta0).  side[q]
// per side (x low, x high, y low, y high, z low, z high): 0 periodic, 1 wall,
// 2 outflow.  beta0: plane-parallel (b0c, b0e) or, with prof != null, the
// radial profile prof[m] at r = (m + 1/2) dr about (cx, cy, cz), linear in r
// between profile points and constant beyond the ends.
struct GenArgs {
    int nx, ny, nz;
    int side[6];
    double h;
    const double* rho;
    const double* b0c;
    const double* b0e;
    int nr;
    double dr;
    const double* prof;
    double cx, cy, cz;
    const double* S;         // null: coefficients only
    const double* u;
    const double* v;
    const double* w;
    const double* w0;        // per-layer dp0/dt term (plane-parallel), nullable
    double* bx;
    double* by;
    double* bz;
    double* bnd[6];          // outflow boundary-face coefficients (null for other sides)
    double* f;
    double* partials;
};
// Level-0 coefficients (low faces: interior and periodic faces beta0_face /
// (0.5 (rho_L + rho_R)), walls and outflow sides 0; outflow boundary faces
// beta0_face / rho_cell into bnd), the right-hand side f = D(beta0 U) -
// beta0_c (S - w0) with every face velocity weighted by its own face's beta0,
// and partial rows as launch_coeff_rhs.
hipError_t launch_coeff_rhs_gen(const GenArgs& a, int* nparts, hipStream_t st);
// beta0 of the radial profile at the cell centres (nx*ny*nz, C order).
hipError_t launch_map_radial(const GenArgs& a, double* out, hipStream_t st);
// Velocity correction with general sides: U -= (phi_c - phi_nb) / h / rho_face
// on interior, periodic and outflow faces (outflow: ghost -phi_c, rho_face =
// rho_cell), the potential phi - mean (mean = *phi_sum / N, or 0 with
// phi_sum = null); periodic duplicate faces refreshed; phi_out (nullable) =
// phi - mean.
hipError_t launch_correct_gen(const GenArgs& a, const double* phi, const double* phi_sum, double* u,
                              double* v, double* w, double* phi_out, hipStream_t st);
// Coarse boundary-face coefficients: mean of the 2x2 fine faces of each
// outflow side (same order as the interior faces).
template <typename T>
hipError_t launch_avg_bnd(const Shape& fine, const Bnd<T>& fb, T* const cb[6], hipStream_t st);
// out[c] = bnd_diag of every cell (the per-cell boundary diagonal).
template <typename T>
hipError_t launch_bnd_diag3(const Shape& s, const Bnd<T>& bnd, T* out, hipStream_t st);

// Level-0 coefficients and right-hand side, plus per-block partial sums
// {sum f, sum |f|, #non-finite inputs, #non-positive rho/beta0}.
hipError_t launch_coeff_rhs(const Shape& s, int px, int py, int pz, double h,
                            const double* rho, const double* b0c, const double* b0e,
                            const double* S, const double* u, const double* v, const double* w,
                            double* bx, double* by, double* bz, double* f,
                            double* partials, int* nparts, hipStream_t st, const double* w0 = nullptr,
                            float* rho32 = nullptr);
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
// The same, then the next residual scale from out[0] as launch_next_scale
// computes it (one launch instead of two).
hipError_t launch_reduce_scale(const double* partials, int nparts, double* out, double* scales, size_t n,
                               hipStream_t st);
// f -= shift; partial row = {sum f^2 (after), 0, 0, 0}.
hipError_t launch_shift_norm(const Shape& s, double* f, double shift, double* partials,
                             int* nparts, hipStream_t st);
// Coarse coefficients = mean of the 4 coincident fine faces; with m32
// (three FP32 arrays), also their FP32 mirrors.
template <typename T>
hipError_t launch_avg_coeff(const Shape& fine, const T* bx, const T* by, const T* bz,
                            T* cbx, T* cby, T* cbz, hipStream_t st, float* const* m32 = nullptr);
// One red-black GS sweep (red then black), in place.
template <typename T>
hipError_t launch_rbgs(const Shape& s, double h, T* phi, const T* f, const T* bx,
                       const T* by, const T* bz, int nsweeps, hipStream_t st, const Bnd<T>* bnd = nullptr);
// f_c = R (f - L phi); phi_c = 0.
template <typename T>
hipError_t launch_resid_restrict(const Shape& fine, double h, const T* phi, const T* f,
                                 const T* bx, const T* by, const T* bz, T* fc, T* phic,
                                 hipStream_t st, const Bnd<T>* bnd = nullptr);
// phi += P phic.
template <typename T>
hipError_t launch_prolong(const Shape& fine, T* phi, const T* phic, hipStream_t st);
// Partial rows {sum r^2, max |r|, #non-finite, 0} of r = f - L phi.
template <typename T>
hipError_t launch_resid_norm(const Shape& s, double h, const T* phi, const T* f, const T* bx,
                             const T* by, const T* bz, double* partials, int* nparts,
                             hipStream_t st, const Bnd<T>* bnd = nullptr);
// Finest level, coefficients recomputed from rho: residual partial rows (r
// stored when r_out != nullptr) and fused residual + restriction.
hipError_t launch_resid_norm_rho(const Shape& s, double h, const RhoArgs& ra, const double* phi,
                                 const double* f, double* r_out, double* partials, int* nparts,
                                 hipStream_t st, const Bnd<double>* bnd = nullptr);
hipError_t launch_resid_restrict_rho(const Shape& fine, double h, const RhoArgs& ra, const double* phi,
                                     const double* f, double* fc, double* phic, hipStream_t st,
                                     const Bnd<double>* bnd = nullptr);
// Coarsest level: build M = -A + c 1 1^T (singular operator) or M = -A
// (outflow sides, bnd given) from the coefficients and invert it in place
// (one workgroup).  minv holds N*N doubles.
hipError_t launch_coarse_setup(const Shape& s, double h, const double* bx, const double* by,
                               const double* bz, double* minv, hipStream_t st,
                               const Bnd<double>* bnd = nullptr, int singular = 1);
// Coarsest level: phi = zero-mean solution of L phi = f (f's mean removed
// first); with singular = 0 plainly phi = M^-1 (-f).
hipError_t launch_coarse_solve(int N, const double* minv, const double* f, double* phi,
                               hipStream_t st, int singular = 1);
// Partial rows {sum phi, 0, 0, 0}.
hipError_t launch_sum(const Shape& s, const double* a, double* partials, int* nparts,
                      hipStream_t st);
// Velocity correction on non-wall faces with the zero-mean potential
// phi - (*phi_sum)/N; writes phi_out (nullable) = phi - mean.
hipError_t launch_correct(const Shape& s, int px, int py, int pz, double h, const double* b0c,
                          const double* b0e, const double* bx, const double* by,
                          const double* bz, const double* phi, const double* phi_sum,
                          double* u, double* v, double* w, double* phi_out, hipStream_t st);
// First coarse level's coefficients from level 0's recomputed from rho.
hipError_t launch_avg_coeff_rho(const Shape& fine, int px, int py, int pz, const double* rho, const double* b0c,
                                const double* b0e, double* cbx, double* cby, double* cbz, float* const* m32,
                                hipStream_t st);
// Fills and copies (graph-safe replacements for memset / memcpy).
template <typename T>
hipError_t launch_fill(T* a, size_t n, T value, hipStream_t st);
hipError_t launch_copy(double* dst, const double* src, size_t n, hipStream_t st);

// Mixed precision helpers.
// r = f - L phi (FP64), partial rows {sum r^2, max|r|, #nonfinite, 0}; r stored.
hipError_t launch_resid_store(const Shape& s, double h, const double* phi, const double* f,
                              const double* bx, const double* by, const double* bz, double* r,
                              double* partials, int* nparts, hipStream_t st, const Bnd<double>* bnd = nullptr);
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
                                   hipStream_t st, int singular = 1);

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
    double* copy;            // nullable: a second copy of the row (a gathered block)
};
// Level-0 coefficients (+ right-hand side) of one problem: the arguments of
// launch_coeff_rhs, its point-loop grid gx x gy x gz (coeff_grid) and, in a
// batched launch, its first block.
struct CoeffDesc {
    int nx, ny, nz, px, py, pz;
    double h;
    const double* rho;
    const double* b0c;
    const double* b0e;
    const double* S;         // null: coefficients only
    const double* u;
    const double* v;
    const double* w;
    const double* w0;        // nullable
    double* bx;
    double* by;
    double* bz;
    double* f;
    double* partials;
    int gx, gy, gz;
    int block0;
    float* rho32;            // nullable: FP32 copy of rho, written on the way
};
// A strided loop over N cells with one partial row per block (nb blocks, as
// the single-problem launch): a -= shift with rows {sum a^2} (shift-norm) or
// rows {sum a} (sum).
struct RowDesc {
    size_t N;
    double* a;
    double shift;
    double* partials;
    int nb;
    int block0;
};
// Coarse coefficients of one fine level (nx, ny, nz) into the next.
struct AvgDesc {
    int nx, ny, nz;
    const double* bx;
    const double* by;
    const double* bz;
    double* cbx;
    double* cby;
    double* cbz;
    int block0;
};
// Coarsest-level matrix build and inversion of one problem (no outflow sides).
struct CoarseDesc {
    int nx, ny, nz;
    double h;
    const double* bx;
    const double* by;
    const double* bz;
    double* minv;
    int singular;
};
// Elementwise operations over n values: kEltFill dst[e] = s (FP64),
// kEltToF32 dst[e] = (float)src[e], kEltScaleToF32 dst[e] = (float)(src[e] * s).
enum { kEltFill = 0, kEltToF32 = 1, kEltScaleToF32 = 2 };
struct EltDesc {
    int op;
    int block0;
    size_t n;
    const double* src;
    void* dst;
    double s;
};
// Velocity correction of one problem (the arguments of launch_correct).
struct CorrectDesc {
    int nx, ny, nz, px, py, pz;
    double h;
    const double* b0c;
    const double* b0e;
    const double* bx;
    const double* by;
    const double* bz;
    const double* phi;
    const double* phi_sum;
    double* u;
    double* v;
    double* w;
    double* phi_out;
    int block0;
};
hipError_t launch_rbgs_multi(const CellDesc* d, int nprob, int blocks, int colour, hipStream_t st);
hipError_t launch_resid_restrict_multi(const CellDesc* d, int nprob, int blocks, hipStream_t st);
hipError_t launch_prolong_multi(const CellDesc* d, int nprob, int blocks, hipStream_t st);
hipError_t launch_coarse_solve_multi(const CellDesc* d, int nprob, hipStream_t st);
hipError_t launch_reduce_multi(const ReduceDesc* d, int nprob, hipStream_t st);
// Batched set-up and finishing kernels: problem p owns blocks [d[p].block0,
// d[p+1].block0) of a launch of `blocks` workgroups (one per problem for the
// coarsest set-up), and every problem's values are the ones its
// single-problem launch gives (same per-block work and partial rows).
int coeff_grid(const Shape& s, int g[3]);          // point-loop grid; returns its blocks
int row_blocks(size_t n);                          // blocks of a shift-norm / sum over n cells
int elt_blocks(size_t n);                          // blocks of an elementwise op over n values
int cell_blocks(size_t n);                         // blocks of a one-thread-per-cell loop (256 threads)
hipError_t launch_coeff_rhs_multi(const CoeffDesc* d, int nprob, int blocks, hipStream_t st);
hipError_t launch_shift_norm_multi(const RowDesc* d, int nprob, int blocks, hipStream_t st);
hipError_t launch_sum_multi(const RowDesc* d, int nprob, int blocks, hipStream_t st);
hipError_t launch_avg_coeff_multi(const AvgDesc* d, int nprob, int blocks, hipStream_t st);
// lds: every problem's coarsest level has at most 128 cells (inverted in LDS)
hipError_t launch_coarse_setup_multi(const CoarseDesc* d, int nprob, bool lds, hipStream_t st);
bool coarse_setup_in_lds(size_t n);
hipError_t launch_elt_multi(const EltDesc* d, int nprob, int blocks, hipStream_t st);
hipError_t launch_correct_multi(const CorrectDesc* d, int nprob, int blocks, hipStream_t st);
// Mixed precision: the scale update of launch_next_scale for many problems.
struct ScaleDesc {
    const double* res;       // reduced residual row (sum r^2 first)
    double* scales;          // {scale of the FP32 residual, scale for the next}
    double n;                // cells
};
hipError_t launch_next_scale_multi(const ScaleDesc* d, int nprob, hipStream_t st);

}  // namespace mg
