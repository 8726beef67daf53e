// Host-side hierarchy object and the internal entry points shared by the
// single-problem, batch and serving front ends.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "boxes.h"
#include "mg_internal.h"

// Slots (rows of 4 doubles) in the device scalar block of a hierarchy.
namespace mg {
constexpr int kSlotRhs = 0;    // {sum f, sum |f|, bad rho/beta0, #non-finite}
constexpr int kSlotNorm = 1;   // {||f||^2 after mean removal, ...}
constexpr int kSlotRes = 2;    // {||r||^2, -, max |r|, #non-finite}
constexpr int kSlotPhi = 3;    // {sum phi, ...}
constexpr int kSlotScale = 4;  // mixed precision: {scale of the FP32 residual, scale for the next}
}  // namespace mg

struct mg_hierarchy {
    mg_params p{};
    int device = 0;
    int nlev = 0;
    int px = 0, py = 0, pz = 0;
    int side[6] = {};              // per side: 0 periodic, 1 wall, 2 outflow (x low, x high, ..., z high)
    bool outflow = false;          // some side is an outflow side
    bool singular = true;          // no outflow side: phi defined up to a constant
    mg::Level lev[mg::kMaxLevels];
    void* ws = nullptr;
    size_t ws_bytes = 0;
    bool owns_ws = false;
    bool coeffs_valid = false;
    double* partials = nullptr;   // 2048 rows x 4
    double* scal = nullptr;       // 16 rows x 4 device scalars
    double* host = nullptr;       // pinned mirror of scal
    double* minv = nullptr;       // inverse of the coarsest-level matrix
    double* r64 = nullptr;        // FP64 residual (mixed precision)
    float* rho32 = nullptr;       // FP32 copy of rho (mixed precision, fused finest level)
    bool rho32_on = false;        // rho32 holds the current solve's rho
    bool rho32_fresh = false;     // rho32 written by this call's coefficient kernel
    double* rho_own = nullptr;    // copies made by mg_set_coefficients
    double* b0c_own = nullptr;
    double* b0e_own = nullptr;
    double* w0 = nullptr;         // per-layer dp0/dt term (mac_project_full)
    mg::RhoArgs rho{};            // finest-level coefficient source of the current solve
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t evs0 = nullptr, evs1 = nullptr;   // around the multigrid iterations of a solve
    // Replayable V-cycles (FP64 solve): one cycle plus the next residual
    // norm captured as a hipGraph, keyed by everything baked into it.
    bool graphs_on = true;
    bool bottom_on = true;      // levels below the fused ones in one workgroup launch
    hipStream_t gstream = nullptr;
    hipEvent_t gev = nullptr;
    struct CycleGraph {
        hipGraphExec_t exec = nullptr;
        std::vector<uintptr_t> key;                 // pointers and settings at capture
        std::vector<void*> post_phi, post_phi2;     // level phi buffers (FP64, then FP32) after it
    } graph[2];
    int graph_next = 0;                             // slot replaced by the next capture
    // Finest level split into boxes with halo exchange (mg_set_boxes).
    bool boxes_on = false;
    mg::BoxSet box{};
    void* box_mem = nullptr;
};

namespace mg {
// Radial base state of a solve: beta0 profile prof[m] at r = (m + 1/2) dr
// about c (prof == nullptr: plane-parallel beta0).
struct Radial {
    int nr = 0;
    double dr = 0.0;
    const double* prof = nullptr;
    double c[3] = {0.0, 0.0, 0.0};
};
// Per-side codes (x low, x high, ..., z high) of mg_params::bc.
void sides_from_bc(const mg_params* p, int side[6]);
void set_error(const std::string& s);
int hip_fail(hipError_t e, const char* what, int line);
int count_levels(int nx, int ny, int nz);
int validate_params(const mg_params* p);
size_t workspace_bytes(const mg_params* p);
int setup(const mg_params* p, void* workspace, size_t ws_bytes, mg_hierarchy** out);
int destroy(mg_hierarchy* H);
// In-place set-up on caller memory (no allocation, no events, no graphs).
int setup_static(const mg_params* p, void* ws, size_t ws_bytes, double* host, mg_hierarchy* H);
int project(mg_hierarchy* H, const double* rho, const double* b0c, const double* b0e, const double* S,
            double* u, double* v, double* w, double* phi_out, mg_stats* stats, hipStream_t st,
            const double* w0 = nullptr, const Radial* rad = nullptr);
double model_bytes(const mg_params& p, int cycles, int mixed);
// First level run by the one-workgroup bottom solver (phi and f of it and of
// every coarser level fit in its LDS), or -1.
template <typename T>
int bottom_start(const mg_hierarchy* H);
// Mixed precision: the power of two nearest 1/rms of a residual of 2-norm
// norm2_sqrt over n cells (1 for a zero or non-finite norm).
double residual_scale(double norm2_sqrt, size_t n);
template <typename T>
void bottom_args(mg_hierarchy* H, int l, BottomArgs<T>& a);
int build_coefficients(mg_hierarchy* H, const double* rho, const double* b0c, const double* b0e,
                       const double* S, const double* u, const double* v, const double* w, hipStream_t st,
                       const double* w0 = nullptr, const Radial* rad = nullptr);
// Multi-box finest level of box-cell boxes for params p (MG_ERR_INVALID_ARG
// for a box size mg_set_boxes refuses), and the device bytes of its arrays
// (0 for such a box size).
int box_layout(const mg_params& p, const int32_t box[3], BoxSet* out, size_t* e, size_t* eb);
size_t box_bytes(const mg_params& p, const int32_t box[3]);
// Nodal projection: device bytes of a hierarchy for p (0 if not solvable),
// and new solver controls (rtol, cycles, sweeps) for an existing one of the
// same shape.
size_t nodal_bytes(const mg_params* p);
void nodal_rebind(nodal_handle h, const mg_params* p);
}  // namespace mg
