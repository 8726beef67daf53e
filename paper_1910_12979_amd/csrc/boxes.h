// Multi-box finest level: layout and launchers (internal, not part of the
// C ABI).  The finest level of an n0 x n1 x n2 domain is tiled by
// nb0 x nb1 x nb2 boxes, nb_d = ceil(n_d / B_d), B_d even: box (ib, jb, kb)
// starts at cell (ib B0, jb B1, kb B2) and holds B_d cells along d, except
// the last box of a direction that B_d does not divide, which holds the
// remainder n_d - (nb_d - 1) B_d (even, at least 2); box
// b = (kb nb1 + jb) nb0 + ib, x fastest.  Every box array is ghosted and
// sized for a full box: G0 x G1 x G2 cells, G_d = B_d + 2 kBoxGhost, local
// cell (i, j, k) of the box at ((k + g) G1 + (j + g)) G0 + (i + g),
// g = kBoxGhost, boxes one after another (stride G0 G1 G2 elements); a
// smaller box uses the first E_d + 2g cells of each direction (E_d its cells):
//   phi, phi2  two buffers (the fused sweep is out of place)
//   f          the right-hand side, ghosts included (the neighbour's value)
//   cx, cy, cz face coefficients, cell-aligned low faces in the same layout
//   rho        rho of the ghosted box (plane-parallel beta0: the fused sweep
//              recomputes the coefficients from it, as on the single box)
// plus beta0 at the centres and low faces of each box's ghosted planes
// (b0c, b0e: G2 entries per box).  Ghost cells beyond a wall hold
// phi = f = 0, rho = 1 and coefficient 1 on their faces (finite updates),
// except the wall face itself, which is 0.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace mg {

constexpr int kBoxGhost = 2;

struct BoxSet {
    int n[3];         // domain cells
    int B[3];         // cells of a full box
    int nb[3];        // boxes per direction
    int per[3];       // periodic directions
    int G[3];         // ghosted box dims
    int nbox;
    int fused;        // smoother: fused sweeps (1) or one launch per colour (0)
    size_t stride;    // elements per box
    double* phi;      // current phi
    double* phi2;     // the other buffer
    double* f;
    double* cx;
    double* cy;
    double* cz;
    double* rho;
    double* b0c;
    double* b0e;
    int rho_on;       // this solve's coefficients come from rho (plane-parallel beta0)
    // mixed precision (null otherwise): FP32 arrays in the same layout, the
    // inner V-cycle's finest level: phi (two buffers), f (the scaled FP64
    // residual), rho and the face coefficients
    float* phi32;
    float* phi2_32;
    float* f32;
    float* rho32;
    float* cx32;
    float* cy32;
    float* cz32;
};

size_t boxset_cells(const BoxSet& B);
// Cells along d of the box at box coordinate c.
__host__ __device__ inline int box_ext(const BoxSet& B, int d, int c) {
    const int r = B.n[d] - c * B.B[d];
    return r < B.B[d] ? r : B.B[d];
}
// phi = 0 (phi2 is written by a sweep before it is read); f of every
// ghosted box from the global finest-level f, and with coeffs its face
// arrays from the cell-aligned bx, by, bz (periodic images; walls as above).
// With rho (global, and b0c, b0e) also the boxes' rho and beta0.
hipError_t launch_box_scatter(const BoxSet& B, const double* f, const double* bx, const double* by, const double* bz,
                              const double* rho, const double* b0c, const double* b0e, bool coeffs, hipStream_t st);
// Every ghost cell of phi (colour 0 / 1: only that colour's; -1: all) from
// the box that owns its cell (periodic images; 0 beyond walls).
hipError_t launch_box_exchange(const BoxSet& B, int colour, hipStream_t st);
// nsweeps red-black sweeps, each followed by a halo exchange (per-colour
// smoother: after each colour).  Fused sweeps swap B.phi and B.phi2.  With
// phic (the single coarser level's phi) the sweeps start from phi + P phic:
// folded into the first fused sweep's load, else a prolongation launch.
hipError_t launch_box_smooth(BoxSet& B, double h, int nsweeps, hipStream_t st, const double* phic = nullptr);
// Speculative first sweep of the next cycle (fused smoother, at most
// kMaxPartialRows tiles in all: box_norm_sweep_fits): phi2 = RBGS(phi)
// without swapping, and per tile the partial rows {sum r^2, 0, 0, 0} of the
// residual of phi over the box interiors; *nparts rows.
bool box_norm_sweep_fits(const BoxSet& B);
hipError_t launch_box_sweep_norm(const BoxSet& B, double h, double* partials, int* nparts, hipStream_t st);
// Restricted residual into the (single-box) next level: fc, phic = 0.
hipError_t launch_box_resid_restrict(const BoxSet& B, double h, double* fc, double* phic, hipStream_t st);
// phi += P phic, then a halo exchange.
hipError_t launch_box_prolong(const BoxSet& B, const double* phic, hipStream_t st);
// Partial rows {sum r^2, 0, max |r|, #non-finite} of the residual; *nparts rows (<= 2048).
hipError_t launch_box_resid_norm(const BoxSet& B, double h, double* partials, int* nparts, hipStream_t st);
// Global phi from the box interiors.
hipError_t launch_box_gather(const BoxSet& B, double* phi, hipStream_t st);

// ---- mixed precision (fused boxes only) --------------------------------
// f32 = s f over every ghosted cell, and the FP32 copy of this solve's
// coefficient source (rho, or the three face arrays).
hipError_t launch_box_to_f32(const BoxSet& B, double s, hipStream_t st);
// nsweeps FP32 sweeps of phi32, each followed by an exchange of phi32; the
// first starts from 0 (zero_first) or from phi32 + P phic (phic: level 1's
// FP32 phi); swaps phi32 and phi2_32.
hipError_t launch_box_smooth32(BoxSet& B, double h, int nsweeps, bool zero_first, const float* phic,
                               hipStream_t st);
// FP32 residual of phi32 restricted into level 1's FP32 fc, phic = 0.
hipError_t launch_box_resid_restrict32(const BoxSet& B, double h, float* fc, float* phic, hipStream_t st);
// FP64 refinement over the interiors: phi = phi + phi32 / scales[0], f32 =
// scales[1] (f - L phi), partial rows {sum r^2, 0, 0, 0} of that residual
// (*nparts rows); then exchanges of phi and f32.  Swaps phi and phi2.
hipError_t launch_box_refine(BoxSet& B, double h, const double* scales, double* partials, int* nparts,
                             hipStream_t st);

}  // namespace mg
