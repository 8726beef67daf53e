// Multi-box finest level: layout and launchers (internal, not part of the
// C ABI).  The finest level of an n0 x n1 x n2 domain is tiled by
// nb0 x nb1 x nb2 boxes of B0 x B1 x B2 cells (every B_d even, dividing n_d);
// box b = (kb nb1 + jb) nb0 + ib, x fastest.  Per box, contiguous:
//   phi  (B0+2)(B1+2)(B2+2)  interior plus one ghost layer on each face
//   f    B0 B1 B2
//   cx   (B0+1) B1 B2        x-face coefficients, face f between cells f-1, f
//   cy   B0 (B1+1) B2
//   cz   B0 B1 (B2+1)
// Edge and corner ghosts are never read (the operator is the 7-point one).
// Offsets inside one box are 32-bit: (B0+2)(B1+2)(B2+2) < 2^31.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace mg {

struct BoxSet {
    int n[3];         // domain cells
    int B[3];         // box cells
    int nb[3];        // boxes per direction
    int per[3];       // periodic directions
    int nbox;
    int face_max;     // largest face (cells) of a box
    size_t phi_stride, f_stride, cx_stride, cy_stride, cz_stride;
    double* phi;
    double* f;
    double* cx;
    double* cy;
    double* cz;
};

size_t boxset_cells(const BoxSet& B);
// phi = 0 (ghosts included); f and the face arrays from the global
// finest-level f and cell-aligned bx, by, bz.
hipError_t launch_box_scatter(const BoxSet& B, const double* f, const double* bx, const double* by, const double* bz,
                              hipStream_t st);
// Every ghost face from the neighbouring boxes (periodic images; 0 beyond walls).
hipError_t launch_box_exchange(const BoxSet& B, hipStream_t st);
// nsweeps red-black sweeps, after each colour a halo exchange of that colour.
hipError_t launch_box_smooth(const BoxSet& B, double h, int nsweeps, hipStream_t st);
// Restricted residual into the (single-box) next level: fc, phic = 0.
hipError_t launch_box_resid_restrict(const BoxSet& B, double h, double* fc, double* phic, hipStream_t st);
// phi += P phic, then a halo exchange.
hipError_t launch_box_prolong(const BoxSet& B, const double* phic, hipStream_t st);
// Partial rows {sum r^2, 0, max |r|, #non-finite} of the residual; *nparts rows (<= 2048).
hipError_t launch_box_resid_norm(const BoxSet& B, double h, double* partials, int* nparts, hipStream_t st);
// Global phi from the box interiors.
hipError_t launch_box_gather(const BoxSet& B, double* phi, hipStream_t st);

}  // namespace mg
