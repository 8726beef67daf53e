/*
 * macproj.h -- C ABI of the MI355X (gfx950) variable-coefficient MAC projection.
 *
 * What the library computes (arXiv:1910.12979):
 *   The low Mach number velocity obeys the divergence constraint
 *   div(beta0 U) = beta0 S (Sec. 2, constraint equation; the caller folds the
 *   d p0/dt term into S).  A projection enforces it (Sec. 3: second-order
 *   projection method with multigrid solvers): solve
 *       div((beta0/rho) grad phi) = div(beta0 U) - beta0 S
 *   by geometric multigrid and correct the face velocities
 *       U <- U - (1/rho) grad phi
 *   which is the (beta0/rho) grad(.) pressure-gradient form of the momentum
 *   equation (Sec. 2) with the potential absorbing beta0.  beta0(r) is the
 *   1-D base state (Sec. 2, beta0 definition) taken along the height z.
 *
 * Discretisation: uniform cubic cells of spacing dx, cell-centred phi, rho, S;
 * face-normal velocities (MAC).  Face coefficient
 *     b = beta0_face / (0.5 (rho_left + rho_right)),
 * beta0_face = beta0_cc[k] on x and y faces of layer k, beta0_edge[k] on the
 * z face k.  (L phi)_c = dx^-2 sum_faces b (phi_nb - phi_c).  Solid-wall faces
 * carry no flux and their normal velocity is never modified.  In a periodic
 * direction face n duplicates face 0: it is ignored on input and overwritten
 * with face 0 on output.
 *
 * Outflow sides (MG_BC_OUTFLOW, MG_BC_WALL_OUTFLOW, MG_BC_OUTFLOW_WALL): phi =
 * 0 on the side's faces.  A boundary face's coefficient is beta0_face / rho of
 * its one cell and it enters the operator with the ghost value -phi_c
 * (b (-phi_c - phi_c)); its normal velocity takes part in div(beta0 U) as
 * given and is corrected like an interior face's, with rho_face = rho of the
 * cell.  With any outflow side the operator is non-singular: there is no
 * compatibility check, f and phi keep their means (stats mean_removed and
 * phi_mean are 0), and the coarsest level is solved with -A itself.  Problems
 * with outflow sides (and any solve with a plane-parallel or radial beta0 on
 * such a box) use the general-boundary kernels: interior faces U -= (1/rho_f)
 * grad phi with rho_f = 0.5 (rho_L + rho_R), and the divergence weights every
 * face velocity with its own face's beta0.
 *
 * Multigrid: V(pre, post) cycles of red-black Gauss-Seidel (red =
 * (i+j+k) even, first), 8-cell-average restriction, piecewise-constant
 * prolongation, coarse coefficients = mean of the 4 coincident fine faces,
 * coarsening while every dimension is even and the level has more than 64
 * cells; exact solve on the coarsest level (at most 512 cells).  Stop when
 * ||f - L phi||_2 / ||f||_2 <= rtol (f after mean removal).
 *
 * Layout: every field is float64, C order [k][j][i] (i fastest), contiguous:
 *   rho, S, phi      (nz, ny, nx)
 *   u                (nz, ny, nx+1)   face i between cells i-1 and i
 *   v                (nz, ny+1, nx)
 *   w                (nz+1, ny, nx)
 *   beta0_cc (nz), beta0_edge (nz+1)
 * All field pointers are DEVICE pointers on the current HIP device, owned by
 * the caller, which keeps them alive until the call (or ticket) completes.
 * Streams are hipStream_t passed as void* (NULL = the null stream).
 *
 * Errors: every int-returning call returns MG_OK (0), MG_PENDING (1) or a
 * negative mg_status.  No C++ exception crosses this boundary and the library
 * never exits or aborts.  mg_last_error() gives a thread-local detail string.
 */
#ifndef MACPROJ_H
#define MACPROJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MG_OK = 0,
    MG_PENDING = 1,
    MG_ERR_INVALID_ARG = -1,      /* null pointer, rho <= 0, beta0 <= 0, dx <= 0, bad bc */
    MG_ERR_BAD_SIZE = -2,         /* coarsest level would exceed 512 cells, or n < 1 */
    MG_ERR_INCOMPATIBLE_RHS = -3, /* |sum f| > 1e-8 sum |f|: no solution exists */
    MG_ERR_NOT_CONVERGED = -4,    /* max_cycles reached; outputs and stats still written */
    MG_ERR_NONFINITE = -5,        /* NaN/Inf in an input or in the residual */
    MG_ERR_OOM = -6,
    MG_ERR_HIP = -7,              /* a HIP runtime call failed, detail in mg_last_error() */
    MG_ERR_BUDGET = -8,           /* a request can never fit the server's memory budget */
    MG_ERR_BUSY = -9              /* no free slot right now (non-blocking submit) */
} mg_status;

/* Per direction: both sides periodic, both solid walls, both outflow, or a
 * wall on the low side and an outflow on the high side (and the reverse).
 * One code per direction, where a sketch with separate low/high side arrays
 * would take two: the periodic case pairs the sides anyway, and the two mixed
 * codes cover a wall facing an outflow. */
typedef enum {
    MG_BC_PERIODIC = 0,
    MG_BC_WALL = 1,
    MG_BC_OUTFLOW = 2,
    MG_BC_WALL_OUTFLOW = 3,
    MG_BC_OUTFLOW_WALL = 4
} mg_bc;
typedef enum { MG_FP64 = 0, MG_MIXED = 1 } mg_precision;

typedef struct {
    int32_t n[3];            /* nx, ny, nz (cells) */
    double  dx;              /* uniform cubic spacing */
    int32_t bc[3];           /* per direction: an mg_bc */
    int32_t pre_sweeps;      /* red-black GS sweeps before restriction (default 2) */
    int32_t post_sweeps;     /* sweeps after prolongation (default 2) */
    double  rtol;            /* relative L2 residual target (default 1e-10) */
    int32_t max_cycles;      /* V-cycles (or refinement steps) cap (default 100) */
    int32_t precision;       /* mg_precision */
    int32_t inner_cycles;    /* MG_MIXED: FP32 V-cycles per FP64 refinement step, 1..8 (the first
                                from zero); 0: the default, 2 (nodal solves: 1) */
} mg_params;

#define MG_HIST_MAX 128

typedef struct {
    int32_t status;          /* mg_status of the solve */
    int32_t cycles;          /* V-cycles (FP64) or refinement steps (mixed) */
    int32_t nlevels;
    int32_t hist_len;        /* entries used in resid_hist */
    double  rel_resid0;      /* relative residual of the starting phi = 0: 1 (0 when f = 0) */
    double  rel_resid;       /* final ||f - L phi||_2 / ||f||_2 */
    double  mean_removed;    /* mean of the right-hand side before removal */
    double  sum_f, sum_abs_f, norm_f;
    double  phi_mean;        /* mean removed from phi on exit */
    double  ms_total;        /* device time of the call (HIP events) */
    double  ms_smooth;       /* of which the multigrid iterations (sweeps, transfers, coarsest
                                solves, residual norms, refinement) */
    double  ms_other;        /* the rest: coefficients, right-hand side, checks, correction */
    double  bytes_model;     /* algorithmic HBM bytes of the call */
    double  resid_hist[MG_HIST_MAX]; /* relative residual after c cycles, [0] = 1 */
} mg_stats;

typedef struct mg_hierarchy* mg_handle;

typedef enum { MG_KIND_MAC = 0, MG_KIND_NODAL = 1 } mg_problem_kind;

/* One problem for project_batch / serve_submit.
 * kind MG_KIND_MAC: pointers as for mac_project; box = cells per box of a
 * multi-box finest level as for mg_set_boxes (FP64, periodic or wall sides),
 * {0, 0, 0} for a single box.
 * kind MG_KIND_NODAL: the nodal projection (nodal_project, FP64 or mixed):
 * u, v, w are the cell-centred velocity components, corrected in place, phi
 * (nullable) the node values; beta0_edge is not read (may be NULL); box must
 * be {0, 0, 0}.
 * A zero-filled tail (kind 0, box {0, 0, 0}) is the single-box MAC problem. */
typedef struct {
    mg_params p;
    const double* rho;
    const double* beta0_cc;
    const double* beta0_edge;
    const double* S;
    double* u;
    double* v;
    double* w;
    double* phi;             /* nullable */
    int32_t kind;            /* mg_problem_kind */
    int32_t box[3];
} mg_problem;

/* Fill *p with the defaults (V(2,2), rtol 1e-10, 100 cycles, FP64,
 * periodic x,y and walls in z) for an nx*ny*nz box of spacing dx. */
void mg_default_params(mg_params* p, int32_t nx, int32_t ny, int32_t nz, double dx);

/* Number of multigrid levels for params (0 if the shape is not solvable). */
int32_t mg_num_levels_for(const mg_params* p);

/* Device bytes the hierarchy needs for params (0 on invalid params). */
size_t mg_workspace_bytes(const mg_params* p);

/* Build a hierarchy for the shape in *p on the current device.
 * workspace: NULL -> the library allocates (and frees in mg_destroy);
 * otherwise a device buffer of at least mg_workspace_bytes(p) bytes, 256-byte
 * aligned, owned by the caller and kept alive until mg_destroy.
 * Set-up takes the shape only, not rho, beta0 or a stream: rho and beta0 change
 * every time step of the method, so they are arguments of each projection
 * (mac_project builds the coefficients from them inside the solve), and every
 * call that does device work takes its own stream. */
int mg_setup(const mg_params* p, void* workspace, size_t ws_bytes, mg_handle* out);

/* Release a hierarchy (NULL is allowed). */
int mg_destroy(mg_handle h);

/* Replace the solver controls (rtol, max_cycles, sweeps, precision) of h.
 * The shape, dx and bc must equal those given to mg_setup. */
int mg_set_params(mg_handle h, const mg_params* p);

/* Face coefficients b = beta0/rho_face on every level and the coarsest-level
 * factorisation, from rho (nz,ny,nx), beta0_cc (nz), beta0_edge (nz+1).
 * mac_project calls this itself; exposed for mg_vcycle users. */
int mg_set_coefficients(mg_handle h, const double* rho, const double* beta0_cc,
                        const double* beta0_edge, void* stream);

/* The whole projection: coefficients and right-hand side from (rho, beta0,
 * U, S), compatibility check and mean removal, V-cycles to rtol, mean removal
 * of phi, velocity correction.  u, v, w are updated in place; phi (nullable)
 * receives the zero-mean potential.  Blocks until the work on `stream` is
 * done.  stats may be NULL. */
int mac_project(mg_handle h, const double* rho, const double* beta0_cc,
                const double* beta0_edge, const double* S, double* u, double* v,
                double* w, double* phi, mg_stats* stats, void* stream);

/* One V(pre, post) cycle on level 0 with the current coefficients: phi
 * (nz,ny,nx, in/out) is improved for L phi = rhs (rhs must have zero mean).
 * *rel_resid_out (nullable) = ||rhs - L phi||_2 / ||rhs||_2 afterwards. */
int mg_vcycle(mg_handle h, double* phi, const double* rhs, double* rel_resid_out, void* stream);

/* ---- base state given as p0 and Gamma1 ---------------------------------- */

/* beta0 from the base-state pressure (Sec. 2, definition of beta0): with r
 * the height z, beta0(r) = rho0_base exp(integral from 0 to r of
 * (1/(Gamma1 p0)) dp0/dr').  Gamma1 is taken constant within each of the nz
 * layers, so the integral over any part [a, b] of layer k is exactly
 * ln(p0(b)/p0(a)) / Gamma1[k].  Device arrays: p0_edge (nz+1, at z = k dx;
 * face 0 is r = 0), p0_cc and gamma1_cc (nz, layer centres); outputs
 * beta0_cc (nz) and beta0_edge (nz+1), caller-owned.  Stream-ordered:
 * returns after enqueueing one small kernel.  Non-positive or non-finite p0
 * or Gamma1 give non-finite beta0, which mac_project then rejects
 * (MG_ERR_NONFINITE). */
int mg_beta0_from_p0(int32_t nz, double rho0_base, const double* p0_edge, const double* p0_cc,
                     const double* gamma1_cc, double* beta0_cc, double* beta0_edge, void* stream);

/* mac_project with the full right-hand side of the constraint (Sec. 2):
 * f = D(beta0 U) - beta0 (S - w0[k]), w0[k] = dp0dt_cc[k] / (gamma1_cc[k]
 * p0_cc[k]) per layer, instead of a dp0/dt term folded into S.  p0_cc,
 * gamma1_cc, dp0dt_cc: device arrays of nz layer values.  Everything else
 * (arguments, statuses, blocking) as mac_project. */
int mac_project_full(mg_handle h, const double* rho, const double* beta0_cc, const double* beta0_edge,
                     const double* S, const double* p0_cc, const double* gamma1_cc, const double* dp0dt_cc,
                     double* u, double* v, double* w, double* phi, mg_stats* stats, void* stream);

/* ---- spherical base state ------------------------------------------------ */

/* mac_project with beta0 a function of the radius from a centre (the
 * spherical base state of a star, Sec. 2, beta0 definition, with r the
 * distance from the star's centre): beta0_r (device, nr values) holds beta0 at
 * r_m = (m + 1/2) dr, m = 0..nr-1; beta0 at any point x is the linear
 * interpolation in r = |x - centre| between the two nearest r_m, held at
 * beta0_r[0] below r_0 and at beta0_r[nr-1] above r_{nr-1}.  centre (host, 3
 * values) is in the units of dx with the box's low corner at the origin; cell
 * (i,j,k) is centred at ((i+1/2) dx, (j+1/2) dx, (k+1/2) dx).  Face
 * coefficients use beta0 at the face centre, the beta0 S term beta0 at the cell
 * centre, and every face velocity of div(beta0 U) its own face's beta0.  Any
 * boundary types; arguments, statuses and blocking as mac_project
 * (beta0_r <= 0 somewhere: MG_ERR_INVALID_ARG; non-finite: MG_ERR_NONFINITE). */
int mac_project_radial(mg_handle h, const double* rho, int32_t nr, double dr, const double* beta0_r,
                       const double centre[3], const double* S, double* u, double* v, double* w,
                       double* phi, mg_stats* stats, void* stream);

/* The radial mapping alone: beta0_out (device, nz*ny*nx, C order) = beta0 of
 * the profile at every cell centre of an nx*ny*nz box of spacing dx, as
 * mac_project_radial evaluates it.  Stream-ordered: returns after enqueueing
 * one kernel. */
int mg_map_radial(int32_t nx, int32_t ny, int32_t nz, double dx, int32_t nr, double dr,
                  const double* beta0_r, const double centre[3], double* beta0_out, void* stream);

/* ---- nodal (cell-velocity) projection ----------------------------------- */

/* The other projection of the paper's second-order projection method (Sec. 3):
 * the cell-centred velocities are projected onto the same constraint
 * div(beta0 U) = beta0 S (Sec. 2), with the potential phi on the nodes (cell
 * corners).  Trilinear elements with the cell coefficient sigma = beta0/rho;
 * divided by the node volume h^3:
 *   (L phi)_n = 1/(12 h^2) sum_{cells c at n} sigma_c (sum of phi over the 4
 *               corners of c across a face or the body diagonal from n
 *               - 4 phi_n)
 *   f_n = 1/(4h) sum_c beta0_c (+-u_c +- v_c +- w_c) - 1/8 sum_c beta0_c S_c
 *   (+ for a cell on the high side of the node in that direction),
 * L phi = f solved by multigrid (four-colour Gauss-Seidel, colour (J mod 2)
 * + 2 (K mod 2) in the order 0..3, full-weighting
 * restriction, trilinear prolongation, coarse sigma the mean of the 8 fine
 * cells, exact coarsest solve on at most 512 nodes), then U_c -= (G phi)_c /
 * rho_c with G the cell's mean gradient of phi.  The projection is
 * approximate: L is not D sigma G, so the corrected velocity meets the
 * constraint to truncation error.  Boundaries: periodic (node n is node 0) or
 * solid wall (natural: wall nodes are unknowns).  Precision: FP64, or
 * MG_MIXED: each iteration p.inner_cycles FP32 V-cycles (default one here;
 * the first from zero) on the FP64 residual scaled by a power of two near
 * 1/rms(r), the FP32 correction added to the FP64 phi (divided by that
 * power of two, exactly), r = f - L phi and its norm in FP64, the same stop
 * test; stats.cycles counts iterations.
 * Layout: rho, S, uc, vc, wc (nz, ny, nx) cells; beta0_cc (nz); phi nodes
 * (Nz, Ny, Nx) with N = n (periodic) or n + 1 (walls), C order.  Device
 * pointers, caller-owned. */
typedef struct nodal_hierarchy* nodal_handle;

/* Levels for params (0: not solvable: bc other than periodic/wall, or the
 * coarsest level would exceed 512 nodes). */
int32_t nodal_num_levels_for(const mg_params* p);
/* Allocate a nodal hierarchy (FP64, or MG_MIXED with FP32 copies of every
 * level's arrays). */
int nodal_setup(const mg_params* p, nodal_handle* out);
int nodal_destroy(nodal_handle h);
/* The whole nodal projection: coefficients and right-hand side,
 * compatibility check (|sum f| <= 1e-8 sum |f|) and mean removal, V-cycles to
 * rtol, zero-mean phi (nullable output), correction of uc, vc, wc in place.
 * Blocks until done; statuses as mac_project. */
int nodal_project(nodal_handle h, const double* rho, const double* beta0_cc, const double* S, double* uc,
                  double* vc, double* wc, double* phi, mg_stats* stats, void* stream);
/* Tuning: force the fused nodal sweep's tile configuration (0..7: 64x8,
 * 32x8, 32x16, 64x16 nodes with 32-plane chunks, 64x8 with 64, 32x8 with 16,
 * 32x16 with 64, 64x8 with 16) on every level it takes; -1 restores the
 * per-level default.  Process-wide; results do not depend on it. */
int nodal_tune_sweep(int32_t cfg);
/* Coefficients only (for the single steps below). */
int nodal_set_coefficients(nodal_handle h, const double* rho, const double* beta0_cc, void* stream);
/* enable = 1 (the default): the V-cycle and the residual norm after it run as
 * one captured hipGraph replayed every cycle (all buffers are fixed);
 * results are identical either way. */
int nodal_set_graphs(nodal_handle h, int32_t enable);
/* enable = 1 (the default): the coarse levels whose phi, f and r fit in
 * 136 KB of LDS (with every coarser level's) run as one workgroup per V-cycle
 * (colours, residual, restriction, coarsest solve, prolongation with
 * barriers in between) instead of one launch per step; the per-node
 * arithmetic is the same, so results are identical either way. */
int nodal_set_bottom(nodal_handle h, int32_t enable);
typedef enum { MG_NOD_PHI = 0, MG_NOD_F = 1, MG_NOD_SIGMA = 2 } mg_nodal_array;
/* dims = {Nx, Ny, Nz, nx, ny, nz} of level l; *dx its spacing. */
int nodal_level_info(nodal_handle h, int32_t level, int32_t dims[6], double* dx);
/* Copy a level array (nodes: phi, f; cells: sigma) to or from a device
 * buffer, stream-ordered. */
int nodal_level_copy(nodal_handle h, int32_t level, int32_t array, void* buffer, int32_t to_hierarchy,
                     void* stream);
/* One step on level l: MG_STEP_SMOOTH (arg sweeps), MG_STEP_RESID_RESTRICT,
 * MG_STEP_PROLONG, MG_STEP_COARSE (coarsest level).  Stream-ordered. */
int nodal_level_step(nodal_handle h, int32_t level, int32_t step, int32_t arg, void* stream);

/* ---- single steps of the cycle, for step-by-step verification ---------- */
typedef enum {
    MG_STEP_SMOOTH = 0,          /* `arg` red-black GS sweeps on level l (phi_l, f_l) */
    MG_STEP_RESID_RESTRICT = 1,  /* f_{l+1} = R (f_l - L phi_l); phi_{l+1} = 0 */
    MG_STEP_PROLONG = 2,         /* phi_l += P phi_{l+1} */
    MG_STEP_COARSE = 3,          /* exact solve on the coarsest level */
    MG_STEP_DOWN = 4,            /* fused: `arg` sweeps + residual + restriction */
    MG_STEP_UP = 5               /* fused: prolongation + `arg` sweeps */
} mg_step;

typedef enum { MG_ARR_PHI = 0, MG_ARR_F = 1, MG_ARR_BX = 2, MG_ARR_BY = 3, MG_ARR_BZ = 4 } mg_array;

/* Level l's shape and spacing. */
int mg_level_info(mg_handle h, int32_t level, int32_t dims[3], double* dx);

/* Copy a level array between the hierarchy and a caller device buffer,
 * enqueued on `stream`
 * (to_hierarchy = 1: buffer -> hierarchy).  Cell arrays are (nz,ny,nx); the
 * coefficient arrays hold, per cell, the coefficient of its LOW face in that
 * direction (face n of a periodic direction is face 0; walls and outflow
 * sides hold 0 there: outflow boundary faces are kept separately). */
int mg_level_copy(mg_handle h, int32_t level, int32_t array, void* buffer,
                  int32_t to_hierarchy, void* stream);

/* Run one step (mg_step) on level l.  Like mg_level_copy, stream-ordered:
 * returns after enqueueing the work on `stream`.  On a box with outflow sides
 * the steps take their boundary faces from the last mg_set_coefficients or
 * projection. */
int mg_level_step(mg_handle h, int32_t level, int32_t step, int32_t arg, void* stream);

/* ---- batches and serving ------------------------------------------------ */

/* Solve `count` independent problems (any shapes, each with its own params)
 * with shared launches; stats has `count` entries (nullable).  Each result is
 * the one mac_project (nodal_project for MG_KIND_NODAL) gives for that
 * problem alone.  Single-box MAC problems whose finest level takes the fused
 * sweep run together, iteration by iteration; the others (nodal problems,
 * multi-box problems, small shapes) are solved one at a time on pooled
 * hierarchies, between those iterations.  Blocks until done.
 * stats[i].ms_total is the device time of the whole call, ms_smooth the
 * wall time from problem i's first iteration to its last (the iterations are
 * shared launches), ms_other the difference. */
int project_batch(int32_t count, const mg_problem* probs, mg_stats* stats, void* stream);

/* Continuous-batching server on the current device.  hbm_budget_bytes caps
 * the device memory of resident hierarchies plus in-flight work;
 * max_inflight caps the problems on the device at once. */
int serve_create(size_t hbm_budget_bytes, int32_t max_inflight, void** server);
/* Queue a problem (any kind, as for project_batch: nodal and multi-box
 * problems are solved one at a time on pooled hierarchies, between the
 * shared iterations); never blocks.  The problem's buffers must stay alive
 * until its ticket completes. */
int serve_submit(void* server, const mg_problem* prob, uint64_t* ticket);
/* A ticket is released once a poll or wait has returned its final status
 * (when no other wait is still blocked on it); later calls with it return
 * MG_ERR_INVALID_ARG.
 * MG_PENDING while the ticket is queued or running; else its final status,
 * with *out (nullable) filled. */
int serve_poll(void* server, uint64_t ticket, mg_stats* out);
/* Block until the ticket completes; returns its status.  For served
 * problems stats ms_total is the time from serve_submit to completion
 * (queueing included), ms_smooth the wall time from the request's first
 * iteration to its last, ms_other the difference. */
int serve_wait(void* server, uint64_t ticket, mg_stats* out);
/* Server counters: [0] submitted, [1] completed, [2] queued, [3] in flight,
 * [4] resident bytes, [5] peak in-flight problems. */
int serve_counters(void* server, double out[6]);
/* Finish all tickets and release the server. */
int serve_destroy(void* server);

/* Tuning: force fused-sweep tile configuration cfg (0..11: 32x8x32, 32x8x64,
 * 64x8x32, 32x16x32, 64x4x64, 32x4x64, 32x8x16, 32x8x8, 64x8x64, 64x16x32,
 * 32x32x32, 64x16x64 cells per workgroup tile x planes per chunk) on every
 * level that fits it; -1 restores the per-shape default.
 * Process-wide; results do not depend on it (the sweep is exact per cell). */
int mg_tune_sweep(int32_t cfg);

/* Autotune: time every fused-sweep configuration that fits each level of h
 * (`reps` sweeps each, on `stream`) and keep the fastest per level shape in a
 * process-wide table used by every later solve of that shape.  Needs
 * coefficients (mg_set_coefficients or mac_project); overwrites the
 * hierarchy's own level arrays, never caller data.  Blocks until done.
 * With the environment variable MACPROJ_TUNE_CACHE naming a file, the table
 * is read from it on first use and the whole table is written back after
 * every mg_autotune (a temporary file renamed over it). */
int mg_autotune(mg_handle h, int32_t reps, void* stream);

/* The tuning table and its cache file, host-side only (no device work).
 * Entries are keyed by GPU architecture name (arch, NULL = the current
 * device's gcnArchName), level shape n[3], coefficient source (rho = 1:
 * recomputed from rho on the finest level), precision (fp64 = 1: FP64) and
 * coarse (1: a coarse level of a single-problem V-cycle); the value is a
 * configuration index as for mg_tune_sweep.  The file is JSON
 * {"format": "macproj-sweep-tune-1", "entries": [{"arch", "n", "rho",
 * "fp64", "coarse", "cfg", "tile"}, ...]}; entries whose tile does not match
 * their index in this build are skipped.
 * mg_tune_cache_save/load: path NULL = MACPROJ_TUNE_CACHE; return the number
 * of entries written / taken, or MG_ERR_INVALID_ARG (unreadable, unwritable
 * or malformed file: a malformed file changes nothing).  Loading merges into
 * the table.  mg_tune_cache_clear empties the table (the environment's file
 * is then not read again).  mg_tune_record adds or replaces one entry
 * (MG_ERR_INVALID_ARG for an index out of range or a tile that does not fit
 * the shape); mg_tune_lookup returns the entry's index or -1. */
int mg_tune_cache_save(const char* path);
int mg_tune_cache_load(const char* path);
int mg_tune_cache_clear(void);
int mg_tune_record(const char* arch, const int32_t n[3], int32_t rho, int32_t fp64, int32_t coarse, int32_t cfg);
int mg_tune_lookup(const char* arch, const int32_t n[3], int32_t rho, int32_t fp64, int32_t coarse);

/* Replayable cycles: with enable = 1 (the default) an FP64 solve captures
 * one V-cycle plus the following residual-norm sweep as a hipGraph on the
 * hierarchy's own stream the first time it needs it, and replays it for the
 * later cycles and solves whose buffers, coefficient source, sweep counts
 * and tile choices match (at most two captures are kept per hierarchy).
 * Results are identical either way; 0 runs every cycle as separate launches
 * on the caller's stream. */
int mg_set_graphs(mg_handle h, int32_t enable);

/* Bottom of the V-cycle: with enable = 1 (the default) the levels below the
 * ones the fused sweep covers (when their phi and f fit in 136 KB of LDS) run
 * as one 1024-thread workgroup per V-cycle instead of one launch per step
 * and level.  Results are identical either way. */
int mg_set_bottom(mg_handle h, int32_t enable);

/* Multi-box finest level: the block-structured box layout whose boxes the
 * method distributes over MPI processes and tiles (Sec. 3), one
 * process per GPU (Sec. 6), here with every box on one device and the
 * inter-box halo exchange done by a kernel: box[0..2] = cells per box in
 * x, y, z, each even, >= 2 and at most the domain size.  The domain is tiled
 * by ceil(n/box) boxes per direction, all of box cells except the last one
 * of a direction that box does not divide, which holds the (even) remainder:
 * uneven boxes, as a domain chopped to a maximum box size.  Each box has its
 * own phi (two buffers), f and face coefficients inside a two-cell ghost
 * shell.  Every later mac_project on h smooths, restricts and prolongates
 * the finest level box by box with a halo exchange (ghost cells from the
 * box that owns the cell, the periodic image, or 0 beyond a wall) after
 * every sweep and after each prolongation; when every box, the smallest
 * included, has at least 32 x 8 x 4 cells, the boxes are swept by the fused
 * red-black sweep, otherwise one colour per launch with an exchange of that
 * colour in between.  Levels 1 and coarser are the single-box levels.  The
 * result agrees with the single-box solve to rounding (the same per-cell
 * arithmetic; the residual norm and the restriction may be summed in
 * another order).  box == NULL or {0, 0, 0} returns to a single box.
 * Needs periodic or wall sides and two or more levels; in mixed precision
 * (FP32 box sweeps, FP32 residual + restriction and an FP64 refinement over
 * the boxes, halos exchanged after each) also every box taking the fused
 * sweep and at most 2048 box tiles (MG_ERR_INVALID_ARG otherwise).  The boxes' arrays are allocated here
 * (device memory, freed by mg_destroy or the next mg_set_boxes), 7 x 8
 * bytes per cell of the ghosted boxes (7 x 4 more in mixed precision), each
 * sized for a full box; MG_ERR_HIP if that fails.  Batches and the server take the box size from
 * mg_problem.box. */
int mg_set_boxes(mg_handle h, const int32_t box[3]);

/* Fused-sweep tile used on level l of h: tile[0..2] = cells per workgroup
 * tile in x, y and planes per z-chunk, tile[3] = configuration index (as for
 * mg_tune_sweep).  All four are -1 for a level the fused sweep does not cover
 * (it then runs one kernel per colour). */
int mg_sweep_config(mg_handle h, int32_t level, int32_t tile[4]);

/* ---- allocation-free projection ------------------------------------------ */

/* Device bytes of the fixed scratch array behind mac_project_static. */
#define MG_STATIC_SCRATCH_BYTES (32u << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): mac_project for the
 * problem described by *p (shape, dx, bc, sweeps, rtol, max_cycles,
 * precision), with every multigrid level array, partial-sum row and scalar
 * in a fixed per-device array of MG_STATIC_SCRATCH_BYTES (32 MiB) instead of
 * a hierarchy from mg_setup.  Arguments, layout, ownership of the fields,
 * results, statuses and blocking are those of mac_project; the results equal
 * mac_project's on a hierarchy set up with the same params.  The call
 * allocates no device or pinned host memory and creates no events, streams
 * or graphs: the V-cycles run as separate launches on `stream`, and
 * stats->ms_total is the host wall time of the call.  Problems whose
 * mg_workspace_bytes(p) exceeds MG_STATIC_SCRATCH_BYTES (e.g. more than 64^3
 * cells in a cube) return MG_ERR_BAD_SIZE.  Each device the library runs on
 * holds the array from module load until the process ends; its device
 * address is looked up on the first call made with that device current
 * (devices 0..63).  Every call on a device shares that device's array and
 * host-side state, so calls that overlap on one device (several threads, or
 * several streams in flight) race; each call clears the part of the array it
 * uses before its own work. */
int mac_project_static(const mg_params* p, const double* rho, const double* beta0_cc,
                       const double* beta0_edge, const double* S, double* u, double* v, double* w,
                       double* phi, mg_stats* stats, void* stream);

const char* mg_strerror(int code);
const char* mg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MACPROJ_H */
