// Fused out-of-place red-black Gauss-Seidel sweep (sweep.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "mg_internal.h"

namespace mg {

constexpr int kSweepTX = 32;     // smallest tile width (x) of any configuration
constexpr int kSweepTY = 4;      // smallest tile height (y)
constexpr int kSweepTZMax = 64;  // largest z-chunk
constexpr int kMaxPartialRows = 2048;   // rows of a hierarchy's partial-sum buffer

// Tile configurations of the fused sweep (TX x TY columns, TZ planes per
// chunk); the autotuner picks one per level shape.
struct SweepCfg {
    int tx, ty, tz;
};
constexpr int kNumSweepCfg = 14;
constexpr int kFirstCoarseCfg = 12;     // 4-plane chunks: coarse levels of a single problem
constexpr SweepCfg kSweepCfgs[kNumSweepCfg] = {
    {32, 8, 32}, {32, 8, 64}, {64, 8, 32}, {32, 16, 32}, {64, 4, 64},  {32, 4, 64}, {32, 8, 16},
    {32, 8, 8},  {64, 8, 64}, {64, 16, 32}, {32, 32, 32}, {64, 16, 64}, {32, 8, 4}, {32, 4, 4}};

enum { kInZero = 0, kInPlain = 1, kInProlong = 2, kInCorrect = 3 };
enum { kOpSweep = 0, kOpSweepNorm = 1, kOpResidRestrict = 2, kOpRefine = 3 };

template <typename T>
struct SweepArgs {
    int nx, ny, nz;
    int px, py, pz;            // periodic flags (finest level, coefficient recompute)
    int tz;                    // planes per chunk
    int ntx, nty;              // filled by the launcher
    T h2;
    const T* phi_in;           // unused for kInZero
    T* phi_out;
    const T* f;
    const T* phic;             // coarse phi for kInProlong
    const T* bx;               // stored coefficients (coarse levels)
    const T* by;
    const T* bz;
    const T* rho;              // finest level: coefficients from rho and beta0
    const double* b0c;
    const double* b0e;
    double* partials;          // residual-norm rows (kOpSweepNorm, kOpRefine), one per tile
    T* fc;                     // coarse right-hand side (kOpResidRestrict)
    T* phic_out;               // coarse phi, zeroed (kOpResidRestrict)
    const float* corr;         // kInCorrect: input is phi_in + corr / scales[0]
    float* r32;                // kOpRefine: r32 = (float)(scales[1] * (f - L phi))
    const double* scales;      // device {scale of corr's right-hand side, scale for r32}
    int has_bnd;               // outflow sides: their boundary faces add to the diagonal
    Bnd<T> bnd;                // which sides are outflow sides (non-null)
    const T* dg;               // per-cell boundary diagonal (bnd_diag of every cell)
    int ox, oy, oz;            // launch_sweep_boxes: first cell of a box interior
    int ex, ey, ez;            // launch_sweep_boxes: box cells
    int wlo[3], whi[3];        // launch_sweep_boxes with rho: wall faces (low faces of these cells), -1 none
    int go[3], gn[3], gp[3];   // launch_sweep_boxes with prolongation: box origin, domain cells, periodic
};

template <typename T>
bool sweep_fusable(int nx, int ny, int nz);

template <typename T>
hipError_t launch_sweep(const SweepArgs<T>& a, bool use_rho, int in_mode, int cfg, hipStream_t st);

// Finest-level sweep of phi_in (as stored; coefficients from rho, or stored
// with use_rho = false) that also writes, per tile, the partial row
// {sum r^2, 0, 0, 0} of the residual r = f - L phi_in of its INPUT (a
// non-finite r makes the sum non-finite).  *nparts = rows written.
hipError_t launch_sweep_norm(const SweepArgs<double>& a, bool use_rho, int cfg, int* nparts, hipStream_t st);

// Finest level: f_c = R (f - L phi), phi_c = 0, using the sweep's tiles (each
// face coefficient computed or read once per cell).  Needs even tile
// origins, which every configuration has.
template <typename T>
hipError_t launch_resid_restrict_tiled(const SweepArgs<T>& a, bool use_rho, int cfg, hipStream_t st);

// Refinement step of the mixed-precision solve (finest level, FP64):
// phi_out = phi_in + corr / scales[0]; per tile the partial row
// {sum r^2, 0, 0, 0} of r = f - L phi_out; and r32 = (float)(scales[1] * r).
// The scales are powers of two read from device memory, so a captured launch
// stays valid as they change.  *nparts = rows written.
hipError_t launch_refine(const SweepArgs<double>& a, bool use_rho, int cfg, int* nparts, hipStream_t st);

// Batched form (one launch, many problems): descriptor i (device) is problem
// i's SweepArgs with tz/ntx/nty filled (sweep_geometry); launch tile b is tile
// tmap[b].y of problem tmap[b].x (device, `tiles` entries, every problem's
// tiles in order); `op` is kOpSweep, kOpResidRestrict, or (FP64 with rho
// only) kOpSweepNorm (plain input) or kOpRefine (corrected input).  Tile
// shapes 32x8, 64x8, 32x4 and 64x16.
template <typename T>
hipError_t launch_sweep_multi(const SweepArgs<T>* d, const int2* tmap, int tiles, bool use_rho, int in_mode, int op,
                              int cfg, hipStream_t st);
void sweep_geometry(SweepArgs<double>& a, int cfg);
void sweep_geometry(SweepArgs<float>& a, int cfg);

// One sweep of every box of a multi-box finest level in one launch: nbox
// boxes stored bstride elements apart, each a ghosted array of a.nx x a.ny x
// a.nz cells whose interior (a.ex x a.ey x a.ez cells from (a.ox, a.oy,
// a.oz), ghost width >= 2) is swept out of place from phi_in to phi_out with
// stored coefficients (bx, by, bz, cell-aligned low faces in the same
// layout); the ghosts must hold the neighbouring values, and phi_out's are
// not written.  hipErrorInvalidValue for a shape it does not cover
// (sweep_boxes_fit).  nparts != null: also the per-tile partial rows
// {sum r^2, 0, 0, 0} of the residual of the INPUT over the box interiors
// into a.partials (*nparts rows, at most kMaxPartialRows, else
// hipErrorInvalidValue).
// With a.rho set the coefficients are recomputed from each box's ghosted rho
// and its own beta0 (a.b0c, a.b0e: g.b0stride entries per box, one per
// ghosted plane); g places the domain's walls.
struct BoxGeom {
    int nb[3];                 // boxes per direction
    int per[3];                // periodic directions
    int b0stride;              // beta0 entries per box
    int box[3];                // cells of a full box; the last box of a direction holds n - (nb - 1) box
    int n[3];                  // domain cells
};
bool sweep_boxes_fit(int bx, int by, int bz);
int sweep_boxes_tiles(int bx, int by, int bz);      // tiles per box
// prolong: the input is phi_in + P a.phic (a.phic: the domain's single
// coarser level), the prolongation folded into the load as on a single box.
// restrict_only: no sweep; the residual of phi_in restricted into the
// domain's single coarser level (a.fc, a.phic_out = 0), as the tiled
// single-box residual + restriction does.
hipError_t launch_sweep_boxes(const SweepArgs<double>& a, const BoxGeom& g, int nbox, size_t bstride, int* nparts,
                              hipStream_t st, bool prolong = false, bool restrict_only = false);
// The same over every box in T with an explicit operation: a sweep of phi_in
// as stored, of 0 (kInZero) or of phi_in + P phic; the residual + restriction;
// and (FP64, partial rows) the sweep with the residual norm of its input or
// the mixed-precision refinement (phi_out = phi_in + corr / scales[0] on the
// interiors, r32 = scales[1] (f - L phi_out) there, corr and r32 in the same
// box layout).  nparts must be given exactly for the two row-writing modes.
enum { kBoxSweep = 0, kBoxSweepZero = 1, kBoxSweepProlong = 2, kBoxSweepNorm = 3, kBoxResidRestrict = 4,
       kBoxRefine = 5 };
template <typename T>
hipError_t launch_sweep_boxes_mode(const SweepArgs<T>& a, const BoxGeom& g, int nbox, size_t bstride, int mode,
                                   int* nparts, hipStream_t st);

// Number of tiles (= partial rows) a sweep of this shape launches with cfg.
int sweep_tiles(int nx, int ny, int nz, int cfg);

// Configuration used for a level of shape nx x ny x nz whose coefficients come
// from rho (finest level) or are stored, in FP64 (dbl) or FP32, as the
// finest level of a problem or (coarse) a coarser level of a single-problem
// V-cycle: forced, autotuned, else a measured default.  Configurations
// kFirstCoarseCfg and up are only chosen for coarse levels.  A deterministic function of these, so
// a problem's tiles (and the order of its per-tile norm rows) are the same in
// solo and batched runs.
int sweep_config_for(int nx, int ny, int nz, bool rho, bool dbl = true, bool coarse = false);
bool sweep_cfg_fits(int nx, int ny, int cfg);
void sweep_record_tuned(int nx, int ny, int nz, bool rho, bool dbl, int cfg, bool coarse);
int sweep_tuned_count();
// Force one configuration for every level that fits it (-1 restores the default).
void sweep_force_config(int cfg);
// Incremented whenever a forced or tuned configuration changes (captured
// launches are only valid for the epoch they were recorded in).
unsigned sweep_tune_epoch();

// The tuning table (tune.hip): autotuned configurations keyed by the current
// device's architecture and the level shape / coefficient source /
// precision / coarse flag, persisted through the file named by
// MACPROJ_TUNE_CACHE (read on first use, written by tune_save_env).
int tune_find(int nx, int ny, int nz, bool rho, bool dbl, bool coarse);    // -1: none
void tune_put(int nx, int ny, int nz, bool rho, bool dbl, bool coarse, int cfg);
int tune_count();
unsigned tune_epoch();
void tune_force(int cfg);          // -1: per-shape choice
int tune_forced();
int tune_save_env();               // entries written (0 without MACPROJ_TUNE_CACHE) or an mg_status

}  // namespace mg
