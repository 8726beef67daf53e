// Fused out-of-place red-black Gauss-Seidel sweep (sweep.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace mg {

constexpr int kSweepTX = 32;     // smallest tile width (x) of any configuration
constexpr int kSweepTY = 4;      // smallest tile height (y)
constexpr int kSweepTZMax = 64;  // largest z-chunk

// Tile configurations of the fused sweep (TX x TY columns, TZ planes per
// chunk); the autotuner picks one per level shape.
struct SweepCfg {
    int tx, ty, tz;
};
constexpr int kNumSweepCfg = 6;
constexpr SweepCfg kSweepCfgs[kNumSweepCfg] = {
    {32, 8, 32}, {32, 8, 64}, {64, 8, 32}, {32, 16, 32}, {64, 4, 64}, {32, 4, 64}};

enum { kInZero = 0, kInPlain = 1, kInProlong = 2 };

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
    const double* rho;         // finest level: coefficients from rho and beta0
    const double* b0c;
    const double* b0e;
};

template <typename T>
bool sweep_fusable(int nx, int ny, int nz);

template <typename T>
hipError_t launch_sweep(const SweepArgs<T>& a, bool use_rho, int in_mode, int cfg, hipStream_t st);

// Configuration used for a level of shape nx x ny x nz (autotuned choice or default).
int sweep_config_for(int nx, int ny, int nz);
// Force one configuration for every level that fits it (-1 restores the default).
void sweep_force_config(int cfg);

}  // namespace mg
