// Batched execution engine shared by project_batch and the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "runtime.h"

namespace mg {

// Pinned host ring mirrored in device memory, for per-launch descriptor
// tables.  Reset (off = 0) only after the stream has been synchronised.
struct Staging {
    char* host = nullptr;
    char* dev = nullptr;
    size_t cap = 0;
    size_t off = 0;
    int init(size_t bytes);
    void release();
    int push(const void* src, size_t bytes, hipStream_t st, void** out);
};

// One projection in flight.
struct Job {
    enum { kNew = 0, kSolve = 1, kFinish = 2, kDone = 3 };
    mg_problem pr{};
    mg_hierarchy* H = nullptr;
    mg_stats st{};
    int status = MG_OK;
    int stage = kNew;
    int cycles = 0;
    double fnorm = 0.0;
    double rel = 1.0;
    uint64_t ticket = 0;
    double t_submit = 0.0;
    double t_admit = 0.0;
    double t_done = 0.0;
    size_t bytes = 0;
};

// Problems the batched path runs (FP64 with the fused finest-level sweep);
// the others are solved one at a time by the single-problem path.
bool batchable(const mg_hierarchy* H);

struct Engine {
    Staging staging;
    // coefficients, right-hand side, compatibility check, norm of f
    int setup_new(std::vector<Job*>& fresh, hipStream_t st);
    // stop tests, one V-cycle for every job still solving, finish the rest
    int round(std::vector<Job*>& jobs, hipStream_t st);
};

}  // namespace mg
