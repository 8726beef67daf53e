// Batched execution engine shared by project_batch and the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "runtime.h"
#include "scheduler.h"

namespace mg {

// Descriptor tables of a captured round: pinned host bytes and their device
// copy, uploaded once after the capture and never changed afterwards.
struct Arena {
    char* host = nullptr;
    char* dev = nullptr;
    size_t cap = 0;
    size_t off = 0;
    bool overflow = false;
    int init(size_t bytes);
    void release();
};

// Per-launch descriptor tables.  Eagerly launched work copies each table
// from a pinned host ring to its device mirror on the stream (the ring is
// reset, off = 0, only after the stream has been synchronised); while a
// round is being captured (`rec` set) tables go to that round's arena
// instead, with no copy.
struct Staging {
    char* host = nullptr;
    char* dev = nullptr;
    size_t cap = 0;
    size_t off = 0;
    Arena* rec = nullptr;
    int init(size_t bytes);
    void release();
    int push(const void* src, size_t bytes, hipStream_t st, void** out);
};

// Problems the batched path runs (FP64 with the fused finest-level sweep, or
// mixed precision whose FP32 levels above the bottom are all fused); the
// others are solved one at a time by the single-problem path.
bool batchable(const mg_hierarchy* H);

struct Engine {
    Staging staging;
    // Graph policy for rounds: 0 never capture, 1 capture a round the first
    // time its key is seen, 2 the second time (keys that recur).
    int graph_mode = 1;

    // coefficients, right-hand side, compatibility check, norm of f
    int setup_new(std::vector<Job*>& fresh, hipStream_t st);
    // stop tests, one iteration (V-cycle + norm, or FP32 V-cycle +
    // refinement) for every job still solving, correction of the finished
    int round(std::vector<Job*>& jobs, hipStream_t st);
    // one iteration for the running sets (graph replay, capture or eager)
    int iterate(std::vector<mg_hierarchy*>& h64, const std::vector<int>& pre_done, std::vector<mg_hierarchy*>& hm,
                hipStream_t st);
    void release();
    ~Engine() { release(); }

    // rows of 4 doubles gathered from every problem's scalar block (device,
    // and its pinned host mirror); grown on demand
    double* gdev = nullptr;
    double* ghost = nullptr;
    int grows = 0;
    int ensure_gather(int rows);

    // captured rounds
    struct RoundGraph {
        std::vector<uintptr_t> key;
        hipGraphExec_t exec = nullptr;
        Arena arena;
        std::vector<void*> post;      // level phi pointers of the round's hierarchies after it
        uint64_t used = 0;
    };
    std::vector<RoundGraph> graphs;
    std::vector<std::vector<uintptr_t>> seen;     // recently seen keys (graph_mode 2)
    uint64_t clock = 0;
    hipStream_t gs = nullptr;
    hipEvent_t gev = nullptr;
    uint64_t captures = 0, replays = 0, eager = 0;
    void drop_graphs();
};

}  // namespace mg
