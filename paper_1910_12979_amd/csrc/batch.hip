// Batched execution of many independent projections.
//
// Every problem keeps its own hierarchy and goes through exactly the
// sequence of kernels a single mac_project would run on it (same kernel
// bodies, same per-problem tile geometry and reduction order), so its result
// is bit-identical to the single-problem result.  What is shared is the
// launch: at every step one launch covers that step for all active problems
// (their tiles, cells or blocks concatenated, a descriptor table telling each
// workgroup which problem it belongs to) -- the set-up (coefficients,
// right-hand side, coarse coefficients, coarsest-level inverses, FP32
// mirrors), every step of the V-cycle, and the finishing correction.
//
// Problems stop independently; the active set is revisited once per
// iteration (a V-cycle plus the speculative sweep that measures its
// residual, or an FP32 V-cycle plus the FP64 refinement), which is also
// where the serving loop admits new requests.  An iteration's launches for a
// given active set are captured once as a hipGraph, with their descriptor
// tables in an arena owned by that graph, and replayed while the same set
// (same hierarchies, buffers and settings) recurs; every problem's norm row
// lands in one gathered block copied to the host once per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <type_traits>
#include <vector>

#include "batch.h"
#include "mg_internal.h"
#include "runtime.h"
#include "sweep.h"

namespace mg {

#define BHIP(expr)                                                      \
    do {                                                                \
        hipError_t e_ = (expr);                                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr, __LINE__);     \
    } while (0)

// ---------------------------------------------------------------------------
// descriptor staging: pinned host ring mirrored on the device
// ---------------------------------------------------------------------------
int Arena::init(size_t bytes) {
    cap = bytes;
    off = 0;
    overflow = false;
    if (hipHostMalloc((void**)&host, bytes, hipHostMallocDefault) != hipSuccess) {
        host = nullptr;
        return MG_ERR_OOM;
    }
    if (hipMalloc((void**)&dev, bytes) != hipSuccess) {
        dev = nullptr;
        return MG_ERR_OOM;
    }
    return MG_OK;
}

void Arena::release() {
    if (host) hipHostFree(host);
    if (dev) hipFree(dev);
    host = dev = nullptr;
    cap = off = 0;
}

int Staging::init(size_t bytes) {
    cap = bytes;
    if (hipHostMalloc((void**)&host, bytes, hipHostMallocDefault) != hipSuccess) return MG_ERR_OOM;
    if (hipMalloc((void**)&dev, bytes) != hipSuccess) return MG_ERR_OOM;
    return MG_OK;
}

void Staging::release() {
    if (host) hipHostFree(host);
    if (dev) hipFree(dev);
    host = dev = nullptr;
}

int Staging::push(const void* src, size_t bytes, hipStream_t st, void** out) {
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (rec) {
        // capture: the table goes to the round's arena (uploaded once later);
        // an arena that is too small marks the capture for a retry
        if (rec->off + need > rec->cap) {
            rec->overflow = true;
            rec->off += need;
            *out = rec->dev;
            return MG_OK;
        }
        std::memcpy(rec->host + rec->off, src, bytes);
        *out = rec->dev + rec->off;
        rec->off += need;
        return MG_OK;
    }
    if (off + need > cap) {
        // everything staged so far must have been copied before reuse
        BHIP(hipStreamSynchronize(st));
        off = 0;
        if (need > cap) {
            set_error("descriptor table larger than the staging buffer");
            return MG_ERR_OOM;
        }
    }
    std::memcpy(host + off, src, bytes);
    BHIP(hipMemcpyAsync(dev + off, host + off, bytes, hipMemcpyHostToDevice, st));
    *out = dev + off;
    off += need;
    return MG_OK;
}

namespace {

struct Item {
    mg_hierarchy* H;
    int l;
    int nsweeps;
};

bool rho_level(const mg_hierarchy* H, int l) { return l == 0 && H->rho.rho != nullptr; }

SweepArgs<double> sweep_args(mg_hierarchy* H, int l) {
    Level& F = H->lev[l];
    SweepArgs<double> a{};
    a.nx = F.nx;
    a.ny = F.ny;
    a.nz = F.nz;
    a.px = H->px;
    a.py = H->py;
    a.pz = H->pz;
    a.h2 = F.h * F.h;
    a.phi_in = F.d.phi;
    a.phi_out = F.phi2_d;
    a.f = F.d.f;
    a.phic = l + 1 < H->nlev ? H->lev[l + 1].d.phi : nullptr;
    a.bx = F.d.bx;
    a.by = F.d.by;
    a.bz = F.d.bz;
    a.rho = H->rho.rho;
    a.b0c = H->rho.b0c;
    a.b0e = H->rho.b0e;
    a.partials = H->partials;
    if (l + 1 < H->nlev) {
        a.fc = H->lev[l + 1].d.f;
        a.phic_out = H->lev[l + 1].d.phi;
    }
    return a;
}

bool multi_tile_shape(int cfg) {
    const SweepCfg& c = kSweepCfgs[cfg];
    return (c.tx == 32 && c.ty == 8) || (c.tx == 64 && c.ty == 8) || (c.tx == 32 && c.ty == 4) ||
           (c.tx == 64 && c.ty == 16);
}

// One batched launch of the fused sweep kernel (op) over `grp`, grouped by
// tile configuration; problems whose configuration has no batched form run
// the single-problem kernel (same body).
int launch_fused(std::vector<Item>& grp, bool use_rho, int in_mode, int op, Staging& S, hipStream_t st) {
    std::map<int, std::vector<Item*>> by_cfg;
    for (auto& it : grp) {
        Level& F = it.H->lev[it.l];
        by_cfg[sweep_config_for(F.nx, F.ny, F.nz, use_rho)].push_back(&it);
    }
    for (auto& kv : by_cfg) {
        const int cfg = kv.first;
        if (!multi_tile_shape(cfg)) {
            for (Item* it : kv.second) {
                SweepArgs<double> a = sweep_args(it->H, it->l);
                if (op == kOpSweep) {
                    BHIP(launch_sweep<double>(a, use_rho, in_mode, cfg, st));
                } else if (op == kOpSweepNorm) {
                    int np = 0;
                    BHIP(launch_sweep_norm(a, use_rho, cfg, &np, st));
                } else {
                    BHIP(launch_resid_restrict_tiled(a, use_rho, cfg, st));
                }
            }
            continue;
        }
        std::vector<SweepArgs<double>> descs;
        std::vector<int2> tmap;
        for (Item* it : kv.second) {
            SweepArgs<double> a = sweep_args(it->H, it->l);
            sweep_geometry(a, cfg);
            const int nt = sweep_tiles(a.nx, a.ny, a.nz, cfg);
            for (int t = 0; t < nt; ++t) tmap.push_back(make_int2((int)descs.size(), t));
            descs.push_back(a);
        }
        void* dd = nullptr;
        void* dp = nullptr;
        int rc = S.push(descs.data(), descs.size() * sizeof(SweepArgs<double>), st, &dd);
        if (rc) return rc;
        rc = S.push(tmap.data(), tmap.size() * sizeof(int2), st, &dp);
        if (rc) return rc;
        BHIP(launch_sweep_multi<double>((const SweepArgs<double>*)dd, (const int2*)dp, (int)tmap.size(), use_rho,
                                        in_mode, op, cfg, st));
    }
    return MG_OK;
}

CellDesc cell_desc(mg_hierarchy* H, int l) {
    Level& F = H->lev[l];
    CellDesc c{};
    c.nx = F.nx;
    c.ny = F.ny;
    c.nz = F.nz;
    c.h2 = F.h * F.h;
    c.phi = F.d.phi;
    c.f = F.d.f;
    c.bx = F.d.bx;
    c.by = F.d.by;
    c.bz = F.d.bz;
    if (l + 1 < H->nlev) {
        c.fc = H->lev[l + 1].d.f;
        c.phic = H->lev[l + 1].d.phi;
    }
    c.minv = H->minv;
    return c;
}

// batched small-level launch: `per_problem_threads` work items per problem
template <typename F>
int launch_cells(std::vector<Item*>& its, size_t (*work)(const Level&), F launch, Staging& S, hipStream_t st) {
    if (its.empty()) return MG_OK;
    std::vector<CellDesc> d;
    int blocks = 0;
    for (Item* it : its) {
        CellDesc c = cell_desc(it->H, it->l);
        c.block0 = blocks;
        blocks += (int)((work(it->H->lev[it->l]) + 255) / 256);
        d.push_back(c);
    }
    void* dd = nullptr;
    int rc = S.push(d.data(), d.size() * sizeof(CellDesc), st, &dd);
    if (rc) return rc;
    BHIP(launch((const CellDesc*)dd, (int)d.size(), blocks));
    return MG_OK;
}

size_t half_cells(const Level& L) { return (size_t)(L.nx / 2) * L.ny * L.nz; }
size_t coarse_cells(const Level& L) { return (size_t)(L.nx / 2) * (L.ny / 2) * (L.nz / 2); }
size_t all_cells(const Level& L) { return L.N; }

}  // namespace

// Sweeps on a list of (hierarchy, level, count) items: the batched form of
// the single-problem smooth(): fused out-of-place sweeps where the level
// allows them, per-colour in-place sweeps otherwise.
int multi_smooth(std::vector<Item>& items, int first, Staging& S, hipStream_t st) {
    std::vector<Item*> small;
    int maxk = 0;
    for (auto& it : items) {
        Level& F = it.H->lev[it.l];
        if (!sweep_fusable<double>(F.nx, F.ny, F.nz)) small.push_back(&it);
        maxk = std::max(maxk, it.nsweeps);
    }
    // prolongation alone (no sweep to fold it into)
    {
        std::vector<Item*> pro;
        for (auto& it : items)
            if (first == kInProlong && it.nsweeps == 0) pro.push_back(&it);
        int rc = launch_cells(pro, all_cells,
                              [&](const CellDesc* d, int n, int b) { return launch_prolong_multi(d, n, b, st); }, S, st);
        if (rc) return rc;
    }
    // small levels: prolongation / zero start once, then in-place sweeps
    {
        std::vector<Item*> pro, sm;
        std::vector<EltDesc> zero;
        int zb = 0;
        for (Item* it : small) {
            if (it->nsweeps == 0) continue;
            sm.push_back(it);
            if (first == kInProlong) pro.push_back(it);
            if (first == kInZero) {
                Level& F = it->H->lev[it->l];
                zero.push_back(EltDesc{kEltFill, zb, F.N, nullptr, F.d.phi, 0.0});
                zb += elt_blocks(F.N);
            }
        }
        if (!zero.empty()) {
            void* dd = nullptr;
            int rc = S.push(zero.data(), zero.size() * sizeof(EltDesc), st, &dd);
            if (rc) return rc;
            BHIP(launch_elt_multi((const EltDesc*)dd, (int)zero.size(), zb, st));
        }
        int rc = launch_cells(pro, all_cells,
                              [&](const CellDesc* d, int n, int b) { return launch_prolong_multi(d, n, b, st); }, S, st);
        if (rc) return rc;
        for (int k = 0; k < maxk; ++k) {
            std::vector<Item*> now;
            for (Item* it : sm)
                if (k < it->nsweeps) now.push_back(it);
            for (int colour = 0; colour < 2; ++colour) {
                rc = launch_cells(now, half_cells,
                                  [&](const CellDesc* d, int n, int b) { return launch_rbgs_multi(d, n, b, colour, st); },
                                  S, st);
                if (rc) return rc;
            }
        }
    }
    // fused levels, grouped by coefficient source (rho on the finest level)
    for (int k = 0; k < maxk; ++k) {
        for (int rho = 0; rho < 2; ++rho) {
            std::vector<Item> grp;
            for (auto& it : items) {
                Level& F = it.H->lev[it.l];
                if (k >= it.nsweeps || !sweep_fusable<double>(F.nx, F.ny, F.nz)) continue;
                if (rho_level(it.H, it.l) != (rho == 1)) continue;
                grp.push_back(it);
            }
            if (grp.empty()) continue;
            int rc = launch_fused(grp, rho == 1, k == 0 ? first : (int)kInPlain, kOpSweep, S, st);
            if (rc) return rc;
            for (auto& it : grp) std::swap(it.H->lev[it.l].d.phi, it.H->lev[it.l].phi2_d);
        }
    }
    return MG_OK;
}

// r_l = f_l - L phi_l restricted into f_{l+1}; phi_{l+1} = 0 (batched form).
int multi_resid_restrict(std::vector<Item>& items, Staging& S, hipStream_t st) {
    std::vector<Item> tiled;
    std::vector<Item*> cells;
    for (auto& it : items) {
        Level& F = it.H->lev[it.l];
        if (rho_level(it.H, it.l)) {
            if (sweep_fusable<double>(F.nx, F.ny, F.nz)) {
                tiled.push_back(it);
            } else {
                Level& C = it.H->lev[it.l + 1];
                BHIP(launch_resid_restrict_rho(Shape{F.nx, F.ny, F.nz}, F.h, it.H->rho, F.d.phi, F.d.f, C.d.f, C.d.phi,
                                               st));
            }
        } else {
            cells.push_back(&it);
        }
    }
    if (!tiled.empty()) {
        int rc = launch_fused(tiled, true, kInPlain, kOpResidRestrict, S, st);
        if (rc) return rc;
    }
    return launch_cells(cells, coarse_cells,
                        [&](const CellDesc* d, int n, int b) { return launch_resid_restrict_multi(d, n, b, st); }, S, st);
}

int multi_coarse(std::vector<mg_hierarchy*>& hs, Staging& S, hipStream_t st) {
    if (hs.empty()) return MG_OK;
    std::vector<CellDesc> d;
    for (auto* H : hs) d.push_back(cell_desc(H, H->nlev - 1));
    void* dd = nullptr;
    int rc = S.push(d.data(), d.size() * sizeof(CellDesc), st, &dd);
    if (rc) return rc;
    BHIP(launch_coarse_solve_multi((const CellDesc*)dd, (int)d.size(), st));
    return MG_OK;
}

// Speculative first pre-sweep with the residual norm of each problem's
// current finest-level phi; problem i's reduced row lands in its scalar
// block (kSlotRes) and in row i of `gather`.
int multi_norm_sweep(std::vector<mg_hierarchy*>& hs, double* gather, Staging& S, hipStream_t st) {
    if (hs.empty()) return MG_OK;
    std::vector<Item> grp;
    for (auto* H : hs) grp.push_back(Item{H, 0, 1});
    int rc = launch_fused(grp, true, kInPlain, kOpSweepNorm, S, st);
    if (rc) return rc;
    std::vector<ReduceDesc> rd;
    for (size_t i = 0; i < hs.size(); ++i) {
        mg_hierarchy* H = hs[i];
        Level& L0 = H->lev[0];
        rd.push_back(ReduceDesc{H->partials, sweep_tiles(L0.nx, L0.ny, L0.nz, sweep_config_for(L0.nx, L0.ny, L0.nz, true)),
                                H->scal + kSlotRes * kReduceWidth, gather + i * kReduceWidth});
    }
    void* dd = nullptr;
    rc = S.push(rd.data(), rd.size() * sizeof(ReduceDesc), st, &dd);
    if (rc) return rc;
    BHIP(launch_reduce_multi((const ReduceDesc*)dd, (int)rd.size(), st));
    return MG_OK;
}

// One V-cycle for every job in `jobs` (each at its own depth).  pre_done[i]
// finest-level pre-sweeps were already run by the speculative norm sweep.
int multi_vcycle(std::vector<mg_hierarchy*>& hs, const std::vector<int>& pre_done, Staging& S, hipStream_t st) {
    // levels each problem runs level by level: down to its bottom-solver
    // level, else down to (excluding) its coarsest
    std::vector<int> stop(hs.size());
    int lmax = 0;
    for (size_t i = 0; i < hs.size(); ++i) {
        const int b = bottom_start<double>(hs[i]);
        stop[i] = b > 0 ? b : hs[i]->nlev - 1;
        lmax = std::max(lmax, stop[i]);
    }
    for (int l = 0; l < lmax; ++l) {
        std::vector<Item> items;
        for (size_t i = 0; i < hs.size(); ++i) {
            mg_hierarchy* H = hs[i];
            if (l >= stop[i]) continue;
            items.push_back(Item{H, l, H->p.pre_sweeps - (l == 0 ? pre_done[i] : 0)});
        }
        // finest level: plain input; the other levels start from zero
        int rc = multi_smooth(items, l == 0 ? kInPlain : kInZero, S, st);
        if (rc) return rc;
        rc = multi_resid_restrict(items, S, st);
        if (rc) return rc;
    }
    std::vector<mg_hierarchy*> direct;
    std::vector<BottomArgs<double>> bottoms;
    for (size_t i = 0; i < hs.size(); ++i) {
        if (stop[i] == hs[i]->nlev - 1) {
            direct.push_back(hs[i]);
        } else {
            BottomArgs<double> a;
            bottom_args<double>(hs[i], stop[i], a);
            bottoms.push_back(a);
        }
    }
    int rc = multi_coarse(direct, S, st);
    if (rc) return rc;
    if (!bottoms.empty()) {
        void* dd = nullptr;
        rc = S.push(bottoms.data(), bottoms.size() * sizeof(BottomArgs<double>), st, &dd);
        if (rc) return rc;
        BHIP(launch_bottom_multi((const BottomArgs<double>*)dd, (int)bottoms.size(), st));
    }
    for (int l = lmax - 1; l >= 0; --l) {
        std::vector<Item> items;
        for (size_t i = 0; i < hs.size(); ++i)
            if (l < stop[i]) items.push_back(Item{hs[i], l, hs[i]->p.post_sweeps});
        rc = multi_smooth(items, kInProlong, S, st);
        if (rc) return rc;
    }
    return MG_OK;
}

// ---------------------------------------------------------------------------
// mixed precision: one FP32 V-cycle from zero on every problem's scaled
// residual (fused levels and the one-workgroup bottom), then the FP64
// refinement kernel, the norm rows and the next residual scales
// ---------------------------------------------------------------------------
namespace {

SweepArgs<float> sweep_args_f32(mg_hierarchy* H, int l) {
    Level& F = H->lev[l];
    SweepArgs<float> a{};
    a.nx = F.nx;
    a.ny = F.ny;
    a.nz = F.nz;
    a.px = H->px;
    a.py = H->py;
    a.pz = H->pz;
    a.h2 = (float)(F.h * F.h);
    a.phi_in = F.s.phi;
    a.phi_out = F.phi2_s;
    a.f = F.s.f;
    a.phic = l + 1 < H->nlev ? H->lev[l + 1].s.phi : nullptr;
    a.bx = F.s.bx;
    a.by = F.s.by;
    a.bz = F.s.bz;
    a.rho = l == 0 ? H->rho32 : nullptr;
    a.b0c = H->rho.b0c;
    a.b0e = H->rho.b0e;
    if (l + 1 < H->nlev) {
        a.fc = H->lev[l + 1].s.f;
        a.phic_out = H->lev[l + 1].s.phi;
    }
    return a;
}

// One launch per tile configuration of `op` over the given descriptors: the
// batched kernel where the tile shape has one, else one launch per problem.
template <typename T>
int launch_group(std::vector<SweepArgs<T>>& args, const std::vector<int>& cfgs, bool use_rho, int in_mode, int op,
                 Staging& S, hipStream_t st) {
    std::map<int, std::vector<size_t>> by_cfg;
    for (size_t i = 0; i < args.size(); ++i) by_cfg[cfgs[i]].push_back(i);
    for (auto& kv : by_cfg) {
        const int cfg = kv.first;
        if (!multi_tile_shape(cfg)) {
            for (size_t i : kv.second) {
                if (op == kOpSweep) {
                    BHIP(launch_sweep<T>(args[i], use_rho, in_mode, cfg, st));
                } else if (op == kOpResidRestrict) {
                    BHIP(launch_resid_restrict_tiled<T>(args[i], use_rho, cfg, st));
                } else {
                    if constexpr (std::is_same<T, double>::value) {
                        int np = 0;
                        BHIP(launch_refine(args[i], use_rho, cfg, &np, st));
                    }
                }
            }
            continue;
        }
        std::vector<SweepArgs<T>> descs;
        std::vector<int2> tmap;
        for (size_t i : kv.second) {
            SweepArgs<T> a = args[i];
            sweep_geometry(a, cfg);
            const int nt = sweep_tiles(a.nx, a.ny, a.nz, cfg);
            for (int t = 0; t < nt; ++t) tmap.push_back(make_int2((int)descs.size(), t));
            descs.push_back(a);
        }
        void* dd = nullptr;
        void* dp = nullptr;
        int rc = S.push(descs.data(), descs.size() * sizeof(SweepArgs<T>), st, &dd);
        if (rc) return rc;
        rc = S.push(tmap.data(), tmap.size() * sizeof(int2), st, &dp);
        if (rc) return rc;
        BHIP(launch_sweep_multi<T>((const SweepArgs<T>*)dd, (const int2*)dp, (int)tmap.size(), use_rho, in_mode, op,
                                   cfg, st));
    }
    return MG_OK;
}

// FP32 V-cycle on every problem (all of whose levels above the bottom are
// fused-sweep levels), the batched form of vcycle<float>: from zero, or
// (zero_start false) from the current finest-level correction.
int multi_vcycle_f32(std::vector<mg_hierarchy*>& hs, Staging& S, hipStream_t st, bool zero_start) {
    std::vector<int> stop(hs.size());
    int lmax = 0;
    for (size_t i = 0; i < hs.size(); ++i) {
        stop[i] = bottom_start<float>(hs[i]);
        lmax = std::max(lmax, stop[i]);
    }
    auto sweeps = [&](int l, bool post, int first) -> int {
        int maxk = 0;
        for (size_t i = 0; i < hs.size(); ++i)
            if (l < stop[i]) maxk = std::max(maxk, post ? hs[i]->p.post_sweeps : hs[i]->p.pre_sweeps);
        for (int k = 0; k < maxk; ++k) {
            std::vector<SweepArgs<float>> args;
            std::vector<int> cfgs;
            std::vector<mg_hierarchy*> who;
            for (size_t i = 0; i < hs.size(); ++i) {
                mg_hierarchy* H = hs[i];
                if (l >= stop[i] || k >= (post ? H->p.post_sweeps : H->p.pre_sweeps)) continue;
                const Level& F = H->lev[l];
                args.push_back(sweep_args_f32(H, l));
                cfgs.push_back(sweep_config_for(F.nx, F.ny, F.nz, l == 0, false));
                who.push_back(H);
            }
            if (args.empty()) continue;
            int rc = launch_group<float>(args, cfgs, l == 0, k == 0 ? first : (int)kInPlain, kOpSweep, S, st);
            if (rc) return rc;
            for (auto* H : who) std::swap(H->lev[l].s.phi, H->lev[l].phi2_s);
        }
        return MG_OK;        // (batched mixed problems have post-sweeps: the prolongation is folded in)
    };
    for (int l = 0; l < lmax; ++l) {
        int rc = sweeps(l, false, l == 0 && !zero_start ? (int)kInPlain : (int)kInZero);
        if (rc) return rc;
        std::vector<SweepArgs<float>> args;
        std::vector<int> cfgs;
        for (size_t i = 0; i < hs.size(); ++i) {
            if (l >= stop[i]) continue;
            const Level& F = hs[i]->lev[l];
            args.push_back(sweep_args_f32(hs[i], l));
            cfgs.push_back(sweep_config_for(F.nx, F.ny, F.nz, l == 0, false));
        }
        rc = launch_group<float>(args, cfgs, l == 0, kInPlain, kOpResidRestrict, S, st);
        if (rc) return rc;
    }
    std::vector<BottomArgs<float>> bottoms;
    for (size_t i = 0; i < hs.size(); ++i) {
        BottomArgs<float> a;
        bottom_args<float>(hs[i], stop[i], a);
        bottoms.push_back(a);
    }
    void* dd = nullptr;
    int rc = S.push(bottoms.data(), bottoms.size() * sizeof(BottomArgs<float>), st, &dd);
    if (rc) return rc;
    BHIP(launch_bottom_multi((const BottomArgs<float>*)dd, (int)bottoms.size(), st));
    for (int l = lmax - 1; l >= 0; --l) {
        rc = sweeps(l, true, kInProlong);
        if (rc) return rc;
    }
    return MG_OK;
}

// FP64 refinement of every problem: phi += e32 / scale, residual, FP32
// residual for the next cycle, norm rows reduced (problem i's also into row
// i of `gather`), scales advanced.
int multi_refine(std::vector<mg_hierarchy*>& hs, double* gather, Staging& S, hipStream_t st) {
    std::vector<SweepArgs<double>> args;
    std::vector<int> cfgs;
    std::vector<ReduceDesc> rd;
    std::vector<ScaleDesc> sd;
    for (size_t i = 0; i < hs.size(); ++i) {
        mg_hierarchy* H = hs[i];
        Level& L0 = H->lev[0];
        SweepArgs<double> a{};
        a.nx = L0.nx;
        a.ny = L0.ny;
        a.nz = L0.nz;
        a.px = H->px;
        a.py = H->py;
        a.pz = H->pz;
        a.h2 = L0.h * L0.h;
        a.phi_in = L0.d.phi;
        a.phi_out = L0.phi2_d;
        a.f = L0.d.f;
        a.rho = H->rho.rho;
        a.b0c = H->rho.b0c;
        a.b0e = H->rho.b0e;
        a.partials = H->partials;
        a.corr = L0.s.phi;
        a.r32 = L0.s.f;
        a.scales = H->scal + kSlotScale * kReduceWidth;
        const int cfg = sweep_config_for(L0.nx, L0.ny, L0.nz, true);
        args.push_back(a);
        cfgs.push_back(cfg);
        rd.push_back(ReduceDesc{H->partials, sweep_tiles(L0.nx, L0.ny, L0.nz, cfg), H->scal + kSlotRes * kReduceWidth,
                                gather + i * kReduceWidth});
        sd.push_back(ScaleDesc{H->scal + kSlotRes * kReduceWidth, H->scal + kSlotScale * kReduceWidth, (double)L0.N});
    }
    int rc = launch_group<double>(args, cfgs, true, kInCorrect, kOpRefine, S, st);
    if (rc) return rc;
    for (auto* H : hs) std::swap(H->lev[0].d.phi, H->lev[0].phi2_d);
    void* dd = nullptr;
    rc = S.push(rd.data(), rd.size() * sizeof(ReduceDesc), st, &dd);
    if (rc) return rc;
    BHIP(launch_reduce_multi((const ReduceDesc*)dd, (int)rd.size(), st));
    rc = S.push(sd.data(), sd.size() * sizeof(ScaleDesc), st, &dd);
    if (rc) return rc;
    BHIP(launch_next_scale_multi((const ScaleDesc*)dd, (int)sd.size(), st));
    return MG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// jobs
// ---------------------------------------------------------------------------
bool batchable(const mg_hierarchy* H) {
    const Level& L0 = H->lev[0];
    if (H->outflow) return false;      // outflow sides: solved one by one (mac_project)
    if (H->boxes_on) return false;     // multi-box finest level: solved one by one
    if (H->p.pre_sweeps < 1 || H->nlev < 2 || !sweep_fusable<double>(L0.nx, L0.ny, L0.nz)) return false;
    if (H->p.precision == MG_FP64) return true;
    // mixed precision: every FP32 level above the one-workgroup bottom is a
    // fused-sweep level (the batched FP32 cycle has no per-cell kernels), and
    // every prolongation is folded into a post-sweep
    if (H->p.post_sweeps < 1) return false;
    const int b = bottom_start<float>(H);
    if (b <= 0) return false;
    for (int l = 0; l < b; ++l)
        if (!sweep_fusable<float>(H->lev[l].nx, H->lev[l].ny, H->lev[l].nz)) return false;
    return true;
}

static void fail_job(Job& j, int status) {
    j.st.status = status;
    j.status = status;
    j.stage = Job::kDone;
}

namespace {

double steady_seconds() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr size_t kArenaMin = (size_t)1 << 20;
constexpr size_t kMaxRoundGraphs = 8;
constexpr size_t kMaxSeenKeys = 16;

template <typename D>
int push_table(Staging& S, const std::vector<D>& v, hipStream_t st, const D** out) {
    void* dd = nullptr;
    int rc = S.push(v.data(), v.size() * sizeof(D), st, &dd);
    *out = (const D*)dd;
    return rc;
}

// Every phi buffer pointer of H's levels (FP64 pair, FP32 pair per level).
void phi_state(const mg_hierarchy* H, std::vector<void*>& out) {
    for (int l = 0; l < H->nlev; ++l) {
        const Level& L = H->lev[l];
        out.push_back(L.d.phi);
        out.push_back(L.phi2_d);
        out.push_back(L.s.phi);
        out.push_back(L.phi2_s);
    }
}

void set_phi_state(mg_hierarchy* H, const std::vector<void*>& in, size_t& at) {
    for (int l = 0; l < H->nlev; ++l) {
        Level& L = H->lev[l];
        L.d.phi = (double*)in[at++];
        L.phi2_d = (double*)in[at++];
        L.s.phi = (float*)in[at++];
        L.phi2_s = (float*)in[at++];
    }
}

// Everything an iteration's launches bake in: the hierarchies in order, their
// shapes, settings, coefficient sources and current phi buffers, the tile
// choices and the gathered-row block.
std::vector<uintptr_t> round_key(const std::vector<mg_hierarchy*>& h64, const std::vector<int>& pre_done,
                                 const std::vector<mg_hierarchy*>& hm, const double* gather) {
    std::vector<uintptr_t> k;
    k.push_back((uintptr_t)sweep_tune_epoch());
    k.push_back((uintptr_t)gather);
    auto one = [&k](const mg_hierarchy* H, uintptr_t tag) {
        k.push_back(tag);
        k.push_back((uintptr_t)H);
        k.push_back((uintptr_t)H->ws);
        for (int d = 0; d < 3; ++d) k.push_back((uintptr_t)H->p.n[d]);
        k.push_back((uintptr_t)H->nlev);
        k.push_back((uintptr_t)H->p.pre_sweeps);
        k.push_back((uintptr_t)H->p.post_sweeps);
        k.push_back((uintptr_t)inner_cycles_of(H->p));
        k.push_back((uintptr_t)H->bottom_on);
        k.push_back((uintptr_t)H->rho.rho);
        k.push_back((uintptr_t)H->rho.b0c);
        k.push_back((uintptr_t)H->rho.b0e);
        k.push_back((uintptr_t)H->rho32_on);
        std::vector<void*> ph;
        phi_state(H, ph);
        for (void* q : ph) k.push_back((uintptr_t)q);
    };
    for (size_t i = 0; i < h64.size(); ++i) one(h64[i], 0x100 + (uintptr_t)pre_done[i]);
    for (auto* H : hm) one(H, 0x200);
    return k;
}

}  // namespace

int Engine::ensure_gather(int rows) {
    if (rows <= grows) return MG_OK;
    const int want = std::max(rows, std::max(64, 2 * grows));
    drop_graphs();                       // captured rounds bake in the old block
    if (gdev) hipFree(gdev);
    if (ghost) hipHostFree(ghost);
    gdev = nullptr;
    ghost = nullptr;
    grows = 0;
    if (hipMalloc((void**)&gdev, (size_t)want * kReduceWidth * sizeof(double)) != hipSuccess) {
        gdev = nullptr;
        set_error("allocation of the gathered norm block failed");
        return MG_ERR_OOM;
    }
    if (hipHostMalloc((void**)&ghost, (size_t)want * kReduceWidth * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
        ghost = nullptr;
        set_error("allocation of the host norm block failed");
        return MG_ERR_OOM;
    }
    grows = want;
    return MG_OK;
}

void Engine::drop_graphs() {
    for (auto& g : graphs) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        g.arena.release();
    }
    graphs.clear();
    seen.clear();
}

void Engine::release() {
    drop_graphs();
    if (gdev) hipFree(gdev);
    if (ghost) hipHostFree(ghost);
    gdev = nullptr;
    ghost = nullptr;
    grows = 0;
    if (gs) hipStreamDestroy(gs);
    if (gev) hipEventDestroy(gev);
    gs = nullptr;
    gev = nullptr;
    staging.release();
}

// Coefficients, right-hand side, compatibility and norm of f for new jobs,
// batched over all of them.
int Engine::setup_new(std::vector<Job*>& fresh, hipStream_t st) {
    if (fresh.empty()) return MG_OK;
    int rc = ensure_gather((int)fresh.size());
    if (rc) return rc;
    std::vector<CoeffDesc> cd;
    std::vector<ReduceDesc> rd;
    std::vector<CoarseDesc> co_lds, co_glb;
    std::vector<EltDesc> f32;
    int cblocks = 0, f32blocks = 0, maxlev = 0;
    for (size_t q = 0; q < fresh.size(); ++q) {
        Job* j = fresh[q];
        mg_hierarchy* H = j->H;
        std::memset(&j->st, 0, sizeof j->st);
        j->st.nlevels = H->nlev;
        j->gslot = -1;
        for (int l = 0; l < H->nlev; ++l) {       // the buffers as laid out (the values do not depend on it)
            Level& L = H->lev[l];
            L.d.phi = L.phi_home_d[0];
            L.phi2_d = L.phi_home_d[1];
            L.s.phi = L.phi_home_s[0];
            L.phi2_s = L.phi_home_s[1];
        }
        const mg_problem& p = j->pr;
        const double* rho_src = p.rho;
        if (((uintptr_t)p.rho & 15) != 0) {       // the fused sweeps read rho as 16-byte pairs
            BHIP(launch_copy(H->rho_own, p.rho, H->lev[0].N, st));
            rho_src = H->rho_own;
        }
        H->rho = RhoArgs{rho_src, p.beta0_cc, p.beta0_edge, H->px, H->py, H->pz};
        H->rho32_on = false;
        Level& L0 = H->lev[0];
        int g[3];
        const int nb = coeff_grid(Shape{L0.nx, L0.ny, L0.nz}, g);
        cd.push_back(CoeffDesc{L0.nx, L0.ny, L0.nz, H->px, H->py, H->pz, L0.h, p.rho, p.beta0_cc, p.beta0_edge, p.S,
                               p.u, p.v, p.w, nullptr, L0.d.bx, L0.d.by, L0.d.bz, L0.d.f, H->partials, g[0], g[1],
                               g[2], cblocks});
        cblocks += nb;
        rd.push_back(ReduceDesc{H->partials, nb, H->scal + kSlotRhs * kReduceWidth, gdev + q * kReduceWidth});
        maxlev = std::max(maxlev, H->nlev);
        Level& Lc = H->lev[H->nlev - 1];
        const CoarseDesc c{Lc.nx, Lc.ny, Lc.nz, Lc.h, Lc.d.bx, Lc.d.by, Lc.d.bz, H->minv, H->singular ? 1 : 0};
        (coarse_setup_in_lds(Lc.N) ? co_lds : co_glb).push_back(c);
        if (H->p.precision == MG_MIXED) {
            // FP32 coefficient mirrors of the stored levels (the finest FP32
            // level recomputes its coefficients from an FP32 copy of rho)
            for (int l = 1; l < H->nlev; ++l) {
                Level& L = H->lev[l];
                const double* src[3] = {L.d.bx, L.d.by, L.d.bz};
                float* dst[3] = {L.s.bx, L.s.by, L.s.bz};
                for (int a = 0; a < 3; ++a) {
                    f32.push_back(EltDesc{kEltToF32, f32blocks, L.N, src[a], dst[a], 0.0});
                    f32blocks += elt_blocks(L.N);
                }
            }
        }
    }
    const CoeffDesc* dcd = nullptr;
    if ((rc = push_table(staging, cd, st, &dcd))) return rc;
    BHIP(launch_coeff_rhs_multi(dcd, (int)cd.size(), cblocks, st));
    const ReduceDesc* drd = nullptr;
    if ((rc = push_table(staging, rd, st, &drd))) return rc;
    BHIP(launch_reduce_multi(drd, (int)rd.size(), st));
    for (int l = 0; l + 1 < maxlev; ++l) {      // coarse coefficients, one launch per depth
        std::vector<AvgDesc> av;
        int ab = 0;
        for (Job* j : fresh) {
            mg_hierarchy* H = j->H;
            if (l + 1 >= H->nlev) continue;
            Level& F = H->lev[l];
            Level& C = H->lev[l + 1];
            av.push_back(AvgDesc{F.nx, F.ny, F.nz, F.d.bx, F.d.by, F.d.bz, C.d.bx, C.d.by, C.d.bz, ab});
            ab += cell_blocks(C.N);
        }
        const AvgDesc* dav = nullptr;
        if ((rc = push_table(staging, av, st, &dav))) return rc;
        BHIP(launch_avg_coeff_multi(dav, (int)av.size(), ab, st));
    }
    for (int lds = 0; lds < 2; ++lds) {
        std::vector<CoarseDesc>& v = lds ? co_lds : co_glb;
        if (v.empty()) continue;
        const CoarseDesc* dco = nullptr;
        if ((rc = push_table(staging, v, st, &dco))) return rc;
        BHIP(launch_coarse_setup_multi(dco, (int)v.size(), lds == 1, st));
    }
    if (!f32.empty()) {
        const EltDesc* de = nullptr;
        if ((rc = push_table(staging, f32, st, &de))) return rc;
        BHIP(launch_elt_multi(de, (int)f32.size(), f32blocks, st));
    }
    BHIP(hipMemcpyAsync(ghost, gdev, fresh.size() * kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, st));
    BHIP(hipStreamSynchronize(st));
    staging.off = 0;
    for (Job* j : fresh) j->H->coeffs_valid = true;

    // compatibility and mean removal
    std::vector<Job*> norm;
    std::vector<RowDesc> nd;
    std::vector<ReduceDesc> nr;
    std::vector<EltDesc> el;
    int nblocks = 0, eblocks = 0;
    for (size_t q = 0; q < fresh.size(); ++q) {
        Job* j = fresh[q];
        mg_hierarchy* H = j->H;
        const double* row = ghost + q * kReduceWidth;
        const double sf = row[0], saf = row[1], bad = row[2], nonfin = row[3];
        j->st.sum_f = sf;
        j->st.sum_abs_f = saf;
        if (nonfin > 0.0 || !std::isfinite(sf) || !std::isfinite(saf)) {
            fail_job(*j, MG_ERR_NONFINITE);
            continue;
        }
        if (bad > 0.0) {
            fail_job(*j, MG_ERR_INVALID_ARG);
            continue;
        }
        if (std::fabs(sf) > 1e-8 * saf) {
            fail_job(*j, MG_ERR_INCOMPATIBLE_RHS);
            continue;
        }
        Level& L0 = H->lev[0];
        if (saf == 0.0) {
            el.push_back(EltDesc{kEltFill, eblocks, L0.N, nullptr, L0.d.phi, 0.0});
            eblocks += elt_blocks(L0.N);
            j->st.hist_len = 1;
            j->st.resid_hist[0] = 0.0;
            j->status = MG_OK;
            j->stage = Job::kFinish;
            continue;
        }
        const double mean = sf / (double)L0.N;
        j->st.mean_removed = mean;
        const int rb = row_blocks(L0.N);
        nd.push_back(RowDesc{L0.N, L0.d.f, mean, H->partials, rb, nblocks});
        nblocks += rb;
        nr.push_back(ReduceDesc{H->partials, rb, H->scal + kSlotNorm * kReduceWidth, gdev + norm.size() * kReduceWidth});
        norm.push_back(j);
    }
    if (!nd.empty()) {
        const RowDesc* dnd = nullptr;
        if ((rc = push_table(staging, nd, st, &dnd))) return rc;
        BHIP(launch_shift_norm_multi(dnd, (int)nd.size(), nblocks, st));
        const ReduceDesc* dnr = nullptr;
        if ((rc = push_table(staging, nr, st, &dnr))) return rc;
        BHIP(launch_reduce_multi(dnr, (int)nr.size(), st));
        BHIP(hipMemcpyAsync(ghost, gdev, norm.size() * kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, st));
        BHIP(hipStreamSynchronize(st));
        staging.off = 0;
    }
    for (size_t q = 0; q < norm.size(); ++q) {
        Job* j = norm[q];
        mg_hierarchy* H = j->H;
        Level& L0 = H->lev[0];
        j->fnorm = std::sqrt(ghost[q * kReduceWidth]);
        j->st.norm_f = j->fnorm;
        el.push_back(EltDesc{kEltFill, eblocks, L0.N, nullptr, L0.d.phi, 0.0});
        eblocks += elt_blocks(L0.N);
        if (j->fnorm == 0.0) {
            j->status = MG_OK;
            j->stage = Job::kFinish;
            continue;
        }
        j->cycles = 0;
        j->rel = 1.0;
        j->st.resid_hist[0] = 1.0;
        j->st.hist_len = 1;
        if (H->p.precision == MG_MIXED) {
            // FP32 rho for the finest FP32 sweeps; FP32 residual = s0 f while
            // phi = 0; both device scales = s0
            const double s0 = residual_scale(j->fnorm, L0.N);
            el.push_back(EltDesc{kEltToF32, eblocks, L0.N, H->rho.rho, H->rho32, 0.0});
            eblocks += elt_blocks(L0.N);
            el.push_back(EltDesc{kEltScaleToF32, eblocks, L0.N, L0.d.f, L0.s.f, s0});
            eblocks += elt_blocks(L0.N);
            el.push_back(EltDesc{kEltFill, eblocks, 2, nullptr, H->scal + kSlotScale * kReduceWidth, s0});
            eblocks += elt_blocks(2);
            H->rho32_on = true;
        }
        j->status = MG_ERR_NOT_CONVERGED;
        j->stage = (H->p.rtol >= 1.0) ? Job::kFinish : Job::kSolve;
        if (H->p.rtol >= 1.0) j->status = MG_OK;
    }
    if (!el.empty()) {
        const EltDesc* de = nullptr;
        if ((rc = push_table(staging, el, st, &de))) return rc;
        BHIP(launch_elt_multi(de, (int)el.size(), eblocks, st));
    }
    return MG_OK;
}

// The launches of one iteration: FP64 problems one V-cycle (pre_done[i]
// first pre-sweeps already taken from the last speculative sweep) and the
// next speculative sweep with its residual norm, rows 0.. of the gathered
// block; mixed problems their FP32 V-cycles (the first from zero) and the
// FP64 refinement, rows after those.
static int enqueue_iteration(std::vector<mg_hierarchy*>& h64, const std::vector<int>& pre_done,
                             std::vector<mg_hierarchy*>& hm, double* gather, Staging& S, hipStream_t st) {
    if (!h64.empty()) {
        int rc = multi_vcycle(h64, pre_done, S, st);
        if (rc) return rc;
        rc = multi_norm_sweep(h64, gather, S, st);
        if (rc) return rc;
    }
    if (!hm.empty()) {
        // each problem's inner_cycles FP32 V-cycles: the first from zero
        int rc = multi_vcycle_f32(hm, S, st, true);
        if (rc) return rc;
        for (int c = 1;; ++c) {
            std::vector<mg_hierarchy*> more;
            for (mg_hierarchy* H : hm)
                if (inner_cycles_of(H->p) > c) more.push_back(H);
            if (more.empty()) break;
            rc = multi_vcycle_f32(more, S, st, false);
            if (rc) return rc;
        }
        rc = multi_refine(hm, gather + h64.size() * kReduceWidth, S, st);
        if (rc) return rc;
    }
    return MG_OK;
}

// One round: stop tests for solving jobs (their last iteration's norm rows
// are on the host), one iteration for the rest, then the velocity
// correction of every job that finished.
int Engine::round(std::vector<Job*>& jobs, hipStream_t st) {
    int rc = ensure_gather((int)jobs.size() + 2);
    if (rc) return rc;
    std::vector<mg_hierarchy*> run64, runm;
    std::vector<Job*> jrun64, jrunm;
    std::vector<int> pre_done;
    for (Job* j : jobs) {
        if (j->stage != Job::kSolve) continue;
        mg_hierarchy* H = j->H;
        const bool mixed = H->p.precision == MG_MIXED;
        int pd = 0;
        if (j->cycles > 0) {
            const double* r = j->row;
            j->rel = std::sqrt(r[0]) / j->fnorm;
            if (j->cycles < MG_HIST_MAX) {
                j->st.resid_hist[j->cycles] = j->rel;
                j->st.hist_len = j->cycles + 1;
            }
            if (r[3] > 0.0 || !std::isfinite(j->rel)) {
                fail_job(*j, MG_ERR_NONFINITE);
                continue;
            }
            if (j->rel <= H->p.rtol) {
                j->status = MG_OK;
                j->stage = Job::kFinish;
                continue;
            }
            if (j->cycles >= H->p.max_cycles) {
                j->status = MG_ERR_NOT_CONVERGED;
                j->stage = Job::kFinish;
                continue;
            }
            if (!mixed) {
                std::swap(H->lev[0].d.phi, H->lev[0].phi2_d);   // keep the speculative sweep
                pd = 1;
            }
        } else if (H->p.max_cycles == 0) {
            j->stage = Job::kFinish;
            continue;
        }
        if (mixed) {
            runm.push_back(H);
            jrunm.push_back(j);
        } else {
            run64.push_back(H);
            jrun64.push_back(j);
            pre_done.push_back(pd);
        }
    }
    for (size_t i = 0; i < jrun64.size(); ++i) jrun64[i]->gslot = (int)i;
    for (size_t i = 0; i < jrunm.size(); ++i) jrunm[i]->gslot = (int)(jrun64.size() + i);
    const size_t nrun = jrun64.size() + jrunm.size();
    const double t_round = steady_seconds();
    for (Job* j : jrun64)
        if (j->cycles == 0) j->t_iter0 = t_round;
    for (Job* j : jrunm)
        if (j->cycles == 0) j->t_iter0 = t_round;
    if (nrun > 0) {
        rc = iterate(run64, pre_done, runm, st);
        if (rc) return rc;
        for (Job* j : jrun64) ++j->cycles;
        for (Job* j : jrunm) ++j->cycles;
    }
    // finish: mean removal of phi and the velocity correction, batched; the
    // sums land in the gathered rows after the iteration's
    std::vector<Job*> fin;
    for (Job* j : jobs)
        if (j->stage == Job::kFinish) fin.push_back(j);
    if (!fin.empty()) {
        std::vector<RowDesc> sd;
        std::vector<ReduceDesc> rd;
        std::vector<CorrectDesc> cd;
        int sb = 0, cb = 0;
        for (size_t q = 0; q < fin.size(); ++q) {
            mg_hierarchy* H = fin[q]->H;
            const mg_problem& p = fin[q]->pr;
            Level& L0 = H->lev[0];
            const int rb = row_blocks(L0.N);
            sd.push_back(RowDesc{L0.N, L0.d.phi, 0.0, H->partials, rb, sb});
            sb += rb;
            rd.push_back(ReduceDesc{H->partials, rb, H->scal + kSlotPhi * kReduceWidth,
                                    gdev + (nrun + q) * kReduceWidth});
            cd.push_back(CorrectDesc{L0.nx, L0.ny, L0.nz, H->px, H->py, H->pz, L0.h, p.beta0_cc, p.beta0_edge, L0.d.bx,
                                     L0.d.by, L0.d.bz, L0.d.phi, H->scal + kSlotPhi * kReduceWidth, p.u, p.v, p.w,
                                     p.phi, cb});
            cb += cell_blocks(L0.N);
        }
        const RowDesc* dsd = nullptr;
        if ((rc = push_table(staging, sd, st, &dsd))) return rc;
        BHIP(launch_sum_multi(dsd, (int)sd.size(), sb, st));
        const ReduceDesc* drd = nullptr;
        if ((rc = push_table(staging, rd, st, &drd))) return rc;
        BHIP(launch_reduce_multi(drd, (int)rd.size(), st));
        const CorrectDesc* dcd = nullptr;
        if ((rc = push_table(staging, cd, st, &dcd))) return rc;
        BHIP(launch_correct_multi(dcd, (int)cd.size(), cb, st));
    }
    const size_t rows = nrun + fin.size();
    if (rows > 0)
        BHIP(hipMemcpyAsync(ghost, gdev, rows * kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, st));
    BHIP(hipStreamSynchronize(st));
    staging.off = 0;
    const double t_end = steady_seconds();
    for (Job* j : jrun64) {
        std::memcpy(j->row, ghost + (size_t)j->gslot * kReduceWidth, sizeof j->row);
        j->t_iter1 = t_end;
    }
    for (Job* j : jrunm) {
        std::memcpy(j->row, ghost + (size_t)j->gslot * kReduceWidth, sizeof j->row);
        j->t_iter1 = t_end;
    }
    for (size_t q = 0; q < fin.size(); ++q) {
        Job* j = fin[q];
        mg_hierarchy* H = j->H;
        j->st.phi_mean = ghost[(nrun + q) * kReduceWidth] / (double)H->lev[0].N;
        j->st.rel_resid0 = j->st.resid_hist[0];
        j->st.ms_smooth = j->cycles > 0 ? (j->t_iter1 - j->t_iter0) * 1e3 : 0.0;
        j->st.cycles = j->cycles;
        j->st.rel_resid = j->cycles > 0 ? j->rel : j->st.resid_hist[0];
        if (j->st.hist_len == 1 && j->st.resid_hist[0] == 0.0) j->st.rel_resid = 0.0;
        j->st.bytes_model = model_bytes(H->p, j->cycles, H->p.precision == MG_MIXED);
        j->st.status = j->status;
        j->stage = Job::kDone;
        H->rho = RhoArgs{};
        H->rho32_on = false;
    }
    return MG_OK;
}

// One iteration for the running sets: replay the captured graph of this
// exact work, capture it (graph_mode), or launch it eagerly on `st`.
int Engine::iterate(std::vector<mg_hierarchy*>& h64, const std::vector<int>& pre_done,
                    std::vector<mg_hierarchy*>& hm, hipStream_t st) {
    std::vector<uintptr_t> key;
    RoundGraph* g = nullptr;
    bool capture = false;
    if (graph_mode > 0) {
        key = round_key(h64, pre_done, hm, gdev);
        for (auto& c : graphs)
            if (c.exec && c.key == key) g = &c;
        if (!g) {
            if (graph_mode == 1) {
                capture = true;
            } else {
                for (auto& k : seen)
                    if (k == key) capture = true;
                if (!capture) {
                    if (seen.size() >= kMaxSeenKeys) seen.erase(seen.begin());
                    seen.push_back(key);
                }
            }
        }
    }
    if (!g && !capture) {
        ++eager;
        return enqueue_iteration(h64, pre_done, hm, gdev, staging, st);
    }
    if (!gs) {
        BHIP(hipStreamCreateWithFlags(&gs, hipStreamNonBlocking));
        BHIP(hipEventCreateWithFlags(&gev, hipEventDisableTiming));
    }
    // the graph runs on the engine's own stream, after the caller's earlier work
    BHIP(hipEventRecord(gev, st));
    BHIP(hipStreamWaitEvent(gs, gev, 0));
    if (g) {
        size_t at = 0;
        for (auto* H : h64) set_phi_state(H, g->post, at);
        for (auto* H : hm) set_phi_state(H, g->post, at);
        ++replays;
    } else {
        std::vector<void*> before;
        for (auto* H : h64) phi_state(H, before);
        for (auto* H : hm) phi_state(H, before);
        size_t cap = kArenaMin;
        RoundGraph fresh;
        for (int attempt = 0;; ++attempt) {
            int rc = fresh.arena.init(cap);
            if (rc) {
                fresh.arena.release();
                set_error("allocation of a round's descriptor arena failed");
                return rc;
            }
            staging.rec = &fresh.arena;
            hipError_t e = hipStreamBeginCapture(gs, hipStreamCaptureModeRelaxed);
            if (e != hipSuccess) {
                staging.rec = nullptr;
                fresh.arena.release();
                return hip_fail(e, "hipStreamBeginCapture", __LINE__);
            }
            rc = enqueue_iteration(h64, pre_done, hm, gdev, staging, gs);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(gs, &graph);
            staging.rec = nullptr;
            const bool overflow = fresh.arena.overflow;
            const size_t used = fresh.arena.off;
            if (rc || e != hipSuccess || overflow) {
                if (graph) hipGraphDestroy(graph);
                size_t at = 0;                    // back to the state before the capture
                for (auto* H : h64) set_phi_state(H, before, at);
                for (auto* H : hm) set_phi_state(H, before, at);
                fresh.arena.release();
                if (rc) return rc;
                if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __LINE__);
                if (attempt >= 3) {
                    set_error("descriptor arena kept overflowing");
                    return MG_ERR_OOM;
                }
                cap = std::max(2 * cap, used + kArenaMin);
                continue;
            }
            e = hipGraphInstantiate(&fresh.exec, graph, nullptr, nullptr, 0);
            hipGraphDestroy(graph);
            if (e != hipSuccess) {
                fresh.exec = nullptr;
                size_t at = 0;
                for (auto* H : h64) set_phi_state(H, before, at);
                for (auto* H : hm) set_phi_state(H, before, at);
                fresh.arena.release();
                return hip_fail(e, "hipGraphInstantiate", __LINE__);
            }
            break;
        }
        fresh.key = key;
        for (auto* H : h64) phi_state(H, fresh.post);
        for (auto* H : hm) phi_state(H, fresh.post);
        // the tables, once (the pinned bytes never change afterwards)
        BHIP(hipMemcpyAsync(fresh.arena.dev, fresh.arena.host, fresh.arena.off, hipMemcpyHostToDevice, gs));
        if (graphs.size() >= kMaxRoundGraphs) {        // least recently used out (its work is complete)
            size_t lru = 0;
            for (size_t i = 1; i < graphs.size(); ++i)
                if (graphs[i].used < graphs[lru].used) lru = i;
            if (graphs[lru].exec) hipGraphExecDestroy(graphs[lru].exec);
            graphs[lru].arena.release();
            graphs.erase(graphs.begin() + lru);
        }
        graphs.push_back(std::move(fresh));
        g = &graphs.back();
        ++captures;
    }
    g->used = ++clock;
    BHIP(hipGraphLaunch(g->exec, gs));
    BHIP(hipEventRecord(gev, gs));
    BHIP(hipStreamWaitEvent(st, gev, 0));
    return MG_OK;
}

}  // namespace mg
