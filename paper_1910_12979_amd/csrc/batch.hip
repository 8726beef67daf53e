// Batched execution of many independent projections.
//
// Every problem keeps its own hierarchy and goes through exactly the
// sequence of kernels a single mac_project would run on it (same kernel
// bodies, same per-problem tile geometry and reduction order), so its result
// is bit-identical to the single-problem result.  What is shared is the
// launch: at every step of the V-cycle one launch covers that step for all
// active problems (their tiles or cells concatenated, a descriptor table
// telling each workgroup which problem it belongs to).  Problems stop
// independently; the set of active problems is revisited once per V-cycle,
// which is also where the serving loop admits new requests.
#include <hip/hip_runtime.h>

#include <algorithm>
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
    return (c.tx == 32 && c.ty == 8) || (c.tx == 64 && c.ty == 8) || (c.tx == 32 && c.ty == 4);
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
        std::vector<int> prefix(1, 0);
        for (Item* it : kv.second) {
            SweepArgs<double> a = sweep_args(it->H, it->l);
            sweep_geometry(a, cfg);
            descs.push_back(a);
            prefix.push_back(prefix.back() + sweep_tiles(a.nx, a.ny, a.nz, cfg));
        }
        void* dd = nullptr;
        void* dp = nullptr;
        int rc = S.push(descs.data(), descs.size() * sizeof(SweepArgs<double>), st, &dd);
        if (rc) return rc;
        rc = S.push(prefix.data(), prefix.size() * sizeof(int), st, &dp);
        if (rc) return rc;
        BHIP(launch_sweep_multi<double>((const SweepArgs<double>*)dd, (const int*)dp, (int)descs.size(), prefix.back(),
                                        use_rho, in_mode, op, cfg, st));
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
        for (Item* it : small) {
            if (it->nsweeps == 0) continue;
            sm.push_back(it);
            if (first == kInProlong) pro.push_back(it);
            if (first == kInZero) BHIP(launch_fill<double>(it->H->lev[it->l].d.phi, it->H->lev[it->l].N, 0.0, st));
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
// current finest-level phi; the reduced row lands in host[kSlotRes].
int multi_norm_sweep(std::vector<mg_hierarchy*>& hs, Staging& S, hipStream_t st) {
    if (hs.empty()) return MG_OK;
    std::vector<Item> grp;
    for (auto* H : hs) grp.push_back(Item{H, 0, 1});
    int rc = launch_fused(grp, true, kInPlain, kOpSweepNorm, S, st);
    if (rc) return rc;
    std::vector<ReduceDesc> rd;
    for (auto* H : hs) {
        Level& L0 = H->lev[0];
        ReduceDesc r;
        r.partials = H->partials;
        r.nparts = sweep_tiles(L0.nx, L0.ny, L0.nz, sweep_config_for(L0.nx, L0.ny, L0.nz, true));
        r.out = H->scal + kSlotRes * kReduceWidth;
        rd.push_back(r);
    }
    void* dd = nullptr;
    rc = S.push(rd.data(), rd.size() * sizeof(ReduceDesc), st, &dd);
    if (rc) return rc;
    BHIP(launch_reduce_multi((const ReduceDesc*)dd, (int)rd.size(), st));
    for (auto* H : hs)
        BHIP(hipMemcpyAsync(H->host + kSlotRes * kReduceWidth, H->scal + kSlotRes * kReduceWidth,
                            kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, st));
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
        std::vector<int> prefix(1, 0);
        for (size_t i : kv.second) {
            SweepArgs<T> a = args[i];
            sweep_geometry(a, cfg);
            descs.push_back(a);
            prefix.push_back(prefix.back() + sweep_tiles(a.nx, a.ny, a.nz, cfg));
        }
        void* dd = nullptr;
        void* dp = nullptr;
        int rc = S.push(descs.data(), descs.size() * sizeof(SweepArgs<T>), st, &dd);
        if (rc) return rc;
        rc = S.push(prefix.data(), prefix.size() * sizeof(int), st, &dp);
        if (rc) return rc;
        BHIP(launch_sweep_multi<T>((const SweepArgs<T>*)dd, (const int*)dp, (int)descs.size(), prefix.back(), use_rho,
                                   in_mode, op, cfg, st));
    }
    return MG_OK;
}

// FP32 V-cycle from zero on every problem (all of whose levels above the
// bottom are fused-sweep levels), the batched form of vcycle<float> with a
// zero start.
int multi_vcycle_f32(std::vector<mg_hierarchy*>& hs, Staging& S, hipStream_t st) {
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
        int rc = sweeps(l, false, kInZero);
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
// residual for the next cycle, norm rows reduced, scales advanced, norm row
// copied to pinned host memory.
int multi_refine(std::vector<mg_hierarchy*>& hs, Staging& S, hipStream_t st) {
    std::vector<SweepArgs<double>> args;
    std::vector<int> cfgs;
    std::vector<ReduceDesc> rd;
    std::vector<ScaleDesc> sd;
    for (auto* H : hs) {
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
        rd.push_back(ReduceDesc{H->partials, sweep_tiles(L0.nx, L0.ny, L0.nz, cfg), H->scal + kSlotRes * kReduceWidth});
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
    for (auto* H : hs)
        BHIP(hipMemcpyAsync(H->host + kSlotRes * kReduceWidth, H->scal + kSlotRes * kReduceWidth,
                            kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, st));
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

static void fail_job(Job& j, int status, const char* why) {
    j.st.status = status;
    j.status = status;
    j.stage = Job::kDone;
    (void)why;
}

// Coefficients, right-hand side, compatibility and norm of f for new jobs.
int Engine::setup_new(std::vector<Job*>& fresh, hipStream_t st) {
    if (fresh.empty()) return MG_OK;
    for (Job* j : fresh) {
        mg_hierarchy* H = j->H;
        std::memset(&j->st, 0, sizeof j->st);
        j->st.nlevels = H->nlev;
        const mg_problem& p = j->pr;
        const double* rho_src = p.rho;
        if (((uintptr_t)p.rho & 15) != 0) {
            BHIP(launch_copy(H->rho_own, p.rho, H->lev[0].N, st));
            rho_src = H->rho_own;
        }
        H->rho = RhoArgs{rho_src, p.beta0_cc, p.beta0_edge, H->px, H->py, H->pz};
        int rc = build_coefficients(H, p.rho, p.beta0_cc, p.beta0_edge, p.S, p.u, p.v, p.w, st);
        if (rc) return rc;
        BHIP(hipMemcpyAsync(H->host + kSlotRhs * kReduceWidth, H->scal + kSlotRhs * kReduceWidth,
                            kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    BHIP(hipStreamSynchronize(st));
    staging.off = 0;
    std::vector<Job*> norm;
    for (Job* j : fresh) {
        mg_hierarchy* H = j->H;
        const double* q = H->host + kSlotRhs * kReduceWidth;
        const double sf = q[0], saf = q[1], bad = q[2], nonfin = q[3];
        j->st.sum_f = sf;
        j->st.sum_abs_f = saf;
        if (nonfin > 0.0 || !std::isfinite(sf) || !std::isfinite(saf)) {
            fail_job(*j, MG_ERR_NONFINITE, "non-finite input");
            continue;
        }
        if (bad > 0.0) {
            fail_job(*j, MG_ERR_INVALID_ARG, "rho and beta0 must be positive");
            continue;
        }
        if (std::fabs(sf) > 1e-8 * saf) {
            fail_job(*j, MG_ERR_INCOMPATIBLE_RHS, "incompatible right-hand side");
            continue;
        }
        Level& L0 = H->lev[0];
        if (saf == 0.0) {
            BHIP(launch_fill<double>(L0.d.phi, L0.N, 0.0, st));
            j->st.hist_len = 1;
            j->st.resid_hist[0] = 0.0;
            j->status = MG_OK;
            j->stage = Job::kFinish;
            continue;
        }
        const double mean = sf / (double)L0.N;
        j->st.mean_removed = mean;
        int np = 0;
        BHIP(launch_shift_norm(Shape{L0.nx, L0.ny, L0.nz}, L0.d.f, mean, H->partials, &np, st));
        BHIP(launch_reduce(H->partials, np, H->scal + kSlotNorm * kReduceWidth, st));
        BHIP(hipMemcpyAsync(H->host + kSlotNorm * kReduceWidth, H->scal + kSlotNorm * kReduceWidth,
                            kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, st));
        norm.push_back(j);
    }
    if (norm.empty()) return MG_OK;
    BHIP(hipStreamSynchronize(st));
    for (Job* j : norm) {
        mg_hierarchy* H = j->H;
        Level& L0 = H->lev[0];
        j->fnorm = std::sqrt(H->host[kSlotNorm * kReduceWidth]);
        j->st.norm_f = j->fnorm;
        BHIP(launch_fill<double>(L0.d.phi, L0.N, 0.0, st));
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
            // FP32 rho for the finest FP32 sweeps; FP32 residual = s0 f while phi = 0
            BHIP(launch_coeff_to_f32(H->rho.rho, H->rho32, L0.N, st));
            H->rho32_on = true;
            const double s0 = residual_scale(j->fnorm, L0.N);
            BHIP(launch_scale_to_f32(L0.d.f, L0.s.f, L0.N, s0, st));
            H->host[kSlotScale * kReduceWidth] = s0;
            H->host[kSlotScale * kReduceWidth + 1] = s0;
            BHIP(hipMemcpyAsync(H->scal + kSlotScale * kReduceWidth, H->host + kSlotScale * kReduceWidth,
                                2 * sizeof(double), hipMemcpyHostToDevice, st));
        }
        j->status = MG_ERR_NOT_CONVERGED;
        j->stage = (H->p.rtol >= 1.0) ? Job::kFinish : Job::kSolve;
        if (H->p.rtol >= 1.0) j->status = MG_OK;
    }
    return MG_OK;
}

// One round: stop tests for solving jobs, one V-cycle for the rest, then
// the velocity correction of every job that finished.
int Engine::round(std::vector<Job*>& jobs, hipStream_t st) {
    std::vector<Job*> solving;
    for (Job* j : jobs)
        if (j->stage == Job::kSolve) solving.push_back(j);
    // stop tests: FP64 jobs measure the residual of their last cycle with a
    // speculative first pre-sweep; mixed jobs' last refinement left it on the
    // host already
    std::vector<mg_hierarchy*> tested;
    bool mixed_tested = false;
    for (Job* j : solving)
        if (j->cycles > 0) {
            if (j->H->p.precision == MG_MIXED) mixed_tested = true;
            else tested.push_back(j->H);
        }
    if (!tested.empty()) {
        int rc = multi_norm_sweep(tested, staging, st);
        if (rc) return rc;
    }
    if (!tested.empty() || mixed_tested) {
        BHIP(hipStreamSynchronize(st));
        staging.off = 0;
    }
    std::vector<mg_hierarchy*> run, run_mixed;
    std::vector<int> pre_done;
    for (Job* j : solving) {
        mg_hierarchy* H = j->H;
        const bool mixed = H->p.precision == MG_MIXED;
        int pd = 0;
        if (j->cycles > 0) {
            const double* r = H->host + kSlotRes * kReduceWidth;
            j->rel = std::sqrt(r[0]) / j->fnorm;
            if (j->cycles < MG_HIST_MAX) {
                j->st.resid_hist[j->cycles] = j->rel;
                j->st.hist_len = j->cycles + 1;
            }
            if (r[3] > 0.0 || !std::isfinite(j->rel)) {
                j->status = MG_ERR_NONFINITE;
                fail_job(*j, MG_ERR_NONFINITE, "non-finite residual");
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
            run_mixed.push_back(H);
        } else {
            run.push_back(H);
            pre_done.push_back(pd);
        }
    }
    if (!run.empty()) {
        int rc = multi_vcycle(run, pre_done, staging, st);
        if (rc) return rc;
    }
    if (!run_mixed.empty()) {
        int rc = multi_vcycle_f32(run_mixed, staging, st);
        if (rc) return rc;
        rc = multi_refine(run_mixed, staging, st);
        if (rc) return rc;
    }
    for (Job* j : solving)
        if (j->stage == Job::kSolve) ++j->cycles;
    // finish: mean removal of phi and the velocity correction
    std::vector<Job*> fin;
    for (Job* j : jobs)
        if (j->stage == Job::kFinish) fin.push_back(j);
    for (Job* j : fin) {
        mg_hierarchy* H = j->H;
        Level& L0 = H->lev[0];
        int np = 0;
        BHIP(launch_sum(Shape{L0.nx, L0.ny, L0.nz}, L0.d.phi, H->partials, &np, st));
        BHIP(launch_reduce(H->partials, np, H->scal + kSlotPhi * kReduceWidth, st));
        BHIP(launch_correct(Shape{L0.nx, L0.ny, L0.nz}, H->px, H->py, H->pz, L0.h, j->pr.beta0_cc, j->pr.beta0_edge,
                            L0.d.bx, L0.d.by, L0.d.bz, L0.d.phi, H->scal + kSlotPhi * kReduceWidth, j->pr.u, j->pr.v,
                            j->pr.w, j->pr.phi, st));
        BHIP(hipMemcpyAsync(H->host + kSlotPhi * kReduceWidth, H->scal + kSlotPhi * kReduceWidth,
                            kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    if (!fin.empty()) {
        BHIP(hipStreamSynchronize(st));
        staging.off = 0;
        for (Job* j : fin) {
            mg_hierarchy* H = j->H;
            j->st.phi_mean = H->host[kSlotPhi * kReduceWidth] / (double)H->lev[0].N;
            j->st.cycles = j->cycles;
            j->st.rel_resid = j->cycles > 0 ? j->rel : j->st.resid_hist[0];
            if (j->st.hist_len == 1 && j->st.resid_hist[0] == 0.0) j->st.rel_resid = 0.0;
            j->st.bytes_model = model_bytes(H->p, j->cycles, H->p.precision == MG_MIXED);
            j->st.status = j->status;
            j->stage = Job::kDone;
            H->rho = RhoArgs{};
            H->rho32_on = false;
        }
    }
    return MG_OK;
}

}  // namespace mg
