// Host runtime of the MAC-projection library: hierarchy construction,
// V-cycle driver, FP64 and mixed-precision (FP32 cycle + FP64 iterative
// refinement) solves, velocity correction, and the single-problem C ABI.
//
// Method: the projection of arXiv:1910.12979 (Sec. 2 divergence constraint,
// Sec. 3 multigrid projection).  The multigrid cycle, coarsening rule and
// coarsest solve are spelled out in include/macproj.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <functional>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>

#include "mg_internal.h"
#include "runtime.h"
#include "sweep.h"

namespace mg {

thread_local std::string g_last_error;

void set_error(const std::string& s) { g_last_error = s; }

int hip_fail(hipError_t e, const char* what, int line) {
    char buf[256];
    std::snprintf(buf, sizeof buf, "%s failed (line %d): %s", what, line, hipGetErrorString(e));
    set_error(buf);
    return MG_ERR_HIP;
}

int count_levels(int nx, int ny, int nz) {
    if (nx < 1 || ny < 1 || nz < 1) return 0;
    int n = 1;
    while (nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0 && (long long)nx * ny * nz > kCoarsenMin &&
           n < kMaxLevels) {
        nx /= 2;
        ny /= 2;
        nz /= 2;
        ++n;
    }
    if ((long long)nx * ny * nz > kCoarseMax) return 0;
    return n;
}

void sides_from_bc(const mg_params* p, int side[6]) {
    for (int d = 0; d < 3; ++d) {
        int lo = 1, hi = 1;                        // walls
        switch (p->bc[d]) {
            case MG_BC_PERIODIC: lo = hi = 0; break;
            case MG_BC_OUTFLOW: lo = hi = 2; break;
            case MG_BC_WALL_OUTFLOW: hi = 2; break;
            case MG_BC_OUTFLOW_WALL: lo = 2; break;
            default: break;
        }
        side[2 * d] = lo;
        side[2 * d + 1] = hi;
    }
}

int validate_params(const mg_params* p) {
    if (!p) {
        set_error("null params");
        return MG_ERR_INVALID_ARG;
    }
    if (!(p->dx > 0.0) || !std::isfinite(p->dx)) {
        set_error("dx must be positive and finite");
        return MG_ERR_INVALID_ARG;
    }
    for (int d = 0; d < 3; ++d)
        if (p->bc[d] < MG_BC_PERIODIC || p->bc[d] > MG_BC_OUTFLOW_WALL) {
            set_error("bc must be one of MG_BC_PERIODIC, MG_BC_WALL, MG_BC_OUTFLOW, MG_BC_WALL_OUTFLOW, "
                      "MG_BC_OUTFLOW_WALL");
            return MG_ERR_INVALID_ARG;
        }
    if (p->pre_sweeps < 0 || p->post_sweeps < 0 || p->max_cycles < 0 || p->max_cycles > 100000 ||
        !(p->rtol >= 0.0) || (p->precision != MG_FP64 && p->precision != MG_MIXED) || p->inner_cycles < 0 ||
        p->inner_cycles > 8) {
        set_error("invalid solver controls");
        return MG_ERR_INVALID_ARG;
    }
    if (count_levels(p->n[0], p->n[1], p->n[2]) == 0) {
        set_error("shape not solvable: coarsest level would exceed 512 cells (or n < 1)");
        return MG_ERR_BAD_SIZE;
    }
    return MG_OK;
}

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Walk the workspace layout; with base == nullptr only the size is computed.
size_t layout(mg_hierarchy* H, const mg_params* p, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* ptr = base ? base + off : nullptr;
        off += align_up(bytes);
        return ptr;
    };
    int nl = count_levels(p->n[0], p->n[1], p->n[2]);
    bool mixed = p->precision == MG_MIXED;
    for (int l = 0; l < nl; ++l) {
        size_t N = (size_t)(p->n[0] >> l) * (p->n[1] >> l) * (p->n[2] >> l);
        LevelArrays<double> d;
        d.phi = (double*)take(N * 8);
        d.f = (double*)take(N * 8);
        d.bx = (double*)take(N * 8);
        d.by = (double*)take(N * 8);
        d.bz = (double*)take(N * 8);
        double* phi2_d = (double*)take(N * 8);
        float* phi2_s = nullptr;
        LevelArrays<float> s;
        if (mixed) {
            phi2_s = (float*)take(N * 4);
            s.phi = (float*)take(N * 4);
            s.f = (float*)take(N * 4);
            s.bx = (float*)take(N * 4);
            s.by = (float*)take(N * 4);
            s.bz = (float*)take(N * 4);
        }
        // outflow sides: boundary-face coefficients of the level
        int side[6];
        sides_from_bc(p, side);
        double* bd[6] = {};
        float* bs[6] = {};
        double* dgd = nullptr;
        float* dgs = nullptr;
        for (int q = 0; q < 6; ++q) {
            if (side[q] != 2) continue;
            const size_t nb = bnd_count(q, p->n[0] >> l, p->n[1] >> l, p->n[2] >> l);
            bd[q] = (double*)take(nb * 8);
            if (mixed) bs[q] = (float*)take(nb * 4);
            if (!dgd) {
                dgd = (double*)take(N * 8);
                if (mixed) dgs = (float*)take(N * 4);
            }
        }
        if (H) {
            H->lev[l].d = d;
            H->lev[l].s = s;
            H->lev[l].phi2_d = phi2_d;
            H->lev[l].phi2_s = phi2_s;
            H->lev[l].phi_home_d[0] = d.phi;
            H->lev[l].phi_home_d[1] = phi2_d;
            H->lev[l].phi_home_s[0] = s.phi;
            H->lev[l].phi_home_s[1] = phi2_s;
            H->lev[l].has_bnd = false;
            H->lev[l].dg_d = dgd;
            H->lev[l].dg_s = dgs;
            for (int q = 0; q < 6; ++q) {
                H->lev[l].bnd_d[q] = bd[q];
                H->lev[l].bnd_s[q] = bs[q];
                if (bd[q]) H->lev[l].has_bnd = true;
            }
        }
    }
    size_t Nc = (size_t)(p->n[0] >> (nl - 1)) * (p->n[1] >> (nl - 1)) * (p->n[2] >> (nl - 1));
    double* minv = (double*)take(Nc * Nc * 8);
    size_t rows = 2048;
    for (int c = 0; c < kNumSweepCfg; ++c)
        rows = std::max(rows, (size_t)sweep_tiles(p->n[0], p->n[1], p->n[2], c));
    double* partials = (double*)take(rows * kReduceWidth * 8);
    double* scal = (double*)take(64 * 8);
    double* r64 = nullptr;
    size_t N0 = (size_t)p->n[0] * p->n[1] * p->n[2];
    float* rho32 = nullptr;
    if (mixed) {
        r64 = (double*)take(N0 * 8);
        rho32 = (float*)take(N0 * 4);
    }
    double* rho_own = (double*)take(N0 * 8);
    double* b0c_own = (double*)take((size_t)p->n[2] * 8);
    double* b0e_own = (double*)take((size_t)(p->n[2] + 1) * 8);
    double* w0 = (double*)take((size_t)p->n[2] * 8);
    if (H) {
        H->minv = minv;
        H->partials = partials;
        H->scal = scal;
        H->r64 = r64;
        H->rho32 = rho32;
        H->rho_own = rho_own;
        H->b0c_own = b0c_own;
        H->b0e_own = b0e_own;
        H->w0 = w0;
    }
    return off;
}

}  // namespace

size_t workspace_bytes(const mg_params* p) {
    if (validate_params(p) != MG_OK) return 0;
    return layout(nullptr, p, nullptr);
}

#define HIPCHK(expr)                                    \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #expr, __LINE__); \
    } while (0)

int setup(const mg_params* p, void* workspace, size_t ws_bytes, mg_hierarchy** out) {
    if (!out) {
        set_error("null output handle");
        return MG_ERR_INVALID_ARG;
    }
    *out = nullptr;
    int st = validate_params(p);
    if (st != MG_OK) return st;
    size_t need = layout(nullptr, p, nullptr);
    mg_hierarchy* H = new (std::nothrow) mg_hierarchy();
    if (!H) return MG_ERR_OOM;
    H->p = *p;
    H->px = p->bc[0] == MG_BC_PERIODIC;
    H->py = p->bc[1] == MG_BC_PERIODIC;
    H->pz = p->bc[2] == MG_BC_PERIODIC;
    sides_from_bc(p, H->side);
    H->outflow = false;
    for (int q = 0; q < 6; ++q)
        if (H->side[q] == 2) H->outflow = true;
    H->singular = !H->outflow;
    H->nlev = count_levels(p->n[0], p->n[1], p->n[2]);
    hipGetDevice(&H->device);
    if (workspace) {
        if (ws_bytes < need || ((uintptr_t)workspace % kAlign) != 0) {
            delete H;
            set_error("workspace too small or not 256-byte aligned");
            return MG_ERR_INVALID_ARG;
        }
        H->ws = workspace;
        H->owns_ws = false;
    } else {
        hipError_t e = hipMalloc(&H->ws, need);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete H;
            set_error("hipMalloc of the hierarchy workspace failed");
            return MG_ERR_OOM;
        }
        H->owns_ws = true;
    }
    H->ws_bytes = need;
    layout(H, p, (char*)H->ws);
    for (int l = 0; l < H->nlev; ++l) {
        Level& L = H->lev[l];
        L.nx = p->n[0] >> l;
        L.ny = p->n[1] >> l;
        L.nz = p->n[2] >> l;
        L.N = (size_t)L.nx * L.ny * L.nz;
        L.h = p->dx * (double)(1 << l);
    }
    hipError_t e = hipHostMalloc((void**)&H->host, 64 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        if (H->owns_ws) hipFree(H->ws);
        delete H;
        return hip_fail(e, "hipHostMalloc", __LINE__);
    }
    hipEventCreate(&H->ev0);
    hipEventCreate(&H->ev1);
    hipEventCreate(&H->evs0);
    hipEventCreate(&H->evs1);
    *out = H;
    return MG_OK;
}

// A hierarchy laid out in caller memory without allocating anything: *H is
// reset and filled, ws (device, >= workspace_bytes(p), 256-byte aligned)
// holds every level array, host (64 doubles, any host memory) receives the
// scalar readbacks.  No timing events and no captured graphs: the solve runs
// every cycle as separate launches on the caller's stream.
int setup_static(const mg_params* p, void* ws, size_t ws_bytes, double* host, mg_hierarchy* H) {
    int st = validate_params(p);
    if (st != MG_OK) return st;
    const size_t need = layout(nullptr, p, nullptr);
    if (!ws || !host || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0) {
        set_error("static workspace too small or not 256-byte aligned");
        return MG_ERR_INVALID_ARG;
    }
    *H = mg_hierarchy{};
    H->p = *p;
    H->px = p->bc[0] == MG_BC_PERIODIC;
    H->py = p->bc[1] == MG_BC_PERIODIC;
    H->pz = p->bc[2] == MG_BC_PERIODIC;
    sides_from_bc(p, H->side);
    for (int q = 0; q < 6; ++q)
        if (H->side[q] == 2) H->outflow = true;
    H->singular = !H->outflow;
    H->nlev = count_levels(p->n[0], p->n[1], p->n[2]);
    hipGetDevice(&H->device);
    H->ws = ws;
    H->owns_ws = false;
    H->ws_bytes = need;
    H->graphs_on = false;
    layout(H, p, (char*)ws);
    for (int l = 0; l < H->nlev; ++l) {
        Level& L = H->lev[l];
        L.nx = p->n[0] >> l;
        L.ny = p->n[1] >> l;
        L.nz = p->n[2] >> l;
        L.N = (size_t)L.nx * L.ny * L.nz;
        L.h = p->dx * (double)(1 << l);
    }
    H->host = host;
    return MG_OK;
}

int destroy(mg_hierarchy* H) {
    if (!H) return MG_OK;
    if (H->owns_ws && H->ws) hipFree(H->ws);
    if (H->host) hipHostFree(H->host);
    hipEventDestroy(H->ev0);
    hipEventDestroy(H->ev1);
    hipEventDestroy(H->evs0);
    hipEventDestroy(H->evs1);
    for (auto& g : H->graph)
        if (g.exec) hipGraphExecDestroy(g.exec);
    if (H->gstream) hipStreamDestroy(H->gstream);
    if (H->gev) hipEventDestroy(H->gev);
    if (H->box_mem) hipFree(H->box_mem);
    delete H;
    return MG_OK;
}

static Shape shape_of(const Level& L) { return Shape{L.nx, L.ny, L.nz}; }

// Reduce the partial rows into scal[slot*4 .. slot*4+3].
static int reduce_to(mg_hierarchy* H, int nparts, int slot, hipStream_t st) {
    HIPCHK(launch_reduce(H->partials, nparts, H->scal + slot * kReduceWidth, st));
    return MG_OK;
}

static int read_scalars(mg_hierarchy* H, int first, int count, hipStream_t st) {
    HIPCHK(hipMemcpyAsync(H->host + first, H->scal + first, count * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return MG_OK;
}

// Arguments of the general-boundary kernels for level 0 of H.
static GenArgs gen_args(mg_hierarchy* H, const double* rho, const double* b0c, const double* b0e,
                        const Radial* rad) {
    GenArgs g{};
    Level& L0 = H->lev[0];
    g.nx = L0.nx;
    g.ny = L0.ny;
    g.nz = L0.nz;
    for (int q = 0; q < 6; ++q) {
        g.side[q] = H->side[q];
        g.bnd[q] = L0.bnd_d[q];
    }
    g.h = L0.h;
    g.rho = rho;
    g.b0c = b0c;
    g.b0e = b0e;
    if (rad && rad->prof) {
        g.nr = rad->nr;
        g.dr = rad->dr;
        g.prof = rad->prof;
        g.cx = rad->c[0];
        g.cy = rad->c[1];
        g.cz = rad->c[2];
    }
    g.bx = L0.d.bx;
    g.by = L0.d.by;
    g.bz = L0.d.bz;
    g.f = L0.d.f;
    g.partials = H->partials;
    return g;
}

int build_coefficients(mg_hierarchy* H, const double* rho, const double* b0c, const double* b0e,
                       const double* S, const double* u, const double* v, const double* w,
                       hipStream_t st, const double* w0, const Radial* rad) {
    Level& L0 = H->lev[0];
    int np = 0;
    // level 0 from rho with a plane-parallel beta0 (no outflow side): the
    // first coarse averaging recomputes its coefficients from rho
    const bool plane_rho = !H->outflow && !(rad && rad->prof);
    const bool mixed = H->p.precision == MG_MIXED;
    H->rho32_fresh = false;
    if (H->outflow || (rad && rad->prof)) {
        GenArgs g = gen_args(H, rho, b0c, b0e, rad);
        g.S = S;
        g.u = u;
        g.v = v;
        g.w = w;
        g.w0 = w0;
        HIPCHK(launch_coeff_rhs_gen(g, &np, st));
    } else if (S) {
        // mixed precision: the FP32 copy of rho the FP32 finest-level sweeps
        // read is written on the way
        float* r32 = mixed ? H->rho32 : nullptr;
        HIPCHK(launch_coeff_rhs(shape_of(L0), H->px, H->py, H->pz, L0.h, rho, b0c, b0e, S, u, v, w, L0.d.bx,
                                L0.d.by, L0.d.bz, L0.d.f, H->partials, &np, st, w0, r32));
        H->rho32_fresh = r32 != nullptr;
    } else {
        HIPCHK(launch_coeff(shape_of(L0), H->px, H->py, H->pz, rho, b0c, b0e, L0.d.bx, L0.d.by, L0.d.bz,
                            H->partials, &np, st));
    }
    int rc = reduce_to(H, np, kSlotRhs, st);
    if (rc) return rc;
    // mixed precision: the averaging also writes the FP32 mirrors of every
    // coarse level's coefficients
    for (int l = 0; l + 1 < H->nlev; ++l) {
        Level& F = H->lev[l];
        Level& C = H->lev[l + 1];
        float* const m32[3] = {C.s.bx, C.s.by, C.s.bz};
        if (l == 0 && plane_rho)
            HIPCHK(launch_avg_coeff_rho(shape_of(F), H->px, H->py, H->pz, rho, b0c, b0e, C.d.bx, C.d.by, C.d.bz,
                                        mixed ? m32 : nullptr, st));
        else
            HIPCHK(launch_avg_coeff<double>(shape_of(F), F.d.bx, F.d.by, F.d.bz, C.d.bx, C.d.by, C.d.bz, st,
                                            mixed ? m32 : nullptr));
        if (F.has_bnd) HIPCHK(launch_avg_bnd<double>(shape_of(F), F.bnd64(), C.bnd_d, st));
    }
    Level& Lc = H->lev[H->nlev - 1];
    const Bnd<double> cb = Lc.bnd64();
    HIPCHK(launch_coarse_setup(shape_of(Lc), Lc.h, Lc.d.bx, Lc.d.by, Lc.d.bz, H->minv, st,
                               Lc.has_bnd ? &cb : nullptr, H->singular ? 1 : 0));
    if (mixed) {
        // FP32 coefficient mirrors of level 0 (the coarse ones came with the
        // averaging); a fused finest level with a plane-parallel beta0
        // recomputes its FP32 coefficients from an FP32 copy of rho, so its
        // stored ones are not mirrored
        const bool fused0 = H->rho.rho != nullptr && H->p.pre_sweeps >= 1 && H->nlev > 1 &&
                            sweep_fusable<double>(L0.nx, L0.ny, L0.nz);
        for (int l = 0; l < H->nlev; ++l) {
            Level& L = H->lev[l];
            if (l == 0 && !fused0) {
                HIPCHK(launch_coeff_to_f32(L.d.bx, L.s.bx, L.N, st));
                HIPCHK(launch_coeff_to_f32(L.d.by, L.s.by, L.N, st));
                HIPCHK(launch_coeff_to_f32(L.d.bz, L.s.bz, L.N, st));
            }
            for (int q = 0; q < 6; ++q)
                if (L.bnd_d[q]) HIPCHK(launch_coeff_to_f32(L.bnd_d[q], L.bnd_s[q], bnd_count(q, L.nx, L.ny, L.nz), st));
            if (L.has_bnd) HIPCHK(launch_bnd_diag3<float>(shape_of(L), L.bnd32(), L.dg_s, st));
        }
    }
    for (int l = 0; l < H->nlev; ++l) {
        Level& L = H->lev[l];
        if (L.has_bnd) HIPCHK(launch_bnd_diag3<double>(shape_of(L), L.bnd64(), L.dg_d, st));
    }
    H->coeffs_valid = true;
    return MG_OK;
}

// Sweeps on level l.  `first` selects what the first sweep reads as its
// input: kInPlain (phi as stored), kInZero (phi = 0, nothing read) or
// kInProlong (phi + P phi_{l+1}).  Levels large enough for the fused
// out-of-place sweep ping-pong between the two phi buffers; smaller levels
// use the per-colour kernels in place.
template <typename T>
static int smooth(mg_hierarchy* H, int l, int nsweeps, int first, hipStream_t st) {
    constexpr bool dbl = std::is_same<T, double>::value;
    Level& F = H->lev[l];
    LevelArrays<T>* A;
    T** alt;
    if constexpr (dbl) {
        A = &F.d;
        alt = &F.phi2_d;
    } else {
        A = &F.s;
        alt = &F.phi2_s;
    }
    const T* phic = nullptr;
    if (l + 1 < H->nlev) {
        if constexpr (dbl) phic = H->lev[l + 1].d.phi;
        else phic = H->lev[l + 1].s.phi;
    }
    Shape s = shape_of(F);
    Bnd<T> bnd;
    if constexpr (dbl) bnd = F.bnd64();
    else bnd = F.bnd32();
    if (first == kInProlong && nsweeps == 0) {
        HIPCHK(launch_prolong<T>(s, A->phi, phic, st));
        return MG_OK;
    }
    if (!sweep_fusable<T>(F.nx, F.ny, F.nz)) {
        if (first == kInProlong) HIPCHK(launch_prolong<T>(s, A->phi, phic, st));
        if (first == kInZero) HIPCHK(launch_fill<T>(A->phi, F.N, T(0), st));
        HIPCHK(launch_rbgs<T>(s, F.h, A->phi, A->f, A->bx, A->by, A->bz, nsweeps, st, &bnd));
        return MG_OK;
    }
    // finest level: coefficients from rho (FP64) or its FP32 copy (mixed solve)
    const bool use_rho = l == 0 && (dbl ? H->rho.rho != nullptr : H->rho32_on);
    for (int k = 0; k < nsweeps; ++k) {
        SweepArgs<T> a{};
        a.nx = F.nx;
        a.ny = F.ny;
        a.nz = F.nz;
        a.px = H->px;
        a.py = H->py;
        a.pz = H->pz;
        a.tz = 0;
        a.h2 = (T)(F.h * F.h);
        a.phi_in = A->phi;
        a.phi_out = *alt;
        a.f = A->f;
        a.phic = phic;
        a.bx = A->bx;
        a.by = A->by;
        a.bz = A->bz;
        if constexpr (dbl) a.rho = H->rho.rho;
        else a.rho = H->rho32;
        a.b0c = H->rho.b0c;
        a.b0e = H->rho.b0e;
        a.has_bnd = F.has_bnd ? 1 : 0;
        a.bnd = bnd;
        if constexpr (dbl) a.dg = F.dg_d;
        else a.dg = F.dg_s;
        HIPCHK(launch_sweep<T>(a, use_rho, k == 0 ? first : (int)kInPlain,
                               sweep_config_for(F.nx, F.ny, F.nz, use_rho, dbl, l > 0), st));
        std::swap(A->phi, *alt);
    }
    return MG_OK;
}

// r_l = f_l - L phi_l restricted into f_{l+1}; phi_{l+1} = 0.
template <typename T>
static int resid_restrict(mg_hierarchy* H, int l, hipStream_t st) {
    Level& F = H->lev[l];
    Level& C = H->lev[l + 1];
    Shape s = shape_of(F);
    const Bnd<double> b64 = F.bnd64();
    const Bnd<float> b32 = F.bnd32();
    if constexpr (std::is_same<T, double>::value) {
        const bool rho0 = l == 0 && H->rho.rho;
        if (l == 0 && sweep_fusable<double>(F.nx, F.ny, F.nz)) {
            {   // finest level: the sweep's tiles, coefficients from rho or stored
                SweepArgs<double> a{};
                a.nx = F.nx;
                a.ny = F.ny;
                a.nz = F.nz;
                a.px = H->px;
                a.py = H->py;
                a.pz = H->pz;
                a.h2 = F.h * F.h;
                a.phi_in = F.d.phi;
                a.f = F.d.f;
                a.rho = H->rho.rho;
                a.b0c = H->rho.b0c;
                a.b0e = H->rho.b0e;
                a.bx = F.d.bx;
                a.by = F.d.by;
                a.bz = F.d.bz;
                a.fc = C.d.f;
                a.phic_out = C.d.phi;
                a.has_bnd = F.has_bnd ? 1 : 0;
                a.bnd = b64;
                a.dg = F.dg_d;
                HIPCHK(launch_resid_restrict_tiled(a, rho0, sweep_config_for(F.nx, F.ny, F.nz, rho0), st));
            }
            return MG_OK;
        }
        if (rho0) {
            HIPCHK(launch_resid_restrict_rho(s, F.h, H->rho, F.d.phi, F.d.f, C.d.f, C.d.phi, st, &b64));
            return MG_OK;
        }
        HIPCHK(launch_resid_restrict<double>(s, F.h, F.d.phi, F.d.f, F.d.bx, F.d.by, F.d.bz, C.d.f, C.d.phi, st,
                                             &b64));
    } else {
        if (l == 0 && H->rho32_on) {
            SweepArgs<float> a{};
            a.nx = F.nx;
            a.ny = F.ny;
            a.nz = F.nz;
            a.px = H->px;
            a.py = H->py;
            a.pz = H->pz;
            a.h2 = (float)(F.h * F.h);
            a.phi_in = F.s.phi;
            a.f = F.s.f;
            a.rho = H->rho32;
            a.b0c = H->rho.b0c;
            a.b0e = H->rho.b0e;
            a.fc = C.s.f;
            a.phic_out = C.s.phi;
            a.has_bnd = F.has_bnd ? 1 : 0;
            a.bnd = b32;
            a.dg = F.dg_s;
            HIPCHK(launch_resid_restrict_tiled<float>(a, true, sweep_config_for(F.nx, F.ny, F.nz, true, false), st));
            return MG_OK;
        }
        HIPCHK(launch_resid_restrict<float>(s, F.h, F.s.phi, F.s.f, F.s.bx, F.s.by, F.s.bz, C.s.f, C.s.phi, st,
                                            &b32));
    }
    return MG_OK;
}

template <typename T>
int bottom_start(const mg_hierarchy* H) {
    if (!H->bottom_on) return -1;
    int L = -1;
    for (int l = 1; l + 1 < H->nlev; ++l) {
        const Level& F = H->lev[l];
        if (!sweep_fusable<T>(F.nx, F.ny, F.nz)) {
            L = l;
            break;
        }
    }
    if (L < 0) return -1;
    // the first level from there down whose phi and f, with every coarser
    // level's, fit in the workgroup's LDS (a 24^3 level in FP64 does not:
    // it keeps one launch per step, and the bottom takes 12^3 and below)
    for (int b = L; b + 1 < H->nlev; ++b) {
        if (H->nlev - b > kMaxBottomLevels) continue;
        size_t bytes = 0;
        for (int l = b; l < H->nlev; ++l) bytes += 2 * H->lev[l].N * sizeof(T);
        if (bytes <= kBottomLdsBytes) return b;
    }
    return -1;
}

template <typename T>
void bottom_args(mg_hierarchy* H, int l, BottomArgs<T>& a) {
    constexpr bool dbl = std::is_same<T, double>::value;
    a = BottomArgs<T>{};
    a.nlev = H->nlev - l;
    a.pre = H->p.pre_sweeps;
    a.post = H->p.post_sweeps;
    a.singular = H->singular ? 1 : 0;
    a.minv = H->minv;
    int off = 0;
    for (int b = 0; b < a.nlev; ++b) {
        Level& F = H->lev[l + b];
        const LevelArrays<T>* A;
        if constexpr (dbl) A = &F.d;
        else A = &F.s;
        BottomLevel<T>& v = a.lev[b];
        v.nx = F.nx;
        v.ny = F.ny;
        v.nz = F.nz;
        v.off = off;
        v.h2 = (T)(F.h * F.h);
        v.bx = A->bx;
        v.by = A->by;
        v.bz = A->bz;
        v.has_bnd = F.has_bnd ? 1 : 0;
        if constexpr (dbl) v.bnd = F.bnd64();
        else v.bnd = F.bnd32();
        off += 2 * (int)F.N;
        if (b == 0) {
            a.f = A->f;
            a.phi = A->phi;
        }
    }
}

template int bottom_start<double>(const mg_hierarchy*);
template int bottom_start<float>(const mg_hierarchy*);
template void bottom_args<double>(mg_hierarchy*, int, BottomArgs<double>&);
template void bottom_args<float>(mg_hierarchy*, int, BottomArgs<float>&);

// V-cycle from level l (FP64 or FP32 arrays; the coarsest solve is FP64).
// Coarse levels start from phi = 0; level 0 from its stored phi unless
// zero_start (the mixed solve's correction cycle).
template <typename T>
static int vcycle(mg_hierarchy* H, int l, hipStream_t st, int pre_done = 0, bool zero_start = false) {
    Level& F = H->lev[l];
    if (l > 0 && l == bottom_start<T>(H)) {          // this level and every coarser one in one launch
        BottomArgs<T> a;
        bottom_args<T>(H, l, a);
        HIPCHK(launch_bottom<T>(a, st));
        return MG_OK;
    }
    if (l == H->nlev - 1) {
        const int sing = H->singular ? 1 : 0;
        if constexpr (std::is_same<T, double>::value)
            HIPCHK(launch_coarse_solve((int)F.N, H->minv, F.d.f, F.d.phi, st, sing));
        else
            HIPCHK(launch_coarse_solve_f32((int)F.N, H->minv, F.s.f, F.s.phi, st, sing));
        return MG_OK;
    }
    const bool from_zero = l > 0 ? pre_done == 0 : zero_start;
    int rc = smooth<T>(H, l, H->p.pre_sweeps - pre_done, from_zero ? kInZero : kInPlain, st);
    if (rc) return rc;
    rc = resid_restrict<T>(H, l, st);
    if (rc) return rc;
    rc = vcycle<T>(H, l + 1, st);
    if (rc) return rc;
    return smooth<T>(H, l, H->p.post_sweeps, kInProlong, st);
}

static int vcycle64(mg_hierarchy* H, int l, hipStream_t st) { return vcycle<double>(H, l, st); }
static int vcycle32(mg_hierarchy* H, int l, hipStream_t st) { return vcycle<float>(H, l, st); }

// Relative residual of level 0 (FP64) into host[kSlotRes*4..]; r stored in
// r_store when given.
static int level0_residual(mg_hierarchy* H, double* r_store, hipStream_t st) {
    Level& L0 = H->lev[0];
    int np = 0;
    const Bnd<double> b64 = L0.bnd64();
    if (H->rho.rho) {
        HIPCHK(launch_resid_norm_rho(shape_of(L0), L0.h, H->rho, L0.d.phi, L0.d.f, r_store, H->partials, &np, st,
                                     &b64));
    } else if (r_store) {
        HIPCHK(launch_resid_store(shape_of(L0), L0.h, L0.d.phi, L0.d.f, L0.d.bx, L0.d.by, L0.d.bz, r_store,
                                  H->partials, &np, st, &b64));
    } else {
        HIPCHK(launch_resid_norm<double>(shape_of(L0), L0.h, L0.d.phi, L0.d.f, L0.d.bx, L0.d.by, L0.d.bz,
                                         H->partials, &np, st, &b64));
    }
    int rc = reduce_to(H, np, kSlotRes, st);
    if (rc) return rc;
    return read_scalars(H, kSlotRes * kReduceWidth, kReduceWidth, st);
}

double model_bytes(const mg_params& p, int cycles, int mixed) {
    double N = (double)p.n[0] * p.n[1] * p.n[2];
    if (!mixed) return N * (156.0 + cycles * 326.0);
    return N * (192.0 + cycles * 199.0);
}

// Residual norm of the current finest-level phi measured by a speculative
// first pre-sweep: the sweep reads phi, f and rho anyway, so it also writes
// per-tile partial sums of r = f - L phi(input).  The sweep is out of place
// (into phi2); its output is taken (buffers swapped) only if another cycle
// follows.  Enqueues the sweep, the reduction and the copy of the norm row to
// pinned host memory; the caller synchronises.
static int enqueue_sweep_norm(mg_hierarchy* H, hipStream_t st) {
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
    a.bx = L0.d.bx;
    a.by = L0.d.by;
    a.bz = L0.d.bz;
    a.partials = H->partials;
    a.has_bnd = L0.has_bnd ? 1 : 0;
    a.bnd = L0.bnd64();
    a.dg = L0.dg_d;
    const bool rho0 = H->rho.rho != nullptr;
    int np = 0;
    HIPCHK(launch_sweep_norm(a, rho0, sweep_config_for(L0.nx, L0.ny, L0.nz, rho0), &np, st));
    int rc = reduce_to(H, np, kSlotRes, st);
    if (rc) return rc;
    HIPCHK(hipMemcpyAsync(H->host + kSlotRes * kReduceWidth, H->scal + kSlotRes * kReduceWidth,
                          kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, st));
    return MG_OK;
}

// Everything a captured iteration bakes in: coefficient source, sweep
// counts, tile choices, the kind of iteration and the level buffers it
// starts from.
static std::vector<uintptr_t> graph_key(const mg_hierarchy* H, int kind) {
    std::vector<uintptr_t> k;
    k.push_back((uintptr_t)kind);
    k.push_back((uintptr_t)H->rho.rho);
    k.push_back((uintptr_t)H->rho.b0c);
    k.push_back((uintptr_t)H->rho.b0e);
    k.push_back((uintptr_t)H->p.pre_sweeps);
    k.push_back((uintptr_t)H->p.post_sweeps);
    k.push_back((uintptr_t)inner_cycles_of(H->p));
    k.push_back((uintptr_t)sweep_tune_epoch());
    k.push_back((uintptr_t)H->bottom_on);
    for (int l = 0; l < H->nlev; ++l) {
        k.push_back((uintptr_t)H->lev[l].d.phi);
        k.push_back((uintptr_t)H->lev[l].phi2_d);
        k.push_back((uintptr_t)H->lev[l].s.phi);
        k.push_back((uintptr_t)H->lev[l].phi2_s);
    }
    return k;
}

// A captured iteration is replayable when every level's phi buffers come
// back to where they started within two iterations (an even number of
// out-of-place sweeps per level and cycle; the finest FP64 level may swap
// once per iteration, which two cached captures cover).
static bool graphs_usable(const mg_hierarchy* H) {
    return H->graphs_on && ((H->p.pre_sweeps + H->p.post_sweeps) % 2) == 0;
}

enum { kIterFp64 = 1, kIterMixed = 2 };

// One solver iteration whose last step copies the norm row to pinned host
// memory; the norm is on the host when this returns.  `enqueue` puts the
// iteration's work on a stream and makes the host-side buffer swaps.  Replays
// a captured hipGraph of exactly this work when one matches the current
// state, else captures one (or runs eagerly when graphs are off).  Graph
// work runs on the hierarchy's own stream (the caller's may be the legacy
// stream, which cannot be captured); *on_graph records that the caller's
// stream must later wait for it.
template <typename F>
static int run_iteration(mg_hierarchy* H, hipStream_t st, bool* on_graph, int kind, F&& enqueue) {
    if (!graphs_usable(H)) {
        int rc = enqueue(st);
        if (rc) return rc;
        HIPCHK(hipStreamSynchronize(st));
        return MG_OK;
    }
    if (!H->gstream) {
        HIPCHK(hipStreamCreateWithFlags(&H->gstream, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&H->gev, hipEventDisableTiming));
    }
    hipStream_t gs = H->gstream;
    if (!*on_graph) {                       // order after the caller's earlier work
        HIPCHK(hipEventRecord(H->gev, st));
        HIPCHK(hipStreamWaitEvent(gs, H->gev, 0));
        *on_graph = true;
    }
    const std::vector<uintptr_t> key = graph_key(H, kind);
    mg_hierarchy::CycleGraph* g = nullptr;
    for (auto& c : H->graph)
        if (c.exec && c.key == key) g = &c;
    if (!g) {
        g = &H->graph[H->graph_next];
        H->graph_next = (H->graph_next + 1) % 2;
        if (g->exec) {
            hipGraphExecDestroy(g->exec);
            g->exec = nullptr;
        }
        HIPCHK(hipStreamBeginCapture(gs, hipStreamCaptureModeRelaxed));
        int rc = enqueue(gs);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(gs, &graph);
        if (rc) {
            if (graph) hipGraphDestroy(graph);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture", __LINE__);
        e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g->exec = nullptr;
            return hip_fail(e, "hipGraphInstantiate", __LINE__);
        }
        g->key = key;
        g->post_phi.resize(2 * H->nlev);
        g->post_phi2.resize(2 * H->nlev);
        for (int l = 0; l < H->nlev; ++l) {         // capture left the host pointers as after the iteration
            g->post_phi[l] = H->lev[l].d.phi;
            g->post_phi2[l] = H->lev[l].phi2_d;
            g->post_phi[H->nlev + l] = H->lev[l].s.phi;
            g->post_phi2[H->nlev + l] = H->lev[l].phi2_s;
        }
    } else {
        for (int l = 0; l < H->nlev; ++l) {
            H->lev[l].d.phi = (double*)g->post_phi[l];
            H->lev[l].phi2_d = (double*)g->post_phi2[l];
            H->lev[l].s.phi = (float*)g->post_phi[H->nlev + l];
            H->lev[l].phi2_s = (float*)g->post_phi2[H->nlev + l];
        }
    }
    HIPCHK(hipGraphLaunch(g->exec, gs));
    HIPCHK(hipStreamSynchronize(gs));
    return MG_OK;
}

// FP64: one V-cycle after a taken speculative sweep, then the next
// speculative sweep-norm.
static int cycle_and_norm(mg_hierarchy* H, hipStream_t st, bool* on_graph) {
    return run_iteration(H, st, on_graph, kIterFp64, [H](hipStream_t s) {
        int rc = vcycle<double>(H, 0, s, 1);
        if (rc) return rc;
        return enqueue_sweep_norm(H, s);
    });
}

// Power of two nearest 1 / rms(r), the scale of the FP32 residual: the
// scaled values are O(1) and scaling by 2^k is exact in both directions.
double residual_scale(double norm2_sqrt, size_t n) {
    const double rms = norm2_sqrt / std::sqrt((double)n);
    if (!(rms > 0.0) || !std::isfinite(rms)) return 1.0;
    return std::ldexp(1.0, -std::ilogb(rms));
}

// Mixed-precision solve on a fusable finest level (Sec. 3 multigrid used as
// the inner solver of iterative refinement): each iteration runs
// inner_cycles FP32 V-cycles (the first from zero) on the scaled FP64
// residual, then one FP64 refinement
// kernel adds the correction to phi, recomputes r = f - L phi with exact FP64
// coefficients from rho, writes its per-tile norm rows and the next FP32
// residual; the reduction of those rows then also advances the two
// device-side scales (the residual's, and the power of two nearest
// 1/rms(r) for the next).  The FP32 finest-level sweeps recompute their
// coefficients from an FP32 copy of rho (written by the coefficient kernel
// when it could).  Iterations after the first replay a captured graph.
static int solve_level0_mixed_fused(mg_hierarchy* H, double fnorm, int* cycles_out, double* rel_out,
                                    const std::function<void(int, double)>& record, hipStream_t st) {
    Level& L0 = H->lev[0];
    const bool rho0 = H->rho.rho != nullptr;      // else stored finest-level coefficients (radial beta0)
    if (rho0 && !H->rho32_fresh) HIPCHK(launch_coeff_to_f32(H->rho.rho, H->rho32, L0.N, st));
    H->rho32_fresh = false;
    H->rho32_on = rho0;
    HIPCHK(launch_fill<double>(L0.d.phi, L0.N, 0.0, st));
    const double s0 = residual_scale(fnorm, L0.N);           // residual = f while phi = 0
    HIPCHK(launch_scale_to_f32(L0.d.f, L0.s.f, L0.N, s0, st));
    double* scales = H->scal + kSlotScale * kReduceWidth;
    H->host[kSlotScale * kReduceWidth] = s0;
    H->host[kSlotScale * kReduceWidth + 1] = s0;
    HIPCHK(hipMemcpyAsync(scales, H->host + kSlotScale * kReduceWidth, 2 * sizeof(double), hipMemcpyHostToDevice,
                          st));
    const int cfg = sweep_config_for(L0.nx, L0.ny, L0.nz, rho0);
    const int inner = inner_cycles_of(H->p);
    auto iteration = [H, &L0, cfg, scales, rho0, inner](hipStream_t s) {
        // the FP32 correction: V-cycles on the scaled residual, from zero
        for (int c = 0; c < inner; ++c) {
            int rc = vcycle<float>(H, 0, s, 0, c == 0);
            if (rc) return rc;
        }
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
        a.bx = L0.d.bx;
        a.by = L0.d.by;
        a.bz = L0.d.bz;
        a.corr = L0.s.phi;
        a.r32 = L0.s.f;
        a.scales = scales;
        a.has_bnd = L0.has_bnd ? 1 : 0;
        a.bnd = L0.bnd64();
        a.dg = L0.dg_d;
        int np = 0;
        HIPCHK(launch_refine(a, rho0, cfg, &np, s));
        std::swap(L0.d.phi, L0.phi2_d);
        HIPCHK(launch_reduce_scale(H->partials, np, H->scal + kSlotRes * kReduceWidth, scales, L0.N, s));
        HIPCHK(hipMemcpyAsync(H->host + kSlotRes * kReduceWidth, H->scal + kSlotRes * kReduceWidth,
                              kReduceWidth * sizeof(double), hipMemcpyDeviceToHost, s));
        return (int)MG_OK;
    };
    int status = MG_ERR_NOT_CONVERGED, cycles = 0;
    double rel = 1.0;
    bool on_graph = false;
    while (status == MG_ERR_NOT_CONVERGED && cycles < H->p.max_cycles) {
        int rc = run_iteration(H, st, &on_graph, kIterMixed, iteration);
        if (rc) return rc;
        ++cycles;
        const double* r = H->host + kSlotRes * kReduceWidth;
        rel = std::sqrt(r[0]) / fnorm;
        record(cycles, rel);
        if (r[3] > 0.0 || !std::isfinite(rel)) {
            status = MG_ERR_NONFINITE;
            set_error("non-finite residual during the solve");
            break;
        }
        if (rel <= H->p.rtol) status = MG_OK;
    }
    if (on_graph) {                                  // the caller's stream continues after the graph work
        HIPCHK(hipEventRecord(H->gev, H->gstream));
        HIPCHK(hipStreamWaitEvent(st, H->gev, 0));
    }
    *cycles_out = cycles;
    *rel_out = rel;
    return status;
}

// Level-0 solve on the box-split finest level: f and the coefficients are
// scattered into the boxes, each V-cycle smooths, restricts and prolongates
// box by box with a halo exchange after every colour and after the
// prolongation, levels 1 and coarser are the single-box ones, and phi is
// gathered back into level 0 at the end.
static int solve_level0_boxes(mg_hierarchy* H, double fnorm, mg_stats* stats, hipStream_t st) {
    Level& L0 = H->lev[0];
    Level& L1 = H->lev[1];
    BoxSet& B = H->box;                          // the fused smoother swaps its phi buffers
    B.rho_on = H->rho.rho != nullptr;            // plane-parallel beta0: coefficients from rho
    const bool spec = H->p.pre_sweeps >= 1 && box_norm_sweep_fits(B);
    // the stored face arrays serve the per-colour smoother, the per-cell
    // residual norm and solves without rho
    const bool coeffs = !(B.rho_on && B.fused && spec);
    HIPCHK(launch_box_scatter(B, L0.d.f, L0.d.bx, L0.d.by, L0.d.bz, H->rho.rho, H->rho.b0c, H->rho.b0e, coeffs, st));
    int status = H->p.rtol >= 1.0 ? MG_OK : MG_ERR_NOT_CONVERGED;
    int cycles = 0;
    double rel = 1.0;
    if (stats) {
        stats->resid_hist[0] = 1.0;
        stats->hist_len = 1;
    }
    // fused box sweeps: the residual norm of each cycle's result comes from
    // the next cycle's first pre-sweep, run speculatively (its output is
    // taken only if another cycle follows), as on the single-box level
    int pre_done = 0;
    while (status == MG_ERR_NOT_CONVERGED && cycles < H->p.max_cycles) {
        HIPCHK(launch_box_smooth(B, L0.h, H->p.pre_sweeps - pre_done, st));
        HIPCHK(launch_box_resid_restrict(B, L0.h, L1.d.f, L1.d.phi, st));
        int rc = vcycle<double>(H, 1, st);
        if (rc) return rc;
        HIPCHK(launch_box_smooth(B, L0.h, H->p.post_sweeps, st, L1.d.phi));   // prolongation first
        ++cycles;
        int np = 0;
        if (spec) HIPCHK(launch_box_sweep_norm(B, L0.h, H->partials, &np, st));
        else HIPCHK(launch_box_resid_norm(B, L0.h, H->partials, &np, st));
        rc = reduce_to(H, np, kSlotRes, st);
        if (rc) return rc;
        rc = read_scalars(H, kSlotRes * kReduceWidth, kReduceWidth, st);
        if (rc) return rc;
        const double* r = H->host + kSlotRes * kReduceWidth;
        rel = std::sqrt(r[0]) / fnorm;
        if (stats && cycles < MG_HIST_MAX) {
            stats->resid_hist[cycles] = rel;
            stats->hist_len = cycles + 1;
        }
        if (r[3] > 0.0 || !std::isfinite(rel)) {
            status = MG_ERR_NONFINITE;
            set_error("non-finite residual during the solve");
            break;
        }
        if (rel <= H->p.rtol) {
            status = MG_OK;
        } else if (spec && cycles < H->p.max_cycles) {
            std::swap(B.phi, B.phi2);                // keep the sweep: it is the next cycle's first
            HIPCHK(launch_box_exchange(B, -1, st));
            pre_done = 1;
        }
    }
    HIPCHK(launch_box_gather(B, L0.d.phi, st));
    if (stats) {
        stats->cycles = cycles;
        stats->rel_resid = rel;
    }
    return status;
}

// Mixed-precision solve on the box-split finest level: the single-box mixed
// solve's iteration (one FP32 V-cycle from zero on the FP64 residual scaled
// by a power of two, then one FP64 refinement) with the finest level's FP32
// sweeps, FP32 residual + restriction and the FP64 refinement run box by box
// and the halo of phi32, phi and the scaled residual exchanged after each;
// levels 1 and coarser are the single-box FP32 levels.
static int solve_level0_boxes_mixed(mg_hierarchy* H, double fnorm, mg_stats* stats, hipStream_t st) {
    Level& L0 = H->lev[0];
    Level& L1 = H->lev[1];
    BoxSet& B = H->box;
    if (!B.phi32 || !B.fused || H->p.pre_sweeps < 1 || H->p.post_sweeps < 1) {
        set_error("mixed precision on boxes needs fused boxes and at least one pre- and one post-sweep");
        return MG_ERR_INVALID_ARG;
    }
    B.rho_on = H->rho.rho != nullptr;            // plane-parallel beta0: coefficients from rho
    HIPCHK(launch_box_scatter(B, L0.d.f, L0.d.bx, L0.d.by, L0.d.bz, H->rho.rho, H->rho.b0c, H->rho.b0e, !B.rho_on,
                              st));
    const double s0 = residual_scale(fnorm, L0.N);      // residual = f while phi = 0
    HIPCHK(launch_box_to_f32(B, s0, st));
    double* scales = H->scal + kSlotScale * kReduceWidth;
    H->host[kSlotScale * kReduceWidth] = s0;
    H->host[kSlotScale * kReduceWidth + 1] = s0;
    HIPCHK(hipMemcpyAsync(scales, H->host + kSlotScale * kReduceWidth, 2 * sizeof(double), hipMemcpyHostToDevice,
                          st));
    int status = H->p.rtol >= 1.0 ? MG_OK : MG_ERR_NOT_CONVERGED;
    int cycles = 0;
    double rel = 1.0;
    if (stats) {
        stats->resid_hist[0] = 1.0;
        stats->hist_len = 1;
    }
    const int inner = inner_cycles_of(H->p);
    while (status == MG_ERR_NOT_CONVERGED && cycles < H->p.max_cycles) {
        for (int c = 0; c < inner; ++c) {          // the FP32 correction: V-cycles, the first from zero
            HIPCHK(launch_box_smooth32(B, L0.h, H->p.pre_sweeps, c == 0, nullptr, st));
            HIPCHK(launch_box_resid_restrict32(B, L0.h, L1.s.f, L1.s.phi, st));
            int rc = vcycle<float>(H, 1, st);
            if (rc) return rc;
            HIPCHK(launch_box_smooth32(B, L0.h, H->p.post_sweeps, false, L1.s.phi, st));   // prolongation first
        }
        int np = 0;
        HIPCHK(launch_box_refine(B, L0.h, scales, H->partials, &np, st));
        HIPCHK(launch_reduce_scale(H->partials, np, H->scal + kSlotRes * kReduceWidth, scales, L0.N, st));
        int rc = read_scalars(H, kSlotRes * kReduceWidth, kReduceWidth, st);
        if (rc) return rc;
        ++cycles;
        const double* r = H->host + kSlotRes * kReduceWidth;
        rel = std::sqrt(r[0]) / fnorm;
        if (stats && cycles < MG_HIST_MAX) {
            stats->resid_hist[cycles] = rel;
            stats->hist_len = cycles + 1;
        }
        if (r[3] > 0.0 || !std::isfinite(rel)) {
            status = MG_ERR_NONFINITE;
            set_error("non-finite residual during the solve");
            break;
        }
        if (rel <= H->p.rtol) status = MG_OK;
    }
    HIPCHK(launch_box_gather(B, L0.d.phi, st));
    if (stats) {
        stats->cycles = cycles;
        stats->rel_resid = rel;
    }
    return status;
}

// Solve on level 0 after f (mean-removed) and the coefficients are in place.
static int solve_level0(mg_hierarchy* H, double fnorm, mg_stats* stats, hipStream_t st) {
    if (H->boxes_on)
        return H->p.precision == MG_MIXED ? solve_level0_boxes_mixed(H, fnorm, stats, st)
                                          : solve_level0_boxes(H, fnorm, stats, st);
    Level& L0 = H->lev[0];
    HIPCHK(launch_fill<double>(L0.d.phi, L0.N, 0.0, st));
    int status = MG_ERR_NOT_CONVERGED;
    int cycles = 0;
    double rel = 1.0;
    if (stats) {
        stats->resid_hist[0] = 1.0;
        stats->hist_len = 1;
    }
    auto record = [&](double r) {
        if (stats && cycles < MG_HIST_MAX) {
            stats->resid_hist[cycles] = r;
            stats->hist_len = cycles + 1;
        }
    };
    const bool mixed = H->p.precision == MG_MIXED;
    if (H->p.rtol >= 1.0) status = MG_OK;
    const bool fused = H->p.pre_sweeps >= 1 && H->nlev > 1 && sweep_fusable<double>(L0.nx, L0.ny, L0.nz);
    const bool fused_norm = !mixed && fused;
    if (mixed && fused && status == MG_ERR_NOT_CONVERGED) {
        auto rec = [&](int c, double r) {
            if (stats && c < MG_HIST_MAX) {
                stats->resid_hist[c] = r;
                stats->hist_len = c + 1;
            }
        };
        status = solve_level0_mixed_fused(H, fnorm, &cycles, &rel, rec, st);
        if (status != MG_OK && status != MG_ERR_NOT_CONVERGED && status != MG_ERR_NONFINITE) return status;
    } else if (fused_norm) {
        bool on_graph = false;
        while (status == MG_ERR_NOT_CONVERGED) {
            int rc;
            if (cycles == 0) {
                if (H->p.max_cycles == 0) break;
                rc = vcycle<double>(H, 0, st, 0);
                if (rc == MG_OK) rc = enqueue_sweep_norm(H, st);
                if (rc == MG_OK && hipStreamSynchronize(st) != hipSuccess) rc = MG_ERR_HIP;
            } else {
                std::swap(L0.d.phi, L0.phi2_d);     // keep the sweep: it is this cycle's first
                rc = cycle_and_norm(H, st, &on_graph);
            }
            if (rc) return rc;
            ++cycles;
            const double* r = H->host + kSlotRes * kReduceWidth;
            rel = std::sqrt(r[0]) / fnorm;
            record(rel);
            if (r[3] > 0.0 || !std::isfinite(rel)) {
                status = MG_ERR_NONFINITE;
                set_error("non-finite residual during the solve");
                break;
            }
            if (rel <= H->p.rtol) {
                status = MG_OK;
                break;
            }
            if (cycles >= H->p.max_cycles) break;
        }
        if (on_graph) {                              // the caller's stream continues after the graph work
            HIPCHK(hipEventRecord(H->gev, H->gstream));
            HIPCHK(hipStreamWaitEvent(st, H->gev, 0));
        }
    } else {
        if (mixed) {
            // phi = 0, so the FP64 residual is f itself
            int rc = level0_residual(H, H->r64, st);
            if (rc) return rc;
        }
        while (status == MG_ERR_NOT_CONVERGED && cycles < H->p.max_cycles) {
            if (!mixed) {
                int rc = vcycle64(H, 0, st);
                if (rc) return rc;
            } else {
                // correction from an FP32 cycle on the scaled FP64 residual r64
                double rmax = H->host[kSlotRes * kReduceWidth + 2];
                if (!(rmax > 0.0)) break;
                HIPCHK(launch_to_f32(H->r64, L0.s.f, L0.N, H->scal + kSlotRes * kReduceWidth + 2, st));
                HIPCHK(launch_fill<float>(L0.s.phi, L0.N, 0.0f, st));
                int rc = vcycle32(H, 0, st);
                if (rc) return rc;
                HIPCHK(launch_accumulate(L0.d.phi, L0.s.phi, L0.N, H->scal + kSlotRes * kReduceWidth + 2, st));
            }
            ++cycles;
            int rc = level0_residual(H, mixed ? H->r64 : nullptr, st);
            if (rc) return rc;
            const double* r = H->host + kSlotRes * kReduceWidth;
            rel = std::sqrt(r[0]) / fnorm;
            record(rel);
            if (r[3] > 0.0 || !std::isfinite(rel)) {
                status = MG_ERR_NONFINITE;
                set_error("non-finite residual during the solve");
                break;
            }
            if (rel <= H->p.rtol) status = MG_OK;
        }
    }
    if (stats) {
        stats->cycles = cycles;
        stats->rel_resid = rel;
    }
    return status;
}

static int project_impl(mg_hierarchy* H, const double* rho, const double* b0c, const double* b0e,
                        const double* S, double* u, double* v, double* w, double* phi_out, mg_stats* stats,
                        hipStream_t st, const double* w0, const Radial* rad) {
    const bool radial = rad && rad->prof;
    if (!H || !rho || (!radial && (!b0c || !b0e)) || !S || !u || !v || !w) {
        set_error("null argument to mac_project");
        return MG_ERR_INVALID_ARG;
    }
    mg_stats local;
    std::memset(&local, 0, sizeof local);
    mg_stats* S_ = stats ? stats : &local;
    std::memset(S_, 0, sizeof *S_);
    S_->nlevels = H->nlev;
    // device time from events; a hierarchy without events (laid out by
    // setup_static) reports the host wall time of the call instead
    const auto t_host0 = std::chrono::steady_clock::now();
    if (H->ev0) HIPCHK(hipEventRecord(H->ev0, st));
    Level& L0 = H->lev[0];
    // the fused finest-level sweep reads rho as 16-byte pairs
    const double* rho_src = rho;
    if (((uintptr_t)rho & 15) != 0) {
        HIPCHK(launch_copy(H->rho_own, rho, L0.N, st));
        rho_src = H->rho_own;
    }
    // plane-parallel beta0: the finest-level sweeps recompute their
    // coefficients from rho; a radial beta0 leaves them to the stored ones
    H->rho = radial ? RhoArgs{} : RhoArgs{rho_src, b0c, b0e, H->px, H->py, H->pz};
    int rc = build_coefficients(H, rho, b0c, b0e, S, u, v, w, st, w0, rad);
    if (rc) return rc;
    rc = read_scalars(H, kSlotRhs * kReduceWidth, kReduceWidth, st);
    if (rc) return rc;
    const double* q = H->host + kSlotRhs * kReduceWidth;
    double sf = q[0], saf = q[1], bad = q[2], nonfin = q[3];
    S_->sum_f = sf;
    S_->sum_abs_f = saf;
    if (nonfin > 0.0 || !std::isfinite(sf) || !std::isfinite(saf)) {
        set_error("non-finite value in rho, beta0, U or S");
        return S_->status = MG_ERR_NONFINITE;
    }
    if (bad > 0.0) {
        set_error("rho and beta0 must be positive");
        return S_->status = MG_ERR_INVALID_ARG;
    }
    // an outflow side makes the operator non-singular: any f is admissible
    // and neither f nor phi has its mean removed
    if (H->singular && std::fabs(sf) > 1e-8 * saf) {
        set_error("incompatible right-hand side: |sum f| > 1e-8 sum |f|");
        return S_->status = MG_ERR_INCOMPATIBLE_RHS;
    }
    int status = MG_OK;
    if (saf == 0.0) {
        HIPCHK(launch_fill<double>(L0.d.phi, L0.N, 0.0, st));
        S_->hist_len = 1;
        S_->resid_hist[0] = 0.0;
    } else {
        double mean = H->singular ? sf / (double)L0.N : 0.0;
        S_->mean_removed = mean;
        int np = 0;
        HIPCHK(launch_shift_norm(shape_of(L0), L0.d.f, mean, H->partials, &np, st));
        rc = reduce_to(H, np, kSlotNorm, st);
        if (rc) return rc;
        rc = read_scalars(H, kSlotNorm * kReduceWidth, kReduceWidth, st);
        if (rc) return rc;
        double fnorm = std::sqrt(H->host[kSlotNorm * kReduceWidth]);
        S_->norm_f = fnorm;
        if (fnorm == 0.0) {
            HIPCHK(launch_fill<double>(L0.d.phi, L0.N, 0.0, st));
        } else {
            S_->rel_resid0 = 1.0;
            const auto t_s0 = std::chrono::steady_clock::now();
            if (H->evs0) HIPCHK(hipEventRecord(H->evs0, st));
            status = solve_level0(H, fnorm, S_, st);
            if (status != MG_OK && status != MG_ERR_NOT_CONVERGED) return S_->status = status;
            if (H->evs1) {
                HIPCHK(hipEventRecord(H->evs1, st));
                HIPCHK(hipEventSynchronize(H->evs1));
                float ms = 0.f;
                hipEventElapsedTime(&ms, H->evs0, H->evs1);
                S_->ms_smooth = ms;
            } else {       // every iteration ends with a host synchronisation: wall time of the loop
                S_->ms_smooth =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_s0).count();
            }
        }
    }
    int np = 0;
    if (H->singular) {
        HIPCHK(launch_sum(shape_of(L0), L0.d.phi, H->partials, &np, st));
        rc = reduce_to(H, np, kSlotPhi, st);
        if (rc) return rc;
    }
    if (H->outflow || radial) {
        const GenArgs g = gen_args(H, rho, b0c, b0e, rad);
        HIPCHK(launch_correct_gen(g, L0.d.phi, H->singular ? H->scal + kSlotPhi * kReduceWidth : nullptr, u, v, w,
                                  phi_out, st));
    } else {
        HIPCHK(launch_correct(shape_of(L0), H->px, H->py, H->pz, L0.h, b0c, b0e, L0.d.bx, L0.d.by, L0.d.bz,
                              L0.d.phi, H->scal + kSlotPhi * kReduceWidth, u, v, w, phi_out, st));
    }
    if (H->ev1) HIPCHK(hipEventRecord(H->ev1, st));
    if (H->singular) {
        rc = read_scalars(H, kSlotPhi * kReduceWidth, kReduceWidth, st);
        if (rc) return rc;
        S_->phi_mean = H->host[kSlotPhi * kReduceWidth] / (double)L0.N;
    } else {
        HIPCHK(hipStreamSynchronize(st));
        S_->phi_mean = 0.0;
    }
    if (H->ev0 && H->ev1) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, H->ev0, H->ev1);
        S_->ms_total = ms;
    } else {
        S_->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_host0).count();
    }
    S_->ms_other = std::max(0.0, S_->ms_total - S_->ms_smooth);
    S_->bytes_model = model_bytes(H->p, S_->cycles, H->p.precision == MG_MIXED);
    S_->status = status;
    if (status == MG_ERR_NOT_CONVERGED) set_error("maximum number of cycles reached");
    return status;
}

int project(mg_hierarchy* H, const double* rho, const double* b0c, const double* b0e, const double* S,
            double* u, double* v, double* w, double* phi_out, mg_stats* stats, hipStream_t st, const double* w0,
            const Radial* rad) {
    int rc = project_impl(H, rho, b0c, b0e, S, u, v, w, phi_out, stats, st, w0, rad);
    if (H) H->rho32_on = H->rho32_fresh = false;
    // the caller's rho may not outlive the call: later mg_vcycle / step calls
    // use the stored finest-level coefficients (bit-identical values)
    if (H) H->rho = RhoArgs{};
    return rc;
}

int vcycle_api(mg_hierarchy* H, double* phi, const double* rhs, double* rel_out, hipStream_t st) {
    if (!H || !phi || !rhs) {
        set_error("null argument to mg_vcycle");
        return MG_ERR_INVALID_ARG;
    }
    if (!H->coeffs_valid) {
        set_error("mg_vcycle before mg_set_coefficients / mac_project");
        return MG_ERR_INVALID_ARG;
    }
    Level& L0 = H->lev[0];
    HIPCHK(launch_copy(L0.d.f, rhs, L0.N, st));
    HIPCHK(launch_copy(L0.d.phi, phi, L0.N, st));
    int rc = vcycle64(H, 0, st);
    if (rc) return rc;
    HIPCHK(launch_copy(phi, L0.d.phi, L0.N, st));
    if (rel_out) {
        int np = 0;
        HIPCHK(launch_shift_norm(shape_of(L0), L0.d.f, 0.0, H->partials, &np, st));
        rc = reduce_to(H, np, kSlotNorm, st);
        if (rc) return rc;
        rc = read_scalars(H, kSlotNorm * kReduceWidth, kReduceWidth, st);
        if (rc) return rc;
        double fn = std::sqrt(H->host[kSlotNorm * kReduceWidth]);
        rc = level0_residual(H, nullptr, st);
        if (rc) return rc;
        double rn = std::sqrt(H->host[kSlotRes * kReduceWidth]);
        *rel_out = fn > 0.0 ? rn / fn : 0.0;
    }
    return MG_OK;
}

int level_copy(mg_hierarchy* H, int l, int which, void* buf, int to_h, hipStream_t st) {
    if (!H || !buf || l < 0 || l >= H->nlev) {
        set_error("bad level_copy arguments");
        return MG_ERR_INVALID_ARG;
    }
    Level& L = H->lev[l];
    double* a;
    switch (which) {
        case MG_ARR_PHI: a = L.d.phi; break;
        case MG_ARR_F: a = L.d.f; break;
        case MG_ARR_BX: a = L.d.bx; break;
        case MG_ARR_BY: a = L.d.by; break;
        case MG_ARR_BZ: a = L.d.bz; break;
        default: set_error("bad array id"); return MG_ERR_INVALID_ARG;
    }
    if (to_h) {
        HIPCHK(launch_copy(a, (const double*)buf, L.N, st));
        if (which >= MG_ARR_BX) H->coeffs_valid = true;
    } else {
        HIPCHK(launch_copy((double*)buf, a, L.N, st));
    }
    return MG_OK;
}

int level_step(mg_hierarchy* H, int l, int step, int arg, hipStream_t st) {
    if (!H || l < 0 || l >= H->nlev) {
        set_error("bad level");
        return MG_ERR_INVALID_ARG;
    }
    Level& F = H->lev[l];
    Shape s = shape_of(F);
    bool has_coarse = l + 1 < H->nlev;
    switch (step) {
        case MG_STEP_SMOOTH: {
            if (!has_coarse) break;
            int rc = smooth<double>(H, l, arg, kInPlain, st);
            if (rc) return rc;
            break;
        }
        case MG_STEP_RESID_RESTRICT:
        case MG_STEP_DOWN: {
            if (!has_coarse) {
                set_error("no coarser level");
                return MG_ERR_INVALID_ARG;
            }
            if (step == MG_STEP_DOWN) {
                int rc = smooth<double>(H, l, arg, kInPlain, st);
                if (rc) return rc;
            }
            int rc = resid_restrict<double>(H, l, st);
            if (rc) return rc;
            break;
        }
        case MG_STEP_PROLONG:
        case MG_STEP_UP: {
            if (!has_coarse) {
                set_error("no coarser level");
                return MG_ERR_INVALID_ARG;
            }
            int rc = smooth<double>(H, l, step == MG_STEP_UP ? arg : 0, kInProlong, st);
            if (rc) return rc;
            break;
        }
        case MG_STEP_COARSE:
            if (has_coarse) {
                set_error("MG_STEP_COARSE needs the coarsest level");
                return MG_ERR_INVALID_ARG;
            }
            {
                const Bnd<double> cb = F.bnd64();
                HIPCHK(launch_coarse_setup(s, F.h, F.d.bx, F.d.by, F.d.bz, H->minv, st, F.has_bnd ? &cb : nullptr,
                                           H->singular ? 1 : 0));
                HIPCHK(launch_coarse_solve((int)F.N, H->minv, F.d.f, F.d.phi, st, H->singular ? 1 : 0));
            }
            break;
        default:
            set_error("unknown step");
            return MG_ERR_INVALID_ARG;
    }
    return MG_OK;
}

}  // namespace mg

// ============================================================================
// C ABI
// ============================================================================
using namespace mg;

namespace {
int g_forced_for_tuner() { return tune_forced(); }
}  // namespace

namespace mg {

// Layout of a multi-box finest level of box-cell boxes for params p: the box
// grid, ghosted sizes and whether every box takes the fused sweep, and the
// padded element counts of one box array (e) and of one beta0 table (eb).
int box_layout(const mg_params& p, const int32_t box[3], BoxSet* out, size_t* e, size_t* eb) {
    BoxSet B{};
    int emin[3];                               // the smallest box's cells per direction
    for (int d = 0; d < 3; ++d) {
        const int n = p.n[d];
        if (box[d] < 2 || box[d] % 2 != 0 || box[d] > n) {
            set_error("box sizes must be even, at least 2, and at most the domain size in each direction");
            return MG_ERR_INVALID_ARG;
        }
        B.n[d] = n;
        B.B[d] = box[d];
        B.nb[d] = (n + box[d] - 1) / box[d];  // the last box holds the (even) remainder
        B.G[d] = box[d] + 2 * kBoxGhost;
        emin[d] = n - (B.nb[d] - 1) * box[d];
    }
    B.nbox = B.nb[0] * B.nb[1] * B.nb[2];
    B.stride = (size_t)B.G[0] * B.G[1] * B.G[2];
    B.fused = sweep_boxes_fit(emin[0], emin[1], emin[2]) ? 1 : 0;   // every box takes the fused sweep
    if (B.stride >= ((size_t)1 << 31)) {
        set_error("box too large: its ghosted array must stay below 2^31 cells");
        return MG_ERR_INVALID_ARG;
    }
    *e = (B.stride * B.nbox + 31) / 32 * 32;     // 256-byte aligned sub-arrays
    *eb = ((size_t)B.G[2] * B.nbox + 31) / 32 * 32;
    *out = B;
    return MG_OK;
}

size_t box_bytes(const mg_params& p, const int32_t box[3]) {
    BoxSet B;
    size_t e = 0, eb = 0;
    if (box_layout(p, box, &B, &e, &eb) != MG_OK) return 0;
    return (7 * e + 2 * eb) * sizeof(double) + (p.precision == MG_MIXED ? 7 * e * sizeof(float) : 0);
}

}  // namespace mg

extern "C" {

void mg_default_params(mg_params* p, int32_t nx, int32_t ny, int32_t nz, double dx) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->n[0] = nx;
    p->n[1] = ny;
    p->n[2] = nz;
    p->dx = dx;
    p->bc[0] = MG_BC_PERIODIC;
    p->bc[1] = MG_BC_PERIODIC;
    p->bc[2] = MG_BC_WALL;
    p->pre_sweeps = 2;
    p->post_sweeps = 2;
    p->rtol = 1e-10;
    p->max_cycles = 100;
    p->precision = MG_FP64;
    p->inner_cycles = 0;          // the default: two FP32 V-cycles per refinement step
}

int32_t mg_num_levels_for(const mg_params* p) {
    if (!p) return 0;
    return count_levels(p->n[0], p->n[1], p->n[2]);
}

size_t mg_workspace_bytes(const mg_params* p) { return workspace_bytes(p); }

int mg_setup(const mg_params* p, void* workspace, size_t ws_bytes, mg_handle* out) {
    try {
        return setup(p, workspace, ws_bytes, out);
    } catch (...) {
        set_error("internal error in mg_setup");
        return MG_ERR_HIP;
    }
}

int mg_destroy(mg_handle h) { return destroy(h); }

int mg_set_params(mg_handle h, const mg_params* p) {
    if (!h) {
        set_error("null handle");
        return MG_ERR_INVALID_ARG;
    }
    int st = validate_params(p);
    if (st) return st;
    for (int d = 0; d < 3; ++d)
        if (p->n[d] != h->p.n[d] || p->bc[d] != h->p.bc[d]) {
            set_error("mg_set_params cannot change the shape or boundary types");
            return MG_ERR_INVALID_ARG;
        }
    if (p->dx != h->p.dx) {
        set_error("mg_set_params cannot change dx");
        return MG_ERR_INVALID_ARG;
    }
    if (p->precision == MG_MIXED && h->p.precision != MG_MIXED) {
        set_error("hierarchy was built without FP32 mirrors; set up with MG_MIXED");
        return MG_ERR_INVALID_ARG;
    }
    h->p = *p;
    return MG_OK;
}

int mg_set_coefficients(mg_handle h, const double* rho, const double* beta0_cc, const double* beta0_edge,
                        void* stream) {
    if (!h || !rho || !beta0_cc || !beta0_edge) {
        set_error("null argument to mg_set_coefficients");
        return MG_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    // keep private copies: later mg_vcycle / step calls recompute the
    // finest-level coefficients from them
    const int nz = h->p.n[2];
    HIPCHK(launch_copy(h->rho_own, rho, h->lev[0].N, st));
    HIPCHK(launch_copy(h->b0c_own, beta0_cc, (size_t)nz, st));
    HIPCHK(launch_copy(h->b0e_own, beta0_edge, (size_t)nz + 1, st));
    h->rho = RhoArgs{h->rho_own, h->b0c_own, h->b0e_own, h->px, h->py, h->pz};
    int rc = build_coefficients(h, h->rho_own, h->b0c_own, h->b0e_own, nullptr, nullptr, nullptr, nullptr, st);
    if (rc) return rc;
    rc = read_scalars(h, kSlotRhs * kReduceWidth, kReduceWidth, st);
    if (rc) return rc;
    const double* q = h->host + kSlotRhs * kReduceWidth;
    if (q[3] > 0.0) {
        h->coeffs_valid = false;
        set_error("non-finite rho or beta0");
        return MG_ERR_NONFINITE;
    }
    if (q[2] > 0.0) {
        h->coeffs_valid = false;
        set_error("rho and beta0 must be positive");
        return MG_ERR_INVALID_ARG;
    }
    return MG_OK;
}

int mac_project(mg_handle h, const double* rho, const double* beta0_cc, const double* beta0_edge,
                const double* S, double* u, double* v, double* w, double* phi, mg_stats* stats,
                void* stream) {
    try {
        return project(h, rho, beta0_cc, beta0_edge, S, u, v, w, phi, stats, (hipStream_t)stream);
    } catch (...) {
        set_error("internal error in mac_project");
        return MG_ERR_HIP;
    }
}

int mac_project_full(mg_handle h, const double* rho, const double* beta0_cc, const double* beta0_edge,
                     const double* S, const double* p0_cc, const double* gamma1_cc, const double* dp0dt_cc,
                     double* u, double* v, double* w, double* phi, mg_stats* stats, void* stream) {
    if (!h || !p0_cc || !gamma1_cc || !dp0dt_cc) {
        set_error("null argument to mac_project_full");
        return MG_ERR_INVALID_ARG;
    }
    try {
        hipStream_t st = (hipStream_t)stream;
        const hipError_t e = launch_dp0_term(h->p.n[2], p0_cc, gamma1_cc, dp0dt_cc, h->w0, st);
        if (e != hipSuccess) return hip_fail(e, "launch_dp0_term", __LINE__);
        return project(h, rho, beta0_cc, beta0_edge, S, u, v, w, phi, stats, st, h->w0);
    } catch (...) {
        set_error("internal error in mac_project_full");
        return MG_ERR_HIP;
    }
}

int mg_beta0_from_p0(int32_t nz, double rho0_base, const double* p0_edge, const double* p0_cc,
                     const double* gamma1_cc, double* beta0_cc, double* beta0_edge, void* stream) {
    if (nz < 1 || !(rho0_base > 0.0) || !std::isfinite(rho0_base) || !p0_edge || !p0_cc || !gamma1_cc ||
        !beta0_cc || !beta0_edge) {
        set_error("bad mg_beta0_from_p0 arguments");
        return MG_ERR_INVALID_ARG;
    }
    const hipError_t e = launch_beta0_from_p0(nz, rho0_base, p0_edge, p0_cc, gamma1_cc, beta0_cc, beta0_edge,
                                              (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch_beta0_from_p0", __LINE__);
    return MG_OK;
}

static int radial_args(int32_t nr, double dr, const double* beta0_r, const double centre[3], Radial* r) {
    if (nr < 1 || !(dr > 0.0) || !std::isfinite(dr) || !beta0_r || !centre || !std::isfinite(centre[0]) ||
        !std::isfinite(centre[1]) || !std::isfinite(centre[2])) {
        set_error("bad radial base state arguments");
        return MG_ERR_INVALID_ARG;
    }
    r->nr = nr;
    r->dr = dr;
    r->prof = beta0_r;
    for (int d = 0; d < 3; ++d) r->c[d] = centre[d];
    return MG_OK;
}

int mac_project_radial(mg_handle h, const double* rho, int32_t nr, double dr, const double* beta0_r,
                       const double centre[3], const double* S, double* u, double* v, double* w, double* phi,
                       mg_stats* stats, void* stream) {
    Radial r;
    int rc = radial_args(nr, dr, beta0_r, centre, &r);
    if (rc) return rc;
    try {
        return project(h, rho, nullptr, nullptr, S, u, v, w, phi, stats, (hipStream_t)stream, nullptr, &r);
    } catch (...) {
        set_error("internal error in mac_project_radial");
        return MG_ERR_HIP;
    }
}

int mg_map_radial(int32_t nx, int32_t ny, int32_t nz, double dx, int32_t nr, double dr, const double* beta0_r,
                  const double centre[3], double* beta0_out, void* stream) {
    Radial r;
    int rc = radial_args(nr, dr, beta0_r, centre, &r);
    if (rc) return rc;
    if (nx < 1 || ny < 1 || nz < 1 || !(dx > 0.0) || !beta0_out) {
        set_error("bad mg_map_radial arguments");
        return MG_ERR_INVALID_ARG;
    }
    GenArgs g{};
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.h = dx;
    g.nr = r.nr;
    g.dr = r.dr;
    g.prof = r.prof;
    g.cx = r.c[0];
    g.cy = r.c[1];
    g.cz = r.c[2];
    const hipError_t e = launch_map_radial(g, beta0_out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "launch_map_radial", __LINE__);
    return MG_OK;
}

int mg_vcycle(mg_handle h, double* phi, const double* rhs, double* rel_resid_out, void* stream) {
    return vcycle_api(h, phi, rhs, rel_resid_out, (hipStream_t)stream);
}

int mg_level_info(mg_handle h, int32_t level, int32_t dims[3], double* dx) {
    if (!h || level < 0 || level >= h->nlev || !dims) {
        set_error("bad level");
        return MG_ERR_INVALID_ARG;
    }
    dims[0] = h->lev[level].nx;
    dims[1] = h->lev[level].ny;
    dims[2] = h->lev[level].nz;
    if (dx) *dx = h->lev[level].h;
    return MG_OK;
}

int mg_level_copy(mg_handle h, int32_t level, int32_t array, void* buffer, int32_t to_hierarchy,
                  void* stream) {
    return level_copy(h, level, array, buffer, to_hierarchy, (hipStream_t)stream);
}

int mg_level_step(mg_handle h, int32_t level, int32_t step, int32_t arg, void* stream) {
    return level_step(h, level, step, arg, (hipStream_t)stream);
}

int mg_autotune(mg_handle h, int32_t reps, void* stream) {
    if (!h || reps < 1) {
        set_error("bad mg_autotune arguments");
        return MG_ERR_INVALID_ARG;
    }
    if (!h->coeffs_valid) {
        set_error("mg_autotune needs coefficients (mg_set_coefficients or mac_project first)");
        return MG_ERR_INVALID_ARG;
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const int saved = g_forced_for_tuner();
    int rc = MG_OK;
    for (int l = 0; l + 1 < h->nlev && rc == MG_OK; ++l) {
        Level& F = h->lev[l];
        if (!sweep_fusable<double>(F.nx, F.ny, F.nz)) break;
        const bool rho = l == 0 && h->rho.rho != nullptr;
        float best = 1e30f;
        int best_cfg = -1;
        for (int c = 0; c < kNumSweepCfg && rc == MG_OK; ++c) {
            if (!sweep_cfg_fits(F.nx, F.ny, c) || (l == 0 && c >= kFirstCoarseCfg)) continue;
            sweep_force_config(c);
            rc = smooth<double>(h, l, 1, kInPlain, st);          // warm
            if (rc) break;
            hipEventRecord(e0, st);
            rc = smooth<double>(h, l, reps, kInPlain, st);
            hipEventRecord(e1, st);
            if (hipEventSynchronize(e1) != hipSuccess) rc = MG_ERR_HIP;
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) {
                best = ms;
                best_cfg = c;
            }
        }
        if (best_cfg >= 0) sweep_record_tuned(F.nx, F.ny, F.nz, rho, true, best_cfg, l > 0);
    }
    sweep_force_config(saved);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (rc == MG_OK) {
        const int w = tune_save_env();          // persist the choices when MACPROJ_TUNE_CACHE names a file
        if (w < 0) return w;
    }
    return rc;
}

int mg_tune_sweep(int32_t cfg) {
    if (cfg < -1 || cfg >= kNumSweepCfg) {
        set_error("sweep configuration out of range");
        return MG_ERR_INVALID_ARG;
    }
    sweep_force_config(cfg);
    return MG_OK;
}

int mg_set_bottom(mg_handle h, int32_t enable) {
    if (!h) {
        set_error("null handle");
        return MG_ERR_INVALID_ARG;
    }
    h->bottom_on = enable != 0;
    return MG_OK;
}

int mg_set_boxes(mg_handle h, const int32_t box[3]) {
    if (!h) {
        set_error("null handle");
        return MG_ERR_INVALID_ARG;
    }
    if (!box || (box[0] == 0 && box[1] == 0 && box[2] == 0)) {
        if (h->box_mem) HIPCHK(hipFree(h->box_mem));
        h->box_mem = nullptr;
        h->box = BoxSet{};
        h->boxes_on = false;
        return MG_OK;
    }
    if (h->outflow || h->nlev < 2) {
        set_error("a multi-box finest level needs periodic or wall sides and two or more levels");
        return MG_ERR_INVALID_ARG;
    }
    BoxSet B{};
    size_t e = 0, eb = 0;
    const int rc = box_layout(h->p, box, &B, &e, &eb);
    if (rc) return rc;
    const bool mixed = h->p.precision == MG_MIXED;
    if (mixed && !B.fused) {
        set_error("mixed precision on boxes needs every box to take the fused sweep (at least 32 x 8 x 4 cells)");
        return MG_ERR_INVALID_ARG;
    }
    if (mixed && (long long)sweep_boxes_tiles(B.B[0], B.B[1], B.B[2]) * B.nbox > kMaxPartialRows) {
        set_error("mixed precision on boxes: too many box tiles for the residual-norm rows");
        return MG_ERR_INVALID_ARG;
    }
    B.per[0] = h->px;
    B.per[1] = h->py;
    B.per[2] = h->pz;
    if (h->box_mem) HIPCHK(hipFree(h->box_mem));
    h->box_mem = nullptr;
    h->boxes_on = false;
    void* mem = nullptr;
    HIPCHK(hipMalloc(&mem, (7 * e + 2 * eb) * sizeof(double) + (mixed ? 7 * e * sizeof(float) : 0)));
    double* p = static_cast<double*>(mem);
    B.phi = p;
    B.phi2 = p + e;
    B.f = p + 2 * e;
    B.cx = p + 3 * e;
    B.cy = p + 4 * e;
    B.cz = p + 5 * e;
    B.rho = p + 6 * e;
    B.b0c = p + 7 * e;
    B.b0e = B.b0c + eb;
    if (mixed) {                               // FP32 arrays after the FP64 ones (256-byte aligned)
        float* q = reinterpret_cast<float*>(B.b0e + eb);
        B.phi32 = q;
        B.phi2_32 = q + e;
        B.f32 = q + 2 * e;
        B.rho32 = q + 3 * e;
        B.cx32 = q + 4 * e;
        B.cy32 = q + 5 * e;
        B.cz32 = q + 6 * e;
    }
    h->box_mem = mem;
    h->box = B;
    h->boxes_on = true;
    return MG_OK;
}

int mg_set_graphs(mg_handle h, int32_t enable) {
    if (!h) {
        set_error("null handle");
        return MG_ERR_INVALID_ARG;
    }
    h->graphs_on = enable != 0;
    return MG_OK;
}

int mg_sweep_config(mg_handle h, int32_t level, int32_t tile[4]) {
    if (!h || !tile || level < 0 || level >= h->nlev) {
        set_error("bad mg_sweep_config arguments");
        return MG_ERR_INVALID_ARG;
    }
    tile[0] = tile[1] = tile[2] = tile[3] = -1;
    const Level& F = h->lev[level];
    const bool dbl = h->p.precision == MG_FP64;
    const bool fusable = dbl ? sweep_fusable<double>(F.nx, F.ny, F.nz) : sweep_fusable<float>(F.nx, F.ny, F.nz);
    if (level + 1 >= h->nlev || !fusable) return MG_OK;
    const int c = sweep_config_for(F.nx, F.ny, F.nz, level == 0, dbl, level > 0);
    tile[0] = kSweepCfgs[c].tx;
    tile[1] = kSweepCfgs[c].ty;
    tile[2] = kSweepCfgs[c].tz;
    tile[3] = c;
    return MG_OK;
}

const char* mg_strerror(int code) {
    switch (code) {
        case MG_OK: return "ok";
        case MG_PENDING: return "pending";
        case MG_ERR_INVALID_ARG: return "invalid argument";
        case MG_ERR_BAD_SIZE: return "unsupported size";
        case MG_ERR_INCOMPATIBLE_RHS: return "incompatible right-hand side";
        case MG_ERR_NOT_CONVERGED: return "not converged";
        case MG_ERR_NONFINITE: return "non-finite value";
        case MG_ERR_OOM: return "out of device memory";
        case MG_ERR_HIP: return "HIP runtime error";
        case MG_ERR_BUDGET: return "request exceeds the memory budget";
        case MG_ERR_BUSY: return "busy";
        default: return "unknown status";
    }
}

const char* mg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
