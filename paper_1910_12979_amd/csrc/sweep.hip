// Fused red-black Gauss-Seidel sweep for gfx950.
//
// One launch performs a whole sweep (red cells, then black cells) out of
// place: phi_out = RBGS(phi_in).  A workgroup owns a TX x TY column tile and
// marches through a chunk of z planes.  Per plane, the red update is computed
// on the tile plus a one-cell ring (redundantly with the neighbouring tiles)
// so the black update of every tile cell finds all four in-plane red
// neighbours locally; phi_in is only read, so neighbouring workgroups never
// race.  In-plane neighbours come from LDS planes, z-neighbours from
// registers that slide with the march.
//
// Each thread owns an x-pair of cells (even x, odd x).  At every plane one
// cell of a pair is red and the other black, so the red stage and the black
// stage each update exactly one cell per thread (no lane divergence), and
// pairs move as 16-byte loads and stores.  Global loads run two planes ahead
// of their use through a small register queue so HBM latency is hidden
// behind the work of the planes in between.
//
// Coefficient source: on the finest level the face coefficients
// b = beta0_face / (0.5 (rho_L + rho_R)) are recomputed from rho and beta0
// (8 bytes per cell instead of 24), with the same expression as everywhere
// else so the values are bit-identical to stored ones; coarser levels read
// their stored (averaged) coefficients.
//
// Input variants: phi_in = 0 (first pre-sweep on a coarse level), phi_in as
// stored, or phi_in + P phi_coarse (first post-sweep: the prolongation is
// folded into the load).
//
// The per-cell update order is the same as the reference definition:
//   num = bxl*phi(x-1) + bxh*phi(x+1) + byl*phi(y-1) + byh*phi(y+1)
//       + bzl*phi(z-1) + bzh*phi(z+1);  den = bxl+bxh+byl+byh+bzl+bzh;
//   phi = (num - h^2 f) / den.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <map>
#include <mutex>

#include "devmath.h"
#include "mg_internal.h"
#include "sweep.h"

namespace mg {
namespace {

constexpr int kNumXcd = 8;

template <typename T>
struct V2;
template <>
struct V2<double> {
    using type = double2;
};
template <>
struct V2<float> {
    using type = float2;
};

template <typename T>
__device__ inline void ld2(const T* p, T& a, T& b) {
    typename V2<T>::type v = *reinterpret_cast<const typename V2<T>::type*>(p);
    a = v.x;
    b = v.y;
}

template <typename T>
__device__ inline void st2(T* p, T a, T b) {
    typename V2<T>::type v;
    v.x = a;
    v.y = b;
    *reinterpret_cast<typename V2<T>::type*>(p) = v;
}

__device__ inline int wrap3(int g, int n) {
    if (g < 0) g += n;
    if (g >= n) g -= n;
    if (g >= n) g -= n;
    return g;
}

// Map a launch-order block id to a tile id so that each XCD (blocks are
// dealt round-robin across the 8 XCDs) works on a contiguous range of tiles
// and their shared halos stay in that XCD's L2.
__device__ inline int xcd_tile(int b, int total) {
    if (total % kNumXcd != 0) return b;
    return (b % kNumXcd) * (total / kNumXcd) + b / kNumXcd;
}

// The body of one tile: shared by the single-problem kernel and the batched
// kernel, so a problem's values do not depend on how it was launched.
template <typename T, int TX, int TY, bool kRho, int kIn, int kOp, bool kBnd, bool kBox = false>
__device__ __forceinline__ void sweep_body(const SweepArgs<T>& a, const int tile) {
    constexpr bool kNorm = kOp == kOpSweepNorm;    // sweep + residual norm of its input
    constexpr bool kRR = kOp == kOpResidRestrict;  // residual + restriction only (no sweep)
    constexpr bool kIR = kOp == kOpRefine;         // corrected phi + scaled residual + norm (no sweep)
    constexpr bool kGS = !kRR && !kIR;             // red/black updates
    constexpr int WX = TX + 4, WY = TY + 4, WP = WX / 2;   // ring-2 window, pairs per row
    constexpr int NB = kSweepTZMax + 6;                    // beta0 planes staged per chunk
    // Every LDS plane is double-buffered or tripled so that one barrier per
    // plane step suffices: a step reads what the previous step wrote and
    // writes buffers no one reads before the next barrier.
    __shared__ T sphi[2][WY][WX];                   // phi_in: plane t (read), t+1 (staged)
    __shared__ __align__(16) T sR[2][WY][WX];       // red values (kRR: residuals), planes t, t-1
    __shared__ T sbx[3][WY][WX];                    // low x-face coefficients, planes t+1, t, t-1
    __shared__ T sby[3][WY][WX];
    __shared__ T srho[kRho ? 2 : 1][kRho ? WY : 1][kRho ? WX : 1];   // rho: t+1 (read), t+2 (staged)
    __shared__ double sb0c[kRho ? NB : 1], sb0e[kRho ? NB : 1];

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int tx = tile % a.ntx;
    const int ty = (tile / a.ntx) % a.nty;
    const int tz = tile / (a.ntx * a.nty);
    // tiles cover ex x ey x ez cells from (ox, oy, oz): the whole level, or
    // (kBox) the interior of one box inside its ghosted array
    const int ox = kBox ? a.ox : 0, oy = kBox ? a.oy : 0, oz = kBox ? a.oz : 0;
    const int ex = kBox ? a.ex : nx, ey = kBox ? a.ey : ny, ez = kBox ? a.ez : nz;
    const int x0 = ox + tx * TX, y0 = oy + ty * TY;
    const int z0 = oz + tz * a.tz;
    const int z1 = min(z0 + a.tz, oz + ez);
    const int zb = z0 - 2;                    // first plane touched

    const int lp = threadIdx.x % WP;
    const int ly = threadIdx.x / WP;
    const int lx0 = 2 * lp;
    const int gx0 = x0 - 2 + lx0;             // even; the pair never straddles the wrap
    const int gy = y0 - 2 + ly;
    const int gxw = wrap3(gx0, nx);
    const int gyw = wrap3(gy, ny);
    const bool row_r1 = ly >= 1 && ly < WY - 1;
    const bool r1c0 = row_r1 && lp >= 1;            // even cell inside the ring-1 window
    const bool r1c1 = row_r1 && lp < WP - 1;        // odd cell
    const bool writes = ly >= 2 && ly < WY - 2 && lp >= 1 && lp <= WP - 2 && gx0 < ox + ex && gy < oy + ey;
    // 32-bit element offsets (a fused level holds fewer than 2^32 cells):
    // the per-plane index arithmetic stays in single scalar instructions
    const unsigned plane = (unsigned)nx * (unsigned)ny;
    const size_t col = (size_t)gyw * nx + gxw;
    // the plane part is uniform over the workgroup (scalar); the column part per lane
    auto base = [&](auto* p, int tw) { return p + (size_t)((unsigned)tw * plane); };
    const T h2 = a.h2;
    const T ih2 = T(1) / a.h2;
    const T half = T(0.5);
    const T cscale = kIn == kInCorrect ? (T)(1.0 / a.scales[0]) : T(0);    // exact: a power of two
    // outflow sides (kBnd): the level's per-cell boundary diagonal a.dg (zero
    // away from the outflow sides) is read, like f, two plane steps ahead of
    // its use, and only by threads whose cells can touch an outflow side:
    // x/y sides are fixed for the march (x low only for the even cell, x high
    // only for the odd one: nx is even), z sides occur on the first and last
    // plane only (uniform over the workgroup).
    bool bl = false;
    if constexpr (kBnd)
        bl = (gxw == 0 && a.bnd.s[0]) || (gxw + 1 == nx - 1 && a.bnd.s[1]) || (gyw == 0 && a.bnd.s[2]) ||
             (gyw == ny - 1 && a.bnd.s[3]);
    auto zbnd = [&](int tw) -> bool { return (tw == 0 && a.bnd.s[4]) || (tw == nz - 1 && a.bnd.s[5]); };

    // kInProlong: the parent cell on the next coarser level.  In a box
    // (kBox) the parent of a ghosted cell is that of its global cell (the
    // periodic image; beyond a wall the nearest cell, whose value meets a
    // zero wall coefficient), on the single coarser level of the domain.
    auto gwrap = [](int g, int n, int per) -> int {
        if (g < 0) return per ? g + n : 0;
        if (g >= n) return per ? g - n : n - 1;
        return g;
    };
    size_t ccol = 0, cplane = (size_t)(nx >> 1) * (ny >> 1);
    if (kIn == kInProlong) {
        if (kBox) {
            const int X = gwrap(a.go[0] + gxw - ox, a.gn[0], a.gp[0]);
            const int Y = gwrap(a.go[1] + gyw - oy, a.gn[1], a.gp[1]);
            ccol = (size_t)(Y >> 1) * (a.gn[0] >> 1) + (X >> 1);
            cplane = (size_t)(a.gn[0] >> 1) * (a.gn[1] >> 1);
        } else {
            ccol = (size_t)(gyw >> 1) * (nx >> 1) + (gxw >> 1);
        }
    }

    auto load_phi = [&](int t, T& v0, T& v1) {
        if (kIn == kInZero) {
            v0 = T(0);
            v1 = T(0);
            return;
        }
        int tw = wrap3(t, nz);
        ld2(base(a.phi_in, tw) + col, v0, v1);
        if (kIn == kInProlong) {
            const int Z = kBox ? gwrap(a.go[2] + tw - oz, a.gn[2], a.gp[2]) : tw;
            T c = a.phic[(size_t)(Z >> 1) * (kBox ? cplane : (plane >> 2)) + ccol];
            v0 = v0 + c;
            v1 = v1 + c;
        }
        if (kIn == kInCorrect) {
            float e0, e1;
            ld2(base(a.corr, tw) + col, e0, e1);
            v0 = v0 + cscale * (T)e0;
            v1 = v1 + cscale * (T)e1;
        }
    };
    auto load_f = [&](int t, T& v0, T& v1) {
        int tw = wrap3(t, nz);
        ld2(base(a.f, tw) + col, v0, v1);
    };
    // rho (finest level) or the stored low z-face coefficient of plane t
    auto load_q = [&](int t, T& v0, T& v1) {
        int tw = wrap3(t, nz);
        if (kRho) ld2(base(a.rho, tw) + col, v0, v1);
        else ld2(base(a.bz, tw) + col, v0, v1);
    };
    // low z-face coefficient of plane t from the queue values of planes t-1, t
    auto zface = [&](int t, T q_below, T q_here) -> T {
        if (!kRho) return q_here;
        const T b = pdiv((T)sb0e[t - zb], half * (q_below + q_here));
        const bool wall = kBox ? (t == a.wlo[2] || t == a.whi[2]) : (wrap3(t, nz) == 0 && !a.pz);
        return wall ? T(0) : b;                              // solid wall: no flux
    };

    // ---- prologue
    if (kRho) {
        for (int q = threadIdx.x; q < NB && zb + q <= z1 + 3; q += blockDim.x) {
            int qw = wrap3(zb + q, nz);
            sb0c[q] = a.b0c[qw];
            sb0e[q] = a.b0e[qw];
        }
    }
    // Loads in flight: step s issues plane s+3 (phi, stored bx/by), s+4 (rho
    // or stored bz) and s+2 (f) into one of two register sets, and step s+2
    // consumes that set before re-issuing into it, so every load has two
    // plane-steps of work to arrive.  Loads are always issued (clamped to the
    // last plane the chunk needs; those reloads hit in cache) so the sets are
    // plain load results the compiler never has to merge or copy early.
    struct Fly {
        T p0, p1;      // phi_in
        T q0, q1;      // rho (or stored bz)
        T f0, f1;      // f
        T x0, x1;      // stored bx (coarse levels)
        T y0, y1;      // stored by
        T g0, g1;      // boundary diagonal (kBnd)
    };
    auto issue = [&](int s, Fly& X) {
        load_phi(min(s + 3, z1 + 1), X.p0, X.p1);
        load_q(min(s + 4, z1 + 1), X.q0, X.q1);
        if (!kRho) {
            int tw = wrap3(min(s + 3, z1), nz);
            ld2(base(a.bx, tw) + col, X.x0, X.x1);
            ld2(base(a.by, tw) + col, X.y0, X.y1);
        }
        load_f(min(s + 2, z1), X.f0, X.f1);
        if constexpr (kBnd) {
            const int tw = wrap3(min(s + 2, z1), nz);
            X.g0 = T(0);
            X.g1 = T(0);
            if (bl || zbnd(tw)) ld2(base(a.dg, tw) + col, X.g0, X.g1);
        }
    };
    Fly A, B;
    issue(z0 - 3, A);                                  // consumed by step z0-1
    issue(z0 - 2, B);                                  // consumed by step z0
    // window before the first step's rotation
    T Pm0 = T(0), Pm1 = T(0), Pc0, Pc1, Pp0, Pp1;
    load_phi(z0 - 2, Pc0, Pc1);
    load_phi(z0 - 1, Pp0, Pp1);
    T Rc0, Rc1, Rp0, Rp1, Rq0, Rq1;                    // rho (or bz) of planes t, t+1, t+2 after a rotation
    load_q(z0 - 2, Rc0, Rc1);
    load_q(z0 - 1, Rp0, Rp1);
    load_q(z0, Rq0, Rq1);
    T Fm0 = T(0), Fm1 = T(0), Fc0 = T(0), Fc1 = T(0);
    T Gm0 = T(0), Gm1 = T(0), Gc0 = T(0), Gc1 = T(0);  // boundary diagonal of planes t-1, t (kBnd)
    T cx0 = T(0), cx1 = T(0), cy0 = T(0), cy1 = T(0);  // stored x/y coefficients of plane t+1

    // x/y low-face coefficients of plane t into LDS slot s from the staged rho
    // plane (buffer b); (r0, r1) is the thread's own pair of that plane
    auto rho_coeffs = [&](int t, int s, int b, T r0, T r1) {
        const T b0 = (T)sb0c[t - zb];
        const T rc[2] = {r0, r1};
        // the window's first row/column has no low neighbour and is never read
        const T rl[2] = {srho[b][ly][lx0 > 0 ? lx0 - 1 : 0], r0};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int lx = lx0 + c;
            const T cx = pdiv(b0, half * (rl[c] + rc[c]));
            const T cy = pdiv(b0, half * (srho[b][ly > 0 ? ly - 1 : 0][lx] + rc[c]));
            const bool xwall = kBox ? (gxw + c == a.wlo[0] || gxw + c == a.whi[0]) : ((gxw + c == 0) && !a.px);
            const bool ywall = kBox ? (gyw == a.wlo[1] || gyw == a.whi[1]) : (gyw == 0 && !a.py);
            sbx[s][ly][lx] = xwall ? T(0) : cx;
            sby[s][ly][lx] = ywall ? T(0) : cy;
        }
    };
    // LDS before the first step (t = z0-1): phi_in of z0-1, coefficients of
    // z0-1, rho of z0
    sphi[0][ly][lx0] = Pp0;
    sphi[0][ly][lx0 + 1] = Pp1;
    if (kRho) {
        srho[0][ly][lx0] = Rp0;
        srho[0][ly][lx0 + 1] = Rp1;
        __syncthreads();                               // beta0 and rho of z0-1 staged
        rho_coeffs(z0 - 1, 0, 0, Rp0, Rp1);
        srho[1][ly][lx0] = Rq0;
        srho[1][ly][lx0 + 1] = Rq1;
    } else {
        int tw = wrap3(z0 - 1, nz);
        T t0, t1;
        ld2(base(a.bx, tw) + col, t0, t1);
        sbx[0][ly][lx0] = t0;
        sbx[0][ly][lx0 + 1] = t1;
        ld2(base(a.by, tw) + col, t0, t1);
        sby[0][ly][lx0] = t0;
        sby[0][ly][lx0 + 1] = t1;
    }
    T bm0 = T(0), bm1 = T(0), bc0 = T(0), bc1 = T(0);
    T bp0 = zface(z0 - 1, Rc0, Rp0), bp1 = zface(z0 - 1, Rc1, Rp1);   // low face of plane z0-1
    __syncthreads();

    T Rmm = T(0), Rm = T(0);
    // residual of phi_in (kNorm, kRR) or of the corrected phi (kIR):
    // r = f - (sum_f b (phi_nb - phi_c)) / h^2 in the reference face order
    // only the sum of squares is kept: a non-finite residual makes it non-finite
    double nrm2 = 0.0;
    const double rscale = kIR ? a.scales[1] : 0.0;
    auto resid_at = [&](int c, int t, int s_t, int b, T pm, T pc, T pp, T bzl, T bzh, T fc) -> T {
        const int lx = lx0 + c;
        T r = sbx[s_t][ly][lx] * (sphi[b][ly][lx - 1] - pc);
        r = r + sbx[s_t][ly][lx + 1] * (sphi[b][ly][lx + 1] - pc);
        r = r + sby[s_t][ly][lx] * (sphi[b][ly - 1][lx] - pc);
        r = r + sby[s_t][ly + 1][lx] * (sphi[b][ly + 1][lx] - pc);
        r = r + bzl * (pm - pc);
        r = r + bzh * (pp - pc);
        if constexpr (kBnd) r = r - (c ? Gc1 : Gc0) * pc;
        return fc - r * ih2;
    };
    auto accumulate = [&](T r) {
        const double res = (double)r;
        nrm2 += res * res;
    };
    // restriction (kRR): the even-row thread of each 2x2 column block sums the
    // 8 children in the reference order (x fastest, then y, then z)
    T racc = T(0);
    const bool rrow = (ly & 1) == 0;           // gy = y0 - 2 + ly is even
    // the coarse cell (kBox: on the domain's single coarser level; only box
    // interior cells restrict, so no wrap is needed)
    const size_t ccols = kBox ? (size_t)(a.gn[0] >> 1) * (a.gn[1] >> 1) : (size_t)(nx >> 1) * (ny >> 1);
    const size_t cc = kBox ? (size_t)((a.go[1] + gyw - oy) >> 1) * (a.gn[0] >> 1) + ((a.go[0] + gxw - ox) >> 1)
                           : (size_t)(gyw >> 1) * (nx >> 1) + (gxw >> 1);
    // Step j = t - (z0 - 1) of the march.  The LDS planes are chosen by j
    // mod 2 and j mod 3 (any fixed relabelling of the buffers serves) from
    // J = j mod 6, which the six-step unrolled loop passes as a compile-time
    // constant: every LDS address is then a constant offset, and the z
    // windows rotate through registers without copies.  The variants that
    // would spill unrolled pass J at run time: the outflow ones (kBnd) and
    // the FP64 64x8 ones, which are held to 128 registers; so does the FP32
    // zero-start sweep, whose 64x16 tiles fit two workgroups per CU only
    // within 80 registers (unrolled it takes 84).
    auto step = [&](int t, auto J, Fly& X) {
        const int jj = static_cast<int>(J);
        const int m3 = jj % 3;
        // 0. slide the z window, taking in the set issued two steps ago:
        //    phi[t+1], rho[t+2] (or bz[t+2]), f[t], bx/by[t+1]; then re-issue
        Fm0 = Fc0; Fm1 = Fc1;
        Fc0 = X.f0; Fc1 = X.f1;
        if constexpr (kBnd) {
            Gm0 = Gc0; Gm1 = Gc1;
            Gc0 = X.g0; Gc1 = X.g1;
        }
        Pm0 = Pc0; Pm1 = Pc1;
        Pc0 = Pp0; Pc1 = Pp1;
        Pp0 = X.p0; Pp1 = X.p1;
        Rc0 = Rp0; Rc1 = Rp1;
        Rp0 = Rq0; Rp1 = Rq1;
        Rq0 = X.q0; Rq1 = X.q1;
        bm0 = bc0; bm1 = bc1;
        bc0 = bp0; bc1 = bp1;
        bp0 = zface(t + 1, Rc0, Rp0);
        bp1 = zface(t + 1, Rc1, Rp1);
        if (!kRho) {
            cx0 = X.x0; cx1 = X.x1;
            cy0 = X.y0; cy1 = X.y1;
        }
        issue(t, X);                             // consumed by step t+2
        const int s_t = m3, s_p = m3 == 2 ? 0 : m3 + 1, s_m = m3 == 0 ? 2 : m3 - 1;
        const int cur = jj & 1, nxt = cur ^ 1;
        const int rsel = (gy + t) & 1;           // red cell of the pair at plane t (black at t-1)
        // 1. x/y coefficients of plane t+1 (read by the next step)
        if (t + 1 <= z1) {
            if (kRho) {
                rho_coeffs(t + 1, s_p, nxt, Rp0, Rp1);
            } else {
                sbx[s_p][ly][lx0] = cx0;
                sbx[s_p][ly][lx0 + 1] = cx1;
                sby[s_p][ly][lx0] = cy0;
                sby[s_p][ly][lx0 + 1] = cy1;
            }
        }
        // 2. red update at plane t on the tile plus one ring
        const int lxr = lx0 + rsel;
        T Rcur = rsel ? Pc1 : Pc0;
        T rred = T(0);                           // kNorm: residual of phi_in at the red cell
        if (kGS && (rsel ? r1c1 : r1c0)) {
            const T bxl = sbx[s_t][ly][lxr], bxh = sbx[s_t][ly][lxr + 1];
            const T byl = sby[s_t][ly][lxr], byh = sby[s_t][ly + 1][lxr];
            const T bzl = rsel ? bc1 : bc0, bzh = rsel ? bp1 : bp0;
            T num = bxl * sphi[cur][ly][lxr - 1];
            num = num + bxh * sphi[cur][ly][lxr + 1];
            num = num + byl * sphi[cur][ly - 1][lxr];
            num = num + byh * sphi[cur][ly + 1][lxr];
            num = num + bzl * (rsel ? Pm1 : Pm0);
            num = num + bzh * (rsel ? Pp1 : Pp0);
            T den = bxl + bxh;
            den = den + byl;
            den = den + byh;
            den = den + bzl;
            den = den + bzh;
            if constexpr (kBnd) den = den + (rsel ? Gc1 : Gc0);
            const T pin = Rcur;
            Rcur = pdiv(num - h2 * (rsel ? Fc1 : Fc0), den);
            // the update solves den phi_new = num - h^2 f, so f - L phi_in =
            // den (phi_in - phi_new) / h^2 (exact up to rounding)
            if (kNorm) rred = den * (pin - Rcur) * ih2;
        }
        if (kGS) sR[cur][ly][lxr] = Rcur;
        if (kNorm && t >= z0 && t < z1 && writes) {
            accumulate(rred);
            const int cb = 1 - rsel;             // black cell of the pair: full evaluation
            accumulate(resid_at(cb, t, s_t, cur, cb ? Pm1 : Pm0, cb ? Pc1 : Pc0, cb ? Pp1 : Pp0, cb ? bc1 : bc0,
                                cb ? bp1 : bp0, cb ? Fc1 : Fc0));
        }
        if (kRR && t >= z0 && t < z1 && writes) {
            sR[cur][ly][lx0] = resid_at(0, t, s_t, cur, Pm0, Pc0, Pp0, bc0, bp0, Fc0);
            sR[cur][ly][lx0 + 1] = resid_at(1, t, s_t, cur, Pm1, Pc1, Pp1, bc1, bp1, Fc1);
        }
        if (kIR && t >= z0 && t < z1 && writes) {
            const T r0 = resid_at(0, t, s_t, cur, Pm0, Pc0, Pp0, bc0, bp0, Fc0);
            const T r1 = resid_at(1, t, s_t, cur, Pm1, Pc1, Pp1, bc1, bp1, Fc1);
            const double d0 = (double)r0, d1 = (double)r1;
            nrm2 += d0 * d0;
            nrm2 += d1 * d1;
            st2(base(a.phi_out, t) + col, Pc0, Pc1);
            st2(base(a.r32, t) + col, (float)(rscale * d0), (float)(rscale * d1));
        }
        // 3. (kRR) restriction of plane t-1, whose residuals the previous step wrote
        const int tb = t - 1;
        if (kRR && tb >= z0 && tb < z1 && writes && rrow) {
            const int pb = nxt;                 // plane t-1
            if (((tb - z0) & 1) == 0) racc = T(0);
            racc = racc + sR[pb][ly][lx0];
            racc = racc + sR[pb][ly][lx0 + 1];
            racc = racc + sR[pb][ly + 1][lx0];
            racc = racc + sR[pb][ly + 1][lx0 + 1];
            if (((tb - z0) & 1) == 1) {
                const size_t ci = (size_t)((kBox ? a.go[2] + tb - oz : tb) >> 1) * ccols + cc;
                a.fc[ci] = T(0.125) * racc;
                a.phic_out[ci] = T(0);
            }
        }
        // 4. black update at plane t-1 on the tile; write the pair of plane t-1
        if (kGS && tb >= z0 && writes) {
            const int sb = nxt;                 // plane t-1
            const int lxb = lx0 + rsel;
            const T bxl = sbx[s_m][ly][lxb], bxh = sbx[s_m][ly][lxb + 1];
            const T byl = sby[s_m][ly][lxb], byh = sby[s_m][ly + 1][lxb];
            const T bzl = rsel ? bm1 : bm0, bzh = rsel ? bc1 : bc0;
            T num = bxl * sR[sb][ly][lxb - 1];
            num = num + bxh * sR[sb][ly][lxb + 1];
            num = num + byl * sR[sb][ly - 1][lxb];
            num = num + byh * sR[sb][ly + 1][lxb];
            num = num + bzl * Rmm;
            num = num + bzh * Rcur;
            T den = bxl + bxh;
            den = den + byl;
            den = den + byh;
            den = den + bzl;
            den = den + bzh;
            if constexpr (kBnd) den = den + (rsel ? Gm1 : Gm0);
            const T blk = pdiv(num - h2 * (rsel ? Fm1 : Fm0), den);
            T* dst = base(a.phi_out, tb) + col;
            if (rsel) st2(dst, Rm, blk);
            else st2(dst, blk, Rm);
        }
        Rmm = Rm;
        Rm = Rcur;
        // 5. stage phi_in of plane t+1 and rho of plane t+2 for the next step
        if (t + 1 <= z1) {
            sphi[nxt][ly][lx0] = Pp0;
            sphi[nxt][ly][lx0 + 1] = Pp1;
            if (kRho) {
                srho[cur][ly][lx0] = Rq0;
                srho[cur][ly][lx0 + 1] = Rq1;
            }
        }
        __syncthreads();
    };
    using std::integral_constant;
    int t = z0 - 1;
    constexpr bool kRunPhase = kBnd || (sizeof(T) == 8 && TX == 64 && TY == 8) || (sizeof(T) == 4 && kIn == kInZero);
    if constexpr (kRunPhase) {
        int j = 0;
        for (; t + 1 <= z1; t += 2) {
            step(t, j, A);
            step(t + 1, j + 1, B);
            j = j == 4 ? 0 : j + 2;
        }
        if (t <= z1) step(t, j, A);
    } else {
        for (; t + 5 <= z1; t += 6) {
            step(t, integral_constant<int, 0>{}, A);
            step(t + 1, integral_constant<int, 1>{}, B);
            step(t + 2, integral_constant<int, 2>{}, A);
            step(t + 3, integral_constant<int, 3>{}, B);
            step(t + 4, integral_constant<int, 4>{}, A);
            step(t + 5, integral_constant<int, 5>{}, B);
        }
        if (t <= z1) step(t, integral_constant<int, 0>{}, A);
        if (t + 1 <= z1) step(t + 1, integral_constant<int, 1>{}, B);
        if (t + 2 <= z1) step(t + 2, integral_constant<int, 2>{}, A);
        if (t + 3 <= z1) step(t + 3, integral_constant<int, 3>{}, B);
        if (t + 4 <= z1) step(t + 4, integral_constant<int, 4>{}, A);
    }
    if (kNorm || kIR) {
        // fixed-order block reduction into this tile's partial row (in the
        // red-value buffer, free after the last step's barrier)
        double* red = reinterpret_cast<double*>(&sR[0][0][0]);
        static_assert(sizeof(sR) >= 256 * sizeof(double), "reduction buffer");
        const int nt = blockDim.x;
        for (int i = threadIdx.x; i < 256; i += nt) red[i] = 0.0;   // every slot, also when nt < 256
        __syncthreads();
        for (int k = 0; k < nt; k += 256) {
            if (threadIdx.x >= k && threadIdx.x < k + 256) red[threadIdx.x - k] += nrm2;
            __syncthreads();
        }
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double* row = a.partials + (size_t)tile * kReduceWidth;
            row[0] = red[0];
            row[1] = 0.0;
            row[2] = 0.0;
            row[3] = 0.0;
        }
    }
}

// 64x8-tile FP64 variants are held to 128 VGPRs (4 waves per SIMD), so that
// two of their workgroups (7 waves and 79 KB of LDS each) share a CU; left
// alone the compiler gives several of them a few more registers, which
// halves the workgroups per CU.  Smaller tiles are limited by LDS first.
// The outflow-side variants (kBnd) need more registers and are left alone.
template <typename T, int TX, int TY, bool kBnd>
struct SweepWaves {
    static constexpr int value = (sizeof(T) == 8 && TX == 64 && TY == 8 && !kBnd) ? 4 : 1;
};
#define MG_SWEEP_WAVES(B) __attribute__((amdgpu_waves_per_eu(SweepWaves<T, TX, TY, B>::value)))

// kBnd: the level has outflow sides (their boundary faces add to the
// diagonal); a separate instantiation so the other kernels carry none of it.
template <typename T, int TX, int TY, bool kRho, int kIn, int kOp, bool kBnd>
__global__ __launch_bounds__((TX / 2 + 2) * (TY + 4)) MG_SWEEP_WAVES(kBnd) void k_sweep(SweepArgs<T> a) {
    sweep_body<T, TX, TY, kRho, kIn, kOp, kBnd>(a, xcd_tile(blockIdx.x, gridDim.x));
}

// Boxes of one shape stored one after another bstride elements apart, each
// inside its ghosted array (a.nx, a.ny, a.nz: the ghosted dims; a.ox..:
// the ghost width; a.ex..: the box cells): workgroup tiles enumerate
// (box, tile), every box with its own pointers.  Stored coefficients, plain
// input, one sweep; kOp = kOpSweepNorm also writes the per-tile partial
// rows of the residual of its input, box b's after the rows of the boxes
// before it.  kRho: coefficients from the boxes' ghosted rho and per-box
// beta0 (a.b0c, a.b0e: g.b0stride entries per box, indexed by ghosted
// plane), with the domain's walls placed per box.
template <typename T, int TX, int TY, int kOp, bool kRho, int kIn>
__global__ __launch_bounds__((TX / 2 + 2) * (TY + 4)) __attribute__((amdgpu_waves_per_eu(
    SweepWaves<T, TX, TY, false>::value))) void k_sweep_boxes(SweepArgs<T> a, BoxGeom g, int tpb, size_t bstride) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int b = t / tpb;
    const size_t off = (size_t)b * bstride;
    SweepArgs<T> c = a;
    c.phi_in = a.phi_in + off;
    c.phi_out = a.phi_out + off;
    c.f = a.f + off;
    if (kIn == kInCorrect) c.corr = a.corr + off;          // the FP32 correction, in the same box layout
    if (kOp == kOpRefine) c.r32 = a.r32 + off;
    const int bc[3] = {b % g.nb[0], (b / g.nb[0]) % g.nb[1], b / (g.nb[0] * g.nb[1])};
    // this box's cells (the launch's tiles cover a full box; a smaller last
    // box leaves the tiles past its cells without writes)
    const int E[3] = {min(g.box[0], g.n[0] - bc[0] * g.box[0]), min(g.box[1], g.n[1] - bc[1] * g.box[1]),
                      min(g.box[2], g.n[2] - bc[2] * g.box[2])};
    const int O[3] = {a.ox, a.oy, a.oz};
    c.ex = E[0];
    c.ey = E[1];
    c.ez = E[2];
    if (kIn == kInProlong || kOp == kOpResidRestrict) {
        for (int d = 0; d < 3; ++d) {
            c.go[d] = bc[d] * g.box[d];
            c.gn[d] = g.n[d];
            c.gp[d] = g.per[d];
        }
    }
    if (kRho) {
        c.rho = a.rho + off;
        c.b0c = a.b0c + (size_t)b * g.b0stride;
        c.b0e = a.b0e + (size_t)b * g.b0stride;
        for (int d = 0; d < 3; ++d) {
            c.wlo[d] = (!g.per[d] && bc[d] == 0) ? O[d] : -1;
            c.whi[d] = (!g.per[d] && bc[d] == g.nb[d] - 1) ? O[d] + E[d] : -1;
        }
    } else {
        c.bx = a.bx + off;
        c.by = a.by + off;
        c.bz = a.bz + off;
    }
    if (kOp == kOpSweepNorm || kOp == kOpRefine) c.partials = a.partials + (size_t)b * tpb * kReduceWidth;
    sweep_body<T, TX, TY, kRho, kIn, kOp, false, true>(c, t - b * tpb);
}

// Batched form: tile b of the launch is tile tmap[b].y of problem tmap[b].x
// (one load instead of a search over the problems' tile ranges).
template <typename T, int TX, int TY, bool kRho, int kIn, int kOp = kOpSweep>
__global__ __launch_bounds__((TX / 2 + 2) * (TY + 4)) MG_SWEEP_WAVES(false) void k_sweep_multi(const SweepArgs<T>* __restrict__ descs,
                                                                         const int2* __restrict__ tmap) {
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int2 m = tmap[b];
    const SweepArgs<T> a = descs[m.x];
    sweep_body<T, TX, TY, kRho, kIn, kOp, false>(a, m.y);   // batches have no outflow sides
}

template <typename T, int TX, int TY, bool kRho, int kIn, int kOp = kOpSweep>
hipError_t launch_multi_t(const SweepArgs<T>* d, const int2* tmap, int tiles, hipStream_t st) {
    hipLaunchKernelGGL((k_sweep_multi<T, TX, TY, kRho, kIn, kOp>), dim3(tiles), dim3((TX / 2 + 2) * (TY + 4)), 0,
                       st, d, tmap);
    return hipGetLastError();
}

template <typename T, int TX, int TY, bool kRho, int kIn, int kOp = kOpSweep>
hipError_t launch_t(const SweepArgs<T>& a0, int tzc, hipStream_t st, int* nblocks = nullptr) {
    SweepArgs<T> a = a0;
    a.tz = tzc;
    a.ntx = (a.nx + TX - 1) / TX;
    a.nty = (a.ny + TY - 1) / TY;
    int ntz = (a.nz + tzc - 1) / tzc;
    int blocks = a.ntx * a.nty * ntz;
    if (nblocks) *nblocks = blocks;
    if (a.has_bnd)
        hipLaunchKernelGGL((k_sweep<T, TX, TY, kRho, kIn, kOp, true>), dim3(blocks), dim3((TX / 2 + 2) * (TY + 4)),
                           0, st, a);
    else
        hipLaunchKernelGGL((k_sweep<T, TX, TY, kRho, kIn, kOp, false>), dim3(blocks), dim3((TX / 2 + 2) * (TY + 4)),
                           0, st, a);
    return hipGetLastError();
}

template <typename T, int TX, int TY>
hipError_t launch_mode(const SweepArgs<T>& a, bool use_rho, int in_mode, int tzc, hipStream_t st) {
    if (use_rho) {
        switch (in_mode) {
            case kInZero: return launch_t<T, TX, TY, true, kInZero>(a, tzc, st);
            case kInPlain: return launch_t<T, TX, TY, true, kInPlain>(a, tzc, st);
            default: return launch_t<T, TX, TY, true, kInProlong>(a, tzc, st);
        }
    }
    switch (in_mode) {
        case kInZero: return launch_t<T, TX, TY, false, kInZero>(a, tzc, st);
        case kInPlain: return launch_t<T, TX, TY, false, kInPlain>(a, tzc, st);
        default: return launch_t<T, TX, TY, false, kInProlong>(a, tzc, st);
    }
}

}  // namespace

void sweep_force_config(int cfg) { tune_force(cfg); }

void sweep_record_tuned(int nx, int ny, int nz, bool rho, bool dbl, int cfg, bool coarse) {
    tune_put(nx, ny, nz, rho, dbl, coarse, cfg);
}

unsigned sweep_tune_epoch() { return tune_epoch(); }

int sweep_tuned_count() { return tune_count(); }

bool sweep_cfg_fits(int nx, int ny, int cfg) {
    return cfg >= 0 && cfg < kNumSweepCfg && nx >= kSweepCfgs[cfg].tx && ny >= kSweepCfgs[cfg].ty;
}

int sweep_config_for(int nx, int ny, int nz, bool rho, bool dbl, bool coarse) {
    const int forced = tune_forced();
    if (forced >= 0 && sweep_cfg_fits(nx, ny, forced)) return forced;
    const int tuned = tune_find(nx, ny, nz, rho, dbl, coarse);
    if (tuned >= 0) return tuned;
    // untuned shapes: choices measured on MI355X for cubic levels.  On the
    // largest boxes 64x16-cell tiles (the halo share of the loads and of the
    // redundant red updates is a third lower than with 64x8 tiles): FP64
    // with 64-plane chunks (one 132 KB workgroup per CU), FP32 with 32-plane
    // chunks; then 32x8 tiles with shallower z-chunks so small levels still
    // fill the 256 CUs.  Coarse levels of a single-problem V-cycle go
    // shallower still (a 64^3 level in 4-plane chunks, a 32^3 level in 32x4
    // tiles of 4 planes: there the march through the planes, not the bytes,
    // sets the time); batches, which fill the CUs with many problems, keep
    // the deeper chunks.
    const double cells = (double)nx * ny * nz;
    if (nx >= 64 && ny >= 16 && cells >= 8.0e6) {
        if (dbl && nz >= 64) return 11;
        if (!dbl) return 9;
    }
    if (nx >= 64 && cells >= 8.0e6) return 2;
    if (nx >= 32 && ny >= 8) {
        if (cells >= 1.0e6) return 6;
        if (!coarse) return 7;
        if (cells >= 1.0e5) return 12;
    }
    if (coarse && nx >= 32 && ny >= 4 && cells < 1.0e5) return 13;
    return 5;
}

template <typename T>
bool sweep_fusable(int nx, int ny, int nz) {
    return nx >= kSweepTX && ny >= kSweepTY && nz >= 4 && nx % 2 == 0 && ny % 2 == 0 && nz % 2 == 0 &&
           (unsigned long long)nx * ny * nz < (1ull << 32);      // 32-bit element offsets
}

template <typename T>
hipError_t launch_sweep(const SweepArgs<T>& a, bool use_rho, int in_mode, int cfg, hipStream_t st) {
    const SweepCfg& c = kSweepCfgs[cfg];
    if (a.nx < c.tx || a.ny < c.ty) return hipErrorInvalidValue;
    switch (cfg) {
        case 0: return launch_mode<T, 32, 8>(a, use_rho, in_mode, c.tz, st);
        case 1: return launch_mode<T, 32, 8>(a, use_rho, in_mode, c.tz, st);
        case 2: return launch_mode<T, 64, 8>(a, use_rho, in_mode, c.tz, st);
        case 8: return launch_mode<T, 64, 8>(a, use_rho, in_mode, c.tz, st);
        case 9: return launch_mode<T, 64, 16>(a, use_rho, in_mode, c.tz, st);
        case 10: return launch_mode<T, 32, 32>(a, use_rho, in_mode, c.tz, st);
        case 11: return launch_mode<T, 64, 16>(a, use_rho, in_mode, c.tz, st);
        case 3: return launch_mode<T, 32, 16>(a, use_rho, in_mode, c.tz, st);
        case 4: return launch_mode<T, 64, 4>(a, use_rho, in_mode, c.tz, st);
        case 5: return launch_mode<T, 32, 4>(a, use_rho, in_mode, c.tz, st);
        case 13: return launch_mode<T, 32, 4>(a, use_rho, in_mode, c.tz, st);
        default: return launch_mode<T, 32, 8>(a, use_rho, in_mode, c.tz, st);
    }
}

template <bool kRho>
hipError_t launch_sweep_norm_t(const SweepArgs<double>& a, int cfg, int* nparts, hipStream_t st) {
    const SweepCfg& c = kSweepCfgs[cfg];
    constexpr int N = kOpSweepNorm;
    switch (cfg) {
        case 0: return launch_t<double, 32, 8, kRho, kInPlain, N>(a, c.tz, st, nparts);
        case 1: return launch_t<double, 32, 8, kRho, kInPlain, N>(a, c.tz, st, nparts);
        case 2: return launch_t<double, 64, 8, kRho, kInPlain, N>(a, c.tz, st, nparts);
        case 8: return launch_t<double, 64, 8, kRho, kInPlain, N>(a, c.tz, st, nparts);
        case 9: return launch_t<double, 64, 16, kRho, kInPlain, N>(a, c.tz, st, nparts);
        case 10: return launch_t<double, 32, 32, kRho, kInPlain, N>(a, c.tz, st, nparts);
        case 11: return launch_t<double, 64, 16, kRho, kInPlain, N>(a, c.tz, st, nparts);
        case 3: return launch_t<double, 32, 16, kRho, kInPlain, N>(a, c.tz, st, nparts);
        case 4: return launch_t<double, 64, 4, kRho, kInPlain, N>(a, c.tz, st, nparts);
        case 5: return launch_t<double, 32, 4, kRho, kInPlain, N>(a, c.tz, st, nparts);
        case 13: return launch_t<double, 32, 4, kRho, kInPlain, N>(a, c.tz, st, nparts);
        default: return launch_t<double, 32, 8, kRho, kInPlain, N>(a, c.tz, st, nparts);
    }
}

hipError_t launch_sweep_norm(const SweepArgs<double>& a, bool use_rho, int cfg, int* nparts, hipStream_t st) {
    const SweepCfg& c = kSweepCfgs[cfg];
    if (a.nx < c.tx || a.ny < c.ty) return hipErrorInvalidValue;
    return use_rho ? launch_sweep_norm_t<true>(a, cfg, nparts, st) : launch_sweep_norm_t<false>(a, cfg, nparts, st);
}

template <typename T, bool kRho>
hipError_t launch_resid_restrict_tiled_t(const SweepArgs<T>& a, int cfg, hipStream_t st) {
    const SweepCfg& c = kSweepCfgs[cfg];
    constexpr int R = kOpResidRestrict;
    switch (cfg) {
        case 0: return launch_t<T, 32, 8, kRho, kInPlain, R>(a, c.tz, st);
        case 1: return launch_t<T, 32, 8, kRho, kInPlain, R>(a, c.tz, st);
        case 2: return launch_t<T, 64, 8, kRho, kInPlain, R>(a, c.tz, st);
        case 8: return launch_t<T, 64, 8, kRho, kInPlain, R>(a, c.tz, st);
        case 9: return launch_t<T, 64, 16, kRho, kInPlain, R>(a, c.tz, st);
        case 10: return launch_t<T, 32, 32, kRho, kInPlain, R>(a, c.tz, st);
        case 11: return launch_t<T, 64, 16, kRho, kInPlain, R>(a, c.tz, st);
        case 3: return launch_t<T, 32, 16, kRho, kInPlain, R>(a, c.tz, st);
        case 4: return launch_t<T, 64, 4, kRho, kInPlain, R>(a, c.tz, st);
        case 5: return launch_t<T, 32, 4, kRho, kInPlain, R>(a, c.tz, st);
        case 13: return launch_t<T, 32, 4, kRho, kInPlain, R>(a, c.tz, st);
        default: return launch_t<T, 32, 8, kRho, kInPlain, R>(a, c.tz, st);
    }
}

template <typename T>
hipError_t launch_resid_restrict_tiled(const SweepArgs<T>& a, bool use_rho, int cfg, hipStream_t st) {
    const SweepCfg& c = kSweepCfgs[cfg];
    if (a.nx < c.tx || a.ny < c.ty) return hipErrorInvalidValue;
    return use_rho ? launch_resid_restrict_tiled_t<T, true>(a, cfg, st)
                   : launch_resid_restrict_tiled_t<T, false>(a, cfg, st);
}

template <bool kRho>
hipError_t launch_refine_t(const SweepArgs<double>& a, int cfg, int* nparts, hipStream_t st) {
    const SweepCfg& c = kSweepCfgs[cfg];
    constexpr int R = kOpRefine, I = kInCorrect;
    switch (cfg) {
        case 0: return launch_t<double, 32, 8, kRho, I, R>(a, c.tz, st, nparts);
        case 1: return launch_t<double, 32, 8, kRho, I, R>(a, c.tz, st, nparts);
        case 2: return launch_t<double, 64, 8, kRho, I, R>(a, c.tz, st, nparts);
        case 8: return launch_t<double, 64, 8, kRho, I, R>(a, c.tz, st, nparts);
        case 9: return launch_t<double, 64, 16, kRho, I, R>(a, c.tz, st, nparts);
        case 10: return launch_t<double, 32, 32, kRho, I, R>(a, c.tz, st, nparts);
        case 11: return launch_t<double, 64, 16, kRho, I, R>(a, c.tz, st, nparts);
        case 3: return launch_t<double, 32, 16, kRho, I, R>(a, c.tz, st, nparts);
        case 4: return launch_t<double, 64, 4, kRho, I, R>(a, c.tz, st, nparts);
        case 5: return launch_t<double, 32, 4, kRho, I, R>(a, c.tz, st, nparts);
        case 13: return launch_t<double, 32, 4, kRho, I, R>(a, c.tz, st, nparts);
        default: return launch_t<double, 32, 8, kRho, I, R>(a, c.tz, st, nparts);
    }
}

hipError_t launch_refine(const SweepArgs<double>& a, bool use_rho, int cfg, int* nparts, hipStream_t st) {
    const SweepCfg& c = kSweepCfgs[cfg];
    if (a.nx < c.tx || a.ny < c.ty) return hipErrorInvalidValue;
    return use_rho ? launch_refine_t<true>(a, cfg, nparts, st) : launch_refine_t<false>(a, cfg, nparts, st);
}

template <typename T, int TX, int TY>
hipError_t launch_multi_mode(const SweepArgs<T>* d, const int2* tmap, int tiles, bool use_rho,
                             int in_mode, int op, hipStream_t st) {
    if (use_rho) {
        if constexpr (std::is_same<T, double>::value) {
            if (op == kOpSweepNorm)
                return launch_multi_t<T, TX, TY, true, kInPlain, kOpSweepNorm>(d, tmap, tiles, st);
            if (op == kOpRefine)
                return launch_multi_t<T, TX, TY, true, kInCorrect, kOpRefine>(d, tmap, tiles, st);
        } else {
            if (op == kOpSweepNorm || op == kOpRefine) return hipErrorInvalidValue;
        }
        if (op == kOpResidRestrict)
            return launch_multi_t<T, TX, TY, true, kInPlain, kOpResidRestrict>(d, tmap, tiles, st);
        switch (in_mode) {
            case kInZero: return launch_multi_t<T, TX, TY, true, kInZero>(d, tmap, tiles, st);
            case kInPlain: return launch_multi_t<T, TX, TY, true, kInPlain>(d, tmap, tiles, st);
            default: return launch_multi_t<T, TX, TY, true, kInProlong>(d, tmap, tiles, st);
        }
    }
    if (op == kOpResidRestrict)
        return launch_multi_t<T, TX, TY, false, kInPlain, kOpResidRestrict>(d, tmap, tiles, st);
    switch (in_mode) {
        case kInZero: return launch_multi_t<T, TX, TY, false, kInZero>(d, tmap, tiles, st);
        case kInPlain: return launch_multi_t<T, TX, TY, false, kInPlain>(d, tmap, tiles, st);
        default: return launch_multi_t<T, TX, TY, false, kInProlong>(d, tmap, tiles, st);
    }
}

template <typename T>
hipError_t launch_sweep_multi(const SweepArgs<T>* d, const int2* tmap, int tiles, bool use_rho, int in_mode, int op,
                              int cfg, hipStream_t st) {
    if (tiles <= 0) return hipSuccess;
    const SweepCfg& c = kSweepCfgs[cfg];
    if (c.tx == 32 && c.ty == 8) return launch_multi_mode<T, 32, 8>(d, tmap, tiles, use_rho, in_mode, op, st);
    if (c.tx == 64 && c.ty == 8) return launch_multi_mode<T, 64, 8>(d, tmap, tiles, use_rho, in_mode, op, st);
    if (c.tx == 32 && c.ty == 4) return launch_multi_mode<T, 32, 4>(d, tmap, tiles, use_rho, in_mode, op, st);
    if (c.tx == 64 && c.ty == 16) return launch_multi_mode<T, 64, 16>(d, tmap, tiles, use_rho, in_mode, op, st);
    return hipErrorInvalidValue;      // other tile shapes are single-problem only
}

void sweep_geometry(SweepArgs<double>& a, int cfg) {
    const SweepCfg& c = kSweepCfgs[cfg];
    a.tz = c.tz;
    a.ntx = (a.nx + c.tx - 1) / c.tx;
    a.nty = (a.ny + c.ty - 1) / c.ty;
}
void sweep_geometry(SweepArgs<float>& a, int cfg) {
    const SweepCfg& c = kSweepCfgs[cfg];
    a.tz = c.tz;
    a.ntx = (a.nx + c.tx - 1) / c.tx;
    a.nty = (a.ny + c.ty - 1) / c.ty;
}

int sweep_boxes_tiles(int bx, int by, int bz) {
    const bool wide = bx % 64 == 0 && by % 16 == 0;
    const int TXc = wide ? 64 : 32, TYc = wide ? 16 : 8, tzc = std::min(bz, kSweepTZMax);
    return ((bx + TXc - 1) / TXc) * ((by + TYc - 1) / TYc) * ((bz + tzc - 1) / tzc);
}

bool sweep_boxes_fit(int bx, int by, int bz) {
    return bx >= kSweepTX && by >= 8 && bz >= 4 && bx % 2 == 0 && by % 2 == 0 && bz % 2 == 0;
}

template <typename T, int TX, int TY, int kOp, int kIn>
void launch_boxes_t(const SweepArgs<T>& a, const BoxGeom& g, int tpb, size_t bstride, unsigned blocks,
                    hipStream_t st) {
    if (a.rho)
        hipLaunchKernelGGL((k_sweep_boxes<T, TX, TY, kOp, true, kIn>), dim3(blocks), dim3((TX / 2 + 2) * (TY + 4)),
                           0, st, a, g, tpb, bstride);
    else
        hipLaunchKernelGGL((k_sweep_boxes<T, TX, TY, kOp, false, kIn>), dim3(blocks), dim3((TX / 2 + 2) * (TY + 4)),
                           0, st, a, g, tpb, bstride);
}

template <typename T, int TX, int TY>
void launch_boxes_mode(const SweepArgs<T>& a, const BoxGeom& g, int tpb, size_t bstride, unsigned blocks, int mode,
                       hipStream_t st) {
    switch (mode) {
        case kBoxSweepZero: launch_boxes_t<T, TX, TY, kOpSweep, kInZero>(a, g, tpb, bstride, blocks, st); break;
        case kBoxSweepProlong: launch_boxes_t<T, TX, TY, kOpSweep, kInProlong>(a, g, tpb, bstride, blocks, st); break;
        case kBoxResidRestrict:
            launch_boxes_t<T, TX, TY, kOpResidRestrict, kInPlain>(a, g, tpb, bstride, blocks, st);
            break;
        case kBoxSweepNorm:
            if constexpr (std::is_same<T, double>::value)
                launch_boxes_t<T, TX, TY, kOpSweepNorm, kInPlain>(a, g, tpb, bstride, blocks, st);
            break;
        case kBoxRefine:
            if constexpr (std::is_same<T, double>::value)
                launch_boxes_t<T, TX, TY, kOpRefine, kInCorrect>(a, g, tpb, bstride, blocks, st);
            break;
        default: launch_boxes_t<T, TX, TY, kOpSweep, kInPlain>(a, g, tpb, bstride, blocks, st); break;
    }
}

template <typename T>
hipError_t launch_sweep_boxes_mode(const SweepArgs<T>& a0, const BoxGeom& g, int nbox, size_t bstride, int mode,
                                   int* nparts, hipStream_t st) {
    SweepArgs<T> a = a0;
    if (!sweep_boxes_fit(a.ex, a.ey, a.ez) || a.ox < 2 || a.oy < 2 || a.oz < 2 || a.nx < a.ex + 2 * a.ox ||
        a.ny < a.ey + 2 * a.oy || a.nz < a.ez + 2 * a.oz)
        return hipErrorInvalidValue;
    const bool rows = mode == kBoxSweepNorm || mode == kBoxRefine;
    if (rows != (nparts != nullptr)) return hipErrorInvalidValue;
    if (!std::is_same<T, double>::value && rows) return hipErrorInvalidValue;   // FP64 only
    // the finest level's own tile (64 x 16) where the box takes it, else 32 x 8
    const bool wide = a.ex % 64 == 0 && a.ey % 16 == 0;
    const int TXc = wide ? 64 : 32, TYc = wide ? 16 : 8;
    a.tz = std::min(a.ez, kSweepTZMax);
    a.ntx = (a.ex + TXc - 1) / TXc;
    a.nty = (a.ey + TYc - 1) / TYc;
    const int ntz = (a.ez + a.tz - 1) / a.tz;
    const int tpb = a.ntx * a.nty * ntz;
    const unsigned blocks = (unsigned)tpb * nbox;
    if (rows) {
        if (blocks > (unsigned)kMaxPartialRows) return hipErrorInvalidValue;
        *nparts = (int)blocks;
    }
    if (wide) launch_boxes_mode<T, 64, 16>(a, g, tpb, bstride, blocks, mode, st);
    else launch_boxes_mode<T, 32, 8>(a, g, tpb, bstride, blocks, mode, st);
    return hipGetLastError();
}
template hipError_t launch_sweep_boxes_mode<double>(const SweepArgs<double>&, const BoxGeom&, int, size_t, int, int*,
                                                    hipStream_t);
template hipError_t launch_sweep_boxes_mode<float>(const SweepArgs<float>&, const BoxGeom&, int, size_t, int, int*,
                                                   hipStream_t);

hipError_t launch_sweep_boxes(const SweepArgs<double>& a, const BoxGeom& g, int nbox, size_t bstride, int* nparts,
                              hipStream_t st, bool prolong, bool restrict_only) {
    if (nparts && (prolong || restrict_only)) return hipErrorInvalidValue;
    if (prolong && restrict_only) return hipErrorInvalidValue;
    const int mode = nparts ? kBoxSweepNorm : (restrict_only ? kBoxResidRestrict : (prolong ? kBoxSweepProlong
                                                                                            : kBoxSweep));
    return launch_sweep_boxes_mode(a, g, nbox, bstride, mode, nparts, st);
}

int sweep_tiles(int nx, int ny, int nz, int cfg) {
    const SweepCfg& c = kSweepCfgs[cfg];
    return ((nx + c.tx - 1) / c.tx) * ((ny + c.ty - 1) / c.ty) * ((nz + c.tz - 1) / c.tz);
}

template bool sweep_fusable<double>(int, int, int);
template bool sweep_fusable<float>(int, int, int);
template hipError_t launch_sweep<double>(const SweepArgs<double>&, bool, int, int, hipStream_t);
template hipError_t launch_sweep<float>(const SweepArgs<float>&, bool, int, int, hipStream_t);
template hipError_t launch_resid_restrict_tiled<double>(const SweepArgs<double>&, bool, int, hipStream_t);
template hipError_t launch_resid_restrict_tiled<float>(const SweepArgs<float>&, bool, int, hipStream_t);
template hipError_t launch_sweep_multi<double>(const SweepArgs<double>*, const int2*, int, bool, int, int, int,
                                               hipStream_t);
template hipError_t launch_sweep_multi<float>(const SweepArgs<float>*, const int2*, int, bool, int, int, int,
                                              hipStream_t);

}  // namespace mg
