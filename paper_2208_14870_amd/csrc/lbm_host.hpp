// Host-side internals shared by the single-lattice solver and the batch:
// material -> relaxation rates (Table "scheme"), lattice memory layout inside
// caller-owned device memory, kernel dispatch.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>

#include "lbm.h"
#include "lbm_device.hpp"
#include "lbm_host_base.hpp"

namespace lbm_host {
using namespace lbm;


// Tiles per vertical band of a single lattice's work list for the fused tile
// kernel (single steps stream best in row-major order: 8192^2 FP32 81 against
// 76 GLUPS).
constexpr int kItemBand = 8;

inline unsigned blocks_for(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

constexpr int kErrBlocks = 1024;  // grid of the two-stage FP64 reductions

struct Rates {
    double theta = 1.0 / 3.0, w12 = 1.0, w21 = 1.0, w22 = 1.0;  // free parameters
    double w11 = 0, ws = 0, wd = 0;                              // from the material
};

// Table "scheme": tau_11 = mu/theta, tau_s = 2K/(1+theta), tau_d = 2mu/(1-theta),
// K = lambda + mu, omega = 1/(tau + 1/2) (Eq. relaxation_rate).
inline bool material_rates(double lam, double mu, Rates& r, std::string& err) {
    const double K = lam + mu;
    if (!std::isfinite(lam) || !std::isfinite(mu) || !(mu > 0.0) || !(K > 0.0)) {
        err = "material: need finite lambda, mu with mu > 0 and lambda + mu > 0";
        return false;
    }
    const double th = r.theta;
    r.w11 = 1.0 / (mu / th + 0.5);
    r.ws = 1.0 / (2.0 * K / (1.0 + th) + 0.5);
    r.wd = 1.0 / (2.0 * mu / (1.0 - th) + 0.5);
    return true;
}

// ---------------------------------------------------------------------------
// leading-order error of the scheme (Sec. 4, App. B) and the rates of the
// fourth-order special case (App. C)
// ---------------------------------------------------------------------------

// r_x^(4) = C1 d_xxxx u0x + C2 d_xxxy u0y + C3 d_xxyy u0x + C4 d_xyyy u0y
//         + C5 d_yyyy u0x + D1 d_xx gx + D2 d_xy gy + D3 d_yy gx
// (Eq. leadingCoefficients), in the sign of Eq. ux_order2.  App. B lists the
// constants as functions of the dimensionless Young's modulus E and Poisson
// ratio nu (second-order relaxation times eliminated) and of theta, tau_12,
// tau_21, tau_22.  Matched against the symbols of the exact one-step operator
// (quartic part of the log of its slow two-mode block, quadratic part of its
// effective forcing), the printed list needs four changes, applied here:
// every constant changes sign; the tau terms of D1 and D2 are over
// (1 - theta^2)(1 - nu^2), not (1 - theta^2)(1 - nu^2)^2; the E^3 term of C2
// is over 8 theta (1 - theta^2)(1 - nu^2)^3.  The y row is the x row with
// tau_12 and tau_21 exchanged.
struct ErrorConstants {
    double C[5];
    double D[3];
};

inline ErrorConstants error_constants(double E, double nu, double th, double t12, double t21,
                                      double t22) {
    const double a = 1.0 - th * th, b = 1.0 - nu * nu;
    const double E2 = E * E, E3 = E2 * E, n2 = nu * nu, n3 = n2 * nu, th2 = th * th;
    const double b2 = b * b, b3 = b2 * b, om = 1.0 - nu, op = 1.0 + nu;
    const double q = th2 * op + nu - 2.0 * th - 1.0;
    double c[5], d[3];  // as printed (before the sign change)
    c[0] = (n2 - 2.0 * th * nu + 1.0) * E3 / (a * b3) + th * (nu - th) * t12 * E2 / (a * b2) +
           (th2 - 1.0 + 12.0 * th * (th - nu) * t12 * t22) * E / (12.0 * a * b);
    c[1] = (om * om * om + 4.0 * th * (n3 - n2 + 3.0 * nu + 1.0) +
            th2 * (5.0 * n3 - 15.0 * n2 - nu - 5.0)) * E3 / (8.0 * th * a * b3) -
           (2.0 * th * (om * nu + th2 * op - th * (1.0 + n2)) * t12 +
            (1.0 - th) * om * (1.0 + 2.0 * th - nu - th2 * op) * t21) * E2 / (4.0 * th * a * b2) +
           ((2.0 * th2 - 3.0 * th + 1.0) * (1.0 + 3.0 * th * om - 5.0 * nu) +
            24.0 * th * (th - nu) * t12 * t22) * E / (24.0 * a * b);
    c[2] = (om * om * (3.0 + nu) + 4.0 * th * (-n3 + 3.0 * n2 + nu + 1.0) -
            th2 * (5.0 * n3 - 3.0 * n2 + 7.0 * nu + 7.0)) * E3 / (8.0 * th * a * b3) +
           (-2.0 * (1.0 - th) * th * (nu - 2.0 * th - 1.0) * om * t12 -
            ((1.0 + th) * om * om + th2 * th * op * op + th2 * (n2 - 2.0 * nu - 3.0)) * t21) * E2 /
               (4.0 * th * a * b2) +
           ((1.0 - th) * (om - th * op - 2.0 * th2 * (2.0 + nu)) - 4.0 * a * om * t12 * t22 +
            4.0 * q * t21 * t22) * E / (8.0 * a * b) +
           0.25 * th * t22;
    c[3] = (16.0 * th * nu + om * om * (3.0 + nu) - th2 * (n3 + 9.0 * n2 - 5.0 * nu + 11.0)) * E3 /
               (8.0 * th * a * b3) +
           (a * om * (th * nu + nu + th - 1.0) * t12 - 2.0 * th * q * t21) * E2 / (4.0 * th * a * b2) +
           (a * (2.0 * (2.0 - nu) - 3.0 * th * (5.0 + nu)) - 12.0 * a * om * t12 * t22 +
            12.0 * q * t21 * t22) * E / (24.0 * a * b) +
           0.25 * th * t22;
    c[4] = E3 / (8.0 * th * op * op * op) - (1.0 - th) * t12 * E2 / (4.0 * th * op * op) -
           (3.0 * th - 2.0) * E / (24.0 * op);
    d[0] = (n2 - 2.0 * th * nu + 1.0) * E2 / (a * b2) + th * (nu - th) * t12 * E / (a * b) - 0.25;
    d[1] = (om * om + 8.0 * th * nu - th2 * (5.0 * n2 - 2.0 * nu + 5.0)) * E2 / (4.0 * th * a * b2) -
           q * t21 * E / (2.0 * a * b) - 0.5 * th;
    d[2] = E2 / (4.0 * th * op * op) + t12 * E / (2.0 * op) - 0.25 * th;
    ErrorConstants k;
    for (int i = 0; i < 5; ++i) k.C[i] = -c[i];
    for (int i = 0; i < 3; ++i) k.D[i] = -d[i];
    return k;
}

// E and nu of the 2D relations (Eq. material_relations): K = lambda + mu,
// E = 4 K mu / (K + mu), nu = (K - mu) / (K + mu).
inline void young_poisson(double lam, double mu, double& E, double& nu) {
    const double K = lam + mu;
    E = 4.0 * K * mu / (K + mu);
    nu = (K - mu) / (K + mu);
}

// Rates of the fourth-order special case (Sec. 7.3.3): tau_12 = tau_21 from
// App. C (it cancels C5) and tau_22 from C1 = 0 (C1 is affine in tau_22; the
// tau_22 expression printed in App. C does not cancel C1).  Returns false if
// tau_22 has no root (theta = nu) or a rate falls outside (0, 2).
inline bool fourth_order_rates(double lam, double mu, double th, double& w12, double& w22) {
    double E, nu;
    young_poisson(lam, mu, E, nu);
    const double t11 = mu / th;
    const double t12 = (2.0 - 3.0 * th + 12.0 * th * t11 * t11) / (12.0 * (1.0 - th) * t11);
    const double c0 = error_constants(E, nu, th, t12, t12, 0.0).C[0];
    const double c1 = error_constants(E, nu, th, t12, t12, 1.0).C[0];
    if (!(c1 != c0)) return false;
    const double t22 = -c0 / (c1 - c0);
    w12 = 1.0 / (t12 + 0.5);
    w22 = 1.0 / (t22 + 0.5);
    auto ok = [](double w) { return std::isfinite(w) && w > 0.0 && w < 2.0; };
    return ok(w12) && ok(w22);
}

inline void fill_coefs(SlotDesc& d, const Rates& r) {
    d.cs = 0.25 * (1.0 - r.ws);
    d.cd = 0.25 * (1.0 - r.wd);
    d.c11 = 0.25 * (1.0 - r.w11);
    d.hth = 0.5 * (1.0 - r.theta);
    d.tq = 0.25 * r.theta;
    d.a11 = 1.0 - r.w11;
    d.as = 1.0 - r.ws;
    d.ad = 1.0 - r.wd;
    d.theta = r.theta;
    d.w12 = r.w12;
    d.w21 = r.w21;
    d.a22 = 1.0 - r.w22;
    d.general = (r.w12 != 1.0 || r.w21 != 1.0 || r.w22 != 1.0) ? 1 : 0;
}

// ---------------------------------------------------------------------------
// kernel dispatch
// ---------------------------------------------------------------------------
template <typename S, int MODE, int LAY>
inline hipError_t launch_step_l(bool general, int vy, unsigned grid, hipStream_t st,
                                const StepLaunch& L) {
    if (general) {
        hipLaunchKernelGGL((k_step<S, MODE, true, 1, LAY>), dim3(grid), dim3(kBlock), 0, st, L);
    } else if (vy == 1) {
        hipLaunchKernelGGL((k_step<S, MODE, false, 1, LAY>), dim3(grid), dim3(kBlock), 0, st, L);
    } else if (vy == 2) {
        hipLaunchKernelGGL((k_step<S, MODE, false, 2, LAY>), dim3(grid), dim3(kBlock), 0, st, L);
    } else if (vy == 3) {
        hipLaunchKernelGGL((k_step<S, MODE, false, 3, LAY>), dim3(grid), dim3(kBlock), 0, st, L);
    } else if (vy == 4) {
        hipLaunchKernelGGL((k_step<S, MODE, false, 4, LAY>), dim3(grid), dim3(kBlock), 0, st, L);
    } else if constexpr (std::is_same<S, float>::value && LAY == kLayPull) {
        // the work list of the 24-row FP32 tile (single steps between its launches)
        if (vy != 6) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_step<S, MODE, false, 6, LAY>), dim3(grid), dim3(kBlock), 0, st, L);
    } else {
        return hipErrorInvalidValue;  // rows per thread outside 1..4
    }
    return hipGetLastError();
}

template <typename S, int MODE>
inline hipError_t launch_step_t(bool general, int vy, int layout, unsigned grid, hipStream_t st,
                                const StepLaunch& L) {
    if (layout == kLayNatural) return launch_step_l<S, MODE, kLayNatural>(general, vy, grid, st, L);
    if (layout == kLaySwapped) return launch_step_l<S, MODE, kLaySwapped>(general, vy, grid, st, L);
    return launch_step_l<S, MODE, kLayPull>(general, vy, grid, st, L);
}

template <typename S>
inline hipError_t launch_step_s(int mode, bool general, int vy, int layout, unsigned grid,
                                hipStream_t st, const StepLaunch& L) {
    switch (mode) {
        case kPlain: return launch_step_t<S, kPlain>(general, vy, layout, grid, st, L);
        case kWriteU: return launch_step_t<S, kWriteU>(general, vy, layout, grid, st, L);
        default: return launch_step_t<S, kCheck>(general, vy, layout, grid, st, L);
    }
}

// Non-advancing residual check of an in-place lattice (layout natural or swapped).
template <typename S, int LAY>
inline hipError_t launch_check_state_l(int vy, unsigned grid, hipStream_t st, const StepLaunch& L) {
    if (vy == 1) hipLaunchKernelGGL((k_check_state<S, LAY, 1>), dim3(grid), dim3(kBlock), 0, st, L);
    else if (vy == 2) hipLaunchKernelGGL((k_check_state<S, LAY, 2>), dim3(grid), dim3(kBlock), 0, st, L);
    else if (vy == 3) hipLaunchKernelGGL((k_check_state<S, LAY, 3>), dim3(grid), dim3(kBlock), 0, st, L);
    else if (vy == 4) hipLaunchKernelGGL((k_check_state<S, LAY, 4>), dim3(grid), dim3(kBlock), 0, st, L);
    else return hipErrorInvalidValue;  // rows per thread outside 1..4
    return hipGetLastError();
}
template <typename S>
inline hipError_t launch_check_state_s(int vy, int layout, unsigned grid, hipStream_t st,
                                       const StepLaunch& L) {
    if (layout == kLaySwapped) return launch_check_state_l<S, kLaySwapped>(vy, grid, st, L);
    return launch_check_state_l<S, kLayNatural>(vy, grid, st, L);
}
inline hipError_t launch_check_state(int prec, int vy, int layout, unsigned grid, hipStream_t st,
                                     const StepLaunch& L) {
    if (prec == LBM_FP64) return launch_check_state_s<double>(vy, layout, grid, st, L);
    if (prec == LBM_FP32) return launch_check_state_s<float>(vy, layout, grid, st, L);
    return launch_check_state_s<__half>(vy, layout, grid, st, L);
}

// Whether launch_stepN has a kernel for ns steps on tiles of th rows: every
// tile height runs 2..4 steps, and the heights used for deeper blocking (FP64
// 8, FP32 16 and 24, FP16 16) run 2..8, so a remainder of a launch sequence
// can run as one shorter fused launch.
inline bool stepN_supported(int prec, int ns, int th) {
    if (ns < 2 || ns > 8) return false;
    if (prec == LBM_FP64) return th == 8;
    if (prec == LBM_FP32) return th == 16 || th == 24 || (th == 8 && ns <= 4);
    return th == 16 || (th == 12 && ns <= 4);
}

// Shapes of the fused LDS tile kernel (tile 64 x TH, NT threads) per storage
// type and steps per launch, measured on MI355X.  FP64: 8 rows with 512
// threads (1024^2, five steps: 106 against 98 GLUPS with 256).  Up to four
// steps: FP32 8 rows with 512 threads up to 2^21 sites and 16 rows with 256
// threads above, FP16 12 rows.  Five to eight steps: FP32 and FP16 16 rows
// with 512 threads (two workgroups of 75 KB LDS per CU at eight steps in FP32).
// A tile height chosen by the caller (`rows`, lbm_set_tile_rows) is taken when
// a kernel exists for it at `ns` steps.
inline int fused_th(int prec, int ns, long long sites, int rows = 0) {
    if (rows > 0 && stepN_supported(prec, ns, rows)) return rows;
    if (prec == LBM_FP64) return 8;
    if (prec == LBM_FP32) return (ns <= 4 && sites <= (1LL << 21)) ? 8 : 16;
    return ns <= 4 ? 12 : 16;
}

// Threads per workgroup of the fused LDS tile kernel (as launch_stepN runs it).
inline int fused_nt(int prec, int ns, int th) {
    if (prec == LBM_FP64) return 512;
    if (prec == LBM_FP32) return (th == 8 || th == 24 || ns > 4) ? 512 : 256;
    return th == 16 ? 512 : 256;
}

template <typename S, int TH, int NT, int NS, int NSMAX, bool SR = false>
inline bool launch_stepN_ns(int ns, bool check, unsigned grid, hipStream_t st, const StepLaunch& L) {
    if (ns == NS) {
        if (check)
            hipLaunchKernelGGL((k_stepN<S, TH, NS, NT, kCheck, SR>), dim3(grid), dim3(NT), 0, st, L);
        else hipLaunchKernelGGL((k_stepN<S, TH, NS, NT, kPlain, SR>), dim3(grid), dim3(NT), 0, st, L);
        return true;
    }
    if constexpr (NS < NSMAX)
        return launch_stepN_ns<S, TH, NT, NS + 1, NSMAX, SR>(ns, check, grid, st, L);
    return false;
}

// ns in 2..8 with stepN_supported(prec, ns, th); th is the tile height of the
// work list (fused_th for the sequence's steps per launch).  check: the last
// two steps form a residual check (partials per tile into L.partial, u(n) into
// the slot's u planes), replacing a write-u step and a check step.
inline hipError_t launch_stepN(int prec, int ns, int th, unsigned grid, hipStream_t st,
                               const StepLaunch& L, bool check = false, bool sr = false) {
    bool ok = false;
    if (prec == LBM_FP64 && th == 8)
        ok = launch_stepN_ns<double, 8, 512, 2, 8>(ns, check, grid, st, L);
    else if (prec == LBM_FP32 && th == 8)
        ok = launch_stepN_ns<float, 8, 512, 2, 4>(ns, check, grid, st, L);
    else if (prec == LBM_FP32 && th == 16 && ns <= 4)
        ok = launch_stepN_ns<float, 16, 256, 2, 4>(ns, check, grid, st, L);
    else if (prec == LBM_FP32 && th == 16)
        ok = launch_stepN_ns<float, 16, 512, 5, 8>(ns, check, grid, st, L);
    else if (prec == LBM_FP32 && th == 24)
        ok = launch_stepN_ns<float, 24, 512, 2, 8>(ns, check, grid, st, L);
    else if (prec == LBM_FP16 && th == 12 && sr)
        ok = launch_stepN_ns<__half, 12, 256, 2, 4, true>(ns, check, grid, st, L);
    else if (prec == LBM_FP16 && th == 16 && sr)
        ok = launch_stepN_ns<__half, 16, 512, 2, 8, true>(ns, check, grid, st, L);
    else if (prec == LBM_FP16 && th == 12)
        ok = launch_stepN_ns<__half, 12, 256, 2, 4>(ns, check, grid, st, L);
    else if (prec == LBM_FP16 && th == 16)
        ok = launch_stepN_ns<__half, 16, 512, 2, 8>(ns, check, grid, st, L);
    if (!ok) return hipErrorInvalidValue;
    return hipGetLastError();
}

// Whole solves of small lattices in one workgroup (k_solve_small): the largest
// lattices whose two population buffers fit in LDS.
constexpr int kSmallMax64 = 1152, kSmallMax32 = 2304;

inline int small_max_sites(int prec) {
    return prec == LBM_FP64 ? kSmallMax64 : prec == LBM_FP32 ? kSmallMax32 : 0;
}

inline hipError_t launch_solve_small(int prec, bool general, hipStream_t st, const SmallLaunch& P) {
    if (prec == LBM_FP64 && general)
        hipLaunchKernelGGL((k_solve_small<double, kSmallMax64, true>), dim3(1), dim3(kSmallThreads), 0, st, P);
    else if (prec == LBM_FP64)
        hipLaunchKernelGGL((k_solve_small<double, kSmallMax64, false>), dim3(1), dim3(kSmallThreads), 0, st, P);
    else if (prec == LBM_FP32 && general)
        hipLaunchKernelGGL((k_solve_small<float, kSmallMax32, true>), dim3(1), dim3(kSmallThreads), 0, st, P);
    else if (prec == LBM_FP32)
        hipLaunchKernelGGL((k_solve_small<float, kSmallMax32, false>), dim3(1), dim3(kSmallThreads), 0, st, P);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Default fused kernel of a single lattice of N = nx ny sites, measured on
// MI355X (GLUPS at eight steps per launch, kernel alone; FP64 tile at five):
//   FP32  tile / wavefront: 1024^2 242 / 246 (checked chunks of 1000 steps;
//         segments of 22 rows give 1034 waves, a second round: 160), 1100^2
//         212 / 271, 1448^2 231 / 333, 2048^2 239 / 399, 4096^2 263 / 377,
//         8192^2 295 / 432 (two columns per lane);
//   FP16  1448^2 311 / 278, 2048^2 343 / 314, 2896^2 361 / 285, 4096^2 359 / 413,
//         8192^2 380 / 449;
//   FP64  512^2 94 / 54, 600^2 90 / 74, 724^2 87 / 103, 880^2 93 / 143,
//         2048^2 115 / 228, 8192^2 117 / 235.
// So: the wavefront at eight steps for FP32 from 2^20 sites (two columns per
// lane from 2^25 on even widths), FP64 from 458752 (about 677^2) and FP16 from
// 2^24; the tile kernel below.  Segments: as long as leaves one wave per SIMD
// (4 per compute unit) over the strips, at most 128 rows and at least 16: a
// lattice that fills the chip once with long segments reads the fewest halo
// rows (GLUPS at eight steps by segment rows: FP64 1024^2 156 at 32, 165-169
// at 23-24, 110 at 16; FP64 2048^2 191 at 32, 228 at 90-96, 217 at 128; FP32
// 2048^2 343 at 32, 399 at 90; FP64 / FP32 4096^2 best at 128; every type at
// 8192^2 best at 128).  `beyond_tile`: the planes exceed the tile kernel's
// 32-bit offsets, so the wavefront (one column per lane, any width) is the
// only fused kernel.  wave_hs = 0 selects the tile kernel.
inline bool wave_by_default(int prec, long long n) {
    return (prec == LBM_FP64 && n >= 458752) || (prec == LBM_FP32 && n >= (1LL << 20)) ||
           (prec == LBM_FP16 && n >= (1LL << 24));
}
// In a batch, lattices of one storage type fill the chip together, so above
// these totals every lattice of the type takes the wavefront list (GLUPS at
// eight steps, tile / wavefront list, 2000 steps in checked chunks of 100:
// FP64 512 lattices of sides 64..512 (43.9 M sites) 112 / 199, 8 x 1024^2
// 104 / 182, 64 lattices 256..512 (12.4 M) 116 / 162, 512 lattices 64..128
// (5.3 M) 108 / 140, 16 lattices 128..256 (0.74 M) 92 / 78; FP32 in the same
// order 272 / 316, 267 / 308, 279 / 268, 249 / 223, 187 / 124; FP16 43.9 M
// 358 / 381).  Below them only the lattices of wave_by_default do.
inline long long batch_wave_total(int prec) {
    return prec == LBM_FP64 ? (1LL << 22) : prec == LBM_FP32 ? (1LL << 23) : (1LL << 24);
}
struct FusedChoice {
    int wave_hs = 0, wave_v = 1;
};
// Columns per lane of the wavefront at ns steps: two for FP32 / FP16 on even
// widths at up to four steps (ring of four), and for FP32 from 2^25 sites at
// more; one otherwise.
inline int wave_cols(int prec, int ns, int nx, int ny) {
    if (prec == LBM_FP64 || nx % 2 != 0) return 1;
    if (ns <= 4) return 2;
    return (prec == LBM_FP32 && (long long)nx * ny >= (1LL << 25)) ? 2 : 1;
}
inline FusedChoice default_fused(int prec, int ns, int nx, int ny, int cus, bool beyond_tile = false) {
    FusedChoice c;
    const long long n = (long long)nx * ny;
    const bool wave = beyond_tile || wave_by_default(prec, n);
    if (!wave || ns < 2) return c;
    c.wave_v = wave_cols(prec, ns, nx, ny);
    const long long strips = (nx + wave_width_of(ns, c.wave_v) - 1) / wave_width_of(ns, c.wave_v);
    // segments as long as one wave per SIMD allows (fewest halo rows with the
    // chip filled), 16..128 rows
    const long long per = std::max(1LL, 4LL * cus / strips);
    c.wave_hs = (int)std::min<long long>(128, std::max<long long>(16, (ny + per - 1) / per));
    return c;
}

// In place: columns per lane (two on even widths except FP64, and half
// storage beyond four steps) and segment height (256 rows, halved down to 32
// while the lattice would give fewer than 4096 waves): long segments keep the
// row copies small (2 ns rows per segment), enough waves keep the chip busy
// (8192^2 at eight steps, MI355X: FP32 with two columns per lane 275 GLUPS at
// 256 rows (2368 waves), 292 at 128, 262 at 64; FP64 136 at 256 and at 128).
inline int ip_wave_cols(int prec, int ns, int nx) {
    return (prec != LBM_FP64 && nx % 2 == 0 && (prec == LBM_FP32 || ns <= 4)) ? 2 : 1;
}
inline int ip_segment_rows(int ns, int v, int nx, int ny) {
    const long long strips = (nx + wave_width_of(ns, v) - 1) / wave_width_of(ns, v);
    int hs = 256;
    while (hs > 32 && strips * ((ny + hs - 1) / hs) < 4096) hs /= 2;
    return hs;
}
// Halo bytes of in-place launches of up to ns steps (hs = 0: the default
// segment height).  Shallower launches of the same sequence need no more.
inline size_t ip_halo_bytes(int prec, int ns, int nx, int ny, int hs = 0) {
    const int v = ip_wave_cols(prec, ns, nx);
    return wave_halo_bytes(prec, ns, v, nx, ny, hs > 0 ? hs : ip_segment_rows(ns, v, nx, ny));
}

// Default steps per launch for `sites` lattice sites (of one lattice, or of
// all lattices of one storage type in a batch), measured on MI355X: the LDS
// tile kernel is bound by its per-launch memory phase, so deeper blocking pays
// until LDS limits the workgroups per CU.  FP32 and FP16: eight above 2^17
// sites (FP32 1024^2: 232 against 149 GLUPS at four), four on smaller lattices
// (FP32 256^2: 49 against 42).  FP64 (whose LDS tile is twice as large): five
// through the tile kernel (1024^2: 106 against 98 GLUPS at four), eight where
// the register wavefront is the default (wave_by_default, single lattices; a
// batch always runs tiles).
inline int default_time_blocking(int prec, long long sites, bool tiles_only = false) {
    if (prec == LBM_FP64) return (tiles_only || !wave_by_default(prec, sites)) ? 5 : 8;
    return sites > (1LL << 17) ? 8 : 4;
}

inline hipError_t launch_step(int prec, int mode, bool general, int vy, int layout, unsigned grid,
                              hipStream_t st, const StepLaunch& L) {
    if (prec == LBM_FP64) return launch_step_s<double>(mode, general, vy, layout, grid, st, L);
    if (prec == LBM_FP32) return launch_step_s<float>(mode, general, vy, layout, grid, st, L);
    return launch_step_s<__half>(mode, general, vy, layout, grid, st, L);
}

// ---------------------------------------------------------------------------
// one lattice: memory regions, material, scale, tiles (shared by solver and batch)
// ---------------------------------------------------------------------------
struct LatticeMem {
    void* buf[2] = {nullptr, nullptr};  // populations, creation precision
    void* g = nullptr;                  // force, arithmetic type of creation precision
    double* u = nullptr;                // 2 planes
    void* pbuf[2] = {nullptr, nullptr}; // FP64 polish populations
    double* pg = nullptr;               // FP64 force (polish)
};

// Elements between consecutive planes of one array (populations, force,
// displacement).  Large planes get 1024 elements of padding so that the 18
// concurrent streams of a step do not start on the same HBM channels (a
// power-of-two plane size otherwise aligns them); small planes only round up
// to 64 elements.
inline long long plane_of(long long N) {
    const long long r = (N + 63) / 64 * 64;
    return N >= (1LL << 16) ? r + 1024 : r;
}

// In place (one population buffer), no polish reservation.
inline size_t lattice_bytes(long long N, int prec, bool polish, bool inplace = false) {
    const long long P = plane_of(N);
    size_t b = (inplace ? 1 : 2) * al(8 * P * elem_bytes(prec)) + al(2 * P * arith_bytes(prec)) +
               al(2 * P * 8);
    if (polish && prec != LBM_FP64) b += 2 * al(8 * P * 8) + al(2 * P * 8);
    return b;
}

inline void carve_lattice(char* base, long long N, int prec, bool polish, LatticeMem& m,
                          bool inplace = false) {
    const long long P = plane_of(N);
    size_t off = 0;
    for (int i = 0; i < 2; ++i) {
        m.buf[i] = base + off;
        if (!inplace || i == 1) off += al(8 * P * elem_bytes(prec));
    }
    m.g = base + off;
    off += al(2 * P * arith_bytes(prec));
    m.u = reinterpret_cast<double*>(base + off);
    off += al(2 * P * 8);
    if (polish && prec != LBM_FP64) {
        for (int i = 0; i < 2; ++i) {
            m.pbuf[i] = base + off;
            off += al(8 * P * 8);
        }
        m.pg = reinterpret_cast<double*>(base + off);
        off += al(2 * P * 8);
    }
}

struct Lattice {
    int nx = 0, ny = 0;
    long long N = 0;      // sites
    long long plane = 0;  // elements between planes (>= N, see plane_of)
    int prec0 = LBM_FP64;  // creation precision
    int prec = LBM_FP64;   // current storage precision
    bool polish = false;
    LatticeMem mem;
    Rates rates;
    double lam = 0, mu = 0;
    bool has_material = false, has_force = false;
    int e_scale = 0;  // half storage: stored = f * 2^-e
    bool sr = false;       // half storage rounds stochastically (two buffers, no wavefront)
    unsigned sr_seed = 0;
    double gmax = 0;  // max |g| of the force (initial half scale)
    // The mean first moments of the exact trajectory: sum_x m10, sum_x m01 were
    // mbase at step mbase_steps and grow by gsum = sum_x g (FP64) per step.
    double gsum[2] = {0, 0};
    double mbase[2] = {0, 0};
    long long mbase_steps = 0;
    void mean_target(long long steps, double out[2]) const {
        out[0] = mbase[0] + (double)(steps - mbase_steps) * gsum[0];
        out[1] = mbase[1] + (double)(steps - mbase_steps) * gsum[1];
    }
    // a new force from step `steps` on
    void rebase_force(long long steps, double sx, double sy) {
        double m[2];
        mean_target(steps, m);
        mbase[0] = m[0];
        mbase[1] = m[1];
        mbase_steps = steps;
        gsum[0] = sx;
        gsum[1] = sy;
    }
    // The staggered first moments of the exact trajectory (even nx: Jx =
    // sum_x (-1)^x m10 of f(n); even ny: Jy with (-1)^y m01): J(n) = -G/2 +
    // (-1)^(n - jbase_steps) jamp with G = gstag, the staggered sums of the
    // FP64 force.  From f = 0, jamp = G/2: J alternates between 0 and -G.
    double gstag[2] = {0, 0};
    double jamp[2] = {0, 0};
    long long jbase_steps = 0;
    void stag_value(long long steps, double out[2]) const {
        const double sg = ((steps - jbase_steps) & 1) ? -1.0 : 1.0;
        for (int c = 0; c < 2; ++c) out[c] = -0.5 * gstag[c] + sg * jamp[c];
    }
    // the staggered sums of the stored field S = f*(n-1) are -J(n)
    void stag_target_stored(long long steps, double out[2]) const {
        stag_value(steps, out);
        out[0] = -out[0];
        out[1] = -out[1];
    }
    // a new force from step `steps` on (J itself is a property of the state)
    void rebase_stagger(long long steps, double gx_stag, double gy_stag) {
        double j[2];
        stag_value(steps, j);
        gstag[0] = gx_stag;
        gstag[1] = gy_stag;
        set_stagger_state(steps, j);
    }
    // the state at step `steps` has staggered moments j (f = 0: j = 0)
    void set_stagger_state(long long steps, const double j[2]) {
        for (int c = 0; c < 2; ++c) jamp[c] = j[c] + 0.5 * gstag[c];
        jbase_steps = steps;
    }
    // k steps of streaming alone (no collision) flip J k times
    void stream_only_stagger(long long steps, long long k) {
        double j[2];
        stag_value(steps, j);
        if (k & 1) {
            j[0] = -j[0];
            j[1] = -j[1];
        }
        set_stagger_state(steps + k, j);
    }
    int bx_log2 = 6, vy = 1;
    int tb = 4;       // plain steps per launch (2..8: fused multi-step kernel)
    int th = 16;      // tile height of the fused LDS kernel (fused_th)
    int th_user = 0;  // tile height chosen by the caller (0: the default)
    int wave_hs = 0;  // > 0: fused launches use the register wavefront, segments of wave_hs rows
    int wave_v = 1;   // the wavefront's columns per lane
    int cur = 0;      // buffer with the state at flip 0
    bool inplace = false;  // one buffer, in-place streaming (layout alternates per step)
    void* halo = nullptr;  // in place: room for the wavefront's halo copies
    size_t halo_cap = 0;   // its bytes (0: one step per launch only)
    // layout of the stored field for buffer selector `sel` = cur ^ launch parity
    // (in place, the selector flips every step and starts at 0 in kLayNatural)
    int layout(int sel) const { return !inplace ? kLayPull : (sel ? kLaySwapped : kLayNatural); }

    void* state_buf(int i) const {
        return (prec == prec0) ? mem.buf[i] : mem.pbuf[i];
    }
    const void* force() const { return (prec == prec0) ? mem.g : (const void*)mem.pg; }
    int tiles_x() const { return (nx + (1 << eff_bxl()) - 1) >> eff_bxl(); }
    // The fused kernel has a tile 64 wide and th rows high; the general-rates
    // variant runs one row per thread.
    // The tile kernel addresses a plane (populations, and the force in the
    // arithmetic type, which is at least as wide) with 32-bit byte offsets.
    bool tile_fits() const { return plane * (long long)arith_bytes(prec) <= 0xFFFFFFFFLL; }
    bool fused() const { return tb >= 2 && !general() && !inplace && (wave_hs > 0 || tile_fits()); }
    // in place, up to tb steps per launch through the in-place wavefront
    bool ip_blocked() const { return inplace && tb >= 2 && !general() && wave_hs > 0; }
    int eff_bxl() const { return fused() ? 6 : bx_log2; }
    int eff_vy() const { return fused() ? th / 4 : (general() ? 1 : vy); }
    int tile_h() const { return (kBlock >> eff_bxl()) * eff_vy(); }
    int tiles_y() const { return (ny + tile_h() - 1) / tile_h(); }
    int nitems() const { return tiles_x() * tiles_y(); }

    SlotDesc desc() const {
        SlotDesc d;
        std::memset(&d, 0, sizeof(d));
        d.buf[0] = state_buf(0);
        d.buf[1] = state_buf(1);
        d.g = force();
        d.u = mem.u;
        d.plane = plane;
        d.nx = nx;
        d.ny = ny;
        d.cur = cur;
        d.tiles_x = tiles_x();
        d.tiles_y = tiles_y();
        d.bx_log2 = eff_bxl();
        fill_coefs(d, rates);
        const double sc = (prec == LBM_FP16) ? std::ldexp(1.0, -e_scale) : 1.0;
        d.gscale = sc;
        d.inv_scale = 1.0 / sc;
        d.sr = sr_on() ? 1 : 0;
        d.sr_seed = sr_seed;
        return d;
    }
    bool sr_on() const { return sr && prec == LBM_FP16 && !inplace; }
    bool general() const { return rates.w12 != 1.0 || rates.w21 != 1.0 || rates.w22 != 1.0; }
};

// Upper bound of the number of tiles for any admissible tile shape.
inline long long max_items(int nx, int ny) { return (long long)nx * ny / 256 + nx + ny + 2; }

// Default launch shape per storage precision and lattice size (measured on
// MI355X: one workgroup per tile; wide tiles; several rows per thread for
// lattices whose step is short enough that launch overhead matters).
inline void default_tile(int prec, int nx, int ny, int& bx_log2, int& vy) {
    const bool big = (long long)nx * ny >= (1LL << 22);
    if (prec == LBM_FP64) {
        bx_log2 = 7;
        vy = 1;
    } else if (prec == LBM_FP32) {
        bx_log2 = 8;
        vy = big ? 1 : 4;
    } else {
        bx_log2 = big ? 6 : 7;
        vy = 4;
    }
    while (bx_log2 > 3 && (1 << bx_log2) > 2 * nx) --bx_log2;
}

template <typename S>
inline hipError_t launch_extract_u(const SlotDesc& d, int sel, int layout, double* ux, double* uy,
                                   hipStream_t st) {
    hipLaunchKernelGGL(k_extract_u<S>, dim3(blocks_for((long long)d.nx * d.ny)), dim3(kBlock), 0, st,
                       d, sel, layout, ux, uy);
    return hipGetLastError();
}
inline hipError_t extract_u(int prec, const SlotDesc& d, int sel, int layout, double* ux,
                            double* uy, hipStream_t st) {
    if (prec == LBM_FP64) return launch_extract_u<double>(d, sel, layout, ux, uy, st);
    if (prec == LBM_FP32) return launch_extract_u<float>(d, sel, layout, ux, uy, st);
    return launch_extract_u<__half>(d, sel, layout, ux, uy, st);
}

template <typename S>
inline hipError_t launch_stress(const SlotDesc& d, int sel, int layout, const Rates& r, double* a,
                                double* b, double* c, hipStream_t st) {
    hipLaunchKernelGGL(k_extract_stress<S>, dim3(blocks_for((long long)d.nx * d.ny)), dim3(kBlock), 0,
                       st, d, sel, layout, 1.0 - 0.5 * r.ws, 1.0 - 0.5 * r.wd, 1.0 - 0.5 * r.w11,
                       a, b, c);
    return hipGetLastError();
}

template <typename S>
inline hipError_t launch_get_f(const SlotDesc& d, int sel, int layout, double* f, hipStream_t st) {
    hipLaunchKernelGGL(k_get_f<S>, dim3(blocks_for((long long)d.nx * d.ny)), dim3(kBlock), 0, st, d,
                       sel, layout, f);
    return hipGetLastError();
}

template <typename S>
inline hipError_t launch_set_f(const SlotDesc& d, int sel, int layout, const double* f,
                               double scale, hipStream_t st) {
    hipLaunchKernelGGL(k_set_f<S>, dim3(blocks_for((long long)d.nx * d.ny)), dim3(kBlock), 0, st, d,
                       sel, layout, f, scale);
    return hipGetLastError();
}

template <typename S>
inline hipError_t launch_stream_only(unsigned grid, hipStream_t st, const StepLaunch& L,
                                     int layout) {
    if (layout == kLayNatural)
        hipLaunchKernelGGL((k_stream_only<S, kLayNatural>), dim3(grid), dim3(kBlock), 0, st, L);
    else if (layout == kLaySwapped)
        hipLaunchKernelGGL((k_stream_only<S, kLaySwapped>), dim3(grid), dim3(kBlock), 0, st, L);
    else
        hipLaunchKernelGGL((k_stream_only<S, kLayPull>), dim3(grid), dim3(kBlock), 0, st, L);
    return hipGetLastError();
}

inline hipError_t zero_bytes(void* p, size_t bytes, hipStream_t st) {
    const long long words = (long long)(bytes / 4);
    if (words == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(words)), dim3(kBlock), 0, st,
                       reinterpret_cast<unsigned int*>(p), words);
    return hipGetLastError();
}

// Measure the neutral modes of the stored state (blocking): out[0..3] =
// staggered sums and their force terms, out[4..5] = sum m10, sum m01.
// scratch: 8 * kErrBlocks + 12 doubles of device memory; host: 8 pinned doubles.
template <typename S>
inline hipError_t neutral_measure_t(const SlotDesc& d, int sel, double* scratch, double* host,
                                    hipStream_t st) {
    hipLaunchKernelGGL(k_neutral_sums<S>, dim3(kErrBlocks), dim3(kBlock), 0, st, d, sel, scratch);
    double* out = scratch + 8 * kErrBlocks;
    hipLaunchKernelGGL(k_reduce4<0>, dim3(1), dim3(kBlock), 0, st, scratch, kErrBlocks, out);
    hipLaunchKernelGGL(k_reduce4<0>, dim3(1), dim3(kBlock), 0, st, scratch + 4 * kErrBlocks,
                       kErrBlocks, out + 4);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(host, out, 8 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

inline hipError_t neutral_measure(int prec, const SlotDesc& d, int sel, double* scratch,
                                  double* host, hipStream_t st) {
    if (prec == LBM_FP64) return neutral_measure_t<double>(d, sel, scratch, host, st);
    if (prec == LBM_FP32) return neutral_measure_t<float>(d, sel, scratch, host, st);
    return neutral_measure_t<__half>(d, sel, scratch, host, st);
}

// Reset the neutral modes of the stored state to their exact values: the
// staggered sums of the stored field to `stag_target` and the mean first
// moments to `mean_target` (sum_x m10, sum_x m01), both of the exact trajectory
// (Lattice::stag_target_stored, Lattice::mean_target).  Stream-ordered, no
// host wait: the corrections are computed on the device.  scratch:
// 8 * kErrBlocks + 12 doubles of device memory.
template <typename S>
inline hipError_t neutral_reset_t(const SlotDesc& d, int sel, const double mean_target[2],
                                  const double stag_target[2], double* scratch, hipStream_t st) {
    hipLaunchKernelGGL(k_neutral_sums<S>, dim3(kErrBlocks), dim3(kBlock), 0, st, d, sel, scratch);
    double* out = scratch + 8 * kErrBlocks;
    hipLaunchKernelGGL(k_reduce4<0>, dim3(1), dim3(kBlock), 0, st, scratch, kErrBlocks, out);
    hipLaunchKernelGGL(k_reduce4<0>, dim3(1), dim3(kBlock), 0, st, scratch + 4 * kErrBlocks,
                       kErrBlocks, out + 4);
    double* coef = out + 8;
    hipLaunchKernelGGL(k_neutral_coef, dim3(1), dim3(1), 0, st, out, (double)d.nx * d.ny,
                       d.nx % 2 == 0 ? 1 : 0, d.ny % 2 == 0 ? 1 : 0, mean_target[0],
                       mean_target[1], stag_target[0], stag_target[1], 1.0 / d.inv_scale, coef);
    hipLaunchKernelGGL(k_neutral_fix<S>, dim3(blocks_for((long long)d.nx * d.ny)), dim3(kBlock), 0,
                       st, d, sel, coef);
    return hipGetLastError();
}

inline hipError_t neutral_reset(int prec, const SlotDesc& d, int sel, const double mean_target[2],
                                const double stag_target[2], double* scratch, hipStream_t st) {
    if (prec == LBM_FP64) return neutral_reset_t<double>(d, sel, mean_target, stag_target, scratch, st);
    if (prec == LBM_FP32) return neutral_reset_t<float>(d, sel, mean_target, stag_target, scratch, st);
    return neutral_reset_t<__half>(d, sel, mean_target, stag_target, scratch, st);
}

// Statistics of a force given as FP64 device arrays, raw or corrected
// (ForceSrc; two-stage reduction in a fixed order): stats[0..7] = sum gx,
// sum gy, sum gx^2 + gy^2, max |g|, the staggered sums (even nx / ny, else
// 0), 0, 0.  scratch: 8 * kErrBlocks doubles; stats: 8 doubles of device
// memory.  Stream-ordered.
inline hipError_t force_stats(const ForceSrc& src, double* scratch, double* stats, hipStream_t st) {
    hipLaunchKernelGGL(k_force_stats8, dim3(kErrBlocks), dim3(kBlock), 0, st, src, scratch);
    hipLaunchKernelGGL(k_reduce4<kForceMask>, dim3(1), dim3(kBlock), 0, st, scratch, kErrBlocks,
                       stats);
    hipLaunchKernelGGL(k_reduce4<0>, dim3(1), dim3(kBlock), 0, st, scratch + 4 * kErrBlocks,
                       kErrBlocks, stats + 4);
    return hipGetLastError();
}

inline ForceSrc raw_force(const double* gx, const double* gy, int nx, int ny) {
    ForceSrc f;
    f.gx = gx;
    f.gy = gy;
    f.nx = nx;
    f.ny = ny;
    f.n = (long long)nx * ny;
    return f;
}

// Warning bits of a force from its statistics (host): LBM_W_MEAN_REMOVED when
// force_mean_shift removes a mean, LBM_W_STAGGERED_LOAD when a staggered sum
// exceeds 1e-12 N rms (a load with a k = (pi, 0) or (0, pi) component: the
// staggered first moment then oscillates for good and the iteration from
// f = 0 has no steady state).
inline int force_warnings(const double* stats, long long N) {
    double shift[2];
    const double n = (double)N;
    force_mean_shift(stats, n, shift);
    int w = (shift[0] != 0.0 || shift[1] != 0.0) ? LBM_W_MEAN_REMOVED : 0;
    const double lim = 1e-24 * n * (0.5 * stats[2]);  // (1e-12 N rms)^2
    if (stats[4] * stats[4] > lim || stats[5] * stats[5] > lim) w |= LBM_W_STAGGERED_LOAD;
    return w;
}

// Mean-projected copy of the FP64 force (raw or corrected) into the
// lattice's arithmetic type (and the FP64 copy for the polish phase); stats:
// the force's statistics in device memory (force_stats), read by the kernel
// in stream order.
inline hipError_t upload_force(const Lattice& L, const ForceSrc& src, const double* stats,
                               hipStream_t st) {
    const long long N = L.N, P = L.plane;
    if (L.prec0 == LBM_FP64)
        hipLaunchKernelGGL(k_force_upload<double>, dim3(blocks_for(N)), dim3(kBlock), 0, st, src, P,
                           stats, reinterpret_cast<double*>(L.mem.g), (double*)nullptr);
    else
        hipLaunchKernelGGL(k_force_upload<float>, dim3(blocks_for(N)), dim3(kBlock), 0, st, src, P,
                           stats, reinterpret_cast<float*>(L.mem.g), L.mem.pg);
    return hipGetLastError();
}

// The host's record of a force just uploaded (stats on the host): max |g| for
// the half scale, and the sums that drive the neutral modes of the exact
// trajectory from step `steps` on (a removed mean leaves a zero sum).
inline void record_force(Lattice& L, const double* stats, long long steps) {
    double shift[2];
    force_mean_shift(stats, (double)L.N, shift);
    L.gmax = stats[3] + std::max(std::fabs(shift[0]), std::fabs(shift[1]));
    L.rebase_force(steps, shift[0] != 0.0 ? 0.0 : stats[0], shift[1] != 0.0 ? 0.0 : stats[1]);
    L.rebase_stagger(steps, stats[4], stats[5]);
}

// Initial power-of-two scale for half storage: the steady state of a load g
// is bounded by roughly max|g| / (mu k_min^2) with k_min = 2 pi / max(nx, ny);
// the populations are O(|u|).  Chosen so that this bound maps to ~2^12.
inline int initial_half_exponent(const Lattice& L, double gmax) {
    if (!(gmax > 0.0)) return 0;
    const double nmax = (double)std::max(L.nx, L.ny);
    const double kmin = 2.0 * M_PI / nmax;
    const double diff = std::min(L.mu, L.lam + L.mu);
    double bound = gmax / (std::max(diff, 1e-300) * kmin * kmin) + gmax;
    int e = (int)std::ceil(std::log2(bound / 4096.0));
    return std::max(-100, std::min(100, e));
}

}  // namespace lbm_host
