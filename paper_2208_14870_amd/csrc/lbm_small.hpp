// Whole solves of small lattices in one workgroup.
//
// A residual check every few steps makes a small lattice's solve launch-bound
// (the 32 x 32 workload moves 147 KB per step): each check costs a launch and
// a read of the residual by the host.  A lattice whose two population buffers
// fit in LDS runs instead in one workgroup that keeps the state in LDS, steps,
// evaluates the steady-state residual of Sec. 2.1 at the check steps with the
// same FP64 sums as the check kernels, and decides on the device when to stop,
// with the stopping rules of lbm_solve_to_tol (and the FP64 switch of narrow
// storage, which the host then performs).  The collision is the one every
// kernel uses, so the states are those of single steps bit for bit; the
// residual's sums run in another order (rounding only).
#pragma once

#include "lbm_common.hpp"
#include "lbm_fused.hpp"  // block_reduce3n, lds_ld, lds_st

namespace lbm {

constexpr int kSmallThreads = 512;

struct SmallLaunch {
    SlotDesc d;
    int sel;              // buffer holding the state (read at the start, written at the end)
    int have_prev;        // d.u holds u(m0 - 1) (FP64, unscaled)
    long long check;      // check interval K: checks at steps K, 2K, ... of the solve
    long long m0;         // steps the solve has taken before this launch
    long long budget;     // steps this launch may take at most
    long long max_steps;  // the solve's limit
    double tol;
    double r_in;          // the solve's last residual so far (NaN: none)
    double r_switch;      // > 0: narrow storage switches to FP64 (lbm_set_polish)
    int nondec_in;        // checks in a row whose residual did not decrease
    int guard_checks;     // divergence guard: rises in a row that stop the solve (0: off)
    RiseGuard* guard;     // the guard's state (device memory, kept across launches)
    double* out;          // steps after the launch, last residual, outcome, nondec
};

// Clear a divergence guard in device memory (start of a solve, FP64 switch).
static __global__ void k_guard_clear(RiseGuard* g) {
    if (threadIdx.x == 0 && blockIdx.x == 0) g->clear();
}

// Outcome codes in out[2].
constexpr int kSmallConverged = 0, kSmallLimit = 1, kSmallDiverged = 2, kSmallBudget = 3,
              kSmallSwitch = 4;

// One solve (or a budget of its steps) of an nx x ny lattice, nx * ny <= NMAX.
// The state at solve step m is the post-collision field f*(m - 1) (as stored in
// HBM).  A step pulls f(m) from it, forms u(m) while colliding and writes f*(m)
// to the other LDS buffer.  At a check step m the residual uses u(m) and u(m-1),
// the latter kept per site from the step before (or read from d.u at the start
// of a launch).  Stopping as lbm_solve_to_tol does: a residual that is not
// finite, r <= tol, the limit, or the divergence guard at a check step keeps
// the state of step m; the limit between checks keeps the state of the limit.
// With a switch threshold (narrow storage, lbm_set_polish), a check that finds
// the FP64 switch due ends the launch after step m + 1, and the host switches.
template <typename S, int NMAX, bool GENERAL>
static __global__ __launch_bounds__(kSmallThreads) void k_solve_small(SmallLaunch P) {
    using C = typename Store<S>::C;
    constexpr int NM = (NMAX + kSmallThreads - 1) / kSmallThreads;
    constexpr int NW = kSmallThreads / kWave;
    __shared__ S lds[2][8 * NMAX];
    __shared__ double red[3 * NW];
    __shared__ int flag;
    __shared__ double r_shared;
    __shared__ RiseGuard guard;  // updated by thread 0 only
    const SlotDesc& d = P.d;
    const int nx = d.nx, ny = d.ny, N = nx * ny;
    const long long plane = d.plane;
    Coef<C> k;
    k.load(d);
    const S* src = reinterpret_cast<const S*>(d.buf[P.sel]);
    const C* g = reinterpret_cast<const C*>(d.g);
    int sx[NM], sy[NM];  // own sites' coordinates (neighbours are formed per step)
    C gx[NM], gy[NM];
    double upx[NM], upy[NM];
    bool own[NM];
#pragma unroll
    for (int a = 0; a < NM; ++a) {
        const int e = (int)threadIdx.x + a * kSmallThreads;
        own[a] = e < N;
        const int ee = own[a] ? e : 0;
        sx[a] = ee % nx;
        sy[a] = ee / nx;
        gx[a] = own[a] ? glob(g)[ee] * k.gscale : C(0);
        gy[a] = own[a] ? glob(g)[plane + ee] * k.gscale : C(0);
        upx[a] = (own[a] && P.have_prev) ? glob(d.u)[ee] : 0.0;
        upy[a] = (own[a] && P.have_prev) ? glob(d.u)[plane + ee] : 0.0;
        if (own[a]) {
#pragma unroll
            for (int q = 0; q < 8; ++q) lds[0][q * NMAX + e] = glob(src)[q * plane + e];
        }
    }
    __syncthreads();
    int cur = 0;
    long long m = P.m0;
    const long long mend = P.max_steps - P.m0 > P.budget ? P.m0 + P.budget : P.max_steps;
    double r = P.r_in;
    int nondec = P.nondec_in;
    if (threadIdx.x == 0) guard = *P.guard;
    int outcome = kSmallBudget;
    while (true) {
        const bool check = m >= P.check && m % P.check == 0;
        // the budget ends a launch at any step (a check then opens the next
        // launch, with u(m - 1) from d.u); the limit ends the solve unless a
        // check falls on it
        if (m >= mend && !(check && m >= P.max_steps)) {
            outcome = m >= P.max_steps ? kSmallLimit : kSmallBudget;
            break;
        }
        C f[NM][8], ux[NM], uy[NM];
#pragma unroll
        for (int a = 0; a < NM; ++a) {
            if (!own[a]) continue;
            const int x = sx[a], y = sy[a];
            const int xm = (x == 0 ? nx : x) - 1, xp = (x + 1 == nx ? 0 : x + 1);
            const int rm = (y == 0 ? ny - 1 : y - 1) * nx, r0 = y * nx,
                      rp = (y + 1 == ny ? 0 : y + 1) * nx;
            // pull: f_q(x) = f*_q(x - c_q), velocity table order
            const S* b = lds[cur];
            f[a][0] = lds_ld<S>(b + 0 * NMAX + r0 + xm);
            f[a][1] = lds_ld<S>(b + 1 * NMAX + rm + x);
            f[a][2] = lds_ld<S>(b + 2 * NMAX + r0 + xp);
            f[a][3] = lds_ld<S>(b + 3 * NMAX + rp + x);
            f[a][4] = lds_ld<S>(b + 4 * NMAX + rm + xm);
            f[a][5] = lds_ld<S>(b + 5 * NMAX + rm + xp);
            f[a][6] = lds_ld<S>(b + 6 * NMAX + rp + xp);
            f[a][7] = lds_ld<S>(b + 7 * NMAX + rp + xm);
            collide<C, GENERAL>(f[a], gx[a], gy[a], k, ux[a], uy[a]);
        }
        int decision = 0;  // 0 go on, 1 stop at this step, 2 stop after it
        if (check) {
            double dsum = 0.0, ssum = 0.0, unused = 0.0;
#pragma unroll
            for (int a = 0; a < NM; ++a) {
                if (!own[a]) continue;
                const double uxd = (double)ux[a] * d.inv_scale, uyd = (double)uy[a] * d.inv_scale;
                const double dx = uxd - upx[a], dy = uyd - upy[a];
                dsum += dx * dx + dy * dy;
                ssum += uxd * uxd + uyd * uyd;
            }
            block_reduce3n<NW>(dsum, ssum, unused, red);
            if (threadIdx.x == 0) {
                double rr = (ssum == 0.0) ? (dsum == 0.0 ? 0.0 : INFINITY) : sqrt(dsum / ssum);
                if (dsum != dsum || ssum != ssum || !isfinite(ssum)) rr = NAN;
                int dec = 0, oc = kSmallBudget;
                if (!isfinite(rr) && !(ssum == 0.0 && dsum != 0.0)) {
                    dec = 1;
                    oc = kSmallDiverged;
                } else if (rr <= P.tol) {
                    dec = 1;
                    oc = kSmallConverged;
                } else if (m >= P.max_steps) {
                    dec = 1;
                    oc = kSmallLimit;
                } else if (guard.update(sqrt(dsum), P.guard_checks)) {
                    dec = 1;
                    oc = kSmallDiverged;
                } else if (P.r_switch > 0.0) {
                    // the switch of lbm_set_polish, after this step as between
                    // launches of the launch-per-check solve
                    nondec = (rr >= r) ? nondec + 1 : 0;
                    if (rr <= P.r_switch || nondec >= 2) {
                        dec = 2;
                        oc = kSmallSwitch;
                    }
                }
                flag = dec | (oc << 4);
                r_shared = rr;
            }
            __syncthreads();
            // flag and r_shared are next written at the next check, after the
            // barrier that ends this step and those of the next reduction
            decision = flag & 15;
            outcome = flag >> 4;
            r = r_shared;
            if (decision == 1) break;
        }
#pragma unroll
        for (int a = 0; a < NM; ++a) {
            if (!own[a]) continue;
            const int e = (int)threadIdx.x + a * kSmallThreads;
#pragma unroll
            for (int q = 0; q < 8; ++q) lds_st<S>(&lds[cur ^ 1][q * NMAX + e], f[a][q]);
            upx[a] = (double)ux[a] * d.inv_scale;
            upy[a] = (double)uy[a] * d.inv_scale;
        }
        __syncthreads();
        cur ^= 1;
        ++m;
        if (decision == 2) break;
    }
    // the state of step m back to its buffer, u(m - 1) to d.u for a next launch
    S* dst = reinterpret_cast<S*>(d.buf[P.sel]);
#pragma unroll
    for (int a = 0; a < NM; ++a) {
        if (!own[a]) continue;
        const int e = (int)threadIdx.x + a * kSmallThreads;
#pragma unroll
        for (int q = 0; q < 8; ++q) glob(dst)[q * plane + e] = lds[cur][q * NMAX + e];
        glob(d.u)[e] = upx[a];
        glob(d.u)[plane + e] = upy[a];
    }
    if (threadIdx.x == 0) {
        glob(P.out)[0] = (double)m;
        glob(P.out)[1] = r;
        glob(P.out)[2] = (double)outcome;
        glob(P.out)[3] = (double)nondec;
        *P.guard = guard;
    }
}

}  // namespace lbm
