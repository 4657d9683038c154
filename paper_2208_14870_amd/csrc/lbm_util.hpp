// Per-lattice helper kernels: extraction of u, stress and populations,
// conversions, FP64 norms, the work list and the neutral-mode reset.
#pragma once

#include "lbm_common.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// per-lattice helpers (1 thread per site)
// ---------------------------------------------------------------------------

// u(n) = bared first moments of f(n) (read from the stored field in its
// layout), FP64 and unscaled (Table "solution").
template <typename S>
static __global__ __launch_bounds__(kBlock) void k_extract_u(SlotDesc d, int sel, int layout,
                                                             double* ux, double* uy) {
    using C = typename Store<S>::C;
    const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= (long long)d.nx * d.ny) return;
    const int x = (int)(s % d.nx), y = (int)(s / d.nx);
    C f[8];
    load_state<S>(reinterpret_cast<const S*>(d.buf[sel]), d.plane, d.nx, d.ny, x, y, layout, f);
    const C* g = reinterpret_cast<const C*>(d.g);
    const double m10 = (double)((f[0] - f[2]) + ((f[4] - f[6]) - (f[5] - f[7])));
    const double m01 = (double)((f[1] - f[3]) + ((f[4] - f[6]) + (f[5] - f[7])));
    const double gsc = d.gscale;
    ux[s] = (m10 + 0.5 * (double)g[s] * gsc) * d.inv_scale;
    uy[s] = (m01 + 0.5 * (double)g[d.plane + s] * gsc) * d.inv_scale;
}

// Stress from the bared second-order moments of f(n) (Eq. compute_bared with
// zero equilibria, Table "solution" in lattice units): sxx = -(mb_s + mb_d)/2,
// syy = -(mb_s - mb_d)/2, sxy = -mb_11, mb = (1 - omega/2) m.
template <typename S>
static __global__ __launch_bounds__(kBlock) void k_extract_stress(SlotDesc d, int sel, int layout,
                                                                  double bs, double bd, double b11,
                                                                  double* sxx, double* syy,
                                                                  double* sxy) {
    using C = typename Store<S>::C;
    const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= (long long)d.nx * d.ny) return;
    const int x = (int)(s % d.nx), y = (int)(s / d.nx);
    C f[8];
    load_state<S>(reinterpret_cast<const S*>(d.buf[sel]), d.plane, d.nx, d.ny, x, y, layout, f);
    const double h13 = (double)f[0] + (double)f[2], h24 = (double)f[1] + (double)f[3];
    const double sac = (double)f[4] + (double)f[6], sbd = (double)f[5] + (double)f[7];
    const double ms = (h13 + h24) + 2.0 * (sac + sbd);
    const double md = h13 - h24;
    const double m11 = sac - sbd;
    const double mbs = bs * ms, mbd = bd * md, mb11 = b11 * m11;
    sxx[s] = -0.5 * (mbs + mbd) * d.inv_scale;
    syy[s] = -0.5 * (mbs - mbd) * d.inv_scale;
    sxy[s] = -mb11 * d.inv_scale;
}

// Populations f(n) in the paper's order, FP64 unscaled, from the stored field.
template <typename S>
static __global__ __launch_bounds__(kBlock) void k_get_f(SlotDesc d, int sel, int layout,
                                                         double* out) {
    using C = typename Store<S>::C;
    const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= (long long)d.nx * d.ny) return;
    const int x = (int)(s % d.nx), y = (int)(s / d.nx);
    C f[8];
    load_state<S>(reinterpret_cast<const S*>(d.buf[sel]), d.plane, d.nx, d.ny, x, y, layout, f);
    const long long N = (long long)d.nx * d.ny;  // external layout [8][ny][nx]
    for (int q = 0; q < 8; ++q) out[q * N + s] = (double)f[q] * d.inv_scale;
}

// Load a state f(n) given in the paper's order.  kLayPull and kLaySwapped
// store f*(n-1)(x) = f(n)(x + c_q) (the inverse of the gather), in plane q or
// plane opp(q); kLayNatural stores f(n) itself.
template <typename S>
static __global__ __launch_bounds__(kBlock) void k_set_f(SlotDesc d, int sel, int layout,
                                                         const double* in, double scale) {
    const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= (long long)d.nx * d.ny) return;
    const int x = (int)(s % d.nx), y = (int)(s / d.nx);
    const int xm = (x == 0) ? d.nx - 1 : x - 1, xp = (x == d.nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? d.ny - 1 : y - 1, yp = (y == d.ny - 1) ? 0 : y + 1;
    S* dst = reinterpret_cast<S*>(d.buf[sel]);
    const long long N = (long long)d.nx * d.ny;  // external layout [8][ny][nx]
    const int cx[8] = {1, 0, -1, 0, 1, -1, -1, 1};
    const int cy[8] = {0, 1, 0, -1, 1, 1, -1, -1};
    for (int q = 0; q < 8; ++q) {
        const bool nat = layout == kLayNatural;
        const int xs = nat ? x : (cx[q] > 0 ? xp : (cx[q] < 0 ? xm : x));
        const int ys = nat ? y : (cy[q] > 0 ? yp : (cy[q] < 0 ? ym : y));
        const double v = in[q * N + (long long)ys * d.nx + xs] * scale;
        const int plane_q = layout == kLaySwapped ? opp(q) : q;
        Store<S>::st(dst + plane_q * d.plane + s, (typename Store<S>::C)v);
    }
}

// Convert an FP64 array to the arithmetic type (force upload).
template <typename C>
static __global__ __launch_bounds__(kBlock) void k_convert(const double* in, C* out, long long n) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = (C)in[i];
}

// out = in * factor elementwise, between storage types (promotion for the
// FP64 polish phase, power-of-two rescaling of half storage).
template <typename SI, typename SO>
static __global__ __launch_bounds__(kBlock) void k_recast(const SI* in, SO* out, long long n,
                                                   double factor) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double v = (double)Store<SI>::ld(in + i) * factor;
    Store<SO>::st(out + i, (typename Store<SO>::C)v);
}

// Zero fill by a kernel (safe inside captured graphs).
static __global__ __launch_bounds__(kBlock) void k_zero(unsigned int* p, long long nwords) {
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (i < nwords) p[i] = 0u;
}

// Deterministic (fixed-order) block reduction of four values; MAXMASK bit c
// set means entry c is reduced with max instead of +.  Result in thread 0.
template <int MAXMASK>
__device__ __forceinline__ void block_reduce4(double v[4], double* lds) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double w = __shfl_xor(v[c], o, kWave);
            v[c] = ((MAXMASK >> c) & 1) ? fmax(v[c], w) : v[c] + w;
        }
    }
    const int wv = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0)
        for (int c = 0; c < 4; ++c) lds[4 * wv + c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            v[c] = ((MAXMASK >> c) & 1)
                       ? fmax(fmax(lds[c], lds[4 + c]), fmax(lds[8 + c], lds[12 + c]))
                       : (lds[c] + lds[4 + c]) + (lds[8 + c] + lds[12 + c]);
    }
    __syncthreads();
}

// Error norms against a reference field, stage 1: per block
// (sum |e|^2, sum |ref|^2, max |e|_inf, max |ref|_inf), e = u - ref (the grid
// norms of Sec. 7.1 before the dx weighting).
constexpr int kErrMask = 0xC;
static __global__ __launch_bounds__(kBlock) void k_err_norms(const double* ux, const double* uy,
                                                      const double* rx, const double* ry,
                                                      long long n, double* partial) {
    __shared__ double lds[16];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const double ex = ux[i] - rx[i], ey = uy[i] - ry[i];
        v[0] += ex * ex + ey * ey;
        v[1] += rx[i] * rx[i] + ry[i] * ry[i];
        v[2] = fmax(v[2], fmax(fabs(ex), fabs(ey)));
        v[3] = fmax(v[3], fmax(fabs(rx[i]), fabs(ry[i])));
    }
    block_reduce4<kErrMask>(v, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) partial[4 * blockIdx.x + c] = v[c];
}

// Force statistics, stage 1: per block (sum gx, sum gy, sum gx^2 + gy^2,
// max |g|_inf).
constexpr int kForceMask = 0x8;
static __global__ __launch_bounds__(kBlock) void k_force_stats(const double* gx, const double* gy,
                                                        long long n, double* partial) {
    __shared__ double lds[16];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        v[0] += gx[i];
        v[1] += gy[i];
        v[2] += gx[i] * gx[i] + gy[i] * gy[i];
        v[3] = fmax(v[3], fmax(fabs(gx[i]), fabs(gy[i])));
    }
    block_reduce4<kForceMask>(v, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) partial[4 * blockIdx.x + c] = v[c];
}

// Statistics of a body force given as FP64 arrays [ny][nx], stage 1: per block
// two groups of four, (sum gx, sum gy, sum gx^2 + gy^2, max |g|_inf) into
// partial[4 b ..] and (sum (-1)^x gx for even nx, sum (-1)^y gy for even ny,
// 0, 0) into partial[4 (gridDim + b) ..].  The staggered sums drive the
// undamped modes at k = (pi, 0), (0, pi) (see k_neutral_sums).
// The per-step force as the library takes it in: the caller's FP64 arrays,
// or those arrays with the leading-order correction of the improved scheme
// (Sec. 4, Eqs. force_correction_x/y):
//   gx' = gx - (D1 d_xx gx + D2 d_xy gy + D3 d_yy gx),
//   gy' = gy - (E3 d_xx gy + E2 d_xy gx + E1 d_yy gy),
// with (D1, D2, D3) the x row's constants, (E1, E2, E3) the y row's (equal to
// the x row's when tau_12 = tau_21).  The second derivatives are either given
// (d2: six FP64 planes d_xx gx, d_xy gx, d_yy gx, d_xx gy, d_xy gy, d_yy gy)
// or the second-order central differences of g on the periodic lattice.
struct ForceSrc {
    enum { kRaw = 0, kGiven = 1, kCentral = 2 };
    const double* gx = nullptr;
    const double* gy = nullptr;
    const double* d2 = nullptr;
    long long n = 0;
    int nx = 0, ny = 0, mode = kRaw;
    double cx[3] = {0, 0, 0}, cy[3] = {0, 0, 0};

    // d_xx, d_xy, d_yy of one component at (x, y) by central differences
    __device__ void central(const double* g, int x, int y, double out[3]) const {
#pragma clang fp contract(off)
        const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
        const int yp = y + 1 == ny ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
        const long long r = (long long)y * nx, rp = (long long)yp * nx, rm = (long long)ym * nx;
        const double c = g[r + x];
        out[0] = (g[r + xp] - 2.0 * c) + g[r + xm];
        out[1] = ((g[rp + xp] - g[rp + xm]) - (g[rm + xp] - g[rm + xm])) * 0.25;
        out[2] = (g[rp + x] - 2.0 * c) + g[rm + x];
    }
    __device__ void at(long long i, int x, int y, double& vx, double& vy) const {
#pragma clang fp contract(off)
        vx = gx[i];
        vy = gy[i];
        if (mode == kRaw) return;
        double ax[3], ay[3];
        if (mode == kGiven) {
            for (int c = 0; c < 3; ++c) {
                ax[c] = d2[c * n + i];
                ay[c] = d2[(3 + c) * n + i];
            }
        } else {
            central(gx, x, y, ax);
            central(gy, x, y, ay);
        }
        const double hx = vx - ((cx[0] * ax[0] + cx[1] * ay[1]) + cx[2] * ax[2]);
        const double hy = vy - ((cy[2] * ay[0] + cy[1] * ax[1]) + cy[0] * ay[2]);
        vx = hx;
        vy = hy;
    }
};

static __global__ __launch_bounds__(kBlock) void k_force_stats8(ForceSrc src, double* partial) {
    __shared__ double lds[16];
    const int nx = src.nx, ny = src.ny;
    const long long n = src.n;
    const double sx = (nx % 2 == 0) ? 1.0 : 0.0, sy = (ny % 2 == 0) ? 1.0 : 0.0;
    double v[4] = {0.0, 0.0, 0.0, 0.0}, w[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const int x = (int)(i % nx), y = (int)(i / nx);
        double gx, gy;
        src.at(i, x, y, gx, gy);
        v[0] += gx;
        v[1] += gy;
        v[2] += gx * gx + gy * gy;
        v[3] = fmax(v[3], fmax(fabs(gx), fabs(gy)));
        w[0] += ((x & 1) ? -sx : sx) * gx;
        w[1] += ((y & 1) ? -sy : sy) * gy;
    }
    block_reduce4<kForceMask>(v, lds);
    block_reduce4<0>(w, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) {
            partial[4 * blockIdx.x + c] = v[c];
            partial[4 * (gridDim.x + blockIdx.x) + c] = w[c];
        }
}
// st (8 doubles of k_force_stats8 after stage 2).  A zero shift copies g bit
// for bit.
template <typename C>
static __global__ __launch_bounds__(kBlock) void k_force_upload(ForceSrc src, long long plane,
                                                                const double* st, C* out,
                                                                double* out64) {
#pragma clang fp contract(off)
    const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    const long long n = src.n;
    if (i >= n) return;
    double shift[2], gx, gy;
    force_mean_shift(st, (double)n, shift);
    src.at(i, (int)(i % src.nx), (int)(i / src.nx), gx, gy);
    const double vx = gx - shift[0], vy = gy - shift[1];
    out[i] = (C)vx;
    out[plane + i] = (C)vy;
    if (out64) {
        out64[i] = vx;
        out64[plane + i] = vy;
    }
}

// Stage 2: one block combines the block partials in a fixed order.
template <int MAXMASK>
static __global__ __launch_bounds__(kBlock) void k_reduce4(const double* partial, int nparts,
                                                    double* out) {
    __shared__ double lds[16];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nparts; i += kBlock)
        for (int c = 0; c < 4; ++c)
            v[c] = ((MAXMASK >> c) & 1) ? fmax(v[c], partial[4 * i + c])
                                         : v[c] + partial[4 * i + c];
    block_reduce4<MAXMASK>(v, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) out[c] = v[c];
}

// Write the work list of one lattice: tiles in vertical bands `band` tiles
// wide, each band row by row (band >= tiles_x: row-major order).  Each XCD
// walks a contiguous slice of the list, so a tile's neighbours above and
// below (whose rings overlap its own) run shortly before and after it on the
// same XCD and find those rows in its L2 (measured on MI355X with bands of 8
// tiles: 8192^2 FP32 286 against 271 GLUPS, 2048^2 FP64 119 against 111).
static __global__ __launch_bounds__(kBlock) void k_build_items(Item* items, int first, int slot,
                                                        int tiles_x, int count, int band) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= count) return;
    Item it;
    it.slot = slot;
    if (band <= 0 || band >= tiles_x) {
        it.tx = i % tiles_x;
        it.ty = i / tiles_x;
    } else {
        const int tiles_y = count / tiles_x;
        const int per = band * tiles_y;  // items of a full band
        const int b = i / per, j = i - b * per;
        const int w = min(band, tiles_x - b * band);  // the last band may be narrower
        it.ty = j / w;
        it.tx = b * band + j % w;
    }
    it.pad_ = 0;
    items[first + i] = it;
}

// Small device-side stores (stream-ordered, safe inside captured graphs).
static __global__ void k_set_int(int* p, int v) { *p = v; }
static __global__ void k_set_desc(SlotDesc* p, SlotDesc v) { *p = v; }
// the step count of the stochastic-rounding bits, after a launch of ns steps
static __global__ void k_add_sr_step(SlotDesc* p, int ns) { p->sr_step += (unsigned)ns; }

// Neutral modes.  (1) The mean first moments: collision adds g to m10, m01 and
// streaming permutes, so sum_x m10(f(n)) = sum_x m10(f(0)) + n sum_x gx exactly
// (eigenvalue 1 at k = 0).  (2) The staggered first moments: for even nx,
// J = sum_x (-1)^x m10(f(n)) obeys J(n+1) = -J(n) - sum_x (-1)^x gx for any
// relaxation rates (streaming with c_x = +-1 flips (-1)^x), and likewise in y
// with m01, gy: eigenvalue -1 at k = (pi, 0), (0, pi), so that
// J(n) = -G/2 + (-1)^(n - n0) (J(n0) + G/2) oscillates about -G/2 with a
// constant amplitude.  Neither mode is ever damped, so rounding noise from
// narrow storage stays in them for good.  These kernels measure both on the
// stored (post-collision) field S = f*(n-1), whose sums equal those of f(n)
// for the mean and J_S = J(n-1) + G = -J(n) for the staggered mode, and reset
// them to the exact trajectory's values (tracked on the host).
//
// Stage 1: per block two groups of four sums, unscaled FP64:
// (sum (-1)^x m10(S), sum (-1)^y m01(S), sum (-1)^x gx, sum (-1)^y gy) and
// (sum m10(S), sum m01(S), 0, 0).
template <typename S>
static __global__ __launch_bounds__(kBlock) void k_neutral_sums(SlotDesc d, int sel,
                                                                double* partial) {
    __shared__ double lds[16];
    using C = typename Store<S>::C;
    const long long N = (long long)d.nx * d.ny;
    const S* st = reinterpret_cast<const S*>(d.buf[sel]);
    const C* g = reinterpret_cast<const C*>(d.g);
    const double sx = (d.nx % 2 == 0) ? 1.0 : 0.0, sy = (d.ny % 2 == 0) ? 1.0 : 0.0;
    double v[4] = {0.0, 0.0, 0.0, 0.0}, w[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long s = (long long)blockIdx.x * kBlock + threadIdx.x; s < N;
         s += (long long)gridDim.x * kBlock) {
        const int x = (int)(s % d.nx), y = (int)(s / d.nx);
        double f[8];
        for (int q = 0; q < 8; ++q) f[q] = (double)Store<S>::ld(st + q * d.plane + s);
        const double m10 = ((f[0] - f[2]) + ((f[4] - f[6]) - (f[5] - f[7]))) * d.inv_scale;
        const double m01 = ((f[1] - f[3]) + ((f[4] - f[6]) + (f[5] - f[7]))) * d.inv_scale;
        const double px = (x & 1) ? -sx : sx, py = (y & 1) ? -sy : sy;
        v[0] += px * m10;
        v[1] += py * m01;
        v[2] += px * (double)g[s];
        v[3] += py * (double)g[d.plane + s];
        w[0] += m10;
        w[1] += m01;
    }
    block_reduce4<0>(v, lds);
    block_reduce4<0>(w, lds);
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) {
            partial[4 * blockIdx.x + c] = v[c];
            partial[4 * (gridDim.x + blockIdx.x) + c] = w[c];
        }
}

// The four corrections of stage 2 from the stage-1 sums (8 doubles, after the
// second reduction) and the targets, in storage units (sc = 1 / inv_scale):
// the staggered sums of the stored field go to (jx, jy) and the means to
// (tx, ty), the values of the exact trajectory (an update of eps changes
// either by 2 eps N).  One thread, on the device, so the reset needs no host
// round trip; each operation rounds on its own.
static __global__ void k_neutral_coef(const double* sums, double n, int evenx, int eveny,
                                      double tx, double ty, double jx, double jy, double sc,
                                      double* coef) {
#pragma clang fp contract(off)
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double ex = evenx ? (jx - sums[0]) / (2.0 * n) : 0.0;
    const double ey = eveny ? (jy - sums[1]) / (2.0 * n) : 0.0;
    const double mx = (tx - sums[4]) / (2.0 * n);
    const double my = (ty - sums[5]) / (2.0 * n);
    coef[0] = ex * sc;
    coef[1] = ey * sc;
    coef[2] = mx * sc;
    coef[3] = my * sc;
}

// Stage 2: S1 += (ex (-1)^x + mx), S3 -= (ex (-1)^x + mx),
//          S2 += (ey (-1)^y + my), S4 -= (ey (-1)^y + my)
// (changes only m10 / m01 of S: the staggered and the uniform parts; coef =
// {ex, ey, mx, my} in device memory, already in storage units).
template <typename S>
static __global__ __launch_bounds__(kBlock) void k_neutral_fix(SlotDesc d, int sel,
                                                               const double* coef) {
    using C = typename Store<S>::C;
    const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= (long long)d.nx * d.ny) return;
    const int x = (int)(s % d.nx), y = (int)(s / d.nx);
    const double ex = coef[0], ey = coef[1], mx = coef[2], my = coef[3];
    S* st = reinterpret_cast<S*>(d.buf[sel]);
    const double px = ((x & 1) ? -ex : ex) + mx, py = ((y & 1) ? -ey : ey) + my;
    S* p0 = st + 0 * d.plane + s;
    S* p1 = st + 1 * d.plane + s;
    S* p2 = st + 2 * d.plane + s;
    S* p3 = st + 3 * d.plane + s;
    Store<S>::st(p0, (C)((double)Store<S>::ld(p0) + px));
    Store<S>::st(p2, (C)((double)Store<S>::ld(p2) - px));
    Store<S>::st(p1, (C)((double)Store<S>::ld(p1) + py));
    Store<S>::st(p3, (C)((double)Store<S>::ld(p3) - py));
}

}  // namespace lbm
