// Device code of the MI355X (gfx950) lattice Boltzmann elasticity library.
//
// Scheme: Boolakee, Geier, De Lorenzis, arXiv 2208.14870.  One time step is
// Algorithm 1 -- moments, half forcing, equilibria (Table "scheme"),
// relaxation (Eq. collision), second half forcing, back-transformation
// (Eq. moments_post) and streaming (Eq. streaming) -- fused into one pass
// over the lattice in "pull" form: each site gathers the post-collision
// populations of its upstream neighbours from buffer A (periodic wrap by
// index arithmetic, Sec. 6.1), collides them in registers and writes its own
// post-collision populations to buffer B.  The stored state is therefore the
// post-collision field f*(n-1); f(n) is obtained by the same gather.
//
// Populations: D2Q8 (the rest population is never read by any equilibrium
// or relaxed moment, Sec. 3.3.2), one-index order of the velocity table of
// Sec. 5: 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1) 5:(1,1) 6:(-1,1) 7:(-1,-1)
// 8:(1,-1), stored as eight SoA planes [q][y][x], x fastest.
//
// Storage precision S in {double, float, __half}; arithmetic type C is
// double for double storage and float otherwise.  Half storage holds the
// populations times a per-lattice power of two 2^-e (the problem is linear,
// and the rest equilibrium of this scheme is identically zero, so the stored
// value is the deviation from rest); the force is multiplied by the same
// factor inside the kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace lbm {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64s)
constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// per-lattice descriptor (device memory, read once per tile)
// ---------------------------------------------------------------------------
struct SlotDesc {
    void* buf[2];          // two population buffers, 8 planes each
    const void* g;         // force, 2 planes in the arithmetic type
    double* u;             // 2 planes FP64: displacement of the last check launch
    long long plane;       // elements per plane = nx * ny
    int nx, ny;
    int cur;               // buffer index holding the state at launch flip 0
    int tiles_x, tiles_y;  // tile grid of this lattice
    int bx_log2;           // tile width in threads = 1 << bx_log2 (tile height = 256 >> bx_log2)
    int general;           // nonzero: general omega_12/21/22 and theta (host sets the launch variant)
    int pad_;
    // fast-path coefficients (omega_12 = omega_21 = omega_22 = 1)
    double cs, cd, c11, hth, tq;
    // general-path rates
    double a11, as, ad, theta, w12, w21, a22;
    double gscale;     // factor applied to the force (2^-e for half storage, else 1)
    double inv_scale;  // 1 / storage factor, applied to outputs
};

struct Item {
    int slot;
    int tx, ty;
    int pad_;
};

// ---------------------------------------------------------------------------
// storage traits.  Every population is read once and written once per step,
// so loads and stores carry the non-temporal hint (measured on MI355X: best
// for both cache-resident and HBM-resident lattices).
// ---------------------------------------------------------------------------
//
// Pointers taken from a descriptor in memory are generic, and the compiler
// then emits flat instructions, which also count on the LDS/scalar counter:
// a wait for an LDS read or a descriptor load would wait for every flat
// store in flight.  All lattice memory is global, so accesses go through
// an explicit global address-space pointer.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> glob(T* p) { return (gptr<T>)p; }

template <typename S> struct Store;
template <> struct Store<double> {
    using C = double;
    __device__ static __forceinline__ C ld(const double* p) {
        return __builtin_nontemporal_load(glob(p));
    }
    __device__ static __forceinline__ void st(double* p, C v) {
        __builtin_nontemporal_store(v, glob(p));
    }
};
template <> struct Store<float> {
    using C = float;
    __device__ static __forceinline__ C ld(const float* p) {
        return __builtin_nontemporal_load(glob(p));
    }
    __device__ static __forceinline__ void st(float* p, C v) {
        __builtin_nontemporal_store(v, glob(p));
    }
};
template <> struct Store<__half> {
    using C = float;
    __device__ static __forceinline__ C ld(const __half* p) {
        return __half2float(__ushort_as_half(*glob(reinterpret_cast<const unsigned short*>(p))));
    }
    __device__ static __forceinline__ void st(__half* p, C v) {
        __half h = __float2half_rn(v);
        __builtin_nontemporal_store(__half_as_ushort(h), glob(reinterpret_cast<unsigned short*>(p)));
    }
};

// ---------------------------------------------------------------------------
// collision of one site (Algorithm 1, collision block), in registers
// ---------------------------------------------------------------------------
template <typename C>
struct Coef {
    C cs, cd, c11, hth, tq;           // fast path
    C a11, as, ad, theta, w12, w21, a22;  // general path
    C gscale;
    __device__ __forceinline__ void load(const SlotDesc& d) {
        cs = (C)d.cs; cd = (C)d.cd; c11 = (C)d.c11; hth = (C)d.hth; tq = (C)d.tq;
        a11 = (C)d.a11; as = (C)d.as; ad = (C)d.ad; theta = (C)d.theta;
        w12 = (C)d.w12; w21 = (C)d.w21; a22 = (C)d.a22;
        gscale = (C)d.gscale;
    }
};

// f[0..7] in: pre-collision populations; out: post-collision populations.
// gx, gy: (scaled) force.  Returns the bared first-order moments (ux, uy).
//
// Moments (Eqs. moments / replace_raw, transformed directly into the
// collision set as the paper recommends):
//   m10 = f1 - f3 + f5 - f6 - f7 + f8      m01 = f2 - f4 + f5 + f6 - f7 - f8
//   m11 = f5 - f6 + f7 - f8                ms  = f1 + f2 + f3 + f4 + 2(f5+f6+f7+f8)
//   md  = f1 - f2 + f3 - f4                m12 = f5 - f6 - f7 + f8
//   m21 = f5 + f6 - f7 - f8                m22 = f5 + f6 + f7 + f8
// Bared first moments ux = m10 + gx/2, uy = m01 + gy/2 (Eqs. coll10/coll01);
// equilibria m12_eq = theta ux, m21_eq = theta uy, all others 0 (Table
// "scheme"); relaxation m* = omega m_eq + (1 - omega) m (Eq. collision);
// m10* = ux + gx/2, m01* = uy + gy/2 (Eqs. coll10post/coll01post); then
// f* = M^-1 m* with the exact (dyadic) inverse of the transform of Sec. 5.
//
// Fast path (omega_12 = omega_21 = omega_22 = 1, so m12* = theta ux,
// m21* = theta uy, m22* = 0), with cs = (1-omega_s)/4, cd = (1-omega_d)/4,
// c11 = (1-omega_11)/4, hth = (1-theta)/2, tq = theta/4:
//   f1*,f3* = cs ms + cd md +- (hth ux + gx/4)
//   f2*,f4* = cs ms - cd md +- (hth uy + gy/4)
//   f5*,f7* =  c11 m11 +- tq (ux + uy)
//   f6*,f8* = -c11 m11 -+ tq (ux - uy)
//
// Rounding is fixed by the source: contraction is off inside and the fused
// multiply-adds are written out, so every kernel that calls this (single
// step, fused steps, any unrolled copy) rounds every site identically.
__device__ __forceinline__ float fmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Bared first moments ux = m10 + gx/2, uy = m01 + gy/2 of a site (the
// collision's own operations, also used by the residual check without a step).
template <typename C>
__device__ __forceinline__ void bared_u(const C f[8], C gx, C gy, C& ux, C& uy) {
#pragma clang fp contract(off)
    const C p = f[4] - f[6], q = f[5] - f[7];
    ux = ((f[0] - f[2]) + (p - q)) + C(0.5) * gx;
    uy = ((f[1] - f[3]) + (p + q)) + C(0.5) * gy;
}

template <typename C, bool GENERAL>
__device__ __forceinline__ void collide(C f[8], C gx, C gy, const Coef<C>& k, C& ux, C& uy) {
#pragma clang fp contract(off)
    const C p = f[4] - f[6];   // f5 - f7
    const C q = f[5] - f[7];   // f6 - f8
    const C h13 = f[0] + f[2];
    const C h24 = f[1] + f[3];
    const C sac = f[4] + f[6];
    const C sbd = f[5] + f[7];
    const C m12 = p - q;
    const C m21 = p + q;
    const C m10 = (f[0] - f[2]) + m12;
    const C m01 = (f[1] - f[3]) + m21;
    const C m11 = sac - sbd;
    const C ms = (h13 + h24) + C(2) * (sac + sbd);
    const C md = h13 - h24;
    const C hgx = C(0.5) * gx, hgy = C(0.5) * gy;
    ux = m10 + hgx;
    uy = m01 + hgy;
    if constexpr (!GENERAL) {
        const C dd = k.cd * md;
        const C a = fmac(k.cs, ms, dd);
        const C b = fmac(k.cs, ms, -dd);
        const C ex = fmac(k.hth, ux, C(0.5) * hgx);
        const C ey = fmac(k.hth, uy, C(0.5) * hgy);
        const C s = k.c11 * m11;
        const C t1 = k.tq * (ux + uy);
        const C t2 = k.tq * (ux - uy);
        f[0] = a + ex;
        f[2] = a - ex;
        f[1] = b + ey;
        f[3] = b - ey;
        f[4] = s + t1;
        f[6] = s - t1;
        f[5] = -(s + t2);
        f[7] = t2 - s;
    } else {
        const C m22 = sac + sbd;
        const C s10 = ux + hgx, s01 = uy + hgy;
        const C s11 = k.a11 * m11;
        const C sss = k.as * ms;
        const C sdd = k.ad * md;
        const C s12 = k.w12 * (k.theta * ux) + (C(1) - k.w12) * m12;
        const C s21 = k.w21 * (k.theta * uy) + (C(1) - k.w21) * m21;
        const C s22 = k.a22 * m22;
        const C A = C(0.5) * (sss + sdd) - s22;  // m20* - m22*
        const C B = C(0.5) * (sss - sdd) - s22;  // m02* - m22*
        const C ex = s10 - s12, ey = s01 - s21;
        f[0] = C(0.5) * (A + ex);
        f[2] = C(0.5) * (A - ex);
        f[1] = C(0.5) * (B + ey);
        f[3] = C(0.5) * (B - ey);
        f[4] = C(0.25) * ((s22 + s11) + (s12 + s21));
        f[5] = C(0.25) * ((s22 - s11) - (s12 - s21));
        f[6] = C(0.25) * ((s22 + s11) - (s12 + s21));
        f[7] = C(0.25) * ((s22 - s11) + (s12 - s21));
    }
}

// ---------------------------------------------------------------------------
// storage layouts of the populations
// ---------------------------------------------------------------------------
// kLayPull: two buffers; a buffer holds the post-collision field f*(n-1) at
//   its own sites (plane q = f*_q), and a step pulls f(n)(x) = f*(x - c_q).
// In-place streaming (one buffer, the "AA" access pattern) alternates two
// layouts of the same buffer, so that every step reads and writes each
// population once and a site touches only locations no other site touches:
// kLayNatural: the buffer holds f(n) itself (plane q at x = f_q(x)); the step
//   reads a site's own planes and writes f*_q into plane opp(q) of the same
//   site, leaving kLaySwapped.
// kLaySwapped: plane opp(q) at x holds f*_q(x), so f(n)_q(x) is plane opp(q)
//   at x - c_q; the step reads those and writes f*_q into plane q at x + c_q,
//   which is f(n+1)_q there: the buffer is back in kLayNatural.
enum Layout : int { kLayPull = 0, kLayNatural = 1, kLaySwapped = 2 };

// opposite direction: c_opp(q) = -c_q (paper order 1..8 -> 0..7)
__host__ __device__ constexpr int opp(int q) { return q < 4 ? q ^ 2 : 4 + ((q - 4) ^ 2); }

// ---------------------------------------------------------------------------
// pull-gather of the 8 populations arriving at (x, y); SWAP reads plane opp(q)
// ---------------------------------------------------------------------------
template <typename S, bool SWAP = false>
__device__ __forceinline__ void gather(const S* src, long long plane, int nx, int ny, int x, int y,
                                       typename Store<S>::C f[8]) {
    const int xm = (x == 0) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    const long long r0 = (long long)y * nx, rm = (long long)ym * nx, rp = (long long)yp * nx;
    auto pl = [](int q) { return SWAP ? opp(q) : q; };
    f[0] = Store<S>::ld(src + pl(0) * plane + r0 + xm);  // c1 = ( 1, 0) from (x-1, y)
    f[1] = Store<S>::ld(src + pl(1) * plane + rm + x);   // c2 = ( 0, 1) from (x, y-1)
    f[2] = Store<S>::ld(src + pl(2) * plane + r0 + xp);  // c3 = (-1, 0) from (x+1, y)
    f[3] = Store<S>::ld(src + pl(3) * plane + rp + x);   // c4 = ( 0,-1) from (x, y+1)
    f[4] = Store<S>::ld(src + pl(4) * plane + rm + xm);  // c5 = ( 1, 1) from (x-1, y-1)
    f[5] = Store<S>::ld(src + pl(5) * plane + rm + xp);  // c6 = (-1, 1) from (x+1, y-1)
    f[6] = Store<S>::ld(src + pl(6) * plane + rp + xp);  // c7 = (-1,-1) from (x+1, y+1)
    f[7] = Store<S>::ld(src + pl(7) * plane + rp + xm);  // c8 = ( 1,-1) from (x-1, y+1)
}

// push of f*_q to plane q at x + c_q (in-place odd step)
template <typename S>
__device__ __forceinline__ void scatter(S* dst, long long plane, int nx, int ny, int x, int y,
                                        const typename Store<S>::C f[8]) {
    const int xm = (x == 0) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    const long long r0 = (long long)y * nx, rm = (long long)ym * nx, rp = (long long)yp * nx;
    Store<S>::st(dst + 0 * plane + r0 + xp, f[0]);  // c1 = ( 1, 0) to (x+1, y)
    Store<S>::st(dst + 1 * plane + rp + x, f[1]);   // c2 = ( 0, 1) to (x, y+1)
    Store<S>::st(dst + 2 * plane + r0 + xm, f[2]);  // c3 = (-1, 0) to (x-1, y)
    Store<S>::st(dst + 3 * plane + rm + x, f[3]);   // c4 = ( 0,-1) to (x, y-1)
    Store<S>::st(dst + 4 * plane + rp + xp, f[4]);  // c5 = ( 1, 1) to (x+1, y+1)
    Store<S>::st(dst + 5 * plane + rp + xm, f[5]);  // c6 = (-1, 1) to (x-1, y+1)
    Store<S>::st(dst + 6 * plane + rm + xm, f[6]);  // c7 = (-1,-1) to (x-1, y-1)
    Store<S>::st(dst + 7 * plane + rm + xp, f[7]);  // c8 = ( 1,-1) to (x+1, y-1)
}

// f(n) at (x, y) from a buffer in any layout
template <typename S>
__device__ __forceinline__ void load_state(const S* buf, long long plane, int nx, int ny, int x,
                                           int y, int layout, typename Store<S>::C f[8]) {
    if (layout == kLayPull) {
        gather<S, false>(buf, plane, nx, ny, x, y, f);
    } else if (layout == kLaySwapped) {
        gather<S, true>(buf, plane, nx, ny, x, y, f);
    } else {
        const long long s = (long long)y * nx + x;
        for (int q = 0; q < 8; ++q) f[q] = Store<S>::ld(buf + q * plane + s);
    }
}

// ---------------------------------------------------------------------------
// wave64 / block reductions (fixed order: deterministic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
    return v;
}

// Reduce (sum, sum, max) over the 256 threads; result valid in thread 0.
__device__ __forceinline__ void block_reduce3(double& a, double& b, double& m, double* lds) {
    a = wave_sum(a);
    b = wave_sum(b);
    m = wave_max(m);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) {
        lds[3 * w + 0] = a;
        lds[3 * w + 1] = b;
        lds[3 * w + 2] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = (lds[0] + lds[3]) + (lds[6] + lds[9]);
        b = (lds[1] + lds[4]) + (lds[7] + lds[10]);
        m = fmax(fmax(lds[2], lds[5]), fmax(lds[8], lds[11]));
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// the fused stream + collide step over a work list of tiles
// ---------------------------------------------------------------------------
enum StepMode : int {
    kPlain = 0,   // advance only
    kWriteU = 1,  // advance and store u (FP64, unscaled) of this launch
    kCheck = 2,   // advance, store u, and reduce |u - u_prev|^2, |u|^2, max |f*| per tile
};

struct StepLaunch {
    const SlotDesc* slots;
    const Item* items;
    const int* range;   // device pair {begin, end}: items [begin, end) of the work list
    double* partial;    // 3 doubles per item (check mode)
    int flip;           // launch parity: source buffer = buf[cur ^ flip]
    int rows;           // rows per thread of the tiles (the step kernel takes it as VY)
};

// Blocks are spread over the 8 XCDs round-robin by the hardware; item ranges
// are assigned so that each XCD walks one contiguous slice of the work list
// (neighbouring tiles share cache lines of the shifted rows in one L2).
__device__ __forceinline__ void xcd_slice(const int* range, int& last, int& stride, int& start) {
    const int begin = range[0];
    const int nitems = range[1] - begin;
    const int G = gridDim.x;
    const int nx8 = (G % 8 == 0) ? 8 : 1;
    const int xcd = blockIdx.x % nx8;
    const int lb = blockIdx.x / nx8;
    const int first = begin + (int)(((long long)nitems * xcd) / nx8);
    last = begin + (int)(((long long)nitems * (xcd + 1)) / nx8);
    stride = G / nx8;
    start = first + lb;
}

// LAY: kLayPull (read buf[sel], write buf[sel ^ 1]) or an in-place layout
// (read and write buf[sel]; see Layout).
template <typename S, int MODE, bool GENERAL, int VY, int LAY = kLayPull>
static __global__ __launch_bounds__(kBlock) void k_step(StepLaunch L) {
    using C = typename Store<S>::C;
    __shared__ double lds[12];
    int last, stride, it;
    xcd_slice(L.range, last, stride, it);
    for (; it < last; it += stride) {
        const Item item = L.items[it];
        const SlotDesc& d = L.slots[item.slot];
        const int nx = d.nx, ny = d.ny;
        const long long plane = d.plane;
        const int sel = d.cur ^ L.flip;
        // in place, source and destination are one buffer (no restrict): each
        // location is read and then written by the same site only
        const S* src = reinterpret_cast<const S*>(d.buf[sel]);
        S* dst = reinterpret_cast<S*>(d.buf[LAY == kLayPull ? (sel ^ 1) : sel]);
        const C* __restrict__ g = reinterpret_cast<const C*>(d.g);
        Coef<C> k;
        k.load(d);
        const int bxl = d.bx_log2;
        const int lx = threadIdx.x & ((1 << bxl) - 1);
        const int ly = threadIdx.x >> bxl;
        const int th = kBlock >> bxl;  // tile height in threads
        const int x = (item.tx << bxl) + lx;
        const int y0 = item.ty * th * VY + ly;
        double dsum = 0.0, ssum = 0.0, fmaxv = 0.0;
        C f[VY][8];
        bool ok[VY];
#pragma unroll
        for (int j = 0; j < VY; ++j) {
            const int y = y0 + j * th;
            ok[j] = (x < nx) && (y < ny);
            if (ok[j]) load_state<S>(src, plane, nx, ny, x, y, LAY, f[j]);
        }
#pragma unroll
        for (int j = 0; j < VY; ++j) {
            if (!ok[j]) continue;
            const int y = y0 + j * th;
            const long long s = (long long)y * nx + x;
            const C gx = glob(g)[s] * k.gscale;
            const C gy = glob(g)[plane + s] * k.gscale;
            C ux, uy;
            collide<C, GENERAL>(f[j], gx, gy, k, ux, uy);
            if constexpr (LAY == kLayPull) {
#pragma unroll
                for (int q = 0; q < 8; ++q) Store<S>::st(dst + q * plane + s, f[j][q]);
            } else if constexpr (LAY == kLayNatural) {
#pragma unroll
                for (int q = 0; q < 8; ++q) Store<S>::st(dst + opp(q) * plane + s, f[j][q]);
            } else {
                scatter<S>(dst, plane, nx, ny, x, y, f[j]);
            }
            if constexpr (MODE != kPlain) {
                const double uxd = (double)ux * d.inv_scale, uyd = (double)uy * d.inv_scale;
                if constexpr (MODE == kCheck) {
                    const double dx = uxd - glob(d.u)[s], dy = uyd - glob(d.u)[plane + s];
                    dsum += dx * dx + dy * dy;
                    ssum += uxd * uxd + uyd * uyd;
                    double m = 0.0;
#pragma unroll
                    for (int q = 0; q < 8; ++q) m = fmax(m, (double)fabs(f[j][q]));
                    fmaxv = fmax(fmaxv, m);
                }
                glob(d.u)[s] = uxd;
                glob(d.u)[plane + s] = uyd;
            }
        }
        if constexpr (MODE == kCheck) {
            block_reduce3(dsum, ssum, fmaxv, lds);
            if (threadIdx.x == 0) {
                glob(L.partial)[3 * it + 0] = dsum;
                glob(L.partial)[3 * it + 1] = ssum;
                glob(L.partial)[3 * it + 2] = fmaxv;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// NS fused steps per launch (temporal blocking)
// ---------------------------------------------------------------------------
// A workgroup owns an output tile of 64 x TH sites.  Step 1 advances the tile
// plus a ring of NS-1 sites (periodic coordinates) from the stored field in
// HBM and keeps the post-collision populations in LDS, rounded to the storage
// type exactly as a store to HBM would; each middle step gathers from LDS into
// registers, waits for the whole workgroup, collides and writes back in place
// on a ring one site narrower; the last step advances the tile and writes it
// to HBM.  The result is that of NS single steps, with one HBM read and one
// HBM write of the populations per NS updates.
//
// NT threads per workgroup (256, or 512 for the short FP32 tiles, which
// halves each thread's share of a tile's dependent steps).  Every thread keeps
// the same NM sites of the ring region (site e = thread + a * NT, a < NM) in
// all NS steps, so that step 1 issues all its population
// and force loads before it waits once, the force stays in registers, and the
// later steps touch only LDS until the final store.  Sites past the region
// (e >= RN) load a valid address and store nothing.
constexpr int kTW = 64;  // tile width of the fused kernel (the work list uses 2^6 columns)

// LDS copies of the intermediate populations are held in the storage type.
template <typename S>
__device__ __forceinline__ typename Store<S>::C lds_ld(const S* p) {
    return (typename Store<S>::C)(*p);
}
template <>
__device__ __forceinline__ float lds_ld<__half>(const __half* p) { return __half2float(*p); }
template <typename S>
__device__ __forceinline__ void lds_st(S* p, typename Store<S>::C v) { *p = (S)v; }
template <>
__device__ __forceinline__ void lds_st<__half>(__half* p, float v) { *p = __float2half_rn(v); }

__device__ __forceinline__ int wrap_coord(int v, int n) {
    if (v < 0) v += n;
    if (v < 0) v = ((v % n) + n) % n;
    if (v >= n) {
        v -= n;
        if (v >= n) v %= n;
    }
    return v;
}

// Gather of the 8 populations arriving at LDS position r (row stride RW).
template <typename S, int RW, int RN>
__device__ __forceinline__ void lds_gather(const S* lds, int r, typename Store<S>::C f[8]) {
    f[0] = lds_ld<S>(lds + 0 * RN + r - 1);       // c1 = ( 1, 0)
    f[1] = lds_ld<S>(lds + 1 * RN + r - RW);      // c2 = ( 0, 1)
    f[2] = lds_ld<S>(lds + 2 * RN + r + 1);       // c3 = (-1, 0)
    f[3] = lds_ld<S>(lds + 3 * RN + r + RW);      // c4 = ( 0,-1)
    f[4] = lds_ld<S>(lds + 4 * RN + r - RW - 1);  // c5 = ( 1, 1)
    f[5] = lds_ld<S>(lds + 5 * RN + r - RW + 1);  // c6 = (-1, 1)
    f[6] = lds_ld<S>(lds + 6 * RN + r + RW + 1);  // c7 = (-1,-1)
    f[7] = lds_ld<S>(lds + 7 * RN + r + RW - 1);  // c8 = ( 1,-1)
}

// Step 1 of the fused kernel for one tile: gathers the ring region from the
// stored field (periodic coordinates), collides, and writes the post-collision
// populations to LDS; returns the scaled force of the thread's sites.  Every
// slot loads (the last slot's spare lanes re-read the region's last site), so
// all loads are issued before the first use.
template <typename S, int TH, int NS, int NT = kBlock>
__device__ __forceinline__ void stepN_first(const S* __restrict__ src,
                                            const typename Store<S>::C* __restrict__ g,
                                            long long plane, int nx, int ny, int x0, int y0,
                                            const Coef<typename Store<S>::C>& k, S* lds,
                                            typename Store<S>::C gx[], typename Store<S>::C gy[]) {
    using C = typename Store<S>::C;
    constexpr int R = NS - 1;
    constexpr int RW = kTW + 2 * R, RH = TH + 2 * R, RN = RW * RH;
    constexpr int NM = (RN + NT - 1) / NT;
    C f[NM][8];
#pragma unroll
    for (int a = 0; a < NM; ++a) {
        const int e = min((int)threadIdx.x + a * NT, RN - 1);
        const int i = e % RW, j = e / RW;
        const int xw = wrap_coord(x0 - R + i, nx), yw = wrap_coord(y0 - R + j, ny);
        gather<S>(src, plane, nx, ny, xw, yw, f[a]);
        const long long sidx = (long long)yw * nx + xw;
        gx[a] = glob(g)[sidx];
        gy[a] = glob(g)[plane + sidx];
    }
#pragma unroll
    for (int a = 0; a < NM; ++a) {
        const int e = (int)threadIdx.x + a * NT;
        gx[a] *= k.gscale;
        gy[a] *= k.gscale;
        C ux, uy;
        collide<C, false>(f[a], gx[a], gy[a], k, ux, uy);
        if (e < RN) {
#pragma unroll
            for (int q = 0; q < 8; ++q) lds_st<S>(lds + q * RN + e, f[a][q]);
        }
    }
}

template <typename S, int TH, int NS, int NT = kBlock>
static __global__ __launch_bounds__(NT) void k_stepN(StepLaunch L) {
    using C = typename Store<S>::C;
    constexpr int R = NS - 1;  // ring width of the first step
    constexpr int RW = kTW + 2 * R, RH = TH + 2 * R, RN = RW * RH;
    constexpr int NM = (RN + NT - 1) / NT;  // ring sites per thread
    __shared__ S lds[8 * RN];
    int last, stride, it;
    xcd_slice(L.range, last, stride, it);
    for (; it < last; it += stride) {
        const Item item = L.items[it];
        const SlotDesc& d = L.slots[item.slot];
        const int nx = d.nx, ny = d.ny;
        const long long plane = d.plane;
        const int sel = d.cur ^ L.flip;
        const S* __restrict__ src = reinterpret_cast<const S*>(d.buf[sel]);
        S* __restrict__ dst = reinterpret_cast<S*>(d.buf[sel ^ 1]);
        const C* __restrict__ g = reinterpret_cast<const C*>(d.g);
        Coef<C> k;
        k.load(d);
        const int x0 = item.tx * kTW, y0 = item.ty * TH;
        C f[NM][8], gx[NM], gy[NM];
        // step 1: tile + ring R, HBM -> LDS
        stepN_first<S, TH, NS, NT>(src, g, plane, nx, ny, x0, y0, k, lds, gx, gy);
        __syncthreads();
        // middle steps: ring R - m, LDS -> registers -> LDS (in place)
#pragma unroll
        for (int m = 1; m < R; ++m) {
#pragma unroll
            for (int a = 0; a < NM; ++a) {
                const int e = (int)threadIdx.x + a * NT;
                const int i = e % RW, j = e / RW;
                if (e < RN && i >= m && i < RW - m && j >= m && j < RH - m)
                    lds_gather<S, RW, RN>(lds, e, f[a]);
            }
            __syncthreads();
#pragma unroll
            for (int a = 0; a < NM; ++a) {
                const int e = (int)threadIdx.x + a * NT;
                const int i = e % RW, j = e / RW;
                if (e < RN && i >= m && i < RW - m && j >= m && j < RH - m) {
                    C ux, uy;
                    collide<C, false>(f[a], gx[a], gy[a], k, ux, uy);
#pragma unroll
                    for (int q = 0; q < 8; ++q) lds_st<S>(lds + q * RN + e, f[a][q]);
                }
            }
            __syncthreads();
        }
        // last step: the tile, LDS -> HBM
#pragma unroll
        for (int a = 0; a < NM; ++a) {
            const int e = (int)threadIdx.x + a * NT;
            const int i = e % RW, j = e / RW;
            const int x = x0 + i - R, y = y0 + j - R;
            if (e < RN && i >= R && i < R + kTW && j >= R && j < R + TH && x < nx && y < ny) {
                lds_gather<S, RW, RN>(lds, e, f[a]);
                C ux, uy;
                collide<C, false>(f[a], gx[a], gy[a], k, ux, uy);
                const long long sidx = (long long)y * nx + x;
#pragma unroll
                for (int q = 0; q < 8; ++q) Store<S>::st(dst + q * plane + sidx, f[a][q]);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// NS fused steps per launch, register wavefront
// ---------------------------------------------------------------------------
// One wave owns a strip of 64 V columns (V adjacent columns per lane): W
// output columns plus R ring columns per side, and marches up a segment of
// rows.  At row t it loads the stored field's row t (level 0) and advances
// level k = 1..NS at row t - k from level k-1's rows t-k-1, t-k, t-k+1, which
// it keeps in registers: the y neighbours are earlier rows of the same lane,
// the x neighbours are the lane's other column or, across lanes, come through
// a whole-wave DPP shift.  Level NS is stored.  Each level loses one valid
// column per side, so after NS <= R levels the W middle columns hold the
// output.  No LDS and no barrier; every intermediate level is rounded to the
// storage type exactly as a store would round it, so the result equals NS
// single steps bit for bit.  V = 2 (FP32, FP16) needs an even nx, so that a
// lane's column pair stays adjacent across the periodic wrap; its ring is 4
// columns for every NS so that pairs stay aligned.
__device__ __forceinline__ float lane_from_left(float v) {  // lane l <- lane l-1
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane_from_right(float v) {  // lane l <- lane l+1
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double lane_from_left(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_from_right(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// value as the storage type would hold it
template <typename S>
__device__ __forceinline__ typename Store<S>::C as_stored(typename Store<S>::C v) { return v; }
template <>
__device__ __forceinline__ float as_stored<__half>(float v) { return __half2float(__float2half_rn(v)); }

// V consecutive storage elements as arithmetic values (one vector access).
template <typename S, int V> struct VecIO;
template <typename S> struct VecIO<S, 1> {
    using C = typename Store<S>::C;
    __device__ static __forceinline__ void ld(const S* p, C o[1]) { o[0] = Store<S>::ld(p); }
    __device__ static __forceinline__ void st(S* p, const C v[1]) { Store<S>::st(p, v[0]); }
};
typedef float wf2 __attribute__((ext_vector_type(2)));
template <> struct VecIO<float, 2> {
    __device__ static __forceinline__ void ld(const float* p, float o[2]) {
        const wf2 v = __builtin_nontemporal_load(glob(reinterpret_cast<const wf2*>(p)));
        o[0] = v.x;
        o[1] = v.y;
    }
    __device__ static __forceinline__ void st(float* p, const float v[2]) {
        wf2 w;
        w.x = v[0];
        w.y = v[1];
        __builtin_nontemporal_store(w, glob(reinterpret_cast<wf2*>(p)));
    }
};
template <> struct VecIO<__half, 2> {
    __device__ static __forceinline__ void ld(const __half* p, float o[2]) {
        const unsigned u = __builtin_nontemporal_load(glob(reinterpret_cast<const unsigned*>(p)));
        o[0] = __half2float(__ushort_as_half((unsigned short)(u & 0xffffu)));
        o[1] = __half2float(__ushort_as_half((unsigned short)(u >> 16)));
    }
    __device__ static __forceinline__ void st(__half* p, const float v[2]) {
        const unsigned u = (unsigned)__half_as_ushort(__float2half_rn(v[0])) |
                           ((unsigned)__half_as_ushort(__float2half_rn(v[1])) << 16);
        __builtin_nontemporal_store(u, glob(reinterpret_cast<unsigned*>(p)));
    }
};

template <int NS, int V>
__host__ __device__ constexpr int wave_ring() { return V == 1 ? NS : 4; }
template <int NS, int V>
__host__ __device__ constexpr int wave_width() { return kWave * V - 2 * wave_ring<NS, V>(); }

struct WaveLaunch {
    const SlotDesc* slots;
    int flip;
    int strips, segs, hs;  // strips of W output columns, segments of hs rows
};

template <typename S, int NS, int V>
static __global__ __launch_bounds__(kBlock) void k_wave(WaveLaunch L) {
    using C = typename Store<S>::C;
    constexpr int R = wave_ring<NS, V>();
    constexpr int W = wave_width<NS, V>();
    constexpr int PF = 3;  // rows loaded ahead
    // wave index as a scalar: the row loop and the row bases stay scalar
    const int wid = __builtin_amdgcn_readfirstlane((int)blockIdx.x * (kBlock / kWave) +
                                                   (int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & (kWave - 1));
    if (wid >= L.strips * L.segs) return;  // whole waves leave; no barrier follows
    const SlotDesc& d = L.slots[0];
    const int nx = d.nx, ny = d.ny;
    const long long plane = d.plane;
    const int sel = d.cur ^ L.flip;
    const S* __restrict__ src = reinterpret_cast<const S*>(d.buf[sel]);
    S* __restrict__ dst = reinterpret_cast<S*>(d.buf[sel ^ 1]);
    const C* __restrict__ g = reinterpret_cast<const C*>(d.g);
    Coef<C> k;
    k.load(d);
    const int sx = wid % L.strips, sy = wid / L.strips;
    const int xs = sx * W, ya = sy * L.hs, yb = min(ya + L.hs, ny);
    const int x = xs - R + V * lane;  // first column of this lane
    const int xw = wrap_coord(x, nx);
    const bool out_lane = lane >= R / V && lane < (R + W) / V && x < nx;
    // loads of row t: scalar row base + per-lane byte offset of the column
    const unsigned xs_b = (unsigned)xw * (unsigned)sizeof(S), xg_b = (unsigned)xw * (unsigned)sizeof(C);
    auto load_row = [&](int t, C (*a)[V], C (*gg)[V]) {
        const long long r = (long long)wrap_coord(t, ny) * nx;
#pragma unroll
        for (int q = 0; q < 8; ++q)
            VecIO<S, V>::ld(reinterpret_cast<const S*>(
                                reinterpret_cast<const char*>(src + (q * plane + r)) + xs_b),
                            a[q]);
        VecIO<C, V>::ld(reinterpret_cast<const C*>(reinterpret_cast<const char*>(g + r) + xg_b), gg[0]);
        VecIO<C, V>::ld(reinterpret_cast<const C*>(reinterpret_cast<const char*>(g + (plane + r)) + xg_b),
                        gg[1]);
    };
    C A0[6][8][V];      // level 0 rows by iteration mod 6 (three back, three ahead)
    C Gp[6][2][V];      // force rows, same slots
    C A[NS][3][8][V];   // levels 1..NS-1 (index 0 unused), rows mod 3
    C G[NS + 1][2][V];  // force of rows t, t-1, ..., t-NS
#pragma unroll
    for (int j = 0; j <= NS; ++j)
#pragma unroll
        for (int c = 0; c < V; ++c) G[j][0][c] = G[j][1][c] = C(0);
#pragma unroll
    for (int r = 0; r < 6; ++r)
#pragma unroll
        for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int c = 0; c < V; ++c) A0[r][q][c] = C(0);
#pragma unroll
    for (int lv = 0; lv < NS; ++lv)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int c = 0; c < V; ++c) A[lv][r][q][c] = C(0);
    const int t_first = ya - NS;
#pragma unroll
    for (int u = 0; u < PF; ++u) load_row(t_first + u, A0[u], Gp[u]);
    for (int t0 = t_first; t0 < yb + NS; t0 += 6) {
#pragma unroll
        for (int u = 0; u < 6; ++u) {
            const int t = t0 + u;
            load_row(t + PF, A0[(u + PF) % 6], Gp[(u + PF) % 6]);
#pragma unroll
            for (int j = NS; j > 0; --j)
#pragma unroll
                for (int c = 0; c < V; ++c) {
                    G[j][0][c] = G[j - 1][0][c];
                    G[j][1][c] = G[j - 1][1][c];
                }
#pragma unroll
            for (int c = 0; c < V; ++c) {
                G[0][0][c] = Gp[u][0][c] * k.gscale;
                G[0][1][c] = Gp[u][1][c] * k.gscale;
            }
#pragma unroll
            for (int lv = 1; lv <= NS; ++lv) {
                // level lv-1 rows t-lv+1 (this iteration), t-lv, t-lv-1
                const C(*R0)[V] = lv == 1 ? A0[u] : A[lv - 1][u % 3];
                const C(*R1)[V] = lv == 1 ? A0[(u + 5) % 6] : A[lv - 1][(u + 2) % 3];
                const C(*R2)[V] = lv == 1 ? A0[(u + 4) % 6] : A[lv - 1][(u + 1) % 3];
                // value of population q at column c - 1 / c + 1 of a row
                auto left = [&](const C(*row)[V], int q, int c) {
                    return c > 0 ? row[q][c - 1] : lane_from_left(row[q][V - 1]);
                };
                auto right = [&](const C(*row)[V], int q, int c) {
                    return c < V - 1 ? row[q][c + 1] : lane_from_right(row[q][0]);
                };
                C f[V][8];
#pragma unroll
                for (int c = 0; c < V; ++c) {
                    f[c][0] = left(R1, 0, c);   // c1 = ( 1, 0) from (x-1, y)
                    f[c][1] = R2[1][c];         // c2 = ( 0, 1) from (x, y-1)
                    f[c][2] = right(R1, 2, c);  // c3 = (-1, 0) from (x+1, y)
                    f[c][3] = R0[3][c];         // c4 = ( 0,-1) from (x, y+1)
                    f[c][4] = left(R2, 4, c);   // c5 = ( 1, 1) from (x-1, y-1)
                    f[c][5] = right(R2, 5, c);  // c6 = (-1, 1) from (x+1, y-1)
                    f[c][6] = right(R0, 6, c);  // c7 = (-1,-1) from (x+1, y+1)
                    f[c][7] = left(R0, 7, c);   // c8 = ( 1,-1) from (x-1, y+1)
                }
#pragma unroll
                for (int c = 0; c < V; ++c) {
                    C ux, uy;
                    collide<C, false>(f[c], G[lv][0][c], G[lv][1][c], k, ux, uy);
                }
                if (lv < NS) {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
#pragma unroll
                        for (int c = 0; c < V; ++c) A[lv][u % 3][q][c] = as_stored<S>(f[c][q]);
                } else {
                    const int y = t - NS;
                    if (out_lane && y >= ya && y < yb) {
                        const long long o = (long long)y * nx + x;
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            C v[V];
#pragma unroll
                            for (int c = 0; c < V; ++c) v[c] = f[c][q];
                            VecIO<S, V>::st(dst + q * plane + o, v);
                        }
                    }
                }
            }
        }
    }
}

// Streaming alone (no collision): bit-exact check of the index arithmetic,
// in any layout (in place, an even and an odd step together stream twice).
template <typename S, int LAY = kLayPull>
static __global__ __launch_bounds__(kBlock) void k_stream_only(StepLaunch L) {
    using C = typename Store<S>::C;
    int last, stride, it;
    xcd_slice(L.range, last, stride, it);
    for (; it < last; it += stride) {
        const Item item = L.items[it];
        const SlotDesc& d = L.slots[item.slot];
        const int sel = d.cur ^ L.flip;
        const S* src = reinterpret_cast<const S*>(d.buf[sel]);
        S* dst = reinterpret_cast<S*>(d.buf[LAY == kLayPull ? (sel ^ 1) : sel]);
        const int bxl = d.bx_log2;
        const int th = kBlock >> bxl;
        const int x = (item.tx << bxl) + (threadIdx.x & ((1 << bxl) - 1));
        for (int j = 0; j < L.rows; ++j) {
            const int y = item.ty * th * L.rows + (threadIdx.x >> bxl) + j * th;
            if (x >= d.nx || y >= d.ny) continue;
            C f[8];
            load_state<S>(src, d.plane, d.nx, d.ny, x, y, LAY, f);
            const long long s = (long long)y * d.nx + x;
            if (LAY == kLayPull)
                for (int q = 0; q < 8; ++q) Store<S>::st(dst + q * d.plane + s, f[q]);
            else if (LAY == kLayNatural)
                for (int q = 0; q < 8; ++q) Store<S>::st(dst + opp(q) * d.plane + s, f[q]);
            else
                scatter<S>(dst, d.plane, d.nx, d.ny, x, y, f);
        }
    }
}

// Residual check without a step (in-place streaming, which cannot step back
// after the check): u(n) from the stored field in layout LAY; per tile the
// FP64 partials sum |u(n) - u_prev|^2, sum |u(n)|^2 and max |f|; u(n) is
// stored as the next u_prev.
template <typename S, int LAY, int VY>
static __global__ __launch_bounds__(kBlock) void k_check_state(StepLaunch L) {
    using C = typename Store<S>::C;
    __shared__ double lds[12];
    int last, stride, it;
    xcd_slice(L.range, last, stride, it);
    for (; it < last; it += stride) {
        const Item item = L.items[it];
        const SlotDesc& d = L.slots[item.slot];
        const int nx = d.nx, ny = d.ny;
        const long long plane = d.plane;
        const S* src = reinterpret_cast<const S*>(d.buf[d.cur ^ L.flip]);
        const C* g = reinterpret_cast<const C*>(d.g);
        Coef<C> k;
        k.load(d);
        const int bxl = d.bx_log2;
        const int th = kBlock >> bxl;
        const int x = (item.tx << bxl) + (threadIdx.x & ((1 << bxl) - 1));
        double dsum = 0.0, ssum = 0.0, fmaxv = 0.0;
#pragma unroll
        for (int j = 0; j < VY; ++j) {
            const int y = item.ty * th * VY + (threadIdx.x >> bxl) + j * th;
            if (x >= nx || y >= ny) continue;
            C f[8];
            load_state<S>(src, plane, nx, ny, x, y, LAY, f);
            const long long s = (long long)y * nx + x;
            // u exactly as the collision forms it (same type and operations)
            C ux, uy;
            bared_u<C>(f, glob(g)[s] * k.gscale, glob(g)[plane + s] * k.gscale, ux, uy);
            const double uxd = (double)ux * d.inv_scale, uyd = (double)uy * d.inv_scale;
            const double dx = uxd - glob(d.u)[s], dy = uyd - glob(d.u)[plane + s];
            dsum += dx * dx + dy * dy;
            ssum += uxd * uxd + uyd * uyd;
            double m = 0.0;
#pragma unroll
            for (int q = 0; q < 8; ++q) m = fmax(m, (double)fabs(f[q]));
            fmaxv = fmax(fmaxv, m);
            glob(d.u)[s] = uxd;
            glob(d.u)[plane + s] = uyd;
        }
        block_reduce3(dsum, ssum, fmaxv, lds);
        if (threadIdx.x == 0) {
            glob(L.partial)[3 * it + 0] = dsum;
            glob(L.partial)[3 * it + 1] = ssum;
            glob(L.partial)[3 * it + 2] = fmaxv;
        }
    }
}

// Per-slot deterministic sum of the tile partials: one block per slot,
// items of a slot are contiguous in the work list.
struct FinalizeLaunch {
    const int* first;   // per slot: first item
    const int* count;   // per slot: number of items (0 = inactive)
    const double* partial;
    double* result;     // 4 doubles per slot: sum d, sum s, max |f|, unused
    int nslots;
};

static __global__ __launch_bounds__(kBlock) void k_finalize(FinalizeLaunch F) {
    __shared__ double lds[12];
    const int slot = blockIdx.x;
    if (slot >= F.nslots) return;
    const int cnt = F.count[slot];
    if (cnt == 0) return;
    const int f0 = F.first[slot];
    double a = 0.0, b = 0.0, m = 0.0;
    for (int i = threadIdx.x; i < cnt; i += kBlock) {
        a += F.partial[3 * (f0 + i) + 0];
        b += F.partial[3 * (f0 + i) + 1];
        m = fmax(m, F.partial[3 * (f0 + i) + 2]);
    }
    block_reduce3(a, b, m, lds);
    if (threadIdx.x == 0) {
        F.result[4 * slot + 0] = a;
        F.result[4 * slot + 1] = b;
        F.result[4 * slot + 2] = m;
        F.result[4 * slot + 3] = 0.0;
    }
}

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

// Write the work list of one lattice: tiles in row-major tile order.
static __global__ __launch_bounds__(kBlock) void k_build_items(Item* items, int first, int slot,
                                                        int tiles_x, int count) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= count) return;
    Item it;
    it.slot = slot;
    it.tx = i % tiles_x;
    it.ty = i / tiles_x;
    it.pad_ = 0;
    items[first + i] = it;
}

// Small device-side stores (stream-ordered, safe inside captured graphs).
static __global__ void k_set_int(int* p, int v) { *p = v; }
static __global__ void k_set_desc(SlotDesc* p, SlotDesc v) { *p = v; }

// Neutral modes.  (1) The mean first moments: collision adds g to m10, m01 and
// streaming permutes, so sum_x m10(f(n)) = sum_x m10(f(0)) + n sum_x gx exactly
// (eigenvalue 1 at k = 0).  (2) The staggered first moments: for even nx,
// J = sum_x (-1)^x m10(f(n)) obeys J(n+1) = -J(n) - sum_x (-1)^x gx for any
// relaxation rates (streaming with c_x = +-1 flips (-1)^x), and likewise in y
// with m01, gy: eigenvalue -1 at k = (pi, 0), (0, pi).  Neither mode is ever
// damped, so rounding noise from narrow storage stays in them for good.  These
// kernels measure both on the stored (post-collision) field S, whose sums
// equal those of f(n) for the mean and J_S = J_f + G (fixed point G/2) for the
// staggered mode, and reset them.
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

// Stage 2: S1 += (ex (-1)^x + mx), S3 -= (ex (-1)^x + mx),
//          S2 += (ey (-1)^y + my), S4 -= (ey (-1)^y + my)
// (changes only m10 / m01 of S: the staggered and the uniform parts; all
// amounts already in storage units).
template <typename S>
static __global__ __launch_bounds__(kBlock) void k_neutral_fix(SlotDesc d, int sel, double ex,
                                                               double ey, double mx, double my) {
    using C = typename Store<S>::C;
    const long long s = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (s >= (long long)d.nx * d.ny) return;
    const int x = (int)(s % d.nx), y = (int)(s / d.nx);
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
