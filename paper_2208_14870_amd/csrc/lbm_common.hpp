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
    int sr;                // nonzero: half storage rounds stochastically (two buffers only)
    unsigned sr_seed;      // seed of the stochastic rounding
    unsigned sr_step;      // steps done before the next launch (advanced on the device)
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
    __device__ static __forceinline__ void st_h(__half* p, __half h) {
        __builtin_nontemporal_store(__half_as_ushort(h), glob(reinterpret_cast<unsigned short*>(p)));
    }
};

// ---------------------------------------------------------------------------
// stochastic rounding of half storage (optional, lbm_set_stochastic_rounding)
// ---------------------------------------------------------------------------
// Round-to-nearest half storage loses every change of a population smaller
// than half a unit in the last place, so slow modes stall.  Stochastic
// rounding rounds up with probability equal to the discarded fraction, so the
// stored value is unbiased.  The random bits are a fixed function of (site,
// population, step, seed), so the single-step and the fused kernels, which
// store the same value for the same (site, q, step), round it identically, and
// reruns repeat.  Per site and step: the 32-bit finaliser of MurmurHash3
// (Appleby) of the site index mixed with a hash of the step gives one word;
// three xorshift32 steps (Marsaglia 2003) give three more; population q takes
// 13 bits of word q/2.  Rounding: the 13 random bits are added to the low 13
// bits of the FP32 pattern (the bits that FP32 -> FP16 drops for normal half
// values), which are then cleared, so the conversion to half is exact.  Values
// below the half normal range (|v| < 2^-14, far below the stored scale) are
// rounded to nearest by that conversion; canonical NaN and infinity pass
// unchanged.
__host__ __device__ __forceinline__ unsigned sr_fmix(unsigned h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
__host__ __device__ __forceinline__ unsigned sr_xorshift(unsigned x) {
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}
// hash of a step, wave-uniform
__host__ __device__ __forceinline__ unsigned sr_step_hash(unsigned step, unsigned seed) {
    return sr_fmix(step * 0x9e3779b9u ^ seed);
}
struct SrBits {
    unsigned w[4];
    __device__ __forceinline__ void make(unsigned site, unsigned step_hash) {
        w[0] = sr_fmix(site ^ step_hash);
        w[1] = sr_xorshift(w[0] | 1u);
        w[2] = sr_xorshift(w[1]);
        w[3] = sr_xorshift(w[2]);
    }
    __device__ __forceinline__ unsigned r13(int q) const {
        return (q & 1) ? (w[q >> 1] >> 13) & 0x1fffu : w[q >> 1] & 0x1fffu;
    }
};
__device__ __forceinline__ __half half_sr(float v, unsigned r13) {
    const unsigned b = (__float_as_uint(v) + r13) & 0xffffe000u;
    return __float2half_rn(__uint_as_float(b));
}

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

// The collision with the force given as its half and quarter (hgx = gx/2,
// qgx = hgx/2, formed by the caller with exactly these two products, so that
// kernels that keep them per site across steps round as collide() does).
template <typename C, bool GENERAL>
__device__ __forceinline__ void collide_h(C f[8], C hgx, C hgy, C qgx, C qgy, const Coef<C>& k,
                                          C& ux, C& uy) {
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
    const C ms = fmac(C(2), sac + sbd, h13 + h24);  // (h13 + h24) + 2 (sac + sbd): 2x is exact
    const C md = h13 - h24;
    ux = m10 + hgx;
    uy = m01 + hgy;
    if constexpr (!GENERAL) {
        const C dd = k.cd * md;
        const C a = fmac(k.cs, ms, dd);
        const C b = fmac(k.cs, ms, -dd);
        const C ex = fmac(k.hth, ux, qgx);
        const C ey = fmac(k.hth, uy, qgy);
        const C s = k.c11 * m11;
        const C t1 = k.tq * (ux + uy);
        const C t2 = k.tq * (ux - uy);
        f[0] = a + ex;
        f[2] = a - ex;
        f[1] = b + ey;
        f[3] = b - ey;
        f[4] = s + t1;
        f[6] = s - t1;
        f[5] = (-s) - t2;  // -(s + t2) in one instruction (round-to-nearest is odd)
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

template <typename C, bool GENERAL>
__device__ __forceinline__ void collide(C f[8], C gx, C gy, const Coef<C>& k, C& ux, C& uy) {
#pragma clang fp contract(off)
    const C hgx = C(0.5) * gx, hgy = C(0.5) * gy;
    collide_h<C, GENERAL>(f, hgx, hgy, C(0.5) * hgx, C(0.5) * hgy, k, ux, uy);
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

// v modulo n in 0..n-1 (periodic coordinates; any v)
__device__ __forceinline__ int wrap_coord(int v, int n) {
    if (v < 0) v += n;
    if (v < 0) v = ((v % n) + n) % n;
    if (v >= n) {
        v -= n;
        if (v >= n) v %= n;
    }
    return v;
}

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

// ---------------------------------------------------------------------------
// host/device policies shared by every solve path
// ---------------------------------------------------------------------------

// Mean projection of a body force.  The mean of u is conserved by the scheme
// (collision adds g to the first moments, streaming permutes), so a steady
// state needs a zero-mean load (Sec. 7.2).  From the FP64 sums
// st = {sum gx, sum gy, sum gx^2 + gy^2} over n sites, a component's mean is
// removed when it exceeds 1e-12 times the rms of the force; a smaller mean is
// at the level of the sum's own rounding and the force is taken as given.
// Host and device evaluate this with the same correctly rounded operations, so
// they take the same decision.
__host__ __device__ inline void force_mean_shift(const double* st, double n, double shift[2]) {
#pragma clang fp contract(off)
    const double ms = st[2] / (2.0 * n);  // mean square of the components
    for (int c = 0; c < 2; ++c) {
        const double m = st[c] / n;
        shift[c] = (m * m > 1e-24 * ms) ? m : 0.0;
    }
}

// Divergence guard of the pseudo-time iteration, fed at every check with the
// update norm d = ||u(n) - u(n-1)||_2 (the residual's numerator).  With a
// material outside the stability region of Sec. 5 the unstable modes grow
// geometrically, and so does d, without end (the ratio r = d / ||u|| rises
// too, but saturates once they dominate u); d grows by decades long before
// any value overflows.  In a stable solve d decays.  The guard fires when d
// rose at each of at least M consecutive checks and is at least twice the
// largest d of the kWindow checks before that run of rises.  A decaying
// oscillation (a complex pair of eigenvalues) also makes d climb from its dips
// for several checks, but not above its earlier peaks; the factor keeps
// rounding noise at a precision floor from firing it.
struct RiseGuard {
    static constexpr int kWindow = 32;
    double hist[kWindow];  // the last update norms, a ring
    double prev;           // d of the previous check (NaN: none)
    double base;           // the largest d of the window before the current run
    int run;               // checks in a row whose d rose
    int count, pos;        // values in the ring, next slot
    int pad_;
    __host__ __device__ void clear() {
        prev = __builtin_nan("");
        base = __builtin_nan("");
        run = count = pos = pad_ = 0;
    }
    __host__ __device__ bool update(double d, int M) {
        if (d > prev) {
            if (run == 0) {
                base = hist[0];
                for (int h = 1; h < count; ++h)
                    if (hist[h] > base) base = hist[h];
            }
            ++run;
        } else {
            run = 0;
        }
        hist[pos] = d;
        pos = (pos + 1) % kWindow;
        if (count < kWindow) ++count;
        prev = d;
        return M > 0 && run >= M && d >= 2.0 * base;
    }
};

// Blocks are spread over the 8 XCDs round-robin by the hardware; item ranges
// are assigned so that each XCD walks one contiguous slice of the work list
// (neighbouring tiles share cache lines of the shifted rows in one L2).
__device__ __forceinline__ void xcd_slice(const int* range, int& last, int& stride, int& start) {
    const int begin = range[0];
    const int nitems = range[1] - begin;
    const int G = gridDim.x;
    // 8 slices when the grid is a multiple of 8, else one; the quotients by
    // 8 or 1 as shifts of non-negative values
    const int sh = (G % 8 == 0) ? 3 : 0;
    const int xcd = (int)blockIdx.x & ((1 << sh) - 1);
    const int lb = (int)blockIdx.x >> sh;
    const int first = begin + (int)(((long long)nitems * xcd) >> sh);
    last = begin + (int)(((long long)nitems * (xcd + 1)) >> sh);
    stride = G >> sh;
    start = first + lb;
}

}  // namespace lbm
