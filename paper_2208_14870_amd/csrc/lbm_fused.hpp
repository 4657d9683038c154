// Temporal blocking: several steps per launch through an LDS tile or a
// register wavefront, bit-identical to single steps.
#pragma once

#include <type_traits>

#include "lbm_common.hpp"

namespace lbm {

// ---------------------------------------------------------------------------
// NS fused steps per launch (temporal blocking)
// ---------------------------------------------------------------------------
// A workgroup owns an output tile of 64 x TH sites.  Step 1 advances the tile
// plus a ring of NS-1 sites (periodic coordinates) from the stored field in
// HBM and keeps the post-collision populations in LDS, rounded to the storage
// type exactly as a store to HBM would; each middle step advances a ring one
// site narrower from LDS back into LDS; the last step advances the tile and
// writes it to HBM.  The result is that of NS single steps, with one HBM read
// and one HBM write of the populations per NS updates.
//
// The LDS copy alternates between two layouts, as in-place streaming does in
// HBM, so that within a step every LDS location a site writes is read in that
// step by the same site only, and one barrier per step suffices.  Swapped:
// plane opp(q) at r holds f*_q(r), the populations leaving r; step 1 and the
// other odd steps write it at their own site.  Natural: plane q at r holds
// f_q(r), the populations arriving at r; even steps read the swapped copy of
// their upstream neighbours and push into it at the downstream neighbours.
//
// NT threads per workgroup: 256, or 512 for the 8-row FP32 tiles and the
// 16-row FP32 / FP16 tiles of deeper blocking (each thread then carries fewer
// sites of the ring region, in fewer registers).  Every thread keeps
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

// LDS offset of the neighbour r + c_q (row stride RW; q in the order of the
// velocity table, 0-based).
template <int RW>
__device__ __forceinline__ constexpr int lds_shift(int q) {
    return ((q == 0 || q == 4 || q == 7) ? 1 : (q == 2 || q == 5 || q == 6) ? -1 : 0) +
           RW * ((q == 1 || q == 4 || q == 5) ? 1 : (q == 3 || q == 6 || q == 7) ? -1 : 0);
}

// The 8 populations arriving at LDS position r, from the swapped layout (the
// upstream neighbours' post-collision values) or the natural one (own site).
template <typename S, int RW, int RN>
__device__ __forceinline__ void lds_read(const S* lds, int r, bool swapped,
                                         typename Store<S>::C f[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q)
        f[q] = swapped ? lds_ld<S>(lds + opp(q) * RN + r - lds_shift<RW>(q))
                       : lds_ld<S>(lds + q * RN + r);
}

// The post-collision populations of LDS position r: to its own site in the
// swapped layout, or pushed to the downstream neighbours in the natural one.
template <typename S, int RW, int RN>
__device__ __forceinline__ void lds_write(S* lds, int r, bool swapped,
                                          const typename Store<S>::C f[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        if (swapped) lds_st<S>(lds + opp(q) * RN + r, f[q]);
        else lds_st<S>(lds + q * RN + r + lds_shift<RW>(q), f[q]);
    }
}

// lds_write for half storage with stochastic rounding (bits of the writing
// site for this step).
template <int RW, int RN>
__device__ __forceinline__ void lds_write_sr(__half* lds, int r, bool swapped, const float f[8],
                                             const SrBits& b) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const __half h = half_sr(f[q], b.r13(q));
        if (swapped) lds[opp(q) * RN + r] = h;
        else lds[q * RN + r + lds_shift<RW>(q)] = h;
    }
}

// Element i of a plane through a 32-bit byte offset (planes of the tile kernel
// hold fewer than 2^32 bytes): with a wave-uniform base each access is one
// scalar base plus one 32-bit vector offset, instead of 64-bit address
// arithmetic per load.
template <typename S>
__device__ __forceinline__ const S* at_u32(const S* base, unsigned i) {
    return reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(S));
}
template <typename S>
__device__ __forceinline__ S* at_u32(S* base, unsigned i) {
    return reinterpret_cast<S*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(S));
}

// The slots of a thread in the region of the fused kernel, fixed for the whole
// launch: slot a is region site e = threadIdx.x + a NT, at column i and row j of
// the region, and lvl = min(i, RW-1-i, j, RH-1-j) is its distance to the
// region's edge.  Step s (1-based) advances the region shrunk by s-1 sites on
// every side, i.e. the slots with lvl >= s-1, and the last step's tile is
// lvl >= R.  Spare slots (e >= RN) have lvl = -1 and the coordinates of the
// region's last site (a valid address).  Computed once per launch, so that no
// step divides or compares coordinates again, and packed into one register per
// slot (i in bits 0-7, j in bits 8-15, lvl + 1 from bit 16), so that "lvl >= m"
// is one unsigned compare against a constant.
template <int TH, int NS, int NT>
struct SlotGeo {
    static constexpr int R = NS - 1;
    static constexpr int RW = kTW + 2 * R, RH = TH + 2 * R, RN = RW * RH;
    static constexpr int NM = (RN + NT - 1) / NT;
    static_assert(RW < 256 && RH < 256, "region coordinates must fit 8 bits");
    unsigned p[NM];
    __device__ __forceinline__ void init() {
#pragma unroll
        for (int a = 0; a < NM; ++a) {
            const int e0 = (int)threadIdx.x + a * NT;
            const int e = min(e0, RN - 1);
            const int ii = e % RW, jj = e / RW;
            const int lv = e0 < RN ? min(min(ii, RW - 1 - ii), min(jj, RH - 1 - jj)) : -1;
            p[a] = (unsigned)ii | ((unsigned)jj << 8) | ((unsigned)(lv + 1) << 16);
        }
    }
    __device__ __forceinline__ int i(int a) const { return (int)(p[a] & 0xffu); }
    __device__ __forceinline__ int j(int a) const { return (int)((p[a] >> 8) & 0xffu); }
    // lvl >= m (m >= 0)
    __device__ __forceinline__ bool active(int a, int m) const {
        return p[a] >= ((unsigned)(m + 1) << 16);
    }
};

// Step 1 of the fused kernel for one tile, in two parts.  stepN_load issues
// the loads of the ring region from the stored field (periodic coordinates):
// the 8 incoming populations and the force of every slot, so that all loads
// are in flight before the first use.  A tile whose region and its pull halo
// lie inside the lattice (almost every tile of a large lattice) forms its
// addresses without the periodic wrap; the others wrap every coordinate.
// stepN_collide1 scales the force, collides and writes the post-collision
// populations to LDS.
template <typename S, int TH, int NS, int NT = kBlock, bool SR = false>
__device__ __forceinline__ void stepN_load(const S* __restrict__ src,
                                           const typename Store<S>::C* __restrict__ g,
                                           long long plane, int nx, int ny, int x0, int y0,
                                           const SlotGeo<TH, NS, NT>& geo,
                                           typename Store<S>::C f[][8],
                                           typename Store<S>::C gx[], typename Store<S>::C gy[],
                                           unsigned sid[]) {
    using Geo = SlotGeo<TH, NS, NT>;
    constexpr int R = Geo::R, NM = Geo::NM;
    using C = typename Store<S>::C;
    const S* pq[8];  // wave-uniform plane bases
#pragma unroll
    for (int q = 0; q < 8; ++q) pq[q] = src + q * plane;
    const C* g1 = g + plane;
    const unsigned w = (unsigned)nx;
    const bool interior = x0 - R >= 1 && x0 + kTW + R <= nx - 1 && y0 - R >= 1 &&
                          y0 + TH + R <= ny - 1;  // wave-uniform
    if (interior) {
        const unsigned base = (unsigned)(y0 - R) * w + (unsigned)(x0 - R);
#pragma unroll
        for (int a = 0; a < NM; ++a) {
            const unsigned c = base + (unsigned)geo.j(a) * w + (unsigned)geo.i(a);
            const unsigned cm = c - w, cp = c + w;
            // pull: f_q(x) = f*_q(x - c_q), velocity table order
            f[a][0] = Store<S>::ld(at_u32(pq[0], c - 1));
            f[a][1] = Store<S>::ld(at_u32(pq[1], cm));
            f[a][2] = Store<S>::ld(at_u32(pq[2], c + 1));
            f[a][3] = Store<S>::ld(at_u32(pq[3], cp));
            f[a][4] = Store<S>::ld(at_u32(pq[4], cm - 1));
            f[a][5] = Store<S>::ld(at_u32(pq[5], cm + 1));
            f[a][6] = Store<S>::ld(at_u32(pq[6], cp + 1));
            f[a][7] = Store<S>::ld(at_u32(pq[7], cp - 1));
            gx[a] = *glob(at_u32(g, c));
            gy[a] = *glob(at_u32(g1, c));
            if constexpr (SR) sid[a] = c;
        }
        return;
    }
#pragma unroll
    for (int a = 0; a < NM; ++a) {
        const unsigned x = (unsigned)wrap_coord(x0 - R + geo.i(a), nx);
        const unsigned y = (unsigned)wrap_coord(y0 - R + geo.j(a), ny);
        const unsigned xm = (x == 0) ? w - 1 : x - 1;
        const unsigned xp = (x == w - 1) ? 0 : x + 1;
        const unsigned ym = (y == 0) ? (unsigned)ny - 1 : y - 1;
        const unsigned yp = (y == (unsigned)ny - 1) ? 0 : y + 1;
        const unsigned r0 = y * w, rm = ym * w, rp = yp * w;
        f[a][0] = Store<S>::ld(at_u32(pq[0], r0 + xm));
        f[a][1] = Store<S>::ld(at_u32(pq[1], rm + x));
        f[a][2] = Store<S>::ld(at_u32(pq[2], r0 + xp));
        f[a][3] = Store<S>::ld(at_u32(pq[3], rp + x));
        f[a][4] = Store<S>::ld(at_u32(pq[4], rm + xm));
        f[a][5] = Store<S>::ld(at_u32(pq[5], rm + xp));
        f[a][6] = Store<S>::ld(at_u32(pq[6], rp + xp));
        f[a][7] = Store<S>::ld(at_u32(pq[7], rp + xm));
        gx[a] = *glob(at_u32(g, r0 + x));
        gy[a] = *glob(at_u32(g1, r0 + x));
        if constexpr (SR) sid[a] = r0 + x;
    }
}

// Whether the tile kernel keeps the quarter force of every slot in registers
// (FP32 / FP64: LDS, not registers, limits their workgroups per CU) or forms it
// at each collision (half storage: four more registers per thread would cost a
// workgroup per CU).  Either way it is the same product of the half force.
template <typename S>
constexpr bool kKeepQuarter = !std::is_same<S, __half>::value;

// The quarter force of slot a for a collision.
template <typename S, typename C>
__device__ __forceinline__ C quarter(const C hq[][2], const C qg[][2], int a, int c) {
#pragma clang fp contract(off)
    if constexpr (kKeepQuarter<S>) return qg[a][c];
    else return C(0.5) * hq[a][c];
}

// Scales the force of every slot and keeps its half (hg) and, where registers
// allow, its quarter (qg): the products collide() forms, taken once per tile.
// Collides and writes step 1 to LDS; up[a] receives u of the step (for a check
// launch of two steps, u(n - 1)).
template <typename S, int TH, int NS, int NT = kBlock>
__device__ __forceinline__ void stepN_collide1(typename Store<S>::C f[][8],
                                               const Coef<typename Store<S>::C>& k, S* lds,
                                               const SlotGeo<TH, NS, NT>& geo,
                                               const typename Store<S>::C gx[],
                                               const typename Store<S>::C gy[],
                                               typename Store<S>::C hg[][2],
                                               typename Store<S>::C qg[][2],
                                               typename Store<S>::C up[][2],
                                               const unsigned sid[], bool sr, unsigned sh) {
#pragma clang fp contract(off)
    using C = typename Store<S>::C;
    using Geo = SlotGeo<TH, NS, NT>;
    constexpr int RW = Geo::RW, RN = Geo::RN, NM = Geo::NM;
#pragma unroll
    for (int a = 0; a < NM; ++a) {
        const int e = (int)threadIdx.x + a * NT;
        hg[a][0] = C(0.5) * (gx[a] * k.gscale);
        hg[a][1] = C(0.5) * (gy[a] * k.gscale);
        if constexpr (kKeepQuarter<S>) {
            qg[a][0] = C(0.5) * hg[a][0];
            qg[a][1] = C(0.5) * hg[a][1];
        }
        collide_h<C, false>(f[a], hg[a][0], hg[a][1], quarter<S>(hg, qg, a, 0),
                            quarter<S>(hg, qg, a, 1), k, up[a][0], up[a][1]);
        if (geo.active(a, 0)) {
            if constexpr (std::is_same<S, __half>::value) {
                if (sr) {
                    SrBits b;
                    b.make(sid[a], sh);
                    lds_write_sr<RW, RN>(lds, e, true, f[a], b);
                    continue;
                }
            }
            lds_write<S, RW, RN>(lds, e, true, f[a]);
        }
    }
}

// (sum, sum, max) over the NW waves of a workgroup in a fixed order; result
// valid in thread 0.  lds: 3 NW doubles.
template <int NW>
__device__ __forceinline__ void block_reduce3n(double& a, double& b, double& m, double* lds) {
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
        double sa[NW], sb[NW], sm[NW];
#pragma unroll
        for (int v = 0; v < NW; ++v) {
            sa[v] = lds[3 * v];
            sb[v] = lds[3 * v + 1];
            sm[v] = lds[3 * v + 2];
        }
#pragma unroll
        for (int h = 1; h < NW; h *= 2)
#pragma unroll
            for (int v = 0; v + h < NW; v += 2 * h) {
                sa[v] += sa[v + h];
                sb[v] += sb[v + h];
                sm[v] = fmax(sm[v], sm[v + h]);
            }
        a = sa[0];
        b = sb[0];
        m = sm[0];
    }
    __syncthreads();
}

// Steps 2..NS of the fused kernel for one tile whose step 1 is in LDS: middle
// steps on rings R-1 .. 1 (LDS -> registers -> LDS), then the tile from LDS to
// the destination field.  Step k reads the swapped layout when k is even and
// writes the natural one (and the reverse when k is odd); one barrier after
// each step.
//
// MODE kCheck (a launch whose last two steps are the two steps of a residual
// check): each thread keeps u(n - 1) of its tile sites from the step before
// the last (up), and the last step stores u(n) (FP64, unscaled, into u) and
// reduces sum |u(n) - u(n - 1)|^2, sum |u(n)|^2 and max |f*| over the tile into
// partial[0..2], as a check step after a write-u step does.
template <typename S, int TH, int NS, int NT = kBlock, int MODE = kPlain>
__device__ __forceinline__ void stepN_rest(S* __restrict__ dst, long long plane, int nx, int ny,
                                           int x0, int y0, const Coef<typename Store<S>::C>& k,
                                           S* lds, const SlotGeo<TH, NS, NT>& geo,
                                           const typename Store<S>::C hg[][2],
                                           const typename Store<S>::C qg[][2],
                                           typename Store<S>::C up[][2], double* u,
                                           double inv_scale, double* partial, double* red,
                                           const unsigned sid[], bool sr, unsigned step0,
                                           unsigned seed) {
    using C = typename Store<S>::C;
    using Geo = SlotGeo<TH, NS, NT>;
    constexpr int R = Geo::R, RW = Geo::RW, RN = Geo::RN, NM = Geo::NM;
    S* pq[8];  // wave-uniform plane bases
#pragma unroll
    for (int q = 0; q < 8; ++q) pq[q] = dst + q * plane;
#pragma unroll
    for (int m = 1; m < R; ++m) {
        const bool even = (m & 1) != 0;  // step m + 1
#pragma unroll
        for (int a = 0; a < NM; ++a) {
            const int e = (int)threadIdx.x + a * NT;
            if (geo.active(a, m)) {
                C f[8], ux, uy;
                lds_read<S, RW, RN>(lds, e, even, f);
                collide_h<C, false>(f, hg[a][0], hg[a][1], quarter<S>(hg, qg, a, 0),
                                    quarter<S>(hg, qg, a, 1), k, ux, uy);
                bool rounded = false;
                if constexpr (std::is_same<S, __half>::value) {
                    if (sr) {
                        SrBits b;
                        b.make(sid[a], sr_step_hash(step0 + (unsigned)m, seed));
                        lds_write_sr<RW, RN>(lds, e, !even, f, b);
                        rounded = true;
                    }
                }
                if (!rounded) lds_write<S, RW, RN>(lds, e, !even, f);
                if (MODE == kCheck && m == R - 1) {
                    up[a][0] = ux;
                    up[a][1] = uy;
                }
            }
        }
        __syncthreads();
    }
    constexpr bool last_even = (NS % 2) == 0;
    double dsum = 0.0, ssum = 0.0, fmaxv = 0.0;
#pragma unroll
    for (int a = 0; a < NM; ++a) {
        const int e = (int)threadIdx.x + a * NT;
        const int x = x0 + geo.i(a) - R, y = y0 + geo.j(a) - R;
        if (geo.active(a, R) && x < nx && y < ny) {  // the tile, inside the lattice
            C f[8], ux, uy;
            lds_read<S, RW, RN>(lds, e, last_even, f);
            collide_h<C, false>(f, hg[a][0], hg[a][1], quarter<S>(hg, qg, a, 0),
                                quarter<S>(hg, qg, a, 1), k, ux, uy);
            const unsigned sidx = (unsigned)y * (unsigned)nx + (unsigned)x;
            bool rounded = false;
            if constexpr (std::is_same<S, __half>::value) {
                if (sr) {
                    SrBits b;
                    b.make(sidx, sr_step_hash(step0 + (unsigned)R, seed));
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        Store<__half>::st_h(at_u32(pq[q], sidx), half_sr(f[q], b.r13(q)));
                    rounded = true;
                }
            }
            if (!rounded) {
#pragma unroll
                for (int q = 0; q < 8; ++q) Store<S>::st(at_u32(pq[q], sidx), f[q]);
            }
            if constexpr (MODE == kCheck) {
                const double uxd = (double)ux * inv_scale, uyd = (double)uy * inv_scale;
                const double dx = uxd - (double)up[a][0] * inv_scale;
                const double dy = uyd - (double)up[a][1] * inv_scale;
                dsum += dx * dx + dy * dy;
                ssum += uxd * uxd + uyd * uyd;
                double mm = 0.0;
#pragma unroll
                for (int q = 0; q < 8; ++q) mm = fmax(mm, (double)fabs(f[q]));
                fmaxv = fmax(fmaxv, mm);
                const long long s = (long long)y * nx + x;  // u planes are FP64
                glob(u)[s] = uxd;
                glob(u)[plane + s] = uyd;
            }
        }
    }
    __syncthreads();
    if constexpr (MODE == kCheck) {
        block_reduce3n<NT / kWave>(dsum, ssum, fmaxv, red);
        if (threadIdx.x == 0) {
            glob(partial)[0] = dsum;
            glob(partial)[1] = ssum;
            glob(partial)[2] = fmaxv;
        }
    }
}

// MODE kPlain (advance) or kCheck (advance; the last two steps form a
// residual check, partials per tile as the single-step check writes them).
//
// SR: half storage with stochastic rounding (a separate instantiation, so
// that the round-to-nearest kernel keeps its register count and occupancy).
template <typename S, int TH, int NS, int NT = kBlock, int MODE = kPlain, bool SR = false>
static __global__ __launch_bounds__(NT) void k_stepN(StepLaunch L) {
    using C = typename Store<S>::C;
    using Geo = SlotGeo<TH, NS, NT>;
    constexpr int RN = Geo::RN, NM = Geo::NM;
    __shared__ S lds[8 * RN];
    __shared__ double red[3 * (NT / kWave)];
    Geo geo;
    geo.init();
    int last, stride, it;
    xcd_slice(L.range, last, stride, it);
    for (; it < last; it += stride) {
        const Item item = L.items[it];
        const SlotDesc& d = L.slots[item.slot];
        const int sel = d.cur ^ L.flip;
        Coef<C> k;
        k.load(d);
        const int x0 = item.tx * kTW, y0 = item.ty * TH;
        C f[NM][8], gx[NM], gy[NM], hg[NM][2], qg[kKeepQuarter<S> ? NM : 1][2], up[NM][2];
        constexpr bool sr = SR && std::is_same<S, __half>::value;
        unsigned sid[sr ? NM : 1];  // site index per slot (stochastic rounding)
        stepN_load<S, TH, NS, NT, sr>(reinterpret_cast<const S*>(d.buf[sel]),
                                  reinterpret_cast<const C*>(d.g), d.plane, d.nx, d.ny, x0, y0,
                                  geo, f, gx, gy, sid);
        stepN_collide1<S, TH, NS, NT>(f, k, lds, geo, gx, gy, hg, qg, up, sid, sr,
                                      sr ? sr_step_hash(d.sr_step, d.sr_seed) : 0u);
        __syncthreads();
        stepN_rest<S, TH, NS, NT, MODE>(reinterpret_cast<S*>(d.buf[sel ^ 1]), d.plane, d.nx, d.ny,
                                        x0, y0, k, lds, geo, hg, qg, up, d.u, d.inv_scale,
                                        L.partial + 3 * it, red, sid, sr, d.sr_step, d.sr_seed);
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
// lane's column pair stays adjacent across the periodic wrap; its ring is an
// even number of columns (wave_ring) so that pairs stay aligned.  NS = 2..8:
// the deep variants keep a level's rows only as long as the next level reads
// them (the compiler's liveness does this over the unrolled row loop), and
// run at one or two waves per SIMD on registers alone (FP32 with V = 2 at
// eight steps: 423 registers, the excess in accumulation registers).
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

// Ring columns per side: NS for one column per lane; with two, an even number
// of at least four, so that a lane's column pair stays aligned.
template <int NS, int V>
__host__ __device__ constexpr int wave_ring() { return V == 1 ? NS : (NS <= 4 ? 4 : (NS + 1) / 2 * 2); }
template <int NS, int V>
__host__ __device__ constexpr int wave_width() { return kWave * V - 2 * wave_ring<NS, V>(); }

struct WaveLaunch {
    const SlotDesc* slots;
    int flip;
    int strips, segs, hs;  // strips of W output columns, segments of hs rows
    // in place: copies of the ring columns and halo rows taken before the launch
    // (k_wave_halo), by strip boundary and by segment boundary
    const void* hx;
    const void* hy;
};

// In-place wavefront (one buffer).  Every wave reads and writes the memory of
// the sites it outputs; the ring columns and halo rows it reads belong to
// other waves, which overwrite them during the launch, so they are read from
// copies taken by a launch before (k_wave_halo):
//   hx, per strip boundary b (at column b W): the 2R columns b W - R .. b W + R - 1
//     of every row, as [b][plane][row][2R];
//   hy, per segment boundary j (at row j hs): the 2 NS rows j hs - NS ..
//     j hs + NS - 1 of every column, as [j][plane][2 NS][nx]
// (periodic wrap; a strip's left ring is boundary s's first half, its right
// ring the next boundary's second half).  Layouts (see Layout): a launch from
// kLayNatural (odd NS) collides each site's own populations at level 1; one
// from kLaySwapped (even NS) reads f*_q(x) from plane opp(q) and gathers as
// the two-buffer kernel does; both store f*_q(x) into plane opp(q) at x, so the
// buffer ends in kLaySwapped, which is the layout NS steps on.
template <typename S>
static __global__ __launch_bounds__(kBlock) void k_wave_halo(WaveLaunch L, int W, int R, int NS) {
    const SlotDesc& d = L.slots[0];
    const int nx = d.nx, ny = d.ny;
    const long long plane = d.plane;
    const S* __restrict__ buf = reinterpret_cast<const S*>(d.buf[d.cur ^ L.flip]);
    S* __restrict__ hx = reinterpret_cast<S*>(const_cast<void*>(L.hx));
    S* __restrict__ hy = reinterpret_cast<S*>(const_cast<void*>(L.hy));
    const long long px = (long long)ny * 2 * R, py = (long long)2 * NS * nx;  // plane strides
    const long long nxe = (long long)L.strips * px, nye = (long long)L.segs * py;
    const long long step = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nxe + nye; i += step) {
        long long s;
        S* o;
        long long ps;
        if (i < nxe) {
            const long long b = i / px, r = i - b * px;
            const int row = (int)(r / (2 * R)), j = (int)(r - (long long)row * 2 * R);
            s = (long long)row * nx + wrap_coord((int)(b * W) - R + j, nx);
            o = hx + b * 8 * px + r;
            ps = px;
        } else {
            const long long k = i - nxe, b = k / py, r = k - b * py;
            const int hr = (int)(r / nx), col = (int)(r - (long long)hr * nx);
            s = (long long)wrap_coord((int)(b * L.hs) - NS + hr, ny) * nx + col;
            o = hy + b * 8 * py + r;
            ps = py;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) o[q * ps] = buf[q * plane + s];
    }
}

// SR: half storage with stochastic rounding (a separate instantiation): level
// lv of a launch is global step sr_step + lv - 1, and the bits of a column are
// those of its wrapped site, as the single-step kernel draws them.  IP: in
// place (see k_wave_halo), from kLayNatural for odd NS, kLaySwapped for even.
template <typename S, int NS, int V, bool SR = false, bool IP = false>
static __global__ __launch_bounds__(kBlock) void k_wave(WaveLaunch L) {
    using C = typename Store<S>::C;
    constexpr int R = wave_ring<NS, V>();
    constexpr bool kSR = SR && std::is_same<S, __half>::value;
    static_assert(!(SR && IP), "no stochastic rounding in place");
    constexpr bool kNat = IP && (NS % 2 == 1);  // level 0 is f(n) itself
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
    // two buffers: read one, write the other; in place one buffer (no restrict)
    using SrcP = std::conditional_t<IP, const S*, const S* __restrict__>;
    using DstP = std::conditional_t<IP, S*, S* __restrict__>;
    const SrcP src = reinterpret_cast<const S*>(d.buf[sel]);
    const DstP dst = reinterpret_cast<S*>(d.buf[IP ? sel : (sel ^ 1)]);
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
    // in place: ring lanes read the strip boundaries' copies (any row), the
    // others the segment boundaries' copies in halo rows, else the buffer
    const S* hxl = nullptr;
    bool ring = false;
    if constexpr (IP) {
        const int xe = min(xs + W, nx);
        const bool left = lane < R / V, right = x >= xe && x < xe + R;
        ring = left || right;
        const int b = left ? sx : (sx + 1 == L.strips ? 0 : sx + 1);
        hxl = reinterpret_cast<const S*>(L.hx) + (long long)b * 8 * ny * 2 * R +
              (left ? V * lane : R + (x - xe));
    }
    auto load_row = [&](int t, C (*a)[V], C (*gg)[V]) {
        const long long r = (long long)wrap_coord(t, ny) * nx;
        if constexpr (IP) {
            const S* own = src + r;
            long long ops = plane;
            if (t < ya || (t >= yb && t < yb + NS)) {
                const int b = t < ya ? sy : (sy + 1 == L.segs ? 0 : sy + 1);
                const int hr = t < ya ? t - (ya - NS) : NS + (t - yb);
                own = reinterpret_cast<const S*>(L.hy) + (long long)b * 16 * NS * nx +
                      (long long)hr * nx;
                ops = 2LL * NS * nx;
            }
            const S* p = ring ? hxl + (long long)wrap_coord(t, ny) * 2 * R : own + xw;
            const long long ps = ring ? (long long)ny * 2 * R : ops;
#pragma unroll
            for (int q = 0; q < 8; ++q) VecIO<S, V>::ld(p + q * ps, a[q]);
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                VecIO<S, V>::ld(reinterpret_cast<const S*>(
                                    reinterpret_cast<const char*>(src + (q * plane + r)) + xs_b),
                                a[q]);
        }
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
                if (kNat && lv == 1) {
                    // f(n) of the site itself (level 0 of row t - 1)
#pragma unroll
                    for (int c = 0; c < V; ++c)
#pragma unroll
                        for (int q = 0; q < 8; ++q) f[c][q] = R1[q][c];
                } else {
                    // in place from kLaySwapped, level 0 holds f*_q in slot opp(q)
                    auto sq = [&](int q) { return (IP && lv == 1) ? opp(q) : q; };
#pragma unroll
                    for (int c = 0; c < V; ++c) {
                        f[c][0] = left(R1, sq(0), c);   // c1 = ( 1, 0) from (x-1, y)
                        f[c][1] = R2[sq(1)][c];         // c2 = ( 0, 1) from (x, y-1)
                        f[c][2] = right(R1, sq(2), c);  // c3 = (-1, 0) from (x+1, y)
                        f[c][3] = R0[sq(3)][c];         // c4 = ( 0,-1) from (x, y+1)
                        f[c][4] = left(R2, sq(4), c);   // c5 = ( 1, 1) from (x-1, y-1)
                        f[c][5] = right(R2, sq(5), c);  // c6 = (-1, 1) from (x+1, y-1)
                        f[c][6] = right(R0, sq(6), c);  // c7 = (-1,-1) from (x+1, y+1)
                        f[c][7] = left(R0, sq(7), c);   // c8 = ( 1,-1) from (x-1, y+1)
                    }
                }
#pragma unroll
                for (int c = 0; c < V; ++c) {
                    C ux, uy;
                    collide<C, false>(f[c], G[lv][0][c], G[lv][1][c], k, ux, uy);
                }
                SrBits sb[kSR ? V : 1];
                if constexpr (kSR) {
                    const unsigned row = (unsigned)wrap_coord(t - lv, ny) * (unsigned)nx;
                    const unsigned sh = sr_step_hash(d.sr_step + (unsigned)(lv - 1), d.sr_seed);
#pragma unroll
                    for (int c = 0; c < V; ++c) sb[c].make(row + (unsigned)(xw + c), sh);
                }
                if (lv < NS) {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
#pragma unroll
                        for (int c = 0; c < V; ++c) {
                            if constexpr (kSR)
                                A[lv][u % 3][q][c] = __half2float(half_sr(f[c][q], sb[c].r13(q)));
                            else
                                A[lv][u % 3][q][c] = as_stored<S>(f[c][q]);
                        }
                } else {
                    const int y = t - NS;
                    if (out_lane && y >= ya && y < yb) {
                        const long long o = (long long)y * nx + x;
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            C v[V];
#pragma unroll
                            for (int c = 0; c < V; ++c) {
                                v[c] = f[c][q];
                                // rounded here, so the store's own rounding is exact
                                if constexpr (kSR) v[c] = __half2float(half_sr(v[c], sb[c].r13(q)));
                            }
                            // in place: f*_q into plane opp(q) (kLaySwapped)
                            VecIO<S, V>::st(dst + (IP ? opp(q) : q) * plane + o, v);
                        }
                    }
                }
            }
        }
    }
}

}  // namespace lbm
