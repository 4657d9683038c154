// Temporal blocking through an LDS tile: several steps per launch,
// bit-identical to single steps (the register wavefront is in lbm_wave.hpp).
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

}  // namespace lbm
