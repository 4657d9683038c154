// Temporal blocking through a register wavefront (two buffers, or in place
// with halo copies): several steps per launch, bit-identical to single steps.
#pragma once

#include <type_traits>

#include "lbm_common.hpp"

namespace lbm {

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
// The shifts write 0 where no source lane exists (lane 0 from the left, lane 63
// from the right: ring lanes whose values never reach the output), so the
// destination needs no initial value (bound_ctrl).
__device__ __forceinline__ float lane_from_left(float v) {  // lane l <- lane l-1
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_from_right(float v) {  // lane l <- lane l+1
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_from_left(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane_from_right(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x130, 0xf, 0xf, true);
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

// One wave's work in a list over several lattices (a batch): lattice slot,
// strip, and output rows ya .. yb - 1.
struct WaveItem {
    int slot, sx, ya, yb;
};

struct WaveLaunch {
    const SlotDesc* slots;
    // list mode: the waves' items (slots index the descriptor table), the
    // launch's items[wrange[0] .. wrange[1] - 1] (device memory, so that a
    // captured launch stays valid while the list changes)
    const WaveItem* items;
    const int* wrange;
    int flip;
    // strips of W output columns (strip s from column s W, so that its stores
    // start on the strip width: shifting the strips to align the loads instead
    // measured slower, FP32 8192^2 356 against 428 GLUPS), segments of hs rows
    int strips, segs, hs;
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
// LIST: each wave takes its lattice, strip and rows from L.items (a batch of
// lattices; two buffers, no stochastic rounding).
template <typename S, int NS, int V, bool SR = false, bool IP = false, bool LIST = false>
static __global__ __launch_bounds__(kBlock) void k_wave(WaveLaunch L) {
    using C = typename Store<S>::C;
    constexpr int R = wave_ring<NS, V>();
    constexpr bool kSR = SR && std::is_same<S, __half>::value;
    static_assert(!(SR && IP), "no stochastic rounding in place");
    static_assert(!(LIST && (SR || IP)), "lists run two buffers with rounding to nearest");
    constexpr bool kNat = IP && (NS % 2 == 1);  // level 0 is f(n) itself
    constexpr int W = wave_width<NS, V>();
    constexpr int PF = 3;  // rows loaded ahead
    // wave index as a scalar: the row loop and the row bases stay scalar.
    // Blocks go to the 8 XCDs round-robin; each XCD takes a contiguous range of
    // the blocks that have work, so that strips side by side, whose rings
    // overlap, run on one XCD at the same time and share its L2 (a list's grid
    // is rounded up: its surplus blocks leave first, or the work would gather
    // on the first XCDs).
    const int nwaves = LIST ? L.wrange[1] - L.wrange[0] : L.strips * L.segs;
    const int nb = (nwaves + kBlock / kWave - 1) / (kBlock / kWave), b = (int)blockIdx.x;
    if (b >= nb) return;  // whole blocks leave; no barrier follows
    const int lb = (b % 8) * (nb / 8) + min(b % 8, nb % 8) + b / 8;
    const int wid = __builtin_amdgcn_readfirstlane(lb * (kBlock / kWave) + (int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & (kWave - 1));
    if (wid >= nwaves) return;  // whole waves leave
    WaveItem item{0, 0, 0, 0};
    if constexpr (LIST) item = L.items[L.wrange[0] + wid];
    const SlotDesc& d = L.slots[item.slot];
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
    const int sx = LIST ? item.sx : wid % L.strips, sy = LIST ? 0 : wid / L.strips;
    const int xs = sx * W;
    const int ya = LIST ? item.ya : sy * L.hs, yb = LIST ? item.yb : min(ya + L.hs, ny);
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
            // (rows from yb + NS on feed no output; loading them anyway keeps
            // the loop free of branches: skipping them measured slower, FP16
            // 8192^2 375 against 446 GLUPS)
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
