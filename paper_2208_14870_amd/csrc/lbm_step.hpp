// Single-step kernels: the fused stream + collide step in every layout and
// mode, streaming alone, the in-place residual check and the per-lattice
// finalisation of the residual partials.
#pragma once

#include <type_traits>

#include "lbm_common.hpp"

namespace lbm {

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
                bool rounded = false;
                if constexpr (std::is_same<S, __half>::value) {
                    if (d.sr) {  // stochastic rounding of this step's stores
                        SrBits b;
                        b.make((unsigned)s, sr_step_hash(d.sr_step, d.sr_seed));
#pragma unroll
                        for (int q = 0; q < 8; ++q)
                            Store<__half>::st_h(dst + q * plane + s, half_sr(f[j][q], b.r13(q)));
                        rounded = true;
                    }
                }
                if (!rounded) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) Store<S>::st(dst + q * plane + s, f[j][q]);
                }
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

}  // namespace lbm
