// In-place register-wavefront launches (one population buffer): the halo
// copy (k_wave_halo) and k_wave<..., IP> for every storage type, depth and
// lane width, in a translation unit of their own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lbm_wave.hpp"
#include "lbm_host_base.hpp"

namespace lbm_host {

namespace {
template <typename S, int V>
constexpr int kWaveMaxSteps = (V == 2 && std::is_same<S, __half>::value) ? 4 : 8;

template <typename S, int V>
void launch_wave_ip_t(int ns, unsigned grid, hipStream_t st, const WaveLaunch& W) {
    switch (ns) {
        case 2: hipLaunchKernelGGL((k_wave<S, 2, V, false, true>), dim3(grid), dim3(kBlock), 0, st, W); break;
        case 3: hipLaunchKernelGGL((k_wave<S, 3, V, false, true>), dim3(grid), dim3(kBlock), 0, st, W); break;
        case 4: hipLaunchKernelGGL((k_wave<S, 4, V, false, true>), dim3(grid), dim3(kBlock), 0, st, W); break;
        default:
            if constexpr (kWaveMaxSteps<S, V> == 8) {
                if (ns == 5) hipLaunchKernelGGL((k_wave<S, 5, V, false, true>), dim3(grid), dim3(kBlock), 0, st, W);
                else if (ns == 6) hipLaunchKernelGGL((k_wave<S, 6, V, false, true>), dim3(grid), dim3(kBlock), 0, st, W);
                else if (ns == 7) hipLaunchKernelGGL((k_wave<S, 7, V, false, true>), dim3(grid), dim3(kBlock), 0, st, W);
                else hipLaunchKernelGGL((k_wave<S, 8, V, false, true>), dim3(grid), dim3(kBlock), 0, st, W);
            }
            break;
    }
}

template <typename S>
void launch_halo_t(const WaveLaunch& W, int w, int r, int ns, long long elems, hipStream_t st) {
    const long long want = (elems + kBlock - 1) / kBlock;
    const unsigned grid = (unsigned)std::min<long long>(want, 1LL << 16);
    hipLaunchKernelGGL(k_wave_halo<S>, dim3(grid), dim3(kBlock), 0, st, W, w, r, ns);
}
}  // namespace

hipError_t launch_wave_inplace(int prec, int ns, int v, int nx, int ny, int hs,
                               const SlotDesc* slots, int flip, void* halo, hipStream_t st) {
    if (ns < 2 || ns > 8 || hs < 1 || !halo || (v == 2 && (prec == LBM_FP64 || nx % 2 != 0)) ||
        (v == 2 && prec == LBM_FP16 && ns > 4))
        return hipErrorInvalidValue;
    const int w = wave_width_of(ns, v), r = wave_ring_of(ns, v);
    WaveLaunch W;
    W.slots = slots;
    W.items = nullptr;
    W.wrange = nullptr;
    W.flip = flip;
    W.strips = (nx + w - 1) / w;
    W.hs = hs;
    W.segs = (ny + hs - 1) / hs;
    W.hx = halo;
    W.hy = static_cast<char*>(halo) + wave_halo_x_bytes(prec, ns, v, nx, ny);
    const long long elems = (long long)W.strips * 2 * r * ny + (long long)W.segs * 2 * ns * nx;
    if (prec == LBM_FP64) launch_halo_t<double>(W, w, r, ns, elems, st);
    else if (prec == LBM_FP32) launch_halo_t<float>(W, w, r, ns, elems, st);
    else launch_halo_t<__half>(W, w, r, ns, elems, st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long waves = (long long)W.strips * W.segs;
    const unsigned grid = (unsigned)((waves + kBlock / kWave - 1) / (kBlock / kWave));
    if (prec == LBM_FP64) launch_wave_ip_t<double, 1>(ns, grid, st, W);
    else if (prec == LBM_FP32 && v == 2) launch_wave_ip_t<float, 2>(ns, grid, st, W);
    else if (prec == LBM_FP32) launch_wave_ip_t<float, 1>(ns, grid, st, W);
    else if (v == 2) launch_wave_ip_t<__half, 2>(ns, grid, st, W);
    else launch_wave_ip_t<__half, 1>(ns, grid, st, W);
    return hipGetLastError();
}

}  // namespace lbm_host
