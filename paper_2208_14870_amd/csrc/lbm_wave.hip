// Register-wavefront launches with two buffers (k_wave): the instantiations
// for every storage type, depth and lane width, in a translation unit of
// their own so that they compile beside the rest of the library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lbm_wave.hpp"
#include "lbm_host_base.hpp"

namespace lbm_host {

namespace {
// Half storage with two columns per lane runs at most four steps (wave_cols),
// so its deeper variants are not built.
template <typename S, int V>
constexpr int kWaveMaxSteps = (V == 2 && std::is_same<S, __half>::value) ? 4 : 8;

template <typename S, int V, bool SR>
void launch_wave_t(int ns, unsigned grid, hipStream_t st, const WaveLaunch& W) {
    switch (ns) {
        case 2: hipLaunchKernelGGL((k_wave<S, 2, V, SR>), dim3(grid), dim3(kBlock), 0, st, W); break;
        case 3: hipLaunchKernelGGL((k_wave<S, 3, V, SR>), dim3(grid), dim3(kBlock), 0, st, W); break;
        case 4: hipLaunchKernelGGL((k_wave<S, 4, V, SR>), dim3(grid), dim3(kBlock), 0, st, W); break;
        default:
            if constexpr (kWaveMaxSteps<S, V> == 8) {
                if (ns == 5) hipLaunchKernelGGL((k_wave<S, 5, V, SR>), dim3(grid), dim3(kBlock), 0, st, W);
                else if (ns == 6) hipLaunchKernelGGL((k_wave<S, 6, V, SR>), dim3(grid), dim3(kBlock), 0, st, W);
                else if (ns == 7) hipLaunchKernelGGL((k_wave<S, 7, V, SR>), dim3(grid), dim3(kBlock), 0, st, W);
                else hipLaunchKernelGGL((k_wave<S, 8, V, SR>), dim3(grid), dim3(kBlock), 0, st, W);
            }
            break;
    }
}
}  // namespace

hipError_t launch_wave(int prec, int ns, int v, int nx, int ny, int hs, const SlotDesc* slots,
                       int flip, hipStream_t st, bool sr) {
    if (ns < 2 || ns > 8 || hs < 1 || (v == 2 && (prec == LBM_FP64 || nx % 2 != 0)) ||
        (v == 2 && prec == LBM_FP16 && ns > 4) || (sr && prec != LBM_FP16))
        return hipErrorInvalidValue;
    const int w = wave_width_of(ns, v);
    WaveLaunch W;
    W.slots = slots;
    W.items = nullptr;
    W.wrange = nullptr;
    W.flip = flip;
    W.strips = (nx + w - 1) / w;
    W.hs = hs;
    W.segs = (ny + hs - 1) / hs;
    W.hx = W.hy = nullptr;
    const long long waves = (long long)W.strips * W.segs;
    const unsigned grid = (unsigned)((waves + kBlock / kWave - 1) / (kBlock / kWave));
    if (prec == LBM_FP64) launch_wave_t<double, 1, false>(ns, grid, st, W);
    else if (prec == LBM_FP32 && v == 2) launch_wave_t<float, 2, false>(ns, grid, st, W);
    else if (prec == LBM_FP32) launch_wave_t<float, 1, false>(ns, grid, st, W);
    else if (v == 2 && sr) launch_wave_t<__half, 2, true>(ns, grid, st, W);
    else if (sr) launch_wave_t<__half, 1, true>(ns, grid, st, W);
    else if (v == 2) launch_wave_t<__half, 2, false>(ns, grid, st, W);
    else launch_wave_t<__half, 1, false>(ns, grid, st, W);
    return hipGetLastError();
}

}  // namespace lbm_host
