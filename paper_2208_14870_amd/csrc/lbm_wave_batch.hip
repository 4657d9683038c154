// Register-wavefront launches over a list of waves of several lattices (the
// lattices on a batch's wavefront list): k_wave<..., LIST> with one column per
// lane for every storage type and depth, in a translation unit of its own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "lbm_wave.hpp"
#include "lbm_host_base.hpp"

namespace lbm_host {

namespace {
template <typename S>
void launch_wave_list_t(int ns, unsigned grid, hipStream_t st, const WaveLaunch& W) {
    switch (ns) {
        case 2: hipLaunchKernelGGL((k_wave<S, 2, 1, false, false, true>), dim3(grid), dim3(kBlock), 0, st, W); break;
        case 3: hipLaunchKernelGGL((k_wave<S, 3, 1, false, false, true>), dim3(grid), dim3(kBlock), 0, st, W); break;
        case 4: hipLaunchKernelGGL((k_wave<S, 4, 1, false, false, true>), dim3(grid), dim3(kBlock), 0, st, W); break;
        case 5: hipLaunchKernelGGL((k_wave<S, 5, 1, false, false, true>), dim3(grid), dim3(kBlock), 0, st, W); break;
        case 6: hipLaunchKernelGGL((k_wave<S, 6, 1, false, false, true>), dim3(grid), dim3(kBlock), 0, st, W); break;
        case 7: hipLaunchKernelGGL((k_wave<S, 7, 1, false, false, true>), dim3(grid), dim3(kBlock), 0, st, W); break;
        default: hipLaunchKernelGGL((k_wave<S, 8, 1, false, false, true>), dim3(grid), dim3(kBlock), 0, st, W); break;
    }
}
}  // namespace

hipError_t launch_wave_list(int prec, int ns, const SlotDesc* slots, const WaveItem* items,
                            const int* wrange, int nitems, int flip, unsigned grid,
                            hipStream_t st) {
    if (ns < 2 || ns > 8 || nitems < 0 || !items || !wrange ||
        (long long)grid * (kBlock / kWave) < nitems)
        return hipErrorInvalidValue;
    WaveLaunch W;
    W.slots = slots;
    W.items = items;
    W.wrange = wrange;
    W.flip = flip;
    W.strips = W.segs = W.hs = 0;
    W.hx = W.hy = nullptr;
    if (prec == LBM_FP64) launch_wave_list_t<double>(ns, grid, st, W);
    else if (prec == LBM_FP32) launch_wave_list_t<float>(ns, grid, st, W);
    else launch_wave_list_t<__half>(ns, grid, st, W);
    return hipGetLastError();
}

}  // namespace lbm_host
