// Host-side basics shared by every translation unit: alignment and element
// sizes, the register wavefront's strip and halo shapes, and the wavefront
// launchers (compiled in translation units of their own).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

#include "lbm.h"
#include "lbm_common.hpp"

namespace lbm {
struct WaveLaunch;
struct WaveItem;
}

namespace lbm_host {
using namespace lbm;

constexpr size_t kAlign = 256;
inline size_t al(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

inline size_t elem_bytes(int prec) { return prec == LBM_FP64 ? 8 : (prec == LBM_FP32 ? 4 : 2); }
inline size_t arith_bytes(int prec) { return prec == LBM_FP64 ? 8 : 4; }
inline bool valid_prec(int p) { return p == LBM_FP64 || p == LBM_FP32 || p == LBM_FP16; }

// Register-wavefront launch of `ns` plain steps on slot 0 (single lattice),
// segments of hs rows; v: columns per lane (2 needs an even nx and non-FP64
// storage; half storage with two columns runs at most four steps); sr: half
// storage with stochastic rounding.  Defined in lbm_wave.hip.
hipError_t launch_wave(int prec, int ns, int v, int nx, int ny, int hs, const SlotDesc* slots,
                       int flip, hipStream_t st, bool sr = false);

// Ring columns per side and output columns of a wave's strip (64 v columns
// less the ring on each side).
inline int wave_ring_of(int ns, int v) { return v == 1 ? ns : (ns <= 4 ? 4 : (ns + 1) / 2 * 2); }
inline int wave_width_of(int ns, int v) { return kWave * v - 2 * wave_ring_of(ns, v); }

// In place (one buffer): the copies of ring columns and halo rows that a
// launch of ns steps reads (k_wave_halo), in bytes: per strip boundary 2R
// columns of every row, per segment boundary 2 ns rows of every column, eight
// planes each.  The column copies come first, the row copies at
// wave_halo_x_bytes.
inline size_t wave_halo_x_bytes(int prec, int ns, int v, int nx, int ny) {
    const int w = wave_width_of(ns, v), r = wave_ring_of(ns, v);
    const long long strips = (nx + w - 1) / w;
    return al((size_t)(8 * strips * 2LL * r * ny) * elem_bytes(prec));
}
inline size_t wave_halo_bytes(int prec, int ns, int v, int nx, int ny, int hs) {
    const long long segs = (ny + hs - 1) / hs;
    return wave_halo_x_bytes(prec, ns, v, nx, ny) +
           al((size_t)(8 * segs * 2LL * ns * nx) * elem_bytes(prec));
}

// Wavefront over a list of waves of several lattices (a batch; two buffers,
// one column per lane, any widths): the launch runs items[wrange[0] ..
// wrange[1] - 1] (wrange in device memory), each naming its lattice's
// descriptor slot, strip (of 64 - 2 ns' columns for the list's depth ns' >=
// ns: a shallower launch leaves the surplus strips idle) and rows.  nitems:
// the list's current length, to check the grid (workgroups of four waves).
// Defined in lbm_wave_batch.hip.
hipError_t launch_wave_list(int prec, int ns, const SlotDesc* slots, const WaveItem* items,
                            const int* wrange, int nitems, int flip, unsigned grid,
                            hipStream_t st);

// In-place launch of ns steps: the halo copy, then the wavefront.  The buffer
// must be in kLayNatural for odd ns and kLaySwapped for even ns; it ends in
// kLaySwapped.  halo: wave_halo_bytes(prec, ns, v, nx, ny, hs) bytes.  Defined
// in lbm_wave_inplace.hip.
hipError_t launch_wave_inplace(int prec, int ns, int v, int nx, int ny, int hs,
                               const SlotDesc* slots, int flip, void* halo, hipStream_t st);

}  // namespace lbm_host
