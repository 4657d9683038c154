"""Launch-shape autotuner for the step kernel.

Times candidate launch shapes (tile width, rows per thread, persistent grid
or one workgroup per tile, steps per launch, and for a single lattice the
fused kernel: LDS tile with its tile height or register wavefront with its
segment height) with
HIP events on the solver's stream and keeps the fastest.  Results are cached in a JSON file keyed by GPU architecture,
storage precision, workload kind and a size bucket (log2 of the sites per
step), so a shape is measured once per machine and size class.

Tuning advances the state of the object it times; tune a scratch instance
(or reset the solver afterwards).  The shape never changes results: every
shape computes the same per-site arithmetic.
"""
from __future__ import annotations

import json
import math
import os
from typing import Callable, Dict, Iterable, List, Optional, Tuple

import torch

# (bx_log2, rows_per_thread, blocks_per_cu, steps_per_launch, wavefront_rows,
# tile_rows); wavefront_rows 0 = LDS tile kernel for the fused launches,
# tile_rows 0 = the library's default tile height
Shape = Tuple[int, int, int, int, int, int]

DEFAULT_CACHE = os.environ.get("LBM_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache",
                                            "lbm_elastic_autotune.json"))


def candidates(nx: int, min_bx: int = 3, ny: int = 0, wavefront: bool = False,
               fused: bool = True, precision: str = "fp32", inplace: bool = False) -> List[Shape]:
    """Single-step tile shapes; the fused LDS tile kernel at 2..8 steps with one
    workgroup per tile or a persistent grid, and for single FP32 lattices also
    its 24-row tile at five steps or more; and (single lattices) the register
    wavefront at 3..8 steps with a few segment heights.  In place: single-step
    shapes and the in-place wavefront (those the solver's halo room admits are
    timed); fused=False: single-step shapes only."""
    if inplace:
        out = []
        if fused:
            for rows in (64, 128, 256):
                if rows <= max(ny, 32):
                    out += [(6, 4, 0, t, rows, 0) for t in (8, 6, 4)]
        return out + [s for s in candidates(nx, min_bx, ny, fused=False) if s[3] == 1]
    out = [(6, 4, k, t, 0, 0) for t in (8, 7, 6, 5, 4, 3, 2) for k in (0, 4)] if fused else []
    if fused and wavefront and precision == "fp32":
        out += [(6, 4, 0, t, 0, 24) for t in (8, 7, 6, 5)]
    if wavefront and fused:
        for rows in (32, 64, 128, 256):
            if rows <= max(ny, 32):
                out += [(6, 4, 0, t, rows, 0) for t in (8, 6, 4, 3)]
    for b in (5, 6, 7, 8):
        if b < min_bx or (1 << b) > max(2 * nx, 1 << min_bx):
            continue
        for v in (1, 2, 4):
            for k in (0, 4):
                out.append((b, v, k, 1, 0, 0))
    return out


def _apply(obj, shp: Shape):
    if getattr(obj, "inplace", False):
        # in place the depth is checked against the halo room for the segment
        # height: set the height at one step per launch, then the depth
        obj.set_time_blocking(1)
        obj.set_tile(shp[0], shp[1], shp[2])
        if shp[4] > 0:
            obj.set_fused_kernel("wavefront", shp[4])
        obj.set_time_blocking(shp[3])
        return
    obj.set_time_blocking(shp[3])
    obj.set_tile(shp[0], shp[1], shp[2])
    if hasattr(obj, "set_fused_kernel") and not getattr(obj, "inplace", False):
        if shp[4] > 0:
            obj.set_fused_kernel("wavefront", shp[4])
        else:
            obj.set_fused_kernel("tile")
    if hasattr(obj, "set_tile_rows") and not getattr(obj, "inplace", False):
        obj.set_tile_rows(shp[5] if len(shp) > 5 else 0)


def batch_candidates() -> List[Shape]:
    """Batch shapes.  Element 4 says which lattices take the wavefront list:
    0 the default rule (with every shape of candidates(64, 3)), 1 all of them
    and 2 none (at the depths where the wavefront and the tile run best)."""
    return candidates(64, 3) + [(6, 4, 0, 8, 1, 0), (6, 4, 0, 8, 2, 0), (6, 4, 0, 5, 2, 0)]


def _apply_batch(batch, precision: str, shp: Shape):
    _apply(batch, shp)
    batch.set_wavefront_sites(precision, {0: -1, 1: 0}.get(shp[4], 1 << 62))


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _key(kind: str, precision: str, sites: int) -> str:
    return f"{_arch()}|{kind}|{precision}|2^{int(round(math.log2(max(sites, 1))))}|v10"


def _load(path: str) -> Dict[str, list]:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: Dict[str, list]):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def time_shapes(set_shape: Callable[[Shape], None], step: Callable[[int], None],
                shapes: Iterable[Shape], sites: int, target_ms: float = 3.0,
                repeats: int = 3) -> List[Tuple[float, Shape]]:
    """Returns [(microseconds per step, shape)] sorted fastest first.  Step
    counts are whole multiples of the shape's steps per launch, so that only
    the shape's own launches are timed."""
    from .lbm import LbmError
    res = []
    for shp in shapes:
        try:
            set_shape(shp)
        except LbmError:  # a shape this solver does not admit (e.g. halo room)
            continue
        t = max(1, shp[3])
        k = 4 * t
        step(k)  # warm the shape (graph capture, caches)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        step(k)
        e1.record()
        torch.cuda.synchronize()
        per = max(e0.elapsed_time(e1) / k, 1e-4)
        n = max(k, min(4000, int(target_ms / per)) // t * t)
        best = float("inf")
        for _ in range(repeats):
            e0.record()
            step(n)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, 1e3 * e0.elapsed_time(e1) / n)
        res.append((best, shp))
    res.sort()
    return res


def solver_candidates(solver, precision: str) -> List[Shape]:
    """The shapes tune_solver times for a solver: candidates() for its size and
    kind and, when its current plain-step kernel is the wavefront (the
    library's default for the larger lattices), that shape with its segment
    height."""
    inplace = getattr(solver, "inplace", False)
    out = candidates(solver.nx, 0, solver.ny, wavefront=True, precision=precision,
                     inplace=inplace)
    cfg = solver.launch_config()
    if cfg["kernel"] == "wavefront":
        cur = (6, 4, 0, cfg["steps_per_launch"], cfg["rows"], 0)
        if cur not in out:
            out = [cur] + out
    return out


def tune_solver(solver, precision: str, cache_path: Optional[str] = DEFAULT_CACHE,
                force: bool = False) -> Shape:
    """Pick and apply the fastest launch shape for a single-lattice solver."""
    sites = solver.nx * solver.ny
    inplace = getattr(solver, "inplace", False)
    key = _key("single-inplace" if inplace else "single", precision, sites)
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        shp = tuple(cache[key])
        _apply(solver, shp)
        return shp
    res = time_shapes(lambda s: _apply(solver, s), solver.step,
                      solver_candidates(solver, precision), sites)
    shp = res[0][1]
    _apply(solver, shp)
    if cache_path:
        cache[key] = list(shp)
        _store(cache_path, cache)
    return shp


def tune_batch(batch, precision: str, sites: int, cache_path: Optional[str] = DEFAULT_CACHE,
               force: bool = False) -> Shape:
    """Pick and apply the fastest launch shape for a batch (sites = total sites)."""
    key = _key("batch", precision, sites)
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        shp = tuple(cache[key])
        _apply_batch(batch, precision, shp)
        return shp
    res = time_shapes(lambda s: _apply_batch(batch, precision, s), lambda n: batch.step(n),
                      batch_candidates(), sites)
    shp = res[0][1]
    _apply_batch(batch, precision, shp)
    if cache_path:
        cache[key] = list(shp)
        _store(cache_path, cache)
    return shp
