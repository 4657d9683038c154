"""Thin Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the method runs in the HIP kernels of ``liblbm.so``; this
module only loads the library, allocates caller-owned device memory as torch
tensors, passes raw pointers and the current HIP stream, and converts status
codes into exceptions.  There is no CPU fallback: if ``liblbm.so`` is missing
or no GPU is present, every entry point raises.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Tuple

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbm.so")

FP64, FP32, FP16 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16": FP16}
STATUS = {0: "OK", 1: "NOT_CONVERGED", 2: "W_MEAN_REMOVED", 4: "W_STAGGERED_LOAD",
          6: "W_MEAN_REMOVED|W_STAGGERED_LOAD", -1: "E_ARG", -2: "E_MATERIAL",
          -3: "E_WORKSPACE", -4: "E_HIP", -5: "E_DIVERGED", -6: "E_STATE"}
W_MEAN_REMOVED, W_STAGGERED_LOAD = 2, 4
E_ARG, E_MATERIAL, E_WORKSPACE, E_HIP, E_DIVERGED, E_STATE = -1, -2, -3, -4, -5, -6
FORCE_WARNINGS = (0, 2, 4, 6)


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Diverged(LbmError):
    pass


_lib = None


def load() -> ctypes.CDLL:
    """Load liblbm.so (built by __graft_entry__.build()); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, ll, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_double, ctypes.c_size_t
    pll, pd, pi = ctypes.POINTER(ll), ctypes.POINTER(d), ctypes.POINTER(i)
    sigs = {
        "lbm_workspace_bytes": (sz, [i, i, i, i]),
        "lbm_create": (i, [i, i, i, i, vp, sz, vp, ctypes.POINTER(vp)]),
        "lbm_destroy": (i, [vp]),
        "lbm_set_material": (i, [vp, d, d]),
        "lbm_set_rates": (i, [vp, d, d, d, d]),
        "lbm_set_body_force": (i, [vp, vp, vp]),
        "lbm_set_body_force_corrected": (i, [vp, vp, vp, vp]),
        "lbm_leading_error_constants": (i, [d, d, d, d, d, d, pd]),
        "lbm_fourth_order_rates": (i, [d, d, d, pd]),
        "lbm_reset": (i, [vp]),
        "lbm_step": (i, [vp, ll]),
        "lbm_step_checked": (i, [vp, ll, pd]),
        "lbm_solve_to_tol": (i, [vp, d, ll, i, pll, pd]),
        "lbm_set_polish": (i, [vp, d]),
        "lbm_set_small_solve": (i, [vp, ll]),
        "lbm_set_divergence_guard": (i, [vp, i]),
        "lbm_current_precision": (i, [vp]),
        "lbm_steps_done": (ll, [vp]),
        "lbm_get_displacement": (i, [vp, vp, vp]),
        "lbm_get_stress": (i, [vp, vp, vp, vp]),
        "lbm_error_norms": (i, [vp, vp, vp, pd]),
        "lbm_error_norms_noalloc": (i, [i, i, vp, vp, vp, vp, vp, vp]),
        "lbm_get_populations": (i, [vp, vp]),
        "lbm_set_populations": (i, [vp, vp]),
        "lbm_set_tile": (i, [vp, i, i, i]),
        "lbm_debug_stream_only": (i, [vp, ll]),
        "lbm_set_time_blocking": (i, [vp, i]),
        "lbm_set_fused_kernel": (i, [vp, i, i]),
        "lbm_set_stochastic_rounding": (i, [vp, i, ctypes.c_uint]),
        "lbm_set_tile_rows": (i, [vp, i]),
        "lbm_get_launch_config": (i, [vp, pi]),
        "lbm_get_wave_columns": (i, [vp]),
        "lbm_workspace_bytes_inplace": (sz, [i, i, i]),
        "lbm_workspace_bytes_inplace_blocked": (sz, [i, i, i, i, i]),
        "lbm_create_inplace": (i, [i, i, i, vp, sz, vp, ctypes.POINTER(vp)]),
        "lbm_last_error": (ctypes.c_char_p, [vp]),
        "lbm_batch_slot_bytes": (sz, [i, i, i, i]),
        "lbm_batch_create": (i, [i, vp, sz, vp, ctypes.POINTER(vp)]),
        "lbm_batch_destroy": (i, [vp]),
        "lbm_batch_add": (i, [vp, i, i, i, i, d, d, vp, vp, pi]),
        "lbm_batch_remove": (i, [vp, i]),
        "lbm_batch_step": (i, [vp, ll, i]),
        "lbm_batch_residuals": (i, [vp, pd, pll]),
        "lbm_batch_diverged": (i, [vp, pi]),
        "lbm_batch_set_divergence_guard": (i, [vp, i]),
        "lbm_batch_force_warnings": (i, [vp, i]),
        "lbm_batch_promote": (i, [vp, i]),
        "lbm_batch_get_displacement": (i, [vp, i, vp, vp]),
        "lbm_batch_set_tile": (i, [vp, i, i, i]),
        "lbm_batch_info": (i, [vp, pi, ctypes.POINTER(sz), ctypes.POINTER(sz)]),
        "lbm_batch_set_time_blocking": (i, [vp, i]),
        "lbm_batch_set_time_blocking_for": (i, [vp, i, i]),
        "lbm_batch_set_wavefront_sites": (i, [vp, i, ll]),
        "lbm_batch_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return [n for n in dir(load()) if n.startswith("lbm_")]


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev_f64(t: torch.Tensor, shape, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
        raise ValueError(f"{name}: need a contiguous float64 CUDA tensor of shape {shape}")
    return t


def _aligned_buffer(nbytes: int, device) -> Tuple[torch.Tensor, int]:
    buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    addr = buf.data_ptr()
    return buf, (addr + 255) // 256 * 256


def error_norms_noalloc(ux: torch.Tensor, uy: torch.Tensor, ux_ref: torch.Tensor,
                       uy_ref: torch.Tensor, out: torch.Tensor) -> None:
    """lbm_error_norms_noalloc: out (4 float64 on the device) = sum |e|^2,
    sum |ref|^2, max |e|, max |ref| with e = u - ref, enqueued on the current
    stream; allocates nothing."""
    lib = load()
    ny, nx = ux.shape
    fields = [_dev_f64(t, (ny, nx), n) for t, n in
              ((ux, "ux"), (uy, "uy"), (ux_ref, "ux_ref"), (uy_ref, "uy_ref"))]
    out = _dev_f64(out, (4,), "out")
    rc = lib.lbm_error_norms_noalloc(nx, ny, *[ctypes.c_void_p(t.data_ptr()) for t in fields],
                                     ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(_stream_ptr(out.device)))
    if rc != 0:
        raise LbmError(rc, lib.lbm_last_error(None).decode())


def leading_error_constants(lame_lambda: float, lame_mu: float, theta: float = 1.0 / 3.0,
                            w12: float = 1.0, w21: float = 1.0, w22: float = 1.0) -> dict:
    """lbm_leading_error_constants (host only): C1..C5, D1..D3 of the x row and
    the error estimates R1, R2."""
    lib = load()
    out = (ctypes.c_double * 10)()
    rc = lib.lbm_leading_error_constants(float(lame_lambda), float(lame_mu), float(theta),
                                         float(w12), float(w21), float(w22), out)
    if rc != 0:
        raise LbmError(rc, "leading_error_constants: inadmissible material or rates")
    keys = ["C1", "C2", "C3", "C4", "C5", "D1", "D2", "D3", "R1", "R2"]
    return dict(zip(keys, list(out)))


def fourth_order_rates(lame_lambda: float, lame_mu: float, theta: float = 1.0 / 3.0):
    """lbm_fourth_order_rates (host only): (omega_12 = omega_21, omega_22)."""
    lib = load()
    out = (ctypes.c_double * 2)()
    rc = lib.lbm_fourth_order_rates(float(lame_lambda), float(lame_mu), float(theta), out)
    if rc != 0:
        raise LbmError(rc, "fourth_order_rates: no admissible rates for this material")
    return out[0], out[1]


class Solver:
    """One periodic nx x ny lattice (lbm_create ... lbm_destroy); with
    inplace=True, one population buffer with in-place streaming
    (lbm_create_inplace), with room for launches of up to `inplace_steps`
    steps with segments of `inplace_segment_rows` rows (0: the default)
    (lbm_workspace_bytes_inplace_blocked; inplace_steps=1: the minimal
    workspace, one step per launch)."""

    def __init__(self, nx: int, ny: int, precision: str = "fp64", with_polish: bool = False,
                 device: str = "cuda", inplace: bool = False, inplace_steps: int = 8,
                 inplace_segment_rows: int = 0):
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library cannot run")
        self.nx, self.ny = int(nx), int(ny)
        self.device = torch.device(device)
        self.precision = PRECISIONS[precision]
        self.inplace = bool(inplace)
        if self.inplace and with_polish:
            raise ValueError("in-place streaming has no polish phase")
        if self.inplace and int(inplace_steps) >= 2:
            nbytes = self.lib.lbm_workspace_bytes_inplace_blocked(
                self.nx, self.ny, self.precision, int(inplace_steps), int(inplace_segment_rows))
        elif self.inplace:
            nbytes = self.lib.lbm_workspace_bytes_inplace(self.nx, self.ny, self.precision)
        else:
            nbytes = self.lib.lbm_workspace_bytes(self.nx, self.ny, self.precision,
                                                  int(with_polish))
        if nbytes == 0:
            raise ValueError("invalid lattice size or precision")
        self._ws, self._ws_ptr = _aligned_buffer(nbytes, self.device)
        self._nbytes = nbytes
        h = ctypes.c_void_p()
        stream = ctypes.c_void_p(_stream_ptr(self.device))
        if self.inplace:
            rc = self.lib.lbm_create_inplace(self.nx, self.ny, self.precision,
                                             ctypes.c_void_p(self._ws_ptr), nbytes, stream,
                                             ctypes.byref(h))
        else:
            rc = self.lib.lbm_create(self.nx, self.ny, self.precision, int(with_polish),
                                     ctypes.c_void_p(self._ws_ptr), nbytes, stream,
                                     ctypes.byref(h))
        if rc != 0:
            raise LbmError(rc, self.lib.lbm_last_error(None).decode())
        self.h = h
        self._keep = []

    # -- plumbing -----------------------------------------------------------
    def _check(self, rc: int, allow=(0,)) -> int:
        if rc in allow:
            return rc
        msg = self.lib.lbm_last_error(self.h).decode()
        if rc == -5:
            raise Diverged(rc, msg)
        raise LbmError(rc, msg)

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def workspace_bytes(self) -> int:
        return self._nbytes

    # -- API ----------------------------------------------------------------
    def set_material(self, lame_lambda: float, lame_mu: float, check_stability: bool = False):
        """Lattice Lame parameters.  With check_stability, refuse materials whose
        amplification matrix has spectral radius > 1 (Sec. 5): on this lattice's
        own wavevectors for small lattices, on the paper's k-grid otherwise."""
        if check_stability:
            from . import stability
            small = self.nx * self.ny <= 65536
            if not stability.is_stable(lame_lambda, lame_mu,
                                       nx=self.nx if small else None,
                                       ny=self.ny if small else None):
                raise ValueError("material is linearly unstable for this scheme "
                                 "(sup_k rho(L(k)) > 1)")
        self._check(self.lib.lbm_set_material(self.h, float(lame_lambda), float(lame_mu)))

    def set_rates(self, theta: float, w12: float = 1.0, w21: float = 1.0, w22: float = 1.0):
        self._check(self.lib.lbm_set_rates(self.h, theta, w12, w21, w22))

    def set_body_force(self, gx: torch.Tensor, gy: torch.Tensor) -> int:
        """Returns the warning bits of lbm_set_body_force (W_MEAN_REMOVED,
        W_STAGGERED_LOAD) or 0."""
        shp = (self.ny, self.nx)
        gx = _dev_f64(gx, shp, "gx")
        gy = _dev_f64(gy, shp, "gy")
        self._keep = [gx, gy]
        return self._check(self.lib.lbm_set_body_force(self.h, ctypes.c_void_p(gx.data_ptr()),
                                                       ctypes.c_void_p(gy.data_ptr())),
                           allow=FORCE_WARNINGS)

    def set_body_force_corrected(self, gx: torch.Tensor, gy: torch.Tensor,
                                 d2g: Optional[torch.Tensor] = None) -> int:
        """lbm_set_body_force_corrected: the force with the leading-order
        correction of the improved scheme; d2g (6, ny, nx) float64 holds the
        planes d_xx gx, d_xy gx, d_yy gx, d_xx gy, d_xy gy, d_yy gy, or None for
        central differences on the lattice.  Returns the warning bits."""
        shp = (self.ny, self.nx)
        gx = _dev_f64(gx, shp, "gx")
        gy = _dev_f64(gy, shp, "gy")
        ptr = None
        if d2g is not None:
            d2g = _dev_f64(d2g, (6,) + shp, "d2g")
            ptr = ctypes.c_void_p(d2g.data_ptr())
        self._keep = [gx, gy, d2g]
        return self._check(self.lib.lbm_set_body_force_corrected(
            self.h, ctypes.c_void_p(gx.data_ptr()), ctypes.c_void_p(gy.data_ptr()), ptr),
            allow=FORCE_WARNINGS)

    def reset(self):
        self._check(self.lib.lbm_reset(self.h))

    def step(self, nsteps: int):
        self._check(self.lib.lbm_step(self.h, int(nsteps)))

    def step_checked(self, nsteps: int) -> float:
        """Advance nsteps >= 2 steps; returns the residual r(n - 1) of the last
        two steps' displacements (see lbm_step_checked)."""
        r = ctypes.c_double(0.0)
        self._check(self.lib.lbm_step_checked(self.h, int(nsteps), ctypes.byref(r)))
        return r.value

    def solve_to_tol(self, tol: float, max_steps: int, check_every: int = 1):
        """Returns (steps_done, residual, status) with status 0 converged, 1 not."""
        n = ctypes.c_longlong(0)
        r = ctypes.c_double(0.0)
        rc = self._check(self.lib.lbm_solve_to_tol(self.h, float(tol), int(max_steps),
                                                   int(check_every), ctypes.byref(n),
                                                   ctypes.byref(r)), allow=(0, 1))
        return n.value, r.value, rc

    def set_polish(self, r_switch: float):
        self._check(self.lib.lbm_set_polish(self.h, float(r_switch)))

    def set_divergence_guard(self, checks: int):
        """Rises of the update norm in a row that stop solve_to_tol (0: off);
        see lbm_set_divergence_guard."""
        self._check(self.lib.lbm_set_divergence_guard(self.h, int(checks)))

    def set_small_solve(self, steps_per_launch: int):
        """Steps per launch of the one-workgroup solve of small lattices in
        solve_to_tol (0: off); see lbm_set_small_solve."""
        self._check(self.lib.lbm_set_small_solve(self.h, int(steps_per_launch)))

    @property
    def current_precision(self) -> int:
        return self.lib.lbm_current_precision(self.h)

    @property
    def steps_done(self) -> int:
        return self.lib.lbm_steps_done(self.h)

    def set_tile(self, bx_log2: int, rows_per_thread: int, blocks_per_cu: int = 0):
        self._check(self.lib.lbm_set_tile(self.h, int(bx_log2), int(rows_per_thread),
                                          int(blocks_per_cu)))

    def set_time_blocking(self, steps_per_launch: int):
        self._check(self.lib.lbm_set_time_blocking(self.h, int(steps_per_launch)))

    def launch_config(self) -> dict:
        """Steps per launch, fused kernel ("tile", "wavefront" or "single"),
        its rows (tile rows, segment rows, or rows per thread) and threads per
        workgroup; see lbm_get_launch_config."""
        out = (ctypes.c_int * 4)()
        self._check(self.lib.lbm_get_launch_config(self.h, out))
        kind = {0: "tile", 1: "wavefront"}.get(out[1], "single")
        cfg = {"steps_per_launch": out[0], "kernel": kind, "rows": out[2], "threads": out[3]}
        if kind == "wavefront":
            cfg["columns_per_lane"] = self.lib.lbm_get_wave_columns(self.h)
        return cfg

    def set_tile_rows(self, rows: int):
        """Tile height of the LDS tile kernel (0: default); see lbm_set_tile_rows."""
        self._check(self.lib.lbm_set_tile_rows(self.h, int(rows)))

    def set_stochastic_rounding(self, on: bool = True, seed: int = 0):
        """lbm_set_stochastic_rounding (half storage only)."""
        self._check(self.lib.lbm_set_stochastic_rounding(self.h, 1 if on else 0, int(seed) & 0xffffffff))

    def set_fused_kernel(self, kind: str, segment_rows: int = 256):
        """kind "tile" (LDS tile kernel) or "wavefront" (register wavefront with
        segments of `segment_rows` rows); see lbm_set_fused_kernel."""
        k = {"tile": 0, "wavefront": 1}[kind]
        self._check(self.lib.lbm_set_fused_kernel(self.h, k, int(segment_rows)))

    def displacement(self, out: Optional[Tuple[torch.Tensor, torch.Tensor]] = None):
        shp = (self.ny, self.nx)
        if out is None:
            out = (torch.empty(shp, dtype=torch.float64, device=self.device),
                   torch.empty(shp, dtype=torch.float64, device=self.device))
        ux, uy = (_dev_f64(t, shp, "u") for t in out)
        self._check(self.lib.lbm_get_displacement(self.h, ctypes.c_void_p(ux.data_ptr()),
                                                  ctypes.c_void_p(uy.data_ptr())))
        return ux, uy

    def stress(self):
        shp = (self.ny, self.nx)
        outs = [torch.empty(shp, dtype=torch.float64, device=self.device) for _ in range(3)]
        self._check(self.lib.lbm_get_stress(self.h, *[ctypes.c_void_p(t.data_ptr()) for t in outs]))
        return tuple(outs)

    def error_norms(self, ux_ref: torch.Tensor, uy_ref: torch.Tensor) -> dict:
        """Sums of Sec. 7.1 grid norms against a reference field (FP64, on device)."""
        shp = (self.ny, self.nx)
        ux_ref = _dev_f64(ux_ref, shp, "ux_ref")
        uy_ref = _dev_f64(uy_ref, shp, "uy_ref")
        out = (ctypes.c_double * 4)()
        self._check(self.lib.lbm_error_norms(self.h, ctypes.c_void_p(ux_ref.data_ptr()),
                                             ctypes.c_void_p(uy_ref.data_ptr()), out))
        e2, r2, emax, rmax = list(out)
        return {"sum_e2": e2, "sum_ref2": r2, "max_e": emax, "max_ref": rmax,
                "rel_l2": math.sqrt(e2 / r2) if r2 > 0 else float("nan"),
                "rel_linf": emax / rmax if rmax > 0 else float("nan")}

    def populations(self) -> torch.Tensor:
        f = torch.empty((8, self.ny, self.nx), dtype=torch.float64, device=self.device)
        self._check(self.lib.lbm_get_populations(self.h, ctypes.c_void_p(f.data_ptr())))
        return f

    def set_populations(self, f: torch.Tensor):
        f = _dev_f64(f, (8, self.ny, self.nx), "f")
        self._keep.append(f)
        self._check(self.lib.lbm_set_populations(self.h, ctypes.c_void_p(f.data_ptr())))

    def stream_only(self, nsteps: int):
        self._check(self.lib.lbm_debug_stream_only(self.h, int(nsteps)))


class Batch:
    """Many lattices in one arena stepped by one persistent launch per step."""

    def __init__(self, max_slots: int, arena_bytes: int, device: str = "cuda"):
        self.lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HIP library cannot run")
        self.device = torch.device(device)
        self.max_slots = int(max_slots)
        self._arena, ptr = _aligned_buffer(int(arena_bytes), self.device)
        self._stream = torch.cuda.current_stream(self.device)  # the batch's launches run here
        h = ctypes.c_void_p()
        rc = self.lib.lbm_batch_create(self.max_slots, ctypes.c_void_p(ptr), int(arena_bytes),
                                       ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise LbmError(rc, self.lib.lbm_batch_last_error(None).decode())
        self.h = h
        self.shapes = {}
        self._keep = {}

    def _check(self, rc: int, allow=(0,)) -> int:
        if rc in allow:
            return rc
        raise LbmError(rc, self.lib.lbm_batch_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.lbm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def slot_bytes(nx: int, ny: int, precision: str = "fp32", with_polish: bool = False) -> int:
        return load().lbm_batch_slot_bytes(nx, ny, PRECISIONS[precision], int(with_polish))

    def add(self, nx: int, ny: int, lame_lambda: float, lame_mu: float, gx: torch.Tensor,
            gy: torch.Tensor, precision: str = "fp32", with_polish: bool = False) -> Optional[int]:
        """Returns the slot id, or None if the arena has no room."""
        gx = _dev_f64(gx, (ny, nx), "gx")
        gy = _dev_f64(gy, (ny, nx), "gy")
        slot = ctypes.c_int(-1)
        rc = self.lib.lbm_batch_add(self.h, nx, ny, PRECISIONS[precision], int(with_polish),
                                    float(lame_lambda), float(lame_mu),
                                    ctypes.c_void_p(gx.data_ptr()), ctypes.c_void_p(gy.data_ptr()),
                                    ctypes.byref(slot))
        if rc == -3:
            return None
        self._check(rc)
        self.shapes[slot.value] = (ny, nx)
        self._keep[slot.value] = (gx, gy)
        return slot.value

    def remove(self, slot: int):
        self._check(self.lib.lbm_batch_remove(self.h, int(slot)))
        self.shapes.pop(slot, None)
        self._keep.pop(slot, None)

    def step(self, nsteps: int, check: bool = False):
        self._check(self.lib.lbm_batch_step(self.h, int(nsteps), int(check)))

    def residuals(self):
        r = (ctypes.c_double * self.max_slots)()
        n = (ctypes.c_longlong * self.max_slots)()
        self._check(self.lib.lbm_batch_residuals(self.h, r, n))
        return list(r), list(n)

    def diverged(self):
        """Per slot: True once its residual, over the checks read by
        residuals(), became non-finite or its update norm kept rising
        (lbm_batch_diverged)."""
        f = (ctypes.c_int * self.max_slots)()
        self._check(self.lib.lbm_batch_diverged(self.h, f))
        return [bool(v) for v in f]

    def set_divergence_guard(self, checks: int):
        self._check(self.lib.lbm_batch_set_divergence_guard(self.h, int(checks)))

    def force_warnings(self, slot: int) -> int:
        """Warning bits of a slot's force (lbm_batch_force_warnings)."""
        rc = self.lib.lbm_batch_force_warnings(self.h, int(slot))
        if rc < 0:
            self._check(rc)
        return rc

    def promote(self, slot: int):
        self._check(self.lib.lbm_batch_promote(self.h, int(slot)))

    def set_tile(self, bx_log2: int, rows_per_thread: int, blocks_per_cu: int = 0):
        self._check(self.lib.lbm_batch_set_tile(self.h, int(bx_log2), int(rows_per_thread),
                                                int(blocks_per_cu)))

    def set_time_blocking(self, steps_per_launch: int, precision: Optional[str] = None):
        """Steps per launch (1..8) for every storage type, or for `precision` only."""
        if precision is None:
            self._check(self.lib.lbm_batch_set_time_blocking(self.h, int(steps_per_launch)))
        else:
            self._check(self.lib.lbm_batch_set_time_blocking_for(
                self.h, PRECISIONS[precision], int(steps_per_launch)))

    def set_wavefront_sites(self, precision: str, min_sites: int):
        """Lattices of `precision` with at least `min_sites` sites (0: all) take
        their plain fused steps through the wavefront list; -1: the default
        rule (the lattices a single solver steps through the wavefront)."""
        self._check(self.lib.lbm_batch_set_wavefront_sites(self.h, PRECISIONS[precision],
                                                           int(min_sites)))

    def displacements(self, slots):
        """Displacements of several lattices as host arrays [(ux, uy), ...]:
        one device buffer, one copy to page-locked host memory."""
        slots = list(slots)
        if not slots:
            return []
        sizes = [self.shapes[sl][0] * self.shapes[sl][1] for sl in slots]
        buf = torch.empty(2 * sum(sizes), dtype=torch.float64, device=self.device)
        off = 0
        base = buf.data_ptr()
        for sl, n in zip(slots, sizes):
            self._check(self.lib.lbm_batch_get_displacement(
                self.h, int(sl), ctypes.c_void_p(base + 8 * off),
                ctypes.c_void_p(base + 8 * (off + n))))
            off += 2 * n
        # page-locked host memory (torch's caching host allocator): the copy runs
        # at link speed instead of through a pageable staging buffer
        pinned = torch.empty(buf.numel(), dtype=torch.float64, pin_memory=True)
        with torch.cuda.stream(self._stream):
            pinned.copy_(buf, non_blocking=True)
        self._stream.synchronize()  # the extractions and the copy
        host = pinned.numpy()
        out, off = [], 0
        for sl, n in zip(slots, sizes):
            shp = self.shapes[sl]
            out.append((host[off:off + n].reshape(shp), host[off + n:off + 2 * n].reshape(shp)))
            off += 2 * n
        return out

    def displacement(self, slot: int):
        shp = self.shapes[slot]
        ux = torch.empty(shp, dtype=torch.float64, device=self.device)
        uy = torch.empty(shp, dtype=torch.float64, device=self.device)
        self._check(self.lib.lbm_batch_get_displacement(self.h, int(slot),
                                                        ctypes.c_void_p(ux.data_ptr()),
                                                        ctypes.c_void_p(uy.data_ptr())))
        return ux, uy

    def info(self):
        a = ctypes.c_int(0)
        u = ctypes.c_size_t(0)
        f = ctypes.c_size_t(0)
        self._check(self.lib.lbm_batch_info(self.h, ctypes.byref(a), ctypes.byref(u), ctypes.byref(f)))
        return a.value, u.value, f.value
