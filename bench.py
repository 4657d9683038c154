"""Benchmark of the lattice Boltzmann elasticity hot path on one MI355X.

Default workload (the configuration the headline metric is quoted on): a
single periodic 1024 x 1024 lattice, Poisson ratio sweep {0.1, 0.3, 0.45,
0.49} x manufactured sinusoidal load with wavenumbers (1,1) and (4,3), mu = 1,
FP32 population storage (FP64 storage timed the same way for comparison).
One benchmark "step" = one chunk of `--chunk` pseudo-time steps (default
1000) on each of the 8 lattices, ending with the FP64 steady-state residual,
the displacement extraction and the FP64 error norms against the
manufactured solution; the default 20 steps make the 20k pseudo-time steps of
the configuration.  `value` is whole-job MLUPS (site updates per second).

Also reported on the same JSON line:
  roofline      -- dominant kernel of the headline run (the fused tile
                   kernel, several steps per launch).  A launch moves each
                   site's populations and force through HBM once, whatever
                   the number of fused steps: its minimum bytes are 72 B per
                   site (FP32: 8 populations read and written, 2 force values
                   read).  achieved = minimum bytes per launch / average launch
                   duration (HIP events on the library's stream), frac =
                   achieved / 8 TB/s; traffic (and traffic_frac) = the HBM bytes
                   per launch of the committed rocprofv3 counters; valu_frac =
                   the committed VALU instruction count x 64 lanes / duration /
                   the chip's VALU issue rate; effective_gbs = the one-step byte
                   model (72 B per site-update x steps per launch), which passes
                   8 TB/s because the populations cross HBM once per launch;
  fp64          -- the same workload with FP64 storage;
  large_8192    -- 8192 x 8192 FP64 / FP32 / scaled-FP16 step throughput (the
                   working set exceeds the 256 MB last-level cache) and the
                   reduced-precision displacement error on a 256^2 downsample;
  batch         -- 512 uneven lattices in one launch per step; solves/s;
  serving       -- Poisson arrivals, continuous batching, p50/p99 latency;
  cpu_baseline  -- the FP64 CPU oracle on a bounded sample of the workload.
Inputs are seeded and synthetic (no dataset is involved).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_SITE = {"fp64": 144, "fp32": 72, "fp16": 40}  # 8 pops in + 8 out + 2 force
# VALU issue rate of MI355X in lane-instructions per second: 256 compute units x
# 4 SIMDs, each issuing a wave64 VALU instruction over 4 cycles on 16 lanes, at
# 2.4 GHz (packed FP32 is not used)
PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9


# the headers that define each fused kernel family
TRAFFIC_SOURCES = {"tile": ("lbm_common.hpp", "lbm_fused.hpp"),
                   "wave": ("lbm_common.hpp", "lbm_wave.hpp")}


def kernel_family(kernel: str) -> str:
    return "wave" if "k_wave" in kernel else "tile"


def kernel_source_hash(family: str = "tile") -> str:
    """sha256 of a fused kernel family's headers with comments and whitespace
    removed (the code the counters were taken with)."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2208_14870_amd", "csrc")
    for f in TRAFFIC_SOURCES[family]:
        text = open(os.path.join(csrc, f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_counters(name, kernel=None):
    """The committed counter record profiles/<name>.json (HBM bytes per launch
    from FETCH_SIZE / WRITE_SIZE scaled by a 1 GiB copy, VALU instructions per
    launch), or None when the kernel's code changed since the counters were
    taken or the profiled kernel (template arguments included) is not
    `kernel`."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if kernel_source_hash(kernel_family(rec.get("kernel", ""))) != rec.get("source_sha256"):
        return None
    if kernel is not None and kernel not in rec.get("kernel", ""):
        return None
    return rec


def roofline(prec, sites, avg_launch_us, steps_per_launch, kernel, counters=None, note=""):
    """Roofline fields of one fused launch over `sites` sites (see the module
    docstring): minimum HBM bytes per launch against 8 TB/s, and the committed
    counters' traffic and VALU issue against their ceilings."""
    t = avg_launch_us * 1e-6
    min_bytes = BYTES_PER_SITE[prec] * sites
    achieved = min_bytes / t / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "traffic_frac": None,
           "valu_frac": None, "min_bytes_per_launch": min_bytes,
           "site_updates_per_launch": sites * steps_per_launch,
           "effective_gbs": round(BYTES_PER_SITE[prec] * sites * steps_per_launch / t / 1e9, 1),
           "avg_launch_us": round(avg_launch_us, 3), "steps_per_launch": steps_per_launch,
           "kernel": kernel}
    rec = measured_counters(counters, kernel.split(" (")[0]) if counters else None
    if rec:
        tr = rec.get("traffic_bytes_per_launch")
        if tr:
            out["traffic"] = round(tr)
            out["traffic_frac"] = round(tr / t / (PEAK_HBM_GBS * 1e9), 4)
            out["traffic_over_min"] = round(tr / min_bytes, 3)
        valu = rec.get("valu_insts_per_launch")
        if valu:
            out["valu_frac"] = round(64 * valu / t / PEAK_VALU_LANE_OPS, 4)
            out["valu_lane_insts_per_update"] = round(64 * valu / (sites * steps_per_launch), 2)
        out["counters"] = "profiles/" + counters + ".json"
    if note:
        out["note"] = note
    return out


def calib_copy():
    """One device copy of 1 GiB: the calibration kernel for the HBM byte counters."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def copy_bandwidth(gib: int = 2, reps: int = 10) -> dict:
    """Practical HBM ceiling: a plain device copy of `gib` GiB (read + write
    bytes per second, best of `reps`, HIP events)."""
    import torch
    n = (gib << 30) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    gbs = 2 * (gib << 30) / (best * 1e-3) / 1e9
    return {"gbs": round(gbs, 1), "frac_of_peak": round(gbs / PEAK_HBM_GBS, 4),
            "bytes": 2 * (gib << 30), "note": "torch device copy (read + write), best of "
                                              f"{reps}; the practical HBM ceiling beside the "
                                              "8 TB/s datasheet peak"}


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="chunks of --chunk pseudo-time steps")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chunk", type=int, default=1000)
    ap.add_argument("--cases", type=int, default=8, help="how many of the 8 (nu, k) cases")
    ap.add_argument("--no-extras", action="store_true", help="headline FP32 run only")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB device copy (counter calibration)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-oracle-large", action="store_true",
                    help="only time the CPU oracle on the 8192^2 load (20 steps, extrapolated) "
                         "and on lattices sampled from the 512-lattice workload")
    ap.add_argument("--cpu-oracle-only", action="store_true",
                    help="time the CPU oracle only (no GPU) and print its JSON")
    ap.add_argument("--large-only", default="",
                    help="comma list of precisions: run only the 8192^2 leg (for profiling)")
    ap.add_argument("--inplace-only", action="store_true",
                    help="run only the in-place vs two-buffer leg (for profiling)")
    ap.add_argument("--batch-only", default="",
                    help="comma list of precisions: run only the 512-lattice batch leg "
                         "(for profiling)")
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--comparator-only", action="store_true",
                    help="run only the FP64-storage comparator of the headline workload "
                         "(for profiling)")
    ap.add_argument("--accuracy-only", action="store_true",
                    help="only the three convergence studies of the paper (FP64 solves)")
    ap.add_argument("--small-only", action="store_true",
                    help="run only the 32 x 32 launch-bound solve leg")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the two serving legs (overloaded, then sustained)")
    ap.add_argument("--headline-kernel", choices=("default", "tile"), default="default",
                    help="fused kernel of the 1024^2 FP32 headline: the library's default "
                         "(the register wavefront) or the LDS tile kernel, for comparison")
    ap.add_argument("--large-steps", type=int, default=10000)
    ap.add_argument("--large-warm", type=int, default=200)
    ap.add_argument("--large-tb", type=int, default=0,
                    help="steps per launch of the 8192^2 runs (0: library default, "
                         "the register wavefront at eight steps; the default kernel is "
                         "kept at other depths)")
    return ap.parse_args()


def build_cases(ncases):
    from paper_2208_14870_amd import problem as P
    return [P.single_1024(nu, kx, ky) for nu, (kx, ky) in P.SWEEP_1024[:ncases]]


def make_solvers(cases, prec, kernel="default"):
    """Solvers of the cases with their loads; kernel "tile" forces the LDS tile
    kernel for plain fused steps (at the default depth), "default" keeps the
    library's choice."""
    import torch
    from paper_2208_14870_amd import lbm
    out = []
    for c in cases:
        s = lbm.Solver(c.nx, c.ny, prec)
        if kernel == "tile":
            s.set_fused_kernel("tile")
        s.set_material(c.material.lame_lambda, c.material.lame_mu)
        s.set_body_force(torch.from_numpy(c.gx).cuda(), torch.from_numpy(c.gy).cuda())
        ex = (torch.from_numpy(c.ux_exact).cuda(), torch.from_numpy(c.uy_exact).cuda())
        out.append((s, ex))
    return out


def kernel_label(cfg, ctype, sites, sr=False):
    """Name (with its full template arguments, as the profiler names it) and
    algorithmic traffic of the plain-step kernel of a launch config."""
    tb, rows, nt = cfg["steps_per_launch"], cfg["rows"], cfg["threads"]
    per_site = {"double": 144, "float": 72, "__half": 40}[ctype]
    side = int(round(math.sqrt(sites)))
    srs = "true" if sr else "false"
    if cfg["kernel"] == "tile":  # type, tile rows, steps, threads, plain mode, rounding
        return (f"k_stepN<{ctype}, {rows}, {tb}, {nt}, 0, {srs}> (LDS tile 64 x {rows} + ring "
                f"{tb - 1}, {nt} threads): {tb} fused steps per launch, {per_site} B per "
                f"site-update algorithmic, {tb} x {side}^2 site-updates per launch")
    if cfg["kernel"] == "wavefront":  # type, steps, columns per lane, rounding, in place, work list
        v = cfg.get("columns_per_lane", 1)
        return (f"k_wave<{ctype}, {tb}, {v}, {srs}, false, false> (register wavefront, {rows}-row "
                f"segments): {tb} fused steps per launch, "
                f"{per_site} B per site-update algorithmic, {tb} x {side}^2 site-updates per launch")
    return f"k_step<{ctype}, ...>: one step per launch, {per_site} B per site-update algorithmic"


def run_workload(solvers, nchunks, chunk):
    """nchunks x (chunk steps per lattice: plain steps, then one launch whose
    last two steps form the residual check, then displacement + error norms).
    The plain steps run as fused launches (timed with HIP events on the
    library's stream) and the remainder that does not fill a launch.  Returns
    timing and last metrics."""
    import torch
    ev = []
    last = []
    history = []  # residual of the first case after every chunk
    tb = solvers[0][0].launch_config()["steps_per_launch"]
    checked = max(2, tb)  # the chunk's last launch carries the residual check
    per = chunk - checked
    fused, rest = per - per % tb, per % tb
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nchunks):
        for i, (s, (ux, uy)) in enumerate(solvers):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            s.step(fused)
            e1.record()
            ev.append((e0, e1))
            if rest:
                s.step(rest)
            r = s.step_checked(checked)  # residual of the chunk's last two steps
            err = s.error_norms(ux, uy)  # displacement extraction + FP64 norms
            last.append((r, err["rel_l2"], err["rel_linf"]))
            if i == 0:
                history.append(r)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plain_ms = sum(a.elapsed_time(b) for a, b in ev)
    return {"wall_s": wall, "plain_kernel_avg_us": 1e3 * plain_ms / (len(ev) * (fused // tb)),
            "plain_us_per_step": 1e3 * plain_ms / (len(ev) * fused),
            "steps_per_launch": tb, "launch_config": solvers[0][0].launch_config(),
            "last": last[-len(solvers):], "history": history}


def stress_error(solver, case):
    """Stress of the solver's current state (lbm_get_stress, lattice units)
    against the continuum stress of the case's manufactured solution: (relative
    L2 over the three components with sxy counted twice, max |e| / max |exact|)."""
    import numpy as np
    from paper_2208_14870_amd import problem as P
    got = [t.cpu().numpy() for t in solver.stress()]
    want = P.stress_of(case.u_field, case.material, case.nx, case.ny)
    wts = (1.0, 1.0, 2.0)
    num = sum(w * float(np.sum((a - b) ** 2)) for w, a, b in zip(wts, got, want))
    den = sum(w * float(np.sum(b ** 2)) for w, b in zip(wts, want))
    linf = max(float(np.max(np.abs(a - b))) for a, b in zip(got, want))
    return math.sqrt(num / den), linf / max(float(np.max(np.abs(b))) for b in want)


def accuracy_studies(sizes=(20, 40, 80, 160), tol=1e-12, tol_fourth=1e-14):
    """The paper's three convergence studies solved on the GPU in FP64 to
    r <= tol (a check every 100 steps): the standard scheme (Sec. 7.3.1,
    nu = 0.8, E = 0.11), the improved scheme with the analytic force correction
    (Sec. 7.3.2, E = 0.085) and the special case with the fourth-order rates
    (Sec. 7.3.3).  Relative errors of displacement and stress against the
    manufactured solution (L2 ratio and max |e| / max |exact|) and the observed
    orders per halving.  The fourth-order study solves to tol_fourth: its error at
    160 nodes (~5e-8) is below what r <= 1e-12 leaves (r / (mu k^2) ~ 3e-8)."""
    import numpy as np
    import torch
    from paper_2208_14870_amd import lbm, problem as P
    out = {}
    for name, make in (("standard_e1", P.paper_e1), ("improved_e2", P.paper_e2),
                       ("fourth_order_e3", P.paper_e3)):
        rows = []
        for n in sizes:
            c = make(n)
            m = c.material
            s = lbm.Solver(n, n, "fp64")
            s.set_material(m.lame_lambda, m.lame_mu)
            dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
            if name == "standard_e1":
                s.set_body_force(dev(c.gx), dev(c.gy))
            else:
                if name == "fourth_order_e3":
                    w12, w22 = lbm.fourth_order_rates(m.lame_lambda, m.lame_mu)
                    s.set_rates(1.0 / 3.0, w12, w12, w22)
                s.set_body_force_corrected(dev(c.gx), dev(c.gy),
                                           dev(np.concatenate([c.d2gx, c.d2gy])))
            t0 = time.perf_counter()
            steps, r, st = s.solve_to_tol(tol_fourth if name == "fourth_order_e3" else tol,
                                          10 ** 7, 100)
            wall = time.perf_counter() - t0
            ux, uy = (t.cpu().numpy() for t in s.displacement())
            num = float(np.sum((ux - c.ux_exact) ** 2 + (uy - c.uy_exact) ** 2))
            den = float(np.sum(c.ux_exact ** 2 + c.uy_exact ** 2))
            ref = max(float(np.max(np.abs(c.ux_exact))), float(np.max(np.abs(c.uy_exact))))
            dl2 = math.sqrt(num / den)
            dinf = max(float(np.max(np.abs(ux - c.ux_exact))),
                       float(np.max(np.abs(uy - c.uy_exact)))) / ref
            sl2, sinf = stress_error(s, c)
            s.close()
            rows.append({"n": n, "status": st, "steps": steps, "solve_s": round(wall, 3),
                         "disp_rel_l2": dl2, "disp_rel_linf": dinf,
                         "stress_rel_l2": sl2, "stress_rel_linf": sinf})
        for a, b in zip(rows, rows[1:]):
            b["orders"] = {k: round(math.log2(a[k] / b[k]), 3) for k in
                           ("disp_rel_l2", "disp_rel_linf", "stress_rel_l2", "stress_rel_linf")}
        out[name] = rows
    e1, e2 = out["standard_e1"], out["improved_e2"]
    out["improved_over_standard_disp_linf"] = [round(a["disp_rel_linf"] / b["disp_rel_linf"], 2)
                                               for a, b in zip(e1, e2)]
    return out


def small_32(reps: int = 20):
    """The 32 x 32 FP64 manufactured workload (nu = 0.3, mu = 1, mode (1, 1)) solved
    to r <= 1e-10 with a check every step: launch-bound (147 KB per step), so it is
    timed per solve and per step rather than against a roofline (its stop step and
    displacement against the oracle are the smoke check's and the tests').  It runs
    as one workgroup that keeps the state in LDS (lbm_set_small_solve)."""
    import numpy as np
    import torch
    from paper_2208_14870_amd import lbm, problem as P
    case = P.single_32()
    mat = case.material
    gx, gy = torch.from_numpy(case.gx).cuda(), torch.from_numpy(case.gy).cuda()
    s = lbm.Solver(32, 32, "fp64")
    s.set_material(mat.lame_lambda, mat.lame_mu)
    s.set_body_force(gx, gy)
    times, n, r = [], 0, 0.0
    for _ in range(reps + 1):
        s.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n, r, _ = s.solve_to_tol(1e-10, 10000, 1)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ux, uy = (t.cpu().numpy() for t in s.displacement())
    s.close()
    ex = np.sqrt(np.sum((ux - case.ux_exact) ** 2 + (uy - case.uy_exact) ** 2) /
                 np.sum(case.ux_exact ** 2 + case.uy_exact ** 2))
    med = sorted(times[1:])[len(times[1:]) // 2]
    return {"lattice": [32, 32], "storage": "fp64", "tol": 1e-10, "check_every": 1,
            "steps": int(n), "residual": r,
            "solve_ms_median": round(1e3 * med, 3), "us_per_step": round(1e6 * med / n, 2),
            "rel_l2_vs_manufactured": float(ex),
            "path": "one workgroup: state in LDS, residual and stop on the device",
            "note": "a check every step; launch-per-check solve: 2.19 ms (19.4 us per step)"}


def large_lattice(steps=10000, warm=200, precs=("fp64", "fp32", "fp16", "fp16sr"), tb=0):
    """8192 x 8192 random 16-mode load (seed 3): throughput per storage
    precision over `steps` timed steps after `warm` untimed ones, and the
    FP32 / scaled-FP16 displacement error against the FP64 run (the FP64 GPU
    path is checked against the oracle on sampled sites at this size) on the
    256 x 256 downsample (nodes 32i, 32j) after warm + steps steps from rest."""
    import torch
    from paper_2208_14870_amd import lbm, problem as P
    c = P.single_8192()
    gx = torch.from_numpy(c.gx).cuda()
    gy = torch.from_numpy(c.gy).cuda()
    mat = c.material
    del c
    sites = 8192 * 8192
    out, u = {}, {}
    for key in precs:
        prec = "fp16" if key == "fp16sr" else key
        s = lbm.Solver(8192, 8192, prec)
        s.set_material(mat.lame_lambda, mat.lame_mu)
        s.set_body_force(gx, gy)
        if key == "fp16sr":  # half storage with stochastic rounding
            s.set_stochastic_rounding(True, 0)
        if tb:
            s.set_time_blocking(tb)
        s.step(warm)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        s.step(steps)
        e1.record()
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / steps  # per step
        cfg = s.launch_config()
        ux, uy = s.displacement()
        u[key] = (ux[::32, ::32].clone(), uy[::32, ::32].clone())
        del ux, uy
        s.close()
        del s
        tbl = cfg["steps_per_launch"]
        launches = steps // tbl + (1 if steps % tbl else 0)
        ctype = {"fp64": "double", "fp32": "float", "fp16": "__half"}[prec]
        out[key] = {"mlups": round(sites / us, 1), "us_per_step": round(us, 2),
                    "launch_config": cfg,
                    "roofline": roofline(prec, sites, us * steps / launches, tbl,
                                         kernel_label(cfg, ctype, sites, key == "fp16sr"),
                                         (f"k_stepN_{prec}_8192_counters" if cfg["kernel"] == "tile"
                                          else f"k_wave_{prec}_8192_counters")
                                         if key == prec else None)}
        if key == "fp16sr":
            out[key]["rounding"] = "stochastic (13 random bits per stored population)"
    rx, ry = u.get("fp64", (None, None))
    den = float(torch.sum(rx ** 2) + torch.sum(ry ** 2)) if rx is not None else 0.0
    for prec in (p for p in ("fp32", "fp16", "fp16sr") if p in u and rx is not None):
        ax, ay = u[prec]
        num = float(torch.sum((ax - rx) ** 2) + torch.sum((ay - ry) ** 2))
        out[prec]["rel_l2_vs_fp64_downsample_256"] = math.sqrt(num / den)
    out["steps"] = steps
    out["warmup_steps"] = warm
    return out


def inplace_run(n=8192, steps=400, warm=8):
    """In-place streaming (one population buffer) against the two-buffer solver,
    8192 x 8192 random load: one step per launch both ways, then the default
    fused launches (two buffers) against blocked launches in place (the
    in-place wavefront with its halo copies, at eight and at four steps):
    GLUPS and workspace bytes."""
    import torch
    from paper_2208_14870_amd import lbm, problem as P
    c = P.single_8192() if n == 8192 else P.single_1024(0.3, 1, 1, n=n)
    gx = torch.from_numpy(c.gx).cuda()
    gy = torch.from_numpy(c.gy).cuda()
    out = {}
    runs = [("two_buffers", False, 1, 1), ("inplace", True, 1, 1),
            ("two_buffers_fused", False, 8, 0), ("inplace_blocked", True, 8, 8),
            ("inplace_blocked_4", True, 4, 4)]
    for prec in ("fp32", "fp64"):
        row = {}
        for name, inplace, room, tb in runs:
            s = lbm.Solver(n, n, prec, inplace=inplace, inplace_steps=room)
            if tb:
                s.set_time_blocking(tb)
            s.set_material(c.material.lame_lambda, c.material.lame_mu)
            s.set_body_force(gx, gy)
            s.step(warm)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            s.step(steps)
            e1.record()
            torch.cuda.synchronize()
            us = 1e3 * e0.elapsed_time(e1) / steps
            r = {"mlups": round(n * n / us, 1), "workspace_bytes": s.workspace_bytes,
                 "launch_config": s.launch_config()}
            if tb == 1:
                gbs = BYTES_PER_SITE[prec] * n * n / (us * 1e-6) / 1e9
                r.update(gbs=round(gbs, 1), frac=round(gbs / PEAK_HBM_GBS, 4))
            row[name] = r
            s.close()
            del s
        out[prec] = row
    out["lattice"] = [n, n]
    out["steps"] = steps
    return out


def sweep_batched(cases, nchunks: int, chunk: int, warm: int = 1):
    """The headline's 1024^2 sweep with its lattices advanced together: one
    batch (lbm_batch_*) holds every case, each chunk is one sequence of fused
    launches over all of them with the residual check at its end (per-lattice
    arithmetic identical to the solo solver: bit-identical, tested), then the
    residuals, each displacement and its FP64 error norms (library kernels), as
    the headline loop does per lattice.  Reported beside the single-lattice
    headline, not in its place."""
    import torch
    from paper_2208_14870_amd import lbm
    sites = sum(c.nx * c.ny for c in cases)
    arena = len(cases) * lbm.Batch.slot_bytes(1024, 1024, "fp32") + (1 << 28)
    b = lbm.Batch(len(cases), arena)
    exact, slots = [], []
    for c in cases:
        slots.append(b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu,
                           torch.from_numpy(c.gx).cuda(), torch.from_numpy(c.gy).cuda(), "fp32"))
        exact.append((torch.from_numpy(c.ux_exact).cuda(), torch.from_numpy(c.uy_exact).cuda()))
    norms = torch.zeros(len(cases), 4, dtype=torch.float64, device="cuda")

    def chunk_once():
        b.step(chunk, check=True)
        b.residuals()
        for i, sl in enumerate(slots):
            ux, uy = b.displacement(sl)
            lbm.error_norms_noalloc(ux, uy, exact[i][0], exact[i][1], norms[i])

    for _ in range(warm):
        chunk_once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nchunks):
        chunk_once()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nrm = norms.cpu().numpy()
    b.close()
    return {"mlups": round(sites * chunk * nchunks / wall / 1e6, 1), "lattices": len(cases),
            "steps_per_lattice": chunk * nchunks, "wall_s": round(wall, 3),
            "rel_l2_vs_manufactured": [round(math.sqrt(r[0] / r[1]), 6) for r in nrm]}


def batch_run(prec: str, nlat: int = 512, steps: int = 2000, chunk: int = 100):
    """Batched workload: `nlat` lattices (seed 4, sides {64..512}, nu ~ U[0.05, 0.48]),
    one launch per step over the tile work list, graph-replayed chunks with a
    residual check at the end of each chunk."""
    import torch
    from paper_2208_14870_amd import autotune, lbm, problem as P
    cases = P.batch_cases(nlat, seed=4)
    sites = sum(c.nx * c.ny for c in cases)
    arena = int(sites * lbm.Batch.slot_bytes(1024, 1024, prec) / (1024 * 1024) * 1.3) + (1 << 30)
    b = lbm.Batch(nlat + 8, arena)
    for c in cases:
        b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu,
              torch.from_numpy(c.gx).cuda(), torch.from_numpy(c.gy).cuda(), prec)
    shape = autotune.tune_batch(b, prec, sites)
    b.step(chunk, check=True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps // chunk):
        b.step(chunk, check=True)
        b.residuals()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n = steps // chunk * chunk
    us = 1e3 * e0.elapsed_time(e1) / n
    b.close()
    # population passes per chunk: fused launches of shape[3] steps (the last
    # carrying the residual check); approximate for the check's own split
    tb = max(1, int(shape[3])) if len(shape) > 3 else 1
    passes = math.ceil(chunk / tb)
    min_bytes = BYTES_PER_SITE[prec] * sites
    achieved = min_bytes * passes / chunk / (us * 1e-6) / 1e9
    return {"lattices": nlat, "sites": sites, "steps": n, "mlups": sites * n / wall / 1e6,
            "us_per_step": round(us, 2), "tile": list(shape),
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                         "min_bytes_per_pass": min_bytes, "passes_per_chunk": passes,
                         "effective_gbs": round(BYTES_PER_SITE[prec] * sites / (us * 1e-6) / 1e9, 1),
                         "note": f"{passes} population passes per {chunk}-step chunk "
                                 f"({tb} steps per fused launch); minimum bytes per pass = "
                                 f"{BYTES_PER_SITE[prec]} B per site"}}


def batch_solves(prec: str, nlat: int = 512, tol: float = 1e-6, chunk: int = 200,
                 fixed_steps=None, r_switch: float = 0.0):
    """Solve every lattice of the batched workload to r <= tol with per-lattice
    retirement (FP32 switches to FP64 only if its residual stalls); with
    `fixed_steps` each lattice stops after that many steps instead."""
    import torch
    from paper_2208_14870_amd import lbm, problem as P
    from paper_2208_14870_amd.serving import Server
    cases = P.batch_cases(nlat, seed=4)
    reqs = [P.Request(i, 0.0, c.nx, c.material.poisson, 0) for i, c in enumerate(cases)]
    sites = sum(c.nx * c.ny for c in cases)
    arena = int(sites * lbm.Batch.slot_bytes(1024, 1024, prec, True) / (1024 * 1024) * 1.3)
    srv = Server(arena + (1 << 30), max_slots=nlat + 8, chunk=chunk, tol=tol, r_switch=r_switch,
                 precision=prec, polish=(prec != "fp64"), keep_results=True)
    st = srv.run(reqs, 1.0, 600.0, cases={i: c for i, c in enumerate(cases)},
                 fixed_steps=fixed_steps)
    srv.close()
    res = {r.rid: r for r in srv.results}
    return st, res


def serving_run(rate: float = 2000.0, window: float = 1.0, budget: float = 20.0,
                policy: str = "fifo"):
    """Poisson arrivals (seed 5), sides log-uniform 64..2048, 8-mode loads, tol 1e-8,
    FP32 storage with FP64 polish, admission by arena footprint in the order of
    `policy` (arrival order, or highest response ratio next)."""
    import torch
    from paper_2208_14870_amd import problem as P
    from paper_2208_14870_amd.serving import Server
    reqs = P.request_stream(rate, window, seed=5)
    free, _ = torch.cuda.mem_get_info()
    arena = min(64 << 30, int(free * 0.5))
    srv = Server(arena, max_slots=4096, chunk=200, tol=1e-8, r_switch=1e-6, policy=policy)
    st = srv.run(reqs, window, budget)
    # steps to tolerance grow like n^2 (the slowest mode relaxes at ~mu (2 pi/n)^2
    # per step): c = median of steps / n^2 over the completed requests.  This errs
    # high (small lattices retire at whole chunks), which offsets the lower
    # throughput of a lightly loaded server (few resident lattices fill the GPU
    # less, and the FP64 polish of a large lattice dominates)
    fit = sorted(r.steps / float(r.n) ** 2 for r in srv.results)
    st["steps_per_n2"] = fit[len(fit) // 2] if fit else None
    srv.close()
    st["offered_rate_hz"] = rate
    st["admission_window_s"] = window
    st["arena_bytes"] = arena
    return st


def serving_legs():
    """The overloaded serving run (Poisson 2000 req/s for 1 s), then a run at
    0.8x the capacity estimated from work: site-updates per request ~ c n^4
    (steps to tolerance grow like n^2), with n = 64 * 32^U, U ~ U[0, 1), so
    E[n^4] = 64^4 (32^4 - 1) / (4 ln 32); capacity = GLUPS while busy / (c E[n^4]).
    The completion rate of the overloaded run would overstate it, since that
    run completes the small requests first.  Each run is made with admission
    in arrival order and with highest response ratio next, at the same rates."""
    log("serving: Poisson 2000 req/s, sides 64..2048, tol 1e-8 (arrival order)")
    sv = serving_run()
    e_n4 = 64.0 ** 4 * (32.0 ** 4 - 1.0) / (4.0 * math.log(32.0))
    if sv.get("steps_per_n2") and sv["mlups_while_busy"] > 0:
        capacity = sv["mlups_while_busy"] * 1e6 / (sv["steps_per_n2"] * e_n4)
    else:
        capacity = sv["solves_per_s"]
    sustain = max(0.05, 0.8 * capacity)
    log("serving: Poisson 2000 req/s (highest response ratio next)")
    sh = serving_run(policy="hrrn")
    log(f"serving at 0.8x the work-based capacity ({sustain:.2f} req/s), both policies")
    ss = serving_run(rate=sustain, window=15.0, budget=45.0)
    ssh = serving_run(rate=sustain, window=15.0, budget=45.0, policy="hrrn")
    for rec in (ss, ssh):
        rec["capacity_req_s"] = capacity
        rec["capacity_model"] = ("GLUPS while busy / (c E[n^4]), c = median steps / n^2 of "
                                 "the completed requests of the overloaded run")
    return sv, ss, sh, ssh


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds: float):
    """The FP64 CPU oracle, as it stands, on a bounded sample of the workload
    (the first 1024 x 1024 case), timed on this host's cores."""
    import numpy as np
    from oracle import oracle as O
    from paper_2208_14870_amd import problem as P
    c = P.single_1024(0.1, 1, 1)
    om = O.omega_vector(c.material.lame_lambda, c.material.lame_mu)
    f = O.zero_state(c.nx, c.ny)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        f = O.run(f, c.gx, c.gy, om, 2)
        steps += 2
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": c.nx * c.ny * steps / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "cores_visible": len(os.sched_getaffinity(0)),
            "sample": f"1024x1024, nu=0.1, mode (1,1): {steps} of the 20000 pseudo-time steps, "
                      f"{dt:.1f} s, FP64, OpenMP over rows"}


def cpu_oracle_large(nsteps: int = 20):
    """The FP64 CPU oracle on the 8192 x 8192 random load for `nsteps` steps
    (all host cores): a short timing whose MLUPS stand for the 10,200-step run,
    which the oracle would take hours to finish."""
    import numpy as np
    from oracle import oracle as O
    from paper_2208_14870_amd import problem as P
    c = P.single_8192()
    om = O.omega_vector(c.material.lame_lambda, c.material.lame_mu)
    f = O.zero_state(c.nx, c.ny)
    f = O.run(f, c.gx, c.gy, om, 1)  # first touch of the arrays, untimed
    t0 = time.perf_counter()
    f = O.run(f, c.gx, c.gy, om, nsteps)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    mlups = c.nx * c.ny * nsteps / dt / 1e6
    return {"value": mlups, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "extrapolated": True,
            "sample": f"8192x8192 random 16-mode load: {nsteps} steps in {dt:.1f} s, FP64, "
                      f"OpenMP over rows; the 200 + 10000 steps of the workload at this rate "
                      f"would take {c.nx * c.ny * 10200 / mlups / 1e6 / 3600:.1f} h"}


def cpu_oracle_batch_sample(nlat: int = 8, steps: int = 200):
    """The FP64 CPU oracle on `nlat` lattices sampled from the 512-lattice
    workload (seed 4), `steps` steps each, one after another (all host cores)."""
    import numpy as np
    from oracle import oracle as O
    from paper_2208_14870_amd import problem as P
    cases = P.batch_cases(512, seed=4)
    pick = np.random.default_rng(12).choice(len(cases), nlat, replace=False)
    sites, dt = 0, 0.0
    for i in pick:
        c = cases[int(i)]
        om = O.omega_vector(c.material.lame_lambda, c.material.lame_mu)
        t0 = time.perf_counter()
        O.run(O.zero_state(c.nx, c.ny), c.gx, c.gy, om, steps)
        dt += time.perf_counter() - t0
        sites += c.nx * c.ny
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": sites * steps / dt / 1e6, "unit": "MLUPS", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{nlat} lattices of the 512-lattice workload ({sites} sites), "
                      f"{steps} steps each, {dt:.1f} s, FP64, OpenMP over rows"}


def cpu_baseline_one_thread(seconds: float):
    """The same oracle sample on one thread, in a child process (OpenMP reads
    its thread count at start-up)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-oracle-only",
                        "--cpu-seconds", str(seconds)], env=env, capture_output=True, text=True,
                       timeout=seconds * 10 + 120)
    if r.returncode != 0:
        return {"error": r.stderr[-300:]}
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    return {"value": rec["value"], "unit": rec["unit"], "cores": 1, "sample": rec["sample"]}


def main():
    args = parse()
    if args.cpu_oracle_only:
        print(json.dumps(cpu_baseline(args.cpu_seconds)), flush=True)
        return
    if args.cpu_oracle_large:
        print(json.dumps({"cpu_oracle_8192": cpu_oracle_large(),
                          "cpu_oracle_batch_sample": cpu_oracle_batch_sample()}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1 (the "
                          "library has no multi-GPU decomposition: lattices would shard "
                          "whole, a large lattice by slabs with halo exchange)"}))
        sys.exit(2)
    import torch
    from paper_2208_14870_amd import lbm
    lbm.load()
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if args.inplace_only:
        if args.calib_copy:
            calib_copy()
        print(json.dumps({"inplace_8192": inplace_run(steps=args.large_steps,
                                                      warm=args.large_warm)}), flush=True)
        return
    if args.small_only:
        print(json.dumps({"small_32": small_32()}), flush=True)
        return
    if args.accuracy_only:
        print(json.dumps({"accuracy": accuracy_studies()}), flush=True)
        return
    if args.serving_only:
        sv, ss, sh, ssh = serving_legs()
        print(json.dumps({"serving": sv, "serving_sustained": ss, "serving_hrrn": sh,
                          "serving_sustained_hrrn": ssh}), flush=True)
        return
    if args.batch_only:
        if args.calib_copy:
            calib_copy()
        print(json.dumps({"batch": {p: batch_run(p, steps=args.batch_steps)
                                    for p in args.batch_only.split(",")}}), flush=True)
        return
    if args.large_only:
        if args.calib_copy:
            calib_copy()
        precs = tuple(args.large_only.split(","))
        print(json.dumps({"large_8192": large_lattice(args.large_steps, args.large_warm, precs,
                                                      args.large_tb)}),
              flush=True)
        return
    cases = build_cases(args.cases)
    nsites = cases[0].nx * cases[0].ny

    def measure(prec):
        solvers = make_solvers(cases, prec, args.headline_kernel if prec == "fp32" else "default")
        if args.warmup:
            run_workload(solvers, args.warmup, args.chunk)
        for s, _ in solvers:
            s.reset()
        res = run_workload(solvers, args.steps, args.chunk)
        updates = nsites * args.chunk * args.steps * len(solvers)
        res["mlups"] = updates / res["wall_s"] / 1e6
        u = [s.displacement() for s, _ in solvers]
        res["stress_rel_l2"] = [stress_error(s, c)[0] for (s, _), c in zip(solvers, cases)]
        for s, _ in solvers:
            s.close()
        return res, u

    if args.comparator_only:
        if args.calib_copy:
            calib_copy()
        r64, _ = measure("fp64")
        print(json.dumps({"fp64": {"mlups": round(r64["mlups"], 1),
                                   "avg_launch_us": round(r64["plain_kernel_avg_us"], 3),
                                   "steps_per_launch": r64["steps_per_launch"],
                                   "launch_config": r64["launch_config"],
                                   "kernel": kernel_label(r64["launch_config"], "double",
                                                          1024 * 1024)}}), flush=True)
        return
    log("headline: 1024x1024 FP32")
    r32, u32 = measure("fp32")
    out = {
        "metric": "MLUPS & % HBM roofline (FP64 vs FP32 store); batched solves/s + p50/p99 latency",
        "value": round(r32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * r32["wall_s"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded manufactured sinusoidal loads)",
        "config": {"workload": "single periodic 1024x1024 D2Q8 lattice, FP32 populations, "
                               "nu in {0.1,0.3,0.45,0.49} x modes {(1,1),(4,3)}, mu=1, "
                               f"{args.steps * args.chunk} pseudo-time steps per case, "
                               f"residual + displacement + error norms every {args.chunk}",
                   "lattice": [1024, 1024], "cases": len(cases), "chunk": args.chunk,
                   "storage": "fp32", "parallelism": "single GPU"},
        "roofline": roofline("fp32", nsites, r32["plain_kernel_avg_us"], r32["steps_per_launch"],
                             kernel_label(r32["launch_config"], "float", nsites),
                             ("k_wave_fp32_1024_counters"
                              if r32["launch_config"]["kernel"] == "wavefront"
                              else "k_stepN_fp32_1024_counters"),
                             note="1024^2 FP32 (~72 MB of populations and force) fits the "
                                  "256 MB last-level cache: frac is against HBM's peak, the "
                                  "bytes need not come from HBM; the HBM-resident figures "
                                  "are under large_8192"),
        "fp32_last_residual": r32["last"][0][0],
        "fp32_rel_l2_vs_manufactured": [round(x[1], 6) for x in r32["last"]],
        "fp32_rel_linf_vs_manufactured": [round(x[2], 6) for x in r32["last"]],
        "fp32_residual_history_case0": [float("%.4g" % r) for r in r32["history"]],
        "fp32_stress_rel_l2_vs_manufactured": [round(x, 6) for x in r32["stress_rel_l2"]],
    }
    if args.calib_copy:
        calib_copy()
    if not args.no_extras:
        log("comparison: 1024x1024 FP64")
        r64, u64 = measure("fp64")
        num = sum(float(torch.sum((a - b) ** 2) + torch.sum((c - d) ** 2))
                  for (a, c), (b, d) in zip(u32, u64))
        den = sum(float(torch.sum(b ** 2) + torch.sum(d ** 2)) for (b, d) in u64)
        out["fp64"] = {"mlups": round(r64["mlups"], 1),
                       "roofline": roofline("fp64", nsites, r64["plain_kernel_avg_us"],
                                            r64["steps_per_launch"],
                                            kernel_label(r64["launch_config"], "double", nsites),
                                            ("k_wave_fp64_1024_counters"
                                             if r64["launch_config"]["kernel"] == "wavefront"
                                             else "k_stepN_fp64_1024_counters"))}
        out["fp32_speedup_over_fp64"] = round(r32["mlups"] / r64["mlups"], 3)
        log("the same sweep, its 8 lattices advanced together (batch)")
        out["sweep_batched_fp32"] = sweep_batched(cases, args.steps, args.chunk)
        out["fp32_rel_l2_vs_fp64"] = math.sqrt(num / den)
        log("8192x8192 random load: FP64 / FP32 / FP16, 200 + 10000 steps")
        out["hbm_copy"] = copy_bandwidth()
        log("32x32 FP64 to r <= 1e-10, a check every step")
        out["small_32"] = small_32()
        log("accuracy: the paper's three convergence studies (FP64, 20..160 nodes)")
        out["accuracy"] = accuracy_studies()
        out["large_8192"] = large_lattice()
        log("in-place streaming vs two buffers, 8192x8192, one step per launch")
        out["inplace_8192"] = inplace_run()
        log("batched: 512 lattices FP32 / FP64, 2000 steps")
        out["batch"] = {"fp32": batch_run("fp32"), "fp64": batch_run("fp64")}
        log("batched solves to r <= 1e-6 (FP32, FP32 + FP64 polish, FP64)")
        keys = ("completed", "elapsed_s", "solves_per_s", "p50_latency_s", "p99_latency_s")

        def err_vs_fp64(res):
            # FP64 reference at exactly the step count each solve stopped at
            _, ref = batch_solves("fp64", fixed_steps={rid: r.steps for rid, r in res.items()})
            errs = []
            for rid, r64 in ref.items():
                r = res[rid]
                num = float(((r.ux - r64.ux) ** 2).sum() + ((r.uy - r64.uy) ** 2).sum())
                den = float((r64.ux ** 2).sum() + (r64.uy ** 2).sum())
                errs.append(math.sqrt(num / den))
            errs.sort()
            return {"same_step_rel_l2_vs_fp64_max": errs[-1],
                    "same_step_rel_l2_vs_fp64_median": errs[len(errs) // 2]}
        s32, res32 = batch_solves("fp32")
        sp, resp = batch_solves("fp32", r_switch=1e-5)
        s64, _ = batch_solves("fp64")
        out["batch"]["solves"] = {
            "tol": 1e-6,
            "fp32": dict({k: s32[k] for k in keys}, **err_vs_fp64(res32)),
            "fp32_polish_at_1e-5": dict({k: sp[k] for k in keys}, **err_vs_fp64(resp)),
            "fp64": {k: s64[k] for k in keys}}
        (out["serving"], out["serving_sustained"], out["serving_hrrn"],
         out["serving_sustained_hrrn"]) = serving_legs()
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        log("CPU oracle baseline, one thread")
        out["cpu_baseline"]["one_thread"] = cpu_baseline_one_thread(min(6.0, args.cpu_seconds))
        out["paper_context"] = {"mlups": 0.25, "note": "derived from ~1.6 s for ~1e3 steps of "
                                "20x20 on a low-end notebook (Sec. 7.3.1); other hardware"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
