"""Continuous-batching server for periodic elasticity solves.

Requests (a lattice size, a material and a body load) arrive over time.  The
server keeps one device arena; a request is admitted as soon as a slot and
its HBM footprint (FP32 state plus the FP64 polish reservation) are free,
joins the resident batch at the next chunk boundary, and every admitted
lattice advances in the same persistent step launches.  After each chunk of
`chunk` steps the FP64 residual of every lattice is read; a lattice in FP32
switches to FP64 storage once its residual reaches `r_switch` or stops
decreasing, and retires when r <= tol: its displacement is copied to the host
and its memory returns to the arena.  A lattice whose residual becomes
non-finite or whose update norm keeps rising (the library's divergence
guard) is retired as failed.  Latency = result on host - arrival.

Admission order (`policy`): "fifo" takes waiting requests in arrival order,
backfilling smaller ones that fit when the next does not; "hrrn" (highest
response ratio next) takes them in decreasing (wait + S) / S, where S is the
request's predicted service time: the site-updates its solve needs (steps of
its slowest smooth mode to reach the tolerance, times n^2) over the measured
update rate.  Small solves go first, as in shortest-job-first, and a waiting
request's ratio grows with its wait, so a large one is not starved.

Each lattice steps whole chunks from its admission on, with its own promote
and retire decisions taken only from its own residuals, so its result is
the same alone and in any mix (the per-site arithmetic and the per-lattice
reduction order do not depend on the other lattices), whatever the policy.
"""
from __future__ import annotations

import dataclasses
import time
from collections import deque
from typing import Dict, List, Optional

import math

import numpy as np
import torch

from . import lbm, stability
from .problem import Case, Material, Request


def predicted_work(n: int, lame_lambda: float, lame_mu: float, tol: float) -> float:
    """Site-updates an n x n solve from f = 0 needs to reach the residual tol:
    the steps of the slowest smooth mode, the shear mode at the lowest
    wavenumber 2 pi / n (stability.predicted_steps of its |eigenvalue|), times
    n^2.  An estimate: the load's other modes decay faster."""
    A = stability.collision_operator(lame_lambda, lame_mu)
    k = 2.0 * math.pi / n
    rho = max(float(np.max(np.abs(np.linalg.eigvals(stability.amplification(A, k, 0.0))))),
              float(np.max(np.abs(np.linalg.eigvals(stability.amplification(A, 0.0, k))))))
    steps = stability.predicted_steps(rho, tol)
    return float(max(steps, 1)) * n * n


def admission_order(waiting, now: float, rate: float, policy: str):
    """The order in which waiting requests are offered a slot: `waiting` is a
    list of (request, predicted site-updates); "fifo" keeps arrival order,
    "hrrn" sorts by decreasing response ratio (now - t_arrival + S) / S with
    S = work / rate (seconds of GPU time), ties in arrival order."""
    if policy == "fifo":
        return sorted(waiting, key=lambda rw: (rw[0].t_arrival, rw[0].rid))
    if policy != "hrrn":
        raise ValueError(f"unknown admission policy {policy!r}")

    def ratio(rw):
        svc = rw[1] / rate
        return (now - rw[0].t_arrival + svc) / svc
    return sorted(waiting, key=lambda rw: (-ratio(rw), rw[0].t_arrival, rw[0].rid))


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    t_arrival: float
    t_admit: float
    t_done: float
    steps: int
    residual: float
    promoted_at: int
    ux: Optional[np.ndarray] = None
    uy: Optional[np.ndarray] = None

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


@dataclasses.dataclass
class _Active:
    req: Request
    case: Case
    t_admit: float
    last_r: float = float("inf")
    nondecreasing: int = 0
    promoted_at: int = -1
    g: tuple = ()


class Server:
    def __init__(self, arena_bytes: int, max_slots: int = 1024, chunk: int = 200,
                 tol: float = 1e-8, r_switch: float = 1e-6, precision: str = "fp32",
                 polish: bool = True, max_steps: int = 10 ** 8, keep_results: bool = False,
                 tile: Optional[tuple] = None, policy: str = "fifo"):
        self.batch = lbm.Batch(max_slots, arena_bytes)
        if tile is not None:
            self.batch.set_tile(*tile)
        self.chunk = int(chunk)
        self.tol = tol
        self.r_switch = r_switch
        self.precision = precision
        self.polish = polish and precision != "fp64"
        self.max_steps = max_steps
        self.keep = keep_results
        self.active: Dict[int, _Active] = {}
        self.results: List[Result] = []
        self.failed: List[int] = []
        self.site_updates = 0
        admission_order([], 0.0, 1.0, policy)  # rejects an unknown policy
        self.policy = policy
        self.work: Dict[int, float] = {}  # predicted site-updates per request id

    def footprint(self, n: int) -> int:
        return lbm.Batch.slot_bytes(n, n, self.precision, self.polish)

    def _admit(self, req: Request, case: Case, now: float) -> bool:
        gx = torch.from_numpy(case.gx).cuda()
        gy = torch.from_numpy(case.gy).cuda()
        slot = self.batch.add(case.nx, case.ny, case.material.lame_lambda, case.material.lame_mu,
                              gx, gy, self.precision, self.polish)
        if slot is None:
            return False
        self.active[slot] = _Active(req, case, now, g=(gx, gy))
        return True

    def _retire_all(self, done, now_fn):
        """Retire the lattices of one chunk together: their displacements reach
        the host in one copy (the latency ends there), then their memory
        returns to the arena."""
        if not done:
            return
        fields = self.batch.displacements([slot for slot, _, _ in done])
        t = now_fn()
        for (slot, steps, r), (hx, hy) in zip(done, fields):
            a = self.active[slot]
            self.results.append(Result(a.req.rid, a.req.n, a.req.t_arrival, a.t_admit, t, steps,
                                       r, a.promoted_at, hx if self.keep else None,
                                       hy if self.keep else None))
            self.batch.remove(slot)
            del self.active[slot]

    def run(self, requests: List[Request], admit_window_s: float, wall_budget_s: float,
            cases: Optional[Dict[int, Case]] = None,
            fixed_steps: Optional[Dict[int, int]] = None) -> dict:
        """Serve `requests` (arrival times relative to the start).  Arrivals
        after `admit_window_s` are not offered; the loop stops when everything
        offered has retired or after `wall_budget_s` seconds.  With
        `fixed_steps`, request rid retires after exactly that many steps
        (a multiple of the chunk) instead of at the tolerance."""
        pending = deque(sorted((r for r in requests if r.t_arrival < admit_window_s),
                               key=lambda r: r.t_arrival))
        offered = len(pending)
        queue: deque = deque()
        t0 = time.perf_counter()

        def now():
            return time.perf_counter() - t0

        gpu_time = 0.0
        while True:
            t = now()
            while pending and pending[0].t_arrival <= t:
                req = pending.popleft()
                if self.policy != "fifo":
                    mat = cases[req.rid].material if cases is not None else \
                        Material.from_shear_poisson(1.0, req.nu)
                    self.work[req.rid] = predicted_work(req.n, mat.lame_lambda, mat.lame_mu,
                                                        self.tol)
                queue.append(req)
            # admission in the policy's order, backfilling requests that fit
            if self.policy != "fifo" and queue:
                rate = self.site_updates / gpu_time if gpu_time > 0 else 2e11
                queue = deque(r for r, _ in admission_order(
                    [(r, self.work[r.rid]) for r in queue], t, rate, self.policy))
            skipped = deque()
            _, _, largest = self.batch.info()
            while queue:
                req = queue.popleft()
                if (len(self.active) >= self.batch.max_slots or
                        self.footprint(req.n) > largest):
                    skipped.append(req)
                    if largest < self.footprint(64) or len(self.active) >= self.batch.max_slots:
                        break
                    continue
                case = cases[req.rid] if cases is not None else req.case()
                if not self._admit(req, case, now()):
                    skipped.append(req)
                _, _, largest = self.batch.info()
            skipped.extend(queue)
            queue = skipped
            if self.active:
                g0 = time.perf_counter()
                self.batch.step(self.chunk, check=True)
                r, steps = self.batch.residuals()
                diverged = self.batch.diverged()
                gpu_time += time.perf_counter() - g0
                done = []
                for slot in list(self.active):
                    a = self.active[slot]
                    self.site_updates += a.case.nx * a.case.ny * self.chunk
                    rs = r[slot]
                    # a converged residual wins over the guard (as in solve_to_tol)
                    if diverged[slot] and not rs <= self.tol:
                        self.failed.append(a.req.rid)
                        self.batch.remove(slot)
                        del self.active[slot]
                        continue
                    if fixed_steps is not None:
                        if steps[slot] >= fixed_steps[a.req.rid]:
                            done.append((slot, steps[slot], rs))
                        continue
                    if rs <= self.tol or steps[slot] >= self.max_steps:
                        done.append((slot, steps[slot], rs))
                        continue
                    if self.polish and a.promoted_at < 0:
                        a.nondecreasing = a.nondecreasing + 1 if rs >= a.last_r else 0
                        if rs <= self.r_switch or a.nondecreasing >= 2:
                            self.batch.promote(slot)
                            a.promoted_at = steps[slot]
                    a.last_r = rs
                self._retire_all(done, now)
            elif not pending and not queue:
                break
            else:
                nxt = pending[0].t_arrival if pending else t
                time.sleep(max(0.0, min(nxt - now(), 0.005)))
            if now() > wall_budget_s:
                break
        elapsed = now()
        lat = np.array([x.latency for x in self.results]) if self.results else np.array([])
        return {
            "offered": offered,
            "completed": len(self.results),
            "failed": len(self.failed),
            "backlog": len(queue) + len(pending) + len(self.active),
            "elapsed_s": elapsed,
            "solves_per_s": len(self.results) / elapsed if elapsed > 0 else 0.0,
            "p50_latency_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_latency_s": float(np.percentile(lat, 99)) if lat.size else None,
            "gpu_busy_s": gpu_time,
            "policy": self.policy,
            "mlups_while_busy": self.site_updates / gpu_time / 1e6 if gpu_time > 0 else 0.0,
        }

    def close(self):
        self.batch.close()
