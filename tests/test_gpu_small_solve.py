"""Whole solves of small lattices in one workgroup (lbm_set_small_solve): the
same stop step, outcome, state and residual (to the rounding of its sums) as the
launch-per-check solve, including a launch budget that makes the host resume the
solve, the step limit, divergence, general rates and FP32 storage."""
import json

import numpy as np
import pytest

from paper_2208_14870_amd import problem as P
from gpu_common import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def _solve(lbm, n1, n2, prec, mat, gx, gy, rates, tol, max_steps, K, budget, r_switch=0.0):
    s = lbm.Solver(n1, n2, prec, with_polish=r_switch > 0.0)
    s.set_material(mat.lame_lambda, mat.lame_mu)
    if rates:
        s.set_rates(*rates)
    s.set_body_force(dev(gx), dev(gy))
    if r_switch > 0.0:
        s.set_polish(r_switch)
    s.set_small_solve(budget)
    try:
        n, r, status = s.solve_to_tol(tol, max_steps, K)
    except lbm.Diverged:
        n, r, status = s.steps_done, float("nan"), -5
    f = host(s.populations())
    ux, uy = (host(t) for t in s.displacement())
    done = (s.steps_done, s.current_precision)
    s.close()
    return n, r, status, f, ux, uy, done


def test_random_small_solves_equal_the_launch_per_check_solve():
    from paper_2208_14870_amd import lbm
    need_gpu()
    rng = np.random.default_rng(31)
    for case in range(40):
        prec = str(rng.choice(["fp64", "fp32"]))
        cap = 1152 if prec == "fp64" else 2304
        while True:
            nx, ny = int(rng.integers(1, 60)), int(rng.integers(1, 60))
            if nx * ny <= cap:
                break
        mat = P.Material.from_shear_poisson(float(rng.uniform(0.3, 1.5)), float(rng.uniform(0.05, 0.45)))
        rates = (0.4, 1.2, 1.2, 0.8) if rng.random() < 0.25 else None
        kx, ky = int(rng.integers(1, 3)), int(rng.integers(0, 3))
        x = (np.arange(nx) + 0.5) / nx
        y = (np.arange(ny) + 0.5) / ny
        gx = P.remove_mean(1e-4 * np.sin(2 * np.pi * (kx * x[None, :] + ky * y[:, None])))
        gy = P.remove_mean(1e-4 * np.cos(2 * np.pi * (kx * x[None, :] - ky * y[:, None])))
        tol = float(rng.choice([1e-5, 1e-8, 1e-10])) if prec == "fp64" else 1e-5
        K = int(rng.choice([1, 2, 3, 7, 25, 100]))
        max_steps = int(rng.choice([0, 1, 5, 37, 20000]))
        budget = int(rng.choice([1, 7, 64, 65536]))
        say("small " + json.dumps(dict(case=case, nx=nx, ny=ny, prec=prec, general=bool(rates),
                                        tol=tol, K=K, max_steps=max_steps, budget=budget)))
        a = _solve(lbm, nx, ny, prec, mat, gx, gy, rates, tol, max_steps, K, budget)
        b = _solve(lbm, nx, ny, prec, mat, gx, gy, rates, tol, max_steps, K, 0)
        _same(a, b)


def _same(a, b):
    assert a[0] == b[0] and a[2] == b[2] and a[6] == b[6], (a[0], b[0], a[2], b[2], a[6], b[6])
    assert (np.isnan(a[1]) and np.isnan(b[1])) or abs(a[1] - b[1]) <= 1e-9 * abs(b[1])
    for u, v in zip(a[3:6], b[3:6]):
        assert np.array_equal(u, v, equal_nan=True)


def test_small_solves_with_the_fp64_switch():
    """FP32 storage with a polish threshold: the device finds the switch due (r <=
    r_switch or two checks without decrease), the host switches to FP64 and the
    solve goes on in one workgroup; same steps, switch and final state as the
    launch-per-check solve."""
    from paper_2208_14870_amd import lbm
    need_gpu()
    rng = np.random.default_rng(32)
    for case in range(16):
        while True:
            nx, ny = int(rng.integers(2, 40)), int(rng.integers(2, 40))
            if nx * ny <= 1152:
                break
        mat = P.Material.from_shear_poisson(float(rng.uniform(0.3, 1.5)), float(rng.uniform(0.05, 0.45)))
        x = (np.arange(nx) + 0.5) / nx
        y = (np.arange(ny) + 0.5) / ny
        gx = P.remove_mean(1e-4 * np.sin(2 * np.pi * (x[None, :] + y[:, None])))
        gy = P.remove_mean(1e-4 * np.cos(2 * np.pi * (x[None, :] - 2 * y[:, None])))
        K = int(rng.choice([1, 3, 20, 50]))
        r_switch = float(rng.choice([1e-4, 1e-6, 1e-7]))
        budget = int(rng.choice([1, 9, 65536]))
        say("small polish " + json.dumps(dict(case=case, nx=nx, ny=ny, K=K, r_switch=r_switch,
                                               budget=budget)))
        a = _solve(lbm, nx, ny, "fp32", mat, gx, gy, None, 1e-11, 30000, K, budget, r_switch)
        b = _solve(lbm, nx, ny, "fp32", mat, gx, gy, None, 1e-11, 30000, K, 0, r_switch)
        _same(a, b)
        assert a[6][1] == 0  # ended in FP64


def test_small_solve_divergence():
    """Unstable material of Sec. 7.3.5: both paths report divergence at the same step."""
    from paper_2208_14870_amd import lbm
    need_gpu()
    c = P.gaussian_hill_case(32, P.Material.from_young_poisson(0.082, -0.4))
    out = []
    for budget in (65536, 0):
        s = lbm.Solver(32, 32, "fp64")
        s.set_material(c.material.lame_lambda, c.material.lame_mu)
        s.set_body_force(dev(c.gx), dev(c.gy))
        s.set_small_solve(budget)
        with pytest.raises(lbm.Diverged):
            s.solve_to_tol(1e-10, 20000, 500)
        out.append(s.steps_done)
        s.close()
    say(f"diverged after {out[0]} steps (one workgroup) and {out[1]} (launch per check)")
    assert out[0] == out[1]


def test_small_solve_argument_errors():
    from paper_2208_14870_amd import lbm
    need_gpu()
    s = lbm.Solver(8, 8, "fp64")
    with pytest.raises(lbm.LbmError):
        s.set_small_solve(-1)
    s.close()
