"""GPU path (C ABI via the Python binding) against the FP64 CPU oracle.

Bars: streaming/index arithmetic bit-exact; FP64 within 1e-12 relative;
reduced precisions within tolerances derived from their rounding unit
(stated per test).
"""
import functools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_14870_amd import problem as P
from gpu_common import assert_elementwise, dev, host, need_gpu, omega, rel_l2, say

pytestmark = pytest.mark.gpu


def _solver(nx, ny, prec="fp64", polish=False):
    from paper_2208_14870_amd import lbm
    need_gpu()
    return lbm.Solver(nx, ny, prec, with_polish=polish)


def _rand_state(nx, ny, seed, scale=1e-3):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((8, ny, nx)) * scale
    gx = P.remove_mean(rng.standard_normal((ny, nx)) * scale * 0.1)
    gy = P.remove_mean(rng.standard_normal((ny, nx)) * scale * 0.1)
    return f, gx, gy


# ---------------------------------------------------------------------------
# streaming and state transfer: bit-exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec,nx,ny", [
    ("fp64", 1, 1), ("fp64", 2, 2), ("fp64", 3, 3), ("fp64", 5, 3), ("fp64", 67, 33),
    ("fp64", 256, 64), ("fp32", 2, 7), ("fp32", 130, 9), ("fp32", 64, 64), ("fp16", 3, 5),
    ("fp16", 97, 31)])
def test_streaming_bit_exact(prec, nx, ny):
    say(f"streaming bit-exact {prec} {nx}x{ny}")
    s = _solver(nx, ny, prec)
    top = {"fp64": 1 << 40, "fp32": 1 << 23, "fp16": 2000}[prec]
    rng = np.random.default_rng(nx * 1000 + ny)
    f = rng.integers(-top, top, size=(8, ny, nx)).astype(np.float64)
    s.set_populations(dev(f))
    for steps in (1, 4):
        s.stream_only(steps)
        f = O.stream_only(f, steps)
        np.testing.assert_array_equal(host(s.populations()), f)


def test_populations_roundtrip_fp64():
    say("populations roundtrip fp64 37x21")
    s = _solver(37, 21)
    f, _, _ = _rand_state(37, 21, 1)
    s.set_populations(dev(f))
    np.testing.assert_array_equal(host(s.populations()), f)


# ---------------------------------------------------------------------------
# FP64 parity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("nx,ny,steps", [(1, 1, 5), (2, 2, 7), (3, 4, 9), (32, 32, 100),
                                         (67, 45, 50), (130, 7, 30), (64, 257, 20)])
def test_fp64_steps_from_random_state(nx, ny, steps):
    """Arbitrary state and force (ragged tiles, N = 1, 2): n steps agree to 1e-12."""
    say(f"fp64 random state {nx}x{ny} steps {steps}")
    mat = P.Material.from_shear_poisson(0.8, 0.25)
    f0, gx, gy = _rand_state(nx, ny, nx + 7 * ny)
    s = _solver(nx, ny)
    s.set_material(mat.lame_lambda, mat.lame_mu)
    s.set_body_force(dev(gx), dev(gy))
    s.set_populations(dev(f0))
    s.step(1)
    f1 = O.run(f0, gx, gy, omega(mat), 1)
    g1 = host(s.populations())
    assert_elementwise(g1, f1, 1e-14, "f(1)")
    s.step(steps - 1)
    fn = O.run(f1, gx, gy, omega(mat), steps - 1)
    assert_elementwise(host(s.populations()), fn, 1e-12, "f")
    ux, uy = (host(t) for t in s.displacement())
    ox, oy = O.displacement(fn, gx, gy)
    assert_elementwise((ux, uy), (ox, oy), 1e-12, "u")


def test_fp64_config_32_solve_matches_oracle():
    """32 x 32, nu = 0.3, mu = 1, manufactured sinusoid, tol 1e-10, check every
    step: identical stop step, displacement within 1e-12."""
    say("fp64 single-32 solve_to_tol")
    c = P.single_32()
    s = _solver(32, 32)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    n, r, st = s.solve_to_tol(1e-10, 100000, 1)
    f, on, orr, ost = O.solve_to_tol(O.zero_state(32, 32), c.gx, c.gy, omega(c.material), 1e-10,
                                     100000, 1)
    assert st == 0 and ost == 0
    assert n == on
    assert r == pytest.approx(orr, rel=1e-8)
    ux, uy = (host(t) for t in s.displacement())
    ox, oy = O.displacement(f, c.gx, c.gy)
    assert_elementwise((ux, uy), (ox, oy), 1e-12, "u")
    err = s.error_norms(dev(c.ux_exact), dev(c.uy_exact))
    want = O.error_norms(ox, oy, c.ux_exact, c.uy_exact)
    assert err["rel_l2"] == pytest.approx(want["rel_l2_plain"], rel=1e-9)


@pytest.mark.parametrize("K", [2, 7, 64, 250])
def test_fp64_check_interval_matches_oracle(K):
    """Residual checks every K steps: same stop step and residual as the oracle."""
    say(f"fp64 check interval {K}")
    c = P.single_1024(0.3, 1, 1, n=48)
    s = _solver(48, 48)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    n, r, st = s.solve_to_tol(1e-9, 20000, K)
    f, on, orr, ost = O.solve_to_tol(O.zero_state(48, 48), c.gx, c.gy, omega(c.material), 1e-9,
                                     20000, K)
    assert (st, n) == (ost, on)
    assert r == pytest.approx(orr, rel=1e-7)
    ux, uy = (host(t) for t in s.displacement())
    ox, oy = O.displacement(f, c.gx, c.gy)
    assert_elementwise((ux, uy), (ox, oy), 1e-12, "u")


@pytest.mark.parametrize("prec,nx,ny,n,tb", [
    ("fp64", 48, 48, 30, 5), ("fp64", 48, 48, 30, 1), ("fp64", 33, 17, 9, 4),
    ("fp32", 70, 40, 18, 8), ("fp32", 70, 40, 17, 8), ("fp64", 24, 24, 2, 8),
    ("fp16", 64, 64, 21, 8)])
def test_step_checked(prec, nx, ny, n, tb):
    """step_checked(n) advances n steps (f(n) as n plain steps, bit for bit) and
    returns r(n - 1) of the oracle (FP64: to 1e-9; the check may ride on the last
    fused launch of any span)."""
    say(f"step_checked {prec} {nx}x{ny} n {n} tb {tb}")
    from paper_2208_14870_amd import lbm
    mat = P.Material.from_shear_poisson(0.9, 0.3)
    f0, gx, gy = _rand_state(nx, ny, 13 + nx)
    out = []
    for checked in (True, False):
        s = _solver(nx, ny, prec)
        s.set_material(mat.lame_lambda, mat.lame_mu)
        s.set_body_force(dev(gx), dev(gy))
        s.set_populations(dev(f0))
        s.set_time_blocking(tb)
        r = s.step_checked(n) if checked else s.step(n)
        assert s.steps_done == n
        out.append((r, host(s.populations())))
        s.close()
    if prec == "fp16":
        # the half-storage rescale after the check is exact for normal halves
        # and moves subnormal ones by at most half their spacing
        np.testing.assert_allclose(out[0][1], out[1][1], rtol=0, atol=1e-10)
    else:
        np.testing.assert_array_equal(out[0][1], out[1][1])
    assert np.isfinite(out[0][0])
    if prec == "fp64":
        f = O.run(f0, gx, gy, omega(mat), n - 2)
        ua = O.displacement(f, gx, gy)
        f = O.run(f, gx, gy, omega(mat), 1)
        ub = O.displacement(f, gx, gy)
        assert out[0][0] == pytest.approx(O.residual(ub[0], ub[1], ua[0], ua[1]), rel=1e-9)
    with pytest.raises(lbm.LbmError):
        _solver(8, 8, prec).step_checked(1)


def test_fp64_max_steps_not_converged():
    say("fp64 max_steps")
    c = P.single_32()
    s = _solver(32, 32)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    n, r, st = s.solve_to_tol(1e-14, 50, 10)
    assert (n, st) == (50, 1)
    f, on, orr, ost = O.solve_to_tol(O.zero_state(32, 32), c.gx, c.gy, omega(c.material), 1e-14,
                                     50, 10)
    assert (on, ost) == (50, 1)
    assert r == pytest.approx(orr, rel=1e-9)
    ux, uy = (host(t) for t in s.displacement())
    ox, oy = O.displacement(f, c.gx, c.gy)
    assert_elementwise((ux, uy), (ox, oy), 1e-12, "u")


@pytest.mark.parametrize("prec,tile", [("fp64", None), ("fp64", (6, 4, 0)), ("fp32", (8, 4, 0))])
def test_general_rates(prec, tile):
    """theta = 0.4, omega_12 = omega_21 = 1.2, omega_22 = 0.8 (general path), also
    with a multi-row tile request (the general variant runs one row per thread)."""
    say(f"general rates {prec} tile {tile}")
    nx, ny = 40, 24
    mat = P.Material.from_shear_poisson(0.6, 0.35)
    f0, gx, gy = _rand_state(nx, ny, 5)
    s = _solver(nx, ny, prec)
    if tile:
        s.set_tile(*tile)
    s.set_material(mat.lame_lambda, mat.lame_mu)
    s.set_rates(0.4, 1.2, 1.2, 0.8)
    s.set_body_force(dev(gx), dev(gy))
    s.set_populations(dev(f0))
    s.step(60)
    om = O.omega_vector(mat.lame_lambda, mat.lame_mu, 0.4, 1.2, 1.2, 0.8)
    fn = O.run(f0, gx, gy, om, 60, theta=0.4)
    if prec == "fp64":
        assert_elementwise(host(s.populations()), fn, 1e-12, "f")
    else:
        assert rel_l2(host(s.populations()), fn) <= 1e-5


def test_fp64_stress_matches_oracle():
    say("fp64 stress")
    c = P.paper_e1(24)
    s = _solver(24, 24)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    s.step(300)
    f = O.run(O.zero_state(24, 24), c.gx, c.gy, omega(c.material), 300)
    want = O.stress(f, omega(c.material))
    got = [host(t) for t in s.stress()]
    for a, b in zip(got, want):
        assert_elementwise(a, b, 1e-12, "f")


@pytest.mark.parametrize("nx,ny,tile", [(96, 64, (5, 1)), (96, 64, (7, 2)), (100, 90, (4, 4)),
                                        (33, 65, (0, 1)), (33, 65, (8, 4))])
def test_fp64_tile_shapes(nx, ny, tile):
    """Every tile shape gives the oracle's result (ragged edges included)."""
    say(f"fp64 tile {tile} {nx}x{ny}")
    mat = P.Material.from_shear_poisson(1.0, 0.45)
    f0, gx, gy = _rand_state(nx, ny, 11)
    s = _solver(nx, ny)
    s.set_tile(*tile)
    s.set_material(mat.lame_lambda, mat.lame_mu)
    s.set_body_force(dev(gx), dev(gy))
    s.set_populations(dev(f0))
    s.step(25)
    fn = O.run(f0, gx, gy, omega(mat), 25)
    assert_elementwise(host(s.populations()), fn, 1e-12, "f")


def test_fp64_full_size_1024_sampled():
    """1024 x 1024 in the benchmark's launch configuration: 20 steps from a
    random state against the oracle on the whole lattice."""
    say("fp64 1024x1024 20 steps")
    n = 1024
    c = P.single_1024(0.45, 4, 3)
    rng = np.random.default_rng(9)
    f0 = rng.standard_normal((8, n, n)) * 1e-3
    s = _solver(n, n)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    s.set_populations(dev(f0))
    s.step(20)
    fn = O.run(f0, c.gx, c.gy, omega(c.material), 20)
    assert_elementwise(host(s.populations()), fn, 1e-12, "f")


@functools.lru_cache(maxsize=1)
def _case_8192():
    return P.single_8192()


def _window_oracle(case, om, steps, sites, halo):
    """f(steps) from f = 0 at the given sites, each computed by the oracle on a
    periodic window of half-width `halo` > steps around the site (the light cone
    of a site after n steps has radius n, so the window's own wrap never reaches
    the centre)."""
    w = 2 * halo + 1
    out = []
    for (y, x) in sites:
        ys = (np.arange(y - halo, y + halo + 1)) % case.ny
        xs = (np.arange(x - halo, x + halo + 1)) % case.nx
        gx = np.ascontiguousarray(case.gx[np.ix_(ys, xs)])
        gy = np.ascontiguousarray(case.gy[np.ix_(ys, xs)])
        f = O.run(O.zero_state(w, w), gx, gy, om, steps)
        ux, uy = O.displacement(f, gx, gy)
        out.append((ux[halo, halo], uy[halo, halo]))
    return np.array(out)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5), ("fp16", 2e-2)])
def test_full_size_8192_sampled(prec, tol):
    """8192 x 8192 random 16-mode load in the benchmark's launch configuration:
    displacement after 12 steps at sampled sites (corners and edges included)
    against the oracle evaluated site by site on light-cone windows."""
    say(f"8192x8192 {prec} sampled")
    import torch
    c = _case_8192()
    s = _solver(8192, 8192, prec)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    steps = 12
    s.step(steps)
    ux, uy = s.displacement()
    rng = np.random.default_rng(1)
    sites = [(0, 0), (0, 8191), (8191, 0), (8191, 8191), (4096, 0), (0, 4096)]
    sites += [tuple(int(v) for v in rng.integers(0, 8192, 2)) for _ in range(26)]
    iy = torch.tensor([p[0] for p in sites], device="cuda")
    ix = torch.tensor([p[1] for p in sites], device="cuda")
    got = np.stack([host(ux[iy, ix]), host(uy[iy, ix])], axis=1)
    want = _window_oracle(c, omega(c.material), steps, sites, steps + 2)
    scale = np.max(np.abs(want))
    err = np.max(np.abs(got - want)) / scale
    say(f"  max rel err at {len(sites)} sites: {err:.2e}")
    assert err <= tol


@pytest.mark.parametrize("kind,nx", [("default", 36000), ("default", 35999), ("single", 36000)])
def test_beyond_the_tile_kernel_limit(kind, nx):
    """About 1.08e9 FP32 sites, above the 2^30 whose planes the tile kernel
    addresses with 32-bit offsets: by default such lattices run the register
    wavefront at eight steps (two columns per lane on even widths, one on odd),
    which like single steps addresses the planes with 64-bit offsets.
    Displacement after 6 steps from f = 0 at sampled sites (corners and edges
    included) against the oracle on light-cone windows of the same force values."""
    import torch
    need_gpu()
    ny, steps = 30000, 6
    say(f"{nx}x{ny} fp32 {kind}")
    two_pi = 2.0 * np.pi
    x = torch.arange(nx, dtype=torch.float64, device="cuda") + 0.5
    y = torch.arange(ny, dtype=torch.float64, device="cuda") + 0.5
    gx = 1e-4 * torch.outer(torch.cos(two_pi * 2 * y / ny), torch.sin(two_pi * 3 * x / nx))
    gy = 1e-4 * torch.outer(torch.sin(two_pi * 1 * y / ny), torch.cos(two_pi * 2 * x / nx))
    del x, y
    mat = P.Material.from_shear_poisson(1.0, 0.3)
    s = _solver(nx, ny, "fp32")
    s.set_material(mat.lame_lambda, mat.lame_mu)
    s.set_body_force(gx, gy)
    if kind == "single":
        s.set_time_blocking(1)
    cfg = s.launch_config()
    say(f"  launch config {cfg}")
    if kind == "default":
        assert cfg["kernel"] == "wavefront" and cfg["steps_per_launch"] == 8
        assert cfg["columns_per_lane"] == (2 if nx % 2 == 0 else 1)
    else:
        assert cfg["kernel"] == "single"
    s.step(steps)
    ux, uy = s.displacement()
    rng = np.random.default_rng(3)
    sites = [(0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1), (ny // 2, 0), (0, nx // 2)]
    sites += [(int(rng.integers(0, ny)), int(rng.integers(0, nx))) for _ in range(14)]
    iy = torch.tensor([p[0] for p in sites], device="cuda")
    ix = torch.tensor([p[1] for p in sites], device="cuda")
    got = np.stack([host(ux[iy, ix]), host(uy[iy, ix])], axis=1)
    om = omega(mat)
    halo = steps + 2
    want = []
    for (py, px) in sites:
        ys = torch.tensor((np.arange(py - halo, py + halo + 1)) % ny, device="cuda")
        xs = torch.tensor((np.arange(px - halo, px + halo + 1)) % nx, device="cuda")
        wx, wy = host(gx[ys][:, xs]), host(gy[ys][:, xs])
        f = O.run(O.zero_state(2 * halo + 1, 2 * halo + 1), wx, wy, om, steps)
        ox, oy = O.displacement(f, wx, wy)
        want.append((ox[halo, halo], oy[halo, halo]))
    want = np.array(want)
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    say(f"  max rel err at {len(sites)} sites: {err:.2e}")
    s.close()
    del s, gx, gy, ux, uy
    torch.cuda.empty_cache()
    assert err <= 1e-5


@pytest.mark.parametrize("prec,nx,ny,steps", [
    ("fp64", 1, 1, 6), ("fp64", 3, 5, 7), ("fp64", 67, 33, 21), ("fp64", 130, 9, 10),
    ("fp64", 64, 8, 4), ("fp32", 2, 2, 5), ("fp32", 65, 17, 9), ("fp32", 256, 48, 12),
    ("fp16", 5, 3, 5), ("fp16", 97, 31, 8), ("fp64", 1024, 1024, 6)])
def test_time_blocking_identical_to_single_steps(prec, nx, ny, steps):
    """Two to eight steps per launch (tile + ring in LDS) give bit-identical
    populations to single steps (ragged tiles, lattices smaller than the tile,
    step counts that leave remainders, checks interleaved with fused launches),
    and the FP64 result matches the oracle."""
    say(f"time blocking {prec} {nx}x{ny} steps {steps}")
    mat = P.Material.from_shear_poisson(0.9, 0.3)
    f0, gx, gy = _rand_state(nx, ny, 3 + nx)
    res = {}
    for tb in range(1, 9):
        s = _solver(nx, ny, prec)
        s.set_material(mat.lame_lambda, mat.lame_mu)
        s.set_body_force(dev(gx), dev(gy))
        s.set_populations(dev(f0))
        s.set_time_blocking(tb)
        s.step(steps)
        a = host(s.populations())
        n, r, st = s.solve_to_tol(0.0, 11, 5)  # residual checks between fused launches
        res[tb] = (a, host(s.populations()), n, r)
        s.close()
    for tb in range(2, 9):
        np.testing.assert_array_equal(res[tb][0], res[1][0], err_msg=f"{tb} steps per launch")
        np.testing.assert_array_equal(res[tb][1], res[1][1], err_msg=f"{tb} steps per launch")
        # the residual's summation order follows the tile shape: equal to rounding
        assert res[tb][2] == res[1][2] and res[tb][3] == pytest.approx(res[1][3], rel=1e-12)
    if prec == "fp64":
        fn = O.run(f0, gx, gy, omega(mat), steps)
        assert_elementwise(res[2][0], fn, 1e-12, "f")


@pytest.mark.parametrize("nx,ny,steps", [(3, 5, 9), (65, 17, 11), (200, 70, 13), (130, 49, 17)])
def test_tile_rows_24_identical_to_single_steps(nx, ny, steps):
    """The 24-row FP32 tile (lbm_set_tile_rows) at two to eight steps per launch:
    populations bit-identical to single steps, with the remainder steps (six
    rows per thread on the same work list) and the fused residual check of
    solve_to_tol between its launches."""
    say(f"tile rows 24 fp32 {nx}x{ny} steps {steps}")
    mat = P.Material.from_shear_poisson(0.9, 0.3)
    f0, gx, gy = _rand_state(nx, ny, 11 + nx)
    res = {}
    for tb in range(1, 9):
        s = _solver(nx, ny, "fp32")
        s.set_material(mat.lame_lambda, mat.lame_mu)
        s.set_body_force(dev(gx), dev(gy))
        s.set_populations(dev(f0))
        s.set_time_blocking(tb)
        if tb > 1:
            s.set_fused_kernel("tile", 256)
            s.set_tile_rows(24)
            cfg = s.launch_config()
            assert cfg["rows"] == 24 and cfg["kernel"] == "tile", cfg
        s.step(steps)
        a = host(s.populations())
        n, r, st = s.solve_to_tol(0.0, 11, 5)
        res[tb] = (a, host(s.populations()), n, r)
        s.close()
    for tb in range(2, 9):
        np.testing.assert_array_equal(res[tb][0], res[1][0], err_msg=f"{tb} steps per launch")
        np.testing.assert_array_equal(res[tb][1], res[1][1], err_msg=f"{tb} steps per launch")
        assert res[tb][2] == res[1][2] and res[tb][3] == pytest.approx(res[1][3], rel=1e-12)


def test_tile_rows_argument_errors():
    from paper_2208_14870_amd import lbm
    s = _solver(64, 64, "fp64")
    s.set_time_blocking(5)
    with pytest.raises(lbm.LbmError):
        s.set_tile_rows(24)  # no FP64 kernel of that height
    with pytest.raises(lbm.LbmError):
        s.set_tile_rows(20)
    s.set_tile_rows(0)
    assert s.launch_config()["rows"] == 8
    s.close()


@pytest.mark.parametrize("prec,nx,ny,steps,bpc", [
    ("fp32", 1024, 1024, 12, 1), ("fp32", 1024, 1024, 9, 2), ("fp32", 1000, 998, 11, 3),
    ("fp64", 300, 200, 10, 1), ("fp64", 130, 9, 7, 2), ("fp16", 130, 90, 8, 1),
    ("fp32", 65, 17, 9, 3), ("fp32", 3000, 40, 8, 1), ("fp64", 1024, 1024, 8, 2)])
def test_persistent_tile_identical_to_single_steps(prec, nx, ny, steps, bpc):
    """Persistent fused launches (bpc workgroups per CU, fewer than the tiles:
    each workgroup walks several tiles of the work list) give populations
    bit-identical to single steps, with residual checks interleaved."""
    say(f"persistent tile {prec} {nx}x{ny} steps {steps} blocks/CU {bpc}")
    mat = P.Material.from_shear_poisson(0.9, 0.3)
    f0, gx, gy = _rand_state(nx, ny, 7 + nx)
    res = {}
    for tb in (1, 3, 4):
        s = _solver(nx, ny, prec)
        s.set_material(mat.lame_lambda, mat.lame_mu)
        s.set_body_force(dev(gx), dev(gy))
        s.set_populations(dev(f0))
        if tb > 1:
            s.set_tile(6, 2, bpc)
        s.set_time_blocking(tb)
        s.step(steps)
        a = host(s.populations())
        n, r, st = s.solve_to_tol(0.0, 11, 5)
        res[tb] = (a, host(s.populations()), n, r)
        s.close()
    for tb in (3, 4):
        np.testing.assert_array_equal(res[tb][0], res[1][0])
        np.testing.assert_array_equal(res[tb][1], res[1][1])
        assert res[tb][2] == res[1][2] and res[tb][3] == pytest.approx(res[1][3], rel=1e-12)


@pytest.mark.parametrize("prec,nx,ny,steps,rows", [
    ("fp64", 1, 1, 6, 256), ("fp64", 3, 5, 7, 1), ("fp64", 67, 33, 21, 4), ("fp64", 130, 9, 10, 16),
    ("fp64", 257, 48, 12, 7), ("fp32", 2, 2, 5, 3), ("fp32", 65, 17, 9, 5), ("fp32", 200, 70, 12, 32),
    ("fp16", 5, 3, 5, 2), ("fp16", 97, 31, 8, 9), ("fp64", 1024, 1024, 8, 256),
    ("fp32", 4, 3, 6, 1), ("fp32", 256, 48, 10, 16), ("fp16", 2, 2, 5, 3), ("fp16", 130, 20, 8, 6),
    ("fp32", 1024, 64, 8, 32), ("fp32", 300, 130, 19, 24), ("fp16", 301, 77, 17, 12),
    ("fp64", 260, 90, 17, 20)])
def test_wavefront_identical_to_single_steps(prec, nx, ny, steps, rows):
    """The register-wavefront fused kernel at 2..8 steps per launch (one column
    per lane: strips of 64 - 2k columns; two columns per lane for FP32/FP16 on
    even widths: strips of 128 - 2 ring, the ring 4 up to four steps and k
    rounded up to even above; segments of `rows` rows, several strips and
    segments, ragged edges, lattices narrower than a strip) gives populations
    bit-identical to single steps, with residual checks interleaved; the FP64
    result matches the oracle."""
    say(f"wavefront {prec} {nx}x{ny} steps {steps} rows {rows}")
    mat = P.Material.from_shear_poisson(0.9, 0.3)
    f0, gx, gy = _rand_state(nx, ny, 5 + nx)
    res = {}
    depths = (1, 2, 3, 4, 5, 6, 7, 8)
    for tb in depths:
        s = _solver(nx, ny, prec)
        s.set_material(mat.lame_lambda, mat.lame_mu)
        s.set_body_force(dev(gx), dev(gy))
        s.set_populations(dev(f0))
        s.set_time_blocking(tb)
        s.set_fused_kernel("wavefront", rows)
        s.step(steps)
        a = host(s.populations())
        n, r, st = s.solve_to_tol(0.0, 11, 5)
        res[tb] = (a, host(s.populations()), n, r)
    for tb in depths[1:]:
        np.testing.assert_array_equal(res[tb][0], res[1][0])
        np.testing.assert_array_equal(res[tb][1], res[1][1])
        assert res[tb][2] == res[1][2] and res[tb][3] == pytest.approx(res[1][3], rel=1e-12)
    if prec == "fp64" and nx * ny <= 20000:
        fn = O.run(f0, gx, gy, omega(mat), steps)
        assert_elementwise(res[3][0], fn, 1e-12, "f")


def test_fused_kernel_argument_errors():
    """Steps per launch outside 1..8 and a segment height of 0 are refused; a
    wavefront solver keeps the wavefront at deeper blocking (with two columns
    per lane the ring widens to the depth), with results unchanged."""
    from paper_2208_14870_amd import lbm
    s = _solver(16, 16, "fp32")
    with pytest.raises(lbm.LbmError):
        s.set_fused_kernel("wavefront", 0)
    with pytest.raises(KeyError):
        s.set_fused_kernel("other", 4)
    s.set_fused_kernel("tile")
    for bad in (0, 9):
        with pytest.raises(lbm.LbmError):
            s.set_time_blocking(bad)
    s.set_time_blocking(6)
    s.set_fused_kernel("wavefront", 16)
    assert s.launch_config()["kernel"] == "wavefront"
    mat = P.Material.from_shear_poisson(0.9, 0.3)
    f0, gx, gy = _rand_state(40, 24, 11)
    out = []
    for deep in (False, True):
        s = _solver(40, 24, "fp32")
        s.set_material(mat.lame_lambda, mat.lame_mu)
        s.set_body_force(dev(gx), dev(gy))
        s.set_populations(dev(f0))
        s.set_time_blocking(4)
        s.set_fused_kernel("wavefront", 8)
        if deep:
            s.set_time_blocking(8)  # the wavefront at eight steps
        s.step(16)
        out.append(host(s.populations()))
        s.close()
    np.testing.assert_array_equal(out[0], out[1])


def test_launch_config_defaults():
    """Default plain-step launches: eight steps per launch through the LDS tile
    (16 rows, 512 threads) for FP32 and FP16 above 2^17 sites, four below; FP64
    five steps through 8-row tiles of 512 threads below 458752 sites; the register
    wavefront at eight steps for FP64 from 458752 sites, FP32 from 2^20 (two
    columns per lane from 2^25 on even widths) and FP16 from 2^24, with
    segments as long as one wave per SIMD (1024 on 256 compute units) allows,
    16 to 128 rows (1024^2 FP64: 22 strips of 48 columns, 46 per strip, 23
    rows; 2048^2: 43 strips, 23 per strip, 90 rows); the caller's
    depth keeps the default kernel, the caller's kernel stays; in place the
    in-place wavefront at the deepest depth the workspace has room for (one
    step per launch in the minimal workspace), segments of 256 rows halved
    while the lattice would give fewer than 4096 waves."""
    from paper_2208_14870_amd import lbm
    need_gpu()
    cfg = lambda n, m, p, **kw: lbm.Solver(n, m, p, **kw).launch_config()
    assert cfg(1024, 1000, "fp32") == {"steps_per_launch": 8, "kernel": "tile", "rows": 16,
                                       "threads": 512}
    assert cfg(2048, 1024, "fp16") == {"steps_per_launch": 8, "kernel": "tile", "rows": 16,
                                       "threads": 512}
    assert cfg(256, 256, "fp16") == {"steps_per_launch": 4, "kernel": "tile", "rows": 12,
                                     "threads": 256}
    assert cfg(256, 256, "fp32") == {"steps_per_launch": 4, "kernel": "tile", "rows": 8,
                                     "threads": 512}
    assert cfg(512, 512, "fp64") == {"steps_per_launch": 5, "kernel": "tile", "rows": 8,
                                     "threads": 512}
    for n, m, p, rows, v in ((1024, 1024, "fp64", 23, 1), (1024, 1024, "fp32", 23, 1),
                             (4096, 4096, "fp64", 128, 1),
                             (724, 724, "fp64", 16, 1), (1100, 1100, "fp32", 25, 1),
                             (2048, 2048, "fp64", 90, 1),
                             (2048, 2048, "fp32", 90, 1), (4096, 4096, "fp32", 128, 1),
                             (8192, 8192, "fp32", 128, 2), (8191, 8192, "fp32", 128, 1),
                             (4096, 4096, "fp16", 128, 1)):
        assert cfg(n, m, p) == {"steps_per_launch": 8, "kernel": "wavefront", "rows": rows,
                                "threads": 256, "columns_per_lane": v}, (n, m, p)
    s = lbm.Solver(2900, 2900, "fp64")
    c = s.launch_config()
    assert c["kernel"] == "wavefront" and c["steps_per_launch"] == 8
    s.set_time_blocking(6)
    assert s.launch_config()["kernel"] == "wavefront"
    s.set_time_blocking(3)
    assert s.launch_config()["kernel"] == "wavefront"
    s.set_fused_kernel("tile")
    s.set_time_blocking(4)  # the caller's choice stays
    assert s.launch_config() == {"steps_per_launch": 4, "kernel": "tile", "rows": 8, "threads": 512}
    s.set_time_blocking(1)
    assert s.launch_config()["kernel"] == "single"
    s.close()
    c = cfg(256, 256, "fp32", inplace=True, inplace_steps=1)
    assert c["steps_per_launch"] == 1 and c["kernel"] == "single"
    assert cfg(256, 256, "fp32", inplace=True) == {
        "steps_per_launch": 8, "kernel": "wavefront", "rows": 32, "threads": 256,
        "columns_per_lane": 2}
    assert cfg(256, 255, "fp16", inplace=True, inplace_steps=4) == {
        "steps_per_launch": 4, "kernel": "wavefront", "rows": 32, "threads": 256,
        "columns_per_lane": 2}
    assert cfg(2049, 8192, "fp64", inplace=True)["rows"] == 64  # 43 strips x 128 segments


# ---------------------------------------------------------------------------
# reduced precision (error against the FP64 oracle stated as a number)
# ---------------------------------------------------------------------------

def test_fp32_error_vs_oracle_config_32():
    """FP32 storage + FP32 arithmetic, 32 x 32 solved to r <= 1e-6 (reachable in
    FP32): displacement within 1e-5 relative of the FP64 oracle at the same
    step count.  FP32 rounding (6e-8) amplified by the slowest mode's
    1/(1 - lambda) ~ 30 steps and the residual stopping error stays below it."""
    say("fp32 single-32")
    c = P.single_32()
    s = _solver(32, 32, "fp32")
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    n, r, st = s.solve_to_tol(1e-6, 10000, 1)
    assert st == 0
    f = O.run(O.zero_state(32, 32), c.gx, c.gy, omega(c.material), n)
    ox, oy = O.displacement(f, c.gx, c.gy)
    ux, uy = (host(t) for t in s.displacement())
    err = rel_l2(ux, ox, uy, oy)
    say(f"  fp32 rel err vs fp64 oracle at step {n}: {err:.3e}")
    assert err <= 1e-5


def test_fp32_1024_error_vs_oracle():
    """1024 x 1024, 20 steps from a random state: FP32 within 1e-6 of FP64."""
    say("fp32 1024x1024 20 steps")
    n = 1024
    c = P.single_1024(0.3, 1, 1)
    rng = np.random.default_rng(2)
    f0 = rng.standard_normal((8, n, n)) * 1e-3
    s = _solver(n, n, "fp32")
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    s.set_populations(dev(f0))
    s.step(20)
    fn = O.run(f0, c.gx, c.gy, omega(c.material), 20)
    err = rel_l2(host(s.populations()), fn)
    say(f"  fp32 population rel err: {err:.3e}")
    assert err <= 1e-6


def test_fp16_error_vs_oracle():
    """Scaled FP16 storage, FP32 arithmetic: 64 x 64 manufactured problem
    after 2000 steps; half rounding (4.9e-4) amplified by slow modes -- stated,
    bound 5e-2."""
    say("fp16 64x64")
    c = P.single_1024(0.3, 1, 1, n=64)
    s = _solver(64, 64, "fp16")
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    s.step(2000)
    f = O.run(O.zero_state(64, 64), c.gx, c.gy, omega(c.material), 2000)
    ox, oy = O.displacement(f, c.gx, c.gy)
    ux, uy = (host(t) for t in s.displacement())
    err = rel_l2(ux, ox, uy, oy)
    say(f"  fp16 rel err vs fp64 oracle: {err:.3e}")
    assert err <= 5e-2


@pytest.mark.parametrize("n,scale", [(8, 1e-3), (5, 1e-3), (64, 1.0)])
def test_fp16_set_populations_fits_the_state(n, scale):
    """Half storage picks its power-of-two scale from a state set by the caller:
    a state far above the force's steady-state bound (tiny lattice, large
    populations) neither overflows the half range nor loses its digits; 30
    steps without a check stay finite and within half rounding of the FP64
    oracle."""
    say(f"fp16 set_populations {n}x{n} scale {scale}")
    f0, gx, gy = _rand_state(n, n, 11, scale)
    gx, gy = gx * 1e-2, gy * 1e-2
    mat = P.Material.from_shear_poisson(1.0, 0.3)
    s = _solver(n, n, "fp16")
    s.set_material(mat.lame_lambda, mat.lame_mu)
    s.set_body_force(dev(gx), dev(gy))
    s.set_populations(dev(f0))
    back = host(s.populations())
    assert np.all(np.isfinite(back))
    assert rel_l2(back, f0) <= 1e-3  # stored within half rounding
    s.step(30)
    got = host(s.populations())
    want = O.run(f0, gx, gy, omega(mat), 30)
    err = rel_l2(got, want)
    say(f"  rel err vs fp64 oracle after 30 steps: {err:.3e}")
    assert np.all(np.isfinite(got)) and err <= 3e-3


@pytest.mark.parametrize("order", ["pops_force_material", "material_pops_force", "force_material_pops"])
def test_fp16_set_calls_in_any_order(order):
    """Half storage: the state, force and material may be set in any order
    before the first step.  When a later force or material raises the scale's
    exponent, the stored state is rescaled by that power of two instead of
    being read at the wrong scale; results agree with the usual order to
    subnormal-half rounding and with the FP64 oracle to half rounding."""
    say(f"fp16 set order {order}")
    n = 24
    f0, gx, gy = _rand_state(n, n, 21, 1e-4)
    gx, gy = gx * 100.0, gy * 100.0  # a force whose bound dominates the state's
    mat = P.Material.from_shear_poisson(1.0, 0.3)
    out = []
    for o in (order, "force_material_pops"):
        s = _solver(n, n, "fp16")
        for step in o.split("_"):
            if step == "pops":
                s.set_populations(dev(f0))
            elif step == "force":
                s.set_body_force(dev(gx), dev(gy))
            else:
                s.set_material(mat.lame_lambda, mat.lame_mu)
        s.step(20)
        out.append(host(s.populations()))
        s.close()
    want = O.run(f0, gx, gy, omega(mat), 20)
    scale = np.max(np.abs(want))
    say(f"  max diff between orders {np.max(np.abs(out[0] - out[1])) / scale:.2e}, "
        f"rel err vs oracle {rel_l2(out[0], want):.2e}")
    assert np.max(np.abs(out[0] - out[1])) <= 1e-9 * scale
    assert rel_l2(out[0], want) <= 3e-3


def test_fp16_small_state_without_force_keeps_its_digits():
    """A zero force sets no bound on the half scale: a small state keeps its
    own scale (no subnormal halves)."""
    say("fp16 small state, zero force")
    n = 16
    f0, _, _ = _rand_state(n, n, 22, 1e-6)
    z = np.zeros((n, n))
    mat = P.Material.from_shear_poisson(1.0, 0.3)
    s = _solver(n, n, "fp16")
    s.set_material(mat.lame_lambda, mat.lame_mu)
    s.set_body_force(dev(z), dev(z))
    s.set_populations(dev(f0))
    back = host(s.populations())
    s.step(10)
    got = host(s.populations())
    s.close()
    assert rel_l2(back, f0) <= 1e-3
    assert rel_l2(got, O.run(f0, z, z, omega(mat), 10)) <= 3e-3


def test_fp16_reset_is_a_fresh_solver():
    """After checked runs that rescale half storage, reset gives the exponent a
    fresh solver starts with: the next run is bit-identical to a fresh one."""
    say("fp16 reset")
    c = P.single_1024(0.3, 1, 1, n=64)
    runs = []
    s = _solver(64, 64, "fp16")
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    s.solve_to_tol(1e-4, 3000, 50)
    s.reset()
    s.step(200)
    runs.append(host(s.populations()))
    s.close()
    s = _solver(64, 64, "fp16")
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    s.step(200)
    runs.append(host(s.populations()))
    s.close()
    assert np.array_equal(runs[0], runs[1])


def test_fp16_force_raised_mid_run():
    """Half storage: a force 100 times larger set after 100 steps coarsens the
    scale (the live state is rescaled by the power of two), so 400 plain steps
    without a check stay finite and within half rounding of the oracle."""
    say("fp16 force raised mid-run")
    c = P.single_1024(0.3, 1, 1, n=32)
    om = omega(c.material)
    s = _solver(32, 32, "fp16")
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    s.step(100)
    s.set_body_force(dev(100.0 * c.gx), dev(100.0 * c.gy))
    s.step(400)
    got = host(s.populations())
    s.close()
    f = O.run(O.zero_state(32, 32), c.gx, c.gy, om, 100)
    want = O.run(f, 100.0 * c.gx, 100.0 * c.gy, om, 400)
    err = rel_l2(got, want)
    say(f"  rel err vs oracle {err:.2e}")
    assert np.all(np.isfinite(got)) and err <= 3e-3


def test_fp16_zero_state_keeps_the_force_scale():
    """Setting an all-zero state leaves the scale the force chose: the run is
    bit-identical to a fresh solver's."""
    say("fp16 zero state")
    c = P.single_1024(0.3, 1, 1, n=64)
    out = []
    for set_zero in (False, True):
        s = _solver(64, 64, "fp16")
        s.set_material(c.material.lame_lambda, c.material.lame_mu)
        s.set_body_force(dev(c.gx), dev(c.gy))
        if set_zero:
            s.set_populations(dev(np.zeros((8, 64, 64))))
        s.step(50)
        out.append(host(s.populations()))
    assert np.array_equal(out[0], out[1])


def test_fp32_polish_reaches_fp64_tolerance():
    """FP32 storage with the FP64 polish phase reaches r <= 1e-11 and then agrees
    with the FP64 steady state to the residual's stopping error."""
    say("fp32 polish single-32")
    c = P.single_32()
    s = _solver(32, 32, "fp32", polish=True)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    s.set_polish(1e-6)
    n, r, st = s.solve_to_tol(1e-11, 100000, 1)
    assert st == 0 and r <= 1e-11
    from paper_2208_14870_amd import lbm
    assert s.current_precision == lbm.FP64
    f, on, _, _ = O.solve_to_tol(O.zero_state(32, 32), c.gx, c.gy, omega(c.material), 1e-13,
                                 100000, 1)
    ox, oy = O.displacement(f, c.gx, c.gy)
    ux, uy = (host(t) for t in s.displacement())
    err = rel_l2(ux, ox, uy, oy)
    say(f"  polished rel err vs converged fp64 oracle: {err:.3e}")
    assert err <= 1e-9


@pytest.mark.parametrize("prec,n", [("fp32", 64), ("fp32", 96), ("fp16", 64)])
def test_polish_random_load_converges(prec, n):
    """Random 8-mode load: FP32/FP16 noise excites the undamped staggered modes;
    the switch to FP64 resets them, so the polished solve reaches r <= 1e-10 and
    matches the FP64 oracle at the same step (half storage switches when its
    residual stalls)."""
    say(f"{prec} polish random load {n}")
    req = P.Request(0, 0.0, n, 0.3, 1234)
    c = req.case()
    s = _solver(n, n, prec, polish=True)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    s.set_polish(1e-6)
    steps, r, st = s.solve_to_tol(1e-10, 20000, 100)
    assert st == 0 and r <= 1e-10, (steps, r)
    f = O.run(O.zero_state(n, n), c.gx, c.gy, omega(c.material), steps)
    ox, oy = O.displacement(f, c.gx, c.gy)
    ux, uy = (host(t) for t in s.displacement())
    err = rel_l2(ux, ox, uy, oy)
    say(f"  steps {steps} r {r:.2e} rel err vs oracle {err:.2e}")
    assert err <= 1e-6


# ---------------------------------------------------------------------------
# failure handling
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,K,small", [(48, 1, False), (48, 7, False), (32, 1, True),
                                       (32, 1, False), (32, 64, True)])
def test_divergence_is_reported(n, K, small):
    """Unstable material of Sec. 7.3.5 (nu = -0.4, E~ = 0.082): the residual rise
    rule stops the solve with LBM_E_DIVERGED at the same check step as the
    oracle with the same rule (a few thousand steps at most, long before any
    value overflows), and the state of that step stays readable: its
    displacement equals the oracle's to the rounding of the two sides
    (FMA on the GPU, none in the oracle) times what the unstable modes make of
    it, rho^n with rho = sup rho(L(k)) over the lattice's wavevectors."""
    say(f"fp64 divergence {n}x{n} K {K} one-workgroup {small}")
    from paper_2208_14870_amd import lbm
    c = P.gaussian_hill_case(n, P.Material.from_young_poisson(0.082, -0.4))
    s = _solver(n, n)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    s.set_small_solve(65536 if small else 0)
    with pytest.raises(lbm.Diverged):
        s.solve_to_tol(1e-12, 100000, K)
    steps = s.steps_done
    f, on, orr, ost = O.solve_to_tol(O.zero_state(n, n), c.gx, c.gy, omega(c.material), 1e-12,
                                     100000, K, rise_checks=8)
    say(f"  stopped at step {steps}; oracle {on} (status {ost}, r {orr:.3e})")
    assert ost == -2 and steps == on and steps <= 2500
    ux, uy = (host(t) for t in s.displacement())
    ox, oy = O.displacement(f, c.gx, c.gy)
    from paper_2208_14870_amd import stability
    rho = stability.sup_rho(c.material.lame_lambda, c.material.lame_mu,
                            stability.lattice_grid(n, n))[0]
    bar = max(1e-12, 1e-13 * rho ** steps)
    say(f"  rho {rho:.6f}: rho^n {rho ** steps:.2e}, bar {bar:.1e}")
    assert_elementwise((ux, uy), (ox, oy), bar, "u")


def test_divergence_guard_off_and_argument():
    """With the rise rule off (0 checks) the same unstable solve runs to its step
    limit; a negative count is an argument error."""
    from paper_2208_14870_amd import lbm
    c = P.gaussian_hill_case(32, P.Material.from_young_poisson(0.082, -0.4))
    s = _solver(32, 32)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    with pytest.raises(lbm.LbmError):
        s.set_divergence_guard(-1)
    s.set_divergence_guard(0)
    n, r, st = s.solve_to_tol(1e-12, 3000, 1)
    assert st == 1 and n == 3000 and np.isfinite(r)


def _staggered_load(n, amp=1e-3):
    """Zero-mean load with a smooth part and a k = (pi, 0) component in gx."""
    x = np.arange(n) + 0.5
    X, Y = np.meshgrid(x, x)
    gx = amp * (np.sin(2 * np.pi * X / n) * np.cos(2 * np.pi * Y / n)
                + 0.2 * (-1.0) ** np.arange(n)[None, :])
    gy = amp * np.cos(2 * np.pi * X / n) * np.sin(2 * np.pi * Y / n)
    return gx - gx.mean(), gy - gy.mean()


@pytest.mark.parametrize("n,small", [(16, True), (16, False), (64, False)])
def test_staggered_load_same_outcome_fp64_and_polish(n, small):
    """A load with a k = (pi, 0) component has no steady state from f = 0: the
    staggered first moment oscillates for good.  set_body_force warns
    (LBM_W_STAGGERED_LOAD); FP64 storage and FP32 storage with the FP64 polish
    both end NOT_CONVERGED at the step limit, and since the switch resets the
    undamped modes to the exact trajectory's values, the polished state then
    equals the FP64 oracle's at the same step."""
    from paper_2208_14870_amd import lbm
    need_gpu()
    gx, gy = _staggered_load(n)
    mat = P.Material.from_shear_poisson(1.0, 0.3)
    limit = 3000
    out = {}
    for prec in ("fp64", "fp32"):
        say(f"staggered load {n}x{n} {prec} one-workgroup {small}")
        s = lbm.Solver(n, n, prec, with_polish=(prec == "fp32"))
        s.set_material(mat.lame_lambda, mat.lame_mu)
        w = s.set_body_force(dev(gx), dev(gy))
        assert w == lbm.W_STAGGERED_LOAD, w
        if prec == "fp32":
            s.set_polish(1e-6)
        s.set_small_solve(65536 if small else 0)
        # checks every two steps: the check steps share a parity, so the
        # residual settles at its floor and the "stopped decreasing" switch fires
        steps, r, st = s.solve_to_tol(1e-8, limit, 2)
        out[prec] = (steps, r, st, s.current_precision,
                     tuple(host(t) for t in s.displacement()))
        s.close()
    f, on, orr, ost = O.solve_to_tol(O.zero_state(n, n), gx, gy, omega(mat), 1e-8, limit, 2)
    ox, oy = O.displacement(f, gx, gy)
    say(f"  fp64 {out['fp64'][:3]}, fp32+polish {out['fp32'][:4]}, oracle {(on, orr, ost)}")
    assert ost == 1 and on == limit
    for prec in ("fp64", "fp32"):
        steps, r, st, cur, u = out[prec]
        assert st == 1 and steps == limit and r == pytest.approx(orr, rel=1e-6)
        assert cur == 0  # the polish ran in FP64
        assert_elementwise(u, (ox, oy), 1e-12 if prec == "fp64" else 1e-9, prec)


def test_mean_removed_and_rejected_force():
    """lbm_set_body_force: a force with a mean returns LBM_W_MEAN_REMOVED and
    solves the mean-projected problem (as the oracle does from the numpy
    projection); a non-finite force returns LBM_E_ARG and leaves the previous
    force in place."""
    from paper_2208_14870_amd import lbm
    need_gpu()
    c = P.single_32()
    mat = c.material
    gx = c.gx + 0.25 * np.sqrt(np.mean(c.gx ** 2))
    gy = c.gy.copy()
    for prec, bar in (("fp64", 1e-12), ("fp32", 1e-5)):
        say(f"mean removal {prec}")
        s = lbm.Solver(32, 32, prec)
        s.set_material(mat.lame_lambda, mat.lame_mu)
        assert s.set_body_force(dev(gx), dev(gy)) == lbm.W_MEAN_REMOVED
        bad = gx.copy()
        bad[3, 5] = np.nan
        with pytest.raises(lbm.LbmError):
            s.set_body_force(dev(bad), dev(gy))
        s.step(150)
        ux, uy = (host(t) for t in s.displacement())
        px = gx - gx.mean()
        f = O.run(O.zero_state(32, 32), px, gy, omega(mat), 150)
        ox, oy = O.displacement(f, px, gy)
        if prec == "fp64":
            assert_elementwise((ux, uy), (ox, oy), bar, "u")
        else:
            assert rel_l2(ux, ox, uy, oy) <= bar
        s.close()


def test_stability_check_refuses_unstable_material():
    say("stability check")
    m = P.Material.from_young_poisson(0.082, -0.4)
    s = _solver(48, 48)
    with pytest.raises(ValueError):
        s.set_material(m.lame_lambda, m.lame_mu, check_stability=True)
    ok = P.Material.from_shear_poisson(1.0, 0.3)
    s.set_material(ok.lame_lambda, ok.lame_mu, check_stability=True)


def test_invalid_arguments():
    say("argument validation")
    from paper_2208_14870_amd import lbm
    s = _solver(8, 8)
    with pytest.raises(lbm.LbmError):
        s.set_material(1.0, 0.0)
    with pytest.raises(lbm.LbmError):
        s.set_material(-3.0, 1.0)
    with pytest.raises(lbm.LbmError):
        s.step(1)  # no material / force yet
    s.set_material(1.0, 1.0)
    rng = np.random.default_rng(0)
    w = s.set_body_force(dev(rng.standard_normal((8, 8)) + 1.0), dev(rng.standard_normal((8, 8))))
    assert w & lbm.W_MEAN_REMOVED  # white noise also has staggered components
    with pytest.raises(lbm.LbmError):
        s.set_tile(9, 1)
    with pytest.raises(lbm.LbmError):
        s.solve_to_tol(1e-6, 10, 0)
