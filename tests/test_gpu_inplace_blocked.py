"""Temporal blocking in place (the in-place register wavefront with halo
copies): identical to single steps bit for bit for every depth, lane width,
segment height and starting layout, on ragged, narrow and short lattices."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_14870_amd import problem as P
from gpu_common import assert_elementwise, dev, host, need_gpu, omega, say

pytestmark = pytest.mark.gpu


def _rand(nx, ny, seed, scale=1e-3):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((8, ny, nx)) * scale
    gx = P.remove_mean(rng.standard_normal((ny, nx)) * scale * 0.1)
    gy = P.remove_mean(rng.standard_normal((ny, nx)) * scale * 0.1)
    return f, gx, gy


def _solver(nx, ny, prec, mat, gx, gy, f0, inplace, tb, hs=None):
    from paper_2208_14870_amd import lbm
    s = lbm.Solver(nx, ny, prec, inplace=inplace, inplace_steps=max(tb, 2),
                   inplace_segment_rows=hs or 0)
    s.set_material(mat.lame_lambda, mat.lame_mu)
    s.set_body_force(dev(gx), dev(gy))
    s.set_populations(dev(f0))
    if hs is not None and inplace:
        # the segment height first (one step per launch meanwhile), so that
        # the depth is checked against the room for this height
        s.set_time_blocking(1)
        s.set_fused_kernel("wavefront", hs)
    s.set_time_blocking(tb)
    return s


# (precision, nx, ny, steps per launch, segment rows or None for the default)
CASES = [
    ("fp64", 67, 33, 8, None), ("fp64", 48, 40, 8, 16), ("fp64", 49, 9, 5, 3),
    ("fp64", 5, 3, 8, 1), ("fp64", 1, 1, 4, None), ("fp64", 100, 70, 2, 32),
    ("fp32", 300, 70, 8, 32), ("fp32", 112, 64, 8, None), ("fp32", 114, 37, 7, 10),
    ("fp32", 2, 6, 8, 2), ("fp32", 65, 17, 6, None), ("fp32", 256, 48, 3, 16),
    ("fp32", 120, 20, 4, 7),
    ("fp16", 97, 31, 8, None), ("fp16", 240, 50, 4, 16), ("fp16", 4, 4, 8, 1),
    ("fp16", 130, 66, 5, 33),
]


@pytest.mark.parametrize("prec,nx,ny,tb,hs", CASES)
def test_blocked_inplace_identical_to_single_steps(prec, nx, ny, tb, hs):
    """Step counts 1, 2, 5, 8, 13, 3 (cumulative odd and even, so launches
    start from both layouts and remainders run as shorter launches or single
    steps): populations, displacement and stress equal the two-buffer
    solver's single steps exactly; FP64 matches the oracle."""
    need_gpu()
    say(f"blocked inplace {prec} {nx}x{ny} tb {tb} hs {hs}")
    mat = P.Material.from_shear_poisson(0.8, 0.3)
    f0, gx, gy = _rand(nx, ny, 3 + nx + ny)
    a = _solver(nx, ny, prec, mat, gx, gy, f0, False, 1)
    b = _solver(nx, ny, prec, mat, gx, gy, f0, True, tb, hs)
    cfg = b.launch_config()
    assert cfg["steps_per_launch"] == tb and cfg["kernel"] == "wavefront"
    if hs is not None:
        assert cfg["rows"] == hs
    done = 0
    for n in (1, 2, 5, 8, 13, 3):
        a.step(n)
        b.step(n)
        done += n
        np.testing.assert_array_equal(host(b.populations()), host(a.populations()),
                                      err_msg=f"after {done} steps")
    for ta, tb_ in zip(a.displacement(), b.displacement()):
        np.testing.assert_array_equal(host(tb_), host(ta))
    for ta, tb_ in zip(a.stress(), b.stress()):
        np.testing.assert_array_equal(host(tb_), host(ta))
    if prec == "fp64" and nx * ny <= 5000:
        fn = O.run(f0, gx, gy, omega(mat), done)
        assert_elementwise(host(b.populations()), fn, 1e-12, "f")
    a.close()
    b.close()


@pytest.mark.parametrize("prec,K", [("fp64", 7), ("fp32", 50), ("fp16", 25), ("fp64", 64)])
def test_blocked_inplace_solve_to_tol(prec, K):
    """solve_to_tol through blocked launches: the two-buffer solver's stop
    step, residual and state."""
    need_gpu()
    say(f"blocked inplace solve {prec} K={K}")
    from paper_2208_14870_amd import lbm
    c = P.single_1024(0.3, 1, 1, n=96)
    res = []
    for inplace in (False, True):
        s = lbm.Solver(96, 96, prec, inplace=inplace, inplace_steps=8)
        s.set_material(c.material.lame_lambda, c.material.lame_mu)
        s.set_body_force(dev(c.gx), dev(c.gy))
        s.set_time_blocking(1 if not inplace else 8)
        tol = {"fp64": 1e-10, "fp32": 1e-6, "fp16": 1e-3}[prec]
        r = s.solve_to_tol(tol, 60000, K)
        res.append((r, host(s.populations())))
        s.close()
    (ra, fa), (rb, fb) = res
    assert ra[0] == rb[0] and ra[2] == rb[2]
    assert rb[1] == pytest.approx(ra[1], rel=1e-12)
    np.testing.assert_array_equal(fb, fa)


def test_blocked_inplace_large_lattice():
    """A 2048 x 1536 FP32 lattice at the default in-place shape (eight steps,
    two columns per lane) against the two-buffer default (the fused kernels,
    which equal single steps): 37 steps, every population."""
    need_gpu()
    say("blocked inplace 2048x1536 fp32")
    from paper_2208_14870_amd import lbm
    nx, ny = 2048, 1536
    mat = P.Material.from_shear_poisson(1.0, 0.3)
    load, _ = P.random_fourier_load(nx, 8, 3, 12, mat, ny=ny)
    gx, gy = load.evaluate(nx, ny)
    gx, gy = P.remove_mean(gx), P.remove_mean(gy)
    out = []
    for inplace in (False, True):
        s = lbm.Solver(nx, ny, "fp32", inplace=inplace)
        s.set_material(mat.lame_lambda, mat.lame_mu)
        s.set_body_force(dev(gx), dev(gy))
        if inplace:
            cfg = s.launch_config()
            assert cfg["kernel"] == "wavefront" and cfg["steps_per_launch"] == 8
            assert cfg["columns_per_lane"] == 2
        s.step(37)
        out.append(host(s.populations()))
        s.close()
    np.testing.assert_array_equal(out[1], out[0])
