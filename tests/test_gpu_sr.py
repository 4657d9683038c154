"""Stochastic rounding of half storage (lbm_set_stochastic_rounding).

FP16 storage has no oracle parity (the oracle is FP64); what is tested here is
the HIP path against itself and against the FP64 path: every kernel rounds a
population of a given (site, step) with the same random bits, so fused
launches are bit-identical to single steps and reruns repeat; and the
rounding is unbiased, so the FP16 result follows the FP64 one far closer than
round-to-nearest storage does once the slow modes' per-step changes fall
below half an ulp.
"""
import numpy as np
import pytest

from paper_2208_14870_amd import problem as P
from gpu_common import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def _lbm():
    from paper_2208_14870_amd import lbm
    return lbm


def _solver(nx, ny, prec="fp16", **kw):
    need_gpu()
    return _lbm().Solver(nx, ny, prec, **kw)


def _setup(s, mat, gx, gy):
    s.set_material(mat.lame_lambda, mat.lame_mu)
    s.set_body_force(dev(gx), dev(gy))


def _load(nx, ny, seed, mat):
    load, _ = P.random_fourier_load(nx, 8, 3, seed, mat, ny=ny)
    gx, gy = load.evaluate(nx, ny)
    return P.remove_mean(gx), P.remove_mean(gy)


@pytest.mark.parametrize("nx,ny,steps", [(100, 72, 37), (64, 16, 24), (33, 65, 19), (300, 200, 41)])
def test_sr_fused_identical_to_single_steps(nx, ny, steps):
    """Two to eight steps per launch, through the LDS tile and the register
    wavefront, round every population as single steps do (ragged tiles and
    strips, wrapped rings, a residual check and the half rescale between fused
    launches); another seed gives other bits."""
    say(f"stochastic rounding fused vs single {nx}x{ny} steps {steps}")
    mat = P.Material.from_shear_poisson(0.8, 0.3)
    gx, gy = _load(nx, ny, 5 + nx, mat)
    res = {}
    runs = [(1, "tile")] + [(tb, k) for tb in (2, 5, 8) for k in ("tile", "wavefront")]
    for tb, kind in runs:
        s = _solver(nx, ny)
        _setup(s, mat, gx, gy)
        s.set_stochastic_rounding(True, 1234)
        s.set_time_blocking(tb)
        s.set_fused_kernel(kind, 16)
        s.step(steps)
        a = host(s.populations())
        n, r, st = s.solve_to_tol(0.0, 13, 6)  # checks (and rescales) between launches
        res[(tb, kind)] = (a, host(s.populations()), n)
        s.close()
    ref = res[(1, "tile")]
    for key in runs[1:]:
        np.testing.assert_array_equal(res[key][0], ref[0], err_msg=f"{key}")
        np.testing.assert_array_equal(res[key][1], ref[1], err_msg=f"{key}")
        assert res[key][2] == ref[2]
    s = _solver(nx, ny)
    _setup(s, mat, gx, gy)
    s.set_stochastic_rounding(True, 99)
    s.step(steps)
    other = host(s.populations())
    s.close()
    assert not np.array_equal(other, ref[0])


def test_sr_rerun_and_reset_repeat():
    """A second run after lbm_reset, and a second solver, give the same bits;
    switching the rounding off gives round-to-nearest again."""
    mat = P.Material.from_shear_poisson(1.0, 0.3)
    gx, gy = _load(128, 128, 3, mat)
    s = _solver(128, 128)
    _setup(s, mat, gx, gy)
    s.set_stochastic_rounding(True, 7)
    s.step(200)
    a = host(s.populations())
    s.reset()
    s.step(200)
    b = host(s.populations())
    np.testing.assert_array_equal(a, b)
    s.set_stochastic_rounding(False, 7)
    s.reset()
    s.step(200)
    c = host(s.populations())
    s.close()
    t = _solver(128, 128)
    _setup(t, mat, gx, gy)
    t.step(200)
    np.testing.assert_array_equal(c, host(t.populations()))
    t.close()
    assert not np.array_equal(a, c)


def test_sr_follows_fp64_where_rne_stalls():
    """512^2, a smooth 8-mode load from rest, 12000 steps: the slow modes change
    by less than half an ulp per step late in the run, so round-to-nearest
    storage lags the FP64 run; stochastic rounding stays within a few times
    its noise level.  Both errors are against the FP64 GPU run at the same step
    (relative L2 of u); stochastic rounding must be at least 3x closer."""
    n, steps = 512, 12000
    mat = P.Material.from_shear_poisson(1.0, 0.3)
    gx, gy = _load(n, n, 3, mat)
    u = {}
    for key, prec, sr in (("fp64", "fp64", False), ("rne", "fp16", False), ("sr", "fp16", True)):
        s = _solver(n, n, prec)
        _setup(s, mat, gx, gy)
        if sr:
            s.set_stochastic_rounding(True, 11)
        s.step(steps)
        u[key] = [host(t) for t in s.displacement()]
        s.close()
    rx, ry = u["fp64"]
    den = float(np.sum(rx ** 2 + ry ** 2))
    err = {k: float(np.sqrt(np.sum((u[k][0] - rx) ** 2 + (u[k][1] - ry) ** 2) / den))
           for k in ("rne", "sr")}
    say(f"  rel L2 vs FP64 after {steps} steps at {n}^2: {err}")
    assert err["sr"] * 3.0 <= err["rne"], err
    assert err["sr"] <= 1e-3, err


def test_sr_argument_errors():
    lbm = _lbm()
    s = _solver(32, 32, "fp32")
    with pytest.raises(lbm.LbmError) as ei:
        s.set_stochastic_rounding(True)
    assert ei.value.code == lbm.E_STATE
    s.close()
    t = _solver(32, 32, "fp16", inplace=True)
    with pytest.raises(lbm.LbmError):
        t.set_stochastic_rounding(True)
    t.close()
    u = _solver(256, 256, "fp16")
    u.set_stochastic_rounding(True)
    u.set_time_blocking(4)
    u.set_fused_kernel("wavefront", 64)
    assert u.launch_config()["kernel"] == "wavefront"
    u.close()
