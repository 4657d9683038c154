"""The autotuner picks a valid launch shape and the results do not change."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_14870_amd import problem as P
from gpu_common import assert_elementwise, dev, host, need_gpu, omega, rel_l2, say

pytestmark = pytest.mark.gpu


def test_tune_solver_and_cache(tmp_path):
    say("autotune solver 256x256 fp64")
    need_gpu()
    from paper_2208_14870_amd import autotune, lbm
    c = P.single_1024(0.3, 1, 1, n=256)
    s = lbm.Solver(256, 256, "fp64")
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    cache = str(tmp_path / "tune.json")
    cands = autotune.solver_candidates(s, "fp64")
    assert cands == autotune.candidates(256, 0, 256, wavefront=True, precision="fp64")
    shp = autotune.tune_solver(s, "fp64", cache_path=cache)
    assert shp in cands
    assert autotune.tune_solver(s, "fp64", cache_path=cache) == shp  # from the cache
    s.reset()
    s.step(50)
    f = O.run(O.zero_state(256, 256), c.gx, c.gy, omega(c.material), 50)
    ox, oy = O.displacement(f, c.gx, c.gy)
    ux, uy = (host(t) for t in s.displacement())
    assert_elementwise((ux, uy), (ox, oy), 1e-12, "u")


def test_tune_batch(tmp_path):
    say("autotune batch")
    need_gpu()
    from paper_2208_14870_amd import autotune, lbm
    cases = P.batch_cases(6, seed=4, sides=(64, 96, 128))
    b = lbm.Batch(16, 1 << 30)
    for c in cases:
        b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(c.gx), dev(c.gy), "fp32")
    shp = autotune.tune_batch(b, "fp32", sum(c.nx * c.ny for c in cases),
                              cache_path=str(tmp_path / "t.json"))
    assert shp in autotune.batch_candidates()


def test_tune_inplace_solver(tmp_path):
    """In-place solvers are tuned over single-step shapes and the in-place
    wavefront shapes their halo room admits; the tuned solver's populations
    equal the two-buffer solver's single steps bit for bit.  With the minimal
    workspace only single-step shapes remain."""
    say("autotune in-place solver 128x128 fp32")
    need_gpu()
    from paper_2208_14870_amd import autotune, lbm
    c = P.single_1024(0.3, 1, 1, n=128)
    ref = lbm.Solver(128, 128, "fp32")
    ref.set_time_blocking(1)
    ref.set_material(c.material.lame_lambda, c.material.lame_mu)
    ref.set_body_force(dev(c.gx), dev(c.gy))
    ref.step(37)
    want = host(ref.populations())
    ref.close()
    for room in (8, 1):
        s = lbm.Solver(128, 128, "fp32", inplace=True, inplace_steps=room)
        s.set_material(c.material.lame_lambda, c.material.lame_mu)
        s.set_body_force(dev(c.gx), dev(c.gy))
        cands = autotune.solver_candidates(s, "fp32")
        shp = autotune.tune_solver(s, "fp32", cache_path=str(tmp_path / f"t{room}.json"))
        assert shp in cands
        if room == 1:
            assert shp[3] == 1 and shp[4] == 0
        s.reset()
        s.step(37)
        np.testing.assert_array_equal(host(s.populations()), want)
        s.close()


def test_solver_candidates_include_the_default_wavefront():
    """A solver whose default plain-step kernel is the wavefront (1024^2 FP32:
    eight steps, 23-row segments) has that shape among the tuner's candidates;
    a tile-kernel solver (512^2 FP32) has the plain candidate list."""
    need_gpu()
    from paper_2208_14870_amd import autotune, lbm
    s = lbm.Solver(1024, 1024, "fp32")
    assert autotune.solver_candidates(s, "fp32")[0] == (6, 4, 0, 8, 23, 0)
    s.close()
    s = lbm.Solver(512, 512, "fp32")
    assert autotune.solver_candidates(s, "fp32") == autotune.candidates(
        512, 0, 512, wavefront=True, precision="fp32")
    s.close()
