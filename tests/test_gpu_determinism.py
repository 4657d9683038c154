"""Rerun identity: the same work in fresh solvers or batches gives the same bits
(populations, residual history, displacement).  Every reduction is a fixed-order
two-stage sum without atomics, and every fused kernel rounds a site exactly as a
single step does, so a rerun that differs would point to a race."""
import numpy as np
import pytest

from paper_2208_14870_amd import problem as P
from gpu_common import dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def _single(prec, n, m, chunks):
    from paper_2208_14870_amd import lbm
    c = P.random_load_case(n, 8, 4, 5, P.Material.from_shear_poisson(1.0, 0.3), "rerun", False)
    s = lbm.Solver(n, n, prec)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    s.set_body_force(dev(c.gx), dev(c.gy))
    hist = [s.step_checked(m) for _ in range(chunks)]
    f = host(s.populations())
    ux, uy = (host(t) for t in s.displacement())
    cfg = s.launch_config()
    s.close()
    return hist, f, ux, uy, cfg


@pytest.mark.parametrize("prec,n", [("fp64", 300), ("fp32", 512), ("fp16", 512), ("fp32", 2048)])
def test_single_solver_rerun_identity(prec, n):
    need_gpu()
    a = _single(prec, n, 37, 4)
    b = _single(prec, n, 37, 4)
    say(f"{prec} {n}^2 ({a[4]['kernel']}, {a[4]['steps_per_launch']} steps per launch): "
        f"residuals {a[0]}")
    assert a[0] == b[0]
    for x, y in zip(a[1:4], b[1:4]):
        assert np.array_equal(x, y)


def _batch():
    from paper_2208_14870_amd import lbm
    cases = P.batch_cases(12, seed=9)
    b = lbm.Batch(32, 1 << 30)
    slots = []
    for i, c in enumerate(cases):
        prec = ("fp32", "fp64", "fp16")[i % 3]
        slots.append(b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu,
                           dev(c.gx), dev(c.gy), prec))
    hist = []
    for _ in range(3):
        b.step(50, check=True)
        r, _ = b.residuals()
        hist.append([r[s] for s in slots])
    out = [tuple(host(t) for t in b.displacement(s)) for s in slots]
    b.close()
    return hist, out


def test_batch_rerun_identity():
    need_gpu()
    ha, oa = _batch()
    hb, ob = _batch()
    say(f"batch residuals after 3 chunks: {ha[-1][:4]} ...")
    assert ha == hb
    for (ax, ay), (bx, by) in zip(oa, ob):
        assert np.array_equal(ax, bx) and np.array_equal(ay, by)
