"""Checks of the seeded input generators (continuum problem, not the scheme)."""
import math

import numpy as np
import pytest

from paper_2208_14870_amd import problem as P


def _fd_operator(ux, uy, mat):
    """-mu lap(u) - K grad(div u) by 4th-order periodic central differences
    (lattice spacing 1)."""
    def d1(a, ax):
        return (-np.roll(a, -2, ax) + 8 * np.roll(a, -1, ax) - 8 * np.roll(a, 1, ax)
                + np.roll(a, 2, ax)) / 12.0

    def d2(a, ax):
        return (-np.roll(a, -2, ax) + 16 * np.roll(a, -1, ax) - 30 * a + 16 * np.roll(a, 1, ax)
                - np.roll(a, 2, ax)) / 12.0
    X, Y = 1, 0
    lapx = d2(ux, X) + d2(ux, Y)
    lapy = d2(uy, X) + d2(uy, Y)
    div = d1(ux, X) + d1(uy, Y)
    return (-(mat.lame_mu * lapx + mat.bulk * d1(div, X)),
            -(mat.lame_mu * lapy + mat.bulk * d1(div, Y)))


@pytest.mark.parametrize("maker", [
    lambda: P.single_32(),
    lambda: P.single_1024(0.45, 4, 3, n=128),
    lambda: P.paper_e1(64),
    lambda: P.random_load_case(96, 8, 4, 7, P.Material.from_shear_poisson(1.0, 0.2)),
])
def test_manufactured_force_matches_finite_differences(maker):
    """Eq. manu_eq: the analytic load equals -mu lap(u) - K grad(div u) of the
    sampled solution up to the finite-difference truncation error."""
    c = maker()
    bx, by = _fd_operator(c.ux_exact, c.uy_exact, c.material)
    scale = max(np.max(np.abs(c.gx)), np.max(np.abs(c.gy)))
    h4 = (2 * math.pi * 8 / c.nx) ** 4  # (k h)^4 of the highest mode present
    assert np.max(np.abs(bx - c.gx)) <= max(h4, 1e-12) * scale
    assert np.max(np.abs(by - c.gy)) <= max(h4, 1e-12) * scale


def test_trig_product_evaluation():
    n = 20
    a = 2 * math.pi / n
    f = P.trig_product((0.3, -0.7), ("c", "s"), ("s", "c"), a, 2 * a)
    ux, uy = f.evaluate(n, n)
    x = np.arange(n) + 0.5
    X, Y = np.meshgrid(x, x)
    np.testing.assert_allclose(ux, 0.3 * np.cos(a * X) * np.sin(2 * a * Y), atol=1e-15)
    np.testing.assert_allclose(uy, -0.7 * np.sin(a * X) * np.cos(2 * a * Y), atol=1e-15)


def test_material_relations():
    """Eq. material_relations (2D): lambda = E nu/(1-nu^2), mu = E/(2(1+nu)),
    K = E/(2(1-nu))."""
    m = P.Material.from_young_poisson(0.11, 0.8)
    assert m.lame_mu == pytest.approx(0.11 / 3.6)
    assert m.bulk == pytest.approx(0.11 / 0.4)
    assert m.poisson == pytest.approx(0.8)
    m2 = P.Material.from_shear_poisson(1.0, 0.3)
    assert m2.lame_lambda == pytest.approx(2 * 0.3 / 0.7)
    assert m2.bulk == pytest.approx(1.3 / 0.7)


def test_random_load_rms_and_solution():
    mat = P.Material.from_shear_poisson(1.0, 0.3)
    load, sol = P.random_fourier_load(128, 16, 8, 3, mat)
    ux, uy = sol.evaluate(128, 128)
    assert math.sqrt(np.mean(ux ** 2 + uy ** 2)) == pytest.approx(1e-3, rel=1e-10)
    again = P.body_force_of(sol, mat)
    np.testing.assert_allclose(again.amp, load.amp, rtol=1e-12, atol=1e-20)


def test_seeded_generators_are_deterministic():
    a = P.batch_cases(6, seed=4)
    b = P.batch_cases(6, seed=4)
    assert [c.label for c in a] == [c.label for c in b]
    np.testing.assert_array_equal(a[3].gx, b[3].gx)
    r1 = P.request_stream(2000.0, 0.05, seed=5)
    r2 = P.request_stream(2000.0, 0.05, seed=5)
    assert [(r.n, r.nu, r.seed) for r in r1] == [(r.n, r.nu, r.seed) for r in r2]
    assert all(64 <= r.n <= 2048 for r in r1)


def test_loads_are_mean_free():
    for c in (P.single_32(), P.paper_e1(20), P.batch_cases(3)[1]):
        assert abs(np.mean(c.gx)) < 1e-18 and abs(np.mean(c.gy)) < 1e-18
