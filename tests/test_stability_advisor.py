"""The library's stability tool against the independent per-mode model of the
tests and the paper's stability statements (Sec. 5, Sec. 7.3.5)."""
import math

import numpy as np
import pytest

from paper_2208_14870_amd import problem as P
from paper_2208_14870_amd import stability as ST
import spectral as S


def test_moment_matrix_matches_printed():
    np.testing.assert_array_equal(ST.moment_matrix(), S.printed_M())


@pytest.mark.parametrize("nu,E", [(0.3, 2.6), (-0.4, 0.082), (0.8, 0.11), (0.999, 0.05)])
def test_operator_matches_mode_model(nu, E):
    m = P.Material.from_young_poisson(E, nu)
    A = ST.collision_operator(m.lame_lambda, m.lame_mu)
    mm = S.ModeModel(m.lame_lambda, m.lame_mu)
    np.testing.assert_allclose(A, mm.A, atol=1e-14)
    for kx, ky in ((0.3, 0.1), (math.pi, 0.0), (2.0, 1.5)):
        np.testing.assert_allclose(ST.amplification(A, kx, ky), mm.L(kx, ky), atol=1e-14)


def test_paper_statements():
    m = P.Material.from_young_poisson(0.082, -0.4)
    assert not ST.is_stable(m.lame_lambda, m.lame_mu)
    for nu in (0.05, 0.3, 0.49):
        m = P.Material.from_shear_poisson(1.0, nu)
        assert ST.is_stable(m.lame_lambda, m.lame_mu)
    rng = ST.stable_young_range(-0.4, [0.05, 0.082, 0.2, 1.0])
    assert 0.082 not in rng and 0.2 in rng and 1.0 in rng


def test_lattice_grid_check():
    m = P.Material.from_young_poisson(0.082, -0.4)
    assert not ST.is_stable(m.lame_lambda, m.lame_mu, nx=48, ny=48)


# ---------------------------------------------------------------------------
# accuracy and convergence advisor
# ---------------------------------------------------------------------------
from oracle import oracle as O  # noqa: E402

MAT = P.Material.from_shear_poisson(1.0, 0.3)


@pytest.mark.parametrize("k", [(0.3, 0.1), (2 * math.pi / 32, 2 * math.pi / 32), (1.1, -0.4)])
def test_steady_response_matches_mode_model(k):
    """Against the independent per-mode model of the tests (general rates too)."""
    for kw in ({}, {"theta": 0.4, "w12": 1.2, "w21": 1.2, "w22": 0.8}):
        R = ST.steady_response(MAT.lame_lambda, MAT.lame_mu, *k, **kw)
        mm = S.ModeModel(MAT.lame_lambda, MAT.lame_mu, **kw)
        want = np.stack([mm.steady_u(*k, np.array([1.0, 0.0])),
                         mm.steady_u(*k, np.array([0.0, 1.0]))], axis=1)
        np.testing.assert_allclose(R, want, atol=1e-13)


def test_steady_response_is_the_oracle_steady_state():
    """A one-mode load with both components: the oracle, iterated to r <= 1e-13,
    reaches the field the 2 x 2 response predicts at the nodes (i + 1/2, j + 1/2)."""
    n, kx, ky = 24, 2 * math.pi * 2 / 24, 2 * math.pi * 1 / 24
    ghat = np.array([1e-4, -0.6e-4])
    x = np.arange(n) + 0.5
    ph = np.exp(1j * (kx * x[None, :] + ky * x[:, None]))
    gx, gy = (ghat[0] * ph).real, (ghat[1] * ph).real
    om = O.omega_vector(MAT.lame_lambda, MAT.lame_mu)
    f, steps, r, st = O.solve_to_tol(O.zero_state(n, n), gx, gy, om, 1e-13, 100000, 10)
    ux, uy = O.displacement(f, gx, gy)
    uhat = ST.steady_response(MAT.lame_lambda, MAT.lame_mu, kx, ky) @ ghat
    wx, wy = (uhat[0] * ph).real, (uhat[1] * ph).real
    err = np.sqrt(np.sum((ux - wx) ** 2 + (uy - wy) ** 2) / np.sum(wx ** 2 + wy ** 2))
    assert st == 0 and err <= 1e-9


def test_continuum_response_closed_forms():
    """Shear (g perpendicular to k): u = g / (mu k^2); longitudinal (g along k):
    u = g / ((mu + K) k^2)."""
    K = MAT.lame_lambda + MAT.lame_mu
    k = 0.2
    R = ST.continuum_response(MAT.lame_lambda, MAT.lame_mu, k, 0.0)
    np.testing.assert_allclose(R, np.diag([1 / ((MAT.lame_mu + K) * k * k), 1 / (MAT.lame_mu * k * k)]),
                               rtol=1e-14)


def test_mode_error_is_second_order():
    """The steady-state error of the mode (1, 1) falls by about 4 per halving of the
    spacing (Sec. 7.3.1 reports second order), approaching 4."""
    errs = [ST.mode_error(MAT.lame_lambda, MAT.lame_mu, 2 * math.pi / n, 2 * math.pi / n)
            for n in (16, 32, 64, 128, 256)]
    ratios = [a / b for a, b in zip(errs, errs[1:])]
    assert all(r1 < r2 for r1, r2 in zip(ratios, ratios[1:]))
    assert 3.8 <= ratios[2] <= 4.2 and 3.95 <= ratios[3] <= 4.05


def test_slowest_decay_is_the_shear_mode():
    """For a large lattice the slowest smooth mode decays as 1 - mu k^2 with
    k = 2 pi / n (Sec. 5, long-wave limit)."""
    rho, k = ST.slowest_decay(MAT.lame_lambda, MAT.lame_mu, 256, 256)
    kmin = 2 * math.pi / 256
    assert abs(abs(k[0]) + abs(k[1]) - kmin) < 1e-12
    assert abs(rho - (1 - MAT.lame_mu * kmin ** 2)) <= 2e-6


@pytest.mark.parametrize("n,tol,kind,branch", [(32, 1e-8, "shear", -1), (32, 1e-10, "shear", -1),
                                               (48, 1e-8, "shear", -1), (32, 1e-8, "long", -3)])
def test_predicted_steps_match_the_oracle(n, tol, kind, branch):
    """A one-mode load along x excites one branch of L(k) (shear: the slowest
    eigenvalue; longitudinal: the next slowest pair); the oracle's stop step with
    a check every step equals the prediction from that eigenvalue."""
    x = np.arange(n) + 0.5
    ph = np.sin(2 * math.pi * x / n)[None, :] * np.ones((n, 1))
    z = np.zeros((n, n))
    gx, gy = (z, 1e-4 * ph) if kind == "shear" else (1e-4 * ph, z)
    om = O.omega_vector(MAT.lame_lambda, MAT.lame_mu)
    f, steps, r, st = O.solve_to_tol(O.zero_state(n, n), gx, gy, om, tol, 200000, 1)
    A = ST.collision_operator(MAT.lame_lambda, MAT.lame_mu)
    ev = sorted(np.abs(np.linalg.eigvals(ST.amplification(A, 2 * math.pi / n, 0.0))))
    assert st == 0 and steps == ST.predicted_steps(ev[branch], tol)


def test_advise_picks_the_fastest_stable_accurate_modulus():
    rows, best = ST.advise(-0.4, 48, young=[0.05, 0.082, 0.2, 1.0, 3.0], tol=1e-8,
                           max_error=0.02)
    by = {r["young"]: r for r in rows}
    assert not by[0.082]["stable"] and by[1.0]["stable"]
    ok = [r for r in rows if r["stable"] and r["error_k11"] <= 0.02]
    assert best is not None and best["steps"] == min(r["steps"] for r in ok)
    assert best["young"] != 0.082


def test_advise_by_error_estimate_picks_the_papers_modulus():
    """Sec. 4 / Sec. 7.3.2: picking E~ by the smallest R1 (the estimate with the
    force correction) at nu = 0.8 gives about the 0.085 the paper uses; the
    advisor's R1, R2 are the library's host computation, equal to the oracle's
    (which is pinned against the exact discrete symbols)."""
    young = np.geomspace(0.02, 0.5, 120)
    rows, best = ST.advise(0.8, 40, young=young, criterion="R1")
    assert best is not None and best["stable"]
    assert abs(best["young"] - 0.085) <= 0.1 * 0.085, best["young"]
    for r in rows[::17]:
        want = O.error_estimates(O.leading_error_constants(r["young"], 0.8))
        assert r["R1"] == pytest.approx(want[0], rel=1e-10)
        assert r["R2"] == pytest.approx(want[1], rel=1e-10)
    _, by_r2 = ST.advise(0.8, 40, young=young, criterion="R2")
    assert by_r2["R2"] >= 4.0 * best["R1"]
    with pytest.raises(ValueError):
        ST.advise(0.8, 40, young=young, criterion="fast")
