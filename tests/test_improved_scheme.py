"""Pins of the oracle's improved and fourth-order schemes (Sec. 4, Sec. 7.3.2,
Sec. 7.3.3, App. B, App. C).

The constants of the leading-order error (App. B) are checked against the
exact scheme itself: tests/spectral.py reads them off the slow two-mode law of
the one-step operator built from the printed M and Table "scheme" (mpmath, 60
digits, |k| = 1e-7), independently of the oracle's transcription.  The
schemes built on them are checked against what the paper reports: the error
reduction of the force correction and fourth-order convergence in the special
case, on real-space oracle runs to steady state.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_14870_amd import problem as P
import spectral as S

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
FACTS = json.load(open(os.path.join(GOLD, "paper_facts.json")))

# (material, theta, w12, w21, w22): the paper's E1 point, a general-rate point
# with theta != 1/3 and tau_12 != tau_21, and a negative Poisson ratio
CONSTANT_CASES = [
    (P.Material.from_young_poisson(0.11, 0.8), 1.0 / 3.0, 1.0, 1.0, 1.0),
    (P.Material.from_young_poisson(0.9, 0.3), 0.25, 0.7, 1.3, 0.9),
    (P.Material.from_young_poisson(1.1, -0.5), 0.6, 1.2, 0.8, 1.7),
]


@pytest.mark.parametrize("case", range(len(CONSTANT_CASES)))
def test_constants_equal_the_exact_scheme(case):
    """C1..C5, D1..D3 of both rows (App. B with the readings listed in the
    oracle) against the symbols of the exact scheme, to 1e-9 relative."""
    mat, th, w12, w21, w22 = CONSTANT_CASES[case]
    sx, sy = S.leading_error_symbols(mat.lame_lambda, mat.lame_mu, th, w12, w21, w22)
    ox, oy = O.material_error_constants(mat.lame_lambda, mat.lame_mu, th, w12, w21, w22)
    for got, want in ((ox, sx), (oy, sy)):
        for key in want:
            assert abs(got[key] - want[key]) <= 1e-9 * abs(want[key]), (key, got[key], want[key])


def test_fourth_order_rates_cancel_c1_and_c5():
    """App. C's tau_12 = tau_21 cancels C5 and the oracle's tau_22 cancels C1,
    as read off the exact scheme (both far below the other constants)."""
    mat = P.Material.from_young_poisson(0.085, 0.8)
    w12, w21, w22 = O.fourth_order_rates(mat.lame_lambda, mat.lame_mu)
    assert w12 == w21 and 0.0 < w12 < 2.0 and 0.0 < w22 < 2.0
    sx, _ = S.leading_error_symbols(mat.lame_lambda, mat.lame_mu, 1.0 / 3.0, w12, w21, w22)
    scale = max(abs(sx[k]) for k in ("C2", "C3", "C4"))
    assert abs(sx["C1"]) <= 1e-10 * scale and abs(sx["C5"]) <= 1e-10 * scale, sx


def _steady_error(case, rates=(1.0, 1.0, 1.0), correction=None):
    """Oracle steady state (r <= 1e-13) of a manufactured case; returns the
    relative Linf error against the continuum solution (max over both
    components of |u - u_exact|, over max |u_exact|)."""
    m = case.material
    om = O.omega_vector(m.lame_lambda, m.lame_mu, w12=rates[0], w21=rates[1], w22=rates[2])
    gx, gy = case.gx, case.gy
    if correction is not None:
        cx, cy = O.material_error_constants(m.lame_lambda, m.lame_mu, w12=rates[0],
                                            w21=rates[1], w22=rates[2])
        if correction == "analytic":
            d2x, d2y = case.d2gx, case.d2gy
        else:
            d2x, d2y = O.central_second_derivatives(gx), O.central_second_derivatives(gy)
        gx, gy = O.corrected_force(gx, gy, d2x, d2y, cx, cy)
    f, n, r, st = O.solve_to_tol(O.zero_state(case.nx, case.ny), gx, gy, om, 1e-13, 400000, 100)
    assert st == 0, (n, r)
    ux, uy = O.displacement(f, gx, gy)
    ref = max(np.abs(case.ux_exact).max(), np.abs(case.uy_exact).max())
    return max(np.abs(ux - case.ux_exact).max(), np.abs(uy - case.uy_exact).max()) / ref


def test_improved_scheme_error_reduction():
    """Sec. 7.3.2: the corrected force at E~ = 0.085 against the standard
    scheme at E~ = 0.11 (nu = 0.8, 20 nodes per side).  The paper reports
    roughly an order of magnitude; the exact scheme gives 7.6 at this size
    (7.9 at 40), so the band is [6, 10].  The correction with the printed
    sign of the constants (the opposite sign) makes the error larger than
    without any correction."""
    fx = FACTS["e2_improved_scheme"]
    assert (fx["poisson"], fx["young_dimless"]) == (0.8, 0.085)
    e_std = _steady_error(P.paper_e1(20))
    case = P.paper_e2(20)
    e_imp = _steady_error(case, correction="analytic")
    assert 6.0 <= e_std / e_imp <= 10.0, (e_std, e_imp)
    # the opposite sign: negate the constants
    m = case.material
    cx, cy = O.material_error_constants(m.lame_lambda, m.lame_mu)
    flip = lambda c: {k: -v for k, v in c.items()}
    gx, gy = O.corrected_force(case.gx, case.gy, case.d2gx, case.d2gy, flip(cx), flip(cy))
    om = O.omega_vector(m.lame_lambda, m.lame_mu)
    f, n, r, st = O.solve_to_tol(O.zero_state(20, 20), gx, gy, om, 1e-13, 400000, 100)
    ux, uy = O.displacement(f, gx, gy)
    e_flip = max(np.abs(ux - case.ux_exact).max(), np.abs(uy - case.uy_exact).max()) / max(
        np.abs(case.ux_exact).max(), np.abs(case.uy_exact).max())
    assert e_flip > _steady_error(case), e_flip


def test_improved_scheme_with_central_differences():
    """The correction from second-order central differences of the sampled
    load instead of analytic derivatives: the difference is O(k^4), so the
    error reduction stays (6.9 at 20 nodes) and the error still falls by about
    4 per halving (second order)."""
    e_std = _steady_error(P.paper_e1(20))
    e20 = _steady_error(P.paper_e2(20), correction="central")
    e40 = _steady_error(P.paper_e2(40), correction="central")
    assert e_std / e20 >= 6.0, (e_std, e20)
    assert 3.6 <= e20 / e40 <= 4.4, (e20, e40)


def test_fourth_order_special_case():
    """Sec. 7.3.3: with the fourth-order rates and the force correction, the
    load without mixed derivatives converges at fourth order (the paper's
    commented table: 4.00 in both displacement norms).  Ratios per halving from
    10 to 20 to 40 nodes: the exact scheme gives 15.6 and 15.98."""
    fx = FACTS["e3_fourth_order"]
    assert fx["convergence_orders_commented_table"]["linf_disp"] == 4.0
    m = P.paper_e3(10).material
    rates = O.fourth_order_rates(m.lame_lambda, m.lame_mu)
    errs = [_steady_error(P.paper_e3(n), rates, "analytic") for n in (10, 20, 40)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 14.5 <= r1 <= 17.5 and 15.5 <= r2 <= 16.5, errs
    assert math.log2(r2) >= 3.95
    # the same load with the standard rates (and the correction) stays second order
    e20s = _steady_error(P.paper_e3(20), correction="analytic")
    e40s = _steady_error(P.paper_e3(40), correction="analytic")
    assert 3.6 <= e20s / e40s <= 4.4


def test_error_estimate_picks_the_papers_modulus():
    """Sec. 4 / Sec. 7.3.2: minimising R1 (the error left after the force
    correction) over E~ at nu = 0.8 gives about the E~ = 0.085 the paper uses
    for the improved scheme (0.083 here), and the minimum of R2 (no
    correction) is several times larger (the paper's order of magnitude)."""
    E = np.geomspace(0.02, 0.5, 400)
    r = np.array([O.error_estimates(O.leading_error_constants(e, 0.8)) for e in E])
    e_r1 = E[np.argmin(r[:, 0])]
    assert abs(e_r1 - 0.085) <= 0.1 * 0.085, e_r1
    assert r[:, 1].min() / r[:, 0].min() >= 4.0
