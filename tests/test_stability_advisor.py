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
