"""Admission order of the serving loop (host logic, no GPU): arrival order,
and highest response ratio next with predicted work from the slowest mode."""
import pytest

from paper_2208_14870_amd import problem as P
from paper_2208_14870_amd.serving import admission_order, predicted_work


def _req(rid, t, n=64):
    return P.Request(rid, t, n, 0.3, rid)


def test_fifo_keeps_arrival_order():
    w = [(_req(2, 0.3), 1e9), (_req(0, 0.1), 5e12), (_req(1, 0.2), 1e6)]
    assert [r.rid for r, _ in admission_order(w, 1.0, 1e11, "fifo")] == [0, 1, 2]


def test_hrrn_takes_small_jobs_first_and_ages_large_ones():
    rate = 1e11  # site-updates per second
    # arrived together: the smaller predicted work goes first
    w = [(_req(0, 0.0), 1e12), (_req(1, 0.0), 1e9), (_req(2, 0.0), 1e10)]
    assert [r.rid for r, _ in admission_order(w, 0.5, rate, "hrrn")] == [1, 2, 0]
    # a large request (S = 10 s) that has waited 100 s (ratio 11) goes before a
    # small one that just arrived (ratio 1): no starvation
    w = [(_req(0, 0.0), 1e12), (_req(1, 100.0), 1e9)]
    assert [r.rid for r, _ in admission_order(w, 100.0, rate, "hrrn")] == [0, 1]
    # the same large request after 1 s of waiting (ratio 1.1) yields to the small
    # one after 1 s (ratio 101)
    w = [(_req(0, 0.0), 1e12), (_req(1, 0.0), 1e9)]
    assert [r.rid for r, _ in admission_order(w, 1.0, rate, "hrrn")] == [1, 0]
    with pytest.raises(ValueError):
        admission_order(w, 1.0, rate, "lifo")


def test_predicted_work_scales_as_n4():
    """Steps of the slowest (shear) mode, 1 - rho = mu k^2 with k = 2 pi / n,
    are ln(mu k^2 / tol) / (mu k^2): n^2 up to a logarithm, so the work grows
    like n^4 less a logarithmic factor (x16 per doubling, minus ~10-15 %)."""
    m = P.Material.from_shear_poisson(1.0, 0.3)
    w = [predicted_work(n, m.lame_lambda, m.lame_mu, 1e-8) for n in (128, 256, 512)]
    assert all(x > 0 for x in w)
    for a, b in zip(w, w[1:]):
        assert 13.0 < b / a < 16.0
