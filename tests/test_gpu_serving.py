"""Continuous-batching server: admission by footprint, per-request retirement,
identical results alone and in the mix."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_14870_amd import problem as P
from gpu_common import need_gpu, omega, rel_l2, say

pytestmark = pytest.mark.gpu


def _requests():
    rng = np.random.default_rng(11)
    sizes = [64, 72, 96, 64, 128, 80, 96, 112, 64, 144]
    return [P.Request(i, 0.01 * i, n, float(rng.uniform(0.05, 0.49)), int(rng.integers(1 << 30)))
            for i, n in enumerate(sizes)]


def _server(arena=1 << 30, **kw):
    from paper_2208_14870_amd.serving import Server
    need_gpu()
    return Server(arena, max_slots=64, chunk=100, tol=1e-8, keep_results=True, **kw)


@pytest.mark.parametrize("policy", ["fifo", "hrrn"])
def test_serving_completes_and_alone_equals_mix(policy):
    """Every request completes, and each result equals the same request served
    alone, whatever the admission order."""
    say(f"serving mix of 10 + 3 alone ({policy})")
    reqs = _requests()
    cases = {r.rid: r.case() for r in reqs}
    srv = _server(policy=policy)
    stats = srv.run(reqs, admit_window_s=10.0, wall_budget_s=60.0, cases=cases)
    srv.close()
    assert stats["completed"] == len(reqs) and stats["backlog"] == 0 and stats["failed"] == 0
    mix = {r.rid: r for r in srv.results}
    for rid in (0, 4, 9):
        alone = _server()
        req = [r for r in reqs if r.rid == rid][0]
        st = alone.run([P.Request(rid, 0.0, req.n, req.nu, req.seed)], 10.0, 60.0, cases=cases)
        alone.close()
        assert st["completed"] == 1
        a, m = alone.results[0], mix[rid]
        say(f"  rid {rid} n {req.n}: steps alone {a.steps} mix {m.steps}, promoted {a.promoted_at}")
        assert a.steps == m.steps and a.promoted_at == m.promoted_at
        np.testing.assert_array_equal(a.ux, m.ux)
        np.testing.assert_array_equal(a.uy, m.uy)
        assert a.residual == m.residual


def test_serving_result_matches_oracle():
    """FP32 phase + FP64 polish result against the FP64 oracle at the same step."""
    say("serving vs oracle")
    req = P.Request(0, 0.0, 64, 0.3, 1234)
    case = req.case()
    srv = _server()
    srv.run([req], 1.0, 30.0, cases={0: case})
    srv.close()
    res = srv.results[0]
    assert res.residual <= 1e-8
    f = O.run(O.zero_state(64, 64), case.gx, case.gy, omega(case.material), res.steps)
    ox, oy = O.displacement(f, case.gx, case.gy)
    err = rel_l2(res.ux, ox, res.uy, oy)
    say(f"  steps {res.steps}, promoted at {res.promoted_at}, rel err vs oracle {err:.2e}")
    assert err <= 1e-6


@pytest.mark.parametrize("policy", ["fifo", "hrrn"])
def test_serving_admission_respects_footprint(policy):
    """An arena that holds only a few lattices at once still serves everything."""
    say(f"serving small arena ({policy})")
    from paper_2208_14870_amd import lbm
    reqs = _requests()
    per = lbm.Batch.slot_bytes(144, 144, "fp32", True)
    srv = _server(arena=3 * per + (8 << 20), policy=policy)
    stats = srv.run(reqs, 10.0, 60.0, cases={r.rid: r.case() for r in reqs})
    srv.close()
    assert stats["completed"] == len(reqs)
    # arrival order is kept except for backfilling
    assert all(x.latency >= 0 for x in srv.results)


def test_serving_retires_a_diverging_request():
    """A request whose material is linearly unstable (Sec. 7.3.5: nu = -0.4,
    E~ = 0.082, Gaussian-hill load) grows until the batch's divergence guard
    flags it; the server then retires it as failed and frees its slot, while
    the requests beside it finish exactly as they do alone."""
    say("serving with one diverging request")
    reqs = [P.Request(0, 0.0, 64, 0.3, 77), P.Request(1, 0.0, 48, 0.0, 0),
            P.Request(2, 0.0, 72, 0.2, 78)]
    cases = {0: reqs[0].case(), 2: reqs[2].case(),
             1: P.gaussian_hill_case(48, P.Material.from_young_poisson(0.082, -0.4))}
    from paper_2208_14870_amd.serving import Server
    need_gpu()
    srv = Server(1 << 30, max_slots=16, chunk=1000, tol=1e-8, keep_results=True)
    stats = srv.run(reqs, admit_window_s=1.0, wall_budget_s=90.0, cases=cases)
    active, _, _ = srv.batch.info()
    srv.close()
    say(f"  {stats['completed']} completed, failed {srv.failed}, backlog {stats['backlog']}")
    assert srv.failed == [1] and stats["completed"] == 2 and stats["backlog"] == 0
    assert active == 0
    for rid in (0, 2):
        alone = Server(1 << 30, max_slots=16, chunk=1000, tol=1e-8, keep_results=True)
        alone.run([reqs[rid]], 1.0, 60.0, cases=cases)
        alone.close()
        a = alone.results[0]
        m = [r for r in srv.results if r.rid == rid][0]
        assert a.steps == m.steps and a.residual == m.residual
        np.testing.assert_array_equal(a.ux, m.ux)
        np.testing.assert_array_equal(a.uy, m.uy)
