"""The library used from plain C (tests/capi_consumer.c, built by build()): the
32 x 32 manufactured problem solved to tolerance through include/lbm.h with
device memory from the HIP runtime, no Python binding and no torch, against
the oracle."""
import json
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_14870_amd import problem as P
from gpu_common import assert_elementwise, need_gpu, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "capi_consumer")


@pytest.mark.parametrize("precision,tol,bar", [(0, 1e-10, 1e-12), (1, 1e-6, 1e-5)])
def test_c_consumer_solves_to_tolerance(tmp_path, precision, tol, bar):
    need_gpu()
    assert os.path.exists(EXE), "C consumer not built (run __graft_entry__.build())"
    case = P.single_32()
    mat = case.material
    fin, fout = str(tmp_path / "force.bin"), str(tmp_path / "u.bin")
    np.concatenate([case.gx.ravel(), case.gy.ravel()]).astype(np.float64).tofile(fin)
    say(f"C consumer, precision {precision}, tol {tol}")
    r = subprocess.run([EXE, "32", "32", repr(mat.lame_lambda), repr(mat.lame_mu), str(precision),
                        repr(tol), "10000", "1", fin, fout],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    u = np.fromfile(fout, dtype=np.float64).reshape(2, 32, 32)
    om = O.omega_vector(mat.lame_lambda, mat.lame_mu)
    f, n, res, st = O.solve_to_tol(O.zero_state(32, 32), case.gx, case.gy, om, tol, 10000, 1)
    ox, oy = O.displacement(f, case.gx, case.gy)
    err = np.sqrt(np.sum((u[0] - ox) ** 2 + (u[1] - oy) ** 2) / np.sum(ox ** 2 + oy ** 2))
    say(f"  C: steps {rec['steps']} r {rec['residual']:.3e} | oracle steps {n} | rel diff {err:.2e}")
    assert rec["status"] == 0 and st == 0 and rec["force_status"] == 0
    if precision == 0:
        assert rec["steps"] == n
    assert err <= bar


def test_c_consumer_mean_removed(tmp_path):
    """A force with a non-zero mean: the library subtracts the FP64 mean
    (LBM_W_MEAN_REMOVED) and solves the mean-free problem, which the oracle
    solves from the numpy-projected force."""
    need_gpu()
    assert os.path.exists(EXE), "C consumer not built (run __graft_entry__.build())"
    case = P.single_32()
    mat = case.material
    gx = case.gx + 0.3 * np.sqrt(np.mean(case.gx ** 2))
    gy = case.gy - 0.1 * np.sqrt(np.mean(case.gy ** 2))
    fin, fout = str(tmp_path / "force.bin"), str(tmp_path / "u.bin")
    np.concatenate([gx.ravel(), gy.ravel()]).astype(np.float64).tofile(fin)
    say("C consumer, force with a mean")
    r = subprocess.run([EXE, "32", "32", repr(mat.lame_lambda), repr(mat.lame_mu), "0",
                        "1e-10", "10000", "1", fin, fout],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["force_status"] == 2 and rec["status"] == 0
    u = np.fromfile(fout, dtype=np.float64).reshape(2, 32, 32)
    px, py = gx - gx.mean(), gy - gy.mean()
    om = O.omega_vector(mat.lame_lambda, mat.lame_mu)
    f, n, res, st = O.solve_to_tol(O.zero_state(32, 32), px, py, om, 1e-10, 10000, 1)
    ox, oy = O.displacement(f, px, py)
    assert st == 0 and rec["steps"] == n
    assert_elementwise((u[0], u[1]), (ox, oy), 1e-12, "u")


@pytest.mark.parametrize("precision", [0, 1])
def test_c_consumer_inplace_blocked(tmp_path, precision):
    """From plain C: an in-place solver with room for eight steps per launch
    (lbm_workspace_bytes_inplace_blocked, lbm_create_inplace) takes the in-place
    wavefront and reaches the two-buffer solver's stop step, residual and
    displacement exactly; the minimal in-place workspace runs one step per
    launch to the same result."""
    need_gpu()
    assert os.path.exists(EXE), "C consumer not built (run __graft_entry__.build())"
    case = P.single_1024(0.3, 4, 3, n=96)
    mat = case.material
    fin = str(tmp_path / "force.bin")
    np.concatenate([case.gx.ravel(), case.gy.ravel()]).astype(np.float64).tofile(fin)
    tol = 1e-9 if precision == 0 else 1e-6
    out = {}
    for ip in (0, 1, 8):
        fout = str(tmp_path / f"u{ip}.bin")
        say(f"C consumer 96x96, precision {precision}, inplace_steps {ip}")
        r = subprocess.run([EXE, "96", "96", repr(mat.lame_lambda), repr(mat.lame_mu),
                            str(precision), repr(tol), "40000", "37", fin, fout, str(ip)],
                           capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stderr
        rec = json.loads(r.stdout.strip().splitlines()[-1])
        out[ip] = (rec, np.fromfile(fout, dtype=np.float64))
    assert out[8][0]["steps_per_launch"] == 8 and out[8][0]["kernel"] == 1
    assert out[1][0]["steps_per_launch"] == 1
    for ip in (1, 8):
        assert out[ip][0]["status"] == out[0][0]["status"] == 0
        assert out[ip][0]["steps"] == out[0][0]["steps"]
        assert out[ip][0]["residual"] == pytest.approx(out[0][0]["residual"], rel=1e-12)
        np.testing.assert_array_equal(out[ip][1], out[0][1])
