"""Batched lattices (one persistent launch per step over a tile work list)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_14870_amd import problem as P
from gpu_common import assert_elementwise, dev, host, need_gpu, omega, rel_l2, say

pytestmark = pytest.mark.gpu

GIB = 1 << 30


def _batch(max_slots=16, arena=GIB):
    from paper_2208_14870_amd import lbm
    need_gpu()
    return lbm.Batch(max_slots, arena)


def _cases():
    specs = [(64, 64, 0.3, (1, 1)), (96, 96, 0.1, (2, 1)), (33, 65, 0.45, (1, 2)),
             (128, 40, 0.2, (3, 1)), (7, 5, 0.3, (1, 1)), (192, 192, 0.48, (4, 3))]
    out = []
    for nx, ny, nu, (kx, ky) in specs:
        mat = P.Material.from_shear_poisson(1.0, nu)
        u = P.trig_product((1e-3, 1e-3), ("s", "c"), ("c", "s"), 2 * np.pi * kx / nx,
                           2 * np.pi * ky / ny)
        out.append(P.manufactured_case(nx, mat, u, f"b{nx}x{ny}", ny=ny))
    return out


def test_batch_fp64_matches_oracle():
    say("batch fp64 6 lattices 40 steps")
    b = _batch()
    cases = _cases()
    slots = [b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(c.gx), dev(c.gy),
                   "fp64") for c in cases]
    b.step(40)
    for c, s in zip(cases, slots):
        f = O.run(O.zero_state(c.nx, c.ny), c.gx, c.gy, omega(c.material), 40)
        ox, oy = O.displacement(f, c.gx, c.gy)
        ux, uy = (host(t) for t in b.displacement(s))
        assert_elementwise((ux, uy), (ox, oy), 1e-12, c.label)


def test_batch_residual_matches_single_solver_and_oracle():
    """Residual of a checked chunk equals the single-lattice solver's and the
    oracle's r(n - 1) after n steps."""
    say("batch fp64 residual")
    from paper_2208_14870_amd import lbm
    c = _cases()[1]
    b = _batch()
    s = b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(c.gx), dev(c.gy), "fp64")
    b.step(30, check=True)
    r, n = b.residuals()
    assert n[s] == 30
    f29 = O.run(O.zero_state(c.nx, c.ny), c.gx, c.gy, omega(c.material), 28)
    u28 = O.displacement(f29, c.gx, c.gy)
    f29 = O.run(f29, c.gx, c.gy, omega(c.material), 1)
    u29 = O.displacement(f29, c.gx, c.gy)
    want = O.residual(u29[0], u29[1], u28[0], u28[1])
    assert r[s] == pytest.approx(want, rel=1e-9)


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp16"])
def test_alone_vs_mix_identical(prec):
    """A lattice gives bit-identical displacement and residual alone and in a mix."""
    say(f"batch alone vs mix {prec}")
    cases = _cases()
    probe = cases[2]
    b1 = _batch()
    s1 = b1.add(probe.nx, probe.ny, probe.material.lame_lambda, probe.material.lame_mu,
                dev(probe.gx), dev(probe.gy), prec)
    b1.step(100, check=True)
    r1, _ = b1.residuals()
    u1 = [host(t) for t in b1.displacement(s1)]
    b2 = _batch()
    ids = {}
    for c in cases:
        ids[c.label] = b2.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu,
                              dev(c.gx), dev(c.gy), prec)
    b2.step(100, check=True)
    r2, _ = b2.residuals()
    u2 = [host(t) for t in b2.displacement(ids[probe.label])]
    np.testing.assert_array_equal(u1[0], u2[0])
    np.testing.assert_array_equal(u1[1], u2[1])
    assert r1[s1] == r2[ids[probe.label]]


def test_mixed_precisions_match_single_solvers():
    """One batch holding FP64, FP32 and FP16 lattices (each precision its own
    launch per step) gives every lattice the displacement of a single-lattice
    solver of the same precision, bit for bit."""
    say("batch mixed precisions vs single solvers")
    from paper_2208_14870_amd import lbm
    cases = _cases()
    precs = ["fp64", "fp32", "fp16", "fp32", "fp16", "fp64"]
    b = _batch()
    slots = [b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(c.gx), dev(c.gy),
                   p) for c, p in zip(cases, precs)]
    b.step(37)
    for c, p, sl in zip(cases, precs, slots):
        s = lbm.Solver(c.nx, c.ny, p)
        s.set_material(c.material.lame_lambda, c.material.lame_mu)
        s.set_body_force(dev(c.gx), dev(c.gy))
        s.step(37)
        for a, t in zip(b.displacement(sl), s.displacement()):
            np.testing.assert_array_equal(host(a), host(t), err_msg=f"{p} {c.label}")
        s.close()


def test_per_precision_time_blocking():
    """Each storage type runs its own steps per launch (and keeps its own
    launch parity): FP64 at 3, FP32 at 7, FP16 at 1 then 5 steps per launch,
    with residual checks and a promotion of a polish lattice in between, give
    every lattice the populations of a batch stepping once per launch."""
    say("batch per-precision time blocking")
    from paper_2208_14870_amd import lbm
    cases = _cases()
    precs = ["fp64", "fp32", "fp16", "fp32", "fp16", "fp64"]
    runs = []
    for mixed in (False, True):
        b = _batch()
        slots = [b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(c.gx),
                       dev(c.gy), p, with_polish=(p != "fp64")) for c, p in zip(cases, precs)]
        if mixed:
            b.set_time_blocking(3, "fp64")
            b.set_time_blocking(7, "fp32")
            b.set_time_blocking(1, "fp16")
            for bad in (0, 9):
                with pytest.raises(lbm.LbmError):
                    b.set_time_blocking(bad, "fp32")
            with pytest.raises(KeyError):
                b.set_time_blocking(4, "bf16")
        else:
            b.set_time_blocking(1)
        b.step(23, check=True)
        r1, _ = b.residuals()
        b.promote(slots[1])
        if mixed:
            b.set_time_blocking(5, "fp16")
        b.step(30)
        b.step(17, check=True)
        r2, n2 = b.residuals()
        u = [tuple(host(t) for t in b.displacement(sl)) for sl in slots]
        runs.append((u, [r1[sl] for sl in slots], [r2[sl] for sl in slots], [n2[sl] for sl in slots]))
        b.close()
    (u0, a0, b0, n0), (u1, a1, b1, n1) = runs
    assert n0 == n1 == [70] * len(cases)
    for k, p in enumerate(precs):
        for x, y in zip(u0[k], u1[k]):
            np.testing.assert_array_equal(x, y, err_msg=f"{p} {cases[k].label}")
        for r0, r1_ in ((a0[k], a1[k]), (b0[k], b1[k])):
            assert np.isfinite(r0) and r1_ == pytest.approx(r0, rel=1e-12)


@pytest.mark.parametrize("chunks", [(200, 201), (13, 9), (16, 2)])
def test_fused_check_equals_single_step_check(chunks):
    """A checked chunk ends in one fused launch whose last two steps form the
    residual check (a full launch, the remainder, or a full launch after one
    single step): displacements equal those of a batch that checks with single
    steps, residuals equal to rounding (their summation follows the launch)."""
    say(f"batch fused check {chunks}")
    cases = _cases()
    precs = ["fp32", "fp64", "fp16", "fp32", "fp64", "fp16"]
    runs = []
    for tb in (1, 8):
        b = _batch()
        slots = [b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(c.gx),
                       dev(c.gy), p) for c, p in zip(cases, precs)]
        b.set_time_blocking(tb)
        out = []
        for n in chunks:
            b.step(n, check=True)
            r, steps = b.residuals()
            out.append(([r[sl] for sl in slots], [steps[sl] for sl in slots]))
        u = [tuple(host(t) for t in b.displacement(sl)) for sl in slots]
        runs.append((out, u))
        b.close()
    (o1, u1), (o8, u8) = runs
    for (r1, n1), (r8, n8) in zip(o1, o8):
        assert n1 == n8
        for a, b_ in zip(r1, r8):
            assert np.isfinite(a) and b_ == pytest.approx(a, rel=1e-12, abs=1e-300)
    for k, p in enumerate(precs):
        for x, y in zip(u1[k], u8[k]):
            np.testing.assert_array_equal(x, y, err_msg=f"{p} {cases[k].label}")


def test_displacements_of_several_slots():
    """One copy of several lattices' displacements (page-locked host memory)
    equals the per-slot reads, for mixed precisions and shapes."""
    say("batch displacements of several slots")
    cases = _cases()
    precs = ["fp64", "fp32", "fp16", "fp32", "fp16", "fp64"]
    b = _batch()
    slots = [b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(c.gx), dev(c.gy),
                   p) for c, p in zip(cases, precs)]
    b.step(21)
    pick = [slots[4], slots[0], slots[2], slots[5]]
    many = b.displacements(pick)
    assert b.displacements([]) == []
    for sl, (hx, hy) in zip(pick, many):
        ux, uy = b.displacement(sl)
        assert hx.shape == tuple(ux.shape) and hy.shape == tuple(uy.shape)
        np.testing.assert_array_equal(hx, host(ux))
        np.testing.assert_array_equal(hy, host(uy))
    b.close()


def test_deferred_work_list():
    """Adds and removals between steps only mark the work list stale: several of
    them followed by one step give the same results as single solvers; reading
    a displacement right after an add (FP16: its scale is set from the force
    read back at the rebuild) works; a lattice not yet checked reports NaN."""
    say("batch deferred rebuild")
    from paper_2208_14870_amd import lbm
    cases = _cases()
    precs = ["fp16", "fp32", "fp64", "fp16", "fp32", "fp64"]
    b = _batch()
    s0 = b.add(cases[0].nx, cases[0].ny, cases[0].material.lame_lambda,
               cases[0].material.lame_mu, dev(cases[0].gx), dev(cases[0].gy), "fp16",
               with_polish=True)
    got = b.displacement(s0)  # forces the rebuild before any step
    ref = lbm.Solver(cases[0].nx, cases[0].ny, "fp16", with_polish=True)
    ref.set_material(cases[0].material.lame_lambda, cases[0].material.lame_mu)
    ref.set_body_force(dev(cases[0].gx), dev(cases[0].gy))
    for a, t in zip(got, ref.displacement()):  # zero populations: half the force term
        np.testing.assert_array_equal(host(a), host(t))
    ref.close()
    slots = {0: s0}
    for i in (1, 2, 3):
        c = cases[i]
        slots[i] = b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(c.gx),
                         dev(c.gy), precs[i])
    b.remove(slots.pop(2))
    b.remove(slots.pop(3))
    for i in (4, 5):
        c = cases[i]
        slots[i] = b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(c.gx),
                         dev(c.gy), precs[i])
    b.step(20, check=True)
    r, n = b.residuals()
    for i, sl in slots.items():
        assert n[sl] == 20 and np.isfinite(r[sl])
        c = cases[i]
        s = lbm.Solver(c.nx, c.ny, precs[i])
        s.set_material(c.material.lame_lambda, c.material.lame_mu)
        s.set_body_force(dev(c.gx), dev(c.gy))
        s.step(20)
        for a, t in zip(b.displacement(sl), s.displacement()):
            np.testing.assert_array_equal(host(a), host(t), err_msg=f"{precs[i]} {c.label}")
        s.close()
    late = b.add(cases[2].nx, cases[2].ny, cases[2].material.lame_lambda,
                 cases[2].material.lame_mu, dev(cases[2].gx), dev(cases[2].gy), "fp32")
    r, n = b.residuals()
    assert n[late] == 0 and np.isnan(r[late])


def test_join_and_leave_mid_run():
    """Lattices added later and removals do not disturb the others."""
    say("batch join/leave")
    cases = _cases()
    b = _batch()
    a = b.add(cases[0].nx, cases[0].ny, cases[0].material.lame_lambda, cases[0].material.lame_mu,
              dev(cases[0].gx), dev(cases[0].gy), "fp64")
    x = b.add(cases[3].nx, cases[3].ny, cases[3].material.lame_lambda, cases[3].material.lame_mu,
              dev(cases[3].gx), dev(cases[3].gy), "fp64")
    b.step(17)
    b.remove(x)
    c = cases[4]
    late = b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(c.gx), dev(c.gy),
                 "fp64")
    b.step(23)
    for case, slot, n in ((cases[0], a, 40), (c, late, 23)):
        f = O.run(O.zero_state(case.nx, case.ny), case.gx, case.gy, omega(case.material), n)
        ox, oy = O.displacement(f, case.gx, case.gy)
        ux, uy = (host(t) for t in b.displacement(slot))
        assert_elementwise((ux, uy), (ox, oy), 1e-12, "u")


def test_promote_to_fp64():
    """FP32 lattice with polish reservation switches to FP64 mid-run."""
    say("batch promote")
    c = _cases()[0]
    b = _batch()
    s = b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(c.gx), dev(c.gy),
              "fp32", with_polish=True)
    b.step(200)
    b.promote(s)
    b.step(300)
    f = O.run(O.zero_state(c.nx, c.ny), c.gx, c.gy, omega(c.material), 500)
    ox, oy = O.displacement(f, c.gx, c.gy)
    ux, uy = (host(t) for t in b.displacement(s))
    err = rel_l2(ux, ox, uy, oy)
    say(f"  fp32->fp64 rel err vs oracle: {err:.3e}")
    assert err <= 1e-5


def test_arena_admission():
    """A lattice that does not fit is refused and nothing changes."""
    say("batch admission")
    from paper_2208_14870_amd import lbm
    per = lbm.Batch.slot_bytes(256, 256, "fp32")
    b = _batch(max_slots=64, arena=64 << 20)
    c = P.single_1024(0.3, 1, 1, n=256)
    got = []
    while True:
        s = b.add(256, 256, c.material.lame_lambda, c.material.lame_mu, dev(c.gx), dev(c.gy),
                  "fp32")
        if s is None:
            break
        got.append(s)
    assert 1 <= len(got) <= (64 << 20) // per
    active, used, largest = b.info()
    assert active == len(got) and largest < per
    b.remove(got[0])
    assert b.add(256, 256, c.material.lame_lambda, c.material.lame_mu, dev(c.gx), dev(c.gy),
                 "fp32") is not None


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_force_projection_equals_solo(prec):
    """A batch slot mean-projects its force on the device by the rule of
    lbm_set_body_force: its populations equal a solo solver's given the same
    force bit for bit, and lbm_batch_force_warnings reports the same bits."""
    from paper_2208_14870_amd import lbm
    c = _cases()[3]  # 128 x 40
    gx = c.gx + 0.4 * np.sqrt(np.mean(c.gx ** 2))
    gy = c.gy + 0.05e-3 * (-1.0) ** np.arange(c.ny)[:, None]  # a (0, pi) component
    say(f"batch force projection {prec}")
    b = _batch()
    slot = b.add(c.nx, c.ny, c.material.lame_lambda, c.material.lame_mu, dev(gx), dev(gy), prec)
    other = b.add(64, 64, c.material.lame_lambda, c.material.lame_mu,
                  dev(np.zeros((64, 64))), dev(np.zeros((64, 64))), prec)
    assert b.force_warnings(slot) == lbm.W_MEAN_REMOVED | lbm.W_STAGGERED_LOAD
    assert b.force_warnings(other) == 0
    b.step(37)
    s = lbm.Solver(c.nx, c.ny, prec)
    s.set_material(c.material.lame_lambda, c.material.lame_mu)
    assert s.set_body_force(dev(gx), dev(gy)) == lbm.W_MEAN_REMOVED | lbm.W_STAGGERED_LOAD
    s.step(37)
    ua = [host(t) for t in b.displacement(slot)]
    ub = [host(t) for t in s.displacement()]
    assert all(np.array_equal(a, bb) for a, bb in zip(ua, ub))
    if prec == "fp64":
        px = gx - gx.mean()
        f = O.run(O.zero_state(c.nx, c.ny), px, gy - gy.mean(), omega(c.material), 37)
        assert_elementwise(tuple(ua), O.displacement(f, px, gy - gy.mean()), 1e-12, "u")
    s.close()
    b.close()


def test_batch_divergence_flag():
    """The batch's divergence guard: an unstable lattice (Sec. 7.3.5) is flagged
    after its update norm kept rising over checked chunks, its neighbour is not,
    and the neighbour's state equals a batch without the unstable lattice."""
    from paper_2208_14870_amd import lbm
    say("batch divergence flag")
    bad = P.gaussian_hill_case(32, P.Material.from_young_poisson(0.082, -0.4))
    good = _cases()[0]
    b = _batch()
    sb = b.add(32, 32, bad.material.lame_lambda, bad.material.lame_mu, dev(bad.gx), dev(bad.gy),
               "fp64")
    sg = b.add(good.nx, good.ny, good.material.lame_lambda, good.material.lame_mu,
               dev(good.gx), dev(good.gy), "fp64")
    ref = _batch()
    rg = ref.add(good.nx, good.ny, good.material.lame_lambda, good.material.lame_mu,
                 dev(good.gx), dev(good.gy), "fp64")
    flagged_at = None
    for chunk in range(60):
        b.step(20, check=True)
        ref.step(20, check=True)
        b.residuals()
        flags = b.diverged()
        assert not flags[sg]
        if flags[sb] and flagged_at is None:
            flagged_at = (chunk + 1) * 20
            break
    say(f"  flagged after {flagged_at} steps")
    assert flagged_at is not None and flagged_at <= 1200
    ua = [host(t) for t in b.displacement(sg)]
    ub = [host(t) for t in ref.displacement(rg)]
    assert all(np.array_equal(a, bb) for a, bb in zip(ua, ub))
    b.close()
    ref.close()
