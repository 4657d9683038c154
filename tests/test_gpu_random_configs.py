"""Seeded random configurations of the whole solver surface.

Single lattices: random shapes (1..300 per side), storage types, fused kernels
(LDS tile at 2..8 steps per launch, register wavefront at 2..8 with random
segment heights, in-place streaming one step per launch and blocked through
the in-place wavefront), random step counts and residual-checked
runs, each against the same lattice stepped once per launch: populations and
displacement bit-identical, the checked residual equal to rounding of its
reduction order (the partial sums follow the tile shape), and FP64 within 1e-12
of the oracle on small lattices.

Solves: solve_to_tol under random check intervals and depths, with and
without the FP64 polish, gives the same stop step and state as single steps.

Outputs: populations, displacement, stress and error norms after random step
counts (two buffers or in place) against the oracle and numpy.

Batches: random mixes of lattices with a depth per storage type, plain and
checked chunks, removals and late additions; every lattice still resident
equals a solo solver stepped as many steps (bit-identical; half storage to
1e-9 of max |u|, since checks rescale it and subnormal halves round apart).
"""
import json

import numpy as np
import pytest

from oracle import oracle as O
from paper_2208_14870_amd import problem as P
from gpu_common import assert_elementwise, dev, host, need_gpu, say

pytestmark = pytest.mark.gpu


def _side(rng):
    r = rng.random()
    if r < 0.25:
        return int(rng.integers(1, 9))
    if r < 0.7:
        return int(rng.integers(9, 140))
    return int(rng.integers(140, 300))


def _material(rng):
    return P.Material.from_shear_poisson(float(rng.uniform(0.2, 2.0)), float(rng.uniform(0.05, 0.45)))


def _load(rng, nx, ny, scale=1e-5):
    gx = P.remove_mean(rng.standard_normal((ny, nx)) * scale)
    gy = P.remove_mean(rng.standard_normal((ny, nx)) * scale)
    return gx, gy


def _run_single(lbm, cfg, mat, f0, gx, gy, reference):
    nx, ny = cfg["nx"], cfg["ny"]
    kind = cfg["kind"]
    inplace = not reference and kind in ("inplace", "inplace_blocked")
    s = lbm.Solver(nx, ny, cfg["prec"], inplace=inplace,
                   inplace_steps=cfg["tb"] if kind == "inplace_blocked" else 1,
                   inplace_segment_rows=cfg["seg"] if kind == "inplace_blocked" else 0)
    s.set_material(mat.lame_lambda, mat.lame_mu)
    s.set_body_force(dev(gx), dev(gy))
    if reference or kind == "inplace":
        s.set_time_blocking(1)
    elif kind == "inplace_blocked":
        s.set_time_blocking(1)
        s.set_fused_kernel("wavefront", cfg["seg"])
        s.set_time_blocking(cfg["tb"])
    else:
        s.set_time_blocking(cfg["tb"])
        s.set_fused_kernel("tile" if cfg["kind"] == "tile" else "wavefront", cfg["seg"])
    s.set_populations(dev(f0))
    r = s.step_checked(cfg["steps"]) if cfg["checked"] else None
    if not cfg["checked"]:
        s.step(cfg["steps"])
    f = host(s.populations())
    ux, uy = (host(t) for t in s.displacement())
    s.close()
    return f, ux, uy, r


@pytest.mark.parametrize("seed", [1, 2])
def test_random_single_lattices(seed):
    from paper_2208_14870_amd import lbm
    need_gpu()
    rng = np.random.default_rng(seed)
    for case in range(100):
        nx, ny = _side(rng), _side(rng)
        kind = str(rng.choice(["tile", "tile", "wavefront", "inplace", "inplace_blocked"]))
        tb = 1 if kind == "inplace" else int(rng.integers(2, 9))
        steps = int(rng.integers(1, 40))
        cfg = dict(case=case, nx=nx, ny=ny, prec=str(rng.choice(["fp64", "fp32", "fp16"])),
                   kind=kind, tb=tb, seg=int(rng.choice([1, 3, 8, 17, 64, 256])), steps=steps,
                   checked=bool(rng.random() < 0.3) and steps >= 2 and kind != "inplace")
        say("case " + json.dumps(cfg))
        mat = _material(rng)
        f0 = rng.standard_normal((8, ny, nx)) * 1e-3
        gx, gy = _load(rng, nx, ny)
        fa, uxa, uya, ra = _run_single(lbm, cfg, mat, f0, gx, gy, reference=True)
        fb, uxb, uyb, rb = _run_single(lbm, cfg, mat, f0, gx, gy, reference=False)
        assert np.all(np.isfinite(fb))
        assert np.array_equal(fa, fb) and np.array_equal(uxa, uxb) and np.array_equal(uya, uyb)
        if cfg["checked"]:
            assert abs(ra - rb) <= 1e-12 * max(abs(ra), abs(rb), 1e-300)
        if cfg["prec"] == "fp64" and nx * ny <= 6000:
            fo = O.run(f0, gx, gy, O.omega_vector(mat.lame_lambda, mat.lame_mu), steps)
            assert_elementwise(fb, fo, 1e-12, "f")


@pytest.mark.parametrize("seed", [1, 2])
def test_random_batches(seed):
    from paper_2208_14870_amd import lbm
    need_gpu()
    rng = np.random.default_rng(1000 + seed)
    compared = 0
    for trial in range(20):
        b = lbm.Batch(64, 256 << 20)
        tbs = {p: int(rng.integers(1, 9)) for p in ("fp64", "fp32", "fp16")}
        for p, k in tbs.items():
            b.set_time_blocking(k, p)
        # which lattices take the wavefront list: the default rule, all, or a
        # random minimum size
        wave = {p: int(rng.choice([-1, 0, int(rng.integers(1, 20000))]))
                for p in ("fp64", "fp32", "fp16")}
        for p, m in wave.items():
            b.set_wavefront_sites(p, m)
        say(f"trial {trial}: depths {tbs}, wavefront list {wave}")
        lat = {}

        def add():
            nx = int(rng.choice([rng.integers(1, 9), rng.integers(9, 200)]))
            ny = int(rng.choice([rng.integers(1, 9), rng.integers(9, 200)]))
            prec = str(rng.choice(["fp64", "fp32", "fp16"]))
            mat = _material(rng)
            gx, gy = _load(rng, nx, ny)
            slot = b.add(nx, ny, mat.lame_lambda, mat.lame_mu, dev(gx), dev(gy), prec)
            assert slot is not None
            lat[slot] = (nx, ny, prec, mat, gx, gy)

        for _ in range(int(rng.integers(1, 12))):
            add()
        plan = []
        for _ in range(int(rng.integers(1, 4))):
            check = bool(rng.random() < 0.5)
            chunk = int(rng.integers(2 if check else 1, 30))
            plan.append((chunk, check))
            b.step(chunk, check=check)
            if rng.random() < 0.3 and lat:
                victim = int(rng.choice(list(lat)))
                b.remove(victim)
                del lat[victim]
            if rng.random() < 0.3:
                add()
        _, steps = b.residuals()
        say(f"trial {trial} depths {tbs} wavefront list {wave} plan {plan} lattices "
            + str([(sl, v[0], v[1], v[2], int(steps[sl])) for sl, v in lat.items()]))
        for slot, (nx, ny, prec, mat, gx, gy) in lat.items():
            bx, by = (host(t) for t in b.displacement(slot))
            s = lbm.Solver(nx, ny, prec)
            s.set_material(mat.lame_lambda, mat.lame_mu)
            s.set_body_force(dev(gx), dev(gy))
            s.set_time_blocking(1)
            s.step(int(steps[slot]))
            sx, sy = (host(t) for t in s.displacement())
            s.close()
            if prec == "fp16":
                sc = max(np.max(np.abs(sx)), np.max(np.abs(sy)), 1e-300)
                assert np.max(np.abs(bx - sx)) <= 1e-9 * sc and np.max(np.abs(by - sy)) <= 1e-9 * sc
            else:
                assert np.array_equal(bx, sx) and np.array_equal(by, sy)
            compared += 1
        b.close()
    say(f"lattices compared: {compared}")
    assert compared > 0


def test_random_solves():
    """solve_to_tol under random check intervals, depths and kernels (FP32 and
    FP16 with or without the FP64 polish, in place where there is no polish):
    the same stop step, status, final storage type and residual (to 1e-9) as
    single steps, and the same displacement (FP16 to 1e-9 of max |u|)."""
    from paper_2208_14870_amd import lbm
    need_gpu()
    rng = np.random.default_rng(77)
    for case in range(30):
        nx, ny = int(rng.integers(3, 70)), int(rng.integers(3, 70))
        prec = str(rng.choice(["fp64", "fp32", "fp16"]))
        polish = prec != "fp64" and bool(rng.random() < 0.7)
        kind = str(rng.choice(["tile", "wavefront"] if polish
                              else ["tile", "tile", "wavefront", "inplace", "inplace_blocked"]))
        tb = 1 if kind == "inplace" else int(rng.integers(2, 9))
        K = int(rng.choice([1, 2, 3, 7, 50, 100, 333]))
        tol = float(rng.choice([1e-6, 1e-8, 1e-10])) if (prec == "fp64" or polish) else 1e-5
        mat = _material(rng)
        kx, ky = int(rng.integers(1, 3)), int(rng.integers(0, 3))
        x = (np.arange(nx) + 0.5) / nx
        y = (np.arange(ny) + 0.5) / ny
        gx = P.remove_mean(1e-4 * np.sin(2 * np.pi * (kx * x[None, :] + ky * y[:, None])))
        gy = P.remove_mean(1e-4 * np.cos(2 * np.pi * (kx * x[None, :] - ky * y[:, None])))
        seg = int(rng.choice([1, 8, 64]))
        say("solve " + json.dumps(dict(case=case, nx=nx, ny=ny, prec=prec, polish=polish, kind=kind,
                                        tb=tb, K=K, tol=tol)))
        out = []
        for reference in (True, False):
            blocked = not reference and kind == "inplace_blocked"
            s = lbm.Solver(nx, ny, prec, with_polish=polish,
                           inplace=(not reference and kind.startswith("inplace")),
                           inplace_steps=tb if blocked else 1,
                           inplace_segment_rows=seg if blocked else 0)
            s.set_material(mat.lame_lambda, mat.lame_mu)
            s.set_body_force(dev(gx), dev(gy))
            if polish:
                s.set_polish(1e-5)
            if reference or kind == "inplace":
                s.set_time_blocking(1)
            elif blocked:
                s.set_time_blocking(1)
                s.set_fused_kernel("wavefront", seg)
                s.set_time_blocking(tb)
            else:
                s.set_time_blocking(tb)
                s.set_fused_kernel("tile" if kind == "tile" else "wavefront", seg)
            n, r, status = s.solve_to_tol(tol, 20000, K)
            ux, uy = (host(t) for t in s.displacement())
            out.append((n, r, status, s.current_precision, ux, uy))
            s.close()
        (na, ra, sa, pa, uxa, uya), (nb, rb, sb, pb, uxb, uyb) = out
        assert (na, sa, pa) == (nb, sb, pb)
        assert abs(ra - rb) <= 1e-9 * max(abs(ra), 1e-300)
        if prec == "fp16":
            sc = max(np.max(np.abs(uxa)), np.max(np.abs(uya)), 1e-300)
            assert np.max(np.abs(uxa - uxb)) <= 1e-9 * sc and np.max(np.abs(uya - uyb)) <= 1e-9 * sc
        else:
            assert np.array_equal(uxa, uxb) and np.array_equal(uya, uyb)


def test_random_outputs_against_the_oracle():
    """Populations, displacement and stress after random step counts (two
    buffers or in place, at 1..8 steps per launch, odd and even counts) from
    random states, against the oracle: FP64 1e-12, FP32 2e-6 (populations) /
    2e-5, FP16 3e-3 / 3e-2 relative; error norms against numpy to 1e-12."""
    from paper_2208_14870_amd import lbm
    need_gpu()
    rng = np.random.default_rng(7)
    for case in range(40):
        nx, ny = int(rng.integers(1, 90)), int(rng.integers(1, 90))
        prec = str(rng.choice(["fp64", "fp32", "fp16"]))
        inplace = bool(rng.random() < 0.4)
        tb = int(rng.integers(1, 9))  # in place: blocked through the in-place wavefront from 2
        steps = int(rng.integers(0, 12))
        say("outputs " + json.dumps(dict(case=case, nx=nx, ny=ny, prec=prec, inplace=inplace,
                                          tb=tb, steps=steps)))
        mat = _material(rng)
        f0 = rng.standard_normal((8, ny, nx)) * 1e-3
        gx, gy = _load(rng, nx, ny)
        s = lbm.Solver(nx, ny, prec, inplace=inplace)
        s.set_material(mat.lame_lambda, mat.lame_mu)
        s.set_body_force(dev(gx), dev(gy))
        s.set_time_blocking(tb)
        s.set_populations(dev(f0))
        if steps:
            s.step(steps)
        f = host(s.populations())
        ux, uy = (host(t) for t in s.displacement())
        sig = np.stack([host(t) for t in s.stress()])
        rx, ry = rng.standard_normal((ny, nx)), rng.standard_normal((ny, nx))
        norms = s.error_norms(dev(rx), dev(ry))
        s.close()
        om = O.omega_vector(mat.lame_lambda, mat.lame_mu)
        fo = O.run(f0, gx, gy, om, steps) if steps else f0
        oux, ouy = O.displacement(fo, gx, gy)
        osig = np.stack(O.stress(fo, om))

        def rel(a, b):
            return float(np.sqrt(np.sum((a - b) ** 2) / max(np.sum(b ** 2), 1e-300)))

        tol = {"fp64": 1e-12, "fp32": 2e-6, "fp16": 3e-3}[prec]
        if prec == "fp64":
            assert_elementwise(f, fo, tol, "f")
            assert_elementwise((ux, uy), (oux, ouy), tol, "u")
            assert_elementwise(tuple(sig), tuple(osig), tol, "stress")
        else:
            assert rel(f, fo) <= tol
            assert rel(np.stack([ux, uy]), np.stack([oux, ouy])) <= 10 * tol
            assert rel(sig, osig) <= 10 * tol
        ex, ey = ux - rx, uy - ry
        want = (float(np.sum(ex ** 2 + ey ** 2)), float(np.sum(rx ** 2 + ry ** 2)),
                float(max(np.max(np.abs(ex)), np.max(np.abs(ey)))),
                float(max(np.max(np.abs(rx)), np.max(np.abs(ry)))))
        got = (norms["sum_e2"], norms["sum_ref2"], norms["max_e"], norms["max_ref"])
        for g, w in zip(got, want):
            assert abs(g - w) <= 1e-12 * w
