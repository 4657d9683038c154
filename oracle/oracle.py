"""Python face of the FP64 CPU oracle (``lbm_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The slow, plain reference for the lattice
Boltzmann scheme for 2D quasi-static linear elasticity of Boolakee, Geier and
De Lorenzis (arXiv 2208.14870).  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the GPU library never
does, and this module imports nothing from it.

Every function here marshals numpy arrays into the C routines, or is a plain
numpy formula that cites the passage it follows:

* ``rates``           -- Table "scheme" (relaxation times from Lame parameters)
* ``step`` / ``run``  -- Algorithm 1 (collide pass, then periodic streaming)
* ``displacement``    -- Table "solution": u = bared first-order moments
* ``stress``          -- Eq. compute_bared + Table "solution" (lattice units)
* ``solve_to_tol``    -- pseudo-time stepping until ||u(n)-u(n-1)||/||u(n)|| <= tol
* ``error_norms``     -- grid norms of Sec. 7.1 (L2 with dx^2 weight, Linf)
* ``leading_error_constants`` -- C1..C5, D1..D3 of Eq. leadingCoefficients (App. B)
* ``fourth_order_rates`` -- tau_12 = tau_21 of App. C and tau_22 from C1 = 0
* ``corrected_force``  -- Eqs. force_correction_x/y (improved scheme, Sec. 4)
* ``error_estimates``  -- R1, R2 of Eq. rss_estimate

State layout: ``f[q, y, x]`` float64, q = 0..7 for populations 1..8 of the
one-index table of Sec. 5, x fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

THETA = 1.0 / 3.0  # Sec. 3.3.2: theta = 1/3 makes omega_11 = omega_d

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain FP64: no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c99",
               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i, l, d = ctypes.c_int, ctypes.c_long, ctypes.c_double
        lib.oracle_rates.argtypes = [d, d, d, dp]
        lib.oracle_rates.restype = i
        lib.oracle_omega_vector.argtypes = [d, d, d, d, d, d, dp]
        lib.oracle_moment_matrix.argtypes = [dp]
        lib.oracle_collide_node.argtypes = [dp, d, d, dp, d, dp, dp]
        lib.oracle_collide_all.argtypes = [i, i, dp, dp, dp, dp, d, dp]
        lib.oracle_stream.argtypes = [i, i, dp, dp]
        lib.oracle_run.argtypes = [i, i, dp, dp, dp, dp, d, l]
        lib.oracle_run.restype = i
        lib.oracle_displacement.argtypes = [i, i, dp, dp, dp, dp, dp]
        lib.oracle_stress.argtypes = [i, i, dp, dp, dp, dp, dp]
        lib.oracle_residual.argtypes = [l, dp, dp, dp, dp]
        lib.oracle_residual.restype = d
        lib.oracle_solve_to_tol.argtypes = [i, i, dp, dp, dp, dp, d, d, l, i, i,
                                            ctypes.POINTER(l), dp]
        lib.oracle_solve_to_tol.restype = i
        lib.oracle_stream_only.argtypes = [i, i, dp, l]
        lib.oracle_stream_only.restype = i
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

def rates(lame_lambda: float, lame_mu: float, theta: float = THETA):
    """(omega_11, omega_s, omega_d) from Table "scheme" and Eq. relaxation_rate."""
    out = np.zeros(3)
    rc = _load().oracle_rates(lame_lambda, lame_mu, theta, _p(out))
    if rc != 0:
        raise ValueError("inadmissible material: need mu > 0, lambda + mu > 0, 0 < theta < 1")
    return tuple(out)


def omega_vector(lame_lambda: float, lame_mu: float, theta: float = THETA,
                 w12: float = 1.0, w21: float = 1.0, w22: float = 1.0) -> np.ndarray:
    """Relaxation rates in the moment order 10, 01, 11, s, d, 12, 21, 22."""
    w11, ws, wd = rates(lame_lambda, lame_mu, theta)
    out = np.zeros(8)
    _load().oracle_omega_vector(w11, ws, wd, w12, w21, w22, _p(out))
    return out


def moment_matrix() -> np.ndarray:
    """The 8x8 population-to-moment transform as the oracle assembles it."""
    out = np.zeros(64)
    _load().oracle_moment_matrix(_p(out))
    return out.reshape(8, 8)


# ---------------------------------------------------------------------------
# single node and lattice passes
# ---------------------------------------------------------------------------

def collide_node(f8, gx: float, gy: float, omega: np.ndarray, theta: float = THETA):
    """Post-collision populations and displacement of one node."""
    f8 = _f64(f8)
    fs = np.zeros(8)
    u = np.zeros(2)
    _load().oracle_collide_node(_p(f8), gx, gy, _p(_f64(omega)), theta, _p(fs), _p(u))
    return fs, u


def collision_matrix(omega: np.ndarray, theta: float = THETA) -> np.ndarray:
    """The linear collision operator (g = 0) by columns: A[:, j] = collide(e_j)."""
    A = np.zeros((8, 8))
    for j in range(8):
        e = np.zeros(8)
        e[j] = 1.0
        A[:, j], _ = collide_node(e, 0.0, 0.0, omega, theta)
    return A


def forcing_matrix(omega: np.ndarray, theta: float = THETA) -> np.ndarray:
    """Response of the post-collision populations to (gx, gy) at f = 0."""
    B = np.zeros((8, 2))
    B[:, 0], _ = collide_node(np.zeros(8), 1.0, 0.0, omega, theta)
    B[:, 1], _ = collide_node(np.zeros(8), 0.0, 1.0, omega, theta)
    return B


def zero_state(nx: int, ny: int) -> np.ndarray:
    """f(x, 0) = 0: equilibrium initialisation for u0 = 0 (Eq. init_cond, Sec. 6.2)."""
    return np.zeros((8, ny, nx))


def collide_all(f, gx, gy, omega, theta: float = THETA) -> np.ndarray:
    f = _f64(f)
    ny, nx = f.shape[1:]
    out = np.zeros_like(f)
    _load().oracle_collide_all(nx, ny, _p(f), _p(_f64(gx)), _p(_f64(gy)), _p(_f64(omega)),
                               theta, _p(out))
    return out


def stream(fstar) -> np.ndarray:
    fstar = _f64(fstar)
    ny, nx = fstar.shape[1:]
    out = np.zeros_like(fstar)
    _load().oracle_stream(nx, ny, _p(fstar), _p(out))
    return out


def run(f, gx, gy, omega, nsteps: int, theta: float = THETA) -> np.ndarray:
    """f(n + nsteps) from f(n); returns a new array."""
    f = _f64(f).copy()
    ny, nx = f.shape[1:]
    rc = _load().oracle_run(nx, ny, _p(f), _p(_f64(gx)), _p(_f64(gy)), _p(_f64(omega)),
                            theta, int(nsteps))
    if rc != 0:
        raise MemoryError("oracle_run")
    return f


def stream_only(f, nsteps: int) -> np.ndarray:
    f = _f64(f).copy()
    ny, nx = f.shape[1:]
    if _load().oracle_stream_only(nx, ny, _p(f), int(nsteps)) != 0:
        raise MemoryError("oracle_stream_only")
    return f


def displacement(f, gx, gy):
    f = _f64(f)
    ny, nx = f.shape[1:]
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    _load().oracle_displacement(nx, ny, _p(f), _p(_f64(gx)), _p(_f64(gy)), _p(ux), _p(uy))
    return ux, uy


def stress(f, omega):
    f = _f64(f)
    ny, nx = f.shape[1:]
    sxx, syy, sxy = (np.zeros((ny, nx)) for _ in range(3))
    _load().oracle_stress(nx, ny, _p(f), _p(_f64(omega)), _p(sxx), _p(syy), _p(sxy))
    return sxx, syy, sxy


def residual(ux, uy, uxp, uyp) -> float:
    ux, uy, uxp, uyp = (_f64(a) for a in (ux, uy, uxp, uyp))
    return float(_load().oracle_residual(ux.size, _p(ux), _p(uy), _p(uxp), _p(uyp)))


def solve_to_tol(f, gx, gy, omega, tol: float, max_steps: int, check_every: int = 1,
                 theta: float = THETA, rise_checks: int = 0):
    """Returns (f(n), n, r(n), status) with status 0 converged, 1 max_steps, -2
    diverged (a non-finite residual, or with rise_checks > 0 an update norm
    ||u(n) - u(n-1)|| that rose at rise_checks checks in a row to at least
    twice the largest of the 32 update norms before those rises)."""
    f = _f64(f).copy()
    ny, nx = f.shape[1:]
    n = ctypes.c_long(0)
    r = ctypes.c_double(0.0)
    st = _load().oracle_solve_to_tol(nx, ny, _p(f), _p(_f64(gx)), _p(_f64(gy)),
                                     _p(_f64(omega)), theta, tol, int(max_steps),
                                     int(check_every), int(rise_checks), ctypes.byref(n),
                                     ctypes.byref(r))
    if st == -1:
        raise MemoryError("oracle_solve_to_tol")
    return f, n.value, r.value, st


# ---------------------------------------------------------------------------
# error measures (Sec. 7.1)
# ---------------------------------------------------------------------------

def error_norms(ux, uy, ux_ref, uy_ref, dx: float = 1.0) -> dict:
    """Grid norms of e = u - u_ref (Sec. 7.1): L2 = (dx^2 sum |e_i|_2^2)^(1/2),
    Linf = max_i |e_i|_inf; relative forms divide by the L2 grid norm of the
    reference, as the paper reports them, and also give the plain relative
    L2 ratio sqrt(sum|e|^2 / sum|u_ref|^2)."""
    ex = np.asarray(ux, np.float64) - ux_ref
    ey = np.asarray(uy, np.float64) - uy_ref
    e2 = float(np.sum(ex * ex + ey * ey))
    r2 = float(np.sum(np.asarray(ux_ref) ** 2 + np.asarray(uy_ref) ** 2))
    l2 = np.sqrt(dx * dx * e2)
    linf = float(max(np.max(np.abs(ex)), np.max(np.abs(ey))))
    ref_l2 = np.sqrt(dx * dx * r2)
    return {
        "l2": l2,
        "linf": linf,
        "rel_l2": l2 / ref_l2 if ref_l2 > 0 else float("nan"),
        "rel_linf": linf / ref_l2 if ref_l2 > 0 else float("nan"),
        "rel_l2_plain": np.sqrt(e2 / r2) if r2 > 0 else float("nan"),
    }


# ---------------------------------------------------------------------------
# leading-order error, improved scheme and fourth-order rates (Sec. 4, App. B, C)
# ---------------------------------------------------------------------------

def young_poisson(lame_lambda: float, lame_mu: float):
    """Dimensionless Young's modulus and Poisson ratio of the 2D relations
    (Eq. material_relations): K = lambda + mu, E = 4 K mu / (K + mu),
    nu = (K - mu) / (K + mu)."""
    K = lame_lambda + lame_mu
    return 4.0 * K * lame_mu / (K + lame_mu), (K - lame_mu) / (K + lame_mu)


def tau_of(omega: float) -> float:
    """Eq. relaxation_rate: tau = 1/omega - 1/2."""
    return 1.0 / omega - 0.5


def leading_error_constants(young: float, nu: float, theta: float = THETA, tau12: float = 0.5,
                            tau21: float = 0.5, tau22: float = 0.5) -> dict:
    """C1..C5 and D1..D3 of the body-force term r_x^(4) of the leading-order
    error equation (Eqs. ux_order2 / leadingCoefficients) from the expressions
    of App. B, with the second-order relaxation times replaced by (E, nu).

    Four readings, each fixed by the exact one-mode response of the scheme
    (the quartic part of the logarithm of its slow 2 x 2 block and the
    quadratic part of its effective forcing, both to 1e-12 relative for theta
    in (0, 1), tau_12 != tau_21 and nu < 0):
      1. sign: the printed constants are the negatives of the coefficients in
         Eq. ux_order2, so every constant below carries a leading minus;
      2. D1: its tau_12 term has the denominator (1 - theta^2)(1 - nu^2)
         (printed with (1 - nu^2)^2);
      3. D2: its tau_21 term has the denominator (1 - theta^2)(1 - nu^2)
         (printed with (1 - nu^2)^2);
      4. C2: its E^3 term has the denominator 8 theta (1 - theta^2)(1 - nu^2)^3
         (printed without theta).
    The x row; the y row follows with tau_12 and tau_21 exchanged."""
    E, v, th = float(young), float(nu), float(theta)
    t12, t21, t22 = float(tau12), float(tau21), float(tau22)
    a = 1.0 - th * th
    b = 1.0 - v * v
    q = th * th * (1.0 + v) + v - 2.0 * th - 1.0   # a factor shared by several terms
    C1 = ((v * v - 2.0 * th * v + 1.0) / (a * b ** 3) * E ** 3
          + th * (v - th) * t12 / (a * b * b) * E * E
          + (-1.0 + th * th + 12.0 * th * (th - v) * t12 * t22) / (12.0 * a * b) * E)
    C2 = (((1.0 - v) ** 3 + 4.0 * th * (v ** 3 - v * v + 3.0 * v + 1.0)
           + th * th * (5.0 * v ** 3 - 15.0 * v * v - v - 5.0)) / (8.0 * th * a * b ** 3) * E ** 3
          + (2.0 * th * ((1.0 - v) * v + th * th * (1.0 + v) - th * (1.0 + v * v)) * t12
             + (1.0 - th) * (1.0 - v) * (1.0 + 2.0 * th - v - th * th * (1.0 + v)) * t21)
          / (-4.0 * th * a * b * b) * E * E
          + ((2.0 * th * th - 3.0 * th + 1.0) * (1.0 + 3.0 * th * (1.0 - v) - 5.0 * v)
             + 24.0 * th * (th - v) * t12 * t22) / (24.0 * a * b) * E)
    C3 = (((1.0 - v) ** 2 * (3.0 + v) + 4.0 * th * (-v ** 3 + 3.0 * v * v + v + 1.0)
           - th * th * (5.0 * v ** 3 - 3.0 * v * v + 7.0 * v + 7.0)) / (8.0 * th * a * b ** 3) * E ** 3
          + (-2.0 * (1.0 - th) * th * (v - 2.0 * th - 1.0) * (1.0 - v) * t12
             - ((1.0 + th) * (1.0 - v) ** 2 + th ** 3 * (1.0 + v) ** 2
                + th * th * (v * v - 2.0 * v - 3.0)) * t21) / (4.0 * th * a * b * b) * E * E
          + ((1.0 - th) * (1.0 - v - th * (1.0 + v) - 2.0 * th * th * (2.0 + v))
             - 4.0 * a * (1.0 - v) * t12 * t22 + 4.0 * q * t21 * t22) / (8.0 * a * b) * E
          + th * t22 / 4.0)
    C4 = ((16.0 * th * v + (1.0 - v) ** 2 * (3.0 + v)
           - th * th * (v ** 3 + 9.0 * v * v - 5.0 * v + 11.0)) / (8.0 * th * a * b ** 3) * E ** 3
          + (a * (1.0 - v) * (th * v + v + th - 1.0) * t12 - 2.0 * th * q * t21)
          / (4.0 * th * a * b * b) * E * E
          + (a * (2.0 * (2.0 - v) - 3.0 * th * (5.0 + v)) - 12.0 * a * (1.0 - v) * t12 * t22
             + 12.0 * q * t21 * t22) / (24.0 * a * b) * E
          + th * t22 / 4.0)
    C5 = (E ** 3 / (8.0 * th * (1.0 + v) ** 3) - (1.0 - th) * t12 / (4.0 * th * (1.0 + v) ** 2) * E * E
          - (3.0 * th - 2.0) / (24.0 * (1.0 + v)) * E)
    D1 = ((v * v - 2.0 * th * v + 1.0) / (a * b * b) * E * E + th * (v - th) * t12 / (a * b) * E
          - 0.25)
    D2 = (((1.0 - v) ** 2 + 8.0 * th * v - th * th * (5.0 * v * v - 2.0 * v + 5.0))
          / (4.0 * th * a * b * b) * E * E - q * t21 / (2.0 * a * b) * E - th / 2.0)
    D3 = E * E / (4.0 * th * (1.0 + v) ** 2) + t12 / (2.0 * (1.0 + v)) * E - th / 4.0
    printed = {"C1": C1, "C2": C2, "C3": C3, "C4": C4, "C5": C5, "D1": D1, "D2": D2, "D3": D3}
    return {k: -val for k, val in printed.items()}


def material_error_constants(lame_lambda: float, lame_mu: float, theta: float = THETA,
                             w12: float = 1.0, w21: float = 1.0, w22: float = 1.0):
    """(x-row constants, y-row constants) for a material and rates."""
    E, v = young_poisson(lame_lambda, lame_mu)
    t12, t21, t22 = tau_of(w12), tau_of(w21), tau_of(w22)
    return (leading_error_constants(E, v, theta, t12, t21, t22),
            leading_error_constants(E, v, theta, t21, t12, t22))


def error_estimates(consts: dict):
    """Eq. rss_estimate: R1 = |C|_2 (error left after the force correction),
    R2 = |(C, D)|_2 (without it)."""
    c = sum(consts["C%d" % i] ** 2 for i in range(1, 6))
    d = sum(consts["D%d" % i] ** 2 for i in range(1, 4))
    return float(np.sqrt(c)), float(np.sqrt(c + d))


def fourth_order_rates(lame_lambda: float, lame_mu: float, theta: float = THETA):
    """(omega_12, omega_21, omega_22) of the fourth-order special case (Sec.
    7.3.3): tau_12 = tau_21 from App. C, which makes C5 = 0; tau_22 as the
    root of C1 = 0, which is affine in tau_22 (App. C's printed tau_22 does
    not make C1 vanish; reading adopted: the condition C1 = 0 it is meant to
    satisfy)."""
    E, v = young_poisson(lame_lambda, lame_mu)
    t11 = lame_mu / theta
    t12 = (2.0 - 3.0 * theta + 12.0 * theta * t11 * t11) / (12.0 * (1.0 - theta) * t11)
    c0 = leading_error_constants(E, v, theta, t12, t12, 0.0)["C1"]
    c1 = leading_error_constants(E, v, theta, t12, t12, 1.0)["C1"]
    t22 = -c0 / (c1 - c0)
    return 1.0 / (t12 + 0.5), 1.0 / (t12 + 0.5), 1.0 / (t22 + 0.5)


def central_second_derivatives(g) -> np.ndarray:
    """Second-order central differences on the periodic lattice (unit
    spacing): planes (d_xx, d_xy, d_yy) of a field [ny][nx]."""
    g = _f64(g)
    xp, xm = np.roll(g, -1, axis=1), np.roll(g, 1, axis=1)
    yp, ym = np.roll(g, -1, axis=0), np.roll(g, 1, axis=0)
    dxx = xp - 2.0 * g + xm
    dyy = yp - 2.0 * g + ym
    pp = np.roll(xp, -1, axis=0)   # g(x+1, y+1)
    mp_ = np.roll(xm, -1, axis=0)  # g(x-1, y+1)
    pm = np.roll(xp, 1, axis=0)    # g(x+1, y-1)
    mm = np.roll(xm, 1, axis=0)    # g(x-1, y-1)
    dxy = ((pp - mp_) - (pm - mm)) * 0.25
    return np.stack([dxx, dxy, dyy])


def corrected_force(gx, gy, d2gx, d2gy, consts_x: dict, consts_y: dict):
    """Eqs. force_correction_x/y in lattice units:
    gx' = gx - (D1 d_xx gx + D2 d_xy gy + D3 d_yy gx),
    gy' = gy - (D3' d_xx gy + D2' d_xy gx + D1' d_yy gy),
    with d2gx = (d_xx gx, d_xy gx, d_yy gx), d2gy likewise, the x-row
    constants D and the y-row constants D' (equal when tau_12 = tau_21)."""
    cx, cy = consts_x, consts_y
    gx, gy = _f64(gx), _f64(gy)
    hx = gx - ((cx["D1"] * d2gx[0] + cx["D2"] * d2gy[1]) + cx["D3"] * d2gx[2])
    hy = gy - ((cy["D3"] * d2gy[0] + cy["D2"] * d2gx[1]) + cy["D1"] * d2gy[2])
    return hx, hy
