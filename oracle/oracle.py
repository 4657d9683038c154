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
