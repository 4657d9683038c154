"""Host-side linear stability check of the scheme (Sec. 5).

One step acts on a plane wave f = a exp(i k.x) as a -> L(k) a with
L(k) = diag(exp(-i k.c_q)) A, A = M^-1 Lambda M_eq + M^-1 (I - Lambda) M
(Eq. lbmvector): M maps populations to the moments 10, 01, 11, s, d, 12,
21, 22 (Eqs. moments, replace_raw), M_eq produces the equilibria of Table
"scheme" (m12_eq = theta m10, m21_eq = theta m01, all others zero) and
Lambda = diag(0, 0, omega_11, omega_s, omega_d, omega_12, omega_21,
omega_22).  The scheme is stable if sup_k rho(L(k)) <= 1.  Following
Sec. 5 the supremum is sampled with |k| in [0, pi] (50 points) and the angle
in [0, pi/4] (5 points); a lattice-specific check uses the lattice's own
wavevectors 2 pi (a/nx, b/ny).

This is a planning tool for choosing material / time-step parameters; the
GPU library does not call it.
"""
from __future__ import annotations

import math
from typing import Iterable, Optional, Tuple

import numpy as np

# velocities of the one-index table of Sec. 5
C = np.array([(1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)], float)


def moment_matrix() -> np.ndarray:
    """Rows 10, 01, 11, s, d, 12, 21, 22 from m_ab = sum_q i^a j^b f_q."""
    i, j = C[:, 0], C[:, 1]
    return np.stack([i, j, i * j, i ** 2 + j ** 2, i ** 2 - j ** 2, i * j ** 2, i ** 2 * j,
                     i ** 2 * j ** 2])


def rates(lame_lambda: float, lame_mu: float, theta: float = 1.0 / 3.0):
    """Table "scheme": omega = 1/(tau + 1/2) with tau_11 = mu/theta,
    tau_s = 2K/(1+theta), tau_d = 2mu/(1-theta), K = lambda + mu."""
    K = lame_lambda + lame_mu
    if not (lame_mu > 0 and K > 0 and 0 < theta < 1):
        raise ValueError("need mu > 0, lambda + mu > 0, 0 < theta < 1")
    return (1.0 / (lame_mu / theta + 0.5), 1.0 / (2 * K / (1 + theta) + 0.5),
            1.0 / (2 * lame_mu / (1 - theta) + 0.5))


def collision_operator(lame_lambda: float, lame_mu: float, theta: float = 1.0 / 3.0,
                       w12: float = 1.0, w21: float = 1.0, w22: float = 1.0) -> np.ndarray:
    M = moment_matrix()
    Meq = np.zeros((8, 8))
    Meq[0], Meq[1] = M[0], M[1]
    Meq[5], Meq[6] = theta * M[0], theta * M[1]
    w11, ws, wd = rates(lame_lambda, lame_mu, theta)
    lam = np.diag([0.0, 0.0, w11, ws, wd, w12, w21, w22])
    Minv = np.linalg.inv(M)
    return Minv @ lam @ Meq + Minv @ (np.eye(8) - lam) @ M


def amplification(A: np.ndarray, kx: float, ky: float) -> np.ndarray:
    return np.diag(np.exp(-1j * (C[:, 0] * kx + C[:, 1] * ky))) @ A


def paper_grid(n_k: int = 50, n_phi: int = 5) -> Iterable[Tuple[float, float]]:
    for kh in np.linspace(0.0, math.pi, n_k):
        for ph in np.linspace(0.0, math.pi / 4, n_phi):
            yield kh * math.cos(ph), kh * math.sin(ph)


def lattice_grid(nx: int, ny: int) -> Iterable[Tuple[float, float]]:
    for a in range(nx):
        for b in range(ny):
            yield 2 * math.pi * a / nx, 2 * math.pi * b / ny


def sup_rho(lame_lambda: float, lame_mu: float, grid: Optional[Iterable] = None,
            **kw) -> Tuple[float, Tuple[float, float]]:
    """(sup rho(L(k)) over the grid, the maximising k)."""
    A = collision_operator(lame_lambda, lame_mu, **kw)
    best, arg = -1.0, (0.0, 0.0)
    for kx, ky in (paper_grid() if grid is None else grid):
        r = float(np.max(np.abs(np.linalg.eigvals(amplification(A, kx, ky)))))
        if r > best:
            best, arg = r, (kx, ky)
    return best, arg


def is_stable(lame_lambda: float, lame_mu: float, tol: float = 1e-12,
              nx: Optional[int] = None, ny: Optional[int] = None, **kw) -> bool:
    """sup rho <= 1 + tol on the paper's grid, or on the wavevectors of an
    nx x ny lattice when given."""
    grid = lattice_grid(nx, ny) if nx else None
    return sup_rho(lame_lambda, lame_mu, grid, **kw)[0] <= 1.0 + tol


def stable_young_range(nu: float, young: Iterable[float]) -> list:
    """The dimensionless Young's moduli (Eq. scalingE) of `young` that are stable at
    Poisson ratio nu (2D relations of Eq. material_relations)."""
    out = []
    for E in young:
        lam, mu = E * nu / (1 - nu * nu), E / (2 * (1 + nu))
        if is_stable(lam, mu):
            out.append(E)
    return out
