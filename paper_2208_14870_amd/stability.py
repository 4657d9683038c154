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
GPU library does not call it (its error estimates R1, R2 come from the
library's host-only lbm_leading_error_constants).
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


# ---------------------------------------------------------------------------
# accuracy and convergence of one Fourier mode (planning advisor)
# ---------------------------------------------------------------------------

def forcing_operator(theta: float = 1.0 / 3.0, w12: float = 1.0, w21: float = 1.0) -> np.ndarray:
    """Populations one collision adds for a force g (8 x 2): the first moments gain
    g (half before the equilibria, half after: Eqs. coll10, coll10post) and the
    third-order moments m12, m21 relax towards theta times the bared first
    moments, so they gain w12 theta g/2 and w21 theta g/2."""
    G = np.zeros((8, 2))
    G[0, 0] = G[1, 1] = 1.0
    G[5, 0] = w12 * theta / 2.0
    G[6, 1] = w21 * theta / 2.0
    return np.linalg.solve(moment_matrix(), G)


def steady_response(lame_lambda: float, lame_mu: float, kx: float, ky: float,
                    theta: float = 1.0 / 3.0, w12: float = 1.0, w21: float = 1.0,
                    w22: float = 1.0) -> np.ndarray:
    """The scheme's exact steady state for one load mode g = g_hat exp(i k.x),
    k != 0, as the 2 x 2 map g_hat -> u_hat: the populations after the
    collision-and-stream step satisfy f = D(A f + B g) with D = diag(exp(-i k.c)),
    so f = (I - D A)^-1 D B g, and u = (M f)[10, 01] + g/2 (the bared first
    moments)."""
    A = collision_operator(lame_lambda, lame_mu, theta=theta, w12=w12, w21=w21, w22=w22)
    D = np.diag(np.exp(-1j * (C[:, 0] * kx + C[:, 1] * ky)))
    B = forcing_operator(theta, w12, w21)
    F = np.linalg.solve(np.eye(8) - D @ A, D @ B)
    return (moment_matrix() @ F)[:2] + 0.5 * np.eye(2)


def continuum_response(lame_lambda: float, lame_mu: float, kx: float, ky: float) -> np.ndarray:
    """Steady state of mu lap u + K grad div u + g = 0 (lattice units) for one
    mode: (mu |k|^2 I + K k k^T)^-1."""
    K = lame_lambda + lame_mu
    k = np.array([kx, ky])
    return np.linalg.inv(lame_mu * (k @ k) * np.eye(2) + K * np.outer(k, k))


def mode_error(lame_lambda: float, lame_mu: float, kx: float, ky: float, **kw) -> float:
    """Relative discretisation error of the steady state for one load mode: the
    spectral norm of (discrete - continuum response) over that of the continuum
    response.  Second order: it falls by 4 when k halves."""
    Rd = steady_response(lame_lambda, lame_mu, kx, ky, **kw)
    Rc = continuum_response(lame_lambda, lame_mu, kx, ky)
    return float(np.linalg.norm(Rd - Rc, 2) / np.linalg.norm(Rc, 2))


def slowest_decay(lame_lambda: float, lame_mu: float, nx: int, ny: int,
                  **kw) -> Tuple[float, Tuple[float, float]]:
    """Largest |eigenvalue| of L(k) over the smooth wavevectors of an nx x ny
    lattice (both components, folded into [-pi, pi), at most pi/2 in size), and
    its k: the slowest decay of a smooth load's response.  k = 0, the mean, never
    decays and is left out.  (Wavevectors next to the staggered ones with a
    component pi, whose eigenvalue -1 never decays either, mirror the smooth
    ones' slowest |eigenvalue|; a smooth load from f = 0 does not excite them.)"""
    A = collision_operator(lame_lambda, lame_mu, **kw)
    best, arg = 0.0, (0.0, 0.0)
    for kx, ky in lattice_grid(nx, ny):
        fx = kx - 2 * math.pi if kx >= math.pi else kx
        fy = ky - 2 * math.pi if ky >= math.pi else ky
        if (fx == 0.0 and fy == 0.0) or abs(fx) > math.pi / 2 or abs(fy) > math.pi / 2:
            continue
        r = float(np.max(np.abs(np.linalg.eigvals(amplification(A, fx, fy)))))
        if r > best:
            best, arg = r, (fx, fy)
    return best, arg


def predicted_steps(rho: float, tol: float) -> int:
    """Steps until the residual ||u(n) - u(n-1)|| / ||u(n)|| of a mode decaying as
    rho^n from f = 0 falls to tol: u(n) = u(1 - rho^n), so the residual is about
    (1 - rho) rho^(n-1) (an estimate: the load's other modes decay faster)."""
    if not (0.0 < rho < 1.0):
        return 0 if rho <= 0.0 else -1
    return int(math.ceil(1.0 + math.log(tol / (1.0 - rho)) / math.log(rho)))


def error_estimates(lame_lambda: float, lame_mu: float, theta: float = 1.0 / 3.0):
    """(R1, R2) of Eq. rss_estimate: the root-sum-square of the leading-order
    error constants left with the improved scheme's force correction (C1..C5),
    and without it (C1..C5, D1..D3) (Sec. 4, App. B), from the library's host
    function lbm_leading_error_constants (no GPU involved)."""
    from . import lbm
    c = lbm.leading_error_constants(lame_lambda, lame_mu, theta)
    return c["R1"], c["R2"]


def advise(nu: float, n: int, young: Optional[Iterable[float]] = None, tol: float = 1e-8,
           max_error: Optional[float] = None,
           criterion: str = "steps") -> Tuple[list, Optional[dict]]:
    """Choice of the dimensionless Young's modulus (Eq. scalingE: the ratio of time
    step to damping for a given physical E) for an n x n lattice at Poisson ratio
    nu.  For each candidate: stability on the paper's grid, the steps to reach tol
    for the slowest decaying lattice mode, the steady-state error of the lowest
    diagonal load mode k = 2 pi (1, 1)/n, and the error estimates R1 (with the
    force correction) and R2 (without) of Sec. 4.  Returns (rows, the pick or
    None): criterion "steps" picks the stable row with the fewest steps whose
    error is at most max_error; "R1" / "R2" pick the stable row with the
    smallest estimate, as Sec. 4 picks E~ for the improved / standard scheme."""
    if criterion not in ("steps", "R1", "R2"):
        raise ValueError("criterion must be 'steps', 'R1' or 'R2'")
    young = np.geomspace(0.01, 10.0, 25) if young is None else young
    rows = []
    for E in young:
        lam, mu = E * nu / (1 - nu * nu), E / (2 * (1 + nu))
        stable = is_stable(lam, mu)
        rho, _ = slowest_decay(lam, mu, n, n)
        k = 2 * math.pi / n
        r1, r2 = error_estimates(lam, mu)
        rows.append({"young": float(E), "lame_lambda": lam, "lame_mu": mu, "stable": stable,
                     "rho": rho, "steps": predicted_steps(rho, tol),
                     "error_k11": mode_error(lam, mu, k, k), "R1": r1, "R2": r2})
    if criterion == "steps":
        ok = [r for r in rows if r["stable"] and r["steps"] > 0 and
              (max_error is None or r["error_k11"] <= max_error)]
        return rows, (min(ok, key=lambda r: r["steps"]) if ok else None)
    ok = [r for r in rows if r["stable"]]
    return rows, (min(ok, key=lambda r: r[criterion]) if ok else None)
