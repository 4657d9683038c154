"""Independent per-Fourier-mode model of the scheme (test-side pin).

Built only from what the paper prints for the linear stability analysis
(Sec. 5): the transform M (golden file of the printed matrix), the
equilibrium map of Table "scheme", the diagonal relaxation matrix Lambda and
the one-step operator of Eq. lbmvector, A = M^-1 Lambda M_eq + M^-1 (I - Lambda) M,
with the propagation factor diag(exp(-i k.c)) of the stability matrix L.
The forcing enters as in Eqs. coll10/coll10post (first-order moments gain g)
and through the equilibria m12_eq = theta*mbar10, m21_eq = theta*mbar01,
which see g/2.

It shares nothing with the oracle: the oracle builds its transform from the
moment definitions and runs Algorithm 1 node by node in real space; this
module works on one Fourier mode at a time with 8x8 complex matrices.

Reading adopted for the equilibrium map: the matrix M_eq printed in Sec. 5
has, in rows 12 and 21, theta times the rows of m12 and m21 themselves,
which would make the equilibria depend on m12 and m21.  Table "scheme" and
Sec. 3.3.2 define m12_eq = theta*mbar10 and m21_eq = theta*mbar01, so those
rows are theta times the rows of m10 and m01 here.
"""
from __future__ import annotations

import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def printed_M() -> np.ndarray:
    return np.loadtxt(os.path.join(GOLDEN, "moment_matrix_M.txt"))


def printed_velocities() -> np.ndarray:
    v = np.loadtxt(os.path.join(GOLDEN, "velocities.txt"), dtype=int)
    return v[:, 1:3].astype(float)  # (8, 2): c_i


def rates_from_table(lame_lambda: float, lame_mu: float, theta: float = 1.0 / 3.0):
    """Table "scheme": tau_11 = mu/theta, tau_s = 2K/(1+theta), tau_d = 2mu/(1-theta);
    omega = 1/(tau + 1/2)."""
    K = lame_lambda + lame_mu
    t11, ts, td = lame_mu / theta, 2 * K / (1 + theta), 2 * lame_mu / (1 - theta)
    return 1 / (t11 + 0.5), 1 / (ts + 0.5), 1 / (td + 0.5)


class ModeModel:
    """8x8 operators of the scheme for given material / rates."""

    def __init__(self, lame_lambda: float, lame_mu: float, theta: float = 1.0 / 3.0,
                 w12: float = 1.0, w21: float = 1.0, w22: float = 1.0):
        self.theta = theta
        w11, ws, wd = rates_from_table(lame_lambda, lame_mu, theta)
        self.M = printed_M()
        self.Minv = np.linalg.inv(self.M)
        self.c = printed_velocities()
        Meq = np.zeros((8, 8))
        Meq[0] = self.M[0]  # 10 (rate 0: not relaxed)
        Meq[1] = self.M[1]  # 01
        Meq[5] = theta * self.M[0]  # m12_eq = theta * m10
        Meq[6] = theta * self.M[1]  # m21_eq = theta * m01
        self.Meq = Meq
        self.Lam = np.diag([0.0, 0.0, w11, ws, wd, w12, w21, w22])
        I = np.eye(8)
        self.A = self.Minv @ self.Lam @ Meq + self.Minv @ (I - self.Lam) @ self.M
        # forcing: m10* gains gx, m01* gains gy; m12*, m21* gain w*theta*g/2
        G = np.zeros((8, 2))
        G[0, 0] = 1.0
        G[1, 1] = 1.0
        G[5, 0] = w12 * theta / 2
        G[6, 1] = w21 * theta / 2
        self.B = self.Minv @ G
        self.rates = (w11, ws, wd)

    def propagation(self, kx: float, ky: float) -> np.ndarray:
        """diag(exp(-i k.c_q)): f(x + c, n+1) = f*(x, n) for a mode e^{i k.x}."""
        return np.diag(np.exp(-1j * (self.c[:, 0] * kx + self.c[:, 1] * ky)))

    def L(self, kx: float, ky: float) -> np.ndarray:
        return self.propagation(kx, ky) @ self.A

    def spectral_radius(self, kx: float, ky: float) -> float:
        return float(np.max(np.abs(np.linalg.eigvals(self.L(kx, ky)))))

    def transient_u(self, kx: float, ky: float, ghat: np.ndarray, n: int) -> np.ndarray:
        """Complex displacement amplitude after n steps from f = 0 under the load
        mode ghat (complex 2-vector): f(n+1) = D (A f(n) + B g); u = (M f)[0:2] + g/2."""
        D = self.propagation(kx, ky)
        f = np.zeros(8, complex)
        for _ in range(n):
            f = D @ (self.A @ f + self.B @ ghat)
        return (self.M @ f)[:2] + ghat / 2

    def steady_u(self, kx: float, ky: float, ghat: np.ndarray) -> np.ndarray:
        """Steady state f = (I - L)^-1 D B g (k != 0)."""
        D = self.propagation(kx, ky)
        f = np.linalg.solve(np.eye(8) - D @ self.A, D @ self.B @ ghat)
        return (self.M @ f)[:2] + ghat / 2


def sample_mode(amp_u: np.ndarray, kx: float, ky: float, nx: int, ny: int):
    """Real field Re(amp e^{i k.x}) at nodes (i + 1/2, j + 1/2), both components."""
    x = np.arange(nx) + 0.5
    y = np.arange(ny) + 0.5
    ph = np.exp(1j * (kx * x[None, :] + ky * y[:, None]))
    return (amp_u[0] * ph).real, (amp_u[1] * ph).real


def paper_k_grid(npts_k: int = 50, npts_phi: int = 5):
    """Wave vectors of the stability scan in Sec. 5: |k| in [0, pi] at 50 points,
    angle in [0, pi/4] at 5 points."""
    for kh in np.linspace(0.0, np.pi, npts_k):
        for ph in np.linspace(0.0, np.pi / 4, npts_phi):
            yield kh * np.cos(ph), kh * np.sin(ph)


def sup_rho(model: ModeModel, grid=None) -> float:
    grid = paper_k_grid() if grid is None else grid
    return max(model.spectral_radius(kx, ky) for kx, ky in grid)
