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


# ---------------------------------------------------------------------------
# leading-order error symbols of the exact scheme (mpmath, high precision)
# ---------------------------------------------------------------------------

def _mp_operators(lame_lambda, lame_mu, theta, w12, w21, w22, mp):
    """The one-step operator A and forcing B of ModeModel, in mpmath."""
    Mp = mp.matrix(printed_M().tolist())
    Minv = Mp ** -1
    th = mp.mpf(theta)
    K = mp.mpf(lame_lambda) + mp.mpf(lame_mu)
    mu = mp.mpf(lame_mu)
    t11, ts, td = mu / th, 2 * K / (1 + th), 2 * mu / (1 - th)
    w = [mp.mpf(0), mp.mpf(0), 1 / (t11 + mp.mpf(1) / 2), 1 / (ts + mp.mpf(1) / 2),
         1 / (td + mp.mpf(1) / 2), mp.mpf(w12), mp.mpf(w21), mp.mpf(w22)]
    Meq = mp.zeros(8, 8)
    for c in range(8):
        Meq[0, c], Meq[1, c] = Mp[0, c], Mp[1, c]
        Meq[5, c], Meq[6, c] = th * Mp[0, c], th * Mp[1, c]
    Lam = mp.diag(w)
    A = Minv * Lam * Meq + Minv * (mp.eye(8) - Lam) * Mp
    G = mp.zeros(8, 2)
    G[0, 0] = G[1, 1] = 1
    G[5, 0], G[6, 1] = w[5] * th / 2, w[6] * th / 2
    return Mp, A, Minv * G


def slow_symbols(lame_lambda, lame_mu, kx, ky, theta=1.0 / 3.0, w12=1.0, w21=1.0, w22=1.0):
    """For one wavevector k, the exact scheme restricted to its two slow modes,
    written as a continuous-time law for the bared first moments:
    du/dt = S(k) u + G(k) g.  S = W log(Lambda_s) W^-1 with Lambda_s the two
    eigenvalues of L(k) nearest 1 and W the first moments of their
    eigenvectors; G = -S T(k) with T the exact steady response (both laws have
    the same decay and the same steady state).  Returns (S, G) as mpmath
    2 x 2 matrices at the caller's mpmath precision."""
    import mpmath as mpm

    Mp, A, B = _mp_operators(lame_lambda, lame_mu, theta, w12, w21, w22, mpm)
    c = printed_velocities()
    kx, ky = mpm.mpf(kx), mpm.mpf(ky)
    D = mpm.diag([mpm.exp(-1j * (int(c[q, 0]) * kx + int(c[q, 1]) * ky)) for q in range(8)])
    L = D * A
    ev, R = mpm.eig(L)
    idx = sorted(range(8), key=lambda i: abs(ev[i] - 1))[:2]
    W = mpm.matrix(2, 2)
    for a, i in enumerate(idx):
        for r in range(2):
            W[r, a] = sum(Mp[r, q] * R[q, i] for q in range(8))
    S = W * mpm.diag([mpm.log(ev[i]) for i in idx]) * W ** -1
    F = (mpm.eye(8) - L) ** -1 * D * B
    T = mpm.matrix(2, 2)
    for r in range(2):
        for s_ in range(2):
            T[r, s_] = sum(Mp[r, q] * F[q, s_] for q in range(8)) + (mpm.mpf(1) / 2 if r == s_ else 0)
    return S, -S * T


def leading_error_symbols(lame_lambda, lame_mu, theta=1.0 / 3.0, w12=1.0, w21=1.0, w22=1.0,
                          k=1e-7, dps=60):
    """Constants of the leading-order error law du2/dt = L0 u2 + r4, with
    r4_x = C1 u0x_xxxx + C2 u0y_xxxy + C3 u0x_xxyy + C4 u0y_xyyy + C5 u0x_yyyy
           + D1 gx_xx + D2 gy_xy + D3 gx_yy,
    read off the exact slow law at small |k|: S + (mu|k|^2 I + K k k^T) is the
    quartic symbol of the C terms, G - I the quadratic symbol of the D terms
    (d_x -> i k_x), at dps decimal digits.  Returns (x-row dict, y-row dict)."""
    import mpmath

    old = mpmath.mp.dps
    mpmath.mp.dps = dps
    try:
        return _leading_error_symbols(lame_lambda, lame_mu, theta, w12, w21, w22, k)
    finally:
        mpmath.mp.dps = old


def _leading_error_symbols(lame_lambda, lame_mu, theta, w12, w21, w22, k):
    import mpmath

    K = mpmath.mpf(lame_lambda) + mpmath.mpf(lame_mu)
    mu = mpmath.mpf(lame_mu)
    kk = mpmath.mpf(k)

    def quartic(kx, ky):
        S, G = slow_symbols(lame_lambda, lame_mu, kx, ky, theta, w12, w21, w22)
        A0 = mpmath.matrix([[mu * (kx * kx + ky * ky) + K * kx * kx, K * kx * ky],
                            [K * kx * ky, mu * (kx * kx + ky * ky) + K * ky * ky]])
        return S + A0, G - mpmath.eye(2)

    out = []
    for row in (0, 1):
        ox = 1 - row  # the other component
        s_a, g_a = quartic(kk, 0)          # along x
        s_b, g_b = quartic(0, kk)          # along y
        s_d, g_d = quartic(kk, kk)         # diagonal
        s_e, _ = quartic(2 * kk, kk)       # (2, 1) direction
        if row == 0:
            c1 = s_a[0, 0] / kk ** 4
            c5 = s_b[0, 0] / kk ** 4
            d1 = -g_a[0, 0] / kk ** 2
            d3 = -g_b[0, 0] / kk ** 2
        else:  # the y row mirrors x <-> y: C1 multiplies u0y_yyyy, C5 u0y_xxxx
            c1 = s_b[1, 1] / kk ** 4
            c5 = s_a[1, 1] / kk ** 4
            d1 = -g_b[1, 1] / kk ** 2
            d3 = -g_a[1, 1] / kk ** 2
        c3 = s_d[row, row] / kk ** 4 - c1 - c5
        d2 = -g_d[row, ox] / kk ** 2
        sum_d = s_d[row, ox] / kk ** 4      # C2 + C4
        if row == 0:
            sum_e = s_e[0, 1] / kk ** 4     # k = (2k, k): 8 C2 + 2 C4
            c2 = (sum_e - 2 * sum_d) / 6
        else:
            sum_e = s_e[1, 0] / kk ** 4     # C2 u0x_yyyx + C4 u0x_yxxx: 2 C2 + 8 C4
            c2 = (8 * sum_d - sum_e) / 6
        c4 = sum_d - c2
        out.append({k_: float(mpmath.re(v)) for k_, v in
                    (("C1", c1), ("C2", c2), ("C3", c3), ("C4", c4), ("C5", c5),
                     ("D1", d1), ("D2", d2), ("D3", d3))})
    return out[0], out[1]
