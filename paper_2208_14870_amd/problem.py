"""Problem definition and seeded synthetic inputs (FP64, host side).

This module describes the *continuum* problem that the lattice Boltzmann
scheme solves -- the damped Navier-Cauchy equation on a periodic box
(Sec. 2.1, Eqs. linelasdamp/periodicity) with the 2D material relations of
Eq. material_relations -- and generates the seeded inputs of every workload:
manufactured solutions with their analytic body forces (Sec. 7.2, Eq.
manu_eq), random smooth Fourier forces, batches of uneven lattices and
request streams.  It contains none of the lattice Boltzmann arithmetic: both
the GPU library and the CPU oracle receive the arrays made here and nothing
else from this module.

Units: lattice units (dx = dt = 1, kappa = 1, U = 1).  A lattice of n nodes
per side covers the periodic box [0, n) with nodes at i + 1/2 (the lattice is
offset by half a spacing from the domain edge, Sec. 6.1).  Material
parameters are the lattice diffusivities lambda~, mu~, K~ = lambda~ + mu~
(Eq. scaling_example), and the per-step force g equals the body load b in
these units.

Fields are arrays of shape (ny, nx), x fastest, float64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Sequence, Tuple

import numpy as np


# ---------------------------------------------------------------------------
# material relations (Eq. material_relations, 2D -- not plane strain/stress)
# ---------------------------------------------------------------------------

@dataclasses.dataclass(frozen=True)
class Material:
    """Isotropic material in lattice units: Lame parameters lambda, mu."""
    lame_lambda: float
    lame_mu: float

    @property
    def bulk(self) -> float:
        """K = lambda + mu."""
        return self.lame_lambda + self.lame_mu

    @property
    def young(self) -> float:
        """E = 2 mu (1 + nu)."""
        return 2.0 * self.lame_mu * (1.0 + self.poisson)

    @property
    def poisson(self) -> float:
        """nu = lambda / (lambda + 2 mu) in the 2D relations."""
        return self.lame_lambda / (self.lame_lambda + 2.0 * self.lame_mu)

    @staticmethod
    def from_young_poisson(E: float, nu: float) -> "Material":
        """lambda = E nu/(1 - nu^2), mu = E/(2(1 + nu))."""
        return Material(E * nu / (1.0 - nu * nu), E / (2.0 * (1.0 + nu)))

    @staticmethod
    def from_shear_poisson(mu: float, nu: float) -> "Material":
        """lambda = 2 mu nu/(1 - nu), so that K = mu (1 + nu)/(1 - nu)."""
        return Material(2.0 * mu * nu / (1.0 - nu), mu)


# ---------------------------------------------------------------------------
# plane-wave fields and the continuum operator
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class PlaneWaveField:
    """Vector field v(x) = sum_m Re(A_m exp(i k_m . x)), A_m in C^2, k_m in R^2
    (angular wavenumbers in lattice units)."""
    k: np.ndarray  # (M, 2) float
    amp: np.ndarray  # (M, 2) complex

    def evaluate(self, nx: int, ny: int) -> Tuple[np.ndarray, np.ndarray]:
        """Sample both components at the nodes (i + 1/2, j + 1/2)."""
        x = np.arange(nx, dtype=np.float64) + 0.5
        y = np.arange(ny, dtype=np.float64) + 0.5
        m = len(self.k)
        if m == 0:
            return np.zeros((ny, nx)), np.zeros((ny, nx))
        # Re(A e^{i(kx x + ky y)}) = Re(A e^{i kx x}) cos(ky y) - Im(A e^{i kx x}) sin(ky y):
        # one small matrix product per component keeps large lattices cheap.
        ex = np.exp(1j * np.outer(self.k[:, 0], x))  # (M, nx)
        cy = np.cos(np.outer(y, self.k[:, 1]))  # (ny, M)
        sy = np.sin(np.outer(y, self.k[:, 1]))
        out = []
        for c in range(2):
            ax = self.amp[:, c:c + 1] * ex  # (M, nx)
            out.append(cy @ ax.real - sy @ ax.imag)
        return out[0], out[1]

    def second_derivatives(self, nx: int, ny: int) -> Tuple[np.ndarray, np.ndarray]:
        """Analytic second derivatives at the nodes: for each component the
        planes (d_xx, d_xy, d_yy), shape (3, ny, nx) each (d_x of a mode is
        i k_x, so d_xx -> -k_x^2, d_xy -> -k_x k_y, d_yy -> -k_y^2)."""
        planes = ([], [])
        for fac in (-self.k[:, 0] ** 2, -self.k[:, 0] * self.k[:, 1], -self.k[:, 1] ** 2):
            vx, vy = PlaneWaveField(self.k, self.amp * fac[:, None]).evaluate(nx, ny)
            planes[0].append(vx)
            planes[1].append(vy)
        return np.stack(planes[0]), np.stack(planes[1])

    def scaled(self, s: float) -> "PlaneWaveField":
        return PlaneWaveField(self.k.copy(), self.amp * s)

    def rms(self) -> float:
        """Root-mean-square over the box for distinct, non-zero wavevectors
        (each real plane wave has mean square |A|^2 / 2)."""
        return float(np.sqrt(0.5 * np.sum(np.abs(self.amp) ** 2)))


def body_force_of(u: PlaneWaveField, mat: Material) -> PlaneWaveField:
    """Manufactured body load b = -mu lap(u) - K grad(div u) (Eq. manu_eq with a
    time-independent solution), mode by mode: b_hat = mu |k|^2 A + K k (k . A)."""
    k2 = np.sum(u.k ** 2, axis=1)[:, None]
    kdotA = np.sum(u.k * u.amp, axis=1)[:, None]
    return PlaneWaveField(u.k.copy(), mat.lame_mu * k2 * u.amp + mat.bulk * u.k * kdotA)


def solution_of(b: PlaneWaveField, mat: Material) -> PlaneWaveField:
    """Continuum steady state for a plane-wave load: solve
    (mu |k|^2 I + K k k^T) A = b_hat per mode (k != 0)."""
    amps = np.zeros_like(b.amp)
    for m, (kv, bh) in enumerate(zip(b.k, b.amp)):
        op = mat.lame_mu * float(kv @ kv) * np.eye(2) + mat.bulk * np.outer(kv, kv)
        amps[m] = np.linalg.solve(op.astype(complex), bh)
    return PlaneWaveField(b.k.copy(), amps)


def stress_of(u: PlaneWaveField, mat: Material, nx: int, ny: int):
    """Continuum Cauchy stress of a displacement field at the nodes, lattice
    units (Eq. stress with the 2D relations): sigma = K div(u) I +
    mu (grad u + grad u^T - div(u) I).  Returns (sxx, syy, sxy)."""
    def grad(c, axis):  # d u_c / d x_axis, mode by mode (multiply by i k)
        return PlaneWaveField(u.k, u.amp * (1j * u.k[:, axis])[:, None]).evaluate(nx, ny)[c]
    dxx, dxy = grad(0, 0), grad(0, 1)
    dyx, dyy = grad(1, 0), grad(1, 1)
    div = dxx + dyy
    K, mu = mat.bulk, mat.lame_mu
    return (K * div + mu * (2.0 * dxx - div), K * div + mu * (2.0 * dyy - div),
            mu * (dxy + dyx))


def trig_product(coef: Sequence[float], fx: Sequence[str], fy: Sequence[str], kx: float,
                 ky: float) -> PlaneWaveField:
    """Field with components coef[c] * T(kx x) * T'(ky y), T in {cos, sin}, as two
    plane waves (product-to-sum identities; cos -> 1, sin -> -i as Re factors)."""
    amp_p = np.zeros(2, complex)  # wavevector (kx, ky)
    amp_m = np.zeros(2, complex)  # wavevector (kx, -ky)
    for c in range(2):
        a, tx, ty = coef[c], fx[c], fy[c]
        if (tx, ty) == ("c", "c"):  # cos a cos b = [cos(a+b) + cos(a-b)]/2
            p, m = 0.5, 0.5
        elif (tx, ty) == ("c", "s"):  # cos a sin b = [sin(a+b) - sin(a-b)]/2
            p, m = -0.5j, 0.5j
        elif (tx, ty) == ("s", "c"):  # sin a cos b = [sin(a+b) + sin(a-b)]/2
            p, m = -0.5j, -0.5j
        elif (tx, ty) == ("s", "s"):  # sin a sin b = [cos(a-b) - cos(a+b)]/2
            p, m = -0.5, 0.5
        else:
            raise ValueError((tx, ty))
        amp_p[c] = a * p
        amp_m[c] = a * m
    return PlaneWaveField(np.array([[kx, ky], [kx, -ky]], float), np.stack([amp_p, amp_m]))


def remove_mean(a: np.ndarray) -> np.ndarray:
    """Project out the mean (FP64).  A periodic steady state needs a zero-mean
    load because the mean of u is conserved from u0 = 0 (Sec. 7.2)."""
    return a - np.mean(a, dtype=np.float64)


@dataclasses.dataclass
class Case:
    """One periodic elasticity problem on an nx x ny lattice (lattice units)."""
    nx: int
    ny: int
    material: Material
    gx: np.ndarray
    gy: np.ndarray
    ux_exact: np.ndarray | None = None  # continuum solution at the nodes, if known
    uy_exact: np.ndarray | None = None
    label: str = ""
    # analytic second derivatives of the load, planes (d_xx, d_xy, d_yy) per
    # component, when known (input of the improved scheme's force correction)
    d2gx: np.ndarray | None = None
    d2gy: np.ndarray | None = None
    u_field: PlaneWaveField | None = None  # the manufactured solution, if any


def manufactured_case(n: int, mat: Material, u: PlaneWaveField, label: str = "",
                      ny: int | None = None) -> Case:
    ny = n if ny is None else ny
    b = body_force_of(u, mat)
    gx, gy = b.evaluate(n, ny)
    ux, uy = u.evaluate(n, ny)
    d2gx, d2gy = b.second_derivatives(n, ny)
    return Case(n, ny, mat, remove_mean(gx), remove_mean(gy), ux, uy, label, d2gx, d2gy, u)


def sin_cos_solution(n: int, amp: float, kx: int = 1, ky: int = 1) -> PlaneWaveField:
    """u = (A sin(a_x x) cos(a_y y), A cos(a_x x) sin(a_y y)), a = 2 pi k / n."""
    ax, ay = 2.0 * math.pi * kx / n, 2.0 * math.pi * ky / n
    return trig_product((amp, amp), ("s", "c"), ("c", "s"), ax, ay)


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def single_32(amp: float = 1e-3) -> Case:
    """32 x 32, nu = 0.3, mu = 1, sinusoidal manufactured solution, mode (1,1)."""
    mat = Material.from_shear_poisson(1.0, 0.3)
    return manufactured_case(32, mat, sin_cos_solution(32, amp), "single-32")


def single_1024(nu: float, kx: int, ky: int, amp: float = 1e-3, n: int = 1024) -> Case:
    """1024 x 1024, mu = 1, Poisson ratio nu, sinusoidal solution with mode (kx, ky)."""
    mat = Material.from_shear_poisson(1.0, nu)
    return manufactured_case(n, mat, sin_cos_solution(n, amp, kx, ky),
                             f"single-{n}-nu{nu}-k{kx}{ky}")


SWEEP_1024 = [(nu, k) for nu in (0.1, 0.3, 0.45, 0.49) for k in ((1, 1), (4, 3))]


def paper_e1(n: int) -> Case:
    """The first convergence study (Sec. 7.3.1): nu = 0.8, E~ = 0.11 and
    u/U = (9e-4 cos(2 pi x~) sin(2 pi y~), 7e-4 sin(2 pi x~) cos(2 pi y~)) on [0, L]^2
    with n nodes per side (dx = L/n)."""
    mat = Material.from_young_poisson(0.11, 0.8)
    a = 2.0 * math.pi / n
    u = trig_product((9e-4, 7e-4), ("c", "s"), ("s", "c"), a, a)
    return manufactured_case(n, mat, u, f"paper-e1-{n}")


def paper_e2(n: int) -> Case:
    """The convergence study of the improved scheme (Sec. 7.3.2): the load of
    the first study at nu = 0.8, E~ = 0.085 (with its analytic second
    derivatives for the force correction)."""
    mat = Material.from_young_poisson(0.085, 0.8)
    a = 2.0 * math.pi / n
    u = trig_product((9e-4, 7e-4), ("c", "s"), ("s", "c"), a, a)
    return manufactured_case(n, mat, u, f"paper-e2-{n}")


def paper_e3(n: int, young: float = 0.085, nu: float = 0.8) -> Case:
    """The special case with no mixed derivatives (Sec. 7.3.3):
    u/U = (9e-4 (cos(2 pi x~) + sin(2 pi y~)), 7e-4 (sin(2 pi x~) + cos(2 pi y~))).
    The paper does not state the material; the improved scheme's nu = 0.8,
    E~ = 0.085 by default."""
    mat = Material.from_young_poisson(young, nu)
    a = 2.0 * math.pi / n
    # cos -> amplitude 1, sin -> -i (Re(A e^{i k.x}))
    u = PlaneWaveField(np.array([[a, 0.0], [0.0, a]]),
                       np.array([[9e-4, -7e-4j], [-9e-4j, 7e-4]], complex))
    return manufactured_case(n, mat, u, f"paper-e3-{n}")


def gaussian_hill_case(n: int, mat: Material,
                       sig: Sequence[float] = (120 ** -0.5, 123 ** -0.5, 118 ** -0.5,
                                               125 ** -0.5),
                       amp: float = 1e-3) -> Case:
    """Gaussian-hill manufactured solution of the stability study (Sec. 7.3.5,
    Eqs. gaussian_x/gaussian_y, Table std_gauss) on [0, L]^2 with n nodes per side;
    the erf offset makes the continuum solution mean-free.  The body load is the
    analytic b = -mu lap(u) - K grad(div u) in lattice units."""
    x = (np.arange(n) + 0.5) / n  # x~ = x / L
    X, Y = np.meshgrid(x, x)  # (ny, nx)
    h = 1.0 / n  # d/dx (lattice) = h * d/dx~

    def hill(s1, s2):
        G = np.exp(-((X - 0.5) ** 2) / s1 ** 2) * np.exp(-((Y - 0.5) ** 2) / s2 ** 2)
        off = math.pi * s1 * s2 * math.erf(1.0 / (2 * s1)) * math.erf(1.0 / (2 * s2))
        gxx = (4 * (X - 0.5) ** 2 / s1 ** 4 - 2 / s1 ** 2) * G
        gyy = (4 * (Y - 0.5) ** 2 / s2 ** 4 - 2 / s2 ** 2) * G
        gxy = (4 * (X - 0.5) * (Y - 0.5) / (s1 ** 2 * s2 ** 2)) * G
        return amp * (G - off), amp * gxx * h * h, amp * gyy * h * h, amp * gxy * h * h

    ux, uxxx, uxyy, uxxy = hill(sig[0], sig[1])
    uy, uyxx, uyyy, uyxy = hill(sig[2], sig[3])
    mu, K = mat.lame_mu, mat.bulk
    bx = -(mu * (uxxx + uxyy) + K * (uxxx + uyxy))
    by = -(mu * (uyxx + uyyy) + K * (uxxy + uyyy))
    return Case(n, n, mat, remove_mean(bx), remove_mean(by), ux, uy, f"gauss-{n}")


def random_fourier_load(n: int, nmodes: int, kmax: int, seed: int, mat: Material,
                        u_rms: float = 1e-3, ny: int | None = None) -> Tuple[PlaneWaveField,
                                                                             PlaneWaveField]:
    """Random smooth load: `nmodes` distinct wavevectors (integers in
    [-kmax, kmax]^2 minus 0, one per +-k pair); per component an amplitude
    ~ N(0,1) |k|^-2 and a phase ~ U[0, 2 pi); g_c = sum a cos(2 pi k.x/n + phi).
    Rescaled so that the continuum solution has RMS `u_rms`.
    Returns (load, continuum solution) as plane-wave fields."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    cand = [(i, j) for i in range(-kmax, kmax + 1) for j in range(-kmax, kmax + 1)
            if (i, j) != (0, 0) and (i > 0 or (i == 0 and j > 0))]  # one per +-k pair
    pick = rng.choice(len(cand), size=nmodes, replace=False)
    ks = np.array([cand[p] for p in pick], float)
    kvec = 2.0 * math.pi * np.stack([ks[:, 0] / n, ks[:, 1] / ny], axis=1)
    kmag = np.sqrt(np.sum(ks ** 2, axis=1))
    a = rng.standard_normal((nmodes, 2)) * kmag[:, None] ** -2.0
    phi = rng.uniform(0.0, 2.0 * math.pi, size=(nmodes, 2))
    load = PlaneWaveField(kvec, a * np.exp(1j * phi))
    sol = solution_of(load, mat)
    s = u_rms / sol.rms()
    return load.scaled(s), sol.scaled(s)


def random_load_case(n: int, nmodes: int, kmax: int, seed: int, mat: Material,
                     label: str = "", with_exact: bool = True) -> Case:
    load, sol = random_fourier_load(n, nmodes, kmax, seed, mat)
    gx, gy = load.evaluate(n, n)
    ux = uy = None
    if with_exact:
        ux, uy = sol.evaluate(n, n)
    return Case(n, n, mat, remove_mean(gx), remove_mean(gy), ux, uy, label)


def single_8192(seed: int = 3, n: int = 8192, with_exact: bool = False) -> Case:
    """8192 x 8192, nu = 0.3, mu = 1, 16 random Fourier modes with |k|_inf <= 8,
    amplitudes decaying as |k|^-2, solution RMS 1e-3."""
    mat = Material.from_shear_poisson(1.0, 0.3)
    return random_load_case(n, 16, 8, seed, mat, f"single-{n}-random16", with_exact)


BATCH_SIDES = (64, 96, 128, 192, 256, 384, 512)


def batch_cases(count: int = 512, seed: int = 4, sides: Sequence[int] = BATCH_SIDES) -> List[Case]:
    """Batch of independent lattices: side uniform over `sides`, nu ~ U[0.05, 0.48],
    mu = 1, sinusoidal solution of amplitude 1e-3 with mode (kx, ky) ~ U{1..4}^2."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(sides))
        nu = float(rng.uniform(0.05, 0.48))
        kx, ky = (int(v) for v in rng.integers(1, 5, size=2))
        mat = Material.from_shear_poisson(1.0, nu)
        out.append(manufactured_case(n, mat, sin_cos_solution(n, 1e-3, kx, ky),
                                     f"batch-{i}-n{n}-nu{nu:.3f}-k{kx}{ky}"))
    return out


@dataclasses.dataclass
class Request:
    """One elasticity solve arriving at `t_arrival` seconds after the start."""
    rid: int
    t_arrival: float
    n: int
    nu: float
    seed: int

    def case(self) -> Case:
        mat = Material.from_shear_poisson(1.0, self.nu)
        return random_load_case(self.n, 8, 4, self.seed, mat, f"req-{self.rid}", False)


def request_stream(rate_hz: float = 2000.0, duration_s: float = 5.0, seed: int = 5,
                   nmin: int = 64, nmax: int = 2048) -> List[Request]:
    """Poisson arrivals (exponential gaps) at `rate_hz`; side log-uniform in
    [nmin, nmax] (n = round(nmin * (nmax/nmin)^U)); nu ~ U[0.05, 0.49]; each
    request carries its own seed for an 8-mode load with |k|_inf <= 4."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        u = float(rng.uniform())
        n = int(round(nmin * (nmax / nmin) ** u))
        nu = float(rng.uniform(0.05, 0.49))
        out.append(Request(len(out), t, n, nu, int(rng.integers(1 << 31))))
    return out
