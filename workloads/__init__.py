"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module draws random numbers and evaluates the analytic problem data
(sources, exact solutions, puncture background fields) at caller-supplied
coordinates.  It holds none of the discretisation's or the solver's
arithmetic: node positions come from whichever side (oracle or HIP library)
asks for the data, and everything returned here is plain problem input.

All random draws use ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import dataclasses

import numpy as np

# Seeds of the standard workloads.
SEED_C2 = 2
SEED_C3 = 3
SEED_C5 = 5
SEED_RANDOM_X0 = 7
SEED_APPLY = 11
SEED_ARRIVALS = 999
SEED_REQUEST_BASE = 1000


# ---------------------------------------------------------------------------
# Manufactured solution of the Poisson test (Sec. IV.A, eq. prodofsin, in 3D)
# ---------------------------------------------------------------------------
def sin_product_solution(x, y, z):
    """u = sin(pi x) sin(pi y) sin(pi z) on [0,1]^3."""
    return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def sin_product_source(x, y, z):
    """f = -Laplace(u) = 3 pi^2 sin(pi x) sin(pi y) sin(pi z)."""
    return 3.0 * np.pi ** 2 * sin_product_solution(x, y, z)


# ---------------------------------------------------------------------------
# Random-Fourier source with homogeneous Dirichlet data on a box
# ---------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class FourierModes:
    amplitudes: np.ndarray  # [M]
    wavenumbers: np.ndarray  # [M, 3], integers in 1..kmax
    lower: tuple
    upper: tuple


def fourier_modes(seed: int, lower=(0.0, 0.0, 0.0), upper=(1.0, 1.0, 1.0),
                  n_modes: int = 16, kmax: int = 4) -> FourierModes:
    """Draw ``n_modes`` modes: integer wavenumbers uniform in 1..kmax per axis
    and amplitudes from N(0,1)."""
    rng = np.random.default_rng(seed)
    k = rng.integers(1, kmax + 1, size=(n_modes, 3))
    a = rng.standard_normal(n_modes)
    return FourierModes(a, k, tuple(float(v) for v in lower),
                        tuple(float(v) for v in upper))


def _mode_products(m: FourierModes, x, y, z):
    lo, hi = m.lower, m.upper
    L = [hi[d] - lo[d] for d in range(3)]
    out = []
    for a, k in zip(m.amplitudes, m.wavenumbers):
        s = (np.sin(np.pi * k[0] * (x - lo[0]) / L[0])
             * np.sin(np.pi * k[1] * (y - lo[1]) / L[1])
             * np.sin(np.pi * k[2] * (z - lo[2]) / L[2]))
        lam = np.pi ** 2 * sum((k[d] / L[d]) ** 2 for d in range(3))
        out.append((a, s, lam))
    return out


def fourier_source(m: FourierModes, x, y, z):
    """f(x) = sum_m a_m prod_d sin(pi k_md (x_d - lo_d) / L_d)."""
    return sum(a * s for a, s, _ in _mode_products(m, x, y, z))


def fourier_solution(m: FourierModes, x, y, z):
    """Exact solution of -Laplace(u) = f with u = 0 on the box boundary."""
    return sum(a * s / lam for a, s, lam in _mode_products(m, x, y, z))


# ---------------------------------------------------------------------------
# Puncture-type nonlinear problem: Laplace(u) + beta (alpha (1+u) + 1)^-7 = 0
# ---------------------------------------------------------------------------
@dataclasses.dataclass(frozen=True)
class Punctures:
    centers: np.ndarray  # [n, 3]
    masses: np.ndarray  # [n]
    momenta: np.ndarray  # [n, 3]


def puncture_params(seed: int = SEED_C3, separation: float = 3.0,
                    mass: float = 0.5, max_momentum: float = 0.2) -> Punctures:
    """Two punctures at x = +-separation with seeded momenta |P| <= max_momentum
    (direction = normalised N(0, I3), magnitude uniform on [0, max_momentum])."""
    rng = np.random.default_rng(seed)
    centers = np.array([[separation, 0.0, 0.0], [-separation, 0.0, 0.0]])
    masses = np.array([mass, mass])
    mom = []
    for _ in range(2):
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        mom.append(d * rng.uniform(0.0, max_momentum))
    return Punctures(centers, masses, np.array(mom))


def puncture_background(pp: Punctures, x, y, z, r_min: float = 1e-14):
    """Brandt-Bruegmann background with Bowen-York extrinsic curvature.

    1/alpha = sum_n M_n / (2 r_n);  beta = (1/8) alpha^7 Abar_ij Abar^ij with
    Abar^ij = sum_n 3/(2 r_n^2) [P^i l^j + P^j l^i - (delta^ij - l^i l^j) P.l],
    l = (x - C_n)/r_n.  Returns (alpha, beta) at the given points.
    """
    X = np.stack([np.asarray(x, float), np.asarray(y, float), np.asarray(z, float)])
    inv_alpha = np.zeros(X.shape[1:])
    A = np.zeros((3, 3) + X.shape[1:])
    for c, M, P in zip(pp.centers, pp.masses, pp.momenta):
        dx = X - c.reshape((3,) + (1,) * (X.ndim - 1))
        r = np.maximum(np.sqrt((dx ** 2).sum(axis=0)), r_min)
        l = dx / r
        inv_alpha += M / (2.0 * r)
        Pl = sum(P[i] * l[i] for i in range(3))
        pref = 3.0 / (2.0 * r ** 2)
        for i in range(3):
            for j in range(3):
                A[i, j] += pref * (P[i] * l[j] + P[j] * l[i]
                                   - ((1.0 if i == j else 0.0) - l[i] * l[j]) * Pl)
    alpha = 1.0 / inv_alpha
    AA = (A ** 2).sum(axis=(0, 1))
    beta = 0.125 * alpha ** 7 * AA
    return alpha, beta


# ---------------------------------------------------------------------------
# A coupled linear system of several variables (the structure of linearised
# XCTS-like equations, Sec. IV.B, on a flat box)
# ---------------------------------------------------------------------------
SEED_SYSTEM = 21
# Neumann faces (f = 2 d + side) of each variable of the standard system:
# variable 0 plays the conformal factor with Neumann conditions on three
# faces, the others Dirichlet conditions or one Neumann face
SYSTEM_NEUMANN = ((0, 2, 4), (), (1,), (), ())


def system_coupling(seed: int, nvars: int, x, y, z, strength: float = 10.0) -> np.ndarray:
    """Pointwise coupling field c_AB(x) of shape (nvars, nvars, npoints):
    symmetric in A, B, with diagonal strength * (1 + 0.5 cos(.)) and
    off-diagonal entries of size at most strength * 0.25 / nvars (positive
    definite at every point by diagonal dominance), smooth random phases."""
    rng = np.random.default_rng(seed)
    x, y, z = (np.asarray(v, float).reshape(-1) for v in (x, y, z))
    c = np.empty((nvars, nvars, x.size))
    for a in range(nvars):
        for b in range(a, nvars):
            k = rng.uniform(1.0, 3.0, 3)
            ph = rng.uniform(0.0, 2.0 * np.pi, 3)
            wave = np.cos(k[0] * np.pi * x + ph[0]) * np.cos(k[1] * np.pi * y + ph[1]) \
                * np.cos(k[2] * np.pi * z + ph[2])
            if a == b:
                c[a, a] = strength * (1.0 + 0.5 * wave)
            else:
                c[a, b] = c[b, a] = strength * 0.25 / nvars * wave
    return c


# ---------------------------------------------------------------------------
# Generic seeded fields and the request stream of the serving workload
# ---------------------------------------------------------------------------
def wedge_coordinates(X, r_in: float, r_out: float):
    """Node coordinates of one wedge of a spherical shell (the blocks of the
    shell domain of Sec. IV.B), from logical coordinates X = (xi, eta, zeta)
    in [-1, 1]^3 (shape (3, ...)): equiangular in the two angles
    (a = tan(pi xi / 4), b = tan(pi eta / 4)), logarithmic in the radius
    r = r_in (r_out / r_in)^((zeta + 1) / 2), and x = r (a, b, 1) / |(a, b, 1)|,
    the wedge around the +z axis."""
    X = np.asarray(X, dtype=float)
    a = np.tan(np.pi / 4.0 * X[0])
    b = np.tan(np.pi / 4.0 * X[1])
    r = r_in * (r_out / r_in) ** ((X[2] + 1.0) / 2.0)
    s = r / np.sqrt(1.0 + a * a + b * b)
    return np.stack([s * a, s * b, s])


def _kerr_schild_fields(xyz, mass):
    """Background fields of a Schwarzschild black hole in Kerr-Schild
    coordinates (eq. kerrschild_bg) at the node coordinates xyz (3, ...).

    With H = M/r, l = x/r: g_ij = delta_ij + 2H l_i l_j, so g^ij = delta^ij -
    alpha^2 2H l^i l^j and sqrt(g) = (1 + 2H)^(1/2); the Kerr-Schild lapse
    alpha = (1 + 2H)^(-1/2), shift beta^i = 2H alpha^2 l^i and extrinsic
    curvature K_ij = (2 M alpha / r^2)(delta_ij - (2 + H) l_i l_j) (tangential
    eigenvalue a = 2 M alpha / r^2, radial -a alpha^2 (1 + H) of K^i_j), so
    K_ij K^ij = 2 a^2 + a^2 alpha^4 (1 + H)^2 and K = 2 M alpha^3 / r^2 (1 + 3H).
    With psi = 1, u_ij = 0 and no matter, (L beta)^ij = 2 alpha A^ij (A the
    trace-free part of K), so (L beta)_ij (L beta)^ij = 4 alpha^2 A_ij A^ij,
    and R = K_ij K^ij - K^2 (the vacuum Hamiltonian constraint)."""
    x = np.asarray(xyz, dtype=float)
    M = float(mass)
    r = np.sqrt((x * x).sum(axis=0))
    lv = x / r
    H = M / r
    alpha = 1.0 / np.sqrt(1.0 + 2.0 * H)
    ginv = (np.eye(3).reshape((3, 3) + (1,) * r.ndim) -
            (2.0 * H * alpha ** 2) * lv[:, None] * lv[None, :])
    sqrtg = np.sqrt(1.0 + 2.0 * H)
    a = 2.0 * M * alpha / r ** 2
    kr = -a * alpha ** 2 * (1.0 + H)
    KK = 2.0 * a * a + kr * kr
    K = 2.0 * a + kr
    AA = KK - K * K / 3.0
    dalpha = alpha ** 3 * M / r ** 2
    dK = 2.0 * M * ((3.0 * alpha ** 2 * dalpha / r ** 2 - 2.0 * alpha ** 3 / r ** 3) * (1.0 + 3.0 * H)
                    - 3.0 * M * alpha ** 3 / r ** 4)
    return dict(ginv=ginv, sqrtg=sqrtg, alpha=alpha, K2=K * K, R=KK - K * K,
                LL=4.0 * alpha ** 2 * AA, beta_dK=2.0 * H * alpha ** 2 * dK)


def kerr_schild_lapse(xyz, mass: float = 1.0):
    """The lapse equation of the XCTS system (eq. xcts_lapse) on the
    Kerr-Schild background (eq. kerrschild_bg), with psi = 1 and the shift
    held at its Kerr-Schild value (eq. kerrschild_shift), at the node
    coordinates xyz (3, ...).  For Phi = alpha psi it reads
      Laplace_g Phi = c_-1 / Phi + c_1 Phi + c_0,
      c_-1 = 7/32 (L beta)_ij (L beta)^ij,  c_1 = 5/12 K^2 + R / 8,
      c_0 = beta^i d_i K,
    with exact solution Phi = alpha (eq. kerrschild_lapse).  Returns g^ij
    (3, 3, ...), sqrt(g), alpha, the coefficients (3, ...) and their powers
    (-1, 1, 0)."""
    f = _kerr_schild_fields(xyz, mass)
    coefs = np.stack([7.0 / 32.0 * f["LL"], 5.0 / 12.0 * f["K2"] + f["R"] / 8.0, f["beta_dK"]])
    return f["ginv"], f["sqrtg"], f["alpha"], coefs, (-1, 1, 0)


def kerr_schild_xcts(xyz, mass: float = 1.0):
    """The Hamiltonian and lapse equations of the XCTS system (eqs.
    xcts_hamiltonian, xcts_lapse) for psi and Phi = alpha psi on the
    Kerr-Schild background, the shift held at its Kerr-Schild value, at the
    node coordinates xyz (3, ...).  With alpha_bar = Phi psi^-7,
    A_ij A^ij = (L beta)^2 psi^14 / (4 Phi^2), so the right-hand sides are
    sums of monomials in (psi, Phi):
      Laplace_g psi = R/8 psi + K^2/12 psi^5 - (L beta)^2/32 psi^7 Phi^-2,
      Laplace_g Phi = 7 (L beta)^2/32 psi^6 Phi^-1 + 5 K^2/12 psi^4 Phi
                      + R/8 Phi + beta^i d_i K psi^5,
    with exact solution psi = 1, Phi = alpha (eqs. kerrschild_psi,
    kerrschild_lapse).  Returns g^ij, sqrt(g), alpha and, per variable, the
    list of (coefficient field, (power of psi, power of Phi))."""
    f = _kerr_schild_fields(xyz, mass)
    LL, K2, R = f["LL"], f["K2"], f["R"]
    terms = [[(R / 8.0, (1, 0)), (K2 / 12.0, (5, 0)), (-LL / 32.0, (7, -2))],
             [(7.0 * LL / 32.0, (6, -1)), (5.0 * K2 / 12.0, (4, 1)), (R / 8.0, (0, 1)),
              (f["beta_dK"], (5, 0))]]
    return f["ginv"], f["sqrtg"], f["alpha"], terms


def pullback_metric(X, lower, upper, amplitude: float, direction=(1.0, 0.7, 0.4)):
    """A curved background metric with known harmonic functions: the pullback
    g = J^T J of the flat metric under the box map
    phi(X) = X + a c prod_d sin(pi (X_d - lo_d) / L_d) (which keeps the box
    boundary in place), with its analytic Jacobian J.  X: node coordinates,
    shape (3, ...).  Returns phi(X) (3, ...), g^ij (3, 3, ...) and sqrt(det g)
    (...); for h harmonic in flat space, u = h(phi(X)) solves the
    Laplace-Beltrami equation of g."""
    X = np.asarray(X, dtype=float)
    lo = np.asarray(lower, float)
    L = np.asarray(upper, float) - lo
    c = np.asarray(direction, float)
    ext = (slice(None),) + (None,) * (X.ndim - 1)
    S = [np.sin(np.pi * (X[d] - lo[d]) / L[d]) for d in range(3)]
    Co = [np.cos(np.pi * (X[d] - lo[d]) / L[d]) for d in range(3)]
    bump = S[0] * S[1] * S[2]
    dbump = [np.pi / L[0] * Co[0] * S[1] * S[2], np.pi / L[1] * S[0] * Co[1] * S[2],
             np.pi / L[2] * S[0] * S[1] * Co[2]]
    J = np.empty((3, 3) + X.shape[1:])
    for i in range(3):
        for j in range(3):
            J[i, j] = (1.0 if i == j else 0.0) + amplitude * c[i] * dbump[j]
    phi = X + amplitude * c[ext] * bump
    g = np.einsum("ki...,kj...->...ij", J, J)
    ginv = np.moveaxis(np.linalg.inv(g), (-2, -1), (0, 1))
    return phi, ginv, np.sqrt(np.linalg.det(g))


def random_normal(seed: int, n: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(n)


def random_uniform(seed: int, n: int, lo=-0.5, hi=0.5) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n)


@dataclasses.dataclass(frozen=True)
class Request:
    index: int
    seed: int
    arrival: float  # seconds after the stream starts
    elements: tuple  # (nx, ny, nz)
    p: int
    side: float  # domain [0, side]^3


def request_stream(n: int = 256, rate: float = 1.0, seed: int = SEED_ARRIVALS,
                   cube_elements: bool = False, p_range=(3, 8), n_range=(2, 6),
                   sides=(1, 2, 3, 4)) -> list:
    """Poisson-process arrivals (exponential gaps of mean 1/rate).  Request i
    draws its grid, degree and side from seed 1000+i."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n):
        r = np.random.default_rng(SEED_REQUEST_BASE + i)
        if cube_elements:
            m = int(r.integers(n_range[0], n_range[1] + 1))
            el = (m, m, m)
        else:
            el = tuple(int(v) for v in r.integers(n_range[0], n_range[1] + 1, size=3))
        p = int(r.integers(p_range[0], p_range[1] + 1))
        side = float(sides[int(r.integers(0, len(sides)))])
        out.append(Request(i, SEED_REQUEST_BASE + i, float(t[i]), el, p, side))
    return out
