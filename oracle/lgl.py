"""Legendre-Gauss-Lobatto collocation (Sec. II, eqs. field_expansion, lagrprod).

Test infrastructure only: imported by the tests, smoke() and the benchmark's
CPU leg, never by the product path.

Fields are nodal values at N = p+1 LGL points per dimension; the basis is the
tensor product of 1D Lagrange polynomials through those points.  The 1D
Lagrange polynomials are evaluated with the textbook barycentric weights.
"""
from __future__ import annotations

import functools

import numpy as np
from numpy.polynomial import legendre as L


@functools.lru_cache(maxsize=None)
def nodes(N: int) -> np.ndarray:
    """LGL points on [-1, 1]: the endpoints and the roots of P'_{N-1}."""
    if N < 2:
        raise ValueError("need at least two LGL points")
    Pn = L.Legendre.basis(N - 1)
    inner = np.sort(np.real(Pn.deriv().roots())) if N > 2 else np.zeros(0)
    x = np.concatenate([[-1.0], inner, [1.0]])
    # one Newton polish on P'_{N-1} for the interior roots
    if N > 2:
        d1, d2 = Pn.deriv(1), Pn.deriv(2)
        x[1:-1] -= d1(x[1:-1]) / d2(x[1:-1])
    return x


@functools.lru_cache(maxsize=None)
def weights(N: int) -> np.ndarray:
    """LGL quadrature weights w_i = 2 / (N (N-1) P_{N-1}(x_i)^2)."""
    x = nodes(N)
    P = L.Legendre.basis(N - 1)(x)
    return 2.0 / (N * (N - 1) * P ** 2)


def barycentric_weights(x: np.ndarray) -> np.ndarray:
    """lambda_j = 1 / prod_{m != j} (x_j - x_m)."""
    n = len(x)
    lam = np.ones(n)
    for j in range(n):
        for m in range(n):
            if m != j:
                lam[j] /= (x[j] - x[m])
    return lam


@functools.lru_cache(maxsize=None)
def diff_matrix(N: int) -> np.ndarray:
    """D_ij = l_j'(x_i), the collocation derivative on the LGL points."""
    x = nodes(N)
    lam = barycentric_weights(x)
    D = np.zeros((N, N))
    for i in range(N):
        for j in range(N):
            if i != j:
                D[i, j] = (lam[j] / lam[i]) / (x[i] - x[j])
        D[i, i] = -D[i].sum()
    return D


def lagrange_matrix(x_nodes: np.ndarray, targets: np.ndarray) -> np.ndarray:
    """M[a, b] = l_b(targets[a]) by the product formula."""
    n = len(x_nodes)
    M = np.ones((len(targets), n))
    for a, t in enumerate(targets):
        for b in range(n):
            for m in range(n):
                if m != b:
                    M[a, b] *= (t - x_nodes[m]) / (x_nodes[b] - x_nodes[m])
    return M


@functools.lru_cache(maxsize=None)
def child_interpolation(N: int):
    """Prolongation from a parent element to its lower/upper half child in one
    dimension (Sec. III.C, eq. prol): the child's points sit at parent-logical
    coordinates (xi - 1)/2 (lower half) and (xi + 1)/2 (upper half)."""
    x = nodes(N)
    return lagrange_matrix(x, (x - 1.0) / 2.0), lagrange_matrix(x, (x + 1.0) / 2.0)
