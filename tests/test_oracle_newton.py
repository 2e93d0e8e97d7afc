"""Pins of the oracle's Newton-Raphson solver (Sec. III.A)."""
import numpy as np

import workloads as W
from oracle import mesh, newton, operator


def test_manufactured_polynomial_solution():
    # choose u* in Q_p, continuous and zero on the boundary, and set
    # b = A u* + M S(u*): the discrete nonlinear system is solved by u*
    L = np.array([1.0, 1.0, 1.0])
    m = mesh.BoxMesh([0, 0, 0], L, (2, 2, 2), 3)
    x, y, z = m.node_coordinates()
    ustar = 4 * x * (1 - x) * y * (1 - y) * z * (1 - z)
    alpha = 0.5 + 0.2 * x
    beta = 2.0 + y
    b = operator.apply_operator(m, ustar, 1.5, source=newton.puncture_source(alpha, beta, ustar))
    u, info = newton.newton_solve(m, 1.5, alpha, beta, b=b, newton_rtol=1e-12, linear_rtol=1e-10,
                                  levels=2)
    np.testing.assert_allclose(u, ustar.reshape(-1), atol=1e-11)
    h = np.array(info["history"])
    # quadratic convergence with tight linear solves: log residual roughly doubles
    assert info["steps"] <= 6
    k = np.argmax(h < 1e-3)
    assert h[k + 1] < 1e2 * h[k] ** 2


def test_linearisation_matches_finite_difference():
    alpha, beta, u = 0.7, 3.0, 0.2
    eps = 1e-6
    fd = (newton.puncture_source(alpha, beta, u + eps) - newton.puncture_source(alpha, beta, u - eps)) / (2 * eps)
    assert abs(fd - newton.puncture_source_derivative(alpha, beta, u)) < 1e-8


def test_backtrack_quadratic_step_is_minimiser():
    # for g(lambda) = f0 + slope lambda + c lambda^2 the first backtrack returns
    # the exact minimiser -slope / (2 c), clamped to [0.1, 0.5]
    f0, slope, c = 1.0, -2.0, 3.0
    g = lambda l: f0 + slope * l + c * l * l
    lam = newton.backtrack(f0, slope, 1.0, g(1.0), None, None, first=True)
    assert abs(lam - 1.0 / 3.0) < 1e-15


def test_backtrack_cubic_step_is_minimiser():
    # for a cubic g the cubic interpolation through g(0), g'(0), g(l1), g(l2)
    # is exact, so the step is the cubic's local minimiser
    f0, slope, a, bq = 1.0, -1.0, 4.0, 2.0
    g = lambda l: f0 + slope * l + bq * l * l + a * l ** 3
    l1, l2 = 1.0, 0.4
    lam = newton.backtrack(f0, slope, l2, g(l2), l1, g(l1), first=False)
    exact = (-bq + np.sqrt(bq * bq - 3 * a * slope)) / (3 * a)
    assert abs(lam - min(max(exact, 0.1 * l2), 0.5 * l2)) < 1e-14


def test_puncture_background_finite_and_positive():
    pp = W.puncture_params(W.SEED_C3)
    m = mesh.BoxMesh([-20, -20, -20], [20, 20, 20], (6, 6, 6), 7)
    x, y, z = m.node_coordinates()
    alpha, beta = W.puncture_background(pp, x, y, z)
    assert np.all(np.isfinite(alpha)) and np.all(np.isfinite(beta))
    assert np.all(alpha > 0) and np.all(beta >= 0)
    assert np.all(np.linalg.norm(pp.momenta, axis=1) <= 0.2)
