"""Pins of the oracle's LGL tables against closed forms and exactness
properties (Sec. II, eqs. field_expansion, lagrprod)."""
import math
import os

import numpy as np
import pytest

from oracle import lgl


def _closed_forms(golden_dir):
    out = {}
    with open(os.path.join(golden_dir, "lgl_closed_forms.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, rest = line.split(":")
            xs, ws = rest.split("|")
            env = {"sqrt": math.sqrt}
            out[int(n)] = (np.array([eval(t, env) for t in xs.split()]),
                           np.array([eval(t, env) for t in ws.split()]))
    return out


def test_closed_form_nodes_and_weights(golden_dir):
    for N, (x, w) in _closed_forms(golden_dir).items():
        np.testing.assert_allclose(lgl.nodes(N), x, atol=1e-15)
        np.testing.assert_allclose(lgl.weights(N), w, atol=1e-15)


@pytest.mark.parametrize("N", range(2, 14))
def test_weights_sum_and_endpoint(N):
    w = lgl.weights(N)
    p = N - 1
    assert abs(w.sum() - 2.0) < 1e-14
    assert abs(w[0] - 2.0 / (p * (p + 1))) < 1e-15
    assert abs(w[-1] - 2.0 / (p * (p + 1))) < 1e-15


@pytest.mark.parametrize("N", range(2, 14))
def test_quadrature_exact_to_degree_2N_minus_3(N):
    # an N-point rule that contains both endpoints and integrates all
    # polynomials of degree <= 2N-3 exactly is the LGL rule (unique)
    x, w = lgl.nodes(N), lgl.weights(N)
    for k in range(2 * N - 2):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13
    # and not degree 2N-2
    k = 2 * N - 2
    assert abs(np.dot(w, x ** k) - 2.0 / (k + 1)) > 1e-10


@pytest.mark.parametrize("N", range(2, 14))
def test_diff_matrix_exact_on_polynomials(N):
    x = lgl.nodes(N)
    D = lgl.diff_matrix(N)
    for k in range(N):
        d = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        np.testing.assert_allclose(D @ x ** k, d, atol=1e-12 * max(1, k))


@pytest.mark.parametrize("N", range(2, 14))
def test_summation_by_parts(N):
    # W D + D^T W = diag(-1, 0, ..., 0, 1) because LGL quadrature is exact
    # for the degree-(2N-3) products l_i l_j'
    D, W = lgl.diff_matrix(N), np.diag(lgl.weights(N))
    B = np.zeros((N, N))
    B[0, 0], B[-1, -1] = -1.0, 1.0
    np.testing.assert_allclose(W @ D + D.T @ W, B, atol=1e-12)


@pytest.mark.parametrize("N", range(2, 14))
def test_child_interpolation_reproduces_polynomials(N):
    x = lgl.nodes(N)
    P_lo, P_hi = lgl.child_interpolation(N)
    for k in range(N):
        np.testing.assert_allclose(P_lo @ x ** k, ((x - 1) / 2) ** k, atol=1e-13)
        np.testing.assert_allclose(P_hi @ x ** k, ((x + 1) / 2) ** k, atol=1e-13)
