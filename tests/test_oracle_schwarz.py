"""Pins of the oracle's Schwarz smoother (Sec. III.D, III.E)."""
import os

import numpy as np
import pytest

from oracle import lgl, mesh, operator, schwarz


def test_subdomain_size_matches_paper(golden_dir):
    # Sec. III.E: 5 variables, 8^3 points, N_overlap = 2 -> 6400 x 6400, > 300 MB
    vals = {}
    with open(os.path.join(golden_dir, "subdomain_size.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = int(v)
    n = schwarz.subdomain_size(vals["points_per_dim"], vals["overlap"],
                               n_vars=vals["n_vars"])
    assert n == vals["matrix_size"]
    assert n * n * 8 / 1e6 > vals["min_dense_megabytes"]


def test_subdomain_layout_size_and_uniqueness():
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (3, 3, 3), 4)
    for e in range(m.E):
        idx, coords, normal = schwarz.subdomain_layout(m, e, 2)
        nfaces = sum(m.neighbor(e, d, s) is not None for d, s in schwarz.FACE_ORDER)
        assert len(idx) == m.N ** 3 + nfaces * 2 * m.N ** 2
        assert len(np.unique(idx)) == len(idx)
        # no point beyond the neighbour's far face, and none at |xi_S| = 3
        assert np.all(np.abs(coords) < 3.0 - 1e-12)


@pytest.mark.parametrize("delta", [0.3, 0.7, 1.0, 1.5, 2.0])
def test_weight_function_values(delta):
    # eq. schwarz_weight_function: w(+-1) = 1/2, w(+-3) = 0, w(0) = 1 for delta <= 1
    w = schwarz.weight_1d(np.array([-3.0, -1.0, 0.0, 1.0, 3.0]), delta)
    np.testing.assert_allclose(w[[1, 3]], 0.5, atol=1e-15)
    np.testing.assert_allclose(w[[0, 4]], 0.0, atol=1e-15)
    if delta <= 1.0:
        assert abs(w[2] - 1.0) < 1e-15
    # smoothstep: phi(1) = 1, phi'(+-1) = 0 (second-order smoothstep)
    assert abs(schwarz.smoothstep(1.0) - 1.0) < 1e-15
    eps = 1e-6
    assert abs(schwarz.smoothstep(1.0) - schwarz.smoothstep(1.0 - eps)) < 1e-10


@pytest.mark.parametrize("N,ov,expected", [(4, 2, 1 + np.sqrt(1 / 5)), (5, 2, 1.0), (4, 3, 2.0),
                                           (6, 1, 1 - np.sqrt(1 / 3 + 2 * np.sqrt(7) / 21))])
def test_overlap_width(N, ov, expected):
    assert abs(schwarz.overlap_width(N, ov) - expected) < 1e-14


@pytest.mark.parametrize("n,p,ov", [((3, 3, 3), 2, 2), ((4, 2, 3), 3, 2), ((2, 3, 1), 3, 1),
                                    ((3, 2, 2), 4, 3), ((1, 1, 1), 3, 2), ((3, 1, 2), 5, 2)])
def test_weights_partition_of_unity(n, p, ov):
    # sum_S R_S^T w_S = 1 at every point
    m = mesh.BoxMesh([0, 0, 0], [1, 1.2, 0.9], n, p)
    tot = np.zeros(m.ndof)
    for e in range(m.E):
        idx = schwarz.subdomain_layout(m, e, ov)[0]
        np.add.at(tot, idx, schwarz.subdomain_weights(m, e, ov))
    np.testing.assert_allclose(tot, 1.0, atol=1e-14)


@pytest.mark.parametrize("n,p,ov,size", [((3, 3, 3), 2, 2, (1, 1, 1)), ((4, 3, 2), 2, 1, (1, 2, 0.5)),
                                         ((3, 2, 2), 3, 2, (1, 1, 1))])
def test_subdomain_operator_is_submatrix_and_depends_on_class_only(n, p, ov, size):
    # A_S = R_S A R_S^T (Sec. III.D.2) for every element equals the class
    # operator computed on a small patch
    m = mesh.BoxMesh([0, 0, 0], size, n, p)
    A = operator.assemble(m, 1.5)
    cache = {}
    for e in range(m.E):
        idx = schwarz.subdomain_layout(m, e, ov)[0]
        literal = A[np.ix_(idx, idx)]
        key = schwarz.element_class(m, e)
        if key not in cache:
            cache[key] = schwarz.subdomain_operator(m, key, 1.5, ov)
        np.testing.assert_allclose(cache[key], literal, atol=1e-13 * np.abs(literal).max())
        np.testing.assert_allclose(literal, schwarz.subdomain_operator_literal(m, e, 1.5, ov),
                                   atol=1e-13 * np.abs(literal).max())


def test_single_element_step_is_exact():
    # one subdomain covering the whole domain: one Schwarz step solves A u = b
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (1, 1, 1), 4)
    rng = np.random.default_rng(0)
    b = rng.standard_normal(m.ndof)
    S = schwarz.SchwarzSmoother(m, 1.5, 2)
    u = S.smooth(np.zeros(m.ndof), b, 1)
    np.testing.assert_allclose(u, np.linalg.solve(operator.assemble(m, 1.5), b), rtol=1e-12, atol=1e-12)


def test_step_matches_dense_formula():
    # u + sum_S R_S^T W_S A_S^-1 R_S (b - A u), with dense restriction matrices
    # built from the point sets and the submatrices of the assembled A
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (3, 2, 2), 2)
    A = operator.assemble(m, 1.5)
    rng = np.random.default_rng(1)
    u0, b = rng.standard_normal(m.ndof), rng.standard_normal(m.ndof)
    B = np.zeros((m.ndof, m.ndof))
    for e in range(m.E):
        idx = schwarz.subdomain_layout(m, e, 2)[0]
        R = np.zeros((len(idx), m.ndof))
        R[np.arange(len(idx)), idx] = 1.0
        AS = R @ A @ R.T
        B += R.T @ np.diag(schwarz.subdomain_weights(m, e, 2)) @ np.linalg.inv(AS) @ R
    expected = u0 + B @ (b - A @ u0)
    S = schwarz.SchwarzSmoother(m, 1.5, 2)
    np.testing.assert_allclose(S.smooth(u0, b, 1), expected, rtol=1e-11, atol=1e-11)


def test_fixed_point_and_smoothing():
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 2, 2), 3)
    A = operator.assemble(m, 1.5)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(m.ndof)
    S = schwarz.SchwarzSmoother(m, 1.5, 2)
    np.testing.assert_allclose(S.smooth(x, A @ x, 2), x, rtol=1e-11, atol=1e-11)
    # the smoother reduces the error of a random initial guess
    e0 = rng.uniform(-0.5, 0.5, m.ndof)
    e3 = S.smooth(e0, np.zeros(m.ndof), 3)
    assert np.linalg.norm(e3) < 0.5 * np.linalg.norm(e0)


def test_gmres_fixed_with_exact_preconditioner():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((20, 20)) + 20 * np.eye(20)
    r = rng.standard_normal(20)
    x = schwarz.gmres_fixed(lambda v: A @ v, lambda v: np.linalg.solve(A, v), r, 3)
    np.testing.assert_allclose(A @ x, r, rtol=1e-12, atol=1e-12)
    # with an inexact preconditioner three iterations reduce the residual
    D = np.diag(np.diag(A))
    x = schwarz.gmres_fixed(lambda v: A @ v, lambda v: np.linalg.solve(D, v), r, 3)
    assert np.linalg.norm(A @ x - r) < np.linalg.norm(r)
