"""Pins of the oracle's DG operator (Sec. II, eqs. dg_op_auxvars,
dg_op_primal, numflux, penalty, bc).

The strongest pin is an independent brute-force assembly of the textbook
symmetric interior-penalty bilinear form with LGL quadrature,
  a(u, w) = sum_e int grad u . grad w
            - sum_F int ({d_n u}[w] + {d_n w}[u]) + sigma int [u][w]
with Dirichlet ghost faces contributing -int (d_n u w + d_n w u) + 2 sigma int u w.
Under LGL quadrature the strong form of the paper equals this weak form
(summation by parts), so any dropped term, wrong sign or index in the
oracle's strong-form code shows up as a mismatch.
"""
import numpy as np
import pytest

import workloads as W
from oracle import lgl, mesh, operator


def weak_sipg_matrix(m: mesh.BoxMesh, C):
    N = m.N
    n = m.ndof
    w = lgl.weights(N)
    D = lgl.diff_matrix(N)
    I = np.eye(N)
    J = np.prod(m.h) / 8.0
    Wv = np.kron(np.kron(w, w), w)  # [k, j, i] order, i fastest
    # per-element derivative operators in the canonical [k][j][i] order
    G = [np.kron(np.kron(I, I), D) * 2 / m.h[0],
         np.kron(np.kron(I, D), I) * 2 / m.h[1],
         np.kron(np.kron(D, I), I) * 2 / m.h[2]]
    K = np.zeros((n, n))
    n3 = N ** 3
    for e in range(m.E):
        sl = slice(e * n3, (e + 1) * n3)
        for d in range(3):
            K[sl, sl] += G[d].T @ np.diag(J * Wv) @ G[d]

    def face_ops(e, d, side):
        """trace T and outward normal derivative Dn of element e on face
        (d, side), as (N^2 x n) matrices, with face weights."""
        T = np.zeros((N * N, n))
        Dn = np.zeros((N * N, n))
        wf = np.zeros(N * N)
        trans = [t for t in range(3) if t != d]
        JF = np.prod([m.h[t] / 2 for t in trans])
        q = 0
        for b1 in range(N):
            for b0 in range(N):
                for mm in range(N):
                    node = [0, 0, 0]
                    node[d] = mm
                    node[trans[0]], node[trans[1]] = b0, b1
                    i, j, k = node
                    col = ((e * N + k) * N + j) * N + i
                    fidx = N - 1 if side > 0 else 0
                    if mm == fidx:
                        T[q, col] = 1.0
                    Dn[q, col] += side * (2 / m.h[d]) * D[fidx, mm]
                wf[q] = JF * w[b0] * w[b1]
                q += 1
        return T, Dn, wf

    for e in range(m.E):
        for d in range(3):
            sigma = C * N ** 2 / m.h[d]
            # interior face toward +d, and boundary faces
            for side in (-1, +1):
                nb = m.neighbor(e, d, side)
                Ta, Dna, wf = face_ops(e, d, side)
                Wf = np.diag(wf)
                if nb is None:
                    K += -(Dna.T @ Wf @ Ta + Ta.T @ Wf @ Dna) + 2 * sigma * Ta.T @ Wf @ Ta
                elif side > 0:
                    Tb, Dnb, _ = face_ops(nb, d, -1)
                    jump = Ta - Tb  # [u] = u_a - u_b, normal from a
                    avg = 0.5 * (Dna - Dnb)  # {d_n u} along a's normal
                    K += -(avg.T @ Wf @ jump + jump.T @ Wf @ avg) + sigma * jump.T @ Wf @ jump
    return K


CASES = [((1, 1, 1), 1, (1, 1, 1), 1.5), ((2, 1, 1), 2, (1, 1, 1), 1.0),
         ((2, 2, 1), 3, (1.0, 0.5, 2.0), 1.5), ((3, 2, 2), 2, (1, 1, 1), 1.5),
         ((1, 2, 3), 3, (0.7, 1.3, 1.9), 2.5), ((2, 2, 2), 4, (1, 1, 1), 1.5)]


@pytest.mark.parametrize("n,p,size,C", CASES)
def test_strong_form_equals_weak_sipg(n, p, size, C):
    m = mesh.BoxMesh([0.1, -0.2, 0.3], np.array([0.1, -0.2, 0.3]) + np.array(size), n, p)
    A = operator.assemble(m, C)
    K = weak_sipg_matrix(m, C)
    np.testing.assert_allclose(A, K, atol=1e-12 * np.abs(K).max())


@pytest.mark.parametrize("n,p,size,C", CASES)
def test_symmetric_positive_definite(n, p, size, C):
    m = mesh.BoxMesh([0, 0, 0], size, n, p)
    A = operator.assemble(m, C)
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    np.linalg.cholesky(A)  # raises if not SPD


@pytest.mark.parametrize("n,p", [((2, 2, 2), 2), ((3, 2, 1), 3), ((2, 3, 2), 4), ((1, 1, 2), 6),
                                 ((2, 1, 1), 9), ((1, 2, 1), 10), ((1, 1, 2), 11), ((2, 1, 1), 12)])
def test_polynomial_reproduction(n, p):
    # u = prod x_d (L_d - x_d) is continuous, in Q_p for p >= 2 and zero on the
    # boundary: every jump vanishes, so A u_I = M (-Laplace u)_I exactly
    L = np.array([1.0, 1.4, 0.8])
    m = mesh.BoxMesh([0, 0, 0], L, n, p)
    x, y, z = m.node_coordinates()
    fx, fy, fz = x * (L[0] - x), y * (L[1] - y), z * (L[2] - z)
    u = fx * fy * fz
    lap = -2 * (fy * fz + fx * fz + fx * fy)
    Au = operator.apply_operator(m, u, 1.5)
    b = operator.apply_mass(m, -lap)
    np.testing.assert_allclose(Au, b, atol=1e-13 * np.abs(b).max())


def test_h_scaling_cubes():
    # A scales like h for cubic elements: A(2h) = 2 A(h)
    A1 = operator.assemble(mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 2, 2), 3), 1.5)
    A2 = operator.assemble(mesh.BoxMesh([0, 0, 0], [2, 2, 2], (2, 2, 2), 3), 1.5)
    np.testing.assert_allclose(A2, 2 * A1, atol=1e-12 * np.abs(A1).max())


def test_mass_is_lgl_quadrature():
    m = mesh.BoxMesh([0, 0, 0], [1.0, 2.0, 0.5], (2, 1, 3), 4)
    M = operator.mass_diagonal(m)
    # total mass of one element = its volume
    assert abs(M.sum() - np.prod(m.h)) < 1e-14


def test_spectral_convergence_manufactured_solution():
    # Sec. IV.A: the solution error approaches the DG discretisation error,
    # which decays exponentially with p for the smooth sin-product solution
    errs = []
    for p in range(2, 8):
        m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 2, 2), p)
        x, y, z = m.node_coordinates()
        b = operator.apply_mass(m, W.sin_product_source(x, y, z)).reshape(-1)
        A = operator.assemble(m, 1.5)
        u = np.linalg.solve(A, b)
        ue = W.sin_product_solution(x, y, z).reshape(-1)
        errs.append(np.sqrt(np.mean((u - ue) ** 2)))
    errs = np.array(errs)
    assert np.all(errs[1:] < errs[:-1])
    rates = np.log(errs[:-1] / errs[1:])
    assert rates.mean() > 1.5  # better than a factor e^1.5 per degree
    assert errs[-1] < 1e-5


def test_neumann_faces_pure_neumann_kernel_and_mixed_spd():
    # eq. bc with homogeneous Neumann data on every face: constants are in the
    # kernel of A (no flux crosses the boundary and a constant has no jump);
    # with Dirichlet on at least one face A is symmetric positive definite
    all_n = mesh.BoxMesh([0, 0, 0], [1, 1.2, 0.8], (2, 2, 1), 3, neumann=range(6))
    one = np.ones((all_n.E, 4, 4, 4))
    assert np.abs(operator.apply_operator(all_n, one, 1.5)).max() < 1e-12
    m = mesh.BoxMesh([0, 0, 0], [1, 1.2, 0.8], (2, 2, 1), 3, neumann=(1, 2, 3, 4, 5))
    A = operator.assemble(m, 1.5)
    assert np.allclose(A, A.T, atol=1e-12)
    assert np.linalg.eigvalsh(A).min() > 0
    # the Dirichlet operator does not annihilate constants
    d = mesh.BoxMesh([0, 0, 0], [1, 1.2, 0.8], (2, 2, 1), 3)
    assert np.abs(operator.apply_operator(d, one, 1.5)).max() > 1e-3


def test_mixed_dirichlet_neumann_manufactured_solution_converges():
    # u = sin(pi x / 2) cos(pi y) cos(pi z) on [0,1]^3: zero at x = 0
    # (Dirichlet) and zero normal derivative on the five other faces; the
    # discrete solution converges exponentially in p
    errs = []
    for p in (2, 3, 4, 5):
        m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 2, 2), p, neumann=(1, 2, 3, 4, 5))
        x, y, z = m.node_coordinates()
        u = np.sin(np.pi * x / 2) * np.cos(np.pi * y) * np.cos(np.pi * z)
        f = (np.pi ** 2 / 4 + 2 * np.pi ** 2) * u
        A = operator.assemble(m, 1.5)
        uh = np.linalg.solve(A, operator.apply_mass(m, f).reshape(-1))
        errs.append(np.abs(uh - u.reshape(-1)).max())
    assert errs[-1] < 1e-3 and all(b < a / 3 for a, b in zip(errs, errs[1:])), errs


def test_high_order_operator_is_symmetric_positive_definite():
    # p = 10 (11^3 points per element) on two elements of unequal widths
    m = mesh.BoxMesh([0, 0, 0], [1.0, 0.6, 0.8], (2, 1, 1), 10)
    A = operator.assemble(m, 1.5)
    assert np.abs(A - A.T).max() <= 1e-12 * np.abs(A).max()
    np.linalg.cholesky(A)
