"""Pins of the oracle's DG operator on curved (isoparametric) elements
(Sec. II, eqs. massmat, stiffmat, liftop with the element Jacobian), each
against something other than the code it checks: the affine box operator
(pinned by its own tests), exact derivatives of polynomial maps, the exact
reproduction of linear functions, and convergence to a manufactured
solution."""
import numpy as np
import pytest

import workloads as W
from oracle import curved, mesh as omesh, operator as oop

C = 1.5


@pytest.mark.parametrize("elements,p,neumann", [((3, 2, 2), 3, ()), ((2, 2, 3), 4, (1, 4)),
                                                ((1, 3, 2), 2, (0,))])
def test_affine_coordinates_give_the_box_operator(elements, p, neumann):
    box = omesh.BoxMesh((0, 0, 0), (1.0, 1.2, 0.9), elements, p, neumann=neumann)
    cm = curved.CurvedMesh(box, np.stack(box.node_coordinates()))
    u = W.random_normal(41, box.ndof)
    ref = oop.apply_operator(box, u.reshape(box.E, box.N, box.N, box.N), C).reshape(-1)
    got = curved.apply_operator(cm, u, C)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.allclose(curved.mass_diagonal(cm),
                       np.broadcast_to(oop.mass_diagonal(box), cm.det.shape), rtol=1e-14, atol=0)


def test_geometry_of_a_polynomial_map_is_exact():
    # a quadratic map is its own degree-p interpolant (p >= 2), so the
    # collocation Jacobian equals the analytic one
    box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (2, 1, 2), 3)
    X = np.stack(box.node_coordinates())
    e = 0.1
    x = np.stack([X[0] + e * X[0] * X[1], X[1] + e * X[1] ** 2, X[2] + e * X[0] * X[2]])
    cm = curved.CurvedMesh(box, x)
    # dx/dX analytic; dX/dxi = h/2 per axis
    dxdX = np.zeros(X.shape[1:] + (3, 3))
    dxdX[..., 0, 0] = 1 + e * X[1]
    dxdX[..., 0, 1] = e * X[0]
    dxdX[..., 1, 1] = 1 + 2 * e * X[1]
    dxdX[..., 2, 0] = e * X[2]
    dxdX[..., 2, 2] = 1 + e * X[0]
    J = dxdX * (box.h / 2.0)[None, None, None, None, None, :]
    assert np.allclose(cm.jac, J, rtol=0, atol=1e-13)
    assert np.allclose(cm.det, np.linalg.det(J), rtol=1e-13, atol=0)
    assert np.allclose(np.einsum("...ij,...jk->...ik", cm.inv, J), np.eye(3), atol=1e-13)


def test_linear_functions_are_reproduced_exactly_inside():
    # u = a.x + c is a degree-p polynomial in xi on every element and
    # continuous across faces: its lifted gradient is the constant a, so
    # -M D_i v_i vanishes and every interior face flux cancels
    box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (4, 4, 4), 3)
    cm = curved.CurvedMesh(box, curved.deformed_box(box, 0.1))
    x = cm.xyz
    u = 0.3 * x[0] - 0.7 * x[1] + 0.2 * x[2] + 1.0
    Au = curved.apply_operator(cm, u, C).reshape(box.E, -1)
    inner = [e for e in range(box.E) if not any(f for pair in box.external_flags(e) for f in pair)]
    assert len(inner) == 8
    assert np.abs(Au[inner]).max() <= 1e-13 * np.abs(Au).max()


def test_converges_to_a_manufactured_solution_on_a_curved_grid():
    # -Delta u = 3 pi^2 u with u = prod sin(pi x_d) on the deformed unit cube
    # (the map keeps the boundary, where u = 0)
    errs = []
    for p in (2, 3, 4, 5):
        box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (2, 2, 2), p)
        cm = curved.CurvedMesh(box, curved.deformed_box(box, 0.1))
        X = cm.xyz
        uex = (np.sin(np.pi * X[0]) * np.sin(np.pi * X[1]) * np.sin(np.pi * X[2])).reshape(-1)
        b = curved.apply_mass(cm, 3 * np.pi ** 2 * uex).reshape(-1)
        us = np.linalg.solve(curved.assemble(cm, C), b)
        errs.append(np.abs(us - uex).max())
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 2e-4 and errs[0] / errs[-1] > 200, errs


def test_operator_on_curved_elements():
    # the strong form with a varying metric is not symmetric (D_i applies the
    # metric after the derivative), but its asymmetry vanishes with the
    # deformation and its symmetric part stays positive definite
    box = omesh.BoxMesh((0, 0, 0), (1, 1.2, 0.9), (3, 2, 2), 2)
    asym = []
    for amp in (0.0, 0.05, 0.1):
        A = curved.assemble(curved.CurvedMesh(box, curved.deformed_box(box, amp)), C)
        asym.append(np.abs(A - A.T).max() / np.abs(A).max())
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
    assert asym[0] < 1e-14 and 0 < asym[1] < asym[2] < 0.05, asym


def test_wedge_of_a_spherical_shell():
    # one wedge of the shell of Sec. IV.B (equiangular, logarithmic radius):
    # the map is orientation preserving, its inner and outer faces lie on the
    # spheres, and the discrete solution with the harmonic 1/r as Dirichlet
    # data converges to 1/r exponentially in p
    errs = []
    for p in (2, 4, 6):
        box = omesh.BoxMesh((-1, -1, -1), (1, 1, 1), (2, 2, 2), p)
        xyz = W.wedge_coordinates(np.stack(box.node_coordinates()), 2.0, 10.0)
        cm = curved.CurvedMesh(box, xyz)
        r = np.sqrt(np.sum(cm.xyz ** 2, axis=0))
        zeta = np.stack(box.node_coordinates())[2]
        assert np.allclose(r[np.isclose(zeta, -1.0)], 2.0, rtol=1e-14)
        assert np.allclose(r[np.isclose(zeta, 1.0)], 10.0, rtol=1e-14)
        uex = (1.0 / r).reshape(-1)
        A = curved.assemble(cm, C)
        rhs = -curved.apply_operator(cm, np.zeros(box.ndof), C, dirichlet_values=uex)
        us = np.linalg.solve(A, rhs)
        errs.append(np.abs(us - uex).max() / np.abs(uex).max())
    assert errs[0] > 10 * errs[1] > 100 * errs[2], errs
    assert errs[-1] < 1e-5, errs


def _unit_metric(shape):
    G = np.zeros((3, 3) + shape)
    for i in range(3):
        G[i, i] = 1.0
    return G, np.ones(shape)


def test_background_metric_flat_and_constant():
    # with g = delta the metric operator is the flat one; a constant metric
    # g = A^T A on the box is the flat operator on the box mapped by x = A X
    box = omesh.BoxMesh((0, 0, 0), (1, 1.2, 0.9), (3, 2, 2), 3, neumann=(1,))
    cm = curved.CurvedMesh(box, curved.deformed_box(box, 0.1))
    u = W.random_normal(42, box.ndof)
    G, sg = _unit_metric(cm.det.shape)
    ref = curved.apply_operator(cm, u, C)
    assert np.abs(curved.apply_operator_metric(cm, u, C, G, sg) - ref).max() <= 1e-14 * np.abs(ref).max()
    A = np.array([[1.0, 0.3, 0.1], [0.0, 0.9, 0.2], [0.1, 0.0, 1.1]])
    X = np.stack(box.node_coordinates())
    ref = curved.apply_operator(curved.CurvedMesh(box, np.einsum("ij,j...->i...", A, X)), u, C)
    gi = np.linalg.inv(A.T @ A)
    G = np.broadcast_to(gi[:, :, None, None, None, None], (3, 3) + cm.det.shape)
    got = curved.apply_operator_metric(curved.CurvedMesh(box, X), u, C, G,
                                       np.full(cm.det.shape, np.linalg.det(A)))
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_background_metric_converges_to_a_harmonic_function():
    # the pullback of the flat metric under a curved map: u = 1/|phi(X) - x0|
    # solves the Laplace-Beltrami equation; with it as Dirichlet data the
    # discrete solution converges exponentially in p, and dropping the
    # Christoffel source (a constant sqrt(g)) leaves an O(1e-2) error
    x0 = np.array([-0.5, -0.5, -0.5])

    def solve(p, drop_source=False):
        box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (2, 2, 2), p)
        X = np.stack(box.node_coordinates())
        phi, ginv, sqrtg = W.pullback_metric(X, box.lower, box.upper, 0.15)
        if drop_source:
            sqrtg = np.ones_like(sqrtg)
        cm = curved.CurvedMesh(box, X)
        uex = (1.0 / np.sqrt(np.sum((phi - x0[:, None, None, None, None]) ** 2, axis=0))).reshape(-1)
        n = box.ndof
        A = np.stack([curved.apply_operator_metric(cm, e, C, ginv, sqrtg) for e in np.eye(n)], axis=1)
        rhs = -curved.apply_operator_metric(cm, np.zeros(n), C, ginv, sqrtg, dirichlet_values=uex)
        return np.abs(np.linalg.solve(A, rhs) - uex).max() / np.abs(uex).max()

    errs = [solve(p) for p in (2, 3, 4)]
    assert errs[0] > 5 * errs[1] > 25 * errs[2] and errs[2] < 5e-5, errs
    assert solve(4, drop_source=True) > 100 * errs[2]
