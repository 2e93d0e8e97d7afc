"""Pins of the oracle's multigrid transfer and V-cycle (Sec. III.C)."""
import numpy as np
import pytest

import workloads as W
from oracle import krylov, mesh, multigrid, operator, schwarz


def test_coarsening_rules():
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (8, 6, 3), 2)
    levels = multigrid.hierarchy(m, 10)
    assert [lv[0].n for lv in levels] == [(8, 6, 3), (4, 3, 3), (2, 3, 3), (1, 3, 3)]
    assert levels[-1][1] is None
    assert [lv[0].n for lv in multigrid.hierarchy(m, 2)] == [(8, 6, 3), (4, 3, 3)]


@pytest.mark.parametrize("n,p", [((2, 2, 2), 3), ((4, 2, 1), 2), ((2, 3, 2), 4)])
def test_prolongation_reproduces_polynomials(n, p):
    # eq. prol is Lagrange interpolation: a Q_p polynomial on the coarse grid
    # is reproduced exactly at the fine points
    fine = mesh.BoxMesh([0, 0, 0], [1, 2, 1], n, p)
    coarse, split = multigrid.coarsen(fine)
    poly = lambda x, y, z: (1 + x ** p - 2 * y ** (p - 1) * z + x * y * z ** p)
    uc = poly(*coarse.node_coordinates()).reshape(-1)
    uf = multigrid.prolongate(fine, coarse, split, uc)
    np.testing.assert_allclose(uf, poly(*fine.node_coordinates()).reshape(-1), atol=1e-12)


def test_restriction_is_transpose():
    fine = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (4, 2, 2), 3)
    coarse, split = multigrid.coarsen(fine)
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal(coarse.ndof), rng.standard_normal(fine.ndof)
    lhs = np.dot(multigrid.prolongate(fine, coarse, split, x), y)
    rhs = np.dot(x, multigrid.restrict(fine, coarse, split, y))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _dense(f, n):
    return np.stack([f(np.eye(n)[j]) for j in range(n)], axis=1)


def test_vcycle_matches_dense_composition():
    # Two-grid V-cycle written with dense matrices: with the smoothing step
    # u <- u + B (b - A u) on each level,
    #   presmooth 3 from 0, r = b - A u, uc = coarse cycle(R r), u += P uc,
    #   postsmooth 3; on the coarsest grid 3 + 3 steps from 0.
    fine = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 2, 2), 2)
    coarse, split = multigrid.coarsen(fine)
    Af, Ac = operator.assemble(fine, 1.5), operator.assemble(coarse, 1.5)
    Sf, Sc = schwarz.SchwarzSmoother(fine, 1.5, 2), schwarz.SchwarzSmoother(coarse, 1.5, 2)
    Bf = _dense(Sf.correction, fine.ndof)
    Bc = _dense(Sc.correction, coarse.ndof)
    P = _dense(lambda v: multigrid.prolongate(fine, coarse, split, v), coarse.ndof)
    R = P.T

    def smooth(A, B, u, b, k):
        for _ in range(k):
            u = u + B @ (b - A @ u)
        return u

    rng = np.random.default_rng(1)
    b = rng.standard_normal(fine.ndof)
    u = smooth(Af, Bf, np.zeros(fine.ndof), b, 3)
    bc = R @ (b - Af @ u)
    uc = smooth(Ac, Bc, smooth(Ac, Bc, np.zeros(coarse.ndof), bc, 3), bc, 3)
    u = smooth(Af, Bf, u + P @ uc, b, 3)
    V = multigrid.VCycle(fine, 1.5, levels=2)
    np.testing.assert_allclose(V(b), u, rtol=1e-11, atol=1e-11)


def test_vcycle_is_linear():
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (4, 2, 2), 2)
    V = multigrid.VCycle(m, 1.5, levels=3)
    rng = np.random.default_rng(2)
    r1, r2 = rng.standard_normal(m.ndof), rng.standard_normal(m.ndof)
    np.testing.assert_allclose(V(2.5 * r1 + r2), 2.5 * V(r1) + V(r2), rtol=1e-11, atol=1e-11)


def test_mg_schwarz_iterations_flat_under_h_refinement():
    # Sec. IV.A: the multigrid-Schwarz preconditioner keeps the FGMRES
    # iteration count independent of the number of elements
    its = []
    for n, levels in [(4, 3), (8, 4)]:
        m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (n, n, n), 3)
        x, y, z = m.node_coordinates()
        b = operator.apply_mass(m, W.sin_product_source(x, y, z)).reshape(-1)
        A = lambda v, m=m: operator.apply_operator(m, v.reshape(m.E, 4, 4, 4), 1.5).reshape(-1)
        _, k, hist = krylov.fgmres(A, b, precondition=multigrid.VCycle(m, 1.5, levels=levels),
                                   rtol=1e-10)
        its.append(k)
        assert hist[-1] <= 1e-10
    assert abs(its[1] - its[0]) <= 2  # 8 and 9 iterations


def test_wcycle_matches_dense_composition():
    # Three-level W-cycle (gamma = 2) written with dense matrices: every
    # coarser level is visited twice per visit of its parent, the second
    # visit starting from the first one's result; smoothing u <- u + B (b - A u)
    fine = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (8, 4, 4), 1)
    V = multigrid.VCycle(fine, 1.5, levels=3, gamma=2)
    lv = [m for m, _ in V.levels]
    A = [operator.assemble(m, 1.5) for m in lv]
    B = [_dense(schwarz.SchwarzSmoother(m, 1.5, 2).correction, m.ndof) for m in lv]
    P = [_dense(lambda v, l=l: multigrid.prolongate(lv[l], lv[l + 1], V.levels[l][1], v),
                lv[l + 1].ndof) for l in range(2)]

    def smooth(l, u, b, k):
        for _ in range(k):
            u = u + B[l] @ (b - A[l] @ u)
        return u

    def cycle(l, b, u):
        u = smooth(l, u, b, 3)
        if l == 2:
            return smooth(l, u, b, 3)
        bc = P[l].T @ (b - A[l] @ u)
        uc = np.zeros(lv[l + 1].ndof)
        for _ in range(2):
            uc = cycle(l + 1, bc, uc)
        return smooth(l, u + P[l] @ uc, b, 3)

    b = np.random.default_rng(3).standard_normal(fine.ndof)
    np.testing.assert_allclose(V(b), cycle(0, b, np.zeros(fine.ndof)), rtol=1e-11, atol=1e-11)
    # gamma = 1 is the V-cycle; the W-cycle is a different, also linear map
    v1 = multigrid.VCycle(fine, 1.5, levels=3)(b)
    assert np.linalg.norm(V(b) - v1) > 1e-6 * np.linalg.norm(v1)
    np.testing.assert_allclose(V(3.0 * b), 3.0 * V(b), rtol=1e-11, atol=1e-11)


def test_additive_mg_matches_dense_sum_over_levels():
    # z = sum_l P_{0<-l} S_l R_{l<-0} r, with S_l the six-step smoothing
    # operator from zero of level l and P_{0<-l} = P_0 ... P_{l-1}, R = P^T
    fine = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (8, 4, 4), 1)
    Add = multigrid.AdditiveMG(fine, 1.5, levels=3)
    V = multigrid.VCycle(fine, 1.5, levels=3)
    lv = [m for m, _ in V.levels]
    A = [operator.assemble(m, 1.5) for m in lv]
    B = [_dense(schwarz.SchwarzSmoother(m, 1.5, 2).correction, m.ndof) for m in lv]
    P = [_dense(lambda v, l=l: multigrid.prolongate(lv[l], lv[l + 1], V.levels[l][1], v),
                lv[l + 1].ndof) for l in range(2)]
    S = []
    for l in range(3):  # six steps u <- u + B (b - A u) from zero, as a matrix of b
        E = np.eye(lv[l].ndof) - B[l] @ A[l]
        S.append(sum(np.linalg.matrix_power(E, i) for i in range(6)) @ B[l])
    to0 = [np.eye(fine.ndof), P[0], P[0] @ P[1]]
    r = np.random.default_rng(5).standard_normal(fine.ndof)
    want = sum(to0[l] @ S[l] @ to0[l].T @ r for l in range(3))
    np.testing.assert_allclose(Add(r), want, rtol=1e-10, atol=1e-11)
    # it preconditions FGMRES, with more iterations than the multiplicative cycle
    Af = lambda v: A[0] @ v
    _, k_add, _ = krylov.fgmres(Af, r, precondition=Add, rtol=1e-10)
    _, k_mul, _ = krylov.fgmres(Af, r, precondition=V, rtol=1e-10)
    assert k_add > k_mul


def test_fcycle_matches_dense_composition():
    # F-cycle: an F-visit of the coarser level, then a V-visit from its result
    fine = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (8, 8, 4), 1)
    F = multigrid.VCycle(fine, 1.5, levels=4, gamma="F")
    lv = [m for m, _ in F.levels]
    A = [operator.assemble(m, 1.5) for m in lv]
    B = [_dense(schwarz.SchwarzSmoother(m, 1.5, 2).correction, m.ndof) for m in lv]
    P = [_dense(lambda v, l=l: multigrid.prolongate(lv[l], lv[l + 1], F.levels[l][1], v),
                lv[l + 1].ndof) for l in range(3)]

    def smooth(l, u, b, k):
        for _ in range(k):
            u = u + B[l] @ (b - A[l] @ u)
        return u

    def cycle(l, b, u, kind):
        u = smooth(l, u, b, 3)
        if l == 3:
            return smooth(l, u, b, 3)
        bc = P[l].T @ (b - A[l] @ u)
        uc = np.zeros(lv[l + 1].ndof)
        for k in (("F", "V") if kind == "F" else ("V",)):
            uc = cycle(l + 1, bc, uc, k)
        return smooth(l, u + P[l] @ uc, b, 3)

    b = np.random.default_rng(7).standard_normal(fine.ndof)
    np.testing.assert_allclose(F(b), cycle(0, b, np.zeros(fine.ndof), "F"), rtol=1e-11, atol=1e-11)
    for other in (1, 2):
        o = multigrid.VCycle(fine, 1.5, levels=4, gamma=other)(b)
        assert np.linalg.norm(F(b) - o) > 1e-6 * np.linalg.norm(o)
