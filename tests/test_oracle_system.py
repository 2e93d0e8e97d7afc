"""Pins of the oracle's multi-variable system and its Laplacian-approximation
subdomain solver (Sec. III.E.1, eq. lapl_approx), each against something
other than the code it checks: dense matrices assembled by applying the
scalar operator to unit vectors, literal restrictions R_S A R_S^T of the
global system matrix, and exact solves."""
import numpy as np
import pytest

import workloads as W
from oracle import krylov, mesh as omesh, multigrid, operator as oop, schwarz, system

C = 1.5


def _coupling(m, nvars, seed=5, strength=10.0):
    x, y, z = m.node_coordinates()
    c = W.system_coupling(seed, nvars, x, y, z, strength)
    mass = np.broadcast_to(oop.mass_diagonal(m), (m.E, m.N, m.N, m.N)).reshape(-1)
    return c * mass[None, None, :]


def _dense_system(sysop, D):
    n = sysop.V * sysop.ndof
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = sysop.apply(e, D).reshape(-1)
    return A


def _dense_prolongation(fine, coarse, split):
    P = np.empty((fine.ndof, coarse.ndof))
    for j in range(coarse.ndof):
        e = np.zeros(coarse.ndof)
        e[j] = 1.0
        P[:, j] = multigrid.prolongate(fine, coarse, split, e)
    return P


def test_without_coupling_the_system_step_is_the_scalar_steps():
    neu = ((0, 2), (), (5,))
    sysop = system.SystemOperator((0, 0, 0), (1, 1.2, 0.8), (3, 2, 2), 2, neu, C)
    m = sysop.mesh
    D = np.zeros((3, 3, m.ndof))
    b = W.random_normal(1, 3 * m.ndof).reshape(3, -1)
    u0 = W.random_uniform(2, 3 * m.ndof).reshape(3, -1)
    got = system.SystemSchwarzSmoother(sysop.meshes, C, D, subdomain_iters=0).smooth(u0, b, 2)
    for a in range(3):
        ref = schwarz.SchwarzSmoother(sysop.meshes[a], C, 2).smooth(u0[a], b[a], 2)
        assert np.allclose(got[a], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_one_element_step_with_full_gmres_is_the_exact_system_solve():
    # one element: its subdomain is the whole domain with weight 1, so enough
    # GMRES iterations make one step the exact solve of A_sys u = b
    neu = ((0, 2, 4), ())
    sysop = system.SystemOperator((0, 0, 0), (1, 1, 1), (1, 1, 1), 2, neu, C)
    m = sysop.mesh
    D = _coupling(m, 2)
    D[0, 1] *= 1.7  # not symmetric, so a transposed coupling would show
    A = _dense_system(sysop, D)
    b = W.random_normal(3, 2 * m.ndof)
    u0 = W.random_uniform(4, 2 * m.ndof)
    sm = system.SystemSchwarzSmoother(sysop.meshes, C, D, subdomain_iters=2 * m.ndof)
    got = sm.smooth(u0, b, 1).reshape(-1)
    exact = np.linalg.solve(A, b)
    assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < 1e-9


@pytest.mark.parametrize("laplacian_bc", ["matched", "dirichlet"])
def test_step_with_full_gmres_equals_the_dense_formula(laplacian_bc):
    # A_S,sys = R_S A_sys R_S^T taken literally from the global system matrix
    # (coupling and each variable's boundary conditions included); with
    # enough iterations the preconditioner no longer matters
    neu = ((0,), ())
    sysop = system.SystemOperator((0, 0, 0), (1.4, 1, 1), (2, 1, 1), 2, neu, C)
    m = sysop.mesh
    V, n = 2, m.ndof
    D = _coupling(m, V, seed=6)
    D[1, 0] *= 0.4  # not symmetric, so a transposed coupling would show
    A = _dense_system(sysop, D)
    b = W.random_normal(5, V * n)
    u0 = W.random_uniform(6, V * n)
    r = b - A @ u0
    expect = u0.copy()
    for e in range(m.E):
        idx = schwarz.subdomain_layout(m, e, 2)[0]
        w = schwarz.subdomain_weights(m, e, 2)
        rows = np.concatenate([a * n + idx for a in range(V)])
        dS = np.linalg.solve(A[np.ix_(rows, rows)], r[rows])
        expect[rows] += np.tile(w, V) * dS
    k = V * len(schwarz.subdomain_layout(m, 0, 2)[0])
    sm = system.SystemSchwarzSmoother(sysop.meshes, C, D, subdomain_iters=k, laplacian_bc=laplacian_bc)
    got = sm.smooth(u0, b, 1).reshape(-1)
    assert np.linalg.norm(got - expect) / np.linalg.norm(expect) < 1e-9


def test_matched_boundary_conditions_make_the_poisson_subdomain_solve_exact():
    # without coupling the matched Laplacian approximation is the subdomain
    # operator itself, so one GMRES iteration solves every subdomain problem;
    # the Dirichlet approximation does so only for subdomains away from the
    # Neumann face (GMRES takes one coefficient for the stacked vector, so a
    # mismatched variable spoils the other variable's part too)
    neu = ((0,), ())
    sysop = system.SystemOperator((0, 0, 0), (1, 1, 1), (3, 2, 1), 2, neu, C)
    m = sysop.mesh
    D = np.zeros((2, 2, m.ndof))
    matched = system.SystemSchwarzSmoother(sysop.meshes, C, D, subdomain_iters=1)
    naive = system.SystemSchwarzSmoother(sysop.meshes, C, D, subdomain_iters=1,
                                         laplacian_bc="dirichlet")
    r = W.random_normal(7, 2 * m.ndof).reshape(2, -1)
    touching = 0
    for e in range(m.E):
        idx = schwarz.subdomain_layout(m, e, 2)[0]
        rS = r[:, idx].reshape(-1)
        exact = np.concatenate([np.linalg.solve(
            schwarz.subdomain_operator_literal(sysop.meshes[a], e, C, 2), r[a, idx]) for a in range(2)])
        got = matched.subdomain_solve(e, rS)
        assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < 1e-10
        rel = np.linalg.norm(naive.subdomain_solve(e, rS) - exact) / np.linalg.norm(exact)
        if m.elem_coords(e)[0] == 0:  # the subdomain touches the Neumann face x-
            touching += 1
            assert rel > 1e-3
        else:
            assert rel < 1e-10
    assert touching == 2


def _poisson_dense(mesh):
    n = mesh.ndof
    N = mesh.N
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = oop.apply_operator(mesh, e.reshape(mesh.E, N, N, N), C).reshape(-1)
    return A


def test_two_level_system_cycle_equals_the_dense_composition():
    # k = 0: the smoother is linear, C_l r = sum_S R_S^T w_S M_S R_S r with
    # M_S = blockdiag_A (R_S A^(A) R_S^T)^-1 from each variable's dense Poisson
    # matrix; the coarse couplings are D_1 = P^T D_0
    neu = ((0, 2), ())
    V = 2
    sysop = system.SystemOperator((0, 0, 0), (1, 1, 1), (2, 2, 2), 2, neu, C)
    fine = sysop.mesh
    split = multigrid.coarsen(fine)[1]
    coarse = multigrid.coarsen(fine)[0]
    D0 = _coupling(fine, V, seed=8)
    P = _dense_prolongation(fine, coarse, split)
    D1 = np.einsum("ji,abj->abi", P, D0)
    sys_c = system.SystemOperator(coarse.lower, coarse.upper, coarse.n, coarse.p, neu, C)
    A0, A1 = _dense_system(sysop, D0), _dense_system(sys_c, D1)

    def smoother_matrix(s_op):
        m = s_op.mesh
        n = m.ndof
        pois = [_poisson_dense(mv) for mv in s_op.meshes]
        Cm = np.zeros((V * n, V * n))
        for e in range(m.E):
            idx = schwarz.subdomain_layout(m, e, 2)[0]
            w = schwarz.subdomain_weights(m, e, 2)
            for a in range(V):
                rows = a * n + idx
                Cm[np.ix_(rows, rows)] += np.diag(w) @ np.linalg.inv(pois[a][np.ix_(idx, idx)])
        return Cm

    C0, C1 = smoother_matrix(sysop), smoother_matrix(sys_c)
    Pb = np.kron(np.eye(V), P)
    pre = post = 1

    def smooth(Cm, A, u, b, steps):
        for _ in range(steps):
            u = u + Cm @ (b - A @ u)
        return u

    b = W.random_normal(9, V * fine.ndof)
    u = smooth(C0, A0, np.zeros_like(b), b, pre)
    bc = Pb.T @ (b - A0 @ u)
    uc = smooth(C1, A1, np.zeros_like(bc), bc, pre + post)
    u = smooth(C0, A0, u + Pb @ uc, b, post)
    cyc = system.SystemVCycle(sysop, D0, levels=2, pre=pre, post=post, subdomain_iters=0)
    got = cyc(b)
    assert np.linalg.norm(got - u) / np.linalg.norm(u) < 1e-11


def test_matched_preconditioner_needs_fewer_outer_iterations():
    # the effect Sec. IV.B reports: with a Neumann variable, the Dirichlet
    # Laplacian approximation slows the solve and the matched one does not.
    # With one subdomain GMRES iteration the approximation decides the
    # subdomain solve (9 against 15 outer iterations here); with three,
    # GMRES makes up for the mismatch on this flat box
    neu = ((0, 2, 4), ())
    V = 2
    sysop = system.SystemOperator((0, 0, 0), (1, 1, 1), (4, 4, 2), 2, neu, C)
    m = sysop.mesh
    D = _coupling(m, V, seed=10)
    b = W.random_normal(11, V * m.ndof)
    A = lambda x: sysop.apply(x, D).reshape(-1)
    its = {}
    for bc in ("matched", "dirichlet"):
        cyc = system.SystemVCycle(sysop, D, levels=2, subdomain_iters=1, laplacian_bc=bc)
        x, its[bc], _ = krylov.fgmres(A, b, precondition=cyc, rtol=1e-10, max_iter=60)
        assert np.linalg.norm(b - A(x)) / np.linalg.norm(b) <= 1e-10
    assert its["matched"] + 3 <= its["dirichlet"], its
