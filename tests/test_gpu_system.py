"""GPU parity of multi-variable systems (Sec. III.E.1, eq. lapl_approx)
against the oracle, through the C ABI: the coupled operator, Schwarz steps
with the matched and the Dirichlet Laplacian approximation (k = 0 and k = 3
subdomain GMRES iterations), the V-cycle, and FGMRES solves in FP64 and
mixed precision."""
import numpy as np
import pytest

import workloads as W
from oracle import krylov, operator as oop, system
from tests.gpu_util import announce, rel_max, to_gpu, to_np

pytestmark = pytest.mark.gpu

C = 1.5


def _coupling(m, nvars, seed):
    x, y, z = m.node_coordinates()
    c = W.system_coupling(seed, nvars, x, y, z)
    mass = np.broadcast_to(oop.mass_diagonal(m), (m.E, m.N, m.N, m.N)).reshape(-1)
    D = c * mass[None, None, :]
    D[0, 1] *= 1.5  # not symmetric: a transposed coupling would show
    return D


def test_system_apply_matches_oracle():
    import paper_2111_06767_amd as dg
    announce("system apply 3 variables (3,2,2) p=3")
    neu = ((0, 2), (), (5,))
    sysop = system.SystemOperator((0, 0, 0), (1, 0.8, 1.1), (3, 2, 2), 3, neu, C)
    m = sysop.mesh
    D = _coupling(m, 3, 31)
    u = W.random_normal(32, 3 * m.ndof)
    ref = sysop.apply(u, D).reshape(-1)
    S = dg.System((0, 0, 0), (1, 0.8, 1.1), (3, 2, 2), 3, neu, mg_levels=1)
    assert S.ndof == m.ndof
    got0 = to_np(S.apply(to_gpu(u)))
    ref0 = sysop.apply(u).reshape(-1)
    assert rel_max(got0, ref0) < 1e-13
    S.set_coupling(to_gpu(D.reshape(-1)))
    got = to_np(S.apply(to_gpu(u)))
    assert rel_max(got, ref) < 1e-13, rel_max(got, ref)
    S.close()


@pytest.mark.parametrize("laplacian_bc", ["matched", "dirichlet"])
@pytest.mark.parametrize("k", [0, 3])
def test_system_schwarz_step_matches_oracle(laplacian_bc, k):
    import paper_2111_06767_amd as dg
    announce(f"system schwarz step {laplacian_bc} k={k}")
    neu = ((0, 2), ())
    lower, upper, el, p = (0, 0, 0), (1.2, 1, 0.9), (4, 2, 2), 3
    sysop = system.SystemOperator(lower, upper, el, p, neu, C)
    m = sysop.mesh
    D = _coupling(m, 2, 33)
    b = W.random_normal(34, 2 * m.ndof)
    u0 = W.random_uniform(35, 2 * m.ndof)
    sm = system.SystemSchwarzSmoother(sysop.meshes, C, D, subdomain_iters=k, laplacian_bc=laplacian_bc)
    ref = sm.smooth(u0, b, 2).reshape(-1)
    S = dg.System(lower, upper, el, p, neu, laplacian_bc=laplacian_bc, mg_levels=1,
                  subdomain_iters=k)
    S.set_coupling(to_gpu(D.reshape(-1)))
    u = to_gpu(u0)
    S.smooth(to_gpu(b), u, 2)
    got = to_np(u)
    assert rel_max(got, ref) < 1e-10, rel_max(got, ref)
    S.close()


def test_system_vcycle_matches_oracle():
    import paper_2111_06767_amd as dg
    announce("system vcycle 2 levels k=3")
    neu = ((0, 2, 4), (1,))
    lower, upper, el, p = (0, 0, 0), (1, 1, 1), (4, 4, 2), 2
    sysop = system.SystemOperator(lower, upper, el, p, neu, C)
    m = sysop.mesh
    D = _coupling(m, 2, 36)
    r = W.random_normal(37, 2 * m.ndof)
    ref = system.SystemVCycle(sysop, D, levels=2, subdomain_iters=3)(r)
    S = dg.System(lower, upper, el, p, neu, mg_levels=2, subdomain_iters=3)
    S.set_coupling(to_gpu(D.reshape(-1)))
    got = to_np(S.precondition(to_gpu(r)))
    assert rel_max(got, ref) < 1e-10, rel_max(got, ref)
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_system_solve_matches_oracle(precision):
    import paper_2111_06767_amd as dg
    announce(f"system solve {precision}")
    neu = ((0, 2, 4), ())
    lower, upper, el, p = (0, 0, 0), (1, 1, 1), (4, 4, 2), 2
    sysop = system.SystemOperator(lower, upper, el, p, neu, C)
    m = sysop.mesh
    D = _coupling(m, 2, 38)
    b = W.random_normal(39, 2 * m.ndof)
    A = lambda x: sysop.apply(x, D).reshape(-1)
    cyc = system.SystemVCycle(sysop, D, levels=2, subdomain_iters=1)
    x_ref, its_ref, _ = krylov.fgmres(A, b, precondition=cyc, rtol=1e-10, max_iter=60)
    S = dg.System(lower, upper, el, p, neu, mg_levels=2, subdomain_iters=1, precision=precision,
                  max_iter=60)
    S.set_coupling(to_gpu(D.reshape(-1)))
    u, st = S.solve(to_gpu(b))
    u = to_np(u)
    assert st["converged"] and st["rel_residual"] <= 1e-10
    assert abs(st["iterations"] - its_ref) <= 1, (st["iterations"], its_ref)
    assert np.linalg.norm(b - A(u)) / np.linalg.norm(b) <= 1e-10
    assert np.linalg.norm(u - x_ref) / np.linalg.norm(x_ref) <= 1e-9
    S.close()


def test_matched_boundary_types_need_fewer_iterations_on_gpu():
    # the effect of Sec. IV.B: with a Neumann variable and one subdomain
    # GMRES iteration, the Dirichlet Laplacian approximation needs clearly
    # more outer iterations than the matched one (9 against 15 in the oracle)
    import paper_2111_06767_amd as dg
    announce("system matched vs dirichlet")
    neu = ((0, 2, 4), ())
    lower, upper, el, p = (0, 0, 0), (1, 1, 1), (4, 4, 2), 2
    m = system.SystemOperator(lower, upper, el, p, neu, C).mesh
    D = to_gpu(_coupling(m, 2, 10).reshape(-1))
    b = to_gpu(W.random_normal(11, 2 * m.ndof))
    its = {}
    for bc in ("matched", "dirichlet"):
        S = dg.System(lower, upper, el, p, neu, laplacian_bc=bc, mg_levels=2, subdomain_iters=1,
                      max_iter=60)
        S.set_coupling(D)
        _, st = S.solve(b)
        assert st["converged"]
        its[bc] = st["iterations"]
        S.close()
    assert its["matched"] + 3 <= its["dirichlet"], its


def test_system_limits():
    import paper_2111_06767_amd as dg
    announce("system limits")
    with pytest.raises(dg.DgsError):
        dg.System((0, 0, 0), (1, 1, 1), (2, 2, 2), 2, [()] * 6)
    with pytest.raises(dg.DgsError):  # interior subdomains of 1000 + 6 * 2 * 100 points
        dg.System((0, 0, 0), (1, 1, 1), (3, 3, 3), 9, [(), ()], mg_levels=1)
    with pytest.raises(dg.DgsError):  # every face Neumann
        dg.System((0, 0, 0), (1, 1, 1), (2, 2, 2), 2, [tuple(range(6))])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_five_variable_system_full_size_through_oracle_operator(precision):
    # the benchmark's system: five variables on 8^3 elements, p = 6, with their
    # own Neumann faces and pointwise couplings; the GPU solution's residual
    # taken with the oracle's system operator
    import paper_2111_06767_amd as dg
    announce(f"five-variable system 8^3 p=6 {precision} through the oracle operator")
    nv = len(W.SYSTEM_NEUMANN)
    lower, upper, el, p = (0, 0, 0), (1, 1, 1), (8, 8, 8), 6
    sysop = system.SystemOperator(lower, upper, el, p, W.SYSTEM_NEUMANN, C)
    m = sysop.mesh
    x, y, z = m.node_coordinates()
    c = W.system_coupling(W.SEED_SYSTEM, nv, x, y, z)
    mass = np.broadcast_to(oop.mass_diagonal(m), (m.E, m.N, m.N, m.N)).reshape(-1)
    D = c * mass[None, None, :]
    b = np.concatenate([oop.apply_mass(m, W.fourier_source(W.fourier_modes(W.SEED_SYSTEM + 1 + a), x, y, z)
                                       .reshape(m.E, m.N, m.N, m.N)).reshape(-1) for a in range(nv)])
    S = dg.System(lower, upper, el, p, W.SYSTEM_NEUMANN, mg_levels=3, subdomain_iters=3,
                  precision=precision, max_iter=100)
    S.set_coupling(to_gpu(D.reshape(-1)))
    u, st = S.solve(to_gpu(b))
    S.close()
    assert st["converged"] and st["iterations"] <= 12, st
    r = b - sysop.apply(to_np(u), D).reshape(-1)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b)
