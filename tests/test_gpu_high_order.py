"""GPU parity at polynomial degrees 9..12 (10 to 13 points per dimension)
against the oracle, through the C ABI: the operator in every launch shape,
Schwarz steps (subdomains of up to 4225 points), the linearised smoother
with its subdomain GMRES, and a preconditioned solve."""
import numpy as np
import pytest

import workloads as W
from oracle import krylov, mesh as omesh, multigrid, operator as oop, schwarz
from tests.gpu_util import announce, rel_max, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("elements,p", [((2, 2, 1), 9), ((1, 2, 2), 10), ((2, 1, 2), 11),
                                        ((3, 2, 1), 12)])
def test_high_order_apply_matches_oracle(elements, p):
    import paper_2111_06767_amd as dg
    announce(f"apply p={p} elements={elements}")
    upper = (1.0, 0.8, 1.3)
    m = omesh.BoxMesh((0, 0, 0), upper, elements, p)
    u = W.random_normal(W.SEED_APPLY + p, m.ndof)
    ref = oop.apply_operator(m, u.reshape(m.E, m.N, m.N, m.N), 1.5).reshape(-1)
    prob = dg.Problem((0, 0, 0), upper, elements, p, penalty=1.5, mg_levels=1)
    outs = []
    for shape in (1, 2, 0):
        prob.set_apply_shape(shape)
        outs.append(to_np(prob.apply(to_gpu(u))))
        assert rel_max(outs[-1], ref) < 1e-13, (shape, rel_max(outs[-1], ref))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    with pytest.raises(dg.DgsError):
        prob.set_apply_shape(-1)  # bricks are a p = 7 shape
    prob.close()


@pytest.mark.parametrize("elements,p", [((2, 2, 1), 9), ((2, 1, 1), 12)])
def test_high_order_schwarz_matches_oracle(elements, p):
    import paper_2111_06767_amd as dg
    announce(f"schwarz p={p} elements={elements}")
    upper = (1.0, 1.2, 0.9)
    m = omesh.BoxMesh((0, 0, 0), upper, elements, p)
    prob = dg.Problem((0, 0, 0), upper, elements, p, penalty=1.5, mg_levels=1)
    b = W.random_normal(81, m.ndof)
    u0 = W.random_uniform(82, m.ndof)
    S = schwarz.SchwarzSmoother(m, 1.5, 2)
    ref = S.smooth(u0, b, 1)
    u = to_gpu(u0)
    prob.smooth(to_gpu(b), u, 1)
    assert rel_max(to_np(u), ref) < 1e-11, rel_max(to_np(u), ref)
    prob.close()


def test_high_order_linearised_schwarz_matches_oracle():
    # p = 11 on 2x2x2: every subdomain has 1728 + 3 * 2 * 144 = 2592 points,
    # beyond 2048, so the Arnoldi kernel runs its 17-points-per-thread form
    import paper_2111_06767_amd as dg
    announce("linearised schwarz p=11 2x2x2")
    m = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (2, 2, 2), 11)
    c = np.random.default_rng(83).uniform(0.5, 20.0, m.ndof).reshape(m.E, m.N, m.N, m.N)
    d = (oop.mass_diagonal(m) * c).reshape(-1)
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (2, 2, 2), 11, mg_levels=1, subdomain_iters=3)
    prob.set_diagonal(to_gpu(d))
    S = schwarz.SchwarzSmoother(m, 1.5, 2, diag=d, subdomain_iters=3)
    b = W.random_normal(84, m.ndof)
    u0 = W.random_uniform(85, m.ndof)
    ref = S.smooth(u0, b, 1)
    u = to_gpu(u0)
    prob.smooth(to_gpu(b), u, 1)
    assert rel_max(to_np(u), ref) < 1e-10, rel_max(to_np(u), ref)
    prob.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_high_order_solve_matches_oracle(precision):
    import paper_2111_06767_amd as dg
    announce(f"solve p=10 2x2x2 {precision}")
    m = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (2, 2, 2), 10)
    x, y, z = m.node_coordinates()
    b = oop.apply_mass(m, W.sin_product_source(x, y, z)).reshape(-1)
    N = m.N
    A = lambda v: oop.apply_operator(m, v.reshape(m.E, N, N, N), 1.5).reshape(-1)
    u_ref, its_ref, _ = krylov.fgmres(A, b, precondition=multigrid.VCycle(m, 1.5, levels=2),
                                      rtol=1e-10)
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (2, 2, 2), 10, mg_levels=2, precision=precision)
    u, st = prob.solve(to_gpu(b))
    u = to_np(u)
    assert st["converged"] and st["rel_residual"] <= 1e-10
    assert abs(st["iterations"] - its_ref) <= 1, (st["iterations"], its_ref)
    assert np.linalg.norm(b - A(u)) / np.linalg.norm(b) <= 1e-10
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) <= 1e-9
    prob.close()


def test_degree_limits():
    import paper_2111_06767_amd as dg
    announce("degree limits")
    assert len(dg.lgl_nodes(12)) == 13
    with pytest.raises(dg.DgsError):
        dg.Problem((0, 0, 0), (1, 1, 1), (1, 1, 1), 13)
    with pytest.raises(dg.DgsError):
        dg.lgl_nodes(13)
