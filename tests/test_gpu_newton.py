"""GPU parity of the linearised-operator smoother (subdomain GMRES with the
Laplacian-approximation preconditioner) and of the Newton-Raphson solver
against the oracle, through the C ABI."""
import numpy as np
import pytest

import workloads as W
from oracle import mesh as omesh, multigrid, newton as onewton, operator as oop, schwarz
from tests.gpu_util import announce, rel_max, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _diag(m, seed):
    # a positive mass-weighted pointwise term, like M dS/du of the puncture source
    c = np.random.default_rng(seed).uniform(0.5, 20.0, m.ndof).reshape(m.E, m.N, m.N, m.N)
    return (oop.mass_diagonal(m) * c).reshape(-1)


BOX = (1.0, 1.2, 0.9)


# the unit-cube cases give axes of equal element width: classes shared across
# axes, the subdomain's diagonal read through exchanged-axis frames
@pytest.mark.parametrize("elements,p,k,upper", [((2, 2, 2), 3, 3, BOX), ((3, 2, 2), 2, 3, BOX),
                                                ((2, 2, 2), 4, 0, BOX), ((3, 3, 2), 3, 2, BOX),
                                                ((3, 3, 3), 3, 3, (1, 1, 1)),
                                                ((2, 3, 3), 2, 2, (1, 1.5, 1.5))])
def test_linearised_schwarz_matches_oracle(elements, p, k, upper):
    import paper_2111_06767_amd as dg
    announce(f"linearised schwarz elements={elements} p={p} k={k} upper={upper}")
    prob = dg.Problem((0, 0, 0), upper, elements, p, subdomain_iters=k)
    m = omesh.BoxMesh((0, 0, 0), upper, elements, p)
    d = _diag(m, 5)
    prob.set_diagonal(to_gpu(d))
    S = schwarz.SchwarzSmoother(m, 1.5, 2, diag=d, subdomain_iters=k)
    b = W.random_normal(51, m.ndof)
    u0 = W.random_uniform(52, m.ndof)
    for steps in (1, 2):
        ref = S.smooth(u0, b, steps)
        u = to_gpu(u0)
        prob.smooth(to_gpu(b), u, steps)
        err = rel_max(to_np(u), ref)
        assert err < 1e-10, (steps, err)


def test_linearised_vcycle_and_solve_match_oracle():
    import paper_2111_06767_amd as dg
    from oracle import krylov
    announce("linearised vcycle 4x2x2 p=3")
    m = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (4, 2, 2), 3)
    d = _diag(m, 6)
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (4, 2, 2), 3, mg_levels=2, subdomain_iters=3)
    prob.set_diagonal(to_gpu(d))
    V = multigrid.VCycle(m, 1.5, levels=2, diag=d, subdomain_iters=3)
    r = W.random_normal(61, m.ndof)
    got = to_np(prob.precondition(to_gpu(r)))
    assert rel_max(got, V(r)) < 1e-10
    J = lambda x: oop.apply_operator(m, x.reshape(m.E, 4, 4, 4), 1.5).reshape(-1) + d * x
    x_ref, its_ref, _ = krylov.fgmres(J, r, precondition=V, rtol=1e-10)
    x, st = prob.solve(to_gpu(r))
    assert st["converged"] and abs(st["iterations"] - its_ref) <= 1
    assert np.linalg.norm(to_np(x) - x_ref) / np.linalg.norm(x_ref) < 1e-9
    prob.set_diagonal(None)  # back to the plain operator


def _puncture(elements, p):
    m = omesh.BoxMesh((-20, -20, -20), (20, 20, 20), elements, p)
    x, y, z = m.node_coordinates()
    alpha, beta = W.puncture_background(W.puncture_params(W.SEED_C3), x, y, z)
    return m, alpha.reshape(-1), beta.reshape(-1)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_newton_matches_oracle_small(precision):
    import paper_2111_06767_amd as dg
    announce(f"newton 2x2x2 p=4 {precision}")
    m, alpha, beta = _puncture((2, 2, 2), 4)
    u_ref, info = onewton.newton_solve(m, 1.5, alpha, beta, newton_rtol=1e-10, linear_rtol=1e-4,
                                       levels=2, subdomain_iters=3)
    prob = dg.Problem((-20, -20, -20), (20, 20, 20), (2, 2, 2), 4, mg_levels=2, subdomain_iters=3,
                      precision=precision)
    u, st = prob.newton_solve(to_gpu(alpha), to_gpu(beta), newton_rtol=1e-10, linear_rtol=1e-4)
    u = to_np(u)
    assert st["converged"]
    # the oracle's own residual of the GPU solution
    F = lambda v: oop.apply_operator(m, v.reshape(m.E, 5, 5, 5), 1.5,
                                     source=onewton.puncture_source(alpha, beta, v).reshape(m.E, 5, 5, 5))
    r0 = np.linalg.norm(F(np.zeros(m.ndof)))
    assert np.linalg.norm(F(u)) / r0 <= 1e-10
    assert np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref) <= 1e-9
    if precision == "fp64":
        assert st["newton_steps"] == info["steps"]


def test_newton_puncture_full_size():
    # the 6^3, p = 7 puncture problem on [-20, 20]^3: the GPU solution satisfies
    # the oracle's nonlinear DG equations to the Newton tolerance
    import paper_2111_06767_amd as dg
    announce("newton 6x6x6 p=7 puncture")
    m, alpha, beta = _puncture((6, 6, 6), 7)
    F = lambda v: oop.apply_operator(m, v.reshape(m.E, 8, 8, 8), 1.5,
                                     source=onewton.puncture_source(alpha, beta, v).reshape(m.E, 8, 8, 8))
    r0 = np.linalg.norm(F(np.zeros(m.ndof)))
    sols = {}
    for precision in ("fp64", "mixed"):
        prob = dg.Problem((-20, -20, -20), (20, 20, 20), (6, 6, 6), 7, mg_levels=2, subdomain_iters=3,
                          precision=precision)
        u, st = prob.newton_solve(to_gpu(alpha), to_gpu(beta), newton_rtol=1e-10, linear_rtol=1e-4)
        u = to_np(u)
        assert st["converged"], st
        assert np.linalg.norm(F(u)) / r0 <= 1e-10
        sols[precision] = u
    assert np.linalg.norm(sols["mixed"] - sols["fp64"]) / np.linalg.norm(sols["fp64"]) <= 1e-9
