"""GPU checks at the benchmark sizes, through the C ABI.

* 8^3, p = 6 and 16^3, p = 7 solves (mixed and FP64) of the random-Fourier
  Poisson problems: the oracle's own operator re-checks the true residual of
  the GPU solution, the error against the exact solution of the continuous
  problem is bounded, and at 8^3 the solution equals the oracle's FGMRES
  solution (same iteration count).
* The 40^3, p = 7 operator apply (the out-of-cache shape, in the launch shape
  the benchmark times) on sampled elements against the oracle.
"""
import numpy as np
import pytest

import workloads as W
from oracle import krylov, mesh as omesh, multigrid, operator as oop
from tests.gpu_util import announce, rel_max, to_gpu, to_np

pytestmark = pytest.mark.gpu

C = 1.5


def _fourier_problem(n, p, seed):
    m = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (n, n, n), p)
    x, y, z = m.node_coordinates()
    modes = W.fourier_modes(seed)
    f = W.fourier_source(modes, x, y, z)
    b = oop.apply_mass(m, f.reshape(m.E, m.N, m.N, m.N)).reshape(-1)
    uex = W.fourier_solution(modes, x, y, z).reshape(-1)
    return m, b, uex


def _oracle_residual(m, u, b):
    r = b - oop.apply_operator(m, u.reshape(m.E, m.N, m.N, m.N), C).reshape(-1)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def c2_oracle():
    """The oracle's FGMRES solve of the 8^3, p = 6 problem (V-cycle
    preconditioned, 3 levels, tolerance 1e-10)."""
    m, b, uex = _fourier_problem(8, 6, W.SEED_C2)
    A = lambda v: oop.apply_operator(m, v.reshape(m.E, m.N, m.N, m.N), C).reshape(-1)
    V = multigrid.VCycle(m, C, levels=3)
    u, its, _ = krylov.fgmres(A, b, precondition=V, rtol=1e-10)
    return m, b, uex, u, its


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c2_solve_matches_oracle_solve(c2_oracle, precision):
    import paper_2111_06767_amd as dg
    announce(f"full-size solve 8^3 p=6 {precision}")
    m, b, uex, u_or, its_or = c2_oracle
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (8, 8, 8), 6, penalty=C, mg_levels=3,
                      precision=precision)
    u, st = prob.solve(to_gpu(b))
    un = to_np(u)
    prob.close()
    assert st["iterations"] == its_or, (st["iterations"], its_or)
    assert st["rel_residual"] <= 1e-10
    assert _oracle_residual(m, un, b) <= 1e-10
    assert np.linalg.norm(un - u_or) / np.linalg.norm(u_or) <= 1e-9
    # discretisation error of the DG solution against the continuous one
    assert np.sqrt(np.mean((un - uex) ** 2)) <= 5e-9


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_c5_solve_residual_through_oracle_operator(precision):
    import paper_2111_06767_amd as dg
    announce(f"full-size solve 16^3 p=7 {precision}")
    m, b, uex = _fourier_problem(16, 7, W.SEED_C5)
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (16, 16, 16), 7, penalty=C, mg_levels=4,
                      precision=precision)
    u, st = prob.solve(to_gpu(b))
    un = to_np(u)
    prob.close()
    assert st["rel_residual"] <= 1e-10
    assert st["iterations"] <= 12  # h-independent convergence of the MG-Schwarz V-cycle
    assert _oracle_residual(m, un, b) <= 1e-10
    assert np.sqrt(np.mean((un - uex) ** 2)) <= 1e-9


def test_apply_40cubed_p7_sampled():
    """Elements sampled over the 40^3 box (corners, faces, edges and the
    interior) against the oracle on the 3x3x3 patch around each."""
    import paper_2111_06767_amd as dg
    announce("apply parity 40^3 p=7 sampled")
    n, p = 40, 7
    N = p + 1
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (n, n, n), p, penalty=C, mg_levels=1)
    u = W.random_normal(W.SEED_APPLY, prob.ndof)
    got = to_np(prob.apply(to_gpu(u))).reshape(n, n, n, N, N, N)
    prob.close()
    ug = u.reshape(n, n, n, N, N, N)
    h = 1.0 / n
    rng = np.random.default_rng(1)
    samples = [np.array(c) for c in [(0, 0, 0), (n - 1, n - 1, n - 1), (0, 17, n - 1), (21, 0, 5)]]
    samples += [rng.integers(0, n, 3) for _ in range(6)]
    for c in samples:
        lo = np.maximum(c - 1, 0)
        hi = np.minimum(c + 2, n)
        sub = ug[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        pm = omesh.BoxMesh(lo * h, hi * h, tuple(hi - lo), p)
        ref = oop.apply_operator(pm, sub.reshape(-1, N, N, N), C)[pm.elem_index(*(c - lo))]
        assert rel_max(got[c[2], c[1], c[0]], ref) < 1e-13, c


@pytest.mark.parametrize("name,opts", [("cg", dict()), ("restarted_fgmres_4", dict(restart=4)),
                                       ("wcycle", dict(cycle=2)), ("fcycle", dict(cycle=3)),
                                       ("additive_mg", dict(additive=1))])
def test_c2_solver_variants_through_oracle_operator(name, opts):
    # the benchmark's c2 variants (8^3, p = 6, mixed precision): CG, restarted
    # FGMRES and the W-, F- and additive cycles, each checked by the oracle's
    # residual of its solution
    import paper_2111_06767_amd as dg
    announce(f"c2 variant {name}")
    m, b, uex = _fourier_problem(8, 6, W.SEED_C2)
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (8, 8, 8), 6, penalty=C, mg_levels=3, precision="mixed",
                      **opts)
    u, st = (prob.solve_cg if name == "cg" else prob.solve)(to_gpu(b))
    un = to_np(u)
    prob.close()
    assert st["converged"], st
    assert _oracle_residual(m, un, b) <= 1e-10
