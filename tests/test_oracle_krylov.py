"""Pins of the oracle's flexible GMRES (Sec. III.B, Saad Alg. 9.6)."""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import krylov, mesh, operator, multigrid
import workloads as W


def test_unpreconditioned_matches_dense_solve_and_scipy():
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 2, 1), 2)
    A = operator.assemble(m, 1.5)
    rng = np.random.default_rng(0)
    b = rng.standard_normal(m.ndof)
    x, k, hist = krylov.fgmres(lambda v: A @ v, b, rtol=1e-12, max_iter=m.ndof)
    assert k <= m.ndof
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-10)
    # same Krylov space as textbook GMRES without restart: equal iterates
    xs, info = spla.gmres(A, b, rtol=1e-12, restart=m.ndof, maxiter=1)
    np.testing.assert_allclose(x, xs, rtol=1e-8, atol=1e-9)
    assert np.all(np.diff(hist) <= 1e-15)  # monotone residual


def test_exact_preconditioner_converges_in_one_iteration():
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 1, 1), 3)
    A = operator.assemble(m, 1.5)
    b = np.random.default_rng(1).standard_normal(m.ndof)
    x, k, _ = krylov.fgmres(lambda v: A @ v, b, precondition=lambda v: np.linalg.solve(A, v))
    assert k == 1
    np.testing.assert_allclose(A @ x, b, rtol=1e-10, atol=1e-10)


def test_nonzero_initial_guess_and_estimate_is_true_residual():
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 2, 2), 3)
    x_, y_, z_ = m.node_coordinates()
    b = operator.apply_mass(m, W.sin_product_source(x_, y_, z_)).reshape(-1)
    A = lambda v: operator.apply_operator(m, v.reshape(m.E, 4, 4, 4), 1.5).reshape(-1)
    x0 = W.random_uniform(W.SEED_RANDOM_X0, m.ndof)
    x, k, hist = krylov.fgmres(A, b, x0=x0, precondition=multigrid.VCycle(m, 1.5, levels=2),
                               rtol=1e-10)
    r0 = np.linalg.norm(b - A(x0))
    true = np.linalg.norm(b - A(x)) / r0
    assert true <= 2e-10
    assert abs(true - hist[-1]) <= 1e-11
