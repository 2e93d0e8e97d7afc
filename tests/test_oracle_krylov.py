"""Pins of the oracle's flexible GMRES (Sec. III.B, Saad Alg. 9.6)."""
import numpy as np
import pytest
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


def _spd(n, seed, cond=30.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q @ np.diag(np.geomspace(1.0, cond, n)) @ Q.T


def _galerkin_iterate(A, b, K):
    """The point of the space spanned by the columns of K that minimises the
    A-norm of the error: the k-th conjugate-gradient iterate when K spans the
    k-th (preconditioned) Krylov space."""
    Q, _ = np.linalg.qr(K)
    return Q @ np.linalg.solve(Q.T @ A @ Q, Q.T @ b)


def test_cg_iterates_minimise_the_energy_error_over_krylov_spaces():
    # x_k = argmin over x in K_k(A, b) of ||x - x*||_A, built independently
    # from an orthonormal basis of the Krylov space; with a fixed SPD
    # preconditioner M the space is K_k(M A, M b)
    n = 12
    A = _spd(n, 3)
    b = np.random.default_rng(4).standard_normal(n)
    Mp = _spd(n, 5, cond=4.0)
    for precond in (None, Mp):
        M = (lambda v: v.copy()) if precond is None else (lambda v: precond @ v)
        for k in range(1, 6):
            x, its, _ = krylov.cg(lambda v: A @ v, b, precondition=M, rtol=1e-300, max_iter=k)
            assert its == k
            cols = [M(b)]
            for _ in range(k - 1):
                cols.append(M(A @ cols[-1]))
            ref = _galerkin_iterate(A, b, np.stack(cols, axis=1))
            np.testing.assert_allclose(x, ref, rtol=1e-9, atol=1e-12)


def test_cg_solves_spd_dg_poisson_and_stops_at_rtol():
    # the DG Poisson operator is symmetric positive definite; unpreconditioned
    # CG reaches the dense solution, and with the (non-symmetric) V-cycle the
    # flexible update still converges to the same solution
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 2, 1), 2)
    A = operator.assemble(m, 1.5)
    assert np.allclose(A, A.T) and np.linalg.eigvalsh(A).min() > 0
    b = np.random.default_rng(6).standard_normal(m.ndof)
    ref = np.linalg.solve(A, b)
    x, k, hist = krylov.cg(lambda v: A @ v, b, rtol=1e-12, max_iter=10 * m.ndof)
    np.testing.assert_allclose(x, ref, rtol=1e-8, atol=1e-10)
    assert hist[-1] <= 1e-12 and all(h > 1e-12 for h in hist[:-1])
    V = multigrid.VCycle(m, 1.5, levels=2)
    x, k2, hist = krylov.cg(lambda v: A @ v, b, precondition=V, rtol=1e-10)
    assert k2 < k and hist[-1] <= 1e-10
    np.testing.assert_allclose(x, ref, rtol=1e-8, atol=1e-10)
    # a zero right-hand side needs no iteration
    x0, k0, h0 = krylov.cg(lambda v: A @ v, np.zeros(m.ndof))
    assert k0 == 0 and h0 == [1.0] and not np.any(x0)


def test_restarted_fgmres_equals_scipy_restarted_gmres_and_converges():
    # unpreconditioned FGMRES(m) is GMRES(m): after c cycles its iterate is
    # scipy's GMRES with restart=m and maxiter=c cycles
    m_ = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 2, 1), 2)
    A = operator.assemble(m_, 1.5)
    b = np.random.default_rng(8).standard_normal(m_.ndof)
    for m, c in ((5, 2), (8, 3)):
        x, k, hist = krylov.fgmres(lambda v: A @ v, b, rtol=1e-300, max_iter=m * c, restart=m)
        assert k == m * c and len(hist) == k + 1
        xs, _ = spla.gmres(A, b, rtol=1e-300, atol=0.0, restart=m, maxiter=c)
        np.testing.assert_allclose(x, xs, rtol=1e-8, atol=1e-10)
        # the history is relative to the first residual and drops across cycles
        assert hist[0] == 1.0 and hist[m] < 1.0 and hist[-1] < hist[m]
    # with the V-cycle it converges to the dense solution; a restart longer
    # than the run changes nothing
    V = multigrid.VCycle(m_, 1.5, levels=2)
    ref = np.linalg.solve(A, b)
    x1, k1, h1 = krylov.fgmres(lambda v: A @ v, b, precondition=V, rtol=1e-10)
    x2, k2, h2 = krylov.fgmres(lambda v: A @ v, b, precondition=V, rtol=1e-10, restart=k1)
    assert k2 == k1 and np.array_equal(x1, x2) and h1 == h2
    x3, k3, h3 = krylov.fgmres(lambda v: A @ v, b, precondition=V, rtol=1e-10, restart=3)
    assert k3 >= k1 and h3[-1] <= 1e-10
    np.testing.assert_allclose(x3, ref, rtol=1e-8, atol=1e-10)


def _ill_conditioned(seed, n, decades, nonsymmetric):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = Q @ np.diag(np.logspace(0, decades, n)) @ Q.T
    if nonsymmetric:
        A = A + 1e2 * rng.standard_normal((n, n))
    return A, rng.standard_normal(n)


@pytest.mark.parametrize("seed", [1, 4, 5, 7])
def test_fgmres_confirms_the_estimate_with_the_true_residual(seed):
    # ill-conditioned systems (n = 120, Jacobi preconditioner) on which the
    # Givens estimate reaches the tolerance one or two iterations before the
    # true residual b - A x does: the run goes on from the true residual and
    # returns a solution that meets the tolerance
    A, b = _ill_conditioned(seed, 120, 6, True)
    d = np.diag(A).copy()
    x, k, hist = krylov.fgmres(lambda v: A @ v, b, precondition=lambda v: v / d, rtol=1e-12)
    assert hist[-1] <= 1e-12 and k < 200
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)
    # a tolerance below the rounding floor is never reported as met
    x, k, hist = krylov.fgmres(lambda v: A @ v, b, precondition=lambda v: v / d, rtol=1e-15,
                               max_iter=150)
    assert k == 150 or np.linalg.norm(b - A @ x) <= 1e-15 * np.linalg.norm(b)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cg_reports_convergence_only_at_the_true_residual(seed):
    # at a tolerance near the rounding floor the recursive residual runs
    # ahead of the true one: a run that stops before the iteration limit
    # must have its true residual at the tolerance
    A, b = _ill_conditioned(seed, 150, 4, False)
    d = np.diag(A).copy()
    for rtol in (1e-12, 1e-13):
        x, k, hist = krylov.cg(lambda v: A @ v, b, precondition=lambda v: v / d, rtol=rtol,
                               max_iter=1500)
        assert k == 1500 or np.linalg.norm(b - A @ x) <= rtol * np.linalg.norm(b)
