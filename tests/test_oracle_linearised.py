"""Pins of the oracle's linearised smoother and linearised multigrid cycle.

The linearised problem (Sec. III.A, eq. linearized) adds a pointwise term to
the Poisson operator: A + diag(d), d the mass-weighted derivative of the
nonlinear source.  Each subdomain problem (A_S + diag(R_S d)) du_S = r_S is
solved by a fixed number of GMRES iterations preconditioned with the explicit
inverse of the Poisson A_S (Laplacian approximation, Sec. III.E.1), and the
coarse grids carry the restricted term d_{l+1} = R d_l.

Every expected value here is built without the smoother's own code path:
subdomain operators come from the assembled global matrix and dense
restriction matrices, Krylov spaces from explicit matrix powers, and the
multigrid cycle from dense matrix compositions.
"""
import numpy as np
import pytest

from oracle import mesh, multigrid, operator, schwarz


def _restriction(m, e, ov):
    idx = schwarz.subdomain_layout(m, e, ov)[0]
    R = np.zeros((len(idx), m.ndof))
    R[np.arange(len(idx)), idx] = 1.0
    return R


def _random_diag(m, seed, scale):
    # a positive pointwise term with no structure that a point permutation keeps
    return np.random.default_rng(seed).uniform(0.2, 1.8, m.ndof) * scale


def _minimiser_right_preconditioned(K_op, Minv, r, k):
    """argmin |r - K_op x| over x in Minv K_k(K_op Minv, r), the space that k
    right-preconditioned GMRES iterations from zero search (Saad 2003,
    Sec. 9.3.2).  The Krylov basis is the explicit power sequence, made
    orthonormal by a QR factorisation."""
    KM = K_op @ Minv
    cols = [r]
    for _ in range(k - 1):
        cols.append(KM @ cols[-1])
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    X = Minv @ Q
    y = np.linalg.lstsq(K_op @ X, r, rcond=None)[0]
    return X @ y


def test_one_element_step_solves_the_linearised_system():
    # one subdomain covering the whole domain and as many subdomain GMRES
    # iterations as unknowns: one step solves (A + diag(d)) u = b exactly
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (1, 1, 1), 2)
    A = operator.assemble(m, 1.5)
    d = _random_diag(m, 11, np.abs(np.diag(A)).mean())
    b = np.random.default_rng(12).standard_normal(m.ndof)
    S = schwarz.SchwarzSmoother(m, 1.5, 2, diag=d, subdomain_iters=m.ndof)
    u = S.smooth(np.zeros(m.ndof), b, 1)
    want = np.linalg.solve(A + np.diag(d), b)
    np.testing.assert_allclose(u, want, rtol=1e-10, atol=1e-10 * np.abs(want).max())
    # and it differs from the Poisson solve: the term is not dropped
    poisson = np.linalg.solve(A, b)
    assert np.linalg.norm(u - poisson) > 1e-3 * np.linalg.norm(poisson)


def test_step_with_exact_subdomain_solves_matches_dense_formula():
    # u + sum_S R_S^T W_S (A_S + D_S)^-1 R_S (b - (A + D) u), D_S = diag(R_S d),
    # with the subdomain GMRES run to as many iterations as the largest n_S
    m = mesh.BoxMesh([0, 0, 0], [1, 1.3, 0.8], (3, 2, 2), 1)
    ov = 2  # capped at N - 1 = 1 layer
    A = operator.assemble(m, 1.5)
    d = _random_diag(m, 13, np.abs(np.diag(A)).mean())
    D = np.diag(d)
    rng = np.random.default_rng(14)
    u0, b = rng.standard_normal(m.ndof), rng.standard_normal(m.ndof)
    B = np.zeros((m.ndof, m.ndof))
    nmax = 0
    for e in range(m.E):
        R = _restriction(m, e, ov)
        nmax = max(nmax, R.shape[0])
        AS = R @ (A + D) @ R.T
        B += R.T @ np.diag(schwarz.subdomain_weights(m, e, ov)) @ np.linalg.inv(AS) @ R
    want = u0 + B @ (b - (A + D) @ u0)
    S = schwarz.SchwarzSmoother(m, 1.5, ov, diag=d, subdomain_iters=nmax)
    np.testing.assert_allclose(S.smooth(u0, b, 1), want, rtol=1e-9, atol=1e-9 * np.abs(want).max())


@pytest.mark.parametrize("n,p,ov,k", [((3, 2, 2), 2, 2, 3), ((2, 3, 1), 3, 1, 3),
                                      ((3, 2, 2), 2, 2, 1), ((2, 2, 2), 2, 2, 5)])
def test_fixed_gmres_step_is_the_krylov_minimiser(n, p, ov, k):
    # each subdomain's correction is the minimiser of |r_S - (A_S + D_S) x|
    # over x in M K_k((A_S + D_S) M, r_S) with M = A_S^-1 (Poisson): right
    # preconditioning, zero initial guess, exactly k iterations
    m = mesh.BoxMesh([0, 0, 0], [1, 0.9, 1.2], n, p)
    A = operator.assemble(m, 1.5)
    d = _random_diag(m, 15, 3.0 * np.abs(np.diag(A)).mean())
    rng = np.random.default_rng(16)
    u0, b = rng.standard_normal(m.ndof), rng.standard_normal(m.ndof)
    r = b - (A + np.diag(d)) @ u0
    du = np.zeros(m.ndof)
    for e in range(m.E):
        R = _restriction(m, e, ov)
        AS = R @ A @ R.T
        x = _minimiser_right_preconditioned(AS + np.diag(R @ d), np.linalg.inv(AS), R @ r, k)
        du += R.T @ (schwarz.subdomain_weights(m, e, ov) * x)
    S = schwarz.SchwarzSmoother(m, 1.5, ov, diag=d, subdomain_iters=k)
    got = S.smooth(u0, b, 1)
    np.testing.assert_allclose(got, u0 + du, rtol=1e-9, atol=1e-9 * np.abs(du).max())
    # the pointwise term matters at this strength: the Poisson inverse alone
    # (k = 0) gives a different correction
    S0 = schwarz.SchwarzSmoother(m, 1.5, ov, diag=d, subdomain_iters=0)
    assert np.linalg.norm(S0.smooth(u0, b, 1) - got) > 1e-3 * np.linalg.norm(du)


def test_left_preconditioning_would_differ():
    # guard on the pin above: the left-preconditioned minimiser (of
    # |M (r - K x)| over K_k(M K, M r)) is a different vector here, so the
    # pin separates the two sides of preconditioning
    m = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 2, 2), 2)
    A = operator.assemble(m, 1.5)
    d = _random_diag(m, 17, 3.0 * np.abs(np.diag(A)).mean())
    r = np.random.default_rng(18).standard_normal(m.ndof)
    R = _restriction(m, 0, 2)
    AS = R @ A @ R.T
    K, Minv, rS = AS + np.diag(R @ d), np.linalg.inv(AS), R @ r
    right = _minimiser_right_preconditioned(K, Minv, rS, 3)
    cols = [Minv @ rS]
    for _ in range(2):
        cols.append(Minv @ K @ cols[-1])
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    left = Q @ np.linalg.lstsq(Minv @ K @ Q, Minv @ rS, rcond=None)[0]
    assert np.linalg.norm(right - left) > 1e-4 * np.linalg.norm(right)


def _dense(f, n):
    return np.stack([f(np.eye(n)[j]) for j in range(n)], axis=1)


@pytest.mark.parametrize("k", [0, "exact"])
def test_two_level_linearised_cycle_matches_dense_composition(k):
    # V-cycle on A_l + diag(d_l) with d_1 = P^T d_0 (the restriction of the
    # massive term), smoothing u <- u + B_l (b - (A_l + D_l) u), with
    #   k = 0:      B_l = sum_S R_S^T W_S A_S^-1 R_S (the Poisson inverse alone)
    #   k = exact:  B_l = sum_S R_S^T W_S (A_S + D_S)^-1 R_S
    fine = mesh.BoxMesh([0, 0, 0], [1, 1, 1], (2, 2, 2), 2)
    coarse, split = multigrid.coarsen(fine)
    ov = 2
    A0, A1 = operator.assemble(fine, 1.5), operator.assemble(coarse, 1.5)
    P = _dense(lambda v: multigrid.prolongate(fine, coarse, split, v), coarse.ndof)
    d0 = _random_diag(fine, 19, 2.0 * np.abs(np.diag(A0)).mean())
    d1 = P.T @ d0
    K0, K1 = A0 + np.diag(d0), A1 + np.diag(d1)

    def smoother_matrix(m, A, d):
        B = np.zeros((m.ndof, m.ndof))
        nmax = 0
        for e in range(m.E):
            R = _restriction(m, e, ov)
            nmax = max(nmax, R.shape[0])
            AS = R @ A @ R.T
            if k == "exact":
                AS = AS + np.diag(R @ d)
            B += R.T @ np.diag(schwarz.subdomain_weights(m, e, ov)) @ np.linalg.inv(AS) @ R
        return B, nmax

    B0, n0 = smoother_matrix(fine, A0, d0)
    B1, n1 = smoother_matrix(coarse, A1, d1)

    def smooth(K, B, u, b, steps):
        for _ in range(steps):
            u = u + B @ (b - K @ u)
        return u

    b = np.random.default_rng(20).standard_normal(fine.ndof)
    u = smooth(K0, B0, np.zeros(fine.ndof), b, 3)
    bc = P.T @ (b - K0 @ u)
    uc = smooth(K1, B1, smooth(K1, B1, np.zeros(coarse.ndof), bc, 3), bc, 3)
    want = smooth(K0, B0, u + P @ uc, b, 3)
    iters = 0 if k == 0 else max(n0, n1)
    V = multigrid.VCycle(fine, 1.5, levels=2, overlap=ov, diag=d0, subdomain_iters=iters)
    got = V(b)
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())
    # the coarse term is not optional: leaving it out changes the cycle
    B1z, _ = smoother_matrix(coarse, A1, np.zeros(coarse.ndof))
    uc_z = smooth(A1, B1z, smooth(A1, B1z, np.zeros(coarse.ndof), bc, 3), bc, 3)
    without = smooth(K0, B0, u + P @ uc_z, b, 3)
    assert np.linalg.norm(without - want) > 1e-6 * np.linalg.norm(want)
