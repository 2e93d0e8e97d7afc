"""Newton-Raphson with a backtracking line search (Sec. III.A, eq. linearized).

Test infrastructure only: imported by the tests, smoke() and the benchmark's
CPU leg, never by the product path.

The nonlinear DG residual is F(u) = A u + M S(u) - b, with the linear flux
part A of Sec. II and a pointwise source S.  Each step solves the linearised
problem (dA/du)(u) du = b - A(u) with preconditioned flexible GMRES to a
relative tolerance, then backtracks the step length lambda until the
sufficient-decrease condition holds, and updates u <- u + lambda du.

Puncture source (the nonlinear workload): the equation
Laplace(u) + beta (alpha (1+u) + 1)^-7 = 0 in flux form -Laplace(u) + S_u = 0
has S_u(u) = -beta (alpha (1+u) + 1)^-7 and dS_u/du = 7 alpha beta
(alpha (1+u) + 1)^-8.

Power-law sources on curved elements (newton_solve_powers): S(u) =
sum_t c_t(x) u^(k_t), the form one XCTS equation (eq. xcts) takes when the
other variables are held fixed, with Dirichlet data through the ghost state
of eq. bc; pinned by the Kerr-Schild lapse equation on a wedge (exponential
convergence to the analytic lapse), by Newton with dense linear solves, and
by the one-step solve of an affine source.

Readings:
* f(u) = 1/2 ||F(u)||^2; the predicted decrease is that of the linear model,
  so the initial slope is -||F(u)||^2; sufficient decrease
  f(u + lambda du) <= f(u) + a lambda slope with a = 1e-4.
* backtracking as in Dennis & Schnabel (the algorithm the paper names):
  quadratic interpolation on the first backtrack, cubic afterwards, the new
  lambda clamped to [0.1, 0.5] times the previous one, lambda = 1 first, at
  most ``max_backtracks`` backtracks per step.
* convergence when ||F(u)|| <= newton_rtol ||F(u_0)||.
"""
from __future__ import annotations

import numpy as np

from . import curved
from .mesh import BoxMesh
from .operator import apply_operator, mass_diagonal
from .krylov import fgmres
from .multigrid import VCycle


def puncture_source(alpha, beta, u):
    return -beta * (alpha * (1.0 + u) + 1.0) ** -7


def puncture_source_derivative(alpha, beta, u):
    return 7.0 * alpha * beta * (alpha * (1.0 + u) + 1.0) ** -8


def backtrack(f0, slope, lam, f_lam, lam_prev, f_prev, first):
    """Next trial step length (quadratic first, cubic afterwards)."""
    if first:
        t = -slope * lam ** 2 / (2.0 * (f_lam - f0 - slope * lam))
    else:
        r1 = f_lam - f0 - lam * slope
        r2 = f_prev - f0 - lam_prev * slope
        a = (r1 / lam ** 2 - r2 / lam_prev ** 2) / (lam - lam_prev)
        b = (-lam_prev * r1 / lam ** 2 + lam * r2 / lam_prev ** 2) / (lam - lam_prev)
        if a == 0.0:
            t = -slope / (2.0 * b)
        else:
            disc = max(b * b - 3.0 * a * slope, 0.0)
            t = (-b + np.sqrt(disc)) / (3.0 * a)
    t = min(t, 0.5 * lam)
    return max(t, 0.1 * lam)


def newton_solve(mesh: BoxMesh, C, alpha, beta, b=None, u0=None, newton_rtol=1e-10,
                 linear_rtol=1e-4, max_newton=20, levels=2, overlap=2, pre=3, post=3,
                 subdomain_iters=3, sufficient_decrease=1e-4, max_backtracks=10,
                 max_linear_iter=200):
    """Returns (u, info) with the residual history and iteration counts."""
    N = mesh.N
    shape = (mesh.E, N, N, N)
    alpha = np.asarray(alpha, float).reshape(shape)
    beta = np.asarray(beta, float).reshape(shape)
    b = np.zeros(shape) if b is None else np.asarray(b, float).reshape(shape)
    u = np.zeros(shape) if u0 is None else np.asarray(u0, float).reshape(shape).copy()
    M = mass_diagonal(mesh)

    def F(v):
        return apply_operator(mesh, v, C, source=puncture_source(alpha, beta, v)) - b

    Fu = F(u)
    norm0 = np.linalg.norm(Fu)
    hist = [1.0]
    linear_its = []
    steps = 0
    backtracks = 0
    for _ in range(max_newton):
        nrm = np.linalg.norm(Fu)
        if nrm <= newton_rtol * norm0 or nrm == 0.0:
            break
        d = (M * puncture_source_derivative(alpha, beta, u)).reshape(-1)

        def J(x):
            return apply_operator(mesh, x.reshape(shape), C).reshape(-1) + d * x

        V = VCycle(mesh, C, levels=levels, overlap=overlap, pre=pre, post=post,
                   diag=d, subdomain_iters=subdomain_iters)
        du, its, _ = fgmres(J, -Fu.reshape(-1), precondition=V, rtol=linear_rtol,
                            max_iter=max_linear_iter)
        linear_its.append(its)
        du = du.reshape(shape)
        f0 = 0.5 * nrm ** 2
        slope = -nrm ** 2
        lam, lam_prev, f_prev = 1.0, None, None
        for bt in range(max_backtracks + 1):
            Ft = F(u + lam * du)
            ft = 0.5 * np.linalg.norm(Ft) ** 2
            if ft <= f0 + sufficient_decrease * lam * slope or bt == max_backtracks:
                break
            new = backtrack(f0, slope, lam, ft, lam_prev, f_prev, first=(bt == 0))
            lam_prev, f_prev, lam = lam, ft, new
            backtracks += 1
        u = u + lam * du
        Fu = Ft
        steps += 1
        hist.append(np.linalg.norm(Fu) / norm0)
    return u.reshape(-1), dict(steps=steps, history=hist, linear_iterations=linear_its,
                               backtracks=backtracks)


def power_source(coefs, powers, u):
    """S(u) = sum_t c_t u^(k_t) and dS/du, for integer powers k_t."""
    S = np.zeros_like(u)
    dS = np.zeros_like(u)
    for c, k in zip(coefs, powers):
        S += c * u ** float(k)
        if k != 0:
            dS += c * k * u ** float(k - 1)
    return S, dS


def newton_solve_powers(cm, C, coefs, powers, ginv=None, sqrtg=None, dirichlet=None, b=None,
                        u0=None, newton_rtol=1e-10, linear_rtol=1e-4, max_newton=20, levels=2,
                        overlap=2, pre=3, post=3, subdomain_iters=3, sufficient_decrease=1e-4,
                        max_backtracks=10, max_linear_iter=200, dense=False):
    """Newton-Raphson on curved elements for F(u) = A(u; u_b) + M S(u) - b with
    the pointwise source S(u) = sum_t c_t u^(k_t) (Sec. III.A; on a
    background metric when ginv and sqrtg are given, Sec. II).  A(u; u_b) is
    the curved operator with the Dirichlet data u_b (nodal, read at boundary
    nodes; None: homogeneous); M its diagonal mass.  Each linearisation
    A + diag(M S'(u)) is solved by FGMRES preconditioned by the box grid's
    V-cycle on A_box + diag(M S'(u)) (or, with dense=True, by a dense solve),
    then the step length is backtracked as in newton_solve.  u0: initial guess
    (ones if None).  Returns (u, info)."""
    box = cm.box
    n = box.ndof
    coefs = [np.asarray(c, float).reshape(-1) for c in np.asarray(coefs, float).reshape(len(powers), -1)]
    if ginv is None:
        Mdiag = curved.mass_diagonal(cm).reshape(-1)

        def A(v, ub=None):
            return curved.apply_operator(cm, v, C, dirichlet_values=ub)
    else:
        Mdiag = (np.asarray(sqrtg, float).reshape(cm.det.shape) * curved.mass_diagonal(cm)).reshape(-1)

        def A(v, ub=None):
            return curved.apply_operator_metric(cm, v, C, ginv, sqrtg, dirichlet_values=ub)
    ub = None if dirichlet is None else np.asarray(dirichlet, float).reshape(-1)
    b = np.zeros(n) if b is None else np.asarray(b, float).reshape(-1)
    u = np.ones(n) if u0 is None else np.asarray(u0, float).reshape(-1).copy()

    def F(v):
        return A(v, ub) + Mdiag * power_source(coefs, powers, v)[0] - b

    Fu = F(u)
    norm0 = np.linalg.norm(Fu)
    hist = [1.0]
    linear_its = []
    steps = backtracks = 0
    for _ in range(max_newton):
        nrm = np.linalg.norm(Fu)
        if nrm <= newton_rtol * norm0 or nrm == 0.0:
            break
        d = Mdiag * power_source(coefs, powers, u)[1]

        def J(x):
            return A(x) + d * x

        if dense:
            Jm = np.stack([J(e) for e in np.eye(n)], axis=1)
            du = np.linalg.solve(Jm, -Fu)
            linear_its.append(0)
        else:
            V = VCycle(box, C, levels=levels, overlap=overlap, pre=pre, post=post, diag=d,
                       subdomain_iters=subdomain_iters)
            du, its, _ = fgmres(J, -Fu, precondition=V, rtol=linear_rtol, max_iter=max_linear_iter)
            linear_its.append(its)
        f0 = 0.5 * nrm ** 2
        slope = -nrm ** 2
        lam, lam_prev, f_prev = 1.0, None, None
        for bt in range(max_backtracks + 1):
            Ft = F(u + lam * du)
            ft = 0.5 * np.linalg.norm(Ft) ** 2
            if ft <= f0 + sufficient_decrease * lam * slope or bt == max_backtracks:
                break
            new = backtrack(f0, slope, lam, ft, lam_prev, f_prev, first=(bt == 0))
            lam_prev, f_prev, lam = lam, ft, new
            backtracks += 1
        u = u + lam * du
        Fu = Ft
        steps += 1
        hist.append(np.linalg.norm(Fu) / norm0)
    return u, dict(steps=steps, history=hist, linear_iterations=linear_its, backtracks=backtracks)


def monomial_source(terms, u):
    """S_a(u) = sum over the terms (c, k) of variable a of c prod_b u_b^(k_b),
    and D_ab = dS_a/du_b, for u of shape (V, n)."""
    V, n = u.shape
    S = np.zeros((V, n))
    D = np.zeros((V, V, n))
    for a in range(V):
        for c, k in terms[a]:
            c = np.asarray(c, float).reshape(-1)
            S[a] += c * np.prod([u[q] ** float(k[q]) for q in range(V)], axis=0)
            for b in range(V):
                if k[b] == 0:
                    continue
                f = c * k[b] * u[b] ** float(k[b] - 1)
                for q in range(V):
                    if q != b:
                        f = f * u[q] ** float(k[q])
                D[a, b] += f
    return S, D


def system_newton_solve_powers(meshes, xyz, C, terms, ginv=None, sqrtg=None, dirichlet=None, b=None,
                               u0=None, newton_rtol=1e-10, linear_rtol=1e-4, max_newton=20, levels=2,
                               overlap=2, pre=3, post=3, subdomain_iters=3, laplacian_bc="matched",
                               sufficient_decrease=1e-4, max_backtracks=10, max_linear_iter=200,
                               dense=False):
    """Newton-Raphson (Sec. III.A) for a coupled system of V variables on
    curved elements: F_a(u) = A_a(u_a; u_b,a) + M S_a(u) - b_a with sources
    that are sums of monomials in all variables (``terms[a]`` lists (c, k),
    k the V powers), e.g. the XCTS equations (eq. xcts) with some variables
    held fixed.  ``meshes[a]`` is variable a's box grid (its own Neumann
    faces), all with the node coordinates xyz; on a background metric when
    ginv and sqrtg are given.  Each linearisation blockdiag(A_a) + M dS/du is
    solved by FGMRES preconditioned by the system V-cycle of the box grids
    with the couplings D = M dS/du (Sec. III.E.1; or by a dense solve), then
    the step length is backtracked as in newton_solve.  u0: (V, n), ones if
    None.  Returns (u of shape (V, n), info)."""
    from .system import SystemOperator, SystemVCycle
    V = len(meshes)
    cms = [curved.CurvedMesh(m, xyz) for m in meshes]
    n = meshes[0].ndof
    if ginv is None:
        Mdiag = curved.mass_diagonal(cms[0]).reshape(-1)

        def A(a, v, ub=None):
            return curved.apply_operator(cms[a], v, C, dirichlet_values=ub)
    else:
        Mdiag = (np.asarray(sqrtg, float).reshape(cms[0].det.shape) *
                 curved.mass_diagonal(cms[0])).reshape(-1)

        def A(a, v, ub=None):
            return curved.apply_operator_metric(cms[a], v, C, ginv, sqrtg, dirichlet_values=ub)
    ub = [None] * V if dirichlet is None else np.asarray(dirichlet, float).reshape(V, n)
    b = np.zeros((V, n)) if b is None else np.asarray(b, float).reshape(V, n)
    u = np.ones((V, n)) if u0 is None else np.asarray(u0, float).reshape(V, n).copy()
    m0 = meshes[0]
    sysop = SystemOperator(m0.lower, m0.upper, m0.n, m0.p, [m.neumann for m in meshes], C)

    def F(v):
        return np.stack([A(a, v[a], ub[a]) for a in range(V)]) + Mdiag * monomial_source(terms, v)[0] - b

    Fu = F(u)
    norm0 = np.linalg.norm(Fu)
    hist = [1.0]
    linear_its = []
    steps = backtracks = 0
    for _ in range(max_newton):
        nrm = np.linalg.norm(Fu)
        if nrm <= newton_rtol * norm0 or nrm == 0.0:
            break
        D = Mdiag * monomial_source(terms, u)[1]

        def J(x):
            x = x.reshape(V, n)
            return (np.stack([A(a, x[a]) for a in range(V)]) + np.einsum("abn,bn->an", D, x)).reshape(-1)

        if dense:
            Jm = np.stack([J(e) for e in np.eye(V * n)], axis=1)
            du = np.linalg.solve(Jm, -Fu.reshape(-1))
            linear_its.append(0)
        else:
            P = SystemVCycle(sysop, D, levels=levels, overlap=overlap, pre=pre, post=post,
                             subdomain_iters=subdomain_iters, laplacian_bc=laplacian_bc)
            du, its, _ = fgmres(J, -Fu.reshape(-1), precondition=P, rtol=linear_rtol,
                                max_iter=max_linear_iter)
            linear_its.append(its)
        du = du.reshape(V, n)
        f0 = 0.5 * nrm ** 2
        slope = -nrm ** 2
        lam, lam_prev, f_prev = 1.0, None, None
        for bt in range(max_backtracks + 1):
            Ft = F(u + lam * du)
            ft = 0.5 * np.linalg.norm(Ft) ** 2
            if ft <= f0 + sufficient_decrease * lam * slope or bt == max_backtracks:
                break
            new = backtrack(f0, slope, lam, ft, lam_prev, f_prev, first=(bt == 0))
            lam_prev, f_prev, lam = lam, ft, new
            backtracks += 1
        u = u + lam * du
        Fu = Ft
        steps += 1
        hist.append(np.linalg.norm(Fu) / norm0)
    return u, dict(steps=steps, history=hist, linear_iterations=linear_its, backtracks=backtracks)
