"""Flexible GMRES (Sec. III.B; Saad 2003, Alg. 9.6) and preconditioned
conjugate gradients for symmetric positive definite problems (Sec. III.B;
Saad 2003, Alg. 9.1).

Test infrastructure only: imported by the tests, smoke() and the benchmark's
CPU leg, never by the product path.

One operator application and one preconditioner application per iteration;
the new basis vector is orthogonalised against all previous ones (modified
Gram-Schmidt), the small least-squares problem is updated with Givens
rotations, and the iteration stops when the residual estimate drops below
rtol times the initial residual norm.  The solution is x0 + Z y with Z the
preconditioned vectors.

Readings: no restart unless asked for; the residual is the Euclidean 2-norm
of the massive DG residual b - A x over all points; the stopping test uses
the Givens estimate (FGMRES) or the recursively updated residual (CG), and
the true residual b - A x then confirms it: when it is still above the
tolerance, the iteration goes on from the true residual (a new cycle), within
the same iteration limit.
"""
from __future__ import annotations

import numpy as np


def fgmres(apply_A, b, x0=None, precondition=None, rtol=1e-10, max_iter=200, restart=None):
    """Returns (x, iterations, history of relative residual estimates).

    restart=m: restarted FGMRES(m), cycles of at most m iterations, each
    started from the true residual of the previous cycle's solution; the
    tolerance and the history stay relative to the first cycle's ||r_0||
    and max_iter bounds the iterations of all cycles together."""
    b = np.asarray(b, float).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, float).reshape(-1).copy()
    M = precondition if precondition is not None else (lambda v: v.copy())
    m = max_iter if not restart else min(restart, max_iter)
    hist = [1.0]
    beta0 = None
    total = 0
    done = False
    while True:
        r0 = b - apply_A(x)
        beta = np.linalg.norm(r0)
        if beta0 is None:
            beta0 = beta
        if beta == 0.0:
            return x, total, hist
        if done and beta <= rtol * beta0:  # the true residual confirms the estimate
            return x, total, hist
        if total >= max_iter:
            return x, total, hist
        x, k, done = _fgmres_cycle(apply_A, M, x, r0, beta, beta0, rtol,
                                   min(m, max_iter - total), hist)
        total += k


def _fgmres_cycle(apply_A, M, x0, r0, beta, beta0, rtol, m, hist):
    """One cycle of at most m iterations from x0 with residual r0 = b - A x0
    (beta = ||r0||); appends the estimates |g_{j+1}| / beta0 to hist and
    returns (x, iterations, converged)."""
    V = [r0 / beta]
    Z = []
    H = np.zeros((m + 1, m))
    cs = np.zeros(m)
    sn = np.zeros(m)
    g = np.zeros(m + 1)
    g[0] = beta
    done = False
    j = 0
    for j in range(m):
        z = M(V[j])
        Z.append(z)
        w = apply_A(z)
        for i in range(j + 1):  # modified Gram-Schmidt
            H[i, j] = np.dot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        for i in range(j):  # apply previous rotations
            t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
            H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
            H[i, j] = t
        den = np.hypot(H[j, j], H[j + 1, j])
        cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
        H[j, j] = den
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        hist.append(abs(g[j + 1]) / beta0)
        done = abs(g[j + 1]) <= rtol * beta0
        if not done and H_next_zero(w):
            done = True
        if done:
            break
        V.append(w / np.linalg.norm(w))
    k = j + 1
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    x = x0 + sum(y[i] * Z[i] for i in range(k))
    return x, k, done


def H_next_zero(w):
    """Lucky breakdown: the new Krylov vector vanished."""
    return not np.any(w)


def cg(apply_A, b, x0=None, precondition=None, rtol=1e-10, max_iter=200):
    """Preconditioned conjugate gradients (Sec. III.B; Saad 2003, Alg. 9.1)
    for symmetric positive definite A.  Returns (x, iterations, history of
    ||r_k|| / ||r_0||).

    Reading: the direction update takes beta_k = (z_{k+1}, r_{k+1} - r_k) /
    (z_k, r_k) (the Polak-Ribiere form).  For a fixed symmetric positive
    definite preconditioner (z_{k+1}, r_k) vanishes and this is Saad's
    (z_{k+1}, r_{k+1}) / (z_k, r_k); unlike that form it keeps working when
    the preconditioner is not a fixed symmetric matrix, as the multigrid
    V-cycle with weighted additive Schwarz smoothing is not.  The iteration
    stops when the recursively updated residual satisfies ||r_k|| <= rtol
    ||r_0||; the true residual then confirms it, or CG starts again from the
    true residual.  One operator application, one preconditioner application
    and one round of dot products per iteration."""
    b = np.asarray(b, float).reshape(-1)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, float).reshape(-1).copy()
    M = precondition if precondition is not None else (lambda v: v.copy())
    hist = [1.0]
    nr0 = None
    k = 0
    while True:  # runs, each from the true residual of x
        r = b - apply_A(x)
        nr_start = np.linalg.norm(r)
        if nr0 is None:
            nr0 = nr_start
        if nr0 == 0.0 or (k > 0 and nr_start <= rtol * nr0) or k >= max_iter:
            return x, k, hist
        z = M(r)
        p = z.copy()
        rz = np.dot(r, z)
        hit = False
        while k < max_iter:
            k += 1
            q = apply_A(p)
            alpha = rz / np.dot(p, q)
            x = x + alpha * p
            r_next = r - alpha * q
            nr = np.linalg.norm(r_next)
            hist.append(nr / nr0)
            if nr <= rtol * nr0:
                hit = True
                break
            z = M(r_next)
            rz_next = np.dot(r_next, z)
            beta = (rz_next - np.dot(r, z)) / rz
            p = z + beta * p
            r, rz = r_next, rz_next
        if not hit:
            return x, k, hist
