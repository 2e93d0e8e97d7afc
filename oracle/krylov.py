"""Flexible GMRES (Sec. III.B; Saad 2003, Alg. 9.6).

One operator application and one preconditioner application per iteration;
the new basis vector is orthogonalised against all previous ones (modified
Gram-Schmidt), the small least-squares problem is updated with Givens
rotations, and the iteration stops when the residual estimate drops below
rtol times the initial residual norm.  The solution is x0 + Z y with Z the
preconditioned vectors.

Readings: no restart; the residual is the Euclidean 2-norm of the massive DG
residual b - A x over all points; the stopping test uses the Givens estimate.
"""
from __future__ import annotations

import numpy as np


def fgmres(apply_A, b, x0=None, precondition=None, rtol=1e-10, max_iter=200):
    """Returns (x, iterations, history of relative residual estimates)."""
    b = np.asarray(b, float).reshape(-1)
    x0 = np.zeros_like(b) if x0 is None else np.asarray(x0, float).reshape(-1).copy()
    M = precondition if precondition is not None else (lambda v: v.copy())
    r0 = b - apply_A(x0)
    beta = np.linalg.norm(r0)
    hist = [1.0]
    if beta == 0.0:
        return x0, 0, hist
    V = [r0 / beta]
    Z = []
    H = np.zeros((max_iter + 1, max_iter))
    cs = np.zeros(max_iter)
    sn = np.zeros(max_iter)
    g = np.zeros(max_iter + 1)
    g[0] = beta
    j = 0
    for j in range(max_iter):
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
        hist.append(abs(g[j + 1]) / beta)
        done = abs(g[j + 1]) <= rtol * beta
        if not done and H_next_zero(w):
            done = True
        if done:
            break
        V.append(w / np.linalg.norm(w))
    k = j + 1
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    x = x0 + sum(y[i] * Z[i] for i in range(k))
    return x, k, hist


def H_next_zero(w):
    """Lucky breakdown: the new Krylov vector vanished."""
    return not np.any(w)
