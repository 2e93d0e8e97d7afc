"""Additive Schwarz smoother on element-centred overlapping subdomains.

Test infrastructure only: imported by the tests, smoke() and the benchmark's
CPU leg, never by the product path.

Follows Sec. III.D:

* geometry (Sec. III.D.1, Fig. subdomain_structure): subdomain S_k is the
  element Omega_k plus N_overlap points into each *face* neighbour, up to but
  excluding the neighbour's face that points away; no edge or corner
  neighbours.
* restriction R_S discards data outside S; R_S^T extends by zero (Sec. III.D.2).
* subdomain operator A_S = R_S A R_S^T (Sec. III.D.2).
* subdomain problem A_S du_S = r_S with r_S = R_S (b - A u)
  (eq. schwarz_subd_problem), solved here exactly with the explicit inverse of
  A_S (Sec. III.E.2, explicit-inverse solver; an LU/dense inverse).
* weighted additive update u <- u + sum_S R_S^T (w_S du_S)
  (eq. schwarz_weighting) with w = W(xi) = prod_i w(xi^i)
  (eq. schwarz_weight_prod) and the quintic smoothstep 1D weight
  (eq. schwarz_weight_function).
* missing corner/edge weight is added to the face neighbours that share it
  (end of Sec. III.D.4).

Subdomain vector order: the central element's N^3 points in element order
(x fastest), then for each existing face neighbour in the order -x, +x, -y,
+y, -z, +z a strip of N_ov layers, layer 0 nearest the shared face, each layer
N^2 points with the lower transverse dimension fastest.

Readings:
* N_ov is capped at N - 1 (the far face is never included).
* overlap width delta = 1 + xi_{N_ov}: the logical distance from the central
  element's face to the neighbour's first point outside the overlap
  (xi ascending from the shared face).
* external boundaries: the 1D weight is extended to 1 toward an external face,
  i.e. phi((xi+1)/delta) is replaced by +1 when the low face is external and
  phi((xi-1)/delta) by -1 when the high face is external.
* the corner/edge weight is split equally among the face neighbours that share
  the edge (1/2 each) or corner (1/3 each).  With a_t = w(xi_t) the central
  element's own transverse weights, the weight of a face-neighbour strip
  normal to d is w(xi_d) * T(a_j, a_k) with
  T = a_j a_k + (1-a_j) a_k / 2 + a_j (1-a_k) / 2 + (1-a_j)(1-a_k) / 3.
* the product in eq. schwarz_weight_prod runs over the d dimensions.
"""
from __future__ import annotations

import numpy as np

from . import lgl
from .mesh import BoxMesh
from .operator import apply_operator

FACE_ORDER = ((0, -1), (0, +1), (1, -1), (1, +1), (2, -1), (2, +1))


def overlap_layers(N, overlap):
    return max(1, min(int(overlap), N - 1))


def overlap_width(N, overlap):
    """delta = 1 + xi_{N_ov} (eq. schwarz_weight_function, Fig. schwarz_weight_function)."""
    return 1.0 + lgl.nodes(N)[overlap_layers(N, overlap)]


def smoothstep(x):
    """phi: quintic smoothstep on [-1, 1], sign(x) outside."""
    x = np.asarray(x, dtype=float)
    inner = (15.0 * x - 10.0 * x ** 3 + 3.0 * x ** 5) / 8.0
    return np.where(np.abs(x) <= 1.0, inner, np.sign(x))


def weight_1d(xi, delta, low_external=False, high_external=False):
    """w(xi) = 1/2 (phi((xi+1)/delta) - phi((xi-1)/delta)), extended to 1 toward
    external faces."""
    lo = np.ones_like(np.asarray(xi, float)) if low_external else smoothstep((np.asarray(xi) + 1.0) / delta)
    hi = -np.ones_like(np.asarray(xi, float)) if high_external else smoothstep((np.asarray(xi) - 1.0) / delta)
    return 0.5 * (lo - hi)


def _transverse(d):
    return tuple(t for t in range(3) if t != d)


def subdomain_layout(mesh: BoxMesh, e, overlap):
    """Global flat indices of the subdomain's points, their subdomain-logical
    coordinates xi_S (n_S x 3) and the dimension normal to the strip each point
    lies in (-1 for the central element), in subdomain order."""
    N = mesh.N
    nov = overlap_layers(N, overlap)
    xi = lgl.nodes(N)
    idx, coords, normal = [], [], []
    for k in range(N):
        for j in range(N):
            for i in range(N):
                idx.append(((e * N + k) * N + j) * N + i)
                coords.append((xi[i], xi[j], xi[k]))
                normal.append(-1)
    for d, s in FACE_ORDER:
        b = mesh.neighbor(e, d, s)
        if b is None:
            continue
        t0, t1 = _transverse(d)
        for layer in range(nov):
            m = layer if s > 0 else N - 1 - layer
            for b1 in range(N):
                for b0 in range(N):
                    node = [0, 0, 0]
                    node[d], node[t0], node[t1] = m, b0, b1
                    i, j, k = node
                    idx.append(((b * N + k) * N + j) * N + i)
                    c = [0.0, 0.0, 0.0]
                    c[d] = 2.0 * s + xi[m]
                    c[t0], c[t1] = xi[b0], xi[b1]
                    coords.append(tuple(c))
                    normal.append(d)
    return np.array(idx, dtype=np.int64), np.array(coords), np.array(normal)


def subdomain_size(N, overlap, n_faces=6, n_vars=1):
    """n_S = n_vars (N^3 + n_faces N_ov N^2)."""
    return n_vars * (N ** 3 + n_faces * overlap_layers(N, overlap) * N ** 2)


def subdomain_weights(mesh: BoxMesh, e, overlap):
    """Weight w_S at every subdomain point (eqs. schwarz_weight_prod,
    schwarz_weight_function, plus the corner/edge redistribution)."""
    _, coords, normal = subdomain_layout(mesh, e, overlap)
    delta = overlap_width(mesh.N, overlap)
    flags = mesh.external_flags(e)
    a = np.stack([weight_1d(coords[:, d], delta, *flags[d]) for d in range(3)], axis=1)
    w = np.empty(len(coords))
    central = normal < 0
    w[central] = np.prod(a[central], axis=1)
    for n in np.nonzero(~central)[0]:
        d = int(normal[n])
        j, k = _transverse(d)
        aj, ak = a[n, j], a[n, k]
        T = aj * ak + 0.5 * (1 - aj) * ak + 0.5 * aj * (1 - ak) + (1 - aj) * (1 - ak) / 3.0
        w[n] = a[n, d] * T
    return w


def element_class(mesh: BoxMesh, e):
    """Boundary class of an element: its six external-face flags."""
    return mesh.external_flags(e)


def patch_for_class(mesh: BoxMesh, flags):
    """A small box mesh (1..3 elements per dimension, same h) whose central
    element has the given external-face flags, and that element's index.
    Data outside the subdomain is zero, so the rows of A that belong to the
    subdomain only see the central element, its face neighbours and zeros."""
    lower, upper, n, c = [], [], [], []
    for d in range(3):
        lo_ext, hi_ext = flags[d]
        cd = 0 if lo_ext else 1
        nd = 1 + (0 if lo_ext else 1) + (0 if hi_ext else 1)
        # place the patch so that its external faces coincide with the box
        if lo_ext:
            l0 = mesh.lower[d]
        elif hi_ext:
            l0 = mesh.upper[d] - nd * mesh.h[d]
        else:
            l0 = mesh.lower[d]
        lower.append(l0)
        upper.append(l0 + nd * mesh.h[d])
        n.append(nd)
        c.append(cd)
    # the box's boundary conditions by face; the patch's cut faces only touch
    # rows outside the subdomain, whatever condition they carry
    patch = BoxMesh(lower, upper, n, mesh.p, neumann=mesh.neumann)
    return patch, patch.elem_index(*c)


def subdomain_operator_literal(mesh: BoxMesh, e, C, overlap):
    """A_S = R_S A R_S^T by applying the global operator to zero-extended
    subdomain unit vectors (tiny meshes only)."""
    idx = subdomain_layout(mesh, e, overlap)[0]
    n = len(idx)
    N = mesh.N
    X = np.zeros((n, mesh.ndof))
    X[np.arange(n), idx] = 1.0
    AX = apply_operator(mesh, X.reshape(n, mesh.E, N, N, N), C).reshape(n, -1)
    return AX[:, idx].T.copy()


def subdomain_operator(mesh: BoxMesh, flags, C, overlap, chunk=256):
    """A_S for any element of the given class, computed on the class patch."""
    patch, ep = patch_for_class(mesh, flags)
    idx = subdomain_layout(patch, ep, overlap)[0]
    n = len(idx)
    N = mesh.N
    A_S = np.empty((n, n))
    for c0 in range(0, n, chunk):
        cols = np.arange(c0, min(n, c0 + chunk))
        X = np.zeros((len(cols), patch.ndof))
        X[np.arange(len(cols)), idx[cols]] = 1.0
        AX = apply_operator(patch, X.reshape(len(cols), patch.E, N, N, N), C)
        A_S[:, cols] = AX.reshape(len(cols), -1)[:, idx].T
    return A_S


def gmres_fixed(apply_A, apply_Minv, r, iterations):
    """Right-preconditioned GMRES with zero initial guess and a fixed number of
    iterations (no tolerance check), used as the subdomain solver of the
    linearised problem."""
    beta = np.linalg.norm(r)
    if beta == 0.0:
        return np.zeros_like(r)
    V = [r / beta]
    Z = []
    H = np.zeros((iterations + 1, iterations))
    m = 0
    for j in range(iterations):
        z = apply_Minv(V[j])
        Z.append(z)
        w = apply_A(z)
        for i in range(j + 1):
            H[i, j] = np.dot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        m = j + 1
        if H[j + 1, j] == 0.0:
            break
        V.append(w / H[j + 1, j])
    g = np.zeros(m + 1)
    g[0] = beta
    y = np.linalg.lstsq(H[:m + 1, :m], g, rcond=None)[0]
    return sum(y[i] * Z[i] for i in range(m))


class SchwarzSmoother:
    """Additive Schwarz smoother on one grid.

    ``diag`` (optional, flat array) adds a pointwise term diag(d) to the
    operator, A + diag(d), as for the linearised nonlinear problem.  Then each
    subdomain problem (A_S + diag(R_S d)) du_S = r_S is solved by
    ``subdomain_iters`` iterations of GMRES preconditioned with the explicit
    inverse of the Poisson A_S (Laplacian approximation, Sec. III.E.1).
    """

    def __init__(self, mesh: BoxMesh, C, overlap=2, diag=None, subdomain_iters=0):
        self.mesh, self.C, self.overlap = mesh, C, overlap
        self.diag = None if diag is None else np.asarray(diag, float).reshape(-1)
        self.subdomain_iters = subdomain_iters
        self.layout = [subdomain_layout(mesh, e, overlap) for e in range(mesh.E)]
        self.weights = [subdomain_weights(mesh, e, overlap) for e in range(mesh.E)]
        self.cls = [element_class(mesh, e) for e in range(mesh.E)]
        self.A_S, self.A_S_inv = {}, {}
        for key in sorted(set(self.cls)):
            A = subdomain_operator(mesh, key, C, overlap)
            self.A_S[key] = A
            self.A_S_inv[key] = np.linalg.inv(A)

    def apply(self, u):
        N = self.mesh.N
        Au = apply_operator(self.mesh, u.reshape(self.mesh.E, N, N, N), self.C).reshape(-1)
        if self.diag is not None:
            Au = Au + self.diag * u.reshape(-1)
        return Au

    def correction(self, r):
        """sum_S R_S^T (w_S du_S) for the residual r."""
        r = r.reshape(-1)
        du = np.zeros_like(r)
        groups = {}
        for e in range(self.mesh.E):
            groups.setdefault(self.cls[e], []).append(e)
        for key, elems in groups.items():
            Ainv = self.A_S_inv[key]
            RS = np.stack([r[self.layout[e][0]] for e in elems])
            if self.diag is None or self.subdomain_iters == 0:
                DU = RS @ Ainv.T
            else:
                A_S = self.A_S[key]
                DU = []
                for row, e in zip(RS, elems):
                    dS = self.diag[self.layout[e][0]]
                    DU.append(gmres_fixed(lambda x: A_S @ x + dS * x,
                                          lambda x: Ainv @ x, row, self.subdomain_iters))
                DU = np.stack(DU)
            for row, e in zip(DU, elems):
                np.add.at(du, self.layout[e][0], self.weights[e] * row)
        return du

    def smooth(self, u, b, steps):
        """``steps`` Schwarz iterations on A u = b starting from u."""
        u = np.array(u, dtype=float).reshape(-1)
        b = np.asarray(b, float).reshape(-1)
        for _ in range(steps):
            r = b - self.apply(u)
            u = u + self.correction(r)
        return u
