"""DG Poisson operator on curved (isoparametric) elements, Sec. II.

Test infrastructure only: imported by tests and the benchmark's CPU leg,
never by the product path.

The block is the box grid of ``mesh.BoxMesh`` (its topology, element
neighbours and boundary faces), but every node carries its own physical
coordinates x(xi): the element map is the degree-p interpolant of the node
coordinates, and the node coordinates of neighbouring elements agree on
shared faces.  The background metric is flat (sqrt(g) = 1).

With LGL quadrature on the element's own points:

* the Jacobian J^i_j = dx^i/dxi^j is the collocation derivative of the
  coordinate fields, with determinant J and inverse invJ^j_i = dxi^j/dx^i;
* eq. massmat: M = J w_i w_j w_k (diagonal);
* eq. stiffmat: D_i = M^-1 MD_i is the collocation derivative
  (D_i u)_p = invJ^j_i(p) (D^xi_j u)_p, applied at each node with that
  node's metric;
* eq. liftop on a face normal to xi^d: the outward unit normal one-form is
  n_i = s invJ^d_i / |invJ^d|, the surface Jacobian is J |invJ^d| (Nanson's
  formula), and ML = J |invJ^d| w_a w_b is diagonal on the face, so the
  lifting coefficient L = M^-1 ML at a face node is |invJ^d| / w_end.

Fluxes, boundary conditions and the penalty are those of ``operator.py``
(eqs. numflux, bc, penalty), with n_ext = -n_int.

Reading: h in eq. penalty, "a measure of the element size orthogonal to the
boundary", is 2 / |invJ^d| at the face node, taken on each side of the face
(the element width for affine elements).
"""
from __future__ import annotations

import numpy as np

from . import lgl
from .mesh import BoxMesh, NODE_AXIS


def _apply_1d(a, D, axis):
    a = np.moveaxis(a, axis, -1)
    return np.moveaxis(a @ D.T, -1, axis)


class CurvedMesh:
    """A box grid with curved node coordinates xyz of shape (3, E, N, N, N)."""

    def __init__(self, box: BoxMesh, xyz):
        self.box = box
        self.xyz = np.asarray(xyz, float).reshape(3, box.E, box.N, box.N, box.N)
        N = box.N
        D = lgl.diff_matrix(N)
        J = np.empty(self.xyz.shape[1:] + (3, 3))
        for i in range(3):
            for j in range(3):
                J[..., i, j] = _apply_1d(self.xyz[i], D, NODE_AXIS[j])
        self.jac = J
        self.det = np.linalg.det(J)
        if np.any(self.det <= 0):
            raise ValueError("the element maps are not orientation preserving")
        self.inv = np.linalg.inv(J)  # inv[..., j, i] = d xi^j / d x^i

    @property
    def ndof(self):
        return self.box.ndof


def deformed_box(box: BoxMesh, amplitude, direction=(1.0, 0.7, 0.4)):
    """Node coordinates of the box map x = X + amplitude * c * prod_d sin(pi (X_d - lo_d) / L_d),
    which keeps the box boundary in place: shape (3, E, N, N, N)."""
    X = np.stack(box.node_coordinates())
    L = box.upper - box.lower
    bump = np.ones_like(X[0])
    for d in range(3):
        bump = bump * np.sin(np.pi * (X[d] - box.lower[d]) / L[d])
    return X + amplitude * np.asarray(direction, float)[:, None, None, None, None] * bump[None]


def mass_diagonal(cm: CurvedMesh):
    """Diagonal of M (eq. massmat): J w_i w_j w_k at every node, shape (E, N, N, N)."""
    w = lgl.weights(cm.box.N)
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    return cm.det * W[None]


def apply_mass(cm: CurvedMesh, f):
    return np.asarray(f, float).reshape(cm.det.shape) * mass_diagonal(cm)


def _face_index(N, d, idx):
    """Index tuple into an (N, N, N) node block [k, j, i] fixing dimension d."""
    sl = [slice(None)] * 3
    sl[3 + NODE_AXIS[d]] = idx
    return tuple(sl)


def apply_operator(cm: CurvedMesh, u, C, diag=None, dirichlet_values=None):
    """A u for nodal values u (E * N^3), with the optional pointwise term
    diag * u (a massive diagonal, as the linearised operators use).
    ``dirichlet_values`` (nodal, read at Dirichlet boundary nodes) gives
    inhomogeneous boundary data u_b (eq. bc); the default is u_b = 0."""
    box = cm.box
    N, E = box.N, box.E
    D = lgl.diff_matrix(N)
    w = lgl.weights(N)
    W3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
    u = np.asarray(u, float).reshape(E, N, N, N)
    ub = None if dirichlet_values is None else np.asarray(dirichlet_values, float).reshape(E, N, N, N)
    inv = cm.inv
    du = [_apply_1d(u, D, NODE_AXIS[j]) for j in range(3)]
    # unlifted physical gradient g_i = invJ^j_i D^xi_j u
    g = [sum(inv[..., j, i] * du[j] for j in range(3)) for i in range(3)]

    faces = []
    v = [gi.copy() for gi in g]
    for e in range(E):
        for d in range(3):
            for s in (-1, +1):
                own = 0 if s < 0 else N - 1
                fi = (e,) + _face_index(N, d, own)
                invd = inv[fi][..., d, :]  # (N, N, 3): d xi^d / d x^i
                nrm = np.linalg.norm(invd, axis=-1)
                n = s * invd / nrm[..., None]
                u_int = u[fi]
                g_int = np.stack([g[i][fi] for i in range(3)], axis=-1)
                ndu_int = np.sum(n * g_int, axis=-1)
                nb = box.neighbor(e, d, s)
                if nb is not None:
                    fo = (nb,) + _face_index(N, d, N - 1 if s < 0 else 0)
                    u_ext = u[fo]
                    g_ext = np.stack([g[i][fo] for i in range(3)], axis=-1)
                    ndu_ext = np.sum(n * g_ext, axis=-1)
                    nrm_ext = np.linalg.norm(inv[fo][..., d, :], axis=-1)
                elif 2 * d + (s > 0) in box.neumann:
                    u_ext, ndu_ext, nrm_ext = u_int, -ndu_int, nrm
                else:
                    u_b = 0.0 if ub is None else ub[fi]
                    u_ext, ndu_ext, nrm_ext = 2.0 * u_b - u_int, ndu_int, nrm
                # auxiliary lift, eq. dg_op_auxvars: L (1/2 n (u_ext - u_int))
                lift = (nrm / w[own]) * 0.5 * (u_ext - u_int)
                for i in range(3):
                    v[i][fi] += lift * n[..., i]
                h = np.minimum(2.0 / nrm, 2.0 / nrm_ext)
                sigma = C * N ** 2 / h
                ML = cm.det[fi] * nrm * W3[_face_index(N, d, own)] / w[own]
                faces.append((fi, n, u_int, u_ext, ndu_int, ndu_ext, sigma, ML))

    # primal equation, eq. dg_op_primal: -M D_i v_i
    div = np.zeros_like(u)
    for i in range(3):
        for j in range(3):
            div += inv[..., j, i] * _apply_1d(v[i], D, NODE_AXIS[j])
    Au = -mass_diagonal(cm) * div
    for fi, n, u_int, u_ext, ndu_int, ndu_ext, sigma, ML in faces:
        flux_star = 0.5 * (ndu_int + ndu_ext) - sigma * (u_int - u_ext)
        flux_int = sum(n[..., i] * v[i][fi] for i in range(3))
        Au[fi] -= ML * (flux_star - flux_int)
    if diag is not None:
        Au += np.asarray(diag, float).reshape(E, N, N, N) * u
    return Au.reshape(-1)


def metric_source(cm: CurvedMesh, sqrtg):
    """The contraction of the Christoffel symbols Gamma^i_ik = d_k ln sqrt(g)
    of the background metric at every node, (3, E, N, N, N): the collocation
    derivative of the interpolant of sqrt(g), divided by sqrt(g).

    Reading: the paper does not say how derivatives of background fields are
    formed; they are taken here like those of the solution."""
    N = cm.box.N
    D = lgl.diff_matrix(N)
    sg = np.asarray(sqrtg, float).reshape(cm.det.shape)
    ds = [_apply_1d(sg, D, NODE_AXIS[j]) for j in range(3)]
    return np.stack([sum(cm.inv[..., j, i] * ds[j] for j in range(3)) / sg for i in range(3)])


def apply_operator_metric(cm: CurvedMesh, u, C, ginv, sqrtg, dirichlet_values=None):
    """A u on a curved background metric g_ij (Sec. II: sqrt(g) in eqs.
    massmat, stiffmat and liftop), for the Poisson equation
    -nabla_i (g^ij d_j u) = f in the flux form of the paper: F_v = u delta,
    F_u^i = g^ij v_j, S_u = -Gamma^i_ik F_u^k.  ginv is g^ij at the nodes,
    shape (3, 3, E, N, N, N); sqrtg the metric determinant's root.

    Under LGL quadrature sqrt(g) J cancels between M and MD, so D_i is the
    collocation derivative as for the flat metric; M = sqrt(g) J w_i w_j w_k.
    On a face normal to xi^d the unit normal one-form is
    n_i = s invJ^d_i / |invJ^d|_g with |a|_g = sqrt(g^ij a_i a_j), the
    surface element sqrt(g) J |invJ^d|_g (so L = |invJ^d|_g / w_end), and h
    in eq. penalty is 2 / |invJ^d|_g on each side.  The fluxes of eq. numflux
    take n_i F_u^i of each side's own unlifted gradient."""
    box = cm.box
    N, E = box.N, box.E
    D = lgl.diff_matrix(N)
    w = lgl.weights(N)
    W3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
    u = np.asarray(u, float).reshape(E, N, N, N)
    ub = None if dirichlet_values is None else np.asarray(dirichlet_values, float).reshape(E, N, N, N)
    G = np.asarray(ginv, float).reshape((3, 3) + cm.det.shape)
    sg = np.asarray(sqrtg, float).reshape(cm.det.shape)
    gam = metric_source(cm, sg)
    inv = cm.inv
    du = [_apply_1d(u, D, NODE_AXIS[j]) for j in range(3)]
    g = [sum(inv[..., j, i] * du[j] for j in range(3)) for i in range(3)]  # d_i u
    F = [sum(G[i, j] * g[j] for j in range(3)) for i in range(3)]  # g^ij d_j u

    def gnorm(a, at):
        # |a|_g at the face nodes `at`, a of shape (..., 3)
        return np.sqrt(sum(G[i, j][at] * a[..., i] * a[..., j] for i in range(3) for j in range(3)))

    faces = []
    v = [gi.copy() for gi in g]
    for e in range(E):
        for d in range(3):
            for s in (-1, +1):
                own = 0 if s < 0 else N - 1
                fi = (e,) + _face_index(N, d, own)
                invd = inv[fi][..., d, :]
                nrm = gnorm(invd, fi)
                n = s * invd / nrm[..., None]
                u_int = u[fi]
                ndu_int = sum(n[..., i] * F[i][fi] for i in range(3))
                nb = box.neighbor(e, d, s)
                if nb is not None:
                    fo = (nb,) + _face_index(N, d, N - 1 if s < 0 else 0)
                    u_ext = u[fo]
                    ndu_ext = sum(n[..., i] * F[i][fo] for i in range(3))
                    nrm_ext = gnorm(inv[fo][..., d, :], fo)
                elif 2 * d + (s > 0) in box.neumann:
                    u_ext, ndu_ext, nrm_ext = u_int, -ndu_int, nrm
                else:
                    u_b = 0.0 if ub is None else ub[fi]
                    u_ext, ndu_ext, nrm_ext = 2.0 * u_b - u_int, ndu_int, nrm
                lift = (nrm / w[own]) * 0.5 * (u_ext - u_int)
                for i in range(3):
                    v[i][fi] += lift * n[..., i]
                sigma = C * N ** 2 / np.minimum(2.0 / nrm, 2.0 / nrm_ext)
                ML = sg[fi] * cm.det[fi] * nrm * W3[_face_index(N, d, own)] / w[own]
                faces.append((fi, n, u_int, u_ext, ndu_int, ndu_ext, sigma, ML))

    Fv = [sum(G[i, j] * v[j] for j in range(3)) for i in range(3)]  # F_u^i of the lifted v
    div = np.zeros_like(u)
    for i in range(3):
        for j in range(3):
            div += inv[..., j, i] * _apply_1d(Fv[i], D, NODE_AXIS[j])
    M = sg * mass_diagonal(cm)
    src = -sum(gam[i] * Fv[i] for i in range(3))  # S_u = -Gamma^i_ik F_u^k
    Au = -M * div + M * src
    for fi, n, u_int, u_ext, ndu_int, ndu_ext, sigma, ML in faces:
        flux_star = 0.5 * (ndu_int + ndu_ext) - sigma * (u_int - u_ext)
        flux_int = sum(n[..., i] * Fv[i][fi] for i in range(3))
        Au[fi] -= ML * (flux_star - flux_int)
    return Au.reshape(-1)


def assemble(cm: CurvedMesh, C):
    n = cm.ndof
    A = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = apply_operator(cm, e, C)
    return A
