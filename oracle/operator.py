"""Strong DG operator of the Poisson equation in first-order flux form.

Test infrastructure only: imported by the tests, smoke() and the benchmark's
CPU leg, never by the product path.

Follows Sec. II literally:

* Poisson fluxes (eq. poisson_fluxform): F_v^i_j = u delta^i_j, S_v = v
  (so S~_v = 0), F_u^i = v_i, S_u = 0 for the linear operator.
* auxiliary equation (eq. dg_op_auxvars):
      v_j = D_j u + L ((n_i F_v^i_j)* - n_j u)
* primal equation (eq. dg_op_primal), whose left-hand side is A u:
      A u = -MD_i v_i - ML ((n_i F_u^i)* - n_i v_i) + M S_u
* mass, stiffness and lifting matrices (eqs. massmat, stiffmat, liftop) with
  D = M^-1 MD, L = M^-1 ML.
* generalised internal-penalty flux (eq. numflux) with n_ext = -n_int:
      (n F_v)*_j = 1/2 n_j (u_int + u_ext)
      (n F_u)*   = 1/2 n.(grad u_int + grad u_ext) - sigma (u_int - u_ext)
  where grad u is the derivative of each side's own polynomial (the primal
  flux takes the divergence of the auxiliary flux, not the lifted v).
* penalty (eq. penalty): sigma = C (max(p_int, p_ext) + 1)^2 / min(h_int, h_ext).
* boundary conditions through ghost fluxes (eq. bc):
      (n F)_ext = (n F)_int - 2 (n F)_b
  Dirichlet: the auxiliary boundary flux is n u_b and the primal boundary flux
  equals the interior one, i.e. u_ext = 2 u_b - u_int and the exterior normal
  derivative equals the interior one.  Homogeneous Neumann (the faces listed
  in mesh.neumann): the primal boundary flux is 0 and the auxiliary one equals
  the interior one, i.e. u_ext = u_int and the exterior normal derivative is
  the negated interior one.

Readings (where the paper leaves a choice):
* The integrals in eqs. massmat/stiffmat/liftop are evaluated with LGL
  quadrature on the element's own points, so M = J w_i w_j w_k is diagonal and
  ML is diagonal on each face with weight J_F w_a w_b (J_F the surface
  Jacobian).  D_i is then the collocation derivative (2/h_i) D_xi.
* h in the penalty is the element's full width normal to the face; p is the
  polynomial degree, so (p+1)^2 = N^2.  Homogeneous Dirichlet data u_b = 0.
"""
from __future__ import annotations

import numpy as np

from . import lgl
from .mesh import BoxMesh, NODE_AXIS, GRID_ELEM_AXIS


def _apply_1d(a, D, axis):
    """(D a) along the given axis: out_i = sum_m D[i, m] a_m."""
    a = np.moveaxis(a, axis, -1)
    return np.moveaxis(a @ D.T, -1, axis)


def _face_slice(ndim, axis, idx):
    sl = [slice(None)] * ndim
    sl[axis] = slice(idx, idx + 1)
    return tuple(sl)


def _from_neighbor(face_arr, d, s, n_d):
    """out[..., c_d, ...] = face_arr[..., c_d + s, ...] along element axis d of
    a grid view; entries without a neighbour are left at zero."""
    ax = GRID_ELEM_AXIS[d]
    a = np.moveaxis(face_arr, ax, 0)
    out = np.zeros_like(a)
    if n_d > 1:
        if s > 0:
            out[:-1] = a[1:]
        else:
            out[1:] = a[:-1]
    return np.moveaxis(out, 0, ax)


def _boundary_mask(mesh: BoxMesh, d, s, ndim):
    shape = [1] * ndim
    ax = GRID_ELEM_AXIS[d] + ndim
    shape[ax] = mesh.n[d]
    m = np.zeros(mesh.n[d], dtype=bool)
    m[-1 if s > 0 else 0] = True
    return m.reshape(shape)


def mass_diagonal(mesh: BoxMesh):
    """Diagonal of M (eq. massmat under LGL quadrature): J w_i w_j w_k."""
    w = lgl.weights(mesh.N)
    J = np.prod(mesh.h) / 8.0
    W = w[:, None, None] * w[None, :, None] * w[None, None, :]
    return J * W  # (N, N, N) indexed [k, j, i]


def face_mass(mesh: BoxMesh, d):
    """Diagonal of ML on a face normal to d (eq. liftop under LGL quadrature):
    surface Jacobian times the two transverse weights, shaped to broadcast
    against a face slice (N along the two transverse node axes, 1 along d)."""
    w = lgl.weights(mesh.N)
    JF = np.prod([mesh.h[t] / 2.0 for t in range(3) if t != d])
    shape = [mesh.N, mesh.N, mesh.N]
    W = np.ones(shape)
    for t in range(3):
        if t == d:
            continue
        sh = [1, 1, 1]
        sh[NODE_AXIS[t] + 3] = mesh.N
        W = W * w.reshape(sh)
    sl = [slice(None)] * 3
    sl[NODE_AXIS[d] + 3] = slice(0, 1)
    return JF * W[tuple(sl)]


def penalty(mesh: BoxMesh, C, d):
    """sigma = C (p + 1)^2 / h_d for equal p and h on both sides (eq. penalty)."""
    return C * (mesh.p + 1) ** 2 / mesh.h[d]


def apply_operator(mesh: BoxMesh, u, C, source=None, dirichlet_u_b=0.0):
    """A u for nodal values u of shape (..., E, N, N, N).

    ``source`` optionally adds the pointwise term M S_u (an array of S_u at the
    nodes, same shape as u).  ``dirichlet_u_b`` is the boundary value u_b.
    """
    N = mesh.N
    D = lgl.diff_matrix(N)
    Mdiag = mass_diagonal(mesh)
    ug = mesh.grid(np.asarray(u, dtype=float))
    nd = ug.ndim
    lo, hi = 0, N - 1

    # unlifted derivatives  D_j u = (2/h_j) D_xi u   (D = M^-1 MD)
    g = [(2.0 / mesh.h[d]) * _apply_1d(ug, D, NODE_AXIS[d]) for d in range(3)]

    # face data: interior/exterior value and normal derivative for every face
    faces = {}
    for d in range(3):
        for s in (-1, +1):
            own = lo if s < 0 else hi
            other = hi if s < 0 else lo
            sl_own = _face_slice(nd, NODE_AXIS[d], own)
            sl_oth = _face_slice(nd, NODE_AXIS[d], other)
            u_int = ug[sl_own]
            du_int = g[d][sl_own]  # d u / d x_d on own face
            u_ext = _from_neighbor(ug[sl_oth], d, s, mesh.n[d])
            du_ext = _from_neighbor(g[d][sl_oth], d, s, mesh.n[d])
            bmask = _boundary_mask(mesh, d, s, nd)
            if 2 * d + (s > 0) in mesh.neumann:
                # eq. bc, homogeneous Neumann: the primal boundary flux is 0
                # and the auxiliary one equals the interior flux, i.e.
                # u_ext = u_int and an exterior normal derivative of -du_int
                u_ext = np.where(bmask, u_int, u_ext)
                du_ext = np.where(bmask, -du_int, du_ext)
            else:
                # eq. bc, Dirichlet: u_ext = 2 u_b - u_int, exterior derivative = interior
                u_ext = np.where(bmask, 2.0 * dirichlet_u_b - u_int, u_ext)
                du_ext = np.where(bmask, du_int, du_ext)
            faces[(d, s)] = (sl_own, u_int, u_ext, du_int, du_ext)

    # auxiliary variables, eq. dg_op_auxvars with eq. numfluxaux
    v = []
    for d in range(3):
        lift = np.zeros_like(ug)
        MLf = face_mass(mesh, d)
        for s in (-1, +1):
            sl_own, u_int, u_ext, _, _ = faces[(d, s)]
            n_d = float(s)
            flux_star = 0.5 * (n_d * u_int + n_d * u_ext)  # (n_i F_v^i_d)*
            flux_int = n_d * u_int  # n_i F_v^i_d
            lift[sl_own] += MLf * (flux_star - flux_int)
        v.append(g[d] + lift / Mdiag)  # D u + M^-1 ML (...)

    # primal equation, eq. dg_op_primal with eqs. numfluxprimal, penalty
    Au = np.zeros_like(ug)
    for d in range(3):
        Au -= Mdiag * (2.0 / mesh.h[d]) * _apply_1d(v[d], D, NODE_AXIS[d])  # -MD_d v_d
    for d in range(3):
        MLf = face_mass(mesh, d)
        sigma = penalty(mesh, C, d)
        for s in (-1, +1):
            sl_own, u_int, u_ext, du_int, du_ext = faces[(d, s)]
            n_d = float(s)
            flux_star = 0.5 * (n_d * du_int + n_d * du_ext) - sigma * (u_int - u_ext)
            flux_int = n_d * v[d][sl_own]  # n_i F_u^i = n_i v_i (lifted v)
            Au[sl_own] -= MLf * (flux_star - flux_int)
    if source is not None:
        Au += Mdiag * mesh.grid(np.asarray(source, dtype=float))
    return mesh.flat(Au)


def apply_mass(mesh: BoxMesh, f):
    """b = M f (right-hand side of eq. dg_op_primal)."""
    f = np.asarray(f, dtype=float)
    return f * mass_diagonal(mesh)


def assemble(mesh: BoxMesh, C):
    """Dense matrix of A by applying it to every unit vector (tiny grids only)."""
    n = mesh.ndof
    N = mesh.N
    I = np.eye(n).reshape(n, mesh.E, N, N, N)
    cols = apply_operator(mesh, I, C).reshape(n, n)
    return cols.T.copy()  # column j is A e_j
