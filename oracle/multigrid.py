"""Geometric multigrid V-cycle with Schwarz smoothing (Sec. III.C).

Test infrastructure only: imported by the tests, smoke() and the benchmark's
CPU leg, never by the product path.

* hierarchy (Sec. III.C.1, Fig. mg_hierarchy): level l+1 merges two elements
  into one along every dimension; all elements share one degree p here.
* prolongation (eq. prol): Lagrange interpolation from the parent to the child
  points, whose parent-logical coordinates are (xi-1)/2 or (xi+1)/2 in a
  dimension that is split and xi in a dimension that is not.
* restriction R = P^T with no mass matrices, since it acts on DG residuals that
  already carry them (Sec. III.C.2).
* V-cycle (Sec. III.C.3, eqs. mg_problem, mg_res): presmooth on A_l u_l = b_l,
  restrict the residual b_{l+1} = R r_l, recurse; on the coarsest grid pre- and
  post-smooth; prolongate the correction u_l += P u_{l+1}; postsmooth.
  Coarse operators are the DG discretisation on the coarse grid.

Readings:
* a dimension is split only while its element count is even and greater than
  one; the number of levels is capped by the caller's ``levels`` and by this
  rule.
* the V-cycle starts from u = 0 on every level (it is used once per outer
  iteration as a preconditioner).
* for an operator with a pointwise term diag(d) (the linearised nonlinear
  problem), the coarse term is the restriction d_{l+1} = R d_l of the massive
  diagonal, a row-sum (lumped) Galerkin coarse version of M c, since the
  interpolation reproduces constants.
"""
from __future__ import annotations

import numpy as np

from . import lgl
from .mesh import BoxMesh
from .schwarz import SchwarzSmoother


def coarsen(mesh: BoxMesh):
    """Coarse mesh and the per-dimension split flags, or None if no dimension
    can be merged."""
    split = [mesh.n[d] > 1 and mesh.n[d] % 2 == 0 for d in range(3)]
    if not any(split):
        return None
    n = [mesh.n[d] // 2 if split[d] else mesh.n[d] for d in range(3)]
    return BoxMesh(mesh.lower, mesh.upper, n, mesh.p, neumann=mesh.neumann), split


def hierarchy(mesh: BoxMesh, levels):
    """List of (mesh, split-to-next) from fine to coarse."""
    out = []
    m = mesh
    for _ in range(levels - 1):
        c = coarsen(m)
        if c is None:
            break
        out.append((m, c[1]))
        m = c[0]
    out.append((m, None))
    return out


def _child_matrices(N, split):
    P_lo, P_hi = lgl.child_interpolation(N)
    I = np.eye(N)
    return [(P_lo, P_hi) if split[d] else (I, I) for d in range(3)]


def prolongate(fine: BoxMesh, coarse: BoxMesh, split, uc):
    """u_f = P u_c: each fine element interpolates its parent (eq. prol)."""
    N = fine.N
    mats = _child_matrices(N, split)
    uc = np.asarray(uc, float).reshape(coarse.E, N, N, N)
    uf = np.zeros((fine.E, N, N, N))
    for e in range(fine.E):
        c = fine.elem_coords(e)
        parent = coarse.elem_index(*[c[d] // 2 if split[d] else c[d] for d in range(3)])
        Px = mats[0][c[0] % 2 if split[0] else 0]
        Py = mats[1][c[1] % 2 if split[1] else 0]
        Pz = mats[2][c[2] % 2 if split[2] else 0]
        # out[k,j,i] = sum Pz[k,c] Py[j,b] Px[i,a] u[c,b,a]
        uf[e] = np.einsum('kc,jb,ia,cba->kji', Pz, Py, Px, uc[parent])
    return uf.reshape(-1)


def restrict(fine: BoxMesh, coarse: BoxMesh, split, rf):
    """b_c = P^T r_f (transpose of ``prolongate``)."""
    N = fine.N
    mats = _child_matrices(N, split)
    rf = np.asarray(rf, float).reshape(fine.E, N, N, N)
    bc = np.zeros((coarse.E, N, N, N))
    for e in range(fine.E):
        c = fine.elem_coords(e)
        parent = coarse.elem_index(*[c[d] // 2 if split[d] else c[d] for d in range(3)])
        Px = mats[0][c[0] % 2 if split[0] else 0]
        Py = mats[1][c[1] % 2 if split[1] else 0]
        Pz = mats[2][c[2] % 2 if split[2] else 0]
        bc[parent] += np.einsum('kc,jb,ia,kji->cba', Pz, Py, Px, rf[e])
    return bc.reshape(-1)


class VCycle:
    """One multigrid cycle with ``pre``/``post`` Schwarz steps per level
    (Sec. III.C.3).  ``gamma`` is the number of visits of each coarser level
    per visit of its parent: 1 is the paper's V-cycle, 2 the W-cycle, whose
    second visit starts from the first one's coarse-grid result.  gamma="F"
    is the F-cycle (Sec. V names it): an F-visit of the coarser level followed
    by a V-visit from its result."""

    def __init__(self, mesh: BoxMesh, C, levels=2, overlap=2, pre=3, post=3,
                 diag=None, subdomain_iters=0, gamma=1, on_level=None):
        self.levels = hierarchy(mesh, levels)
        self.pre, self.post = pre, post
        self.gamma = gamma
        self.smoothers = []
        d = None if diag is None else np.asarray(diag, float).reshape(-1)
        for li, (m, split) in enumerate(self.levels):
            self.smoothers.append(SchwarzSmoother(m, C, overlap, diag=d,
                                                  subdomain_iters=subdomain_iters))
            if on_level is not None:  # progress report of a long set-up
                on_level(li, m)
            if split is not None and d is not None:
                d = restrict(m, self.levels[li + 1][0], split, d)

    def __call__(self, b):
        return self._cycle(0, np.asarray(b, float).reshape(-1), None, self.gamma)

    def _cycle(self, l, b, u0, kind):
        mesh, split = self.levels[l]
        sm = self.smoothers[l]
        u = np.zeros_like(b) if u0 is None else u0
        u = sm.smooth(u, b, self.pre)  # presmoothing
        if split is None:  # coarsest grid: pre- and post-smoothing
            return sm.smooth(u, b, self.post)
        coarse = self.levels[l + 1][0]
        r = b - sm.apply(u)  # eq. mg_res
        bc = restrict(mesh, coarse, split, r)
        visits = {1: [1], 2: [2, 2], "F": ["F", 1]}[kind]
        uc = None
        for k in visits:
            uc = self._cycle(l + 1, bc, uc, k)
        u = u + prolongate(mesh, coarse, split, uc)
        return sm.smooth(u, b, self.post)  # postsmoothing


class AdditiveMG:
    """Additive multigrid, the variant Sec. V names: the residual is restricted
    to every level, each level smooths its restriction independently from
    zero, and the prolongated corrections of all levels are summed.

    Reading: every level runs pre + post Schwarz steps (the smoothing count the
    V-cycle gives its coarsest level); with a linearised operator the coarse
    levels carry the restricted diagonal as in VCycle."""

    def __init__(self, mesh: BoxMesh, C, levels=2, overlap=2, pre=3, post=3,
                 diag=None, subdomain_iters=0):
        self.levels = hierarchy(mesh, levels)
        self.steps = pre + post
        self.smoothers = []
        d = None if diag is None else np.asarray(diag, float).reshape(-1)
        for li, (m, split) in enumerate(self.levels):
            self.smoothers.append(SchwarzSmoother(m, C, overlap, diag=d,
                                                  subdomain_iters=subdomain_iters))
            if split is not None and d is not None:
                d = restrict(m, self.levels[li + 1][0], split, d)

    def __call__(self, r):
        b = [np.asarray(r, float).reshape(-1)]
        for li in range(len(self.levels) - 1):
            m, split = self.levels[li]
            b.append(restrict(m, self.levels[li + 1][0], split, b[-1]))
        z = None
        for li in reversed(range(len(self.levels))):
            u = self.smoothers[li].smooth(np.zeros_like(b[li]), b[li], self.steps)
            if z is not None:
                m, split = self.levels[li]
                u = u + prolongate(m, self.levels[li + 1][0], split, z)
            z = u
        return z
