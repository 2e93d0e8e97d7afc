"""Linear elliptic systems of several variables, and the Schwarz subdomain
solver with the Laplacian-approximation preconditioner whose boundary
conditions match each variable's (Sec. III.E.1, eq. lapl_approx).

Test infrastructure only: imported by tests and the benchmark's CPU leg,
never by the product path.

System.  V variables u_A share one box grid.  Variable A has its own set of
box faces with homogeneous Neumann conditions (Dirichlet elsewhere), and

    (A_sys u)_A = A^(A) u_A + sum_B D_AB u_B,

with A^(A) the DG Poisson operator under variable A's boundary conditions
(Sec. II) and D_AB pointwise couplings as they enter the discrete operator
(for a PDE term c_AB u_B: D_AB = M c_AB with the lumped mass), the structure
of the linearised equations of a coupled nonlinear system (eq. linearized),
e.g. the five XCTS variables of Sec. IV.B.

Smoother.  Additive Schwarz (Sec. III.D) on the system: the subdomain
problem A_S,sys du_S = r_S, with A_S,sys = blockdiag_A(A_S^(A)) + D_S over the
V stacked subdomain vectors, is solved by k iterations of right-preconditioned
GMRES (Sec. III.E.1).  The preconditioner is the Laplacian approximation:
independent Poisson subdomain solves, one per variable, by explicit inverses
(Sec. III.E.2).  "matched": variable A's Poisson operator carries A's
boundary-condition type on the subdomain's external faces, so a subdomain
with only internal faces has one Poisson operator for all variables and a
boundary subdomain one per distinct type among the variables; "dirichlet":
every variable takes the Dirichlet one (the naive approximation the paper
compares with).  k = 0 applies the approximation alone.

Multigrid (Sec. III.C): every level coarsens all variables alike; the coarse
couplings are D_{l+1,AB} = R D_{l,AB}, the reading the scalar linearised
cycle takes for its pointwise term.

Readings:
* the subdomain vector stacks the V variables' subdomain vectors, variable 0
  first, each in the scalar layout; GMRES takes the Euclidean inner product
  over the whole stacked vector.
* the Schwarz weights and the subdomain geometry do not depend on the
  boundary-condition type, so every variable uses the same ones.
"""
from __future__ import annotations

import numpy as np

from .mesh import BoxMesh
from .multigrid import hierarchy, prolongate, restrict
from .operator import apply_operator
from .schwarz import (SchwarzSmoother, element_class, gmres_fixed, subdomain_layout,
                      subdomain_weights)


class SystemOperator:
    """A_sys on one grid; ``neumann_sets[A]`` lists variable A's Neumann faces
    (f = 2 d + side)."""

    def __init__(self, lower, upper, elements, p, neumann_sets, C=1.5):
        self.V = len(neumann_sets)
        self.meshes = [BoxMesh(lower, upper, elements, p, neumann=ns) for ns in neumann_sets]
        self.mesh = self.meshes[0]
        self.C = C

    @property
    def ndof(self):
        return self.mesh.ndof

    def apply(self, u, D=None):
        """A_sys u for u of shape (V, ndof); D of shape (V, V, ndof) or None."""
        m = self.mesh
        N = m.N
        u = np.asarray(u, float).reshape(self.V, m.ndof)
        out = np.stack([apply_operator(self.meshes[a], u[a].reshape(m.E, N, N, N), self.C).reshape(-1)
                        for a in range(self.V)])
        if D is not None:
            out = out + np.einsum("abn,bn->an", D, u)
        return out


class SystemSchwarzSmoother:
    """Additive Schwarz steps on A_sys u = b (one grid)."""

    def __init__(self, meshes, C, D, overlap=2, subdomain_iters=3, laplacian_bc="matched"):
        if laplacian_bc not in ("matched", "dirichlet"):
            raise ValueError(laplacian_bc)
        self.meshes, self.C, self.overlap = meshes, C, overlap
        self.V = len(meshes)
        m = meshes[0]
        self.mesh = m
        self.D = np.asarray(D, float).reshape(self.V, self.V, m.ndof)
        self.k = subdomain_iters
        self.layout = [subdomain_layout(m, e, overlap)[0] for e in range(m.E)]
        self.weights = [subdomain_weights(m, e, overlap) for e in range(m.E)]
        self.cls = [element_class(m, e) for e in range(m.E)]
        # true subdomain operators A_S^(A), one scalar smoother per variable
        self.scalar = [SchwarzSmoother(mv, C, overlap) for mv in meshes]
        if laplacian_bc == "matched":
            self.Minv = [sm.A_S_inv for sm in self.scalar]
        else:
            dirichlet = SchwarzSmoother(BoxMesh(m.lower, m.upper, m.n, m.p), C, overlap)
            self.Minv = [dirichlet.A_S_inv] * self.V

    def apply(self, u):
        m = self.mesh
        N = m.N
        u = np.asarray(u, float).reshape(self.V, m.ndof)
        out = np.stack([apply_operator(self.meshes[a], u[a].reshape(m.E, N, N, N), self.C).reshape(-1)
                        for a in range(self.V)])
        return out + np.einsum("abn,bn->an", self.D, u)

    def subdomain_solve(self, e, rS):
        """du_S for subdomain e from its stacked residual rS (V * n_S)."""
        V, key, idx = self.V, self.cls[e], self.layout[e]
        n = len(idx)
        r = rS.reshape(V, n)
        if self.k == 0:
            return np.concatenate([self.Minv[a][key] @ r[a] for a in range(V)])
        A_blocks = [self.scalar[a].A_S[key] for a in range(V)]
        DS = self.D[:, :, idx]

        def apply_sys(x):
            x = x.reshape(V, n)
            return np.concatenate([A_blocks[a] @ x[a] + (DS[a] * x).sum(axis=0) for a in range(V)])

        def apply_M(x):
            x = x.reshape(V, n)
            return np.concatenate([self.Minv[a][key] @ x[a] for a in range(V)])

        return gmres_fixed(apply_sys, apply_M, rS, self.k)

    def correction(self, r):
        """sum_S R_S^T (w_S du_S), variable by variable."""
        V = self.V
        r = np.asarray(r, float).reshape(V, self.mesh.ndof)
        du = np.zeros_like(r)
        for e in range(self.mesh.E):
            idx = self.layout[e]
            dS = self.subdomain_solve(e, r[:, idx].reshape(-1)).reshape(V, len(idx))
            for a in range(V):
                np.add.at(du[a], idx, self.weights[e] * dS[a])
        return du

    def smooth(self, u, b, steps):
        u = np.array(u, dtype=float).reshape(self.V, self.mesh.ndof)
        b = np.asarray(b, float).reshape(self.V, self.mesh.ndof)
        for _ in range(steps):
            u = u + self.correction(b - self.apply(u))
        return u


class SystemVCycle:
    """One multigrid V-cycle (Sec. III.C.3) on the system, ``pre``/``post``
    Schwarz steps per level, pre + post on the coarsest; input and output are
    flat stacked vectors (V * ndof)."""

    def __init__(self, sysop: SystemOperator, D, levels=2, overlap=2, pre=3, post=3,
                 subdomain_iters=3, laplacian_bc="matched"):
        self.V = sysop.V
        self.pre, self.post = pre, post
        hier = [hierarchy(m, levels) for m in sysop.meshes]
        self.levels = []
        D = np.asarray(D, float).reshape(self.V, self.V, sysop.ndof)
        for li in range(len(hier[0])):
            meshes = [h[li][0] for h in hier]
            split = hier[0][li][1]
            sm = SystemSchwarzSmoother(meshes, sysop.C, D, overlap, subdomain_iters, laplacian_bc)
            self.levels.append((meshes[0], split, sm))
            if split is not None:
                coarse = hier[0][li + 1][0]
                D = np.stack([np.stack([restrict(meshes[0], coarse, split, D[a, b])
                                        for b in range(self.V)]) for a in range(self.V)])

    def __call__(self, b):
        return self._cycle(0, np.asarray(b, float).reshape(self.V, -1)).reshape(-1)

    def _cycle(self, l, b):
        mesh, split, sm = self.levels[l]
        u = sm.smooth(np.zeros_like(b), b, self.pre)
        if split is None:
            return sm.smooth(u, b, self.post)
        coarse = self.levels[l + 1][0]
        r = b - sm.apply(u)
        bc = np.stack([restrict(mesh, coarse, split, r[a]) for a in range(self.V)])
        uc = self._cycle(l + 1, bc)
        u = u + np.stack([prolongate(mesh, coarse, split, uc[a]) for a in range(self.V)])
        return sm.smooth(u, b, self.post)
