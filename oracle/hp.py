"""DG Poisson operator, Schwarz smoother and multigrid on hp-nonuniform meshes
(Sec. II blocks and elements, Sec. III.C.1 coarsening, Sec. III.D subdomains).

Test infrastructure only: imported by tests and the benchmark's CPU leg,
never by the product path.

Mesh (Sec. II): the box [lower, upper] is a grid of equal blocks.  Block b is
split 2^L_b,d times along dimension d (its refinement levels; uniform within
the block, free from block to block), and every element carries its own
polynomial degree per dimension (anisotropic p).  Across block boundaries an
element face meets one coarser, one equal or several finer neighbours; the
levels of two face neighbours differ by at most one in each dimension along
the face (two-to-one balance).  Elements are numbered block by block (block
index x fastest), x fastest inside a block; element e holds
Nz x Ny x Nx nodes in [k, j, i] order at offset offsets[e].

Mortars (the faces of Fig. subdomain_structure): a face shared by elements e
and f carries a mortar for each overlapping pair, covering their common part
of the face with max(N_e, N_f) LGL points per face dimension.  Readings (the
paper defers mortar details to its companion DG paper):
* each side's trace and normal derivative are interpolated to the mortar
  points (Lagrange interpolation, exact for the side's own polynomials);
* the fluxes of eq. numflux are evaluated on the mortar, with the penalty of
  eq. penalty from the degrees normal to the face and the element widths
  normal to the face (h = min over both sides, p = max);
* the results are brought back to each element face by the exact L2
  projection onto the face's polynomials (exact mass matrices, Gauss
  quadrature), which is the identity on a conforming face of equal degrees and
  leaves the element's own data unchanged, then lifted with the element's
  LGL face mass as on conforming faces (eq. liftop).
The operator is the strong form of ``operator.py`` elsewhere.  On
nonconforming faces the lumped element mass against the exact projection
makes the operator slightly non-symmetric; its symmetric part stays positive
definite (checked by the tests).

Schwarz subdomains (Sec. III.D.1) extend N_ov points into every face
neighbour, all of a finer face's neighbours included, with N_ov capped at the
neighbour's points normal to the face minus one.  Weights (eqs.
schwarz_weighting, schwarz_weight_prod, schwarz_weight_function): a point's
shares are taken from its own element's weight functions a_d (eq.
schwarz_weight_function with that element's points and overlap), so that they
sum to one at every point: its own subdomain gets prod_d a_d, and the rest
1 - a_d = (low part) + (high part), split by side, goes to the subdomains of
the face neighbours on that side, with the edge and corner shares spread as
on uniform grids (the transverse factor T of ``schwarz.py``) and divided
equally among several neighbours across one face.  On uniform grids these are
exactly the weights of ``schwarz.py``.

Multigrid (Sec. III.C.1): each coarser level halves every block's element
count along each dimension whose level is positive (so coarsening stays inside
blocks), and a merged element takes, per dimension, the smallest degree of its
children.  Prolongation interpolates the parent's polynomial at the child's
points (eq. prol), restriction is its transpose (Sec. III.C.2), and coarse
operators are the DG discretisation on the coarse mesh.
"""
from __future__ import annotations

import functools

import numpy as np
from numpy.polynomial import legendre as Leg

from . import lgl
from .schwarz import smoothstep

FACES = ((0, -1), (0, +1), (1, -1), (1, +1), (2, -1), (2, +1))


def _transverse(d):
    return tuple(t for t in range(3) if t != d)


@functools.lru_cache(maxsize=None)
def exact_mass(N):
    """Exact mass matrix of the N-point LGL Lagrange basis on [-1, 1] (Gauss
    quadrature with N + 1 points is exact for the degree 2N - 2 products)."""
    xg, wg = Leg.leggauss(N + 1)
    B = lgl.lagrange_matrix(lgl.nodes(N), xg)
    return (B * wg[:, None]).T @ B


class HpMesh:
    """Box of bx x by x bz equal blocks with per-block refinement levels and
    per-element degrees.  ``neumann`` lists the box faces 2 d + side that carry
    homogeneous Neumann conditions (the others are Dirichlet, eq. bc)."""

    def __init__(self, lower, upper, blocks, block_levels, degrees, neumann=()):
        self.lower = np.asarray(lower, float)
        self.upper = np.asarray(upper, float)
        self.blocks = tuple(int(b) for b in blocks)
        nb = int(np.prod(self.blocks))
        self.block_levels = np.asarray(block_levels, int).reshape(nb, 3)
        self.neumann = frozenset(int(f) for f in neumann)
        if min(self.blocks) < 1 or self.block_levels.min() < 0:
            raise ValueError("bad block grid")
        self.Lmax = self.block_levels.max(axis=0)
        bsize = (self.upper - self.lower) / np.array(self.blocks, float)
        self.elems = []
        for b in range(nb):
            bx = b % self.blocks[0]
            by = (b // self.blocks[0]) % self.blocks[1]
            bz = b // (self.blocks[0] * self.blocks[1])
            bpos = (bx, by, bz)
            L = self.block_levels[b]
            n = [1 << int(L[d]) for d in range(3)]
            for iz in range(n[2]):
                for iy in range(n[1]):
                    for ix in range(n[0]):
                        idx = (ix, iy, iz)
                        lo = [bpos[d] * (1 << int(self.Lmax[d])) + idx[d] * (1 << int(self.Lmax[d] - L[d]))
                              for d in range(3)]
                        hi = [lo[d] + (1 << int(self.Lmax[d] - L[d])) for d in range(3)]
                        h = bsize / np.array(n, float)
                        plo = self.lower + bsize * np.array(bpos) + h * np.array(idx)
                        self.elems.append(dict(block=b, level=tuple(int(v) for v in L), index=idx,
                                               lo=tuple(lo), hi=tuple(hi), h=h, plo=plo))
        self.E = len(self.elems)
        deg = np.asarray(degrees, int).reshape(self.E, 3)
        if deg.min() < 1:
            raise ValueError("degrees must be at least 1")
        self.N = deg + 1
        sizes = np.prod(self.N, axis=1)
        self.offsets = np.concatenate([[0], np.cumsum(sizes)])
        self.ndof = int(self.offsets[-1])
        self._find_neighbours()

    def _find_neighbours(self):
        self.nbrs = [dict() for _ in range(self.E)]
        for e, ee in enumerate(self.elems):
            for d, s in FACES:
                out = []
                for f, ff in enumerate(self.elems):
                    if f == e:
                        continue
                    touch = ff["hi"][d] == ee["lo"][d] if s < 0 else ff["lo"][d] == ee["hi"][d]
                    if not touch:
                        continue
                    if all(max(ee["lo"][t], ff["lo"][t]) < min(ee["hi"][t], ff["hi"][t])
                           for t in _transverse(d)):
                        for t in _transverse(d):
                            if abs(ee["level"][t] - ff["level"][t]) > 1:
                                raise ValueError("mesh is not two-to-one balanced")
                        out.append(f)
                self.nbrs[e][(d, s)] = out

    def element_view(self, u, e):
        """Nodes of element e from a flat (..., ndof) array, shape (..., Nz, Ny, Nx)."""
        Nx, Ny, Nz = self.N[e]
        return u[..., self.offsets[e]:self.offsets[e + 1]].reshape(u.shape[:-1] + (Nz, Ny, Nx))

    def node_coordinates(self):
        """x, y, z as flat arrays of length ndof."""
        out = np.empty((3, self.ndof))
        for e, ee in enumerate(self.elems):
            Nx, Ny, Nz = self.N[e]
            c = [ee["plo"][d] + ee["h"][d] * (lgl.nodes(int(self.N[e][d])) + 1.0) / 2.0 for d in range(3)]
            X = np.broadcast_to(c[0][None, None, :], (Nz, Ny, Nx))
            Y = np.broadcast_to(c[1][None, :, None], (Nz, Ny, Nx))
            Z = np.broadcast_to(c[2][:, None, None], (Nz, Ny, Nx))
            for d, A in enumerate((X, Y, Z)):
                out[d, self.offsets[e]:self.offsets[e + 1]] = A.reshape(-1)
        return out

    def external(self, e, d, s):
        return len(self.nbrs[e][(d, s)]) == 0


def _apply_1d(a, D, axis):
    a = np.moveaxis(a, axis, -1)
    return np.moveaxis(a @ D.T, -1, axis)


def _face(a, d, s, N):
    """Face slice of an element array (..., Nz, Ny, Nx) normal to d on side s:
    shape (..., N_t1, N_t0) with the lower transverse dimension fastest."""
    idx = 0 if s < 0 else N[d] - 1
    return np.take(a, idx, axis=-1 - d)


def _face_add(a, d, s, N, val):
    idx = 0 if s < 0 else N[d] - 1
    sl = [slice(None)] * a.ndim
    sl[a.ndim - 1 - d] = idx
    a[tuple(sl)] += val


def mortar(mesh: HpMesh, e, d, s, f):
    """Interpolation and projection matrices of the mortar between e's face
    (d, s) and its neighbour f: for t0 < t1 the transverse dimensions,
    ((I_e0, I_e1), (I_f0, I_f1), (P_e0, P_e1)) with I_x: side x's face points
    -> mortar points and P_e: mortar -> e's face points (exact L2 projection)."""
    ee, ff = mesh.elems[e], mesh.elems[f]
    Ie, If, Pe = [], [], []
    for t in _transverse(d):
        a = max(ee["lo"][t], ff["lo"][t])
        b = min(ee["hi"][t], ff["hi"][t])
        M = int(max(mesh.N[e][t], mesh.N[f][t]))
        eta = lgl.nodes(M)
        mats = []
        for g, gg in ((e, ee), (f, ff)):
            w = gg["hi"][t] - gg["lo"][t]
            al = -1.0 + 2.0 * (a - gg["lo"][t]) / w
            be = -1.0 + 2.0 * (b - gg["lo"][t]) / w
            x = al + (be - al) * (eta + 1.0) / 2.0
            mats.append((lgl.lagrange_matrix(lgl.nodes(int(mesh.N[g][t])), x), (be - al) / 2.0))
        (I_e, scale_e), (I_f, _) = mats
        Ne = int(mesh.N[e][t])
        P = np.linalg.solve(exact_mass(Ne), I_e.T @ exact_mass(M)) * scale_e
        Ie.append(I_e)
        If.append(I_f)
        Pe.append(P)
    return tuple(Ie), tuple(If), tuple(Pe)


def _to_mortar(F, I):
    """F (..., n1, n0) -> (..., m1, m0) with I = (I0, I1)."""
    return np.einsum('ab,...bc,dc->...ad', I[1], F, I[0])


def penalty(mesh: HpMesh, C, e, d, f=None):
    """sigma of eq. penalty from the degrees and widths normal to the face."""
    N = mesh.N[e][d] if f is None else max(mesh.N[e][d], mesh.N[f][d])
    h = mesh.elems[e]["h"][d] if f is None else min(mesh.elems[e]["h"][d], mesh.elems[f]["h"][d])
    return C * float(N) ** 2 / h


def mass_element(mesh: HpMesh, e):
    """Diagonal of M on element e, shape (Nz, Ny, Nx)."""
    Nx, Ny, Nz = (int(v) for v in mesh.N[e])
    J = np.prod(mesh.elems[e]["h"]) / 8.0
    return J * (lgl.weights(Nz)[:, None, None] * lgl.weights(Ny)[None, :, None] * lgl.weights(Nx)[None, None, :])


def mass_diagonal(mesh: HpMesh):
    return np.concatenate([mass_element(mesh, e).reshape(-1) for e in range(mesh.E)])


def apply_mass(mesh: HpMesh, f):
    return np.asarray(f, float) * mass_diagonal(mesh)


def _face_mass(mesh: HpMesh, e, d):
    """ML on a face normal to d (LGL face weights times the surface Jacobian),
    shape (N_t1, N_t0)."""
    t0, t1 = _transverse(d)
    h = mesh.elems[e]["h"]
    JF = h[t0] * h[t1] / 4.0
    return JF * np.outer(lgl.weights(int(mesh.N[e][t1])), lgl.weights(int(mesh.N[e][t0])))


def apply_operator(mesh: HpMesh, u, C, dirichlet_values=None):
    """A u for flat nodal values u of shape (..., ndof).  ``dirichlet_values``
    (flat, length ndof, read at Dirichlet boundary nodes) gives inhomogeneous
    boundary data u_b; the default is u_b = 0."""
    u = np.asarray(u, float)
    out = np.zeros_like(u)
    ue = [mesh.element_view(u, e) for e in range(mesh.E)]
    ub = None if dirichlet_values is None else np.asarray(dirichlet_values, float)
    # unlifted physical derivatives of every element
    g = []
    for e in range(mesh.E):
        N, h = mesh.N[e], mesh.elems[e]["h"]
        g.append([(2.0 / h[d]) * _apply_1d(ue[e], lgl.diff_matrix(int(N[d])), -1 - d) for d in range(3)])
    for e in range(mesh.E):
        N, h = mesh.N[e], mesh.elems[e]["h"]
        corr = {}
        for d, s in FACES:
            u_int = _face(ue[e], d, s, N)
            du_int = _face(g[e][d], d, s, N)
            nb = mesh.nbrs[e][(d, s)]
            if not nb:  # eq. bc through the ghost state
                if 2 * d + (s > 0) in mesh.neumann:
                    u_ext, du_ext = u_int, -du_int
                else:
                    u_b = 0.0 if ub is None else _face(mesh.element_view(ub, e), d, s, N)
                    u_ext, du_ext = 2.0 * u_b - u_int, du_int
                sig = penalty(mesh, C, e, d)
                cu = 0.5 * (u_ext - u_int)
                cp = 0.5 * s * (du_int + du_ext) - sig * (u_int - u_ext)
            else:
                cu = np.zeros_like(u_int)
                cp = np.zeros_like(u_int)
                for f in nb:
                    Ie, If, Pe = mortar(mesh, e, d, s, f)
                    Nf = mesh.N[f]
                    u_ext = _to_mortar(_face(ue[f], d, -s, Nf), If)
                    du_ext = _to_mortar(_face(g[f][d], d, -s, Nf), If)
                    ui = _to_mortar(u_int, Ie)
                    dui = _to_mortar(du_int, Ie)
                    sig = penalty(mesh, C, e, d, f)
                    cu_m = 0.5 * (u_ext - ui)
                    cp_m = 0.5 * s * (dui + du_ext) - sig * (ui - u_ext)
                    cu = cu + _to_mortar(cu_m, Pe)
                    cp = cp + _to_mortar(cp_m, Pe)
            corr[(d, s)] = (cu, cp)
        Me = mass_element(mesh, e)
        # auxiliary variable, eq. dg_op_auxvars: v_d = D_d u + L (n_d cu)
        v = [gd.copy() for gd in g[e]]
        for d, s in FACES:
            lift = 2.0 / (h[d] * lgl.weights(int(N[d]))[-1])  # M^-1 ML on the face
            _face_add(v[d], d, s, N, lift * s * corr[(d, s)][0])
        # primal equation, eq. dg_op_primal
        Au = np.zeros_like(ue[e])
        for d in range(3):
            Au -= Me * (2.0 / h[d]) * _apply_1d(v[d], lgl.diff_matrix(int(N[d])), -1 - d)
        for d, s in FACES:
            ML = _face_mass(mesh, e, d)
            _face_add(Au, d, s, N, -ML * (corr[(d, s)][1] - s * _face(v[d], d, s, N)))
        out[..., mesh.offsets[e]:mesh.offsets[e + 1]] = Au.reshape(u.shape[:-1] + (-1,))
    return out


def assemble(mesh: HpMesh, C):
    """Dense A (column j = A e_j), small meshes only."""
    return apply_operator(mesh, np.eye(mesh.ndof), C).T.copy()


# ---------------------------------------------------------------- Schwarz


def overlap_layers(N, overlap):
    return max(1, min(int(overlap), int(N) - 1))


def _own_factors(mesh: HpMesh, e, overlap):
    """Per dimension d: (a_d, low part, high part) at element e's nodes along d."""
    out = []
    for d in range(3):
        N = int(mesh.N[e][d])
        xi = lgl.nodes(N)
        delta = 1.0 + xi[overlap_layers(N, overlap)]
        lo_ext, hi_ext = mesh.external(e, d, -1), mesh.external(e, d, +1)
        lo = np.ones(N) if lo_ext else smoothstep((xi + 1.0) / delta)
        hi = -np.ones(N) if hi_ext else smoothstep((xi - 1.0) / delta)
        out.append((0.5 * (lo - hi), 0.5 * (1.0 - lo), 0.5 * (1.0 + hi)))
    return out


def _T(aj, ak):
    bj, bk = 1.0 - aj, 1.0 - ak
    return aj * ak + 0.5 * bj * ak + 0.5 * aj * bk + bj * bk / 3.0


def subdomain_layout(mesh: HpMesh, e, overlap):
    """Global indices and weights of the points of subdomain S_e: the central
    element's nodes, then for each face in the order -x, +x, -y, +y, -z, +z
    and each neighbour across it (ascending element index) N_ov layers of the
    neighbour's nodes, layer 0 nearest the face, lower transverse dimension
    fastest within a layer."""
    idx, wts = [], []
    fac = _own_factors(mesh, e, overlap)
    Nx, Ny, Nz = (int(v) for v in mesh.N[e])
    base = mesh.offsets[e]
    for k in range(Nz):
        for j in range(Ny):
            for i in range(Nx):
                idx.append(base + (k * Ny + j) * Nx + i)
                wts.append(fac[0][0][i] * fac[1][0][j] * fac[2][0][k])
    for d, s in FACES:
        for f in mesh.nbrs[e][(d, s)]:
            Nf = [int(v) for v in mesh.N[f]]
            nov = overlap_layers(Nf[d], overlap)
            ff = _own_factors(mesh, f, overlap)
            cnt = len(mesh.nbrs[f][(d, -s)])
            t0, t1 = _transverse(d)
            for layer in range(nov):
                m = layer if s > 0 else Nf[d] - 1 - layer  # f's node index along d
                part = ff[d][1][m] if s > 0 else ff[d][2][m]  # f's side facing e
                for b1 in range(Nf[t1]):
                    for b0 in range(Nf[t0]):
                        node = [0, 0, 0]
                        node[d], node[t0], node[t1] = m, b0, b1
                        i, j, k = node
                        idx.append(mesh.offsets[f] + (k * Nf[1] + j) * Nf[0] + i)
                        wts.append(part * _T(ff[t0][0][b0], ff[t1][0][b1]) / cnt)
    return np.array(idx, dtype=np.int64), np.array(wts)


class HpSchwarzSmoother:
    """Additive Schwarz on an hp mesh with A_S = R_S A R_S^T solved by its
    explicit inverse (Sec. III.D.2, Sec. III.E.2)."""

    def __init__(self, mesh: HpMesh, C, overlap=2, A=None):
        self.mesh, self.C = mesh, C
        self.A = assemble(mesh, C) if A is None else A
        self.layout = [subdomain_layout(mesh, e, overlap) for e in range(mesh.E)]
        self.inv = [np.linalg.inv(self.A[np.ix_(ix, ix)]) for ix, _ in self.layout]

    def apply(self, u):
        return self.A @ np.asarray(u, float).reshape(-1)

    def correction(self, r):
        du = np.zeros_like(r)
        for (ix, w), Ainv in zip(self.layout, self.inv):
            np.add.at(du, ix, w * (Ainv @ r[ix]))
        return du

    def smooth(self, u, b, steps):
        u = np.array(u, float).reshape(-1)
        for _ in range(steps):
            u = u + self.correction(b - self.apply(u))
        return u


# ---------------------------------------------------------------- multigrid


def coarsen(mesh: HpMesh):
    """Coarse mesh and, for every fine element, (parent, child position per
    dimension: 0 / 1 for the low / high half of a split dimension, -1 where the
    dimension is not split); None if no block can be coarsened."""
    L = mesh.block_levels
    if L.max() == 0:
        return None
    Lc = np.maximum(L - 1, 0)
    parents, pos = [], []
    keys = {}
    for e, ee in enumerate(mesh.elems):
        b = ee["block"]
        split = [L[b][d] > 0 for d in range(3)]
        pidx = tuple(ee["index"][d] // 2 if split[d] else ee["index"][d] for d in range(3))
        parents.append((b, pidx))
        pos.append(tuple(ee["index"][d] % 2 if split[d] else -1 for d in range(3)))
    # coarse element order: block by block, x fastest (as HpMesh numbers them)
    order = []
    for b in range(len(L)):
        n = [1 << int(Lc[b][d]) for d in range(3)]
        for iz in range(n[2]):
            for iy in range(n[1]):
                for ix in range(n[0]):
                    keys[(b, (ix, iy, iz))] = len(order)
                    order.append((b, (ix, iy, iz)))
    deg = np.full((len(order), 3), 1 << 30)
    parent = [keys[p] for p in parents]
    for e, c in enumerate(parent):
        deg[c] = np.minimum(deg[c], mesh.N[e] - 1)  # the smaller degree per dimension
    coarse = HpMesh(mesh.lower, mesh.upper, mesh.blocks, Lc, deg, neumann=mesh.neumann)
    return coarse, parent, pos


def _child_matrix(Nc, Nf, p):
    x = lgl.nodes(Nf)
    if p < 0:
        t = x
    else:
        t = (x - 1.0) / 2.0 if p == 0 else (x + 1.0) / 2.0
    return lgl.lagrange_matrix(lgl.nodes(Nc), t)


def transfer_matrices(fine: HpMesh, coarse: HpMesh, parent, pos):
    mats = []
    for e in range(fine.E):
        c = parent[e]
        mats.append([_child_matrix(int(coarse.N[c][d]), int(fine.N[e][d]), pos[e][d]) for d in range(3)])
    return mats


def prolongate(fine, coarse, parent, mats, uc):
    uc = np.asarray(uc, float)
    uf = np.zeros(fine.ndof)
    for e in range(fine.E):
        Px, Py, Pz = mats[e]
        v = np.einsum('kc,jb,ia,cba->kji', Pz, Py, Px, coarse.element_view(uc, parent[e]))
        uf[fine.offsets[e]:fine.offsets[e + 1]] = v.reshape(-1)
    return uf


def restrict(fine, coarse, parent, mats, rf):
    rf = np.asarray(rf, float)
    bc = np.zeros(coarse.ndof)
    for e in range(fine.E):
        Px, Py, Pz = mats[e]
        v = np.einsum('kc,jb,ia,kji->cba', Pz, Py, Px, fine.element_view(rf, e))
        c = parent[e]
        bc[coarse.offsets[c]:coarse.offsets[c + 1]] += v.reshape(-1)
    return bc


class HpVCycle:
    """V-cycle (Sec. III.C.3) over the hp hierarchy with ``pre``/``post``
    Schwarz steps; the coarsest level smooths pre + post times."""

    def __init__(self, mesh: HpMesh, C, levels=2, overlap=2, pre=3, post=3):
        self.meshes, self.transfers = [mesh], []
        while len(self.meshes) < levels:
            c = coarsen(self.meshes[-1])
            if c is None:
                break
            coarse, parent, pos = c
            self.transfers.append((parent, transfer_matrices(self.meshes[-1], coarse, parent, pos)))
            self.meshes.append(coarse)
        self.smoothers = [HpSchwarzSmoother(m, C, overlap) for m in self.meshes]
        self.pre, self.post = pre, post

    def __call__(self, b):
        return self._visit(0, np.asarray(b, float).reshape(-1))

    def _visit(self, l, b):
        sm = self.smoothers[l]
        u = sm.smooth(np.zeros_like(b), b, self.pre)
        if l == len(self.meshes) - 1:
            return sm.smooth(u, b, self.post)
        parent, mats = self.transfers[l]
        fine, coarse = self.meshes[l], self.meshes[l + 1]
        bc = restrict(fine, coarse, parent, mats, b - sm.apply(u))
        u = u + prolongate(fine, coarse, parent, mats, self._visit(l + 1, bc))
        return sm.smooth(u, b, self.post)
