"""Axis-aligned box of uniform elements (Sec. II, blocks split into elements).

Test infrastructure only: imported by the tests, smoke() and the benchmark's
CPU leg, never by the product path.

One block, the box [lo, hi], split into n_x * n_y * n_z equal elements.  Each
element carries N = p+1 LGL points per dimension.  Nodal arrays have shape
(..., E, N, N, N) indexed [e, k, j, i] with the x index i fastest and the
element index e = (e_z n_y + e_y) n_x + e_x, so that a flattened array is the
canonical layout idx = ((e N + k) N + j) N + i.

Dimension d = 0, 1, 2 (x, y, z) maps to node axis -1, -2, -3 and, in the
"grid" view (..., n_z, n_y, n_x, N, N, N), to element axis -4, -5, -6.
"""
from __future__ import annotations

import numpy as np

from . import lgl

NODE_AXIS = (-1, -2, -3)
GRID_ELEM_AXIS = (-4, -5, -6)


class BoxMesh:
    """Uniform box grid.  ``neumann`` lists the box faces f = 2 d + side (side
    0 = low, 1 = high) that carry homogeneous Neumann conditions; the others
    are homogeneous Dirichlet (eq. bc)."""

    def __init__(self, lower, upper, elements, p, neumann=()):
        self.neumann = frozenset(int(f) for f in neumann)
        if not self.neumann <= set(range(6)):
            raise ValueError("bad face")
        self.lower = np.asarray(lower, dtype=float)
        self.upper = np.asarray(upper, dtype=float)
        self.n = tuple(int(v) for v in elements)  # (nx, ny, nz)
        if min(self.n) < 1 or p < 1:
            raise ValueError("bad mesh")
        self.p = int(p)
        self.N = self.p + 1
        self.h = (self.upper - self.lower) / np.array(self.n, dtype=float)
        self.E = self.n[0] * self.n[1] * self.n[2]

    @property
    def ndof(self):
        return self.E * self.N ** 3

    # element <-> grid index
    def elem_index(self, ex, ey, ez):
        return (ez * self.n[1] + ey) * self.n[0] + ex

    def elem_coords(self, e):
        ex = e % self.n[0]
        ey = (e // self.n[0]) % self.n[1]
        ez = e // (self.n[0] * self.n[1])
        return ex, ey, ez

    def neighbor(self, e, d, s):
        """Face neighbour across dimension d on side s (+1/-1), or None at the
        external boundary."""
        c = list(self.elem_coords(e))
        c[d] += s
        if c[d] < 0 or c[d] >= self.n[d]:
            return None
        return self.elem_index(*c)

    def external_flags(self, e):
        """((low_x, high_x), (low_y, high_y), (low_z, high_z)) external-face flags."""
        c = self.elem_coords(e)
        return tuple((c[d] == 0, c[d] == self.n[d] - 1) for d in range(3))

    # views
    def grid(self, a):
        nx, ny, nz = self.n
        N = self.N
        return a.reshape(a.shape[:-4] + (nz, ny, nx, N, N, N))

    def flat(self, g):
        N = self.N
        return g.reshape(g.shape[:-6] + (self.E, N, N, N))

    def node_coordinates(self):
        """x, y, z arrays of shape (E, N, N, N)."""
        xi = lgl.nodes(self.N)
        out = []
        for d in range(3):
            e_idx = np.arange(self.n[d])
            # physical coordinate of node m in element e_d
            c = self.lower[d] + self.h[d] * (e_idx[:, None] + (xi[None, :] + 1.0) / 2.0)
            shape = [1] * 6
            shape[GRID_ELEM_AXIS[d] + 6] = self.n[d]
            shape[NODE_AXIS[d] + 6] = self.N
            full = np.broadcast_to(c.reshape(shape),
                                   (self.n[2], self.n[1], self.n[0], self.N, self.N, self.N))
            out.append(self.flat(np.ascontiguousarray(full)))
        return tuple(out)
