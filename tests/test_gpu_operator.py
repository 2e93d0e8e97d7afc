"""GPU parity of the DG operator, mass and node coordinates against the oracle
(element by element on seeded inputs), through the C ABI."""
import numpy as np
import pytest

import workloads as W
from oracle import mesh as omesh, operator as oop
from tests.gpu_util import announce, rel_max, to_gpu, to_np

pytestmark = pytest.mark.gpu

# several tiles of elements and ragged tails, every degree, boxes and 1-element meshes
CASES = [
    ((1, 1, 1), 1, (1, 1, 1)), ((2, 2, 2), 3, (1, 1, 1)), ((3, 2, 5), 2, (1, 2, 0.5)),
    ((4, 4, 4), 4, (1, 1, 1)), ((5, 3, 2), 5, (2, 1, 1)), ((3, 3, 3), 6, (1, 1, 1)),
    ((7, 3, 2), 7, (1, 1.5, 0.8)), ((2, 3, 4), 8, (1, 1, 1)), ((1, 1, 1), 8, (1, 1, 1)),
    ((6, 6, 6), 7, (40, 40, 40)),
]


@pytest.mark.parametrize("elements,p,size", CASES)
def test_apply_matches_oracle(elements, p, size):
    import paper_2111_06767_amd as dg
    announce(f"apply parity elements={elements} p={p} size={size}")
    lower = (0.25, -0.5, 0.0)
    upper = tuple(l + s for l, s in zip(lower, size))
    prob = dg.Problem(lower, upper, elements, p, penalty=1.5)
    m = omesh.BoxMesh(lower, upper, elements, p)
    u = W.random_normal(W.SEED_APPLY + p, m.ndof)
    ref = oop.apply_operator(m, u.reshape(m.E, m.N, m.N, m.N), 1.5).reshape(-1)
    got = to_np(prob.apply(to_gpu(u)))
    assert rel_max(got, ref) < 1e-13, rel_max(got, ref)
    xyz = to_np(prob.node_coordinates()).reshape(3, -1)
    for d, c in enumerate(m.node_coordinates()):
        np.testing.assert_allclose(xyz[d], c.reshape(-1), rtol=0, atol=1e-14 * max(1, abs(upper[d])))
    f = W.random_normal(5, m.ndof)
    b = to_np(prob.apply_mass(to_gpu(f)))
    err = rel_max(b, oop.apply_mass(m, f.reshape(m.E, m.N, m.N, m.N)))
    assert err < 1e-14, err  # a product of four factors, rounded in another order


def test_apply_large_sampled():
    # the 16^3, p = 7 share: compare sampled elements against the oracle on a
    # patch around each sample (the operator only couples face neighbours)
    import paper_2111_06767_amd as dg
    announce("apply parity 16^3 p=7 sampled")
    n, p = 16, 7
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (n, n, n), p)
    N = p + 1
    u = W.random_normal(W.SEED_APPLY, prob.ndof)
    got = to_np(prob.apply(to_gpu(u))).reshape(n, n, n, N, N, N)
    ug = u.reshape(n, n, n, N, N, N)
    h = 1.0 / n
    rng = np.random.default_rng(0)
    for _ in range(6):
        c = rng.integers(0, n, 3)  # (ex, ey, ez)
        lo = np.maximum(c - 1, 0)
        hi = np.minimum(c + 2, n)
        sub = ug[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]]
        # patch mesh with the true boundary only where the box boundary is
        pm = omesh.BoxMesh(lo * h, hi * h, tuple(hi - lo), p)
        full = oop.apply_operator(pm, sub.reshape(-1, N, N, N), 1.5)
        ce = (c - lo)
        e = pm.elem_index(*ce)
        ref = full[e]
        gotc = got[c[2], c[1], c[0]]
        # the patch's own artificial faces only touch elements other than the centre
        assert rel_max(gotc, ref) < 1e-13


def test_apply_is_linear_and_symmetric_on_gpu():
    import torch
    import paper_2111_06767_amd as dg
    announce("apply symmetry 6x5x4 p=5")
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (6, 5, 4), 5)
    x = to_gpu(W.random_normal(1, prob.ndof))
    y = to_gpu(W.random_normal(2, prob.ndof))
    Ax, Ay = prob.apply(x), prob.apply(y)
    a, b = torch.dot(y, Ax).item(), torch.dot(x, Ay).item()
    assert abs(a - b) < 1e-12 * abs(a)
    assert torch.dot(x, Ax).item() > 0


SHAPE_CASES = [((3, 2, 5), 2), ((5, 3, 2), 5), ((4, 4, 4), 6), ((7, 3, 2), 7), ((1, 1, 1), 7),
               ((2, 3, 4), 8), ((9, 8, 7), 7), ((2, 2, 2), 7), ((5, 3, 17), 7), ((3, 5, 9), 4),
               ((1, 2, 13), 3)]


@pytest.mark.parametrize("elements,p", SHAPE_CASES)
def test_every_launch_shape_gives_the_same_apply(elements, p):
    """Elements per workgroup and 2x2x2 bricks (odd grids leave ragged bricks)
    only regroup the elements: every shape returns the same bits, and they
    match the oracle."""
    import paper_2111_06767_amd as dg
    announce(f"apply launch shapes elements={elements} p={p}")
    prob = dg.Problem((0, 0, 0), (1, 1, 1), elements, p, penalty=1.5, mg_levels=1)
    m = omesh.BoxMesh((0, 0, 0), (1, 1, 1), elements, p)
    u = to_gpu(W.random_normal(W.SEED_APPLY + 17 * p, m.ndof))
    shapes = [1, 2, 0] + ([-1] if p == 7 else [])
    outs = {}
    for sh in shapes:
        prob.set_apply_shape(sh)
        assert prob.apply_shape() == sh
        outs[sh] = to_np(prob.apply(u))
    if p != 7:
        with pytest.raises(dg.DgsError):
            prob.set_apply_shape(-1)
    prob.close()
    for sh in shapes[1:]:
        assert np.array_equal(outs[sh], outs[1]), sh
    ref = oop.apply_operator(m, to_np(u).reshape(m.E, m.N, m.N, m.N), 1.5).reshape(-1)
    assert rel_max(outs[1], ref) < 1e-13


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_brick_shape_solve_is_bit_identical(precision):
    """The whole preconditioned solve (residuals with the fused subdomain-row
    gather on every level) with bricks on every level equals the one with one
    element per workgroup, bit for bit."""
    import paper_2111_06767_amd as dg
    announce(f"brick-shape solve 5x4x6 p=7 {precision}")
    b = to_gpu(W.random_normal(3, 5 * 4 * 6 * 512))
    sols = []
    for sh in (1, -1):
        prob = dg.Problem((0, 0, 0), (1, 1, 1), (5, 4, 6), 7, mg_levels=3, precision=precision)
        for lev in range(3):
            prob.set_apply_shape(sh, level=lev)
        u, st = prob.solve(b)
        sols.append((to_np(u), st["iterations"]))
        prob.close()
    for other in sols[1:]:
        assert sols[0][1] == other[1]
        assert np.array_equal(sols[0][0], other[0])


# (elements, p, size, Neumann face mask): one face, opposite faces, all but one,
# the brick shape at p = 7 (shape -1) and 1-element dimensions
NEUMANN_CASES = [((2, 2, 2), 3, (1, 1, 1), 0b000010), ((3, 2, 4), 2, (1, 2, 0.5), 0b001100),
                 ((3, 3, 3), 5, (1, 1, 1), 0b111110), ((4, 4, 2), 7, (1, 1, 1), 0b010101),
                 ((5, 1, 2), 4, (2, 1, 1), 0b101010)]


@pytest.mark.parametrize("elements,p,size,neumann", NEUMANN_CASES)
def test_apply_with_neumann_faces_matches_oracle(elements, p, size, neumann):
    """Homogeneous Neumann box faces (eq. bc ghost fluxes) in every launch
    shape against the oracle's operator."""
    import paper_2111_06767_amd as dg
    announce(f"neumann apply elements={elements} p={p} mask={neumann:06b}")
    lower = (0.25, -0.5, 0.0)
    upper = tuple(l + s for l, s in zip(lower, size))
    faces = [f for f in range(6) if neumann >> f & 1]
    m = omesh.BoxMesh(lower, upper, elements, p, neumann=faces)
    u = W.random_normal(W.SEED_APPLY + p, m.ndof)
    ref = oop.apply_operator(m, u.reshape(m.E, m.N, m.N, m.N), 1.5).reshape(-1)
    prob = dg.Problem(lower, upper, elements, p, penalty=1.5, mg_levels=1, neumann_faces=neumann)
    for shape in (1, 2, 0) + ((-1,) if p == 7 else ()):
        prob.set_apply_shape(shape, level=0)
        got = to_np(prob.apply(to_gpu(u)))
        assert rel_max(got, ref) < 1e-13, (shape, rel_max(got, ref))
    prob.close()
