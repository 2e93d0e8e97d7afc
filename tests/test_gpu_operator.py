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
