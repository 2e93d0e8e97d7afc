"""Pins of the oracle's hp-nonuniform DG operator, Schwarz smoother and
multigrid (Sec. II, Sec. III.C.1, Sec. III.D), each against something other
than the code it checks: the uniform-grid oracle (pinned by its own tests),
exact reproduction of quadratic polynomials across nonconforming faces,
properties of the L2 projection, the partition of unity of the Schwarz
weights, polynomial reproduction by the prolongation, and convergence to a
manufactured solution."""
import numpy as np
import pytest

import workloads as W
from oracle import hp, krylov, mesh as omesh, multigrid, operator as oop, schwarz

C = 1.5

# 2 x 1 x 1 blocks, the left one split once along every dimension: the right
# element meets four smaller ones across its -x face
TWO_BLOCKS = ((2, 1, 1), [(1, 1, 1), (0, 0, 0)])
# 2 x 2 x 1 blocks with anisotropic levels (split along some dimensions only)
ANISO = ((2, 2, 1), [(1, 0, 1), (0, 1, 0), (1, 1, 0), (0, 0, 1)])


def _mesh(spec, upper=(2, 1.5, 1), seed=0, lo=2, hi=5, neumann=()):
    blocks, levels = spec
    E = sum(2 ** sum(lv) for lv in levels)
    deg = np.random.default_rng(seed).integers(lo, hi, size=(E, 3))
    return hp.HpMesh((0, 0, 0), upper, blocks, levels, deg, neumann=neumann)


def test_one_uniform_block_is_the_box_grid():
    box = omesh.BoxMesh((0, 0, 0), (1, 1.2, 0.9), (4, 2, 2), 3, neumann=(1, 4))
    m = hp.HpMesh((0, 0, 0), (1, 1.2, 0.9), (1, 1, 1), [(2, 1, 1)], np.full((16, 3), 3), neumann=(1, 4))
    u = W.random_normal(1, m.ndof)
    ref = oop.apply_operator(box, u.reshape(box.E, box.N, box.N, box.N), C).reshape(-1)
    assert np.abs(hp.apply_operator(m, u, C) - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.allclose(hp.mass_diagonal(m), np.tile(oop.mass_diagonal(box).reshape(-1), box.E), rtol=1e-15)
    for e in (0, 5, 15):
        ix, w = hp.subdomain_layout(m, e, 2)
        assert np.array_equal(ix, schwarz.subdomain_layout(box, e, 2)[0])
        assert np.abs(w - schwarz.subdomain_weights(box, e, 2)).max() <= 1e-15


def test_equal_blocks_form_the_box_grid():
    # 2 x 2 x 1 blocks of 2 x 1 x 2 elements each: the box grid of 4 x 2 x 2
    # elements in another element order; neighbours are found across blocks
    m = hp.HpMesh((0, 0, 0), (2, 1, 1), (2, 2, 1), [(1, 0, 1)] * 4, np.full((16, 3), 2))
    box = omesh.BoxMesh((0, 0, 0), (2, 1, 1), (4, 2, 2), 2)
    perm = []  # box element of each hp element
    for ee in m.elems:
        b = ee["block"]
        bx, by = b % 2, b // 2
        ix, iy, iz = ee["index"]
        perm.append(box.elem_index(2 * bx + ix, by + iy, iz))
    perm = np.array(perm)
    u_box = W.random_normal(2, box.ndof).reshape(box.E, -1)
    ref = oop.apply_operator(box, u_box.reshape(box.E, 3, 3, 3), C).reshape(box.E, -1)
    got = hp.apply_operator(m, u_box[perm].reshape(-1), C).reshape(m.E, -1)
    assert np.abs(got - ref[perm]).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("spec", [TWO_BLOCKS, ANISO])
def test_quadratics_are_reproduced_across_nonconforming_faces(spec):
    # a quadratic is a polynomial of every element's degrees (>= 2) and its
    # gradient is continuous: with its own Dirichlet data every jump vanishes
    # on every mortar, so A u = -M Laplacian(u) at every node
    m = _mesh(spec)
    x, y, z = m.node_coordinates()
    u = 0.3 * x ** 2 - 0.2 * x * y + 0.5 * z ** 2 + 0.1 * y + 0.7
    Au = hp.apply_operator(m, u, C, dirichlet_values=u)
    ref = -hp.mass_diagonal(m) * 1.6
    assert np.abs(Au - ref).max() <= 1e-12 * np.abs(ref).max()
    # a linear function leaves no residual with a degree-1 element present
    m1 = _mesh(spec, seed=3, lo=1, hi=3)
    x, y, z = m1.node_coordinates()
    u = 0.4 * x - 0.3 * y + 0.2 * z + 1
    assert np.abs(hp.apply_operator(m1, u, C, dirichlet_values=u)).max() <= 1e-12


def test_mortar_projection_keeps_the_element_polynomials():
    # interpolating an element's face data to its mortars and projecting it
    # back is the identity (the projection is the L2 projection onto the
    # face's polynomials); on a conforming face of equal degrees every
    # matrix is the identity
    m = _mesh(TWO_BLOCKS, seed=5)
    big = 8
    for f in m.nbrs[big][(0, -1)]:
        Ie, If, Pe = hp.mortar(m, big, 0, -1, f)
        for t in range(2):
            # the big face is covered by four half-by-half mortars
            assert Ie[t].shape[1] == m.N[big][1 + t]
    for t, dims in enumerate((1, 2)):
        acc = np.zeros((m.N[big][dims], m.N[big][dims]))
        seen = set()
        for f in m.nbrs[big][(0, -1)]:
            Ie, _, Pe = hp.mortar(m, big, 0, -1, f)
            key = (m.elems[f]["lo"][dims])
            if key in seen:
                continue
            seen.add(key)
            acc += Pe[t] @ Ie[t]
        assert np.allclose(acc, np.eye(len(acc)), atol=1e-13)
    same = hp.HpMesh((0, 0, 0), (2, 1, 1), (2, 1, 1), [(0, 0, 0)] * 2, [(3, 2, 4), (3, 2, 4)])
    Ie, If, Pe = hp.mortar(same, 0, 0, +1, 1)
    for M in Ie + If + Pe:
        assert np.allclose(M, np.eye(len(M)), atol=1e-14)
    pm = hp.HpMesh((0, 0, 0), (2, 1, 1), (2, 1, 1), [(0, 0, 0)] * 2, [(3, 2, 4), (3, 4, 2)])
    Ie, If, Pe = hp.mortar(pm, 0, 0, +1, 1)
    assert np.allclose(Pe[0] @ Ie[0], np.eye(3), atol=1e-13) and Ie[0].shape == (5, 3)


def test_spectrum_and_symmetry():
    # symmetric wherever every face is conforming with equal degrees;
    # otherwise the eigenvalues stay in the right half plane
    m = hp.HpMesh((0, 0, 0), (2, 1, 1), (2, 2, 1), [(1, 0, 1)] * 4, np.full((16, 3), 2))
    A = hp.assemble(m, C)
    assert np.abs(A - A.T).max() <= 1e-13 * np.abs(A).max()
    for spec in (TWO_BLOCKS, ANISO):
        A = hp.assemble(_mesh(spec), C)
        assert np.abs(A - A.T).max() > 1e-3 * np.abs(A).max()
        assert np.linalg.eigvals(A).real.min() > 0


@pytest.mark.parametrize("spec", [TWO_BLOCKS, ANISO])
def test_schwarz_weights_are_a_partition_of_unity(spec):
    m = _mesh(spec, seed=7)
    for overlap in (1, 2, 3):
        tot = np.zeros(m.ndof)
        for e in range(m.E):
            ix, w = hp.subdomain_layout(m, e, overlap)
            assert len(np.unique(ix)) == len(ix)
            assert w.min() >= 0
            np.add.at(tot, ix, w)
        assert np.abs(tot - 1).max() <= 1e-14


def test_the_coarse_mesh_takes_the_smaller_degree():
    m = _mesh(TWO_BLOCKS, seed=9)
    coarse, parent, pos = hp.coarsen(m)
    assert coarse.E == 2 and parent[:8] == [0] * 8 and parent[8] == 1
    assert np.array_equal(coarse.N[0], m.N[:8].min(axis=0))
    assert np.array_equal(coarse.N[1], m.N[8])
    assert hp.coarsen(coarse) is None


def test_transfers_reproduce_polynomials_and_are_transposes():
    m = _mesh(ANISO, seed=11)
    coarse, parent, pos = hp.coarsen(m)
    mats = hp.transfer_matrices(m, coarse, parent, pos)
    # a polynomial of the coarse degrees prolongates to itself
    q = lambda x, y, z: 0.5 + x - 0.25 * y + 0.125 * x * z
    assert coarse.N.min() >= 2
    uc = q(*coarse.node_coordinates())
    assert np.abs(hp.prolongate(m, coarse, parent, mats, uc) - q(*m.node_coordinates())).max() <= 1e-13
    a, b = W.random_normal(12, coarse.ndof), W.random_normal(13, m.ndof)
    lhs = hp.prolongate(m, coarse, parent, mats, a) @ b
    assert abs(lhs - a @ hp.restrict(m, coarse, parent, mats, b)) <= 1e-12 * abs(lhs)


def test_uniform_vcycle_is_the_box_vcycle():
    box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (4, 4, 2), 2)
    m = hp.HpMesh((0, 0, 0), (1, 1, 1), (1, 1, 1), [(2, 2, 1)], np.full((32, 3), 2))
    r = W.random_normal(3, m.ndof)
    ref = multigrid.VCycle(box, C, levels=2)(r)
    assert np.abs(hp.HpVCycle(m, C, levels=2)(r) - ref).max() <= 1e-12 * np.abs(ref).max()


def test_converges_to_a_manufactured_solution_on_an_hp_mesh():
    # -Laplacian(u) = 3 pi^2 u, u = prod sin(pi x_d) on the unit cube, with
    # the degrees of a nonconforming mesh raised together
    # (2 x 2 x 2 blocks, one of them refined, so that no element spans a
    # symmetric interval of the solution, where odd and even degrees pair up)
    errs = []
    base = np.random.default_rng(1).integers(0, 2, size=(15, 3))
    for p in (2, 3, 4, 5):
        m = hp.HpMesh((0, 0, 0), (1, 1, 1), (2, 2, 2), [(1, 1, 1)] + [(0, 0, 0)] * 7, base + p)
        x, y, z = m.node_coordinates()
        uex = np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)
        us = np.linalg.solve(hp.assemble(m, C), hp.apply_mass(m, 3 * np.pi ** 2 * uex))
        errs.append(np.abs(us - uex).max())
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[0] / errs[-1] > 100, errs


def test_vcycle_preconditioned_fgmres_on_an_hp_mesh():
    m = hp.HpMesh((0, 0, 0), (2, 1, 1), (2, 1, 1), [(1, 1, 1), (2, 2, 2)],
                  np.random.default_rng(1).integers(2, 4, size=(72, 3)))
    cyc = hp.HpVCycle(m, C, levels=3)
    assert [mm.E for mm in cyc.meshes] == [72, 9, 2]
    A = cyc.smoothers[0].A
    b = W.random_normal(4, m.ndof)
    x, its, _ = krylov.fgmres(lambda v: A @ v, b, precondition=cyc, rtol=1e-10)
    assert its <= 12 and np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-8 * np.linalg.norm(x)


def test_unbalanced_meshes_are_refused():
    with pytest.raises(ValueError):
        hp.HpMesh((0, 0, 0), (2, 1, 1), (2, 1, 1), [(2, 2, 2), (0, 0, 0)], np.full((65, 3), 2))
