"""GPU parity of curved (isoparametric) elements against the oracle, through
the C ABI: the operator and the mass on deformed grids and on a wedge of a
spherical shell (Sec. II with the element Jacobian), and FGMRES solves whose
multigrid-Schwarz preconditioner keeps the box grid."""
import numpy as np
import pytest

import workloads as W
from oracle import curved, krylov, mesh as omesh, multigrid, newton as onewton
from tests.gpu_util import announce, rel_max, to_gpu, to_np

pytestmark = pytest.mark.gpu

C = 1.5


def _problem(box, **opts):
    import paper_2111_06767_amd as dg
    return dg.Problem(tuple(box.lower), tuple(box.upper), box.n, box.p, penalty=C,
                      neumann_faces=sum(1 << f for f in box.neumann), **opts)


@pytest.mark.parametrize("elements,p,neumann,amp", [((3, 2, 2), 3, (), 0.1), ((2, 3, 2), 5, (1, 4), 0.08),
                                                    ((2, 2, 2), 7, (0,), 0.05), ((4, 1, 2), 2, (), 0.12),
                                                    ((1, 1, 1), 4, (), 0.1)])
def test_curved_apply_matches_oracle(elements, p, neumann, amp):
    announce(f"curved apply elements={elements} p={p} neumann={neumann}")
    box = omesh.BoxMesh((0, 0, 0), (1.0, 1.1, 0.9), elements, p, neumann=neumann)
    xyz = curved.deformed_box(box, amp)
    cm = curved.CurvedMesh(box, xyz)
    prob = _problem(box, mg_levels=1)
    prob.set_geometry(to_gpu(xyz.reshape(-1)))
    u = W.random_normal(51 + p, box.ndof)
    ref = curved.apply_operator(cm, u, C)
    got = to_np(prob.apply(to_gpu(u)))
    assert rel_max(got, ref) < 1e-12, rel_max(got, ref)
    f = W.random_uniform(52, box.ndof)
    assert rel_max(to_np(prob.apply_mass(to_gpu(f))), curved.apply_mass(cm, f).reshape(-1)) < 1e-14
    prob.close()


def test_box_coordinates_give_the_box_operator():
    announce("curved kernel on box coordinates")
    box = omesh.BoxMesh((0, 0, 0), (1.2, 1.0, 0.8), (3, 2, 2), 4, neumann=(3,))
    prob = _problem(box, mg_levels=1)
    u = to_gpu(W.random_normal(53, box.ndof))
    ref = to_np(prob.apply(u))
    prob.set_geometry(to_gpu(np.stack(box.node_coordinates()).reshape(-1)))
    got = to_np(prob.apply(u))
    assert rel_max(got, ref) < 1e-13
    prob.set_geometry(None)
    assert np.array_equal(to_np(prob.apply(u)), ref)
    prob.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_curved_solve_matches_oracle(precision):
    # the operator is the curved one, the V-cycle that of the box grid: the
    # oracle runs the same FGMRES with its box V-cycle
    announce(f"curved solve {precision}")
    box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (4, 4, 2), 3)
    xyz = curved.deformed_box(box, 0.1)
    cm = curved.CurvedMesh(box, xyz)
    X = cm.xyz
    f = 3 * np.pi ** 2 * np.sin(np.pi * X[0]) * np.sin(np.pi * X[1]) * np.sin(np.pi * X[2])
    b = curved.apply_mass(cm, f).reshape(-1)
    A = lambda v: curved.apply_operator(cm, v, C)
    x_ref, its_ref, _ = krylov.fgmres(A, b, precondition=multigrid.VCycle(box, C, levels=2),
                                      rtol=1e-10)
    prob = _problem(box, mg_levels=2, precision=precision)
    prob.set_geometry(to_gpu(xyz.reshape(-1)))
    u, st = prob.solve(to_gpu(b))
    u = to_np(u)
    assert st["converged"] and st["rel_residual"] <= 1e-10
    assert abs(st["iterations"] - its_ref) <= 1, (st["iterations"], its_ref)
    assert np.linalg.norm(b - A(u)) / np.linalg.norm(b) <= 1e-10
    assert np.linalg.norm(u - x_ref) / np.linalg.norm(x_ref) <= 1e-9
    prob.close()


def test_curved_solve_equals_the_dense_solution():
    announce("curved solve vs dense")
    box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (2, 2, 2), 3)
    xyz = curved.deformed_box(box, 0.15)
    cm = curved.CurvedMesh(box, xyz)
    b = W.random_normal(54, box.ndof)
    exact = np.linalg.solve(curved.assemble(cm, C), b)
    prob = _problem(box, mg_levels=2)
    prob.set_geometry(to_gpu(xyz.reshape(-1)))
    u, st = prob.solve(to_gpu(b))
    assert st["converged"]
    assert np.linalg.norm(to_np(u) - exact) / np.linalg.norm(exact) <= 1e-9
    prob.close()


def test_geometry_checks():
    import paper_2111_06767_amd as dg
    announce("curved geometry checks")
    box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (2, 1, 1), 2)
    prob = _problem(box, mg_levels=1)
    xyz = np.stack(box.node_coordinates())
    flipped = xyz.copy()
    flipped[0, 0] = flipped[0, 0][:, :, ::-1]  # mirror element 0 in x: det < 0
    with pytest.raises(dg.DgsError):
        prob.set_geometry(to_gpu(flipped.reshape(-1)))
    prob.set_geometry(to_gpu(xyz.reshape(-1)))
    n = prob.ndof
    al, be = to_gpu(np.ones(n)), to_gpu(np.ones(n))
    with pytest.raises(dg.DgsError):  # the puncture problem is set on the box grid
        prob.newton_solve(al, be)
    prob.close()
    big = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (1, 1, 1), 8)
    prob = _problem(big, mg_levels=1)
    with pytest.raises(dg.DgsError):
        prob.set_geometry(to_gpu(np.stack(big.node_coordinates()).reshape(-1)))
    prob.close()


def test_wedge_of_a_spherical_shell_matches_oracle():
    # one wedge of the shell of Sec. IV.B, r from 2 to 10 (logarithmic): the
    # operator on its node coordinates, and FGMRES preconditioned by the
    # V-cycle of the logical cube
    announce("curved wedge")
    box = omesh.BoxMesh((-1, -1, -1), (1, 1, 1), (4, 4, 4), 3)
    xyz = W.wedge_coordinates(np.stack(box.node_coordinates()), 2.0, 10.0)
    cm = curved.CurvedMesh(box, xyz)
    prob = _problem(box, mg_levels=2)
    prob.set_geometry(to_gpu(xyz.reshape(-1)))
    u = W.random_normal(56, box.ndof)
    ref = curved.apply_operator(cm, u, C)
    assert rel_max(to_np(prob.apply(to_gpu(u))), ref) < 1e-12
    A = lambda v: curved.apply_operator(cm, v, C)
    b = curved.apply_mass(cm, np.ones(box.ndof)).reshape(-1)
    x_ref, its_ref, _ = krylov.fgmres(A, b, precondition=multigrid.VCycle(box, C, levels=2), rtol=1e-10,
                                      max_iter=100)
    x, st = prob.solve(to_gpu(b))
    x = to_np(x)
    assert st["converged"] and abs(st["iterations"] - its_ref) <= 1, (st["iterations"], its_ref)
    assert np.linalg.norm(b - A(x)) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    prob.close()


def _metric(cm, box, amp):
    """g^ij (as the 6 fields xx, xy, xz, yy, yz, zz) and sqrt(g) of a pullback
    metric at the physical node coordinates, for the oracle and the library."""
    _, G, sg = W.pullback_metric(cm.xyz, box.lower, box.upper, amp)
    six = np.stack([G[0, 0], G[0, 1], G[0, 2], G[1, 1], G[1, 2], G[2, 2]]).reshape(-1)
    return G, sg, six


@pytest.mark.parametrize("elements,p,neumann,geom,amp", [((3, 2, 2), 3, (), 0.1, 0.15),
                                                         ((2, 3, 2), 5, (1, 4), 0.0, 0.2),
                                                         ((2, 2, 2), 7, (0,), 0.05, 0.1),
                                                         ((4, 1, 2), 2, (), 0.12, 0.12)])
def test_metric_apply_matches_oracle(elements, p, neumann, geom, amp):
    # the Laplace-Beltrami operator of a curved background metric (sqrt(g) in
    # M, MD and ML of Sec. II) on curved elements or on the box grid
    announce(f"metric apply elements={elements} p={p} neumann={neumann} geometry={geom} metric={amp}")
    box = omesh.BoxMesh((0, 0, 0), (1.0, 1.1, 0.9), elements, p, neumann=neumann)
    xyz = curved.deformed_box(box, geom)
    cm = curved.CurvedMesh(box, xyz)
    G, sg, six = _metric(cm, box, amp)
    prob = _problem(box, mg_levels=1)
    if geom:
        prob.set_geometry(to_gpu(xyz.reshape(-1)))
    prob.set_metric(to_gpu(six), to_gpu(sg.reshape(-1)))  # box coordinates when geom == 0
    u = W.random_normal(57 + p, box.ndof)
    ref = curved.apply_operator_metric(cm, u, C, G, sg)
    got = to_np(prob.apply(to_gpu(u)))
    assert rel_max(got, ref) < 1e-12, rel_max(got, ref)
    f = W.random_uniform(58, box.ndof)
    ref_m = (sg.reshape(-1) * curved.apply_mass(cm, f).reshape(-1))
    assert rel_max(to_np(prob.apply_mass(to_gpu(f))), ref_m) < 1e-14
    # dropping the metric gives the flat operator of the same elements back
    prob.set_metric(None, None)
    assert rel_max(to_np(prob.apply(to_gpu(u))), curved.apply_operator(cm, u, C)) < 1e-12
    prob.close()


def test_metric_solve_matches_oracle():
    # FGMRES on the metric operator with the flat box V-cycle, on the GPU and
    # in the oracle; then the geometry reset drops the metric too
    announce("metric solve")
    box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (4, 4, 2), 3)
    xyz = curved.deformed_box(box, 0.08)
    cm = curved.CurvedMesh(box, xyz)
    G, sg, six = _metric(cm, box, 0.15)
    X = cm.xyz
    f = np.sin(np.pi * X[0]) * np.sin(np.pi * X[1]) * np.sin(np.pi * X[2])
    b = (sg * curved.apply_mass(cm, f)).reshape(-1)
    A = lambda v: curved.apply_operator_metric(cm, v, C, G, sg)
    x_ref, its_ref, _ = krylov.fgmres(A, b, precondition=multigrid.VCycle(box, C, levels=2),
                                      rtol=1e-10, max_iter=100)
    prob = _problem(box, mg_levels=2)
    prob.set_geometry(to_gpu(xyz.reshape(-1)))
    prob.set_metric(to_gpu(six), to_gpu(sg.reshape(-1)))
    u, st = prob.solve(to_gpu(b))
    u = to_np(u)
    assert st["converged"] and st["rel_residual"] <= 1e-10
    assert abs(st["iterations"] - its_ref) <= 1, (st["iterations"], its_ref)
    assert np.linalg.norm(b - A(u)) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(u - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    prob.set_geometry(None)
    v = W.random_normal(59, box.ndof)
    ref = curved.apply_operator(curved.CurvedMesh(box, np.stack(box.node_coordinates())), v, C)
    assert rel_max(to_np(prob.apply(to_gpu(v))), ref) < 1e-12
    prob.close()


def test_metric_checks():
    import paper_2111_06767_amd as dg
    announce("metric checks")
    box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (2, 1, 1), 2)
    prob = _problem(box, mg_levels=1)
    u = to_gpu(W.random_normal(60, box.ndof))
    flat = to_np(prob.apply(u))
    n = box.ndof
    good = np.concatenate([np.ones(n), np.zeros(n), np.zeros(n), np.ones(n), np.zeros(n), np.ones(n)])
    indefinite = good.copy()
    indefinite[n + 3] = 1.5  # g^xy > sqrt(g^xx g^yy) at one node
    with pytest.raises(dg.DgsError):
        prob.set_metric(to_gpu(indefinite), to_gpu(np.ones(n)))
    bad_root = np.ones(n)
    bad_root[7] = 0.0
    with pytest.raises(dg.DgsError):
        prob.set_metric(to_gpu(good), to_gpu(bad_root))
    with pytest.raises(ValueError):
        prob.set_metric(to_gpu(good), None)
    # refused metrics leave the operator as it was
    assert np.array_equal(to_np(prob.apply(u)), flat)
    # the unit metric on the box coordinates is the box operator
    prob.set_metric(to_gpu(good), to_gpu(np.ones(n)))
    assert rel_max(to_np(prob.apply(u)), flat) < 1e-13
    prob.close()


def _ks_wedge(elements, p):
    box = omesh.BoxMesh((-1, -1, -1), (1, 1, 1), elements, p)
    xyz = W.wedge_coordinates(np.stack(box.node_coordinates()), 2.0, 10.0)
    cm = curved.CurvedMesh(box, xyz)
    G, sg, alpha, coefs, powers = W.kerr_schild_lapse(cm.xyz)
    six = np.stack([G[0, 0], G[0, 1], G[0, 2], G[1, 1], G[1, 2], G[2, 2]]).reshape(-1)
    return box, cm, G, sg, six, alpha.reshape(-1), coefs, powers


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_kerr_schild_lapse_newton_matches_oracle(precision):
    # the XCTS lapse equation on the Kerr-Schild background (psi = 1, shift
    # fixed) on a wedge from r = 2M to 10M, Dirichlet data from the analytic
    # lapse, flat initial guess: Newton with the power-law source on the GPU
    # against the oracle's Newton with the same V-cycle
    announce(f"kerr-schild lapse newton 2x2x2 p=4 {precision}")
    box, cm, G, sg, six, alpha, coefs, powers = _ks_wedge((2, 2, 2), 4)
    u_ref, info = onewton.newton_solve_powers(cm, C, coefs, powers, ginv=G, sqrtg=sg, dirichlet=alpha,
                                              newton_rtol=1e-10, linear_rtol=1e-4, levels=2,
                                              subdomain_iters=3)
    prob = _problem(box, mg_levels=2, subdomain_iters=3, precision=precision)
    prob.set_geometry(to_gpu(cm.xyz.reshape(-1)))
    prob.set_metric(to_gpu(six), to_gpu(sg.reshape(-1)))
    u, st = prob.newton_solve_powers(to_gpu(coefs.reshape(-1)), powers, dirichlet=to_gpu(alpha),
                                     newton_rtol=1e-10, linear_rtol=1e-4)
    u = to_np(u)
    assert st["converged"], st
    # the oracle's own nonlinear residual of the GPU solution
    Mg = (sg * curved.mass_diagonal(cm)).reshape(-1)
    cf = [c.reshape(-1) for c in coefs]
    F = lambda v: (curved.apply_operator_metric(cm, v, C, G, sg, dirichlet_values=alpha)
                   + Mg * onewton.power_source(cf, powers, v)[0])
    assert np.linalg.norm(F(u)) <= 1e-10 * np.linalg.norm(F(np.ones(box.ndof)))
    assert np.linalg.norm(u - u_ref) <= 1e-9 * np.linalg.norm(u_ref)
    if precision == "fp64":
        assert st["newton_steps"] == info["steps"]
    assert np.abs(u - alpha).max() < 1e-4  # the discretisation error at p = 4


def test_power_source_newton_on_box_coordinates():
    # -Laplace(u) + u^3 - 2 u^-2 = f on the box with its own coordinates as
    # curved elements, Dirichlet data u_b = 1 + x y z, homogeneous Neumann on
    # one face, the right-hand side b = M f given
    announce("power-source newton on box coordinates")
    box = omesh.BoxMesh((0, 0, 0), (1, 1.2, 0.9), (3, 2, 2), 3, neumann=(1,))
    X = np.stack(box.node_coordinates())
    cm = curved.CurvedMesh(box, X)
    ub = (1.0 + X[0] * X[1] * X[2]).reshape(-1)
    coefs = np.stack([np.ones(box.ndof), -2.0 * np.ones(box.ndof)])
    f = W.random_uniform(70, box.ndof, 0.5, 1.5)
    b = curved.apply_mass(cm, f).reshape(-1)
    u_ref, info = onewton.newton_solve_powers(cm, C, coefs, (3, -2), dirichlet=ub, b=b, levels=2,
                                              subdomain_iters=3)
    prob = _problem(box, mg_levels=2, subdomain_iters=3)
    prob.set_geometry(to_gpu(X.reshape(-1)))
    u, st = prob.newton_solve_powers(to_gpu(coefs.reshape(-1)), (3, -2), dirichlet=to_gpu(ub), b=to_gpu(b))
    assert st["converged"] and st["newton_steps"] == info["steps"], (st, info["steps"])
    assert np.linalg.norm(to_np(u) - u_ref) <= 1e-9 * np.linalg.norm(u_ref)


def test_power_source_checks():
    import paper_2111_06767_amd as dg
    announce("power-source newton checks")
    box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (2, 1, 1), 2)
    prob = _problem(box, mg_levels=1)
    n = box.ndof
    coef = to_gpu(np.ones(n))
    with pytest.raises(dg.DgsError):  # no curved elements yet
        prob.newton_solve_powers(coef, (1,))
    prob.set_geometry(to_gpu(np.stack(box.node_coordinates()).reshape(-1)))
    with pytest.raises(dg.DgsError):
        prob.newton_solve_powers(coef, (13,))
    with pytest.raises(dg.DgsError):
        prob.newton_solve_powers(to_gpu(np.ones(9 * n)), (1,) * 9)
    with pytest.raises(dg.DgsError):  # u = 0 under a negative power
        prob.newton_solve_powers(coef, (-1,), u=to_gpu(np.zeros(n)))
    prob.close()


def _xcts_system(elements, p):
    mp = omesh.BoxMesh((-1, -1, -1), (1, 1, 1), elements, p, neumann=(4,))  # n.grad psi = 0 at r = 2M
    mf = omesh.BoxMesh((-1, -1, -1), (1, 1, 1), elements, p)
    xyz = W.wedge_coordinates(np.stack(mp.node_coordinates()), 2.0, 10.0)
    G, sg, alpha, terms = W.kerr_schild_xcts(xyz)
    six = np.stack([G[0, 0], G[0, 1], G[0, 2], G[1, 1], G[1, 2], G[2, 2]]).reshape(-1)
    ub = np.stack([np.ones(mp.ndof), alpha.reshape(-1)])
    vars_ = [a for a in range(2) for _ in terms[a]]
    powers = [k for a in range(2) for _, k in terms[a]]
    coef = np.concatenate([np.asarray(c, float).reshape(-1) for a in range(2) for c, _ in terms[a]])
    return mp, mf, xyz, G, sg, six, alpha.reshape(-1), terms, ub, vars_, powers, coef


def _gpu_system(mp, precision, **opts):
    import paper_2111_06767_amd as dg
    return dg.System(tuple(mp.lower), tuple(mp.upper), mp.n, mp.p, [(4,), ()], laplacian_bc="matched",
                     penalty=C, precision=precision, **opts)


def test_system_curved_apply_matches_oracle():
    # the system operator on curved elements and the metric: each variable's
    # metric operator with its own boundary faces, plus pointwise couplings
    announce("system apply on a metric")
    mp, mf, xyz, G, sg, six, alpha, terms, ub, vars_, powers, coef = _xcts_system((2, 2, 2), 3)
    n = mp.ndof
    S = _gpu_system(mp, "fp64", mg_levels=1)
    S.set_geometry(to_gpu(xyz.reshape(-1)))
    S.set_metric(to_gpu(six), to_gpu(sg.reshape(-1)))
    D = W.random_uniform(71, 4 * n, 0.0, 2.0)
    S.set_coupling(to_gpu(D))
    u = W.random_normal(72, 2 * n)
    cms = [curved.CurvedMesh(mp, xyz), curved.CurvedMesh(mf, xyz)]
    ref = np.concatenate([curved.apply_operator_metric(cms[a], u[a * n:(a + 1) * n], C, G, sg) for a in range(2)])
    ref += np.einsum("abn,bn->an", D.reshape(2, 2, n), u.reshape(2, n)).reshape(-1)
    assert rel_max(to_np(S.apply(to_gpu(u))), ref) < 1e-12
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_xcts_hamiltonian_and_lapse_match_oracle(precision):
    # psi and alpha psi of the XCTS system (eqs. xcts_hamiltonian, xcts_lapse)
    # on the Kerr-Schild background with the shift fixed, on a wedge from 2M
    # to 10M: Neumann psi at the inner sphere, Dirichlet data elsewhere, flat
    # initial guess; the system Newton on the GPU against the oracle's
    announce(f"xcts hamiltonian + lapse 2x2x2 p=3 {precision}")
    mp, mf, xyz, G, sg, six, alpha, terms, ub, vars_, powers, coef = _xcts_system((2, 2, 2), 3)
    n = mp.ndof
    u_ref, info = onewton.system_newton_solve_powers([mp, mf], xyz, C, terms, ginv=G, sqrtg=sg, dirichlet=ub,
                                                     levels=2, subdomain_iters=3)
    S = _gpu_system(mp, precision, mg_levels=2, subdomain_iters=3)
    S.set_geometry(to_gpu(xyz.reshape(-1)))
    S.set_metric(to_gpu(six), to_gpu(sg.reshape(-1)))
    u, st = S.newton_solve_powers(to_gpu(coef), vars_, powers, dirichlet=to_gpu(ub.reshape(-1)))
    u = to_np(u).reshape(2, n)
    assert st["converged"], st
    if precision == "fp64":
        assert st["newton_steps"] == info["steps"], (st["newton_steps"], info["steps"])
    assert np.linalg.norm(u - u_ref) <= 1e-9 * np.linalg.norm(u_ref)
    # the oracle's own nonlinear residual of the GPU solution
    cms = [curved.CurvedMesh(mp, xyz), curved.CurvedMesh(mf, xyz)]
    Mg = (sg * curved.mass_diagonal(cms[0])).reshape(-1)

    def F(v):
        Av = np.stack([curved.apply_operator_metric(cms[a], v[a], C, G, sg, dirichlet_values=ub[a])
                       for a in range(2)])
        return Av + Mg * onewton.monomial_source(terms, v)[0]

    assert np.linalg.norm(F(u)) <= 1e-10 * np.linalg.norm(F(np.ones((2, n))))
    assert np.abs(u[0] - 1.0).max() < 1e-5 and np.abs(u[1] - alpha).max() < 1e-3
    S.close()


def test_system_newton_checks():
    import paper_2111_06767_amd as dg
    announce("system newton checks")
    mp = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (2, 1, 1), 2)
    S = _gpu_system(mp, "fp64", mg_levels=1)
    n = mp.ndof
    coef = to_gpu(np.ones(n))
    with pytest.raises(dg.DgsError):  # no curved elements yet
        S.newton_solve_powers(coef, [0], [(1, 0)])
    S.set_geometry(to_gpu(np.stack(mp.node_coordinates()).reshape(-1)))
    with pytest.raises(dg.DgsError):  # variable out of range
        S.newton_solve_powers(coef, [2], [(1, 0)])
    with pytest.raises(dg.DgsError):  # power out of range
        S.newton_solve_powers(coef, [0], [(13, 0)])
    S.close()


def _sampled_patches(n, seed, count=6):
    rng = np.random.default_rng(seed)
    samples = [np.array(c) for c in [(0, 0, 0), (n - 1, n - 1, n - 1), (0, n // 2, n - 1), (n // 3, 0, 2)]]
    return samples + [rng.integers(0, n, 3) for _ in range(count)]


@pytest.mark.parametrize("case", ["deformed_pullback", "wedge_kerr_schild"])
def test_metric_apply_full_size_sampled(case):
    # the 16^3, p = 7 grids of the benchmark's metric and lapse legs: the GPU
    # operator on the whole grid, the oracle on the 3 x 3 x 3 patch of elements
    # around each sampled element (its result depends only on the element and
    # its face neighbours)
    n, p = 16, 7
    N = p + 1
    announce(f"metric apply 16^3 p=7 sampled, {case}")
    if case == "deformed_pullback":
        box = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (n, n, n), p)
        xyz = curved.deformed_box(box, 0.1)
        _, G, sg = W.pullback_metric(xyz, box.lower, box.upper, 0.15)
    else:
        box = omesh.BoxMesh((-1, -1, -1), (1, 1, 1), (n, n, n), p)
        xyz = W.wedge_coordinates(np.stack(box.node_coordinates()), 2.0, 10.0).reshape(3, box.E, N, N, N)
        G, sg, _, _, _ = W.kerr_schild_lapse(xyz)
    six = np.stack([G[0, 0], G[0, 1], G[0, 2], G[1, 1], G[1, 2], G[2, 2]]).reshape(-1)
    prob = _problem(box, mg_levels=1)
    prob.set_geometry(to_gpu(xyz.reshape(-1)))
    prob.set_metric(to_gpu(six), to_gpu(sg.reshape(-1)))
    u = W.random_normal(73, box.ndof)
    got = to_np(prob.apply(to_gpu(u))).reshape(n, n, n, N, N, N)
    prob.close()
    ug = u.reshape(n, n, n, N, N, N)
    xg = xyz.reshape(3, n, n, n, N, N, N)
    Gg = G.reshape(3, 3, n, n, n, N, N, N)
    sgg = sg.reshape(n, n, n, N, N, N)
    hx = (box.upper - box.lower) / n
    for c in _sampled_patches(n, 2):
        lo = np.maximum(c - 1, 0)
        hi = np.minimum(c + 2, n)
        sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
        pm = omesh.BoxMesh(box.lower + lo * hx, box.lower + hi * hx, tuple(hi - lo), p)
        pxyz = xg[(slice(None),) + sl].reshape(3, -1, N, N, N)
        pcm = curved.CurvedMesh(pm, pxyz)
        pG = Gg[(slice(None), slice(None)) + sl].reshape(3, 3, -1, N, N, N)
        psg = sgg[sl].reshape(-1, N, N, N)
        ref = curved.apply_operator_metric(pcm, ug[sl].reshape(-1), C, pG, psg).reshape(-1, N, N, N)
        e = pm.elem_index(*(c - lo))
        assert rel_max(got[c[2], c[1], c[0]], ref[e]) < 1e-12, (case, c)


def test_xcts_matched_laplacian_approximation_needs_fewer_iterations():
    # Sec. III.E.1: subdomain preconditioners with each variable's own
    # boundary types (psi Neumann at the inner sphere) against all-Dirichlet
    # ones, one subdomain GMRES iteration: the same discrete solution, fewer
    # outer iterations with the matched types
    announce("xcts matched vs dirichlet laplacian approximation 4x4x4 p=5")
    mp, mf, xyz, G, sg, six, alpha, terms, ub, vars_, powers, coef = _xcts_system((4, 4, 4), 5)
    its, sols = {}, {}
    for bc in ("matched", "dirichlet"):
        import paper_2111_06767_amd as dg
        S = dg.System(tuple(mp.lower), tuple(mp.upper), mp.n, mp.p, [(4,), ()], laplacian_bc=bc, penalty=C,
                      mg_levels=2, subdomain_iters=1)
        S.set_geometry(to_gpu(xyz.reshape(-1)))
        S.set_metric(to_gpu(six), to_gpu(sg.reshape(-1)))
        u, st = S.newton_solve_powers(to_gpu(coef), vars_, powers, dirichlet=to_gpu(ub.reshape(-1)))
        assert st["converged"] and st["newton_steps"] == 3, st
        its[bc], sols[bc] = st["iterations"], to_np(u)
        S.close()
    assert its["matched"] < its["dirichlet"], its
    assert np.linalg.norm(sols["matched"] - sols["dirichlet"]) <= 1e-9 * np.linalg.norm(sols["dirichlet"])


def test_kerr_schild_full_size_solutions_match_the_analytic_ones():
    # at the benchmark's 16^3 grids of the wedge, the Newton solutions of the
    # lapse equation (p = 7) and of the Hamiltonian + lapse system (p = 5)
    # equal the analytic Kerr-Schild solution (eqs. kerrschild_psi,
    # kerrschild_lapse) to the discretisation error, far below 1e-8
    import paper_2111_06767_amd as dg
    announce("kerr-schild lapse 16^3 p=7 and xcts system 16^3 p=5 against the analytic solution")
    box = omesh.BoxMesh((-1, -1, -1), (1, 1, 1), (16, 16, 16), 7)
    xyz = W.wedge_coordinates(np.stack(box.node_coordinates()), 2.0, 10.0)
    G, sg, alpha, coefs, powers = W.kerr_schild_lapse(xyz)
    six = np.stack([G[0, 0], G[0, 1], G[0, 2], G[1, 1], G[1, 2], G[2, 2]]).reshape(-1)
    prob = _problem(box, mg_levels=4, subdomain_iters=3)
    prob.set_geometry(to_gpu(xyz.reshape(-1)))
    prob.set_metric(to_gpu(six), to_gpu(sg.reshape(-1)))
    u, st = prob.newton_solve_powers(to_gpu(coefs.reshape(-1)), powers, dirichlet=to_gpu(alpha.reshape(-1)))
    prob.close()
    assert st["converged"] and st["newton_steps"] <= 4, st
    assert np.abs(to_np(u) - alpha.reshape(-1)).max() < 1e-8
    mp, mf, xyz2, G2, sg2, six2, alpha2, terms, ub, vars_, pw, coef = _xcts_system((16, 16, 16), 5)
    S = dg.System(tuple(mp.lower), tuple(mp.upper), mp.n, mp.p, [(4,), ()], laplacian_bc="matched", penalty=C,
                  mg_levels=4, subdomain_iters=1)
    S.set_geometry(to_gpu(xyz2.reshape(-1)))
    S.set_metric(to_gpu(six2), to_gpu(sg2.reshape(-1)))
    v, st = S.newton_solve_powers(to_gpu(coef), vars_, pw, dirichlet=to_gpu(ub.reshape(-1)))
    S.close()
    v = to_np(v).reshape(2, -1)
    assert st["converged"] and st["newton_steps"] <= 4, st
    assert np.abs(v[0] - 1.0).max() < 1e-8 and np.abs(v[1] - alpha2).max() < 1e-8
