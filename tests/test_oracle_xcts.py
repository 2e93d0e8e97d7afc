"""Pins of the oracle's Newton solve with a power-law source on curved
elements (Sec. III.A on the curved operator of Sec. II), on the lapse
equation of the XCTS system (eq. xcts_lapse) for a Schwarzschild black hole
in Kerr-Schild coordinates (eqs. kerrschild_bg, kerrschild_lapse,
kerrschild_shift) on one wedge of the shell of Sec. IV.B: the discrete
solution converges exponentially to the analytic lapse, the Krylov-based
Newton reaches the same discrete solution as one with dense linear solves,
and an affine source takes one Newton step to the linear solution.  The
coupled Hamiltonian and lapse equations (eqs. xcts_hamiltonian, xcts_lapse)
for psi and alpha psi, with the paper's Neumann condition on psi at the
inner sphere, converge to psi = 1, alpha psi = alpha (eq. kerrschild_psi)."""
import numpy as np

import workloads as W
from oracle import curved, mesh as omesh, newton

C = 1.5


def _wedge(elements, p):
    box = omesh.BoxMesh((-1, -1, -1), (1, 1, 1), elements, p)
    xyz = W.wedge_coordinates(np.stack(box.node_coordinates()), 2.0, 10.0)
    return curved.CurvedMesh(box, xyz)


def _lapse(cm, **kw):
    G, sg, alpha, coefs, powers = W.kerr_schild_lapse(cm.xyz)
    u, info = newton.newton_solve_powers(cm, C, coefs, powers, ginv=G, sqrtg=sg,
                                         dirichlet=alpha.reshape(-1), **kw)
    return u, alpha.reshape(-1), info


def test_kerr_schild_lapse_converges_to_the_analytic_lapse():
    # Dirichlet data from the analytic lapse on every face of the wedge (r from
    # 2M to 10M); flat initial guess Phi = 1
    errs = []
    for p in (2, 3, 4, 5):
        cm = _wedge((1, 1, 2), p)
        u, alpha, info = _lapse(cm, levels=2)
        assert info["history"][-1] <= 1e-10 and info["steps"] <= 6, info
        errs.append(np.abs(u - alpha).max())
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[0] / errs[-1] > 300, errs


def test_krylov_newton_reaches_the_dense_newton_solution():
    cm = _wedge((1, 1, 2), 3)
    u_k, _, info_k = _lapse(cm, levels=2)
    u_d, _, info_d = _lapse(cm, dense=True)
    assert np.abs(u_k - u_d).max() <= 1e-9 * np.abs(u_d).max()
    assert abs(info_k["steps"] - info_d["steps"]) <= 1


def test_affine_source_takes_one_newton_step():
    # S(u) = c (power 0): F is affine in u, so one full Newton step with a
    # dense solve is the linear solution A(u; u_b) + M c = b
    cm = _wedge((1, 1, 1), 3)
    G, sg, alpha, coefs, _ = W.kerr_schild_lapse(cm.xyz)
    n = cm.ndof
    c = coefs[2].reshape(-1)
    ub = alpha.reshape(-1)
    u, info = newton.newton_solve_powers(cm, C, [c], (0,), ginv=G, sqrtg=sg, dirichlet=ub,
                                         dense=True, newton_rtol=1e-12)
    assert info["steps"] == 1 and info["history"][-1] <= 1e-12
    A = lambda v: curved.apply_operator_metric(cm, v, C, G, sg)
    Ad = np.stack([A(e) for e in np.eye(n)], axis=1)
    g = curved.apply_operator_metric(cm, np.zeros(n), C, G, sg, dirichlet_values=ub)
    Mg = (sg * curved.mass_diagonal(cm)).reshape(-1)
    assert np.abs(u - np.linalg.solve(Ad, -g - Mg * c)).max() <= 1e-10


def _xcts2(elements, p):
    mp = omesh.BoxMesh((-1, -1, -1), (1, 1, 1), elements, p, neumann=(4,))  # n.grad psi = 0 at r = 2M
    mf = omesh.BoxMesh((-1, -1, -1), (1, 1, 1), elements, p)
    xyz = W.wedge_coordinates(np.stack(mp.node_coordinates()), 2.0, 10.0)
    G, sg, alpha, terms = W.kerr_schild_xcts(xyz)
    ub = np.stack([np.ones(mp.ndof), alpha.reshape(-1)])
    return [mp, mf], xyz, G, sg, alpha.reshape(-1), terms, ub


def test_hamiltonian_and_lapse_converge_to_the_kerr_schild_solution():
    e_psi, e_phi = [], []
    for p in (2, 3, 4, 5):
        meshes, xyz, G, sg, alpha, terms, ub = _xcts2((1, 1, 2), p)
        u, info = newton.system_newton_solve_powers(meshes, xyz, C, terms, ginv=G, sqrtg=sg, dirichlet=ub,
                                                    levels=2)
        assert info["history"][-1] <= 1e-10 and info["steps"] <= 6, info
        e_psi.append(np.abs(u[0] - 1.0).max())
        e_phi.append(np.abs(u[1] - alpha).max())
    for errs in (e_psi, e_phi):
        assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert e_psi[0] / e_psi[-1] > 1e3 and e_phi[0] / e_phi[-1] > 300, (e_psi, e_phi)


def test_system_newton_reaches_the_dense_newton_solution():
    meshes, xyz, G, sg, alpha, terms, ub = _xcts2((1, 1, 2), 2)
    kw = dict(ginv=G, sqrtg=sg, dirichlet=ub)
    u_k, info_k = newton.system_newton_solve_powers(meshes, xyz, C, terms, levels=2, **kw)
    u_d, info_d = newton.system_newton_solve_powers(meshes, xyz, C, terms, dense=True, **kw)
    assert np.abs(u_k - u_d).max() <= 1e-9 * np.abs(u_d).max()
    assert abs(info_k["steps"] - info_d["steps"]) <= 1


def test_monomial_derivatives_match_finite_differences():
    _, _, _, _, _, terms, _ = _xcts2((1, 1, 1), 2)
    rng = np.random.default_rng(3)
    u = rng.uniform(0.7, 1.3, size=(2, 27))
    S, D = newton.monomial_source(terms, u)
    for b in range(2):
        h = 1e-6
        up, um = u.copy(), u.copy()
        up[b] += h
        um[b] -= h
        fd = (newton.monomial_source(terms, up)[0] - newton.monomial_source(terms, um)[0]) / (2 * h)
        assert np.abs(fd - D[:, b]).max() <= 1e-6 * np.abs(D[:, b]).max()
