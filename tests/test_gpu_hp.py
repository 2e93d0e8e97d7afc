"""GPU parity of hp-nonuniform meshes against the oracle, through the C ABI:
the operator with mortars on nonconforming faces (Sec. II), the mass and the
node coordinates, Schwarz steps with the inverses of subdomains that reach
into finer and coarser neighbours (Sec. III.D), the V-cycle whose coarse
levels keep the smaller degree (Sec. III.C.1), and FGMRES solves."""
import numpy as np
import pytest

import workloads as W
from oracle import hp, krylov
from tests.gpu_util import announce, rel_max, to_gpu, to_np

pytestmark = pytest.mark.gpu

C = 1.5

# block grid, block levels, upper corner of the box (lower corner at 0)
MESHES = {
    # the right element meets four smaller ones across its -x face
    "two_blocks": ((2, 1, 1), [(1, 1, 1), (0, 0, 0)], (2, 1.5, 1)),
    # anisotropic levels: split along some dimensions only
    "aniso": ((2, 2, 1), [(1, 0, 1), (0, 1, 0), (1, 1, 0), (0, 0, 1)], (2, 1.5, 1)),
    "one_block": ((1, 1, 1), [(1, 2, 1)], (1, 1.3, 0.8)),
    # 64 small elements against 8 larger ones, three multigrid levels
    "big_small": ((2, 1, 1), [(1, 1, 1), (2, 2, 2)], (2, 1, 1)),
}


def _mesh(name, seed, lo=2, hi=5, neumann=()):
    blocks, levels, upper = MESHES[name]
    E = sum(2 ** sum(lv) for lv in levels)
    deg = np.random.default_rng(seed).integers(lo, hi, size=(E, 3))
    return hp.HpMesh((0, 0, 0), upper, blocks, levels, deg, neumann=neumann), deg


def _gpu(m, deg, **opts):
    import paper_2111_06767_amd as dg
    return dg.HpProblem(tuple(m.lower), tuple(m.upper), m.blocks, m.block_levels.tolist(), deg.tolist(),
                        penalty=C, neumann_faces=sum(1 << f for f in m.neumann), **opts)


@pytest.mark.parametrize("name,seed,lo,hi,neumann", [
    ("two_blocks", 0, 2, 5, ()), ("two_blocks", 1, 5, 8, (0, 3)), ("aniso", 2, 1, 4, ()),
    ("aniso", 3, 2, 6, (5,)), ("one_block", 4, 2, 5, (1,)), ("big_small", 5, 1, 4, ()),
])
def test_hp_apply_mass_and_coordinates_match_oracle(name, seed, lo, hi, neumann):
    announce(f"hp apply {name} seed={seed} degrees [{lo},{hi}) neumann={neumann}")
    m, deg = _mesh(name, seed, lo, hi, neumann)
    prob = _gpu(m, deg, mg_levels=1)
    assert prob.ndof == m.ndof
    assert np.abs(to_np(prob.node_coordinates()) - m.node_coordinates()).max() <= 1e-15
    u = W.random_normal(60 + seed, m.ndof)
    ref = hp.apply_operator(m, u, C)
    got = to_np(prob.apply(to_gpu(u)))
    assert rel_max(got, ref) < 1e-12, rel_max(got, ref)
    f = W.random_uniform(61 + seed, m.ndof)
    assert rel_max(to_np(prob.apply_mass(to_gpu(f))), hp.apply_mass(m, f)) < 1e-15
    prob.close()


@pytest.mark.parametrize("name,seed,overlap", [("two_blocks", 6, 2), ("aniso", 7, 1), ("aniso", 8, 3)])
def test_hp_schwarz_steps_match_oracle(name, seed, overlap):
    announce(f"hp schwarz {name} overlap={overlap}")
    m, deg = _mesh(name, seed)
    sm = hp.HpSchwarzSmoother(m, C, overlap=overlap)
    b = W.random_normal(62, m.ndof)
    u0 = W.random_uniform(63, m.ndof)
    ref = sm.smooth(u0, b, 2)
    prob = _gpu(m, deg, mg_levels=1, overlap=overlap)
    u = to_gpu(u0)
    prob.smooth(to_gpu(b), u, 2)
    got = to_np(u)
    assert rel_max(got, ref) < 1e-10, rel_max(got, ref)
    prob.close()


@pytest.mark.parametrize("name,seed,levels", [("two_blocks", 9, 2), ("big_small", 10, 3)])
def test_hp_vcycle_matches_oracle(name, seed, levels):
    announce(f"hp vcycle {name} levels={levels}")
    m, deg = _mesh(name, seed, 2, 4)
    cyc = hp.HpVCycle(m, C, levels=levels)
    r = W.random_normal(64, m.ndof)
    ref = cyc(r)
    prob = _gpu(m, deg, mg_levels=levels)
    assert prob.levels == len(cyc.meshes)
    got = to_np(prob.precondition(to_gpu(r)))
    assert rel_max(got, ref) < 1e-10, rel_max(got, ref)
    prob.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_hp_solve_matches_oracle(precision):
    # mixed precision: FP32 subdomain solves on the finer levels; FGMRES still
    # converges to the same solution
    announce(f"hp solve big_small {precision}")
    m, deg = _mesh("big_small", 11, 2, 4)
    cyc = hp.HpVCycle(m, C, levels=3)
    A = cyc.smoothers[0].A
    x, y, z = m.node_coordinates()
    b = hp.apply_mass(m, W.sin_product_source(x / 2, y, z))
    x_ref, its_ref, _ = krylov.fgmres(lambda v: A @ v, b, precondition=cyc, rtol=1e-10)
    prob = _gpu(m, deg, mg_levels=3, precision=precision)
    u, st = prob.solve(to_gpu(b))
    u = to_np(u)
    assert st["converged"] and st["rel_residual"] <= 1e-10
    assert abs(st["iterations"] - its_ref) <= 1, (st["iterations"], its_ref)
    assert np.linalg.norm(b - A @ u) <= 1e-10 * np.linalg.norm(b)
    assert np.linalg.norm(u - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    prob.close()


def test_graph_replays_match_the_eager_cycle():
    # the V-cycle captured at set-up, replayed several times with other work
    # and synchronisations in between, equals the launches made one by one
    import torch
    announce("hp graph replays")
    m, deg = _mesh("two_blocks", 12, 2, 4)
    g = _gpu(m, deg, mg_levels=2)
    e = _gpu(m, deg, mg_levels=2, use_graphs=0)
    for seed in (66, 67, 68):
        r = to_gpu(W.random_normal(seed, m.ndof))
        zg = g.precondition(r)
        g.apply(r)
        torch.cuda.synchronize()
        ze = e.precondition(r)
        assert torch.equal(zg, ze)
    g.close()
    e.close()


def test_equal_subdomains_share_an_inverse():
    # one cube of 4 x 4 x 4 elements of one degree: up to mirrors and axis
    # exchanges the subdomains are interior, face, edge or corner ones
    announce("hp classes")
    m = hp.HpMesh((0, 0, 0), (1, 1, 1), (1, 1, 1), [(2, 2, 2)], np.full((64, 3), 3))
    prob = _gpu(m, np.full((64, 3), 3), mg_levels=1)
    assert prob.num_classes(0) == 4
    b = W.random_normal(65, m.ndof)
    ref = hp.HpSchwarzSmoother(m, C).smooth(np.zeros(m.ndof), b, 1)
    u = to_gpu(np.zeros(m.ndof))
    prob.smooth(to_gpu(b), u, 1)
    assert rel_max(to_np(u), ref) < 1e-10
    prob.close()


def test_hp_limits():
    import paper_2111_06767_amd as dg
    announce("hp limits")
    with pytest.raises(dg.DgsError):  # degree 8
        dg.HpProblem((0, 0, 0), (1, 1, 1), (1, 1, 1), [(0, 0, 0)], [(8, 2, 2)])
    with pytest.raises(dg.DgsError):  # levels 2 against 0 across a face
        dg.HpProblem((0, 0, 0), (2, 1, 1), (2, 1, 1), [(2, 2, 2), (0, 0, 0)], [(2, 2, 2)] * 65)
    with pytest.raises(dg.DgsError):  # element count
        dg.HpProblem((0, 0, 0), (2, 1, 1), (2, 1, 1), [(1, 1, 1), (0, 0, 0)], [(2, 2, 2)] * 8)
    with pytest.raises(dg.DgsError):  # the V-cycle only
        dg.HpProblem((0, 0, 0), (1, 1, 1), (1, 1, 1), [(0, 0, 0)], [(2, 2, 2)], cycle=2)


def test_hp_checkerboard_full_size():
    # the benchmark's hp workload (2 x 2 x 2 blocks in a checkerboard of 8^3
    # elements of degree 5 and 4^3 of degree 7: every block face nonconforming
    # in h and p; 573,440 points): the operator against the oracle's on the
    # whole mesh, and FP64 and mixed solves through the oracle's operator
    import paper_2111_06767_amd as dg
    announce("hp checkerboard full size")
    levels, degrees = [], []
    for b in range(8):
        fine = (b % 2 + (b // 2) % 2 + b // 4) % 2 == 0
        L = 3 if fine else 2
        levels.append((L, L, L))
        degrees += [(5, 5, 5) if fine else (7, 7, 7)] * (8 ** L)
    m = hp.HpMesh((0, 0, 0), (1, 1, 1), (2, 2, 2), levels, np.asarray(degrees))
    u = W.random_normal(74, m.ndof)
    x, y, z = m.node_coordinates()
    b = hp.apply_mass(m, W.sin_product_source(x, y, z))
    for precision in ("fp64", "mixed"):
        prob = dg.HpProblem((0, 0, 0), (1, 1, 1), (2, 2, 2), levels, degrees, penalty=C, mg_levels=4,
                            precision=precision)
        assert prob.ndof == m.ndof == 573440
        if precision == "fp64":
            got = to_np(prob.apply(to_gpu(u)))
            assert rel_max(got, hp.apply_operator(m, u, C)) < 1e-12
        sol, st = prob.solve(to_gpu(b))
        prob.close()
        assert st["converged"] and st["iterations"] <= 15, st
        r = b - hp.apply_operator(m, to_np(sol), C)
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b), precision
