"""GPU tests of the continuous-batching server: on the per-request path
every request's result is bit-identical alone and in a mix; on the
cross-request batched path (one launch per phase over all active requests)
every result matches its solo solve to the solution tolerance; admission
respects the device budget, and results satisfy the oracle's DG equations."""
import numpy as np
import pytest

import workloads as W
from oracle import mesh as omesh, operator as oop
from tests.gpu_util import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu

REQS = [((2, 3, 2), 3, 1.0), ((3, 2, 2), 4, 2.0), ((2, 2, 2), 5, 1.0), ((4, 2, 3), 3, 3.0),
        ((2, 2, 3), 6, 4.0), ((3, 3, 3), 4, 2.0)]


def _f(elements, p, side, seed):
    import paper_2111_06767_amd as dg
    modes = W.fourier_modes(seed, (0, 0, 0), (side, side, side))
    xyz = dg.points((0, 0, 0), (side,) * 3, elements, p)
    return W.fourier_source(modes, *xyz)


def _alone(elements, p, side, f, **opts):
    import torch
    import paper_2111_06767_amd as dg
    prob = dg.Problem((0, 0, 0), (side,) * 3, elements, p, **opts)
    b = prob.apply_mass(to_gpu(f))
    u, st = prob.solve(b, torch.zeros_like(b))
    return to_np(u), st


@pytest.mark.parametrize("host_threads", [1, 3])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mix_equals_alone(precision, host_threads):
    """Requests advanced by one host thread, or by three worker threads
    sharing the stages, give the bits of a solo solve."""
    import paper_2111_06767_amd as dg
    announce(f"serving mix vs alone {precision} host_threads={host_threads}")
    srv = dg.Server(hbm_budget_bytes=32e9, max_active=4, precision=precision, max_iter=60,
                    host_threads=host_threads, batched=False)
    ids = {}
    for i, (el, p, side) in enumerate(REQS):
        f = _f(el, p, side, 1000 + i)
        ids[srv.submit((0, 0, 0), (side,) * 3, el, p, f)] = (el, p, side, f)
    active_seen = 0
    while True:
        a, q = srv.step()
        active_seen = max(active_seen, a)
        if a == 0 and q == 0:
            break
    assert active_seen > 1  # requests really overlapped
    for rid in srv.finished():
        u, st, times = srv.fetch(rid)
        el, p, side, f = ids[rid]
        ua, sta = _alone(el, p, side, f, precision=precision, max_iter=60)
        assert st["converged"] and st["rel_residual"] <= 1e-10
        assert st["iterations"] == sta["iterations"]
        assert np.array_equal(u, ua), (rid, np.abs(u - ua).max())
        assert times[0] <= times[1] <= times[2]


def test_admission_by_budget_and_rejection():
    import paper_2111_06767_amd as dg
    announce("serving admission")
    # budget for about one 2x2x2 p=4 request at a time
    one = 2 * 2 * 2 * 125 * 8 * (2 * 40 + 1 + 2 + 4 + 16)
    srv = dg.Server(hbm_budget_bytes=1.5 * one, max_active=8, max_iter=40)
    for i in range(3):
        srv.submit((0, 0, 0), (1, 1, 1), (2, 2, 2), 4, _f((2, 2, 2), 4, 1.0, 2000 + i))
    big = srv.submit((0, 0, 0), (1, 1, 1), (4, 4, 4), 4, _f((4, 4, 4), 4, 1.0, 2100))
    while True:
        a, q = srv.step()
        assert a <= 1
        if a == 0 and q == 0:
            break
    done = srv.finished()
    assert len(done) == 4
    for rid in done:
        if rid == big:
            with pytest.raises(dg.DgsError) as ei:
                srv.fetch(rid)
            assert ei.value.code == dg.DGS_ERR_OOM
        else:
            u, st, _ = srv.fetch(rid)
            assert st["converged"]


def test_served_result_solves_oracle_equations():
    import paper_2111_06767_amd as dg
    announce("serving vs oracle residual")
    el, p, side = (3, 2, 2), 4, 2.0
    f = _f(el, p, side, 3000)
    srv = dg.Server(max_active=2)
    rid = srv.submit((0, 0, 0), (side,) * 3, el, p, f)
    while srv.step() != (0, 0):
        pass
    u, st, _ = srv.fetch(rid)
    m = omesh.BoxMesh((0, 0, 0), (side,) * 3, el, p)
    b = oop.apply_mass(m, f.reshape(m.E, m.N, m.N, m.N)).reshape(-1)
    r = b - oop.apply_operator(m, u.reshape(m.E, m.N, m.N, m.N), 1.5).reshape(-1)
    assert np.linalg.norm(r) / np.linalg.norm(b) <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_puncture_requests_in_a_mix_equal_newton_alone(precision):
    """Nonlinear puncture requests (Newton steps as stages) served beside
    Poisson requests give the bits of a solo dgs_newton_solve, and their
    solutions satisfy the oracle's nonlinear DG equations."""
    import paper_2111_06767_amd as dg
    from oracle import newton as onewton
    from tests.test_gpu_newton import _puncture
    announce(f"serving puncture + Poisson mix {precision}")
    opts = dict(precision=precision, max_iter=60, subdomain_iters=3)
    punct = [((2, 2, 2), 4), ((3, 2, 2), 3)]
    fields = [_puncture(el, p) for el, p in punct]
    srv = dg.Server(hbm_budget_bytes=32e9, max_active=4, host_threads=2, **opts)
    ids = []
    for (el, p), (m, alpha, beta) in zip(punct, fields):
        ids.append(("n", el, p, srv.submit_puncture((-20,) * 3, (20,) * 3, el, p, alpha, beta,
                                                     newton_rtol=1e-10, linear_rtol=1e-4)))
        el2, p2, side = REQS[len(ids)]
        ids.append(("p", el2, p2, srv.submit((0, 0, 0), (side,) * 3, el2, p2,
                                             _f(el2, p2, side, 70 + len(ids)))))
    while srv.step() != (0, 0):
        pass
    for kind, el, p, rid in ids:
        u, st, _ = srv.fetch(rid)
        assert st["converged"], (kind, el, p, st)
        if kind != "n":
            continue
        m, alpha, beta = fields[punct.index((el, p))]
        prob = dg.Problem((-20,) * 3, (20,) * 3, el, p, **opts)
        u1, st1 = prob.newton_solve(to_gpu(alpha), to_gpu(beta), newton_rtol=1e-10,
                                    linear_rtol=1e-4)
        prob.close()
        assert st["newton_steps"] == st1["newton_steps"] and st["iterations"] == st1["iterations"]
        assert np.array_equal(u, to_np(u1))
        N = p + 1
        F = lambda v: oop.apply_operator(m, v.reshape(m.E, N, N, N), 1.5,
                                         source=onewton.puncture_source(alpha, beta, v)
                                         .reshape(m.E, N, N, N))
        r0 = np.linalg.norm(F(np.zeros(m.ndof)))
        assert np.linalg.norm(F(u)) / r0 <= 1e-10
    srv.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_reused_problems_give_the_bits_of_fresh_ones(precision):
    """Requests of a shape seen before run on the finished request's resident
    problem (hierarchy, Krylov basis, captured V-cycle graphs); with two slots
    and repeated shapes most requests do, and each still equals a solo solve."""
    import paper_2111_06767_amd as dg
    announce(f"serving problem reuse {precision}")
    shapes = [((2, 3, 2), 3, 1.0), ((3, 2, 2), 4, 2.0), ((2, 2, 2), 5, 1.0)]
    reqs = [shapes[i % 3] + (90 + i,) for i in range(9)]
    srv = dg.Server(hbm_budget_bytes=32e9, max_active=2, precision=precision, max_iter=60,
                    host_threads=2, batched=False)
    ids = []
    for el, p, side, seed in reqs:
        f = _f(el, p, side, seed)
        ids.append((el, p, side, f, srv.submit((0, 0, 0), (side,) * 3, el, p, f)))
    while srv.step() != (0, 0):
        pass
    for el, p, side, f, rid in ids:
        u, st, _ = srv.fetch(rid)
        u1, st1 = _alone(el, p, side, f, precision=precision, max_iter=60)
        assert st["converged"] and st["iterations"] == st1["iterations"]
        assert np.array_equal(u, u1), (el, p)
    srv.close()


def test_server_memory_from_the_callers_allocator():
    """With an allocator the server takes every request's device memory
    (problem workspaces and vectors) from it, gives the bits of the server
    without one, and returns every block."""
    import torch
    import paper_2111_06767_amd as dg
    announce("serving with the torch allocator")
    results = []
    alloc = dg.TorchAllocator()
    for allocator in (None, alloc):
        srv = dg.Server(hbm_budget_bytes=32e9, max_active=3, precision="mixed", max_iter=60,
                        host_threads=2, allocator=allocator)
        ids = []
        for i, (el, p, side) in enumerate(REQS[:4]):
            ids.append(srv.submit((0, 0, 0), (side,) * 3, el, p, _f(el, p, side, 1000 + i)))
        while srv.step() != (0, 0):
            pass
        results.append([srv.fetch(rid)[0] for rid in ids])
        srv.close()
    torch.cuda.synchronize()
    assert alloc.allocated > 0 and not alloc.live
    for a, b in zip(*results):
        assert np.array_equal(a, b)


# grids with single-element coarsest levels (1x1x1, 2x1x1), odd counts, and
# p = 8 (81 lanes per element: two wavefronts per workgroup)
BATCH_REQS = REQS + [((1, 1, 1), 5, 1.0), ((2, 1, 1), 8, 2.0), ((3, 5, 2), 3, 3.0),
                     ((4, 4, 4), 7, 1.0), ((2, 2, 4), 8, 4.0)]


def _oracle_residual(el, p, side, f, u):
    m = omesh.BoxMesh((0, 0, 0), (side,) * 3, el, p)
    b = oop.apply_mass(m, f.reshape(m.E, m.N, m.N, m.N)).reshape(-1)
    r = b - oop.apply_operator(m, u.reshape(m.E, m.N, m.N, m.N), 1.5).reshape(-1)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("restart", [0, 4])
def test_batched_mix_matches_alone(precision, restart):
    """The batched path advances all requests together through shared
    launches (every request's elements in one operator launch per phase,
    every request's classes in one GEMM per precision).  Its GEMM tiles and
    split-K parts differ from the solo solver's autotuned ones, so the
    subdomain corrections round differently: each result is compared with its
    solo solve to a relative 1e-9 (the solution tolerance of the solver
    tests), with the
    same iteration count within one, a true residual at 1e-10, and the
    oracle's residual of the result at 1e-10."""
    import paper_2111_06767_amd as dg
    announce(f"batched serving vs alone {precision} restart={restart}")
    srv = dg.Server(hbm_budget_bytes=32e9, max_active=8, precision=precision, max_iter=60,
                    restart=restart, batched=True)
    ids = {}
    for i, (el, p, side) in enumerate(BATCH_REQS):
        f = _f(el, p, side, 4000 + i)
        ids[srv.submit((0, 0, 0), (side,) * 3, el, p, f)] = (el, p, side, f)
    while srv.step() != (0, 0):
        pass
    steps, bsteps, launches, peak = srv.counters()
    assert peak >= 4 and bsteps > 0
    for rid in srv.finished():
        u, st, times = srv.fetch(rid)
        el, p, side, f = ids[rid]
        ua, sta = _alone(el, p, side, f, precision=precision, max_iter=60, restart=restart)
        assert st["converged"] and st["rel_residual"] <= 1e-10, (el, p, st)
        assert abs(st["iterations"] - sta["iterations"]) <= 1, (el, p, st["iterations"],
                                                               sta["iterations"])
        assert np.linalg.norm(u - ua) / np.linalg.norm(ua) <= 1e-9, (el, p)
        assert _oracle_residual(el, p, side, f, u) <= 1e-10, (el, p)
    srv.close()


def test_batched_launches_do_not_grow_with_the_number_of_requests():
    """Kernel launches per engine step stay flat as the batch grows: one
    launch per phase covers every request."""
    import paper_2111_06767_amd as dg
    announce("batched launches per step")
    per_step = {}
    for count in (1, 8):
        srv = dg.Server(hbm_budget_bytes=32e9, max_active=count, precision="mixed", max_iter=60)
        for i in range(count):
            el, p, side = (3, 3, 2), 4, 1.0  # one shape: the same cycle schedule
            srv.submit((0, 0, 0), (side,) * 3, el, p, _f(el, p, side, 5000 + i))
        while srv.step() != (0, 0):
            pass
        steps, bsteps, launches, peak = srv.counters()
        assert peak == count
        per_step[count] = launches / bsteps
        srv.close()
    assert per_step[8] <= 1.05 * per_step[1], per_step
