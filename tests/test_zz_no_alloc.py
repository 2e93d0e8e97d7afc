"""dgs_cg_solve_noalloc (the CG solve on the library's static device
workspace) against dgs_cg_solve, through the C ABI: two calls in a row, the
second on a smaller problem, each equal to the allocating entry point's
result on the same inputs, and a problem above the workspace limit refused."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_util import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _fourier_rhs(prob, seed):
    xyz = prob.node_coordinates()
    x, y, z = (xyz[d].cpu().numpy() for d in range(3))
    f = W.fourier_source(W.fourier_modes(seed, prob.lower, prob.upper), x, y, z)
    return prob.apply_mass(to_gpu(f))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_cg_equals_cg_on_two_calls(precision):
    import torch
    import paper_2111_06767_amd as dg
    # the larger problem first, then a smaller one: the second call must not
    # see anything the first left in the shared workspace
    for elements, p, seed in (((8, 8, 8), 6, 2), ((4, 2, 2), 3, 3)):
        announce(f"noalloc cg {precision} elements={elements} p={p}")
        prob = dg.Problem((0, 0, 0), (1, 1, 1), elements, p, precision=precision)
        b = _fourier_rhs(prob, seed)
        u_ref, st_ref = prob.solve_cg(b)
        u = torch.zeros_like(b)
        u, st = prob.solve_cg_noalloc(b, u)
        ur, un = to_np(u_ref), to_np(u)
        assert st["converged"] and st_ref["converged"]
        assert st["iterations"] == st_ref["iterations"]
        assert st["rel_residual"] <= 1e-10
        # the same kernels in the same order on the same data: the same bits
        assert np.array_equal(un, ur), float(np.abs(un - ur).max())
        assert st["history"] == st_ref["history"]
        prob.close()


def test_noalloc_cg_refuses_problems_above_its_workspace():
    import torch
    import paper_2111_06767_amd as dg
    announce("noalloc cg size limit")
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (16, 16, 8), 7, mg_levels=1)  # 1,048,576 points: fits
    assert prob.ndof == 1 << 20
    prob.close()
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (16, 16, 9), 7, mg_levels=1)  # 1,179,648: too many
    b = torch.zeros(prob.ndof, dtype=torch.float64, device="cuda")
    u = torch.zeros_like(b)
    with pytest.raises(dg.DgsError) as e:
        prob.solve_cg_noalloc(b, u)
    assert e.value.code == dg.DGS_ERR_INVALID and "static workspace" in str(e.value)
    prob.close()
