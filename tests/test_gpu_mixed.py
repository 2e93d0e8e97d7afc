"""Element-wise error of the mixed-precision smoother against the FP64
oracle, through the C ABI.

In mixed mode every level except the coarsest solves its subdomain problems
in FP32 on the matrix cores: the explicit inverse is rounded to FP32 (unit
roundoff u32 = 2^-24), the gathered residual r_S too, and the product
accumulates in FP32.  Each entry of du_S = A_S^-1 r_S is a sum of n_S
products, so its error is bounded by about (n_S + 2) u32 sum_j |a_ij r_j|;
the tests take that bound with the largest n_S of the level, relative to the
largest |du| (the sums of absolute products stay within a small factor of it
for these SPD inverses: the measured step errors are 0.7 to 3e-7, about
50 times below the bound).
The residual, the weighted scatter and everything outside the subdomain
solves stay FP64, so the step's error is that of du alone; a V-cycle repeats
the step 3 + 3 times per level and the errors add, so its bound is six times
larger per level (measured: below 1e-8 relative to the largest |z|)."""
import numpy as np
import pytest

import workloads as W
from oracle import mesh as omesh, multigrid, schwarz
from tests.gpu_util import announce, to_gpu, to_np

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def _bound(n_s, repeats=1):
    return repeats * (n_s + 2) * U32


@pytest.mark.parametrize("elements,p", [((2, 2, 2), 3), ((4, 2, 2), 4), ((4, 4, 2), 3)])
def test_mixed_schwarz_step_error_against_fp64_oracle(elements, p):
    import paper_2111_06767_amd as dg
    announce(f"mixed schwarz step elements={elements} p={p}")
    m = omesh.BoxMesh((0, 0, 0), (1, 1.1, 0.9), elements, p)
    # two levels, so that the finest is an FP32 level (the coarsest stays FP64)
    prob = dg.Problem((0, 0, 0), (1, 1.1, 0.9), elements, p, mg_levels=2, precision="mixed")
    b = W.random_normal(91, m.ndof)
    u0 = W.random_uniform(92, m.ndof)
    S = schwarz.SchwarzSmoother(m, 1.5, 2)
    ref = S.smooth(u0, b, 1)
    u = to_gpu(u0)
    prob.smooth(to_gpu(b), u, 1)
    got = to_np(u)
    du_ref = ref - u0
    err = np.abs(got - ref).max() / np.abs(du_ref).max()
    n_s = max(len(schwarz.subdomain_layout(m, e, 2)[0]) for e in range(m.E))
    announce(f"  max error / max |du| = {err:.2e} (bound {_bound(n_s):.2e}, n_S = {n_s})")
    assert err <= _bound(n_s), err
    # and it is a real FP32 result, not an FP64 one
    assert err > 1e-12


@pytest.mark.parametrize("elements,p,levels", [((4, 4, 4), 3, 2), ((4, 4, 4), 3, 3), ((4, 2, 2), 5, 2)])
def test_mixed_vcycle_error_against_fp64_oracle(elements, p, levels):
    import paper_2111_06767_amd as dg
    announce(f"mixed vcycle elements={elements} p={p} levels={levels}")
    m = omesh.BoxMesh((0, 0, 0), (1, 1, 1), elements, p)
    prob = dg.Problem((0, 0, 0), (1, 1, 1), elements, p, mg_levels=levels, precision="mixed")
    V = multigrid.VCycle(m, 1.5, levels=levels)
    r = W.random_normal(93, m.ndof)
    ref = V(r)
    got = to_np(prob.precondition(to_gpu(r)))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    n_s = max(len(schwarz.subdomain_layout(m, e, 2)[0]) for e in range(m.E))
    fp32_levels = levels - 1
    announce(f"  max error / max |z| = {err:.2e} (bound {_bound(n_s, 6 * fp32_levels):.2e})")
    assert err <= _bound(n_s, 6 * fp32_levels), err
    assert err > 1e-12
