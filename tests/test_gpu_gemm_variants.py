"""Every tile variant of the grouped subdomain-solve GEMM against the oracle's
Schwarz step (Sec. III.D.2 subdomain solves), through the C ABI.

The variants differ in tile shape, split of the K range and kernel (single or
double-buffered LDS), so their results agree to rounding.  Levels whose
classes hold more than 32 subdomains use the large tiles, smaller ones the
16 x 64 tiles with a variant-dependent number of K parts; both plans are
covered.  With large tiles, variants 2 and 4 use the same tiles, K ranges
and summation order, so they must give the same bits."""
import numpy as np
import pytest

import workloads as W
from oracle import mesh as omesh, schwarz
from tests.gpu_util import announce, rel_max, to_gpu, to_np

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
VARIANTS = range(5)


def _step(prob, b, u0, variant):
    prob.set_gemm_variant(variant, level=0)
    u = to_gpu(u0)
    prob.smooth(to_gpu(b), u, 1)
    return to_np(u)


@pytest.mark.parametrize("elements,p,large", [((6, 6, 6), 3, True), ((4, 4, 2), 4, False)])
def test_every_gemm_variant_matches_oracle_fp64(elements, p, large):
    import paper_2111_06767_amd as dg
    announce(f"gemm variants fp64 elements={elements} p={p}")
    upper = (1.0, 0.9, 1.2)
    m = omesh.BoxMesh((0, 0, 0), upper, elements, p)
    prob = dg.Problem((0, 0, 0), upper, elements, p, penalty=1.5, mg_levels=1)
    b = W.random_normal(101, m.ndof)
    u0 = W.random_uniform(102, m.ndof)
    ref = schwarz.SchwarzSmoother(m, 1.5, 2).smooth(u0, b, 1)
    outs = {}
    for v in VARIANTS:
        outs[v] = _step(prob, b, u0, v)
        assert rel_max(outs[v], ref) < 1e-11, (v, rel_max(outs[v], ref))
    if large:
        # same tiles and K ranges (the small plan splits K differently per variant)
        assert np.array_equal(outs[2], outs[4])
    prob.close()


def test_every_gemm_variant_mixed_precision():
    # two levels: the fine level (216 subdomains of up to 256 points) solves
    # in FP32; every variant stays within the FP32 summation bound of the
    # FP64 oracle, and variants 2 and 4 agree bit for bit
    import paper_2111_06767_amd as dg
    announce("gemm variants mixed 6x6x6 p=3")
    m = omesh.BoxMesh((0, 0, 0), (1, 1, 1), (6, 6, 6), 3)
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (6, 6, 6), 3, penalty=1.5, mg_levels=2,
                      precision="mixed")
    b = W.random_normal(103, m.ndof)
    u0 = W.random_uniform(104, m.ndof)
    ref = schwarz.SchwarzSmoother(m, 1.5, 2).smooth(u0, b, 1)
    n_s = max(len(schwarz.subdomain_layout(m, e, 2)[0]) for e in range(m.E))
    scale = np.abs(ref - u0).max()
    outs = {}
    for v in VARIANTS:
        outs[v] = _step(prob, b, u0, v)
        err = np.abs(outs[v] - ref).max() / scale
        assert 1e-12 < err <= (n_s + 2) * U32, (v, err)
    assert np.array_equal(outs[2], outs[4])
    prob.close()


def test_gemm_variant_override_is_checked():
    import paper_2111_06767_amd as dg
    announce("gemm variant range")
    prob = dg.Problem((0, 0, 0), (1, 1, 1), (2, 2, 2), 3, mg_levels=1)
    for v in VARIANTS:
        prob.set_gemm_variant(v)
        assert prob.gemm_variant() == v
    for bad in (-1, 5):
        with pytest.raises(dg.DgsError):
            prob.set_gemm_variant(bad)
    prob.close()
