"""Host-side checks of the C ABI library: it loads without a GPU and exports
every entry point that include/dgsolve.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "dgsolve.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(dgs_[a-z_]+)\s*\(", text)))


def test_header_lists_the_binding_names():
    import paper_2111_06767_amd as m
    assert sorted(m.EXPORTED) == _declared()


def test_library_exports_every_declared_symbol():
    import paper_2111_06767_amd as m
    if not os.path.exists(m.api.LIB_PATH):
        pytest.skip("library not built")
    lib = m.load_library()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert missing == []


def test_default_options_and_invalid_arguments_without_gpu():
    import ctypes
    import paper_2111_06767_amd as m
    if not os.path.exists(m.api.LIB_PATH):
        pytest.skip("library not built")
    lib = m.load_library()
    o = m.default_options()
    assert (o.overlap, o.pre_smooth, o.post_smooth, o.max_iter) == (2, 3, 3, 200)
    assert o.rtol == 1e-10
    # argument validation happens before any device call
    dom = m.api.Domain((ctypes.c_double * 3)(0, 0, 0), (ctypes.c_double * 3)(1, 1, 1))
    h = ctypes.c_void_p()
    for el, p, C in [((0, 1, 1), 3, 1.5), ((1, 1, 1), 0, 1.5), ((1, 1, 1), 13, 1.5), ((1, 1, 1), 3, 0.0)]:
        code = lib.dgs_create_problem(ctypes.byref(dom), (ctypes.c_int * 3)(*el), p, C,
                                      ctypes.byref(o), m.api.ALLOC_FN(), m.api.FREE_FN(), None,
                                      None, ctypes.byref(h))
        assert code == m.DGS_ERR_INVALID
        assert lib.dgs_last_error().decode() != ""
    bad = m.api.Domain((ctypes.c_double * 3)(0, 0, 0), (ctypes.c_double * 3)(1, 0, 1))
    assert lib.dgs_create_problem(ctypes.byref(bad), (ctypes.c_int * 3)(1, 1, 1), 3, 1.5,
                                  ctypes.byref(o), m.api.ALLOC_FN(), m.api.FREE_FN(), None, None,
                                  ctypes.byref(h)) == m.DGS_ERR_INVALID
    # an allocator needs both functions
    alloc_only = m.api.ALLOC_FN(lambda nbytes, ctx: None)
    assert lib.dgs_create_problem(ctypes.byref(dom), (ctypes.c_int * 3)(1, 1, 1), 3, 1.5,
                                  ctypes.byref(o), alloc_only, m.api.FREE_FN(), None, None,
                                  ctypes.byref(h)) == m.DGS_ERR_INVALID
    assert "together" in lib.dgs_last_error().decode()


def test_subdomain_solves_rejects_null_problem_without_gpu():
    import paper_2111_06767_amd as m
    if not os.path.exists(m.api.LIB_PATH):
        pytest.skip("library not built")
    lib = m.load_library()
    assert lib.dgs_subdomain_solves(None, 0, 1, None, None) == m.DGS_ERR_INVALID


def test_hp_mesh_validation_without_gpu():
    # the hp set-up checks the mesh on the host before any device call
    import ctypes
    import paper_2111_06767_amd as m
    if not os.path.exists(m.api.LIB_PATH):
        pytest.skip("library not built")
    lib = m.load_library()
    dom = m.api.Domain((ctypes.c_double * 3)(0, 0, 0), (ctypes.c_double * 3)(2, 1, 1))
    h = ctypes.c_void_p()

    def create(blocks, levels, degrees, **opts):
        o = m.default_options(**opts)
        lv = [v for row in levels for v in row]
        dg = [v for row in degrees for v in row]
        return lib.dgs_create_hp_problem(ctypes.byref(dom), (ctypes.c_int * 3)(*blocks),
                                         (ctypes.c_int * len(lv))(*lv), (ctypes.c_int * len(dg))(*dg),
                                         len(dg) // 3, 1.5, ctypes.byref(o), None, ctypes.byref(h))

    cases = [
        ((2, 1, 1), [(2, 2, 2), (0, 0, 0)], [(2, 2, 2)] * 65, {}),  # levels 2 against 0 across a face
        ((2, 1, 1), [(1, 1, 1), (0, 0, 0)], [(2, 2, 2)] * 8, {}),  # element count
        ((2, 1, 1), [(0, 0, 0), (0, 0, 0)], [(8, 2, 2), (2, 2, 2)], {}),  # degree 8
        ((2, 1, 1), [(0, 0, 0), (0, 0, 0)], [(0, 2, 2), (2, 2, 2)], {}),  # degree 0
        ((2, 1, 1), [(0, 0, 0), (0, 0, 0)], [(2, 2, 2)] * 2, {"cycle": 2}),
        ((2, 1, 1), [(0, 0, 0), (0, 0, 0)], [(2, 2, 2)] * 2, {"neumann_faces": 63}),
    ]
    for blocks, levels, degrees, opts in cases:
        assert create(blocks, levels, degrees, **opts) == m.DGS_ERR_INVALID, (levels, degrees, opts)
        assert lib.dgs_last_error().decode() != ""
    assert "balanced" in (create(*cases[0][:3]) and lib.dgs_last_error().decode())


def test_curved_and_newton_entries_reject_null_handles_without_gpu():
    # the metric, geometry and power-source Newton entries validate their
    # handles and sizes on the host before any device call
    import ctypes
    import paper_2111_06767_amd as m
    if not os.path.exists(m.api.LIB_PATH):
        pytest.skip("library not built")
    lib = m.load_library()
    pw = (ctypes.c_int * 2)(1, 0)
    va = (ctypes.c_int * 1)(0)
    assert lib.dgs_set_metric(None, None, None, None) == m.DGS_ERR_INVALID
    assert lib.dgs_system_set_metric(None, None, None, None) == m.DGS_ERR_INVALID
    assert lib.dgs_system_set_geometry(None, None, None) == m.DGS_ERR_INVALID
    assert lib.dgs_newton_solve_powers(None, 1, pw, None, None, None, None, 1e-10, 1e-4, 5, None,
                                       None) == m.DGS_ERR_INVALID
    assert lib.dgs_system_newton_solve_powers(None, 1, va, pw, None, None, None, None, 1e-10, 1e-4, 5,
                                              None, None) == m.DGS_ERR_INVALID
    assert lib.dgs_last_error().decode() != ""
