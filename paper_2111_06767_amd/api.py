"""Python binding of the C ABI in include/dgsolve.h (argument marshalling only).

Fields are torch tensors on the GPU (float64, contiguous, canonical nodal
layout); their device pointers and torch's current HIP stream are handed to
the library.  Every computation runs in the library's HIP kernels.  The
library must be built (``__graft_entry__.build()``); loading fails loudly
otherwise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdgsolve.so")

DGS_OK = 0
DGS_NOT_CONVERGED = 1
DGS_ERR_INVALID = -1
DGS_ERR_OOM = -2
DGS_ERR_HIP = -3
DGS_ERR_NONFINITE = -4
DGS_FP64 = 0
DGS_MIXED = 1

# Entry points declared in include/dgsolve.h.
EXPORTED = (
    "dgs_default_options", "dgs_create_problem", "dgs_destroy_problem", "dgs_num_dofs",
    "dgs_node_coordinates", "dgs_apply_mass", "dgs_apply_operator", "dgs_schwarz_smooth",
    "dgs_precondition", "dgs_solve", "dgs_newton_solve", "dgs_last_error", "dgs_set_diagonal",
    "dgs_lgl_nodes", "dgs_server_create", "dgs_server_destroy", "dgs_server_submit",
    "dgs_server_step", "dgs_server_finished", "dgs_server_fetch", "dgs_subdomain_solves",
    "dgs_set_apply_shape", "dgs_get_apply_shape", "dgs_set_gemm_variant", "dgs_get_gemm_variant",
    "dgs_server_submit_puncture", "dgs_cg_solve", "dgs_grid_coordinates",
    "dgs_cg_solve_noalloc", "dgs_server_counters", "dgs_server_timings",
    "dgs_set_geometry", "dgs_create_system", "dgs_destroy_system", "dgs_system_num_dofs", "dgs_system_set_coupling",
    "dgs_system_apply", "dgs_system_smooth", "dgs_system_precondition", "dgs_system_solve",
    "dgs_create_hp_problem", "dgs_destroy_hp_problem", "dgs_hp_num_dofs", "dgs_hp_num_levels",
    "dgs_hp_num_classes", "dgs_hp_node_coordinates", "dgs_hp_apply_operator", "dgs_hp_apply_mass",
    "dgs_hp_smooth", "dgs_hp_precondition", "dgs_hp_solve", "dgs_set_metric", "dgs_newton_solve_powers",
    "dgs_system_set_geometry", "dgs_system_set_metric", "dgs_system_newton_solve_powers",
)


class Domain(ctypes.Structure):
    _fields_ = [("lower", ctypes.c_double * 3), ("upper", ctypes.c_double * 3)]


class Options(ctypes.Structure):
    _fields_ = [("overlap", ctypes.c_int), ("mg_levels", ctypes.c_int),
                ("pre_smooth", ctypes.c_int), ("post_smooth", ctypes.c_int),
                ("precision", ctypes.c_int), ("subdomain_iters", ctypes.c_int),
                ("max_iter", ctypes.c_int), ("rtol", ctypes.c_double),
                ("use_graphs", ctypes.c_int), ("restart", ctypes.c_int),
                ("cycle", ctypes.c_int), ("additive", ctypes.c_int),
                ("neumann_faces", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("newton_steps", ctypes.c_int),
                ("backtracks", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_capacity", ctypes.c_int),
                ("history_len", ctypes.c_int), ("t_setup_s", ctypes.c_double),
                ("t_solve_s", ctypes.c_double)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_double), ("max_active", ctypes.c_int),
                ("penalty", ctypes.c_double), ("solver", Options), ("host_threads", ctypes.c_int),
                ("alloc_fn", ctypes.c_void_p), ("free_fn", ctypes.c_void_p),
                ("alloc_ctx", ctypes.c_void_p), ("batched", ctypes.c_int)]


class DgsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"dgsolve error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libdgsolve.so and declare the argument types of every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch ships its own HIP runtime with the same soname; loading torch first
    # makes the library bind to that one runtime instead of a second copy
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    dp = ctypes.c_void_p  # device pointers
    lib.dgs_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.dgs_default_options.restype = None
    lib.dgs_create_problem.argtypes = [ctypes.POINTER(Domain), ctypes.POINTER(ctypes.c_int),
                                       ctypes.c_int, ctypes.c_double, ctypes.POINTER(Options),
                                       ALLOC_FN, FREE_FN, P, P, ctypes.POINTER(P)]
    lib.dgs_destroy_problem.argtypes = [P]
    lib.dgs_num_dofs.argtypes = [P, ctypes.POINTER(ctypes.c_longlong)]
    lib.dgs_node_coordinates.argtypes = [P, dp, P]
    lib.dgs_apply_mass.argtypes = [P, dp, dp, P]
    lib.dgs_apply_operator.argtypes = [P, dp, dp, P]
    lib.dgs_schwarz_smooth.argtypes = [P, dp, dp, ctypes.c_int, P]
    lib.dgs_precondition.argtypes = [P, dp, dp, P]
    lib.dgs_set_diagonal.argtypes = [P, dp, P]
    lib.dgs_solve.argtypes = [P, dp, dp, ctypes.POINTER(Stats), P]
    lib.dgs_cg_solve.argtypes = [P, dp, dp, ctypes.POINTER(Stats), P]
    lib.dgs_cg_solve_noalloc.argtypes = [P, dp, dp, ctypes.POINTER(Stats), P]
    lib.dgs_newton_solve.argtypes = [P, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int, ctypes.POINTER(Stats), P]
    lib.dgs_lgl_nodes.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.dgs_grid_coordinates.argtypes = [ctypes.POINTER(Domain), ctypes.POINTER(ctypes.c_int),
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                         ctypes.c_longlong]
    lib.dgs_server_create.argtypes = [ctypes.POINTER(ServerOptions), ctypes.POINTER(P)]
    lib.dgs_server_destroy.argtypes = [P]
    lib.dgs_server_submit.argtypes = [P, ctypes.POINTER(Domain), ctypes.POINTER(ctypes.c_int),
                                      ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                      ctypes.c_longlong, ctypes.POINTER(ctypes.c_longlong)]
    lib.dgs_server_submit_puncture.argtypes = [
        P, ctypes.POINTER(Domain), ctypes.POINTER(ctypes.c_int), ctypes.c_int,
        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
        ctypes.POINTER(ctypes.c_double), ctypes.c_longlong, ctypes.c_double, ctypes.c_double,
        ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]
    lib.dgs_server_step.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    lib.dgs_server_counters.argtypes = [P, ctypes.POINTER(ctypes.c_longlong)]
    lib.dgs_server_timings.argtypes = [P, ctypes.POINTER(ctypes.c_double)]
    lib.dgs_server_finished.argtypes = [P, ctypes.POINTER(ctypes.c_longlong), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]
    lib.dgs_server_fetch.argtypes = [P, ctypes.c_longlong, ctypes.POINTER(ctypes.c_double),
                                     ctypes.c_longlong, ctypes.POINTER(Stats),
                                     ctypes.POINTER(ctypes.c_double)]
    lib.dgs_subdomain_solves.argtypes = [P, ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_double), P]
    lib.dgs_set_apply_shape.argtypes = [P, ctypes.c_int, ctypes.c_int]
    lib.dgs_get_apply_shape.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.dgs_set_gemm_variant.argtypes = [P, ctypes.c_int, ctypes.c_int]
    lib.dgs_get_gemm_variant.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    lib.dgs_set_geometry.argtypes = [P, dp, P]
    lib.dgs_set_metric.argtypes = [P, dp, dp, P]
    lib.dgs_newton_solve_powers.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), dp, dp, dp, dp,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                            ctypes.POINTER(Stats), P]
    lib.dgs_create_system.argtypes = [ctypes.POINTER(Domain), ctypes.POINTER(ctypes.c_int),
                                      ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                      ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                      ctypes.POINTER(Options), P, ctypes.POINTER(P)]
    lib.dgs_destroy_system.argtypes = [P]
    lib.dgs_system_num_dofs.argtypes = [P, ctypes.POINTER(ctypes.c_longlong)]
    lib.dgs_system_set_coupling.argtypes = [P, dp, P]
    lib.dgs_system_apply.argtypes = [P, dp, dp, P]
    lib.dgs_system_smooth.argtypes = [P, dp, dp, ctypes.c_int, P]
    lib.dgs_system_precondition.argtypes = [P, dp, dp, P]
    lib.dgs_system_solve.argtypes = [P, dp, dp, ctypes.POINTER(Stats), P]
    lib.dgs_system_set_geometry.argtypes = [P, dp, P]
    lib.dgs_system_set_metric.argtypes = [P, dp, dp, P]
    lib.dgs_system_newton_solve_powers.argtypes = [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                                   ctypes.POINTER(ctypes.c_int), dp, dp, dp, dp,
                                                   ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                   ctypes.POINTER(Stats), P]
    lib.dgs_create_hp_problem.argtypes = [ctypes.POINTER(Domain), ctypes.POINTER(ctypes.c_int),
                                          ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                          ctypes.c_int, ctypes.c_double, ctypes.POINTER(Options), P,
                                          ctypes.POINTER(P)]
    lib.dgs_destroy_hp_problem.argtypes = [P]
    lib.dgs_hp_num_dofs.argtypes = [P]
    lib.dgs_hp_num_levels.argtypes = [P]
    lib.dgs_hp_num_classes.argtypes = [P, ctypes.c_int]
    lib.dgs_hp_node_coordinates.argtypes = [P, dp, P]
    lib.dgs_hp_apply_operator.argtypes = [P, dp, dp, P]
    lib.dgs_hp_apply_mass.argtypes = [P, dp, dp, P]
    lib.dgs_hp_smooth.argtypes = [P, dp, dp, ctypes.c_int, P]
    lib.dgs_hp_precondition.argtypes = [P, dp, dp, P]
    lib.dgs_hp_solve.argtypes = [P, dp, dp, ctypes.POINTER(Stats), P]
    lib.dgs_last_error.argtypes = []
    lib.dgs_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("dgs_default_options", "dgs_last_error"):
            getattr(lib, name).restype = ctypes.c_int
    lib.dgs_hp_num_dofs.restype = ctypes.c_longlong
    _lib = lib
    return lib


def default_options(**kw) -> Options:
    lib = load_library()
    o = Options()
    lib.dgs_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": DGS_FP64, "mixed": DGS_MIXED}[v]
        setattr(o, k, v)
    return o


def _check(code, allow_not_converged=False):
    if code == DGS_OK or (allow_not_converged and code == DGS_NOT_CONVERGED):
        return code
    msg = load_library().dgs_last_error().decode()
    raise DgsError(code, msg)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t, n=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return ctypes.c_void_p(t.data_ptr())


# dgs_alloc_fn / dgs_free_fn
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class TorchAllocator:
    """A problem's device workspace from PyTorch's caching allocator (the
    dgs_alloc_fn / dgs_free_fn pair of dgs_create_problem).  Every block is
    allocated on one stream, torch's current stream when the allocator is
    made unless `stream` names another: the caching allocator only hands a
    freed block out again once that stream's earlier work is done, so the
    problem must run its work on that stream (pass the same stream to every
    call, as Problem does by default).  `live` holds the blocks handed out and
    not yet returned."""

    def __init__(self, stream=None):
        import torch
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self.live = {}
        self.allocated = 0

    def alloc(self, nbytes):
        import torch
        ptr = torch.cuda.caching_allocator_alloc(int(nbytes), self.stream.device.index,
                                                 self.stream)
        self.live[ptr] = int(nbytes)
        self.allocated += 1
        return ptr

    def free(self, ptr):
        import torch
        self.live.pop(ptr)
        torch.cuda.caching_allocator_delete(ptr)


class Problem:
    """A DG Poisson problem on a box (see dgs_create_problem).  `allocator`:
    an object with alloc(nbytes) -> device address and free(address), such as
    TorchAllocator, for the problem's own device memory (None: the library's
    hipMalloc)."""

    def __init__(self, lower, upper, elements, p, penalty=1.5, options: Options | None = None,
                 stream=None, allocator=None, **opts):
        lib = load_library()
        self._lib = lib
        self.options = options if options is not None else default_options(**opts)
        dom = Domain((ctypes.c_double * 3)(*lower), (ctypes.c_double * 3)(*upper))
        el = (ctypes.c_int * 3)(*elements)
        h = ctypes.c_void_p()
        self._h = None
        self.allocator = allocator
        if allocator is not None:
            # kept on the problem: the library calls them until it is destroyed
            self._alloc_cb = ALLOC_FN(lambda nbytes, ctx: allocator.alloc(nbytes))
            self._free_cb = FREE_FN(lambda ptr, ctx: allocator.free(ptr))
        else:
            self._alloc_cb, self._free_cb = ALLOC_FN(), FREE_FN()
        _check(lib.dgs_create_problem(ctypes.byref(dom), el, int(p), float(penalty),
                                      ctypes.byref(self.options), self._alloc_cb, self._free_cb,
                                      None, _stream(stream), ctypes.byref(h)))
        self._h = h
        self.elements = tuple(int(v) for v in elements)
        self.p, self.N = int(p), int(p) + 1
        self.lower, self.upper = tuple(lower), tuple(upper)
        n = ctypes.c_longlong()
        _check(lib.dgs_num_dofs(h, ctypes.byref(n)))
        self.ndof = n.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dgs_destroy_problem(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, n=None):
        import torch
        return torch.empty(self.ndof if n is None else n, dtype=torch.float64, device="cuda")

    def node_coordinates(self, stream=None):
        xyz = self._new(3 * self.ndof)
        _check(self._lib.dgs_node_coordinates(self._h, _ptr(xyz, 3 * self.ndof), _stream(stream)))
        return xyz.view(3, self.ndof)

    def apply_mass(self, f, out=None, stream=None):
        out = self._new() if out is None else out
        _check(self._lib.dgs_apply_mass(self._h, _ptr(f, self.ndof, "f"), _ptr(out, self.ndof, "out"),
                                        _stream(stream)))
        return out

    def apply(self, u, out=None, stream=None):
        out = self._new() if out is None else out
        _check(self._lib.dgs_apply_operator(self._h, _ptr(u, self.ndof, "u"),
                                            _ptr(out, self.ndof, "out"), _stream(stream)))
        return out

    def smooth(self, b, u, steps, stream=None):
        _check(self._lib.dgs_schwarz_smooth(self._h, _ptr(b, self.ndof, "b"), _ptr(u, self.ndof, "u"),
                                            int(steps), _stream(stream)))
        return u

    def precondition(self, r, out=None, stream=None):
        out = self._new() if out is None else out
        _check(self._lib.dgs_precondition(self._h, _ptr(r, self.ndof, "r"), _ptr(out, self.ndof, "z"),
                                          _stream(stream)))
        return out

    def subdomain_solves(self, level=0, reps=1, stream=None):
        """Launch the grouped subdomain-solve GEMM of one Schwarz sweep on
        `level` `reps` times (timing aid); returns its flops per sweep."""
        flops = ctypes.c_double()
        _check(self._lib.dgs_subdomain_solves(self._h, int(level), int(reps), ctypes.byref(flops),
                                              _stream(stream)))
        return flops.value

    def apply_shape(self, level=0):
        """Operator-kernel launch shape of `level`: elements per workgroup
        (1, 2; 0 = default for p) or -1 for 2 x 2 x 2 element bricks (p = 7)."""
        v = ctypes.c_int()
        _check(self._lib.dgs_get_apply_shape(self._h, int(level), ctypes.byref(v)))
        return v.value

    def set_apply_shape(self, shape, level=0):
        """Override the autotuned operator-kernel launch shape of `level`."""
        _check(self._lib.dgs_set_apply_shape(self._h, int(level), int(shape)))

    def gemm_variant(self, level=0):
        """Tile variant (0 to 4) of the subdomain-solve GEMM on `level`."""
        v = ctypes.c_int()
        _check(self._lib.dgs_get_gemm_variant(self._h, int(level), ctypes.byref(v)))
        return v.value

    def set_gemm_variant(self, variant, level=0):
        """Override the autotuned GEMM tile variant of `level`."""
        _check(self._lib.dgs_set_gemm_variant(self._h, int(level), int(variant)))

    def set_geometry(self, xyz=None, stream=None):
        """Curved elements: physical coordinates of every node (a device tensor
        of 3 * ndof: x, then y, then z); None returns to the box grid."""
        ptr = ctypes.c_void_p(None) if xyz is None else _ptr(xyz, 3 * self.ndof, "xyz")
        _check(self._lib.dgs_set_geometry(self._h, ptr, _stream(stream)))

    def set_metric(self, ginv=None, sqrtg=None, stream=None):
        """A curved background metric: g^ij as a device tensor of 6 * ndof (the
        fields xx, xy, xz, yy, yz, zz) and sqrt(g) of ndof; both None return to
        the flat metric."""
        if (ginv is None) != (sqrtg is None):
            raise ValueError("ginv and sqrtg are given together")
        if ginv is None:
            _check(self._lib.dgs_set_metric(self._h, ctypes.c_void_p(None), ctypes.c_void_p(None),
                                            _stream(stream)))
            return
        _check(self._lib.dgs_set_metric(self._h, _ptr(ginv, 6 * self.ndof, "ginv"),
                                        _ptr(sqrtg, self.ndof, "sqrtg"), _stream(stream)))

    def set_diagonal(self, d=None, stream=None):
        """Operator A + diag(d) for smoothing, preconditioning and solves (None: A)."""
        ptr = ctypes.c_void_p(None) if d is None else _ptr(d, self.ndof, "d")
        _check(self._lib.dgs_set_diagonal(self._h, ptr, _stream(stream)))

    def solve(self, b, u=None, history=256, stream=None):
        """Solve A u = b (u = initial guess, zero if None).  Returns (u, stats dict)."""
        import torch
        if u is None:
            u = torch.zeros(self.ndof, dtype=torch.float64, device="cuda")
        st, hist = _make_stats(history)
        code = _check(self._lib.dgs_solve(self._h, _ptr(b, self.ndof, "b"), _ptr(u, self.ndof, "u"),
                                          ctypes.byref(st), _stream(stream)), allow_not_converged=True)
        return u, _stats_dict(st, hist, code)

    def solve_cg(self, b, u=None, history=256, stream=None):
        """Solve A u = b by preconditioned conjugate gradients (dgs_cg_solve).
        Returns (u, stats dict)."""
        import torch
        if u is None:
            u = torch.zeros(self.ndof, dtype=torch.float64, device="cuda")
        st, hist = _make_stats(history)
        code = _check(self._lib.dgs_cg_solve(self._h, _ptr(b, self.ndof, "b"),
                                             _ptr(u, self.ndof, "u"), ctypes.byref(st),
                                             _stream(stream)), allow_not_converged=True)
        return u, _stats_dict(st, hist, code)

    def solve_cg_noalloc(self, b, u, history=256, stream=None):
        """dgs_cg_solve_noalloc: the CG solve with the library's static device
        workspace (no device allocation in the call).  Returns (u, stats dict)."""
        st, hist = _make_stats(history)
        code = _check(self._lib.dgs_cg_solve_noalloc(self._h, _ptr(b, self.ndof, "b"),
                                                     _ptr(u, self.ndof, "u"), ctypes.byref(st),
                                                     _stream(stream)), allow_not_converged=True)
        return u, _stats_dict(st, hist, code)

    def newton_solve(self, alpha, beta, b=None, u=None, newton_rtol=1e-10, linear_rtol=1e-4,
                     max_newton=20, history=256, stream=None):
        import torch
        if u is None:
            u = torch.zeros(self.ndof, dtype=torch.float64, device="cuda")
        if b is None:
            b = torch.zeros(self.ndof, dtype=torch.float64, device="cuda")
        st, hist = _make_stats(history)
        code = _check(self._lib.dgs_newton_solve(
            self._h, _ptr(alpha, self.ndof, "alpha"), _ptr(beta, self.ndof, "beta"),
            _ptr(b, self.ndof, "b"), _ptr(u, self.ndof, "u"), float(newton_rtol), float(linear_rtol),
            int(max_newton), ctypes.byref(st), _stream(stream)), allow_not_converged=True)
        return u, _stats_dict(st, hist, code)

    def newton_solve_powers(self, coef, powers, dirichlet=None, b=None, u=None, newton_rtol=1e-10,
                            linear_rtol=1e-4, max_newton=20, history=256, stream=None):
        """Newton on curved elements for A(u; u_b) + M S(u) = b with the source
        S(u) = sum_t coef_t u^powers_t: coef a device tensor of len(powers) * ndof,
        dirichlet the boundary data (None: homogeneous), u the initial guess
        (ones if None).  Returns (u, stats dict)."""
        import torch
        if u is None:
            u = torch.ones(self.ndof, dtype=torch.float64, device="cuda")
        k = len(powers)
        pw = (ctypes.c_int * max(1, k))(*[int(x) for x in powers])
        null = ctypes.c_void_p(None)
        st, hist = _make_stats(history)
        code = _check(self._lib.dgs_newton_solve_powers(
            self._h, k, pw, _ptr(coef, k * self.ndof, "coef"),
            null if dirichlet is None else _ptr(dirichlet, self.ndof, "dirichlet"),
            null if b is None else _ptr(b, self.ndof, "b"), _ptr(u, self.ndof, "u"),
            float(newton_rtol), float(linear_rtol), int(max_newton), ctypes.byref(st), _stream(stream)),
            allow_not_converged=True)
        return u, _stats_dict(st, hist, code)


def _make_stats(history):
    hist = (ctypes.c_double * max(1, history))()
    st = Stats()
    st.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    st.history_capacity = history
    return st, hist


def _stats_dict(st, hist, code):
    return dict(iterations=st.iterations, newton_steps=st.newton_steps, backtracks=st.backtracks,
                rel_residual=st.rel_residual, history=[hist[i] for i in range(st.history_len)],
                t_setup_s=st.t_setup_s, t_solve_s=st.t_solve_s, converged=(code == DGS_OK))


def lgl_nodes(p):
    """The p+1 LGL points on [-1, 1] (from the library)."""
    import numpy as np
    out = (ctypes.c_double * (p + 1))()
    _check(load_library().dgs_lgl_nodes(int(p), out))
    return np.array(out[:])


def points(lower, upper, elements, p):
    """Host coordinates (3, E*N^3) of every point in the canonical layout
    (dgs_grid_coordinates)."""
    import numpy as np
    n = int(elements[0]) * int(elements[1]) * int(elements[2]) * (int(p) + 1) ** 3
    out = np.empty(3 * n)
    dom = Domain((ctypes.c_double * 3)(*lower), (ctypes.c_double * 3)(*upper))
    _check(load_library().dgs_grid_coordinates(
        ctypes.byref(dom), (ctypes.c_int * 3)(*elements), int(p),
        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n))
    return out.reshape(3, n)


class System:
    """A system of nvars variables with per-variable Neumann faces and
    pointwise couplings (see dgs_create_system).  Vectors are float64 device
    tensors of nvars * ndof entries, variable a's field at a * ndof;
    laplacian_bc "matched" or "dirichlet" selects the subdomain
    preconditioner's boundary types."""

    def __init__(self, lower, upper, elements, p, neumann_faces, laplacian_bc="matched",
                 penalty=1.5, options: Options | None = None, stream=None, **opts):
        lib = load_library()
        self._lib = lib
        self._h = None
        self.options = options if options is not None else default_options(**opts)
        masks = []
        for faces in neumann_faces:
            m = 0
            for f in faces:
                m |= 1 << int(f)
            masks.append(m)
        self.nvars = len(masks)
        dom = Domain((ctypes.c_double * 3)(*lower), (ctypes.c_double * 3)(*upper))
        h = ctypes.c_void_p()
        _check(lib.dgs_create_system(ctypes.byref(dom), (ctypes.c_int * 3)(*elements), int(p),
                                     float(penalty), self.nvars,
                                     (ctypes.c_int * max(1, self.nvars))(*masks),
                                     {"matched": 0, "dirichlet": 1}[laplacian_bc],
                                     ctypes.byref(self.options), _stream(stream), ctypes.byref(h)))
        self._h = h
        n = ctypes.c_longlong()
        _check(lib.dgs_system_num_dofs(h, ctypes.byref(n)))
        self.ndof = n.value
        self.size = self.nvars * self.ndof

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dgs_destroy_system(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self):
        import torch
        return torch.empty(self.size, dtype=torch.float64, device="cuda")

    def set_coupling(self, D=None, stream=None):
        """Couplings D (nvars * nvars * ndof, D_ab at (a * nvars + b) * ndof); None: none."""
        ptr = ctypes.c_void_p(None) if D is None else _ptr(D, self.nvars * self.size, "D")
        _check(self._lib.dgs_system_set_coupling(self._h, ptr, _stream(stream)))

    def apply(self, u, out=None, stream=None):
        out = self._new() if out is None else out
        _check(self._lib.dgs_system_apply(self._h, _ptr(u, self.size, "u"), _ptr(out, self.size, "out"),
                                          _stream(stream)))
        return out

    def smooth(self, b, u, steps=1, stream=None):
        _check(self._lib.dgs_system_smooth(self._h, _ptr(b, self.size, "b"), _ptr(u, self.size, "u"),
                                           int(steps), _stream(stream)))
        return u

    def precondition(self, r, out=None, stream=None):
        out = self._new() if out is None else out
        _check(self._lib.dgs_system_precondition(self._h, _ptr(r, self.size, "r"),
                                                 _ptr(out, self.size, "z"), _stream(stream)))
        return out

    def solve(self, b, u=None, history=256, stream=None):
        import torch
        if u is None:
            u = torch.zeros(self.size, dtype=torch.float64, device="cuda")
        st, hist = _make_stats(history)
        code = _check(self._lib.dgs_system_solve(self._h, _ptr(b, self.size, "b"),
                                                 _ptr(u, self.size, "u"), ctypes.byref(st),
                                                 _stream(stream)), allow_not_converged=True)
        return u, _stats_dict(st, hist, code)

    def set_geometry(self, xyz=None, stream=None):
        """Curved elements for every variable (3 * ndof coordinates; None: the box grid)."""
        ptr = ctypes.c_void_p(None) if xyz is None else _ptr(xyz, 3 * self.ndof, "xyz")
        _check(self._lib.dgs_system_set_geometry(self._h, ptr, _stream(stream)))

    def set_metric(self, ginv=None, sqrtg=None, stream=None):
        """A background metric for every variable (g^ij as 6 * ndof, sqrt(g) as ndof)."""
        if (ginv is None) != (sqrtg is None):
            raise ValueError("ginv and sqrtg are given together")
        null = ctypes.c_void_p(None)
        _check(self._lib.dgs_system_set_metric(
            self._h, null if ginv is None else _ptr(ginv, 6 * self.ndof, "ginv"),
            null if sqrtg is None else _ptr(sqrtg, self.ndof, "sqrtg"), _stream(stream)))

    def newton_solve_powers(self, coef, vars, powers, dirichlet=None, b=None, u=None, newton_rtol=1e-10,
                            linear_rtol=1e-4, max_newton=20, history=256, stream=None):
        """Newton on curved elements for the monomial sources: term t adds
        coef_t prod_q u_q^powers[t][q] to variable vars[t]'s source; coef a
        device tensor of len(vars) * ndof.  u: nvars * ndof (ones if None).
        Returns (u, stats dict)."""
        import torch
        if u is None:
            u = torch.ones(self.size, dtype=torch.float64, device="cuda")
        k = len(vars)
        if len(powers) != k or any(len(pw) != self.nvars for pw in powers):
            raise ValueError("one power per variable for every term")
        va = (ctypes.c_int * max(1, k))(*[int(x) for x in vars])
        pa = (ctypes.c_int * max(1, k * self.nvars))(*[int(x) for pw in powers for x in pw])
        null = ctypes.c_void_p(None)
        st, hist = _make_stats(history)
        code = _check(self._lib.dgs_system_newton_solve_powers(
            self._h, k, va, pa, _ptr(coef, k * self.ndof, "coef"),
            null if dirichlet is None else _ptr(dirichlet, self.size, "dirichlet"),
            null if b is None else _ptr(b, self.size, "b"), _ptr(u, self.size, "u"),
            float(newton_rtol), float(linear_rtol), int(max_newton), ctypes.byref(st), _stream(stream)),
            allow_not_converged=True)
        return u, _stats_dict(st, hist, code)


class Server:
    """Continuous-batching solve server (see dgs_server_* in include/dgsolve.h)."""

    def __init__(self, hbm_budget_bytes=64e9, max_active=16, penalty=1.5, host_threads=0,
                 allocator=None, batched=True, **solver_opts):
        lib = load_library()
        self._lib = lib
        o = ServerOptions()
        o.hbm_budget_bytes = float(hbm_budget_bytes)
        o.max_active = int(max_active)
        o.penalty = float(penalty)
        o.host_threads = int(host_threads)
        o.solver = default_options(**solver_opts)
        o.batched = 1 if batched else 0
        self.allocator = allocator
        if allocator is not None:
            # kept on the server: the library calls them until it is destroyed
            self._alloc_cb = ALLOC_FN(lambda nbytes, ctx: allocator.alloc(nbytes))
            self._free_cb = FREE_FN(lambda ptr, ctx: allocator.free(ptr))
            o.alloc_fn = ctypes.cast(self._alloc_cb, ctypes.c_void_p)
            o.free_fn = ctypes.cast(self._free_cb, ctypes.c_void_p)
        h = ctypes.c_void_p()
        _check(lib.dgs_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._sizes = {}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dgs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, lower, upper, elements, p, f):
        import numpy as np
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        dom = Domain((ctypes.c_double * 3)(*lower), (ctypes.c_double * 3)(*upper))
        rid = ctypes.c_longlong()
        _check(self._lib.dgs_server_submit(self._h, ctypes.byref(dom), (ctypes.c_int * 3)(*elements),
                                           int(p), f.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           f.size, ctypes.byref(rid)))
        self._sizes[rid.value] = f.size
        return rid.value

    def submit_puncture(self, lower, upper, elements, p, alpha, beta, b=None, newton_rtol=1e-10,
                        linear_rtol=1e-4, max_newton=20):
        """Queue the puncture equation A u + M S(u) = b (b = 0 when None), u = 0 on the
        box, solved by Newton from u0 = 0; alpha, beta, b are host arrays at the points."""
        import numpy as np
        dp = ctypes.POINTER(ctypes.c_double)
        a = np.ascontiguousarray(alpha, dtype=np.float64).reshape(-1)
        be = np.ascontiguousarray(beta, dtype=np.float64).reshape(-1)
        bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
        dom = Domain((ctypes.c_double * 3)(*lower), (ctypes.c_double * 3)(*upper))
        rid = ctypes.c_longlong()
        _check(self._lib.dgs_server_submit_puncture(
            self._h, ctypes.byref(dom), (ctypes.c_int * 3)(*elements), int(p), a.ctypes.data_as(dp),
            be.ctypes.data_as(dp), None if bb is None else bb.ctypes.data_as(dp), a.size,
            float(newton_rtol), float(linear_rtol), int(max_newton), ctypes.byref(rid)))
        self._sizes[rid.value] = a.size
        return rid.value

    def counters(self):
        """(server steps, batch-engine steps, their kernel launches, most
        requests the engine advanced together)."""
        c = (ctypes.c_longlong * 4)()
        _check(self._lib.dgs_server_counters(self._h, c))
        return tuple(c[i] for i in range(4))

    def timings(self):
        """Host seconds in dgs_server_step: (admission, set-up and
        per-request work; issuing the engine's steps; waiting for them; the
        engine's host part; retiring finished requests)."""
        t = (ctypes.c_double * 5)()
        _check(self._lib.dgs_server_timings(self._h, t))
        return tuple(t[i] for i in range(5))

    def step(self):
        a, q = ctypes.c_int(), ctypes.c_int()
        _check(self._lib.dgs_server_step(self._h, ctypes.byref(a), ctypes.byref(q)))
        return a.value, q.value

    def finished(self):
        c = ctypes.c_int()
        _check(self._lib.dgs_server_finished(self._h, None, 0, ctypes.byref(c)))
        ids = (ctypes.c_longlong * max(1, c.value))()
        _check(self._lib.dgs_server_finished(self._h, ids, c.value, ctypes.byref(c)))
        return [ids[i] for i in range(c.value)]

    def fetch(self, rid, history=64):
        """(u, stats, times) of a finished request; times = submit, admit, done, footprint."""
        import numpy as np
        n = self._sizes.pop(rid)
        u = np.empty(n)
        st, hist = _make_stats(history)
        times = (ctypes.c_double * 4)()
        code = _check(self._lib.dgs_server_fetch(self._h, rid, u.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                 n, ctypes.byref(st), times), allow_not_converged=True)
        return u, _stats_dict(st, hist, code), list(times)


class HpProblem:
    """An hp-nonuniform mesh (see dgs_create_hp_problem): the box split into
    blocks[0] x blocks[1] x blocks[2] equal blocks, block b refined
    block_levels[b][d] times along d, element e of degree degrees[e][d].
    Vectors are float64 device tensors of ndof entries, element by element."""

    def __init__(self, lower, upper, blocks, block_levels, degrees, penalty=1.5,
                 options: Options | None = None, stream=None, **opts):
        lib = load_library()
        self._lib = lib
        self._h = None
        self.options = options if options is not None else default_options(**opts)
        lv = [int(v) for row in block_levels for v in row]
        dg = [int(v) for row in degrees for v in row]
        ne = len(dg) // 3
        dom = Domain((ctypes.c_double * 3)(*lower), (ctypes.c_double * 3)(*upper))
        h = ctypes.c_void_p()
        _check(lib.dgs_create_hp_problem(ctypes.byref(dom), (ctypes.c_int * 3)(*blocks),
                                         (ctypes.c_int * max(1, len(lv)))(*lv),
                                         (ctypes.c_int * max(1, len(dg)))(*dg), ne, float(penalty),
                                         ctypes.byref(self.options), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.ndof = lib.dgs_hp_num_dofs(h)
        self.levels = lib.dgs_hp_num_levels(h)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.dgs_destroy_hp_problem(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, n=None):
        import torch
        return torch.empty(self.ndof if n is None else n, dtype=torch.float64, device="cuda")

    def num_classes(self, level=0):
        return self._lib.dgs_hp_num_classes(self._h, int(level))

    def node_coordinates(self, stream=None):
        xyz = self._new(3 * self.ndof)
        _check(self._lib.dgs_hp_node_coordinates(self._h, _ptr(xyz, 3 * self.ndof, "xyz"),
                                                 _stream(stream)))
        return xyz.view(3, self.ndof)

    def apply(self, u, out=None, stream=None):
        out = self._new() if out is None else out
        _check(self._lib.dgs_hp_apply_operator(self._h, _ptr(u, self.ndof, "u"), _ptr(out, self.ndof, "out"),
                                               _stream(stream)))
        return out

    def apply_mass(self, f, out=None, stream=None):
        out = self._new() if out is None else out
        _check(self._lib.dgs_hp_apply_mass(self._h, _ptr(f, self.ndof, "f"), _ptr(out, self.ndof, "out"),
                                           _stream(stream)))
        return out

    def smooth(self, b, u, steps=1, stream=None):
        _check(self._lib.dgs_hp_smooth(self._h, _ptr(b, self.ndof, "b"), _ptr(u, self.ndof, "u"),
                                       int(steps), _stream(stream)))
        return u

    def precondition(self, r, out=None, stream=None):
        out = self._new() if out is None else out
        _check(self._lib.dgs_hp_precondition(self._h, _ptr(r, self.ndof, "r"), _ptr(out, self.ndof, "z"),
                                             _stream(stream)))
        return out

    def solve(self, b, u=None, history=256, stream=None):
        import torch
        if u is None:
            u = torch.zeros(self.ndof, dtype=torch.float64, device="cuda")
        st, hist = _make_stats(history)
        code = _check(self._lib.dgs_hp_solve(self._h, _ptr(b, self.ndof, "b"), _ptr(u, self.ndof, "u"),
                                             ctypes.byref(st), _stream(stream)), allow_not_converged=True)
        return u, _stats_dict(st, hist, code)
