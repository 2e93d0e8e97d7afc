"""MI355X (gfx950) DG multigrid-Schwarz elliptic solver (arXiv:2111.06767 hot path).

The computation lives in ``libdgsolve.so`` (HIP kernels + C++ host code behind
the C ABI of ``include/dgsolve.h``); this package only marshals arguments.
"""
from .api import (DGS_ERR_HIP, DGS_ERR_INVALID, DGS_ERR_NONFINITE, DGS_ERR_OOM, DGS_FP64,  # noqa: F401
                  DGS_MIXED, DGS_NOT_CONVERGED, DGS_OK, EXPORTED, DgsError, HpProblem, Options, Problem,
                  Server, System, TorchAllocator, default_options, lgl_nodes, load_library,
                  points)
