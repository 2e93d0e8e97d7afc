"""Plain FP64 CPU oracle of the DG multigrid-Schwarz elliptic solver.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously correct
reference that the HIP library is checked against.  Only the tests, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product library never calls it and shares no code, tables or helpers with it.

Every function follows a passage of arXiv:2111.06767 ("A scalable elliptic
solver with task-based parallelism for the SpECTRE numerical relativity
code"), cited by section and equation label:

* ``lgl``        Legendre-Gauss-Lobatto nodes, weights, Lagrange derivative and
                 interpolation matrices (Sec. II, eqs. field_expansion, lagrprod).
* ``mesh``       axis-aligned box of uniform elements (Sec. II, Fig. element).
* ``operator``   strong DG operator with the generalised internal-penalty flux
                 (Sec. II, eqs. dg_op_auxvars, dg_op_primal, massmat, stiffmat,
                 liftop, numflux, penalty, bc).
* ``schwarz``    element-centred overlapping subdomains, weights and the
                 additive Schwarz step (Sec. III.D, eqs. schwarz_subd_problem,
                 schwarz_weighting, schwarz_weight_prod,
                 schwarz_weight_function; Sec. III.E explicit inverse).
* ``multigrid``  h-coarsened hierarchy, prolongation/restriction, V-cycle
                 (Sec. III.C, eqs. prol, mg_problem, mg_res).
* ``krylov``     flexible GMRES (Sec. III.B; Saad 2003, Alg. 9.6).
* ``newton``     Newton-Raphson with backtracking line search (Sec. III.A,
                 eq. linearized; Dennis & Schnabel backtracking).

Readings of passages that are silent or ambiguous are listed in each module.

Parity status: every function is pinned by tests in ``tests/test_oracle_*``
against closed forms, textbook identities, brute-force weak-form assembly or
dense direct solves, except the values of the discretisation error itself
(only its exponential trend in p is checked): parity unpinned for the
absolute error level.
"""

from . import lgl, mesh, operator, schwarz, multigrid, krylov, newton  # noqa: F401
