/*
 * dgsolve.h -- C ABI of the MI355X (gfx950) DG multigrid-Schwarz elliptic solver.
 *
 * Problem (arXiv:2111.06767, Sec. II, eq. matrix_eq): the discontinuous
 * Galerkin discretisation of the Poisson equation -Laplace(u) = f on an
 * axis-aligned box split into n_x * n_y * n_z equal elements, each with
 * N = p+1 Legendre-Gauss-Lobatto points per dimension, homogeneous Dirichlet
 * boundaries (or homogeneous Neumann on the faces dgs_options.neumann_faces
 * names), and the internal-penalty numerical flux with penalty parameter C
 * (eqs. dg_op_auxvars, dg_op_primal, numflux, penalty, bc).  The linear
 * system A u = b is never assembled: only A u is defined.  Nonlinear problems
 * A(u) = b are solved by repeated linearisation (Sec. III.A).
 *
 * Data layout.  Every field pointer is a DEVICE pointer to a contiguous FP64
 * array owned by the caller, in the canonical nodal layout
 *     idx = ((e * N + k) * N + j) * N + i,   e = (e_z * n_y + e_y) * n_x + e_x,
 * i.e. the x point index i fastest, then y, then z, then the element.  The
 * library owns its internal workspaces: device memory it allocates itself, or
 * through the allocator passed to dgs_create_problem.
 *
 * Streams.  All device work is enqueued on the hipStream_t passed as
 * `stream` (NULL = the null stream).  dgs_apply_operator, dgs_apply_mass,
 * dgs_node_coordinates and dgs_precondition never synchronise the host.
 * dgs_solve, dgs_cg_solve and dgs_newton_solve synchronise once per
 * iteration to read the convergence scalars.
 *
 * Return codes.  DGS_OK (0) on success; DGS_NOT_CONVERGED (1) when an
 * iteration limit was hit (outputs and stats are still valid); negative
 * values are errors, described by dgs_last_error().  No C++ exception
 * crosses this interface.  A problem handle is used by one thread at a time.
 */
#ifndef DGSOLVE_H
#define DGSOLVE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DGS_OK 0
#define DGS_NOT_CONVERGED 1
#define DGS_ERR_INVALID (-1)   /* bad argument: p outside [1,12], element count < 1,
                                  penalty <= 0, empty box, NULL pointer ...      */
#define DGS_ERR_OOM (-2)       /* device allocation failed                       */
#define DGS_ERR_HIP (-3)       /* a HIP runtime call or kernel launch failed     */
#define DGS_ERR_NONFINITE (-4) /* NaN or Inf met in a reduction                  */

#define DGS_FP64 0  /* every step in FP64                                         */
#define DGS_MIXED 1 /* Schwarz subdomain solves in FP32 on MFMA with FP32
                       accumulation; residuals, Gram-Schmidt, updates and the
                       coarsest-level smoothing stay FP64                       */

typedef struct dgs_problem dgs_problem; /* opaque, owned by the library */

/* Axis-aligned box [lower, upper] (Sec. II: a single block). */
typedef struct {
  double lower[3];
  double upper[3];
} dgs_domain;

/* Solver options; dgs_default_options() fills the defaults in brackets. */
typedef struct {
  int overlap;         /* N_overlap points into each face neighbour (Sec. III.D.1) [2] */
  int mg_levels;       /* multigrid levels incl. the finest; 0 = until no
                          dimension can be halved (Sec. III.C.1)                  [0] */
  int pre_smooth;      /* Schwarz presmoothing steps per level (Sec. III.C.3)    [3] */
  int post_smooth;     /* Schwarz postsmoothing steps per level                  [3] */
  int precision;       /* DGS_FP64 or DGS_MIXED                            [DGS_FP64] */
  int subdomain_iters; /* linearised problems only: 0 = apply the Poisson
                          subdomain inverse once; k > 0 = k iterations of GMRES
                          preconditioned by it (Sec. III.E.1), k <= 8            [3] */
  int max_iter;        /* FGMRES iteration limit (no restart)                   [200] */
  double rtol;         /* FGMRES relative residual tolerance                   [1e-10] */
  int use_graphs;      /* 1 = replay each V-cycle from a captured hipGraph        [1] */
  int restart;         /* FGMRES: 0 = no restart; m > 0 = restarted FGMRES(m),
                          cycles of at most m iterations from the true residual
                          (max_iter bounds all cycles together)                 [0] */
  int cycle;           /* multigrid cycle: 1 = V-cycle (Sec. III.C.3); 2 = W-cycle,
                          two visits of each coarser level per visit of its parent;
                          3 = F-cycle, an F-visit of the coarser level and then a
                          V-visit; a second visit starts from the first one's
                          result                                                 [1] */
  int additive;        /* 1 = additive multigrid instead (the variant of Sec. V):
                          the residual restricted to every level, each level
                          smoothed from zero with pre + post steps, the
                          prolongated corrections summed; `cycle` is unused  [0] */
  int neumann_faces;   /* bit f = 2 d + side (side 0 = low, 1 = high face of the box
                          along dimension d) set: that face carries a homogeneous
                          Neumann condition through the ghost fluxes of eq. bc;
                          the others homogeneous Dirichlet.  At least one face
                          must stay Dirichlet (63 is DGS_ERR_INVALID)            [0] */
} dgs_options;

/* Statistics of a solve.  `history` may be NULL; otherwise it receives up to
   `history_capacity` relative residual estimates (entry 0 is 1.0). */
typedef struct {
  int iterations;       /* FGMRES iterations (summed over Newton steps)          */
  int newton_steps;     /* Newton steps taken (dgs_newton_solve only)            */
  int backtracks;       /* line-search backtracks (dgs_newton_solve only)        */
  double rel_residual;  /* final true relative residual ||b-Au|| / ||b-Au0||     */
  double* history;
  int history_capacity;
  int history_len;
  double t_setup_s;     /* wall time of dgs_create_problem                        */
  double t_solve_s;     /* wall time of the last solve call                       */
} dgs_stats;

void dgs_default_options(dgs_options* opt);

/* Device allocator for a problem's own workspace (multigrid fields, class
 * tables, subdomain blocks, Krylov basis), e.g. a shim over PyTorch's caching
 * allocator.  alloc returns `bytes` of device memory on the current device,
 * aligned to 256 bytes, or NULL when it has none; free releases a pointer
 * that alloc returned.  Both are called on the thread that calls the
 * library, free only once the device has finished the problem's work.  The
 * process-wide cache of subdomain inverses, which outlives any problem, is
 * always allocated by the library itself. */
typedef void* (*dgs_alloc_fn)(size_t bytes, void* ctx);
typedef void (*dgs_free_fn)(void* ptr, void* ctx);

/* Create a problem: mesh, LGL tables, multigrid hierarchy, and the explicit
 * inverses of the Schwarz subdomain operators A_S = R_S A R_S^T
 * (Sec. III.D.2, III.E.2), built on the device.
 *   domain    box; upper > lower in every dimension
 *   elements  n_x, n_y, n_z >= 1
 *   p         polynomial degree, 1..12 (N = p+1 points per dimension)
 *   penalty   C > 0 in sigma = C (p+1)^2 / h (eq. penalty)
 *   opt       NULL = defaults
 *   alloc_fn, free_fn, alloc_ctx
 *             the problem's device allocator (both NULL = hipMalloc / hipFree;
 *             one NULL without the other is DGS_ERR_INVALID).  A NULL from
 *             alloc_fn fails the call with DGS_ERR_OOM, a pointer not aligned
 *             to 256 bytes with DGS_ERR_INVALID; what was allocated is freed.
 *   stream    hipStream_t for the set-up work
 *   out       receives the handle; free it with dgs_destroy_problem.          */
int dgs_create_problem(const dgs_domain* domain, const int elements[3], int p, double penalty,
                       const dgs_options* opt, dgs_alloc_fn alloc_fn, dgs_free_fn free_fn,
                       void* alloc_ctx, void* stream, dgs_problem** out);
int dgs_destroy_problem(dgs_problem* prob);

/* Number of degrees of freedom E * N^3. */
int dgs_num_dofs(const dgs_problem* prob, long long* n);

/* Physical coordinates of every point: xyz[d * ndof + idx], d = x, y, z. */
int dgs_node_coordinates(const dgs_problem* prob, double* xyz, void* stream);

/* b = M f with the LGL-quadrature mass matrix M = J w_i w_j w_k (eq. massmat);
 * J = det(J) at each point on curved elements (dgs_set_geometry), times
 * sqrt(g) on a background metric (dgs_set_metric). */
int dgs_apply_mass(const dgs_problem* prob, const double* f, double* b, void* stream);

/* Au = A u: the left-hand side of eq. dg_op_primal for the Poisson fluxes
 * (eq. poisson_fluxform) with homogeneous Dirichlet boundaries, homogeneous
 * Neumann on the faces the options' neumann_faces names (eq. bc); the curved
 * operator once dgs_set_geometry or dgs_set_metric has been called.  u and
 * Au must not overlap. */
int dgs_apply_operator(dgs_problem* prob, const double* u, double* Au, void* stream);

/* u <- u + sum of `steps` additive Schwarz iterations on A u = b on the
 * finest grid (Sec. III.D.5, eq. schwarz_weighting); b and u must not overlap. */
int dgs_schwarz_smooth(dgs_problem* prob, const double* b, double* u, int steps, void* stream);

/* z = one multigrid V-cycle applied to r with zero initial guess
 * (Sec. III.C.3); r and z must not overlap. */
int dgs_precondition(dgs_problem* prob, const double* r, double* z, void* stream);

/* Solve A u = b by flexible GMRES (Sec. III.B) preconditioned with one
 * V-cycle per iteration.  u holds the initial guess on entry and the solution
 * on exit.  Stops when the residual estimate drops below rtol ||b - A u0||;
 * stats->rel_residual is the true relative residual of the result. */
int dgs_solve(dgs_problem* prob, const double* b, double* u, dgs_stats* stats, void* stream);

/* Solve A u = b by preconditioned conjugate gradients (Sec. III.B, the
 * algorithm for symmetric positive definite problems; Saad 2003, Alg. 9.1)
 * with one V-cycle per iteration as the preconditioner.  The direction update
 * uses beta = (z_{k+1}, r_{k+1} - r_k) / (z_k, r_k), which keeps the method
 * usable with the V-cycle, a preconditioner that is not symmetric.  u holds
 * the initial guess on entry and the solution on exit; rtol and max_iter of
 * the options apply to the recursively updated residual, stats->rel_residual
 * is the true relative residual of the result.  DGS_NOT_CONVERGED also when a
 * direction p has p.Ap <= 0 (A not positive definite).  b and u must not
 * overlap; the call synchronises the stream once per iteration. */
int dgs_cg_solve(dgs_problem* prob, const double* b, double* u, dgs_stats* stats, void* stream);

/* dgs_cg_solve without device allocation, for callers that cannot allocate
 * device memory at the call (tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, arithmetic and results as dgs_cg_solve, but the
 * CG work vectors, reduction partials and device scalars live in a static
 * device workspace of the library instead of the problem's lazily allocated
 * Krylov buffers, and the few convergence scalars are staged through static
 * host memory.  The problem itself (created beforehand) supplies the
 * multigrid hierarchy and the captured V-cycle.  Limit: the fine level may
 * have at most 1,048,576 points (E (p+1)^3); larger problems get
 * DGS_ERR_INVALID.  The workspace (about 56 MiB) exists once per GPU for the
 * life of the process and is shared by every call on that GPU: calls that
 * overlap on one GPU (from two host threads, or on two streams) race and must
 * not be made.  Nothing in the workspace needs to start at zero: every entry
 * is written before it is read. */
int dgs_cg_solve_noalloc(dgs_problem* prob, const double* b, double* u, dgs_stats* stats,
                         void* stream);

/* Add a pointwise term: subsequent dgs_schwarz_smooth, dgs_precondition and
 * dgs_solve act on A + diag(d) (d a device field in the nodal layout, e.g. the
 * mass-weighted derivative M S'(u) of a nonlinear source, eq. linearized);
 * d = NULL removes it.  dgs_apply_operator always applies A alone.  The field
 * is copied (and restricted to the coarse grids, d_{l+1} = R d_l); the caller
 * may free d afterwards.  With subdomain_iters = k > 0 each subdomain problem
 * (A_S + diag(R_S d)) du_S = r_S is solved by k iterations of GMRES
 * preconditioned by the explicit Poisson inverse (Laplacian approximation,
 * Sec. III.E.1); with k = 0 the Poisson inverse is applied alone. */
int dgs_set_diagonal(dgs_problem* prob, const double* d, void* stream);

/* Solve the puncture-type equation Laplace(u) + beta (alpha (1+u) + 1)^-7 = f
 * in DG form A u + M S(u) = b with S(u) = -beta (alpha (1+u) + 1)^-7, by
 * Newton-Raphson with a backtracking line search (Sec. III.A).  alpha, beta
 * are nodal fields; b = M f (all zero for the vacuum puncture problem).
 * Each Newton step solves the linearisation to linear_rtol with FGMRES and a
 * multigrid-Schwarz preconditioner on the linearised operator.  u holds the
 * initial guess on entry and the solution on exit.  Converged when
 * ||F(u)|| <= newton_rtol ||F(u0)||. */
int dgs_newton_solve(dgs_problem* prob, const double* alpha, const double* beta, const double* b,
                     double* u, double newton_rtol, double linear_rtol, int max_newton,
                     dgs_stats* stats, void* stream);

/* Solve a nonlinear equation with a pointwise power-law source on curved
 * elements (Sec. III.A, eq. linearized): the DG residual
 *   F(u) = A(u; u_b) + M S(u) - b,  S(u) = sum_t c_t(x) u^(k_t),
 * with A the curved operator (on the background metric when dgs_set_metric
 * gave one), M its diagonal mass, and u_b the Dirichlet data (`dirichlet`,
 * device, ndof values read at the Dirichlet boundary nodes through the
 * ghost u_ext = 2 u_b - u_int of eq. bc; NULL = homogeneous).  The XCTS
 * equations (eq. xcts) take this form for one variable when the others are
 * held fixed, e.g. the lapse equation with S(Phi) = c_-1 / Phi + c_1 Phi +
 * c_0.  powers: host, nterms integers in [-12, 12]; coef: device, nterms
 * fields of ndof values (term t at t * ndof); b: device or NULL (zero).
 * Newton-Raphson with the backtracking line search of dgs_newton_solve;
 * each linearisation A + diag(M S'(u)) is solved to linear_rtol by FGMRES
 * preconditioned by the box grid's multigrid-Schwarz cycle on
 * A_box + diag(M S'(u)).  u holds the initial guess on entry (it must keep
 * u != 0 where negative powers appear) and the solution on exit; converged
 * when ||F(u)|| <= newton_rtol ||F(u0)||.  Needs curved elements
 * (dgs_set_geometry, or dgs_set_metric, which sets the box coordinates);
 * DGS_ERR_INVALID otherwise, for nterms outside [1, 8] or a power outside
 * [-12, 12]; DGS_ERR_NONFINITE when a residual is not finite (u = 0 under
 * a negative power).  Synchronises the stream once per Krylov iteration. */
int dgs_newton_solve_powers(dgs_problem* prob, int nterms, const int* powers, const double* coef,
                            const double* dirichlet, const double* b, double* u, double newton_rtol,
                            double linear_rtol, int max_newton, dgs_stats* stats, void* stream);

/* The subdomain solves of one Schwarz sweep alone (Sec. III.D.2, III.E.2):
 * du_S = s A_S^-1 r_S for every subdomain of multigrid level `level`
 * (0 = finest), one grouped GEMM launch on the matrix cores, repeated `reps`
 * (>= 0) times on `stream`.  It reads the level's gathered residuals r_S as
 * the last smoothing step left them (values do not change the work done) and
 * writes only library workspace, so no caller-visible state changes.  Meant
 * for timing this dominant kernel of a Schwarz step with events recorded on
 * the same stream.  *flops (may be NULL) receives the algorithmic flop count
 * of one sweep, 2 * sum over subdomains S of n_S^2.  DGS_ERR_INVALID for a
 * level outside [0, levels). */
int dgs_subdomain_solves(dgs_problem* prob, int level, int reps, double* flops, void* stream);

/* Launch shape of the operator kernel on multigrid level `level` (Sec. II
 * operator; the shape changes only how elements are grouped into workgroups,
 * never the arithmetic, so every shape gives bit-identical results):
 *   1, 2  elements per workgroup;
 *   0     the default group for p (256 / (p+1)^2 elements);
 *  -1     2 x 2 x 2 bricks of elements, whose in-brick face neighbours are
 *         read from on-chip memory (p = 7 only).
 * The autotuner sets them per level when the problem is created, one for the
 * Schwarz residual launches that store subdomain rows and one for the
 * launches that write a vector (this entry's A u among them);
 * dgs_set_apply_shape sets both (DGS_ERR_INVALID for a level outside
 * [0, levels) or a shape not listed / not available for p), and
 * dgs_get_apply_shape reads the vector-writing one into *shape. */
int dgs_set_apply_shape(dgs_problem* prob, int level, int shape);
int dgs_get_apply_shape(const dgs_problem* prob, int level, int* shape);

/* Curved (isoparametric) elements, Sec. II: eqs. massmat, stiffmat and
 * liftop with the element Jacobian, flat background metric.  xyz (device,
 * 3 * ndof doubles: all x, then all y, then all z, canonical layout) gives
 * the physical coordinates of every node of the finest grid; the element
 * maps are their degree-p interpolants and must agree on shared faces (the
 * box topology and its boundary faces stay those of the problem).  The
 * library computes the Jacobian, its determinant and inverse at every node;
 * then dgs_apply_operator, dgs_apply_mass, dgs_solve and dgs_cg_solve use
 * the curved operator (unit normals n_c = s invJ^d_c/|invJ^d|, surface
 * Jacobian det(J) |invJ^d|, element size 2/|invJ^d| in the penalty), while
 * dgs_precondition and dgs_schwarz_smooth keep the multigrid-Schwarz cycle
 * of the box grid: a preconditioner that approximates the curved operator.
 * NULL returns to the box operator.  p <= 7; DGS_ERR_INVALID for a
 * Jacobian determinant <= 0 anywhere.  dgs_newton_solve refuses a problem
 * with curved elements.  Synchronises the stream once (the determinant
 * check). */
int dgs_set_geometry(dgs_problem* prob, const double* xyz, void* stream);

/* A curved background metric g_ij on the finest grid, Sec. II: the Poisson
 * equation -nabla_i (g^ij d_j u) = f in the flux form F_u^i = g^ij v_j with
 * the source S_u = -Gamma^i_ik F_u^k (Gamma^i_ik = d_k ln sqrt(g)), and
 * sqrt(g) in eqs. massmat, stiffmat and liftop.  ginv (device, 6 * ndof
 * doubles: the fields g^xx, g^xy, g^xz, g^yy, g^yz, g^zz, one after the
 * other, canonical layout) and sqrtg (device, ndof doubles) are copied; the
 * library forms d_k ln sqrt(g) as the collocation derivative of sqrt(g) on
 * each element, divided by sqrt(g).  Unit normals and face measures are
 * taken in the metric norm |a|_g = sqrt(g^ij a_i a_j), and the penalty's
 * element size is 2 / |invJ^d|_g.  Without curved node coordinates
 * (dgs_set_geometry) the box grid's own coordinates are set first.  Then
 * dgs_apply_operator, dgs_apply_mass, dgs_solve and dgs_cg_solve use the
 * metric operator; dgs_precondition and dgs_schwarz_smooth keep the box
 * grid's flat cycle.  Both NULL returns to the flat metric (the curved
 * elements stay); dgs_set_geometry with NULL also drops the metric.
 * DGS_ERR_INVALID if only one of ginv and sqrtg is given, for p > 7, or if
 * g^ij is not positive definite or sqrt(g) not positive and finite at some
 * node (checked on the host, which synchronises the stream). */
int dgs_set_metric(dgs_problem* prob, const double* ginv, const double* sqrtg, void* stream);

/* Tile variant of the grouped subdomain-solve GEMM on multigrid level
 * `level` (Sec. III.D.2 subdomain solves; the variant changes the tiling and
 * the split of the K range, so results agree to rounding):
 *   levels whose classes all have at most 32 subdomains: 16 x 64 tiles with
 *   up to 16 (0), 4 (1), 8 (2), 2 (3) or 1 (4) K parts; other levels:
 *   32 x 128 (0), 64 x 128 (1), 32 x 64 (2), 64 x 64 (3) or 64 x 64 with a
 *   deeper K step in FP64 (4) tiles, with up to 4 K parts.
 * The autotuner sets one per level when the problem is created;
 * dgs_set_gemm_variant overrides it (DGS_ERR_INVALID for a level outside
 * [0, levels) or a variant outside [0, 4]), dgs_get_gemm_variant reads it. */
int dgs_set_gemm_variant(dgs_problem* prob, int level, int variant);
int dgs_get_gemm_variant(const dgs_problem* prob, int level, int* variant);

/* The p+1 Legendre-Gauss-Lobatto points on [-1, 1] (ascending), so that a
 * caller can place its data: point (i, j, k) of element (e_x, e_y, e_z) sits at
 * x = lower_x + h_x (e_x + (xi_i + 1) / 2), and likewise in y and z. */
int dgs_lgl_nodes(int p, double* xi);

/* Host coordinates of every point of a box grid (no problem needed), as
 * dgs_node_coordinates gives them on the device: xyz (host, 3 * n values,
 * n = n_x n_y n_z (p+1)^3) receives xyz[d * n + idx] in the canonical layout.
 * DGS_ERR_INVALID for a bad grid or an n that does not match it. */
int dgs_grid_coordinates(const dgs_domain* domain, const int elements[3], int p, double* xyz,
                         long long n);

/* ---- Serving: continuous batching of many Poisson and puncture solves on one device ----
 * Requests queue until their estimated device footprint fits in
 * hbm_budget_bytes and one of max_active slots is free; every admitted request
 * keeps its mesh, multigrid hierarchy and Krylov basis resident until it
 * finishes, and shares the subdomain inverses of a process-wide cache.  Each
 * dgs_server_step admits what fits and advances the active requests by FGMRES
 * stages (Newton steps for puncture requests), each on its own stream, so
 * requests overlap on the device: a request whose stage has finished is
 * completed and its next stage issued at once, so the device keeps working
 * between calls and a small request does not wait for a large one.  A finished request's problem
 * (hierarchy, Krylov basis, captured V-cycle graphs) stays resident for the
 * next request of the same box, grid and degree (up to 32 are kept, their
 * footprints counted against the budget); other memory is released in
 * batches (freeing waits for the whole device);
 * a request's arithmetic is the same alone or in a mix (dgs_solve on the same
 * inputs gives the same bits).  The server_* calls come from one caller thread
 * at a time; the server's own worker threads share the stage work. */
typedef struct dgs_server dgs_server;
typedef struct {
  double hbm_budget_bytes; /* admission limit on the summed request footprints      */
  int max_active;          /* at most this many requests on the device at once      */
  double penalty;          /* C of every request                                    */
  dgs_options solver;      /* options of every request                              */
  int host_threads;        /* worker threads that issue and complete the active
                              requests' stages in parallel (launching is
                              host-bound for small requests); 0 = 4              */
  dgs_alloc_fn alloc_fn;   /* device allocator of every request's memory (its
                              problem and vectors), as in dgs_create_problem;  */
  dgs_free_fn free_fn;     /* both NULL = hipMalloc / hipFree.  Called from the
                              server's worker threads too, one at a time; a
                              block is freed only after the device is done
                              with it.                                          */
  void* alloc_ctx;
  int batched;             /* 1 = advance the Poisson requests of degree p <= 8
                              together: every server step moves each of them by
                              one FGMRES iteration through launches that cover
                              all of them (one operator launch, one grouped
                              subdomain GEMM per precision and one scatter per
                              Schwarz step of the multigrid cycle, one launch
                              per transfer and per Krylov vector operation),
                              with one synchronisation per step.  Puncture
                              requests and p > 8 take the per-request path.
                              0 = every request on its own stream.              */
} dgs_server_options;

int dgs_server_create(const dgs_server_options* opt, dgs_server** out);
int dgs_server_destroy(dgs_server* server);
/* Queue -Laplace(u) = f with u = 0 on the box: f (host, n = E N^3 values in
 * the canonical layout) is copied.  *id receives the request id. */
int dgs_server_submit(dgs_server* server, const dgs_domain* domain, const int elements[3], int p,
                      const double* f, long long n, long long* id);
/* Queue the puncture equation Laplace(u) + beta (alpha (1+u) + 1)^-7 = f in
 * the DG form A u + M S(u) = b of dgs_newton_solve (Sec. III.A), with u = 0
 * on the box and u0 = 0: alpha, beta and b (host, n values each in the
 * canonical layout; b may be NULL for b = 0) are copied.  Its stages are
 * Newton steps: each linearises, solves the linear system with FGMRES to
 * linear_rtol and line-searches, on a server worker thread.  Converged when
 * ||F(u)|| <= newton_rtol ||F(0)||, else it stops after max_newton steps.
 * dgs_server_fetch fills newton_steps and backtracks.  *id receives the id. */
int dgs_server_submit_puncture(dgs_server* server, const dgs_domain* domain,
                               const int elements[3], int p, const double* alpha,
                               const double* beta, const double* b, long long n,
                               double newton_rtol, double linear_rtol, int max_newton,
                               long long* id);
/* Admit what fits, then advance the active requests: each one whose stage
 * has finished on the device is completed and its next stage issued (if none
 * of a worker's requests has finished, the worker waits for one, so every
 * call makes progress); reports the active and queued counts. */
int dgs_server_step(dgs_server* server, int* n_active, int* n_queued);
/* Counters since dgs_server_create: counters[0] server steps, [1] steps of
 * the batch engine, [2] kernel launches of those steps, [3] the most requests
 * the engine advanced together. */
int dgs_server_counters(const dgs_server* server, long long counters[4]);
/* Host seconds since dgs_server_create spent in dgs_server_step:
 * seconds[0] admission, the set-up of admitted requests and the per-request
 * work of the worker threads (overlapping the batch engine's step on the
 * device), [1] issuing the engine's steps (job tables and launches), [2]
 * waiting for them, [3] the engine's host part (the Givens updates), [4]
 * retiring finished requests (their solutions copied to the host, memory
 * released). */
int dgs_server_timings(const dgs_server* server, double seconds[5]);
/* Ids of finished requests (up to capacity) and their number. */
int dgs_server_finished(dgs_server* server, long long* ids, int capacity, int* count);
/* Copy a finished request's solution (host, n values) and stats, and release
 * it.  times[0..3] = submit, admit and completion time in seconds since the
 * server was created, and the footprint in bytes.  Returns DGS_OK,
 * DGS_NOT_CONVERGED, or DGS_ERR_OOM for a request larger than the budget. */
int dgs_server_fetch(dgs_server* server, long long id, double* u, long long n, dgs_stats* stats,
                     double times[4]);

/* ------------------------------------------------------------------------
 * Systems of several variables (Sec. III.E.1, eq. lapl_approx)
 *
 * nvars (1..5) variables u_a on one box grid.  Variable a has homogeneous
 * Neumann conditions on the faces of neumann_faces[a] (bit f = 2 d + side,
 * at least one face Dirichlet) and Dirichlet conditions elsewhere; the
 * operator is
 *     (A_sys u)_a = A^(a) u_a + sum_b D_ab u_b
 * with A^(a) the DG Poisson operator under a's conditions (Sec. II) and
 * pointwise couplings D_ab as they enter the discrete operator (for a PDE
 * term c_ab u_b, D_ab = M c_ab with the lumped mass), the form of the
 * linearised equations of a coupled system (eq. linearized).
 *
 * Preconditioner: the multigrid V-cycle (Sec. III.C) with additive Schwarz
 * smoothing (Sec. III.D) on the whole system; each subdomain problem
 * (blockdiag_a A_S^(a) + D_S) du_S = r_S is solved by opt->subdomain_iters
 * (k, 0..8) iterations of right-preconditioned GMRES whose preconditioner is
 * the Laplacian approximation: one Poisson inverse per variable, with that
 * variable's boundary types on the subdomain's external faces
 * (laplacian_bc = 0, matched) or the Dirichlet one for every variable
 * (laplacian_bc = 1, the approximation the paper compares with in Sec. IV.B);
 * k = 0 applies the approximation alone.  Coarse couplings are restricted,
 * D_{l+1} = R D_l.  Subdomains are limited to 2048 points (p <= 8 with
 * overlap 2; DGS_ERR_INVALID beyond).
 *
 * Vectors are device arrays of nvars * ndof doubles, variable a's field at
 * a * ndof in the canonical layout; D is nvars * nvars fields (D_ab at
 * (a * nvars + b) * ndof).  opt as for dgs_create_problem (its neumann_faces
 * is ignored); device memory comes from hipMalloc.  All calls are ordered on
 * `stream` (NULL: the default stream).
 * ------------------------------------------------------------------------ */
typedef struct dgs_system dgs_system; /* opaque, owned by the library */

int dgs_create_system(const dgs_domain* domain, const int elements[3], int p, double penalty,
                      int nvars, const int* neumann_faces, int laplacian_bc,
                      const dgs_options* opt, void* stream, dgs_system** out);
int dgs_destroy_system(dgs_system* sys);
/* Points per variable (ndof). */
int dgs_system_num_dofs(const dgs_system* sys, long long* n);
/* Copy the couplings D (device, nvars * nvars * ndof; NULL: no coupling)
 * and restrict them to the coarse levels. */
int dgs_system_set_coupling(dgs_system* sys, const double* D, void* stream);
/* y = A_sys u (device vectors, no overlap). */
int dgs_system_apply(dgs_system* sys, const double* u, double* y, void* stream);
/* `steps` Schwarz steps on the finest level, in place on u. */
int dgs_system_smooth(dgs_system* sys, const double* b, double* u, int steps, void* stream);
/* z = one V-cycle applied to r (z starts from zero). */
int dgs_system_precondition(dgs_system* sys, const double* r, double* z, void* stream);
/* FGMRES (Saad Alg. 9.6, restarts of opt->restart) preconditioned by the
 * V-cycle, from the initial guess in u, to the relative residual opt->rtol
 * confirmed by the true residual; DGS_OK or DGS_NOT_CONVERGED. */
int dgs_system_solve(dgs_system* sys, const double* b, double* u, dgs_stats* stats, void* stream);

/* Curved elements and a background metric for every variable of the system
 * (as dgs_set_geometry and dgs_set_metric on each variable's operator):
 * dgs_system_apply and dgs_system_solve then use the curved operators, the
 * V-cycle keeps the box grids'.  Same arguments and errors as the scalar
 * calls. */
int dgs_system_set_geometry(dgs_system* sys, const double* xyz, void* stream);
int dgs_system_set_metric(dgs_system* sys, const double* ginv, const double* sqrtg, void* stream);

/* Newton-Raphson (Sec. III.A) for the system on curved elements with sources
 * that are sums of monomials in all variables,
 *   F_a(u) = A_a(u_a; u_b,a) + M S_a(u) - b_a,
 *   S_a(u) = sum over the terms t with vars[t] = a of c_t prod_q u_q^k(t,q),
 * the form the XCTS equations (eq. xcts) take when the shift is held fixed.
 * A_a is variable a's curved operator (its own Neumann faces; on the metric
 * when one is set) with Dirichlet data `dirichlet` (device, nvars * ndof,
 * variable a at a * ndof, read at its Dirichlet boundary nodes through the
 * ghost of eq. bc; NULL = homogeneous).  vars: host, nterms variable
 * indices; powers: host, nterms * nvars integers in [-12, 12] (term t at
 * t * nvars); coef: device, nterms fields of ndof values; b: device
 * (nvars * ndof) or NULL (zero); u: device, nvars * ndof, the initial guess
 * on entry and the solution on exit.  Each step sets the couplings
 * D_ab = M dS_a/du_b and solves the linearisation to linear_rtol by FGMRES
 * preconditioned by the system V-cycle (its subdomain problems carry D,
 * Sec. III.E.1), then backtracks the step length as dgs_newton_solve does;
 * converged when ||F(u)|| <= newton_rtol ||F(u0)||.  The couplings are
 * cleared on return.  Needs curved elements on every variable
 * (dgs_system_set_geometry or dgs_system_set_metric); DGS_ERR_INVALID
 * otherwise, for nterms outside [1, 16], a variable index outside
 * [0, nvars) or a power outside [-12, 12]; DGS_ERR_NONFINITE when a residual
 * is not finite. */
int dgs_system_newton_solve_powers(dgs_system* sys, int nterms, const int* vars, const int* powers,
                                   const double* coef, const double* dirichlet, const double* b,
                                   double* u, double newton_rtol, double linear_rtol, int max_newton,
                                   dgs_stats* stats, void* stream);

/* ---- hp-nonuniform meshes (Sec. II: blocks split into elements by h
 * refinement with two-to-one balance, elements of their own degree; Sec.
 * III.C.1: coarsening keeps the smaller degree) ------------------------------
 *
 * The box `domain` is a grid of blocks[0] x blocks[1] x blocks[2] equal
 * blocks, numbered x fastest.  Block b is split 2^L times along dimension d,
 * L = block_levels[3 b + d] in [0, 10]; the levels of face neighbours may
 * differ by at most one along every dimension of their shared face
 * (DGS_ERR_INVALID otherwise).  Elements are numbered block by block and x
 * fastest inside a block; element e has degree degrees[3 e + d] in [1, 7]
 * along dimension d (N_d = degree + 1 points).  num_elements must equal the
 * sum over blocks of 2^(L_x + L_y + L_z).
 *
 * Data layout: element by element, element e's N_x N_y N_z nodes in
 * [k][j][i] order (x fastest), FP64, device pointers owned by the caller.
 *
 * Faces shared by elements of different degree or size carry mortars: both
 * sides' traces and normal derivatives are interpolated to the mortar (the
 * larger degree per face dimension over the common part of the faces), the
 * internal-penalty fluxes (eqs. numflux, penalty, with the degree and width
 * normal to the face) are evaluated there and projected back to each
 * element's face points by the exact L2 projection.  The operator is not
 * symmetric on nonconforming faces (lumped element mass against the exact
 * projection), so the solver is FGMRES; CG is not offered.
 *
 * Schwarz subdomains reach N_overlap points into every face neighbour, all
 * neighbours of a finer face included; each point's weights come from its
 * own element and sum to one.  Subdomains of equal structure share one
 * explicit inverse, built on the device.  Options: overlap, mg_levels,
 * pre_smooth, post_smooth, max_iter, rtol, restart, neumann_faces,
 * precision (DGS_MIXED: FP32 subdomain solves on every level but the
 * coarsest, as for box grids) and use_graphs (the V-cycle captured at set-up
 * and replayed) apply; cycle must be 1 and additive 0 (DGS_ERR_INVALID
 * otherwise); the other fields are unused.  Workspaces are allocated with
 * hipMalloc.  The set-up synchronises the stream. */
typedef struct dgs_hp_problem dgs_hp_problem;
int dgs_create_hp_problem(const dgs_domain* domain, const int blocks[3], const int* block_levels,
                          const int* degrees, int num_elements, double penalty,
                          const dgs_options* opt, void* stream, dgs_hp_problem** out);
int dgs_destroy_hp_problem(dgs_hp_problem* prob);
/* Points of the finest mesh (-1 for NULL). */
long long dgs_hp_num_dofs(const dgs_hp_problem* prob);
/* Multigrid levels, and the number of distinct subdomain inverses of one
 * level (-1 for a bad argument). */
int dgs_hp_num_levels(const dgs_hp_problem* prob);
int dgs_hp_num_classes(const dgs_hp_problem* prob, int level);
/* xyz (device, 3 * ndof): xyz[d * ndof + idx], the node coordinates.
 * Synchronises the stream. */
int dgs_hp_node_coordinates(dgs_hp_problem* prob, double* xyz, void* stream);
/* Au = A u and Mf = M f (eq. massmat) on the finest mesh; no synchronisation. */
int dgs_hp_apply_operator(dgs_hp_problem* prob, const double* u, double* Au, void* stream);
int dgs_hp_apply_mass(dgs_hp_problem* prob, const double* f, double* Mf, void* stream);
/* `steps` additive Schwarz steps on the finest mesh, in place on u. */
int dgs_hp_smooth(dgs_hp_problem* prob, const double* b, double* u, int steps, void* stream);
/* z = one V-cycle applied to r (z starts from zero). */
int dgs_hp_precondition(dgs_hp_problem* prob, const double* r, double* z, void* stream);
/* FGMRES preconditioned by the V-cycle from the initial guess in u, to the
 * relative residual opt->rtol confirmed by the true residual; DGS_OK or
 * DGS_NOT_CONVERGED.  Synchronises once per iteration. */
int dgs_hp_solve(dgs_hp_problem* prob, const double* b, double* u, dgs_stats* stats, void* stream);

/* Message of the last error on the calling thread ("" if none). */
const char* dgs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DGSOLVE_H */
