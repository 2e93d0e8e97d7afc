// Curved elements on a curved background metric g_ij (Sec. II: sqrt(g) in
// eqs. massmat, stiffmat and liftop): the Poisson equation
// -nabla_i (g^ij d_j u) = f in the paper's flux form, F_u^i = g^ij v_j and
// the source S_u = -Gamma^i_ik F_u^k with Gamma^i_ik = d_k ln sqrt(g).
#pragma once

#include "dgs_internal.h"

namespace dgs {

// Per-node background fields of the finest level (device): g^ij as 6 fields
// (xx, xy, xz, yy, yz, zz at f * nd), sqrt(g), and d_k ln sqrt(g) as 3 fields
// (formed at set-up as the collocation derivative of sqrt(g), divided by it).
struct CurvedMetric {
  double* ginv = nullptr;
  double* sqrtg = nullptr;
  double* dlsg = nullptr;
};

// A pointwise source S(u) = sum_t c_t(x) u^(k_t) with integer powers
// (Sec. III.A: the nonlinear sources of eq. linearized; the XCTS sources of
// eq. xcts are of this form once the other variables are fixed).  coef:
// device, nterms fields of n values.
constexpr int kMaxPowerTerms = 8;
constexpr int kMaxPower = 12;
struct PowerSource {
  int nterms = 0;
  int power[kMaxPowerTerms] = {};
  const double* coef = nullptr;
};

// Sources of a system of nv <= kSysMaxVars variables: variable var[t] of
// term t receives c_t prod_b u_b^(power[t][b]) (the XCTS equations, eq. xcts,
// are of this form when the shift is held fixed).  coef: device, nterm
// fields of n values.
constexpr int kMaxMonomials = 16;
struct MonomialSource {
  int nv = 0;
  int nterm = 0;
  int var[kMaxMonomials] = {};
  int power[kMaxMonomials][kSysMaxVars] = {};
  const double* coef = nullptr;
};

// dlsg from sqrtg (the element metric of G)
hipError_t launch_curved_metric_source(int N, const CurvedGeometry& G, CurvedMetric& Mt, long long E,
                                       hipStream_t s);
// A u (+ diag u; residual: b - (A u + diag u)) with the metric: normals and
// face measures in the metric norm, F_u = g v in the divergence and the
// fluxes, M = sqrt(g) J w w w (diag may be NULL)
hipError_t launch_curved_apply_metric(int N, bool residual, const double* u, double* out,
                                      const double* b, const double* diag, const CurvedGeometry& G,
                                      const CurvedMetric& Mt,
                                      const int* nbr, double C, int neumann, long long E, hipStream_t s);
// out = A u with Dirichlet data bvals (device, read at the Dirichlet boundary
// nodes; the ghost u_ext = 2 u_b - u_int of eq. bc), on the background metric
// when Mt is given
hipError_t launch_curved_apply_bc(int N, const double* u, double* out, const double* bvals,
                                  const CurvedGeometry& G, const CurvedMetric* Mt, const int* nbr,
                                  double C, int neumann, long long E, hipStream_t s);
// F += m S(u) - b (F may be NULL; b may be NULL) and d = m dS/du (d may be
// NULL), m the diagonal mass
hipError_t launch_power_source(const PowerSource& ps, const double* u, const double* mdiag,
                               const double* b, double* F, double* d, long long n, hipStream_t s);
// For u of nv fields of n values: F_a += m S_a(u) - b_a (F, b may be NULL)
// and D_ab = m dS_a/du_b at (a nv + b) n (D may be NULL)
hipError_t launch_monomial_source(const MonomialSource& ms, const double* u, const double* mdiag,
                                  const double* b, double* F, double* D, long long n, hipStream_t s);
// b = M f with M = sqrt(g) det(J) w_i w_j w_k
hipError_t launch_curved_mass_metric(int N, const double* f, double* out, const CurvedGeometry& G,
                                     const CurvedMetric& Mt, long long E, hipStream_t s);

}  // namespace dgs
