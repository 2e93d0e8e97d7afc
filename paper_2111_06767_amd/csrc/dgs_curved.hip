// DG Poisson operator on curved (isoparametric) elements (Sec. II: eqs.
// massmat, stiffmat and liftop with the element Jacobian; flat background
// metric).  Every node carries physical coordinates; the element map is the
// degree-p interpolant of them.
//
// With LGL quadrature on the element's own points the metric enters pointwise:
//   J^c_d = dx^c/dxi^d (collocation derivative of the coordinate fields),
//   M = det(J) w_i w_j w_k, (D_c u) = invJ^d_c (D^xi_d u),
//   on a face normal to xi^d: unit normal n_c = s invJ^d_c / |invJ^d|,
//   lifting coefficient |invJ^d| / w_end, ML = det(J) |invJ^d| w_a w_b,
//   element size normal to the face 2 / |invJ^d| (per side) in the penalty.
// Fluxes and boundary ghosts are those of the box operator (eqs. numflux, bc).
//
// Three kernels, one workgroup of N^3 threads (one per node) per element:
// the geometry (invJ and det(J) from the coordinates, at set-up), the
// physical gradient of u, and the operator, which reads the neighbours'
// values and gradients at the shared face nodes.
#include "dgs_curved.h"

#include <algorithm>

namespace dgs {
namespace {

// D^xi along dimension d at node (i, j, k) of an LDS field f[N^3]
template <int N>
__device__ __forceinline__ double dxi(const double* f, const double* D, int d, int i, int j, int k) {
  double s = 0.0;
  if (d == 0) {
#pragma unroll
    for (int m = 0; m < N; ++m) s += D[i * N + m] * f[(k * N + j) * N + m];
  } else if (d == 1) {
#pragma unroll
    for (int m = 0; m < N; ++m) s += D[j * N + m] * f[(k * N + m) * N + i];
  } else {
#pragma unroll
    for (int m = 0; m < N; ++m) s += D[k * N + m] * f[(m * N + j) * N + i];
  }
  return s;
}

// |a|_g = sqrt(g^ab a_a a_b) with g^ab as (xx, xy, xz, yy, yz, zz)
__device__ __forceinline__ double gnorm(const double G[6], double a0, double a1, double a2) {
  return sqrt(G[0] * a0 * a0 + G[3] * a1 * a1 + G[5] * a2 * a2 +
              2.0 * (G[1] * a0 * a1 + G[2] * a0 * a2 + G[4] * a1 * a2));
}

// invJ (9 fields, invJ^d_c at (3 d + c) * nd) and det(J) from the coordinates
template <int N>
__global__ void __launch_bounds__(N * N * N)
k_curved_geometry(const double* __restrict__ xyz, long long nd, const double* __restrict__ Dg,
                  double* __restrict__ inv, double* __restrict__ det) {
  constexpr int N3 = N * N * N;
  __shared__ double D[N * N];
  __shared__ double X[3][N3];
  const int t = threadIdx.x;
  const long long g = (long long)blockIdx.x * N3 + t;
  if (t < N * N) D[t] = Dg[t];
#pragma unroll
  for (int c = 0; c < 3; ++c) X[c][t] = xyz[c * nd + g];
  __syncthreads();
  const int i = t % N, j = (t / N) % N, k = t / (N * N);
  double J[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) J[c][d] = dxi<N>(X[c], D, d, i, j, k);
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  const double dt = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  const double r = 1.0 / dt;
  // inverse = adjugate / det: Inv[d][c] = cofactor(J)[c][d] / det
  double I[3][3];
  I[0][0] = c00 * r;
  I[1][0] = c01 * r;
  I[2][0] = c02 * r;
  I[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * r;
  I[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * r;
  I[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * r;
  I[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * r;
  I[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * r;
  I[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * r;
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int c = 0; c < 3; ++c) inv[(3 * d + c) * nd + g] = I[d][c];
  det[g] = dt;
}

// physical gradient grad_c u = invJ^d_c D^xi_d u (3 fields)
template <int N>
__global__ void __launch_bounds__(N * N * N)
k_curved_grad(const double* __restrict__ u, long long nd, const double* __restrict__ Dg,
              const double* __restrict__ inv, double* __restrict__ grad) {
  constexpr int N3 = N * N * N;
  __shared__ double D[N * N];
  __shared__ double U[N3];
  const int t = threadIdx.x;
  const long long g = (long long)blockIdx.x * N3 + t;
  if (t < N * N) D[t] = Dg[t];
  U[t] = u[g];
  __syncthreads();
  const int i = t % N, j = (t / N) % N, k = t / (N * N);
  double du[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) du[d] = dxi<N>(U, D, d, i, j, k);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) s += inv[(3 * d + c) * nd + g] * du[d];
    grad[c * nd + g] = s;
  }
}

// The operator: v = grad u + lifts of the auxiliary flux jumps (eq.
// dg_op_auxvars), A u = -M D_c v_c - ML ((n F_u)* - n.v) (eq. dg_op_primal),
// plus diag * u when diag is given.  RES: out = b - A u.
// bvals (optional): Dirichlet data at the boundary nodes (otherwise the
// homogeneous ghost).
// MET: on a curved background metric (the fields of CurvedMetric): normals
// and face measures in the metric norm, F_u = g v, M = sqrt(g) J w w w and
// the source -M Gamma^i_ik F_u^k.
template <int N, bool RES, bool MET = false>
__global__ void __launch_bounds__(N * N * N)
k_curved_apply(const double* __restrict__ u, const double* __restrict__ grad,
               const double* __restrict__ inv, const double* __restrict__ det, long long nd,
               const double* __restrict__ Dg, const double* __restrict__ wg,
               const int* __restrict__ nbr, double C, int neumann,
               const double* __restrict__ diag, const double* __restrict__ b,
               double* __restrict__ out, const double* __restrict__ ginv = nullptr,
               const double* __restrict__ sqrtg = nullptr, const double* __restrict__ dlsg = nullptr,
               const double* __restrict__ bvals = nullptr) {
  constexpr int N3 = N * N * N;
  __shared__ double D[N * N];
  __shared__ double V[3][N3];
  const int t = threadIdx.x;
  const long long e = blockIdx.x;
  const long long g = e * N3 + t;
  if (t < N * N) D[t] = Dg[t];
  const int ijk[3] = {t % N, (t / N) % N, t / (N * N)};
  const double ue = u[g];
  const double dt = det[g];
  double I[3][3], gr[3], v[3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int c = 0; c < 3; ++c) I[d][c] = inv[(3 * d + c) * nd + g];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    gr[c] = grad[c * nd + g];
    v[c] = gr[c];
  }
  const double W3 = wg[ijk[0]] * wg[ijk[1]] * wg[ijk[2]];
  // the metric g^ab (symmetric, 6 fields) and F of the unlifted gradient
  double Gm[6] = {1.0, 0.0, 0.0, 1.0, 0.0, 1.0}, Fg[3] = {gr[0], gr[1], gr[2]};
  if constexpr (MET) {
#pragma unroll
    for (int q = 0; q < 6; ++q) Gm[q] = ginv[q * nd + g];
    Fg[0] = Gm[0] * gr[0] + Gm[1] * gr[1] + Gm[2] * gr[2];
    Fg[1] = Gm[1] * gr[0] + Gm[3] * gr[1] + Gm[4] * gr[2];
    Fg[2] = Gm[2] * gr[0] + Gm[4] * gr[1] + Gm[5] * gr[2];
  }
  // the faces this node lies on (at most one per dimension): their normal,
  // exterior value, normal derivatives of both sides, penalty and ML
  double fn[3][3] = {}, fue[3] = {}, fndi[3] = {}, fnde[3] = {}, fsig[3] = {}, fml[3] = {};
  bool on[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int idx = ijk[d];
    on[d] = idx == 0 || idx == N - 1;
    if (!on[d]) continue;
    const int s = idx == 0 ? -1 : 1;
    const double nrm = MET ? gnorm(Gm, I[d][0], I[d][1], I[d][2])
                           : sqrt(I[d][0] * I[d][0] + I[d][1] * I[d][1] + I[d][2] * I[d][2]);
    double n[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) n[c] = s * I[d][c] / nrm;
    const double ndi = n[0] * Fg[0] + n[1] * Fg[1] + n[2] * Fg[2];
    const int f = 2 * d + (s > 0 ? 1 : 0);
    const int nb = nbr[e * 6 + f];
    double uext, ndext, nrmext;
    if (nb >= 0) {
      int m[3] = {ijk[0], ijk[1], ijk[2]};
      m[d] = N - 1 - idx;
      const long long gm = (long long)nb * N3 + (m[2] * N + m[1]) * N + m[0];
      uext = u[gm];
      const double a0 = inv[(3 * d) * nd + gm], a1 = inv[(3 * d + 1) * nd + gm],
                   a2 = inv[(3 * d + 2) * nd + gm];
      const double e0 = grad[gm], e1 = grad[nd + gm], e2 = grad[2 * nd + gm];
      if constexpr (MET) {
        double Ge[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) Ge[q] = ginv[q * nd + gm];
        ndext = n[0] * (Ge[0] * e0 + Ge[1] * e1 + Ge[2] * e2) +
                n[1] * (Ge[1] * e0 + Ge[3] * e1 + Ge[4] * e2) +
                n[2] * (Ge[2] * e0 + Ge[4] * e1 + Ge[5] * e2);
        nrmext = gnorm(Ge, a0, a1, a2);
      } else {
        ndext = n[0] * e0 + n[1] * e1 + n[2] * e2;
        nrmext = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
      }
    } else if ((neumann >> f) & 1) {
      uext = ue;  // homogeneous Neumann ghost (eq. bc)
      ndext = -ndi;
      nrmext = nrm;
    } else {
      // Dirichlet ghost (eq. bc): u_ext = 2 u_b - u_int, homogeneous without data
      uext = bvals ? 2.0 * bvals[g] - ue : -ue;
      ndext = ndi;
      nrmext = nrm;
    }
    // auxiliary lift, L (1/2 n (u_ext - u_int)) with L = |invJ^d| / w_end here
    const double lift = nrm / wg[idx] * 0.5 * (uext - ue);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c] += lift * n[c];
      fn[d][c] = n[c];
    }
    fue[d] = uext;
    fndi[d] = ndi;
    fnde[d] = ndext;
    fsig[d] = C * (double)(N * N) / fmin(2.0 / nrm, 2.0 / nrmext);
    fml[d] = dt * nrm * W3 / wg[idx];
  }
  // F_u of the lifted v (v itself for the flat metric)
  double F[3] = {v[0], v[1], v[2]};
  double sg = 1.0;
  if constexpr (MET) {
    F[0] = Gm[0] * v[0] + Gm[1] * v[1] + Gm[2] * v[2];
    F[1] = Gm[1] * v[0] + Gm[3] * v[1] + Gm[4] * v[2];
    F[2] = Gm[2] * v[0] + Gm[4] * v[1] + Gm[5] * v[2];
    sg = sqrtg[g];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) V[c][t] = F[c];
  __syncthreads();
  // -M D_c v_c with D_c = invJ^d_c D^xi_d
  double div = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) div += I[d][c] * dxi<N>(V[c], D, d, ijk[0], ijk[1], ijk[2]);
  double Au = -sg * dt * W3 * div;
  if constexpr (MET)  // + M S_u, S_u = -Gamma^i_ik F_u^k
    Au -= sg * dt * W3 * (dlsg[g] * F[0] + dlsg[nd + g] * F[1] + dlsg[2 * nd + g] * F[2]);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    if (!on[d]) continue;
    const double flux_star = 0.5 * (fndi[d] + fnde[d]) - fsig[d] * (ue - fue[d]);
    const double flux_int = fn[d][0] * F[0] + fn[d][1] * F[1] + fn[d][2] * F[2];
    Au -= sg * fml[d] * (flux_star - flux_int);
  }
  if (diag) Au += diag[g] * ue;
  out[g] = RES ? b[g] - Au : Au;
}

// d_c ln sqrt(g) = (invJ^d_c D^xi_d sqrt(g)) / sqrt(g) (3 fields)
template <int N>
__global__ void __launch_bounds__(N * N * N)
k_curved_metric_source(const double* __restrict__ sqrtg, long long nd, const double* __restrict__ Dg,
                       const double* __restrict__ inv, double* __restrict__ dlsg) {
  constexpr int N3 = N * N * N;
  __shared__ double D[N * N];
  __shared__ double S[N3];
  const int t = threadIdx.x;
  const long long g = (long long)blockIdx.x * N3 + t;
  if (t < N * N) D[t] = Dg[t];
  S[t] = sqrtg[g];
  __syncthreads();
  const int i = t % N, j = (t / N) % N, k = t / (N * N);
  double ds[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) ds[d] = dxi<N>(S, D, d, i, j, k);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double v = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) v += inv[(3 * d + c) * nd + g] * ds[d];
    dlsg[c * nd + g] = v / S[t];
  }
}

// b = M f = sqrt(g) det(J) w_i w_j w_k f
template <int N>
__global__ void __launch_bounds__(N * N * N)
k_curved_mass_metric(const double* __restrict__ f, const double* __restrict__ det,
                     const double* __restrict__ sqrtg, const double* __restrict__ wg,
                     double* __restrict__ out) {
  constexpr int N3 = N * N * N;
  const int t = threadIdx.x;
  const long long g = (long long)blockIdx.x * N3 + t;
  out[g] = sqrtg[g] * det[g] * wg[t % N] * wg[(t / N) % N] * wg[t / (N * N)] * f[g];
}

// u^k for an integer power k (|k| <= kMaxPower): repeated products, a
// reciprocal for negative powers
__device__ __forceinline__ double ipow(double u, int k) {
  double r = 1.0;
  const int m = k < 0 ? -k : k;
  for (int q = 0; q < m; ++q) r *= u;
  return k < 0 ? 1.0 / r : r;
}

// F = F + m S(u) - b and d = m dS/du(u), S(u) = sum_t c_t u^(k_t) (either
// output may be NULL; b may be NULL)
__global__ void k_power_source(PowerSource ps, const double* __restrict__ u,
                               const double* __restrict__ mdiag, const double* __restrict__ b,
                               double* __restrict__ F, double* __restrict__ d, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double ui = u[i], m = mdiag[i];
    double S = 0.0, dS = 0.0;
    for (int t = 0; t < ps.nterms; ++t) {
      const double c = ps.coef[t * n + i];
      const int k = ps.power[t];
      S += c * ipow(ui, k);
      if (k != 0) dS += c * (double)k * ipow(ui, k - 1);
    }
    if (F) F[i] = F[i] + m * S - (b ? b[i] : 0.0);
    if (d) d[i] = m * dS;
  }
}

// S_a and D_ab = dS_a/du_b of a monomial source at every point; the
// per-variable values stay in registers (compile-time indices, selected by
// the term's variable)
__global__ void k_monomial_source(MonomialSource ms, const double* __restrict__ u,
                                  const double* __restrict__ mdiag, const double* __restrict__ b,
                                  double* __restrict__ F, double* __restrict__ D, long long n) {
  constexpr int V = kSysMaxVars;
  const int nv = ms.nv;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    double uv[V], S[V], Dv[V][V];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      uv[q] = q < nv ? u[q * n + i] : 1.0;
      S[q] = 0.0;
#pragma unroll
      for (int r = 0; r < V; ++r) Dv[q][r] = 0.0;
    }
    for (int t = 0; t < ms.nterm; ++t) {
      const double c = ms.coef[t * n + i];
      const int a = ms.var[t];
      double pw[V];
#pragma unroll
      for (int q = 0; q < V; ++q) pw[q] = ipow(uv[q], ms.power[t][q]);
      double mono = c;
#pragma unroll
      for (int q = 0; q < V; ++q) mono *= pw[q];
      double dm[V];
#pragma unroll
      for (int r = 0; r < V; ++r) {
        const int k = ms.power[t][r];
        double f = k != 0 ? c * (double)k * ipow(uv[r], k - 1) : 0.0;
#pragma unroll
        for (int q = 0; q < V; ++q)
          if (q != r) f *= pw[q];
        dm[r] = f;
      }
#pragma unroll
      for (int q = 0; q < V; ++q) {
        if (q != a) continue;
        S[q] += mono;
#pragma unroll
        for (int r = 0; r < V; ++r) Dv[q][r] += dm[r];
      }
    }
    const double m = mdiag[i];
#pragma unroll
    for (int q = 0; q < V; ++q) {
      if (q >= nv) break;
      if (F) F[q * n + i] += m * S[q] - (b ? b[q * n + i] : 0.0);
      if (D) {
#pragma unroll
        for (int r = 0; r < V; ++r)
          if (r < nv) D[(long long)(q * nv + r) * n + i] = m * Dv[q][r];
      }
    }
  }
}

// b = M f = det(J) w_i w_j w_k f
template <int N>
__global__ void __launch_bounds__(N * N * N)
k_curved_mass(const double* __restrict__ f, const double* __restrict__ det,
              const double* __restrict__ wg, double* __restrict__ out) {
  constexpr int N3 = N * N * N;
  const int t = threadIdx.x;
  const long long g = (long long)blockIdx.x * N3 + t;
  out[g] = det[g] * wg[t % N] * wg[(t / N) % N] * wg[t / (N * N)] * f[g];
}

}  // namespace

// ---------------------------------------------------------------------------
#define DGS_CURVED_SWITCH(N_, CALL)      \
  switch (N_) {                          \
    case 2: CALL(2); break;              \
    case 3: CALL(3); break;              \
    case 4: CALL(4); break;              \
    case 5: CALL(5); break;              \
    case 6: CALL(6); break;              \
    case 7: CALL(7); break;              \
    case 8: CALL(8); break;              \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_curved_geometry(int N, const double* xyz, long long E, const double* D,
                                  double* inv, double* det, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  const long long nd = E * N * N * N;
#define DGS_CALL(NN)                                                                            \
  hipLaunchKernelGGL(k_curved_geometry<NN>, dim3((unsigned)E), dim3(NN * NN * NN), 0, s, xyz, nd, \
                     D, inv, det)
  DGS_CURVED_SWITCH(N, DGS_CALL)
#undef DGS_CALL
  return hipGetLastError();
}

hipError_t launch_curved_apply(int N, bool residual, const double* u, double* out, const double* b,
                               const double* diag, const CurvedGeometry& G, const int* nbr, double C,
                               int neumann, long long E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  const long long nd = E * N * N * N;
#define DGS_CALL(NN)                                                                              \
  hipLaunchKernelGGL(k_curved_grad<NN>, dim3((unsigned)E), dim3(NN * NN * NN), 0, s, u, nd, G.D,   \
                     G.inv, G.grad);                                                              \
  if (residual)                                                                                   \
    hipLaunchKernelGGL((k_curved_apply<NN, true>), dim3((unsigned)E), dim3(NN * NN * NN), 0, s, u, \
                       G.grad, G.inv, G.det, nd, G.D, G.w, nbr, C, neumann, diag, b, out);        \
  else                                                                                            \
    hipLaunchKernelGGL((k_curved_apply<NN, false>), dim3((unsigned)E), dim3(NN * NN * NN), 0, s,   \
                       u, G.grad, G.inv, G.det, nd, G.D, G.w, nbr, C, neumann, diag, b, out)
  DGS_CURVED_SWITCH(N, DGS_CALL)
#undef DGS_CALL
  return hipGetLastError();
}

hipError_t launch_curved_mass(int N, const double* f, double* out, const CurvedGeometry& G,
                              long long E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
#define DGS_CALL(NN)                                                                              \
  hipLaunchKernelGGL(k_curved_mass<NN>, dim3((unsigned)E), dim3(NN * NN * NN), 0, s, f, G.det, G.w, \
                     out)
  DGS_CURVED_SWITCH(N, DGS_CALL)
#undef DGS_CALL
  return hipGetLastError();
}

hipError_t launch_curved_apply_bc(int N, const double* u, double* out, const double* bvals,
                                  const CurvedGeometry& G, const CurvedMetric* Mt, const int* nbr,
                                  double C, int neumann, long long E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  const long long nd = E * N * N * N;
#define DGS_CALL(NN)                                                                                  \
  hipLaunchKernelGGL(k_curved_grad<NN>, dim3((unsigned)E), dim3(NN * NN * NN), 0, s, u, nd, G.D,       \
                     G.inv, G.grad);                                                                  \
  if (Mt)                                                                                             \
    hipLaunchKernelGGL((k_curved_apply<NN, false, true>), dim3((unsigned)E), dim3(NN * NN * NN), 0, s, \
                       u, G.grad, G.inv, G.det, nd, G.D, G.w, nbr, C, neumann, nullptr, nullptr, out,  \
                       Mt->ginv, Mt->sqrtg, Mt->dlsg, bvals);                                         \
  else                                                                                                \
    hipLaunchKernelGGL((k_curved_apply<NN, false, false>), dim3((unsigned)E), dim3(NN * NN * NN), 0, s, \
                       u, G.grad, G.inv, G.det, nd, G.D, G.w, nbr, C, neumann, nullptr, nullptr, out,  \
                       nullptr, nullptr, nullptr, bvals)
  DGS_CURVED_SWITCH(N, DGS_CALL)
#undef DGS_CALL
  return hipGetLastError();
}

hipError_t launch_power_source(const PowerSource& ps, const double* u, const double* mdiag,
                               const double* b, double* F, double* d, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_power_source, dim3(blocks), dim3(256), 0, s, ps, u, mdiag, b, F, d, n);
  return hipGetLastError();
}

hipError_t launch_monomial_source(const MonomialSource& ms, const double* u, const double* mdiag,
                                  const double* b, double* F, double* D, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)std::min<long long>((n + 255) / 256, 1 << 20);
  hipLaunchKernelGGL(k_monomial_source, dim3(blocks), dim3(256), 0, s, ms, u, mdiag, b, F, D, n);
  return hipGetLastError();
}

hipError_t launch_curved_metric_source(int N, const CurvedGeometry& G, CurvedMetric& Mt, long long E,
                                       hipStream_t s) {
  if (E <= 0) return hipSuccess;
  const long long nd = E * N * N * N;
#define DGS_CALL(NN)                                                                               \
  hipLaunchKernelGGL(k_curved_metric_source<NN>, dim3((unsigned)E), dim3(NN * NN * NN), 0, s, Mt.sqrtg, \
                     nd, G.D, G.inv, Mt.dlsg)
  DGS_CURVED_SWITCH(N, DGS_CALL)
#undef DGS_CALL
  return hipGetLastError();
}

hipError_t launch_curved_apply_metric(int N, bool residual, const double* u, double* out,
                                      const double* b, const double* diag, const CurvedGeometry& G,
                                      const CurvedMetric& Mt,
                                      const int* nbr, double C, int neumann, long long E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  const long long nd = E * N * N * N;
#define DGS_CALL(NN)                                                                                  \
  hipLaunchKernelGGL(k_curved_grad<NN>, dim3((unsigned)E), dim3(NN * NN * NN), 0, s, u, nd, G.D,       \
                     G.inv, G.grad);                                                                  \
  if (residual)                                                                                       \
    hipLaunchKernelGGL((k_curved_apply<NN, true, true>), dim3((unsigned)E), dim3(NN * NN * NN), 0, s,  \
                       u, G.grad, G.inv, G.det, nd, G.D, G.w, nbr, C, neumann, diag, b, out, Mt.ginv, \
                       Mt.sqrtg, Mt.dlsg);                                                            \
  else                                                                                                \
    hipLaunchKernelGGL((k_curved_apply<NN, false, true>), dim3((unsigned)E), dim3(NN * NN * NN), 0, s, \
                       u, G.grad, G.inv, G.det, nd, G.D, G.w, nbr, C, neumann, diag, b, out, Mt.ginv, \
                       Mt.sqrtg, Mt.dlsg)
  DGS_CURVED_SWITCH(N, DGS_CALL)
#undef DGS_CALL
  return hipGetLastError();
}

hipError_t launch_curved_mass_metric(int N, const double* f, double* out, const CurvedGeometry& G,
                                     const CurvedMetric& Mt, long long E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
#define DGS_CALL(NN)                                                                                \
  hipLaunchKernelGGL(k_curved_mass_metric<NN>, dim3((unsigned)E), dim3(NN * NN * NN), 0, s, f, G.det, \
                     Mt.sqrtg, G.w, out)
  DGS_CURVED_SWITCH(N, DGS_CALL)
#undef DGS_CALL
  return hipGetLastError();
}

}  // namespace dgs
