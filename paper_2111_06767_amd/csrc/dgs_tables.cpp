// Host-side Legendre-Gauss-Lobatto tables (Sec. II, eqs. field_expansion, lagrprod).
//
// Nodes: the endpoints and the roots of P'_{N-1}, found by Newton iteration
// on P'_{N-1} started from the Chebyshev-Gauss-Lobatto points, with P''
// from Legendre's differential equation.  Weights 2 / (N (N-1) P_{N-1}^2).
// Derivative matrix from the closed form for LGL points
//   D_ij = P_{N-1}(x_i) / (P_{N-1}(x_j) (x_i - x_j)),  i != j,
//   D_00 = -N(N-1)/4,  D_{N-1,N-1} = N(N-1)/4,  other diagonal entries 0.
// Child interpolation (Sec. III.C.2, eq. prol) by the barycentric formula at
// the parent-logical points (x - 1)/2 and (x + 1)/2.
#include <cmath>
#include <cstring>

#include "dgs_internal.h"

namespace dgs {
namespace {

// P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, double x, double& P, double& dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int k = 1; k < n; ++k) {
    double p2 = ((2.0 * k + 1.0) * x * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  // derivative from n (x P_n - P_{n-1}) / (x^2 - 1); valid off the endpoints
  dP = n * (x * p1 - p0) / (x * x - 1.0);
}

}  // namespace

HostTables make_tables(int N) {
  HostTables t;
  t.N = N;
  t.xi.assign(N, 0.0);
  t.w.assign(N, 0.0);
  const int n = N - 1;
  t.xi[0] = -1.0;
  t.xi[N - 1] = 1.0;
  for (int m = 1; m < N - 1; ++m) {
    double x = -std::cos(M_PI * m / n);
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, x, P, dP);
      double d2P = (2.0 * x * dP - n * (n + 1.0) * P) / (1.0 - x * x);
      double dx = dP / d2P;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    t.xi[m] = x;
  }
  std::vector<double> Pn(N);
  for (int m = 0; m < N; ++m) {
    double P, dP;
    if (m == 0 || m == N - 1) {
      P = (m == 0 && (n % 2 == 1)) ? -1.0 : 1.0;  // P_n(-1) = (-1)^n, P_n(1) = 1
    } else {
      legendre(n, t.xi[m], P, dP);
    }
    Pn[m] = P;
    t.w[m] = 2.0 / (N * (N - 1.0) * P * P);
  }
  t.D.assign(N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      if (i != j) t.D[i * N + j] = Pn[i] / (Pn[j] * (t.xi[i] - t.xi[j]));
  t.D[0] = -N * (N - 1.0) / 4.0;
  t.D[(N - 1) * N + N - 1] = N * (N - 1.0) / 4.0;
  // the LGL points are symmetric, so D[N-1-i][N-1-j] = -D[i][j]; impose it on
  // the rounded values so the even-odd evaluation is exact to rounding
  {
    std::vector<double> Ds(N * N);
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j)
        Ds[i * N + j] = 0.5 * (t.D[i * N + j] - t.D[(N - 1 - i) * N + (N - 1 - j)]);
    t.D = Ds;
  }

  // barycentric weights
  std::vector<double> lam(N, 1.0);
  for (int j = 0; j < N; ++j)
    for (int m = 0; m < N; ++m)
      if (m != j) lam[j] /= (t.xi[j] - t.xi[m]);
  auto interp = [&](double target, double* row) {
    for (int b = 0; b < N; ++b) {
      if (target == t.xi[b]) {
        for (int c = 0; c < N; ++c) row[c] = (c == b) ? 1.0 : 0.0;
        return;
      }
    }
    double den = 0.0;
    for (int b = 0; b < N; ++b) den += lam[b] / (target - t.xi[b]);
    for (int b = 0; b < N; ++b) row[b] = lam[b] / (target - t.xi[b]) / den;
  };
  t.Plo.assign(N * N, 0.0);
  t.Phi.assign(N * N, 0.0);
  for (int a = 0; a < N; ++a) {
    interp(0.5 * (t.xi[a] - 1.0), &t.Plo[a * N]);
    interp(0.5 * (t.xi[a] + 1.0), &t.Phi[a * N]);
  }
  return t;
}

void set_derived(OpParams& P, int N, double w_end) {
  for (int d = 0; d < 3; ++d) {
    P.rh[d] = 2.0 / P.h[d];
    P.sig[d] = P.penalty * (double)(N * N) / P.h[d];  // eq. penalty, p_int = p_ext
    P.lf[d] = 1.0 / (P.h[d] * w_end);
  }
  P.J = P.h[0] * P.h[1] * P.h[2] * 0.125;
}

namespace {
void even_odd(const std::vector<double>& M, int N, bool transpose, EvenOdd& eo) {
  auto at = [&](int i, int j) { return transpose ? M[j * N + i] : M[i * N + j]; };
  const int H = N / 2;
  for (int i = 0; i < H; ++i)
    for (int m = 0; m < H; ++m) {
      eo.P[i * H + m] = 0.5 * (at(i, m) + at(i, N - 1 - m));
      eo.Q[i * H + m] = 0.5 * (at(i, m) - at(i, N - 1 - m));
    }
  if (N % 2 == 1) {
    for (int i = 0; i < H; ++i) eo.cf[i] = at(i, H);
    for (int m = 0; m < H; ++m) eo.rc[m] = at(H, m);
  }
}
}  // namespace

DevTables to_dev(const HostTables& t) {
  DevTables d;
  std::memset(&d, 0, sizeof(d));
  const int N = t.N;
  even_odd(t.D, N, false, d.fwd);
  even_odd(t.D, N, true, d.bwd);
  for (int i = 0; i < N; ++i) {
    d.xi[i] = t.xi[i];
    d.w[i] = t.w[i];
  }
  for (int m = 0; m < N; ++m) {
    d.D0[m] = t.D[m];
    d.DN[m] = t.D[(N - 1) * N + m];
  }
  return d;
}

MgTables to_dev_mg(const HostTables& t) {
  MgTables d;
  std::memset(&d, 0, sizeof(d));
  for (int i = 0; i < t.N * t.N; ++i) {
    d.Plo[i] = t.Plo[i];
    d.Phi[i] = t.Phi[i];
  }
  return d;
}

}  // namespace dgs
