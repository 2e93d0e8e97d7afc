// DG operator apply on gfx950 (Sec. II, eqs. dg_op_auxvars, dg_op_primal,
// massmat, stiffmat, liftop, numflux, penalty, bc).
//
// One kernel computes A u for a batch of elements.  Each element is handled by
// N^2 lanes; lane (i, j) owns the z-line of points (i, j, 0..N-1) in
// registers.  Derivatives along z stay in registers, derivatives along x and
// y go through LDS (sum factorisation).  The neighbour data the numerical flux
// needs (the neighbour's trace and its own normal derivative on the shared
// face) is computed from the neighbour's points read straight from global
// memory, so the whole apply is one pass: read u, write A u.
//
// With LGL quadrature the strong form is evaluated through summation by parts,
//   -M D_d v_d + ML_d n_d v_d = D_d^T M v_d      (exact for LGL points),
// so that
//   A u = sum_d D_d^T (M v_d) - sum_faces ML_f (n F_u)*,
//   v_d = D_d u + L_d (1/2) n_d (u_ext - u_int)  on the faces normal to d,
//   (n F_u)* = 1/2 n.(grad u_int + grad u_ext) - sigma (u_int - u_ext).
// Dirichlet faces use the ghost state u_ext = -u_int, grad u_ext = grad u_int.
#include "dgs_internal.h"

namespace dgs {
namespace {

// Point with index m along dimension d and transverse indices (a, b) (lower
// transverse dimension first), as an offset inside one element.
template <int N>
__device__ __forceinline__ int face_line_point(int d, int m, int a, int b) {
  if (d == 0) return (b * N + a) * N + m;
  if (d == 1) return (b * N + m) * N + a;
  return (m * N + b) * N + a;
}

template <int N, int EPB>
__global__ void __launch_bounds__(256)
k_apply(const double* __restrict__ u, double* __restrict__ out, const double* __restrict__ bvec,
        const double* __restrict__ aux0, const double* __restrict__ aux1,
        const int* __restrict__ nbr, OpParams P, DevTables T, int mode) {
  constexpr int N2 = N * N, N3 = N2 * N;
  __shared__ double sD[N * N];
  __shared__ double sw[N];
  __shared__ double su[EPB][N3];
  __shared__ double sq[EPB][N3];
  __shared__ double sf[EPB][6][2][N2];

  const int tid = threadIdx.x;
  for (int t = tid; t < N * N; t += blockDim.x) sD[t] = T.D[t];
  if (tid < N) sw[tid] = T.w[tid];
  const int slot = tid / N2;
  const int ij = tid - slot * N2;
  const int i = ij % N, j = ij / N;
  const long long e = (long long)blockIdx.x * EPB + slot;
  const bool active = (slot < EPB) && (e < P.E);
  const double rh0 = 2.0 / P.h[0], rh1 = 2.0 / P.h[1], rh2 = 2.0 / P.h[2];

  double uk[N];
  int nb[6];
  if (active) {
    const double* ue = u + e * N3;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      uk[k] = ue[k * N2 + ij];
      su[slot][k * N2 + ij] = uk[k];
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) nb[f] = nbr[e * 6 + f];
  }
  __syncthreads();

  // Neighbour trace and neighbour normal derivative on each shared face.
  if (active) {
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      if (nb[f] < 0) continue;
      const int d = f >> 1;
      const int fi = (f & 1) ? 0 : N - 1;  // neighbour's layer on the shared face
      const double* ub = u + (long long)nb[f] * N3;
      double dn = 0.0, ue = 0.0;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const double v = ub[face_line_point<N>(d, m, i, j)];
        dn += sD[fi * N + m] * v;
        if (m == fi) ue = v;
      }
      const double rh = d == 0 ? rh0 : (d == 1 ? rh1 : rh2);
      sf[slot][f][0][ij] = ue;
      sf[slot][f][1][ij] = dn * rh;
    }
  }

  double gx[N], gy[N], gz[N], au[N];
  const double J = P.h[0] * P.h[1] * P.h[2] * 0.125;
  if (active) {
    const double* s = su[slot];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        ax += sD[i * N + m] * s[k * N2 + j * N + m];
        ay += sD[j * N + m] * s[k * N2 + m * N + i];
        az += sD[k * N + m] * uk[m];
      }
      gx[k] = ax * rh0;
      gy[k] = ay * rh1;
      gz[k] = az * rh2;
      au[k] = 0.0;
    }
  }
  __syncthreads();  // neighbour face data visible

  if (active) {
    const double wend = sw[0];
    // faces normal to x: lanes with i = 0 (f = 0) or i = N-1 (f = 1)
    if (i == 0 || i == N - 1) {
      const int f = (i == 0) ? 0 : 1;
      const double sgn = (i == 0) ? -1.0 : 1.0;
      const double sig = P.penalty * (double)(N * N) / P.h[0];
      const double JF = J * rh0;
      const double lf = 1.0 / (P.h[0] * wend);
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const int fn = j + N * k;
        const double ui = uk[k], gi = gx[k];
        double ue, ge;
        if (nb[f] >= 0) {
          ue = sf[slot][f][0][fn];
          ge = sf[slot][f][1][fn];
        } else {
          ue = -ui;
          ge = gi;
        }
        au[k] -= JF * sw[j] * sw[k] * (0.5 * sgn * (gi + ge) - sig * (ui - ue));
        gx[k] += lf * sgn * (ue - ui);
      }
    }
    // faces normal to y: lanes with j = 0 (f = 2) or j = N-1 (f = 3)
    if (j == 0 || j == N - 1) {
      const int f = (j == 0) ? 2 : 3;
      const double sgn = (j == 0) ? -1.0 : 1.0;
      const double sig = P.penalty * (double)(N * N) / P.h[1];
      const double JF = J * rh1;
      const double lf = 1.0 / (P.h[1] * wend);
#pragma unroll
      for (int k = 0; k < N; ++k) {
        const int fn = i + N * k;
        const double ui = uk[k], gi = gy[k];
        double ue, ge;
        if (nb[f] >= 0) {
          ue = sf[slot][f][0][fn];
          ge = sf[slot][f][1][fn];
        } else {
          ue = -ui;
          ge = gi;
        }
        au[k] -= JF * sw[i] * sw[k] * (0.5 * sgn * (gi + ge) - sig * (ui - ue));
        gy[k] += lf * sgn * (ue - ui);
      }
    }
    // faces normal to z: every lane, points k = 0 (f = 4) and k = N-1 (f = 5)
    {
      const double sig = P.penalty * (double)(N * N) / P.h[2];
      const double JF = J * rh2;
      const double lf = 1.0 / (P.h[2] * wend);
      const double wf = JF * sw[i] * sw[j];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int f = 4 + side;
        const int k = side ? N - 1 : 0;
        const double sgn = side ? 1.0 : -1.0;
        const double ui = uk[k], gi = gz[k];
        double ue, ge;
        if (nb[f] >= 0) {
          ue = sf[slot][f][0][ij];
          ge = sf[slot][f][1][ij];
        } else {
          ue = -ui;
          ge = gi;
        }
        au[k] -= wf * (0.5 * sgn * (gi + ge) - sig * (ui - ue));
        gz[k] += lf * sgn * (ue - ui);
      }
    }
  }
  __syncthreads();  // every lane has finished reading su
  if (active) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const double jw = J * sw[i] * sw[j] * sw[k];
      su[slot][k * N2 + ij] = jw * gx[k];
      sq[slot][k * N2 + ij] = jw * gy[k];
      gz[k] *= jw;
    }
  }
  __syncthreads();
  if (active) {
    const double* qx = su[slot];
    const double* qy = sq[slot];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        ax += sD[m * N + i] * qx[k * N2 + j * N + m];
        ay += sD[m * N + j] * qy[k * N2 + m * N + i];
        az += sD[m * N + k] * gz[m];
      }
      double r = au[k] + rh0 * ax + rh1 * ay + rh2 * az;
      const long long g = e * N3 + k * N2 + ij;
      switch (mode) {
        case kApply:
          break;
        case kResidual:
          r = bvec[g] - r;
          break;
        case kApplyDiag:
          r += aux0[g] * uk[k];
          break;
        case kResidualDiag:
          r = bvec[g] - (r + aux0[g] * uk[k]);
          break;
        case kPuncture: {
          const double t = aux0[g] * (1.0 + uk[k]) + 1.0;
          const double t2 = t * t, t4 = t2 * t2;
          const double S = -aux1[g] / (t4 * t2 * t);
          r += J * sw[i] * sw[j] * sw[k] * S - bvec[g];
          break;
        }
        default:
          break;
      }
      out[g] = r;
    }
  }
}

template <int N, int EPB>
hipError_t launch_apply_t(int mode, const double* u, double* out, const double* b,
                          const double* aux0, const double* aux1, const int* nbr,
                          const OpParams& P, const DevTables& T, hipStream_t s) {
  if (P.E <= 0) return hipSuccess;
  const int threads = ((EPB * N * N + 63) / 64) * 64;
  const long long blocks = ((long long)P.E + EPB - 1) / EPB;
  hipLaunchKernelGGL((k_apply<N, EPB>), dim3((unsigned)blocks), dim3(threads), 0, s, u, out, b,
                     aux0, aux1, nbr, P, T, mode);
  return hipGetLastError();
}

template <int N>
hipError_t launch_apply_n(int epb, int mode, const double* u, double* out, const double* b,
                          const double* aux0, const double* aux1, const int* nbr,
                          const OpParams& P, const DevTables& T, hipStream_t s) {
  constexpr int def = (N == 2) ? 64 : (256 / (N * N));  // >= 3 for every N <= 9
  if (epb == 1) return launch_apply_t<N, 1>(mode, u, out, b, aux0, aux1, nbr, P, T, s);
  if (epb == 2) return launch_apply_t<N, 2>(mode, u, out, b, aux0, aux1, nbr, P, T, s);
  return launch_apply_t<N, def>(mode, u, out, b, aux0, aux1, nbr, P, T, s);
}

// b = M f, M = J w_i w_j w_k
__global__ void k_mass(const double* __restrict__ f, double* __restrict__ out, long long total,
                       int N, double J, DevTables T) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int N3 = N * N * N;
  const int loc = (int)(g % N3);
  const int i = loc % N, j = (loc / N) % N, k = loc / (N * N);
  out[g] = J * T.w[i] * T.w[j] * T.w[k] * f[g];
}

__global__ void k_coords(double* __restrict__ xyz, long long total, int N, int nx, int ny,
                         double lx, double ly, double lz, double hx, double hy, double hz,
                         DevTables T) {
  const double* xi = T.xi;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int N3 = N * N * N;
  const long long e = g / N3;
  const int loc = (int)(g % N3);
  const int i = loc % N, j = (loc / N) % N, k = loc / (N * N);
  const int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = (int)(e / ((long long)nx * ny));
  xyz[g] = lx + hx * (ex + 0.5 * (xi[i] + 1.0));
  xyz[total + g] = ly + hy * (ey + 0.5 * (xi[j] + 1.0));
  xyz[2 * total + g] = lz + hz * (ez + 0.5 * (xi[k] + 1.0));
}

}  // namespace

hipError_t launch_apply(int N, int mode, const double* u, double* out, const double* b,
                        const double* aux0, const double* aux1, const int* nbr, const OpParams& P,
                        const DevTables& T, const ApplyConfig& cfg, hipStream_t s) {
  switch (N) {
    case 2: return launch_apply_n<2>(cfg.epb, mode, u, out, b, aux0, aux1, nbr, P, T, s);
    case 3: return launch_apply_n<3>(cfg.epb, mode, u, out, b, aux0, aux1, nbr, P, T, s);
    case 4: return launch_apply_n<4>(cfg.epb, mode, u, out, b, aux0, aux1, nbr, P, T, s);
    case 5: return launch_apply_n<5>(cfg.epb, mode, u, out, b, aux0, aux1, nbr, P, T, s);
    case 6: return launch_apply_n<6>(cfg.epb, mode, u, out, b, aux0, aux1, nbr, P, T, s);
    case 7: return launch_apply_n<7>(cfg.epb, mode, u, out, b, aux0, aux1, nbr, P, T, s);
    case 8: return launch_apply_n<8>(cfg.epb, mode, u, out, b, aux0, aux1, nbr, P, T, s);
    case 9: return launch_apply_n<9>(cfg.epb, mode, u, out, b, aux0, aux1, nbr, P, T, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mass(int N, const double* f, double* out, long long E, const double h[3],
                       const DevTables& T, hipStream_t s) {
  const long long total = E * N * N * N;
  if (total <= 0) return hipSuccess;
  const double J = h[0] * h[1] * h[2] * 0.125;
  hipLaunchKernelGGL(k_mass, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, f, out, total,
                     N, J, T);
  return hipGetLastError();
}

hipError_t launch_coords(int N, double* xyz, const int n[3], const double lower[3],
                         const double h[3], const DevTables& T, hipStream_t s) {
  const long long total = (long long)n[0] * n[1] * n[2] * N * N * N;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coords, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, xyz, total,
                     N, n[0], n[1], lower[0], lower[1], lower[2], h[0], h[1], h[2], T);
  return hipGetLastError();
}

}  // namespace dgs
