// Vector kernels of the Krylov and Newton solvers, and the set-up kernels
// that build the explicit subdomain inverses (Sec. III.B, III.A, III.E.2).
//
// Reductions are two-stage with a fixed block count per vector length and a
// fixed summation order, so every dot product is bitwise reproducible.
#include "dgs_internal.h"
#include "dgs_dot.h"

namespace dgs {
namespace {

__global__ void k_fill(double* x, double v, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) x[g] = v;
}

// Values in [-0.5, 0.5) from a multiplicative hash of the index: operand
// data for timing runs, whose MFMA power draw (and clock) depends on the bits.
template <typename T>
__global__ void k_fill_pattern(T* x, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) {
    const unsigned h = (unsigned)(g * 2654435761ull) ^ (unsigned)(g >> 13);
    x[g] = (T)((double)h * (1.0 / 4294967296.0) - 0.5);
  }
}

__global__ void k_copy(double* __restrict__ y, const double* __restrict__ x, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) y[g] = x[g];
}

__global__ void k_axpy(double* __restrict__ y, double a, const double* __restrict__ x, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) y[g] += a * x[g];
}

__global__ void k_waxpy(double* __restrict__ y, const double* __restrict__ x, double lam,
                        const double* __restrict__ dx, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) y[g] = x[g] + lam * dx[g];
}

// One conjugate-gradient update with the step length formed on the device:
// alpha = rz / (p . q) (0 when p . q <= 0, a breakdown the caller detects from
// the same value), x += alpha p, r_next = r - alpha q.
__global__ void k_cg_step(double* __restrict__ x, double* __restrict__ r_next,
                          const double* __restrict__ r, const double* __restrict__ p,
                          const double* __restrict__ q, double rz, const double* __restrict__ pq,
                          long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const double d = pq[0];
  const double alpha = d > 0.0 ? rz / d : 0.0;
  x[g] += alpha * p[g];
  r_next[g] = r[g] - alpha * q[g];
}

__global__ void __launch_bounds__(kDotThreads)
k_multidot_partial(const double* __restrict__ V, long long ldv, int m, const double* __restrict__ w,
                   long long n, long long chunk, double* __restrict__ partial) {
  __shared__ double red[kDotGroup * (kDotThreads / 64)];
  const long long start = (long long)blockIdx.x * chunk;
  const long long end = start + chunk < n ? start + chunk : n;
  chunk_dots(V, ldv, m, w, start, end, red, partial);
}

// w -= sum_{i < m} coef_i V_i, then partial dots of V_0..V_{m-1} with the new
// w (norm_only = 0), or of w with itself (norm_only = 1, one value per block).
__global__ void __launch_bounds__(kDotThreads)
k_axpy_multidot_partial(const double* __restrict__ V, long long ldv, int m,
                        const double* __restrict__ coef, double* w, long long n, long long chunk,
                        int norm_only, double* __restrict__ partial) {
  __shared__ double red[kDotGroup * (kDotThreads / 64)];
  const long long start = (long long)blockIdx.x * chunk;
  const long long end = start + chunk < n ? start + chunk : n;
  for (long long g = start + threadIdx.x; g < end; g += kDotThreads) {
    double acc = w[g];
    for (int i = 0; i < m; ++i) acc -= coef[i] * V[(long long)i * ldv + g];
    w[g] = acc;
  }
  if (norm_only) {
    double acc[1] = {0.0};
    for (long long g = start + threadIdx.x; g < end; g += kDotThreads) acc[0] += w[g] * w[g];
    group_store<1>(acc, red, partial + blockIdx.x, 1);
  } else {
    chunk_dots(V, ldv, m, w, start, end, red, partial);
  }
}

// h[i] = sum_b partial[b * m + i], one block per i, fixed order
__global__ void __launch_bounds__(kDotThreads)
k_multidot_final(const double* __restrict__ partial, int nblocks, int m, double* __restrict__ h) {
  __shared__ double red[kDotThreads / 64];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kDotThreads) s += partial[(long long)b * m + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) h[i] = s;
}

__global__ void k_multi_axpy(double* __restrict__ w, const double* __restrict__ V, long long ldv,
                             int m, const double* __restrict__ coef, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  double acc = w[g];
  for (int i = 0; i < m; ++i) acc -= coef[i] * V[(long long)i * ldv + g];
  w[g] = acc;
}

__global__ void k_combine(double* __restrict__ x, const double* __restrict__ Z, long long ldz, int m,
                          const double* __restrict__ y, long long n) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  double acc = x[g];
  for (int i = 0; i < m; ++i) acc += y[i] * Z[(long long)i * ldz + g];
  x[g] = acc;
}

__global__ void k_scale_inv_norm(double* y, const double* x, const double* __restrict__ nrm2,
                                 long long n, double* __restrict__ y2, int N, GatherOut go) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const double v = x[g] / sqrt(nrm2[0]);
  y[g] = v;
  if (y2) y2[g] = v;
  if (go.rs) {  // the finest level's r_S rows for the first smoothing step
    const int N3 = N * N * N;
    const long long e = g / N3;
    const int loc = (int)(g - e * N3);
    const int i = loc % N, j = (loc / N) % N, k = loc / (N * N);
    if (go.f32)
      gather_out_point<float>((float*)go.rs, go.pull + e * 7, N, go.nov, i, j, k, v);
    else
      gather_out_point<double>((double*)go.rs, go.pull + e * 7, N, go.nov, i, j, k, v);
  }
}

__global__ void k_puncture_diag(const double* __restrict__ alpha, const double* __restrict__ beta,
                                const double* __restrict__ u, double* __restrict__ d,
                                long long total, int N, double J, DevTables T) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int N3 = N * N * N;
  const int loc = (int)(g % N3);
  const int i = loc % N, j = (loc / N) % N, k = loc / (N * N);
  const double t = alpha[g] * (1.0 + u[g]) + 1.0;
  const double t2 = t * t, t4 = t2 * t2;
  d[g] = J * T.w[i] * T.w[j] * T.w[k] * 7.0 * alpha[g] * beta[g] / (t4 * t4);
}

// ---- set-up: unit columns and column gather for the patch assembly ----------
__global__ void k_unit_columns(double* __restrict__ X, long long stride, const int* __restrict__ idx,
                               int ncols) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncols) X[(long long)c * stride + idx[c]] = 1.0;
}

// A[row * n_pad + c] = AX[c * stride + idx[row]]
__global__ void k_gather_columns(const double* __restrict__ AX, long long stride,
                                 const int* __restrict__ idx, int n, double* __restrict__ A,
                                 int n_pad) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)n * n) return;
  const int row = (int)(g / n), c = (int)(g - (long long)row * n);
  A[(long long)row * n_pad + c] = AX[(long long)c * stride + idx[row]];
}

// out[k * n + row] = scale * Ainv[row * n_pad + k]  (transpose, FP64 and FP32)
__global__ void k_finish_inverse(const double* __restrict__ Ainv, int n_pad, int n, int ld,
                                 double scale, double* __restrict__ out64,
                                 float* __restrict__ out32) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)n * n) return;
  const int k = (int)(g / n), row = (int)(g - (long long)k * n);
  const double v = scale * Ainv[(long long)row * n_pad + k];
  const long long o = (long long)k * ld + row;
  if (out64) out64[o] = v;
  if (out32) out32[o] = (float)v;
}

__global__ void k_scale_copy(const double* __restrict__ A, int n_pad, int n, double scale,
                             double* __restrict__ out64, float* __restrict__ out32) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)n * n) return;
  const int row = (int)(g / n), c = (int)(g - (long long)row * n);
  const double v = scale * A[(long long)row * n_pad + c];
  if (out64) out64[g] = v;
  if (out32) out32[g] = (float)v;
}

inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_fill(double* x, double v, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(256), 0, s, x, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_pattern(void* x, bool f32, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_fill_pattern<float>, dim3(nblk(n)), dim3(256), 0, s, (float*)x, n);
  else
    hipLaunchKernelGGL(k_fill_pattern<double>, dim3(nblk(n)), dim3(256), 0, s, (double*)x, n);
  return hipGetLastError();
}
hipError_t launch_copy(double* y, const double* x, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, dim3(nblk(n)), dim3(256), 0, s, y, x, n);
  return hipGetLastError();
}
hipError_t launch_axpy(double* y, double a, const double* x, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, dim3(nblk(n)), dim3(256), 0, s, y, a, x, n);
  return hipGetLastError();
}
hipError_t launch_cg_step(double* x, double* r_next, const double* r, const double* p,
                          const double* q, double rz, const double* pq, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg_step, dim3(nblk(n)), dim3(256), 0, s, x, r_next, r, p, q, rz, pq, n);
  return hipGetLastError();
}
hipError_t launch_waxpy(double* y, const double* x, double lam, const double* dx, long long n,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_waxpy, dim3(nblk(n)), dim3(256), 0, s, y, x, lam, dx, n);
  return hipGetLastError();
}

int multidot_blocks(long long n) {
  long long b = (n + 511) / 512;  // ~512 points per block: enough blocks for 256 CUs
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return (int)b;
}

hipError_t launch_multidot(const double* V, long long ldv, int m, const double* w, long long n,
                           double* partial, double* h, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int nb = multidot_blocks(n);
  const long long chunk = (n + nb - 1) / nb;
  hipLaunchKernelGGL(k_multidot_partial, dim3(nb), dim3(kDotThreads), 0, s, V, ldv, m, w, n, chunk,
                     partial);
  hipLaunchKernelGGL(k_multidot_final, dim3(m), dim3(kDotThreads), 0, s, partial, nb, m, h);
  return hipGetLastError();
}

hipError_t launch_axpy_multidot(const double* V, long long ldv, int m, const double* coef, double* w,
                                long long n, bool norm_only, double* partial, double* h,
                                hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const int nb = multidot_blocks(n);
  const long long chunk = (n + nb - 1) / nb;
  hipLaunchKernelGGL(k_axpy_multidot_partial, dim3(nb), dim3(kDotThreads), 0, s, V, ldv, m, coef, w,
                     n, chunk, norm_only ? 1 : 0, partial);
  const int mh = norm_only ? 1 : m;
  hipLaunchKernelGGL(k_multidot_final, dim3(mh), dim3(kDotThreads), 0, s, partial, nb, mh, h);
  return hipGetLastError();
}

hipError_t launch_multi_axpy(double* w, const double* V, long long ldv, int m, const double* coef,
                             long long n, hipStream_t s) {
  if (n <= 0 || m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_multi_axpy, dim3(nblk(n)), dim3(256), 0, s, w, V, ldv, m, coef, n);
  return hipGetLastError();
}

hipError_t launch_scale_by_inv_norm(double* y, const double* x, const double* nrm2, long long n,
                                    hipStream_t s, double* y2, int N, const GatherOut& go) {
  if (n <= 0) return hipSuccess;
  if (go.rs && N < 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_scale_inv_norm, dim3(nblk(n)), dim3(256), 0, s, y, x, nrm2, n, y2, N, go);
  return hipGetLastError();
}

hipError_t launch_combine(double* x, const double* Z, long long ldz, int m, const double* y,
                          long long n, hipStream_t s) {
  if (n <= 0 || m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_combine, dim3(nblk(n)), dim3(256), 0, s, x, Z, ldz, m, y, n);
  return hipGetLastError();
}

hipError_t launch_puncture_diag(int N, const double* alpha, const double* beta, const double* u,
                                double* d, long long E, const double h[3], const DevTables& T,
                                hipStream_t s) {
  const long long total = E * N * N * N;
  if (total <= 0) return hipSuccess;
  const double J = h[0] * h[1] * h[2] * 0.125;
  hipLaunchKernelGGL(k_puncture_diag, dim3(nblk(total)), dim3(256), 0, s, alpha, beta, u, d, total,
                     N, J, T);
  return hipGetLastError();
}

hipError_t launch_unit_columns(double* X, long long copy_stride, const int* idx, int ncols,
                               hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unit_columns, dim3(nblk(ncols)), dim3(256), 0, s, X, copy_stride, idx, ncols);
  return hipGetLastError();
}

hipError_t launch_gather_columns(const double* AX, long long copy_stride, const int* idx, int n,
                                 double* A, int n_pad, hipStream_t s) {
  const long long tot = (long long)n * n;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_columns, dim3(nblk(tot)), dim3(256), 0, s, AX, copy_stride, idx, n, A,
                     n_pad);
  return hipGetLastError();
}

hipError_t launch_finish_inverse(const double* Ainv, int n_pad, int n, int ld, double scale,
                                 double* out64, float* out32, hipStream_t s) {
  const long long tot = (long long)n * n;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_finish_inverse, dim3(nblk(tot)), dim3(256), 0, s, Ainv, n_pad, n, ld, scale,
                     out64, out32);
  return hipGetLastError();
}

hipError_t launch_scale_copy(const double* A, int n_pad, int n, double scale, double* out64,
                             float* out32, hipStream_t s) {
  const long long tot = (long long)n * n;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scale_copy, dim3(nblk(tot)), dim3(256), 0, s, A, n_pad, n, scale, out64,
                     out32);
  return hipGetLastError();
}

}  // namespace dgs
