// Additive Schwarz smoother kernels on gfx950 (Sec. III.D, III.E).
//
// A Schwarz step on one level is
//   r = b - A u                                   (fused apply kernel)
//   r_S = R_S r for every subdomain S              (gather, this file)
//   du_S = s * A_S^-1 r_S, one GEMM per class       (MFMA, this file)
//   u += sum_S R_S^T (w_S du_S)                    (pull scatter, this file)
// Subdomains are grouped by boundary class: all subdomains of a class share
// one explicit inverse, so the subdomain solves become dense GEMMs
// [count x n] * [n x n] on the matrix cores.  FP64 uses v_mfma_f64_16x16x4f64,
// the mixed-precision path v_mfma_f32_16x16x4f32 with FP32 accumulation.
#include "dgs_internal.h"

namespace dgs {
namespace {

// r_S = R_S r for the subdomain of element e (one workgroup per subdomain);
// row elem_row[e] of the class block receives the n_S gathered values.
template <typename T>
__global__ void __launch_bounds__(256)
k_gather_rows(const double* __restrict__ r, T* __restrict__ rs, const int* __restrict__ elem_class,
              const long long* __restrict__ elem_row, const int* __restrict__ nbr,
              const ClassInfo* __restrict__ cls, const int* __restrict__ seg_loc, int E, int N3) {
  const int e = blockIdx.x;
  if (e >= E) return;
  const ClassInfo ci = cls[elem_class[e]];
  __shared__ long long src[7];
  if (threadIdx.x < 7) {
    const int el = threadIdx.x == 0 ? e : nbr[(long long)e * 6 + threadIdx.x - 1];
    src[threadIdx.x] = (long long)el * N3;  // negative (absent) is never referenced
  }
  __syncthreads();
  T* out = rs + elem_row[e];
  const int* lay = seg_loc + ci.layout_off;
  for (int k = threadIdx.x; k < ci.n; k += blockDim.x) {
    const int sl = lay[k];
    const int seg = sl / N3;
    const int loc = sl - seg * N3;
    out[k] = (T)r[src[seg] + loc];
  }
}

// Pull-based weighted scatter: every point adds its own subdomain's
// correction and the overlap corrections of the face neighbours' subdomains.
template <typename T>
__global__ void __launch_bounds__(256)
k_scatter(double* __restrict__ u, const T* __restrict__ du, const double* __restrict__ weights,
          const int* __restrict__ elem_class, const long long* __restrict__ elem_row,
          const int* __restrict__ nbr, const ClassInfo* __restrict__ cls, int N, int nov,
          long long total) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int N2 = N * N, N3 = N2 * N;
  const long long e = g / N3;
  const int loc = (int)(g - e * N3);
  const int idx[3] = {loc % N, (loc / N) % N, loc / N2};
  const ClassInfo ce = cls[elem_class[e]];
  double acc = weights[ce.layout_off + loc] * (double)du[elem_row[e] + loc];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int b = nbr[e * 6 + f];
    if (b < 0) continue;
    const int d = f >> 1;
    const int m = idx[d];
    const int layer = (f & 1) ? (N - 1 - m) : m;
    if (layer >= nov) continue;
    const int t0 = d == 0 ? idx[1] : idx[0];
    const int t1 = d == 2 ? idx[1] : idx[2];
    const ClassInfo cb = cls[elem_class[b]];
    const int so = cb.strip_off[f ^ 1];
    const int k = so + layer * N2 + t1 * N + t0;
    acc += weights[cb.layout_off + k] * (double)du[elem_row[b] + k];
  }
  u[g] += acc;
}

// ---------------------------------------------------------------------------
// Grouped subdomain GEMM:  DU_c[count x n] = scale * RS_c[count x n] * B_c[n x n]
// with B_c = (A_S^-1)^T, one 64 x 64 output tile per workgroup, 4 waves of
// 32 x 32, MFMA 16x16x4.
// ---------------------------------------------------------------------------
template <typename T>
struct Mfma;

// Operand layout of both 16x16x4 instructions: lane l supplies A[l % 16][l / 16]
// and B[l / 16][l % 16].  The accumulator layouts differ (measured on gfx950):
// FP64 holds D[l / 16 + 4 r][l % 16], FP32 holds D[4 (l / 16) + r][l % 16].
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 run(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename T>
__global__ void __launch_bounds__(256)
k_sub_gemm(const T* __restrict__ rs, const T* __restrict__ inv, T* __restrict__ du,
           const ClassInfo* __restrict__ cls, const GemmTile* __restrict__ tiles, double scale) {
  constexpr int BM = 64, BN = 64, BK = 16;
  typedef typename Mfma<T>::v4 v4;
  __shared__ T As[BK][BM + 4];
  __shared__ T Bs[BK][BN + 4];
  const GemmTile tl = tiles[blockIdx.x];
  const ClassInfo ci = cls[tl.cls];
  const int n = ci.n, M = ci.count;
  const T* A = rs + ci.rs_off;
  const T* B = inv + ci.inv_off;
  T* C = du + ci.rs_off;
  const int m0 = tl.m0, n0 = tl.n0;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  v4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4{0, 0, 0, 0};

  const int ar = tid >> 2, ac = (tid & 3) * 4;    // A tile loader: row, k
  const int bk = tid >> 4, bc = (tid & 15) * 4;   // B tile loader: k, col
  for (int k0 = 0; k0 < n; k0 += BK) {
    {
      const int row = m0 + ar;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = k0 + ac + q;
        As[ac + q][ar] = (row < M && col < n) ? A[(long long)row * n + col] : (T)0;
      }
      const int krow = k0 + bk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int col = n0 + bc + q;
        Bs[bk][bc + q] = (krow < n && col < n) ? B[(long long)krow * n + col] : (T)0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T a0 = As[kr][wm * 32 + (lane & 15)];
      T a1 = As[kr][wm * 32 + 16 + (lane & 15)];
      T b0 = Bs[kr][wn * 32 + (lane & 15)];
      T b1 = Bs[kr][wn * 32 + 16 + (lane & 15)];
      acc[0][0] = Mfma<T>::run(a0, b0, acc[0][0]);
      acc[0][1] = Mfma<T>::run(a0, b1, acc[0][1]);
      acc[1][0] = Mfma<T>::run(a1, b0, acc[1][0]);
      acc[1][1] = Mfma<T>::run(a1, b1, acc[1][1]);
    }
    __syncthreads();
  }
  const T sc = (T)scale;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + a * 16 + Mfma<T>::row(lane, r);
        const int col = n0 + wn * 32 + b * 16 + (lane & 15);
        if (row < M && col < n) C[(long long)row * n + col] = sc * acc[a][b][r];
      }
}

}  // namespace

hipError_t launch_gather(int N, bool f32, const double* r, void* rs, const int* elem_class,
                         const long long* elem_row, const int* nbr, const ClassInfo* cls,
                         const int* seg_loc, int E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  const int N3 = N * N * N;
  if (f32)
    hipLaunchKernelGGL(k_gather_rows<float>, dim3(E), dim3(256), 0, s, r, (float*)rs, elem_class,
                       elem_row, nbr, cls, seg_loc, E, N3);
  else
    hipLaunchKernelGGL(k_gather_rows<double>, dim3(E), dim3(256), 0, s, r, (double*)rs, elem_class,
                       elem_row, nbr, cls, seg_loc, E, N3);
  return hipGetLastError();
}

hipError_t launch_subdomain_gemm(bool f32, const void* rs, const void* inv, void* du,
                                 const ClassInfo* cls, const GemmTile* tiles, int ntiles,
                                 double scale, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_sub_gemm<float>, dim3(ntiles), dim3(256), 0, s, (const float*)rs,
                       (const float*)inv, (float*)du, cls, tiles, scale);
  else
    hipLaunchKernelGGL(k_sub_gemm<double>, dim3(ntiles), dim3(256), 0, s, (const double*)rs,
                       (const double*)inv, (double*)du, cls, tiles, scale);
  return hipGetLastError();
}

hipError_t launch_scatter(int N, bool f32, double* u, const void* du, const double* weights,
                               const int* elem_class, const long long* elem_row, const int* nbr,
                               const ClassInfo* cls, int nov, long long E, hipStream_t s) {
  const long long total = E * N * N * N;
  if (total <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (f32)
    hipLaunchKernelGGL(k_scatter<float>, dim3(blocks), dim3(256), 0, s, u, (const float*)du,
                       weights, elem_class, elem_row, nbr, cls, N, nov, total);
  else
    hipLaunchKernelGGL(k_scatter<double>, dim3(blocks), dim3(256), 0, s, u, (const double*)du,
                       weights, elem_class, elem_row, nbr, cls, N, nov, total);
  return hipGetLastError();
}

}  // namespace dgs
