// Blocked Gauss-Jordan inversion of a batch of symmetric positive definite
// matrices on gfx950 (set-up of the explicit subdomain inverses, Sec. III.E.2).
//
// In-place Gauss-Jordan without pivoting (A_S is SPD), 64 columns per step:
// with K the step's column block, P = A[K,K]^-1,
//   A[K,K] <- P,  A[K,j] <- P A[K,j],  A[i,K] <- -A[i,K] P,
//   A[i,j] <- A[i,j] - A[i,K] (P A[K,j])            (i, j outside K).
// The diagonal block is inverted in LDS by unblocked elimination; the rest of
// the step is a rank-64 update done with FP64 MFMA tiles, so the whole
// inversion costs about 2 n^3 flops on the matrix cores instead of n passes
// over the matrix.  Matrices are padded to a multiple of 64 with the identity.
#include "dgs_internal.h"

namespace dgs {
namespace {

constexpr int BS = 64;  // block size

typedef double d4 __attribute__((ext_vector_type(4)));

// P = A[K,K]^-1 for every matrix of the batch (one workgroup each).  The 64
// elimination steps are sequential, so the block uses 1024 lanes (four
// entries each) to keep every step short.
constexpr int kDiagThreads = 1024;
__global__ void __launch_bounds__(kDiagThreads) k_bgj_diag(const double* __restrict__ A, int n,
                                                           int kb, double* __restrict__ Pbuf) {
  constexpr int PER = BS * BS / kDiagThreads;
  __shared__ double M[BS][BS + 1];
  __shared__ double col[BS], row[BS];
  const int b = blockIdx.x;
  const double* Ab = A + (long long)b * n * n;
  const int k0 = kb * BS;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int t = threadIdx.x + i * kDiagThreads;
    const int r = t / BS, c = t % BS;
    M[r][c] = Ab[(long long)(k0 + r) * n + k0 + c];
  }
  __syncthreads();
  for (int k = 0; k < BS; ++k) {
    if (threadIdx.x < BS) {
      col[threadIdx.x] = M[threadIdx.x][k];
      row[threadIdx.x] = M[k][threadIdx.x];
    }
    __syncthreads();
    const double p = 1.0 / row[k];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int t = threadIdx.x + i * kDiagThreads;
      const int r = t / BS, c = t % BS;
      double v;
      if (r == k)
        v = (c == k) ? p : row[c] * p;
      else
        v = (c == k) ? -col[r] * p : M[r][c] - col[r] * row[c] * p;
      M[r][c] = v;
    }
    __syncthreads();
  }
  double* Pb = Pbuf + (long long)b * BS * BS;
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int t = threadIdx.x + i * kDiagThreads;
    Pb[t] = M[t / BS][t % BS];
  }
}

// 64x64x64 tile product on MFMA: acc += X(64x64, LDS) * Y(64x64, LDS).
// Wave w computes rows 32 (w / 2) .. +32, cols 32 (w % 2) .. +32.
// FP64 16x16x4 layout: lane supplies X[l%16][l/16], Y[l/16][l%16];
// the result holds D[l/16 + 4 r][l%16].
__device__ __forceinline__ void tile_mma(const double (*X)[BS + 1], const double (*Y)[BS + 1],
                                         d4 (&acc)[2][2], int wave, int lane) {
  const int wm = wave >> 1, wn = wave & 1;
#pragma unroll 4
  for (int k = 0; k < BS; k += 4) {
    const int kk = k + (lane >> 4);
    const double a0 = X[wm * 32 + (lane & 15)][kk];
    const double a1 = X[wm * 32 + 16 + (lane & 15)][kk];
    const double b0 = Y[kk][wn * 32 + (lane & 15)];
    const double b1 = Y[kk][wn * 32 + 16 + (lane & 15)];
    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
  }
}

__device__ __forceinline__ void load_tile(double (*T)[BS + 1], const double* __restrict__ src,
                                          long long ld) {
  for (int t = threadIdx.x; t < BS * BS; t += blockDim.x) {
    const int r = t / BS, c = t % BS;
    T[r][c] = src[(long long)r * ld + c];
  }
}

// Panels of step kb: R = P A[K, tj] (row panel, per column tile) and
// C = A[ti, K] (column panel copy), one workgroup per (matrix, tile).
__global__ void __launch_bounds__(256) k_bgj_panels(const double* __restrict__ A, int n, int kb,
                                                    const double* __restrict__ Pbuf,
                                                    double* __restrict__ Rbuf,
                                                    double* __restrict__ Cbuf) {
  __shared__ double X[BS][BS + 1], Y[BS][BS + 1];
  const int nt = n / BS;
  const int b = blockIdx.x / nt, t = blockIdx.x % nt;
  const double* Ab = A + (long long)b * n * n;
  const int k0 = kb * BS;
  // column panel copy: C[t-th 64 rows][64] = A[t rows, K]
  double* Cb = Cbuf + (long long)b * n * BS;
  for (int q = threadIdx.x; q < BS * BS; q += blockDim.x) {
    const int r = q / BS, c = q % BS;
    Cb[(long long)(t * BS + r) * BS + c] = Ab[(long long)(t * BS + r) * n + k0 + c];
  }
  // row panel: R[:, t cols] = P * A[K, t cols]
  load_tile(X, Pbuf + (long long)b * BS * BS, BS);
  load_tile(Y, Ab + (long long)k0 * n + t * BS, n);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  d4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};
  tile_mma(X, Y, acc, wave, lane);
  double* Rb = Rbuf + (long long)b * BS * n;
  const int wm = wave >> 1, wn = wave & 1;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int row = wm * 32 + i * 16 + (lane >> 4) + 4 * r;
        const int colm = t * BS + wn * 32 + j * 16 + (lane & 15);
        Rb[(long long)row * n + colm] = acc[i][j][r];
      }
}

// The update of step kb for tile (ti, tj) of every matrix.
__global__ void __launch_bounds__(256) k_bgj_update(double* __restrict__ A, int n, int kb,
                                                    const double* __restrict__ Pbuf,
                                                    const double* __restrict__ Rbuf,
                                                    const double* __restrict__ Cbuf) {
  __shared__ double X[BS][BS + 1], Y[BS][BS + 1];
  const int nt = n / BS;
  const int b = blockIdx.x / (nt * nt);
  const int rem = blockIdx.x % (nt * nt);
  const int ti = rem / nt, tj = rem % nt;
  double* Ab = A + (long long)b * n * n;
  const double* Pb = Pbuf + (long long)b * BS * BS;
  const double* Rb = Rbuf + (long long)b * BS * n;
  const double* Cb = Cbuf + (long long)b * n * BS;
  double* T = Ab + (long long)(ti * BS) * n + tj * BS;
  if (ti == kb) {  // row block: P (diagonal) or P A[K, tj]
    for (int q = threadIdx.x; q < BS * BS; q += blockDim.x) {
      const int r = q / BS, c = q % BS;
      T[(long long)r * n + c] = (tj == kb) ? Pb[r * BS + c] : Rb[(long long)r * n + tj * BS + c];
    }
    return;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave >> 1, wn = wave & 1;
  d4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0, 0, 0, 0};
  load_tile(X, Cb + (long long)(ti * BS) * BS, BS);  // A[ti, K] (saved before the step)
  if (tj == kb)
    load_tile(Y, Pb, BS);  // column block: -A[ti,K] P
  else
    load_tile(Y, Rb + tj * BS, n);  // P A[K, tj]
  __syncthreads();
  tile_mma(X, Y, acc, wave, lane);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int row = wm * 32 + i * 16 + (lane >> 4) + 4 * r;
        const int col = wn * 32 + j * 16 + (lane & 15);
        double* p = T + (long long)row * n + col;
        *p = (tj == kb) ? -acc[i][j][r] : *p - acc[i][j][r];
      }
}

}  // namespace

hipError_t launch_block_inverse(double* A, int n, int batch, double* Pbuf, double* Rbuf,
                                double* Cbuf, hipStream_t s) {
  if (n % BS != 0 || batch <= 0) return hipErrorInvalidValue;
  const int nt = n / BS;
  for (int kb = 0; kb < nt; ++kb) {
    hipLaunchKernelGGL(k_bgj_diag, dim3(batch), dim3(kDiagThreads), 0, s, A, n, kb, Pbuf);
    hipLaunchKernelGGL(k_bgj_panels, dim3(batch * nt), dim3(256), 0, s, A, n, kb, Pbuf, Rbuf, Cbuf);
    hipLaunchKernelGGL(k_bgj_update, dim3(batch * nt * nt), dim3(256), 0, s, A, n, kb, Pbuf, Rbuf,
                       Cbuf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace dgs
