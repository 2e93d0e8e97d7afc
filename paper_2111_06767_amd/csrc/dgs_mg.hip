// Multigrid intermesh operators on gfx950 (Sec. III.C.2, eq. prol).
//
// Prolongation interpolates a parent element to each child with the 1D
// Lagrange matrices P_lo / P_hi (child points at parent-logical (xi -+ 1)/2)
// in every dimension that is split, identity otherwise.  Restriction is the
// transpose, summed over the children of each parent (no mass matrices: it
// acts on residuals that already carry them).  Both are pulled per output
// element, so no atomics are needed and results are bitwise reproducible.
#include "dgs_internal.h"

namespace dgs {
namespace {

// Apply a 1D matrix to every line of an N^3 block in LDS along dimension d:
//   out[.., a, ..] = sum_m M(a, m) in[.., m, ..]   (transpose: M(m, a))
template <int N>
__device__ __forceinline__ void line_apply(const double* __restrict__ in, double* __restrict__ out,
                                           const double* __restrict__ Mx, bool transpose, int d,
                                           int tid, int nthreads) {
  constexpr int N2 = N * N, N3 = N2 * N;
  for (int p = tid; p < N3; p += nthreads) {
    const int idx[3] = {p % N, (p / N) % N, p / N2};
    const int a = idx[d];
    const int stride = d == 0 ? 1 : (d == 1 ? N : N2);
    const int base = p - a * stride;
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < N; ++m)
      acc += (transpose ? Mx[m * N + a] : Mx[a * N + m]) * in[base + m * stride];
    out[p] = acc;
  }
}

template <int N>
__global__ void __launch_bounds__(256)
k_restrict(const double* __restrict__ fine, double* __restrict__ coarse, int nfx, int nfy,
           int ncx, int ncy, int ncz, int sx, int sy, int sz, DevTables T) {
  constexpr int N3 = N * N * N;
  __shared__ double buf0[N3], buf1[N3];
  __shared__ double sPlo[N * N], sPhi[N * N];
  const int tid = threadIdx.x;
  for (int t = tid; t < N * N; t += blockDim.x) {
    sPlo[t] = T.Plo[t];
    sPhi[t] = T.Phi[t];
  }
  const long long ec = blockIdx.x;
  const int cx = (int)(ec % ncx), cy = (int)((ec / ncx) % ncy), cz = (int)(ec / ((long long)ncx * ncy));
  double acc[(N3 + 255) / 256];
#pragma unroll
  for (int q = 0; q < (N3 + 255) / 256; ++q) acc[q] = 0.0;
  const int split[3] = {sx, sy, sz};
  for (int oz = 0; oz <= sz; ++oz)
    for (int oy = 0; oy <= sy; ++oy)
      for (int ox = 0; ox <= sx; ++ox) {
        const int fx = sx ? 2 * cx + ox : cx, fy = sy ? 2 * cy + oy : cy, fz = sz ? 2 * cz + oz : cz;
        const long long ef = ((long long)fz * nfy + fy) * nfx + fx;
        __syncthreads();
        for (int p = tid; p < N3; p += blockDim.x) buf0[p] = fine[ef * N3 + p];
        __syncthreads();
        double* cur = buf0;
        double* nxt = buf1;
        const int half[3] = {ox, oy, oz};
        for (int d = 0; d < 3; ++d) {
          if (!split[d]) continue;
          line_apply<N>(cur, nxt, half[d] ? sPhi : sPlo, true, d, tid, blockDim.x);
          __syncthreads();
          double* t = cur;
          cur = nxt;
          nxt = t;
        }
#pragma unroll
        for (int q = 0; q < (N3 + 255) / 256; ++q) {
          const int p = tid + 256 * q;
          if (p < N3) acc[q] += cur[p];
        }
      }
#pragma unroll
  for (int q = 0; q < (N3 + 255) / 256; ++q) {
    const int p = tid + 256 * q;
    if (p < N3) coarse[ec * N3 + p] = acc[q];
  }
}

template <int N>
__global__ void __launch_bounds__(256)
k_prolongate_add(const double* __restrict__ coarse, double* __restrict__ fine, int nfx, int nfy,
                 int ncx, int ncy, int sx, int sy, int sz, DevTables T) {
  constexpr int N3 = N * N * N;
  __shared__ double buf0[N3], buf1[N3];
  __shared__ double sPlo[N * N], sPhi[N * N];
  const int tid = threadIdx.x;
  for (int t = tid; t < N * N; t += blockDim.x) {
    sPlo[t] = T.Plo[t];
    sPhi[t] = T.Phi[t];
  }
  const long long ef = blockIdx.x;
  const int fx = (int)(ef % nfx), fy = (int)((ef / nfx) % nfy), fz = (int)(ef / ((long long)nfx * nfy));
  const int cx = sx ? fx / 2 : fx, cy = sy ? fy / 2 : fy, cz = sz ? fz / 2 : fz;
  const long long ec = ((long long)cz * ncy + cy) * ncx + cx;
  for (int p = tid; p < N3; p += blockDim.x) buf0[p] = coarse[ec * N3 + p];
  __syncthreads();
  const int split[3] = {sx, sy, sz};
  const int half[3] = {fx & 1, fy & 1, fz & 1};
  double* cur = buf0;
  double* nxt = buf1;
  for (int d = 0; d < 3; ++d) {
    if (!split[d]) continue;
    line_apply<N>(cur, nxt, half[d] ? sPhi : sPlo, false, d, tid, blockDim.x);
    __syncthreads();
    double* t = cur;
    cur = nxt;
    nxt = t;
  }
  for (int p = tid; p < N3; p += blockDim.x) fine[ef * N3 + p] += cur[p];
}

template <int N>
hipError_t restrict_n(const double* fine, double* coarse, const int nf[3], const int nc[3],
                      const int split[3], const DevTables& T, hipStream_t s) {
  const long long Ec = (long long)nc[0] * nc[1] * nc[2];
  hipLaunchKernelGGL(k_restrict<N>, dim3((unsigned)Ec), dim3(256), 0, s, fine, coarse, nf[0], nf[1],
                     nc[0], nc[1], nc[2], split[0], split[1], split[2], T);
  return hipGetLastError();
}

template <int N>
hipError_t prolong_n(const double* coarse, double* fine, const int nf[3], const int nc[3],
                     const int split[3], const DevTables& T, hipStream_t s) {
  const long long Ef = (long long)nf[0] * nf[1] * nf[2];
  hipLaunchKernelGGL(k_prolongate_add<N>, dim3((unsigned)Ef), dim3(256), 0, s, coarse, fine, nf[0],
                     nf[1], nc[0], nc[1], split[0], split[1], split[2], T);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_restrict(int N, const double* fine, double* coarse, const int nf[3],
                           const int nc[3], const int split[3], const DevTables& T, hipStream_t s) {
  switch (N) {
    case 2: return restrict_n<2>(fine, coarse, nf, nc, split, T, s);
    case 3: return restrict_n<3>(fine, coarse, nf, nc, split, T, s);
    case 4: return restrict_n<4>(fine, coarse, nf, nc, split, T, s);
    case 5: return restrict_n<5>(fine, coarse, nf, nc, split, T, s);
    case 6: return restrict_n<6>(fine, coarse, nf, nc, split, T, s);
    case 7: return restrict_n<7>(fine, coarse, nf, nc, split, T, s);
    case 8: return restrict_n<8>(fine, coarse, nf, nc, split, T, s);
    case 9: return restrict_n<9>(fine, coarse, nf, nc, split, T, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_prolongate_add(int N, const double* coarse, double* fine, const int nf[3],
                                 const int nc[3], const int split[3], const DevTables& T,
                                 hipStream_t s) {
  switch (N) {
    case 2: return prolong_n<2>(coarse, fine, nf, nc, split, T, s);
    case 3: return prolong_n<3>(coarse, fine, nf, nc, split, T, s);
    case 4: return prolong_n<4>(coarse, fine, nf, nc, split, T, s);
    case 5: return prolong_n<5>(coarse, fine, nf, nc, split, T, s);
    case 6: return prolong_n<6>(coarse, fine, nf, nc, split, T, s);
    case 7: return prolong_n<7>(coarse, fine, nf, nc, split, T, s);
    case 8: return prolong_n<8>(coarse, fine, nf, nc, split, T, s);
    case 9: return prolong_n<9>(coarse, fine, nf, nc, split, T, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgs
