// Per-element multigrid transfer bodies (Sec. III.C.2, eq. prol) shared by the
// solo transfer kernels and the cross-request batched ones.
#pragma once

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

// Restriction of one coarse element, sum-factorised across its children: the
// x pass combines each pair of children that differ in x, the y pass each
// pair of those results that differ in y, the z pass the last pair:
//   T1[oy][oz](a, j, k) = sum_ox sum_m Px_ox(m, a) child[ox][oy][oz](m, j, k)
//   T2[oz](a, b, k)     = sum_oy sum_n Py_oy(n, b) T1[oy][oz](a, n, k)
//   coarse(a, b, c)     = sum_oz sum_o Pz_oz(o, c) T2[oz](a, b, o)
// with P = identity and a single child in a dimension that is not split.
template <int N>
__device__ __forceinline__ double pcoef(const double* sPlo, const double* sPhi, int split, int half,
                                        int m, int a) {
  return split ? (half ? sPhi[m * N + a] : sPlo[m * N + a]) : (m == a ? 1.0 : 0.0);
}

// Restriction of coarse element ec (one workgroup), on caller-provided LDS:
// T1 (4 N^3), T2 (2 N^3), sPlo / sPhi (N^2 each), sPull (7 entries).
template <int N>
__device__ __forceinline__ void restrict_element(
    double (*T1)[N * N * N], double (*T2)[N * N * N], double* sPlo, double* sPhi,
    PullEntry* sPull, const double* __restrict__ fine, double* __restrict__ coarse, int nfx,
    int nfy, int ncx, int ncy, int sx, int sy, int sz, const double* Plo, const double* Phi,
    const GatherOut& go, long long ec) {
  constexpr int N2 = N * N, N3 = N2 * N;
  const int tid = threadIdx.x;
  for (int t = tid; t < N * N; t += blockDim.x) {
    sPlo[t] = Plo[t];
    sPhi[t] = Phi[t];
  }
  if (go.rs && tid < 7) sPull[tid] = go.pull[ec * 7 + tid];
  const int cx = (int)(ec % ncx), cy = (int)((ec / ncx) % ncy), cz = (int)(ec / ((long long)ncx * ncy));
  __syncthreads();
  // x pass, straight from the fine field
  for (int t = tid; t < (sy + 1) * (sz + 1) * N3; t += blockDim.x) {
    const int slot = t / N3, p = t - slot * N3;
    const int oy = slot % (sy + 1), oz = slot / (sy + 1);
    const int a = p % N, jk = p / N;
    const int fy = sy ? 2 * cy + oy : cy, fz = sz ? 2 * cz + oz : cz;
    double acc = 0.0;
    for (int ox = 0; ox <= sx; ++ox) {
      const int fx = sx ? 2 * cx + ox : cx;
      const double* src = fine + (((long long)fz * nfy + fy) * nfx + fx) * N3 + jk * N;
#pragma unroll
      for (int m = 0; m < N; ++m) acc += pcoef<N>(sPlo, sPhi, sx, ox, m, a) * src[m];
    }
    T1[slot][p] = acc;
  }
  __syncthreads();
  // y pass
  for (int t = tid; t < (sz + 1) * N3; t += blockDim.x) {
    const int oz = t / N3, p = t - oz * N3;
    const int a = p % N, b = (p / N) % N, k = p / N2;
    double acc = 0.0;
    for (int oy = 0; oy <= sy; ++oy) {
      const double* src = T1[oz * (sy + 1) + oy] + k * N2 + a;
#pragma unroll
      for (int n = 0; n < N; ++n) acc += pcoef<N>(sPlo, sPhi, sy, oy, n, b) * src[n * N];
    }
    T2[oz][p] = acc;
  }
  __syncthreads();
  // z pass
  for (int p = tid; p < N3; p += blockDim.x) {
    const int ab = p % N2, c = p / N2;
    double acc = 0.0;
    for (int oz = 0; oz <= sz; ++oz) {
      const double* src = T2[oz] + ab;
#pragma unroll
      for (int o = 0; o < N; ++o) acc += pcoef<N>(sPlo, sPhi, sz, oz, o, c) * src[o * N2];
    }
    coarse[ec * N3 + p] = acc;
    if (go.rs) {  // the coarse level's r_S rows for its first smoothing step
      const int i = p % N, j = (p / N) % N;
      if (go.f32)
        gather_out_point<float>((float*)go.rs, sPull, N, go.nov, i, j, c, acc);
      else
        gather_out_point<double>((double*)go.rs, sPull, N, go.nov, i, j, c, acc);
    }
  }
}

// Prolongation to fine element ef (one workgroup), on caller-provided LDS:
// buf0, buf1 (N^3 each), sPlo / sPhi (N^2 each).
template <int N>
__device__ __forceinline__ void prolongate_element(
    double* buf0, double* buf1, double* sPlo, double* sPhi, const double* __restrict__ coarse,
    double* __restrict__ fine, int nfx, int nfy, int ncx, int ncy, int sx, int sy, int sz,
    const double* Plo, const double* Phi, long long ef) {
  constexpr int N3 = N * N * N;
  const int tid = threadIdx.x;
  for (int t = tid; t < N * N; t += blockDim.x) {
    sPlo[t] = Plo[t];
    sPhi[t] = Phi[t];
  }
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

}  // namespace
}  // namespace dgs
