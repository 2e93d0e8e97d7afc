// Multigrid intermesh operators on gfx950 (Sec. III.C.2, eq. prol).
//
// Prolongation interpolates a parent element to each child with the 1D
// Lagrange matrices P_lo / P_hi (child points at parent-logical (xi -+ 1)/2)
// in every dimension that is split, identity otherwise.  Restriction is the
// transpose, summed over the children of each parent (no mass matrices: it
// acts on residuals that already carry them).  Both are pulled per output
// element, so no atomics are needed and results are bitwise reproducible.
#include "dgs_internal.h"
#include "dgs_mg_elem.h"

namespace dgs {
namespace {

template <int N>
__global__ void __launch_bounds__(256)
k_restrict(const double* __restrict__ fine, double* __restrict__ coarse, int nfx, int nfy,
           int ncx, int ncy, int ncz, int sx, int sy, int sz, MgTables T, GatherOut go) {
  constexpr int N3 = N * N * N;
  __shared__ double T1[4][N3], T2[2][N3];
  __shared__ double sPlo[N * N], sPhi[N * N];
  __shared__ PullEntry sPull[7];
  (void)ncz;
  restrict_element<N>(T1, T2, sPlo, sPhi, sPull, fine, coarse, nfx, nfy, ncx, ncy, sx, sy, sz,
                      T.Plo, T.Phi, go, blockIdx.x);
}

template <int N>
__global__ void __launch_bounds__(256)
k_prolongate_add(const double* __restrict__ coarse, double* __restrict__ fine, int nfx, int nfy,
                 int ncx, int ncy, int sx, int sy, int sz, MgTables T) {
  constexpr int N3 = N * N * N;
  __shared__ double buf0[N3], buf1[N3];
  __shared__ double sPlo[N * N], sPhi[N * N];
  prolongate_element<N>(buf0, buf1, sPlo, sPhi, coarse, fine, nfx, nfy, ncx, ncy, sx, sy, sz,
                        T.Plo, T.Phi, blockIdx.x);
}

template <int N>
hipError_t restrict_n(const double* fine, double* coarse, const int nf[3], const int nc[3],
                      const int split[3], const MgTables& T, hipStream_t s, const GatherOut& go) {
  const long long Ec = (long long)nc[0] * nc[1] * nc[2];
  hipLaunchKernelGGL(k_restrict<N>, dim3((unsigned)Ec), dim3(256), 0, s, fine, coarse, nf[0], nf[1],
                     nc[0], nc[1], nc[2], split[0], split[1], split[2], T, go);
  return hipGetLastError();
}

template <int N>
hipError_t prolong_n(const double* coarse, double* fine, const int nf[3], const int nc[3],
                     const int split[3], const MgTables& T, hipStream_t s) {
  const long long Ef = (long long)nf[0] * nf[1] * nf[2];
  hipLaunchKernelGGL(k_prolongate_add<N>, dim3((unsigned)Ef), dim3(256), 0, s, coarse, fine, nf[0],
                     nf[1], nc[0], nc[1], split[0], split[1], split[2], T);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_restrict(int N, const double* fine, double* coarse, const int nf[3],
                           const int nc[3], const int split[3], const MgTables& T, hipStream_t s,
                           const GatherOut& go) {
  switch (N) {
    case 2: return restrict_n<2>(fine, coarse, nf, nc, split, T, s, go);
    case 3: return restrict_n<3>(fine, coarse, nf, nc, split, T, s, go);
    case 4: return restrict_n<4>(fine, coarse, nf, nc, split, T, s, go);
    case 5: return restrict_n<5>(fine, coarse, nf, nc, split, T, s, go);
    case 6: return restrict_n<6>(fine, coarse, nf, nc, split, T, s, go);
    case 7: return restrict_n<7>(fine, coarse, nf, nc, split, T, s, go);
    case 8: return restrict_n<8>(fine, coarse, nf, nc, split, T, s, go);
    case 9: return restrict_n<9>(fine, coarse, nf, nc, split, T, s, go);
    case 10: return restrict_n<10>(fine, coarse, nf, nc, split, T, s, go);
    case 11: return restrict_n<11>(fine, coarse, nf, nc, split, T, s, go);
    case 12: return restrict_n<12>(fine, coarse, nf, nc, split, T, s, go);
    case 13: return restrict_n<13>(fine, coarse, nf, nc, split, T, s, go);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_prolongate_add(int N, const double* coarse, double* fine, const int nf[3],
                                 const int nc[3], const int split[3], const MgTables& T,
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
    case 10: return prolong_n<10>(coarse, fine, nf, nc, split, T, s);
    case 11: return prolong_n<11>(coarse, fine, nf, nc, split, T, s);
    case 12: return prolong_n<12>(coarse, fine, nf, nc, split, T, s);
    case 13: return prolong_n<13>(coarse, fine, nf, nc, split, T, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace dgs
