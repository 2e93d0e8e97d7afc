// Per-element helpers of the DG operator kernels (the solo operator kernel
// and the cross-request batched one): the even-odd derivative product, a face
// neighbour's trace and normal derivative from its line, and the gather-out
// of a z-line of the residual into the subdomain rows.
#pragma once

#include "dgs_internal.h"

namespace dgs {
namespace {

// y = M x for a centro-antisymmetric M through its even-odd split (half the
// multiply-adds of the plain product; the constants are wave-uniform).
template <int N>
__device__ __forceinline__ void eo_apply(const double (&x)[N], double (&y)[N], const EvenOdd& E) {
  constexpr int H = N / 2;
  double ev[H], od[H];
#pragma unroll
  for (int m = 0; m < H; ++m) {
    ev[m] = x[m] + x[N - 1 - m];
    od[m] = x[m] - x[N - 1 - m];
  }
#pragma unroll
  for (int i = 0; i < H; ++i) {
    double a = 0.0, c = 0.0;
#pragma unroll
    for (int m = 0; m < H; ++m) {
      a += E.P[i * H + m] * ev[m];
      c += E.Q[i * H + m] * od[m];
    }
    if constexpr (N % 2 == 1) a += E.cf[i] * x[H];
    y[i] = a + c;
    y[N - 1 - i] = c - a;
  }
  if constexpr (N % 2 == 1) {
    double c = 0.0;
#pragma unroll
    for (int m = 0; m < H; ++m) c += E.rc[m] * od[m];
    y[H] = c;
  }
}

// Neighbour's trace (ue) and normal derivative (ge, along +d) on the shared
// face from its line x[0..N-1] along d; fi is the neighbour's layer on the face.
template <int N>
__device__ __forceinline__ void face_from_line(const double (&x)[N], int side, double rh,
                                               const DevTables& T, double& ue, double& ge) {
  double acc = 0.0;
  if (side) {  // neighbour on the high side: its low face (layer 0)
#pragma unroll
    for (int m = 0; m < N; ++m) acc += T.D0[m] * x[m];
    ue = x[0];
  } else {  // neighbour on the low side: its high face (layer N-1)
#pragma unroll
    for (int m = 0; m < N; ++m) acc += T.DN[m] * x[m];
    ue = x[N - 1];
  }
  ge = acc * rh;
}

// Gather-out of one z-line of the residual (lane (a, b), points k = 0..N-1)
// into the subdomain rows: the element's own row (in its class frame) and the
// overlap strips of its face neighbours' subdomains, at the offsets of the
// scatter's pull table.  A strip entry is layer * N^2 + t1 * N + t0 (layer
// counted from the shared face into this element, t0 / t1 the transverse
// indices in the neighbour's class frame).
template <typename TS, int N>
__device__ __forceinline__ void store_subdomain_rows(const double (&rz)[N], TS* __restrict__ rs,
                                                     const PullEntry* pe, int a, int b, int nov) {
  constexpr int N2 = N * N;
  const PullEntry own = pe[0];
  {
    int s0, s1, s2;
    frame_strides(own.flip, N, s0, s1, s2);
    const int mi = (own.flip & 1) ? N - 1 - a : a;
    const int mj = (own.flip & 2) ? N - 1 - b : b;
    const bool fk = own.flip & 4;
    TS* p = rs + own.du + mi * s0 + mj * s1;
#pragma unroll
    for (int k = 0; k < N; ++k) p[(fk ? N - 1 - k : k) * s2] = (TS)rz[k];
  }
  // x and y faces: the lane's layer is fixed; of the two transverse
  // coordinates one is the lane's other index and one is k
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const PullEntry q = pe[1 + f];
    const int id = f < 2 ? a : b;
    const int layer = (f & 1) ? N - 1 - id : id;
    if (q.du >= 0 && layer < nov) {
      const bool sw = q.flip & 4;
      int tf = f < 2 ? b : a;
      if (sw ? (q.flip & 2) : (q.flip & 1)) tf = N - 1 - tf;
      const bool fkk = sw ? (q.flip & 1) : (q.flip & 2);
      const int sk = sw ? 1 : N;
      TS* p = rs + q.du + layer * N2 + tf * (sw ? N : 1);
#pragma unroll
      for (int k = 0; k < N; ++k) p[(fkk ? N - 1 - k : k) * sk] = (TS)rz[k];
    }
  }
  // z faces: the layer is the point's own k (uniform across the element)
#pragma unroll
  for (int f = 4; f < 6; ++f) {
    const PullEntry q = pe[1 + f];
    if (q.du < 0) continue;
    int t0 = a, t1 = b;
    strip_coords(t0, t1, q.flip, N);
    TS* p = rs + q.du + t1 * N + t0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const int layer = f == 4 ? k : N - 1 - k;
      if (layer < nov) p[layer * N2] = (TS)rz[k];
    }
  }
}

}  // namespace
}  // namespace dgs
