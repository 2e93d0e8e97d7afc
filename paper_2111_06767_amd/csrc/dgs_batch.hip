// Cross-request batched kernels of the serving loop (Sec. III.D.5: once the
// residuals are exchanged every subdomain solve is independent, and so is
// every element of every request).
//
// A launch covers work items of several problems, possibly of different
// polynomial degrees: each problem's share is a job, the jobs of a launch are
// listed by their first workgroup (blk0, ascending), and a workgroup finds its
// job by scanning the list (a few dozen entries at most, read as uniform
// loads).  Degrees are dispatched inside the kernel, so one launch serves the
// elements of every active request: the operator kernel runs one element per
// workgroup with the per-element arithmetic of the solo operator kernel, the
// transfer kernels one coarse (restriction) or fine (prolongation) element per
// workgroup with the solo transfer bodies, and the vector kernels keep the
// solo kernels' fixed chunks and summation orders, so a request's reductions
// are the same numbers alone or in a batch.
#include "dgs_internal.h"
#include "dgs_dot.h"
#include "dgs_elem.h"
#include "dgs_mg_elem.h"

namespace dgs {
namespace {

template <typename J>
__device__ __forceinline__ int job_of(const J* __restrict__ jobs, int njobs, int blk) {
  int j = 0;
  while (j + 1 < njobs && jobs[j + 1].blk0 <= blk) ++j;
  return j;
}

// ---------------------------------------------------------------------------
// Operator: one element per workgroup (box grids), any N <= 9
// ---------------------------------------------------------------------------
constexpr int kBatchMaxN = 9;
constexpr int kBatchS3 = kBatchMaxN * kBatchMaxN * (kBatchMaxN + 1);
// LDS of one element: sU, sA (padded element copies), sw, the pull entries
constexpr int kBatchApplyLds = 2 * kBatchS3 + 16 + 7 * 2;

// The element e of job jb: the solo operator kernel's arithmetic for one
// element per workgroup (its face-neighbour loads, the forward phase with the
// numerical flux at the line ends, the transposed products and the sum).
// MODE: kApply (with the optional copy of u) or kResidual; GO: 0 writes out,
// 1 / 2 writes r_S into FP32 / FP64 subdomain rows.
template <int N, int MODE, int GO>
__device__ __forceinline__ void batch_apply_element(double* lds, const BApplyJob& jb, long long e,
                                                    const DevTables& T) {
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int PIT = N + 1;
  constexpr int S3 = N * N * PIT;
  double* sU = lds;
  double* sA = lds + S3;
  double* sw = lds + 2 * S3;
  PullEntry* sPull = reinterpret_cast<PullEntry*>(lds + 2 * S3 + 16);
  const OpParams& P = jb.P;
  const double* __restrict__ u = jb.u;
  const int tid = threadIdx.x;
  if (tid < N) sw[tid] = T.w[tid];
  const bool active = tid < N2;
  const int t = tid;
  const int a = t % N, b = t / N;
  const double J = P.J;
  auto L = [](int k, int j, int i) { return (k * N + j) * PIT + i; };
  if constexpr (GO != 0) {
    if (tid < 7) sPull[tid] = jb.go.pull[e * 7 + tid];
  }
  double uz[N], xf[4], yf[4], zf[4];
  int nb[6];
  if (active) {
    const double* ue = u + e * N3;
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int ie = (int)e, ex = ie % nx, ey = (ie / nx) % ny, ez = ie / (nx * ny);
    nb[0] = ex > 0 ? ie - 1 : -1;
    nb[1] = ex < nx - 1 ? ie + 1 : -1;
    nb[2] = ey > 0 ? ie - nx : -1;
    nb[3] = ey < ny - 1 ? ie + nx : -1;
    nb[4] = ez > 0 ? ie - nx * ny : -1;
    nb[5] = ez < nz - 1 ? ie + nx * ny : -1;
#pragma unroll
    for (int k = 0; k < N; ++k) {
      uz[k] = ue[k * N2 + t];
      sU[L(k, b, a)] = uz[k];
    }
    // a missing neighbour reads the element itself; its result is replaced by
    // the boundary's ghost state
    auto nbi = [&](int f) -> long long { return nb[f] >= 0 ? (long long)nb[f] : e; };
    const long long xl0 = nbi(0), xh0 = nbi(1), yl = nbi(2), yh = nbi(3), zl = nbi(4), zh = nbi(5);
    double xlo[N], xhi[N], ylo[N], yhi[N], zlo[N], zhi[N];
#pragma unroll
    for (int m = 0; m < N; ++m) {
      xlo[m] = u[xl0 * N3 + b * N2 + a * N + m];
      xhi[m] = u[xh0 * N3 + b * N2 + a * N + m];
    }
#pragma unroll
    for (int m = 0; m < N; ++m) {
      ylo[m] = u[yl * N3 + b * N2 + m * N + a];
      yhi[m] = u[yh * N3 + b * N2 + m * N + a];
      zlo[m] = u[zl * N3 + m * N2 + t];
      zhi[m] = u[zh * N3 + m * N2 + t];
    }
    face_from_line<N>(xlo, 0, P.rh[0], T, xf[0], xf[1]);
    face_from_line<N>(xhi, 1, P.rh[0], T, xf[2], xf[3]);
    face_from_line<N>(ylo, 0, P.rh[1], T, yf[0], yf[1]);
    face_from_line<N>(yhi, 1, P.rh[1], T, yf[2], yf[3]);
    face_from_line<N>(zlo, 0, P.rh[2], T, zf[0], zf[1]);
    face_from_line<N>(zhi, 1, P.rh[2], T, zf[2], zf[3]);
  }
  __syncthreads();

  double qy[N], cz[N];
  double fy[2], fz[2];
  if (active) {
    const double wa = sw[a], wb = sw[b];
    const double jwab = J * wa * wb;
    // ---- x role: line (j, k) = (a, b) ----
    {
      double line[N], g[N];
#pragma unroll
      for (int m = 0; m < N; ++m) line[m] = sU[L(b, a, m)];
      eo_apply<N>(line, g, T.fwd);
#pragma unroll
      for (int m = 0; m < N; ++m) g[m] *= P.rh[0];
      double fx[2];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int ie = side ? N - 1 : 0;
        const double sg = side ? 1.0 : -1.0;
        const bool has = nb[side] >= 0;
        const double ui = line[ie], gi = g[ie];
        double ue = has ? xf[2 * side] : -ui;
        double ge = has ? xf[2 * side + 1] : gi;
        if (P.neumann && !has && ((P.neumann >> (side)) & 1)) {  // Neumann ghost
          ue = ui;
          ge = -gi;
        }
        fx[side] = jwab * P.rh[0] * (0.5 * sg * (gi + ge) - P.sig[0] * (ui - ue));
        g[ie] += P.lf[0] * sg * (ue - ui);
      }
#pragma unroll
      for (int m = 0; m < N; ++m) line[m] = jwab * T.w[m] * g[m];
      eo_apply<N>(line, g, T.bwd);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        double v = g[i] * P.rh[0];
        if (i == 0) v -= fx[0];
        if (i == N - 1) v -= fx[1];
        sA[L(b, a, i)] = v;
      }
    }
    // ---- y role: line (i, k) = (a, b) ----
    {
      double line[N], g[N];
#pragma unroll
      for (int m = 0; m < N; ++m) line[m] = sU[L(b, m, a)];
      eo_apply<N>(line, g, T.fwd);
#pragma unroll
      for (int m = 0; m < N; ++m) g[m] *= P.rh[1];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int je = side ? N - 1 : 0;
        const double sg = side ? 1.0 : -1.0;
        const bool has = nb[2 + side] >= 0;
        const double ui = line[je], gi = g[je];
        double ue = has ? yf[2 * side] : -ui;
        double ge = has ? yf[2 * side + 1] : gi;
        if (P.neumann && !has && ((P.neumann >> (2 + side)) & 1)) {  // Neumann ghost
          ue = ui;
          ge = -gi;
        }
        fy[side] = jwab * P.rh[1] * (0.5 * sg * (gi + ge) - P.sig[1] * (ui - ue));
        g[je] += P.lf[1] * sg * (ue - ui);
      }
#pragma unroll
      for (int m = 0; m < N; ++m) qy[m] = jwab * T.w[m] * g[m];
    }
    // ---- z role: line (i, j) = (a, b), in registers ----
    {
      double g[N];
      eo_apply<N>(uz, g, T.fwd);
#pragma unroll
      for (int m = 0; m < N; ++m) g[m] *= P.rh[2];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int ke = side ? N - 1 : 0;
        const double sg = side ? 1.0 : -1.0;
        const double ui = uz[ke], gi = g[ke];
        const bool has = nb[4 + side] >= 0;
        double ue = has ? zf[2 * side] : -ui;
        double ge = has ? zf[2 * side + 1] : gi;
        if (P.neumann && !has && ((P.neumann >> (4 + side)) & 1)) {  // Neumann ghost
          ue = ui;
          ge = -gi;
        }
        fz[side] = jwab * P.rh[2] * (0.5 * sg * (gi + ge) - P.sig[2] * (ui - ue));
        g[ke] += P.lf[2] * sg * (ue - ui);
      }
#pragma unroll
      for (int m = 0; m < N; ++m) g[m] = jwab * T.w[m] * g[m];
      eo_apply<N>(g, cz, T.bwd);
    }
  }
  __syncthreads();  // every forward read of sU is done: the y part is written below
  if (active) {
    double c[N];
    eo_apply<N>(qy, c, T.bwd);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      double v = c[j] * P.rh[1];
      if (j == 0) v -= fy[0];
      if (j == N - 1) v -= fy[1];
      sU[L(b, j, a)] = v;
    }
  }
  constexpr bool need_b = MODE == kResidual;
  double bz[need_b ? N : 1];
  if (active) {
    if constexpr (need_b) {
#pragma unroll
      for (int k = 0; k < N; ++k) bz[k] = jb.b[e * N3 + k * N2 + t];
    }
  }
  __syncthreads();
  if (active) {
    double rz[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double r = cz[k] * P.rh[2] + sA[L(k, b, a)] + sU[L(k, b, a)];
      if (k == 0) r -= fz[0];
      if (k == N - 1) r -= fz[1];
      if constexpr (MODE == kResidual) r = bz[k] - r;
      rz[k] = r;
    }
    if (jb.ucopy) {
#pragma unroll
      for (int k = 0; k < N; ++k) jb.ucopy[e * N3 + k * N2 + t] = uz[k];
    }
    if constexpr (GO == 0) {
#pragma unroll
      for (int k = 0; k < N; ++k) jb.out[e * N3 + k * N2 + t] = rz[k];
    } else if constexpr (GO == 1) {
      store_subdomain_rows<float, N>(rz, (float*)jb.go.rs, sPull, a, b, jb.go.nov);
    } else {
      store_subdomain_rows<double, N>(rz, (double*)jb.go.rs, sPull, a, b, jb.go.nov);
    }
  }
}

template <int N, int MODE, bool ROWS>
__device__ __forceinline__ void batch_apply_dispatch_go(double* lds, const BApplyJob& jb,
                                                        long long e, const DevTables& T) {
  if constexpr (ROWS) {
    if (jb.go.f32)
      batch_apply_element<N, MODE, 1>(lds, jb, e, T);
    else
      batch_apply_element<N, MODE, 2>(lds, jb, e, T);
  } else {
    batch_apply_element<N, MODE, 0>(lds, jb, e, T);
  }
}

// ROWS: residual written into the subdomain rows (each job's go), else into out
template <int MODE, bool ROWS>
__global__ void __launch_bounds__(128)
k_batch_apply(const BApplyJob* __restrict__ jobs, int njobs, const DevTables* __restrict__ tabs) {
  __shared__ double lds[kBatchApplyLds];
  const int j = job_of(jobs, njobs, (int)blockIdx.x);
  const BApplyJob& jb = jobs[j];
  const long long e = (long long)blockIdx.x - jb.blk0;
  const DevTables& T = tabs[jb.N];
  switch (jb.N) {
    case 2: batch_apply_dispatch_go<2, MODE, ROWS>(lds, jb, e, T); break;
    case 3: batch_apply_dispatch_go<3, MODE, ROWS>(lds, jb, e, T); break;
    case 4: batch_apply_dispatch_go<4, MODE, ROWS>(lds, jb, e, T); break;
    case 5: batch_apply_dispatch_go<5, MODE, ROWS>(lds, jb, e, T); break;
    case 6: batch_apply_dispatch_go<6, MODE, ROWS>(lds, jb, e, T); break;
    case 7: batch_apply_dispatch_go<7, MODE, ROWS>(lds, jb, e, T); break;
    case 8: batch_apply_dispatch_go<8, MODE, ROWS>(lds, jb, e, T); break;
    case 9: batch_apply_dispatch_go<9, MODE, ROWS>(lds, jb, e, T); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Weighted pull-scatter (the solo scatter's arithmetic, FP32 or FP64 partial
// products per job, the split-K parts summed in the same order)
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ double batch_sum_parts(const T* __restrict__ du, long long idx,
                                                  long long stride, int parts) {
  double v = 0.0;
  for (int q = 0; q < parts; ++q) v += (double)du[q * stride + idx];
  return v;
}

template <typename T>
__device__ __forceinline__ void batch_scatter_point(const BScatterJob& jb, long long g) {
  const T* __restrict__ du = (const T*)jb.du;
  const int N = jb.N, N2 = N * N, N3 = N2 * N;
  const long long e = g / N3;
  const int loc = (int)(g - e * N3);
  const int idx[3] = {loc % N, (loc / N) % N, loc / N2};
  const PullEntry* pe = jb.pull + e * 7;
  const PullEntry own = pe[0];
  const int lc = to_class_frame(idx[0], idx[1], idx[2], own.flip, N);
  double acc = jb.weights[own.w + lc] * batch_sum_parts<T>(du, own.du + lc, jb.pstride, jb.parts);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const PullEntry q = pe[1 + f];
    const int d = f >> 1;
    const int layer = (f & 1) ? (N - 1 - idx[d]) : idx[d];
    int t0 = idx[d == 0 ? 1 : 0], t1 = idx[d == 2 ? 1 : 2];
    strip_coords(t0, t1, q.flip, N);
    const bool ok = q.du >= 0 && layer < jb.nov;
    const int k = ok ? layer * N2 + t1 * N + t0 : lc;
    const long long bd = ok ? q.du : own.du;
    const int bw = ok ? q.w : own.w;
    const double v = jb.weights[bw + k] * batch_sum_parts<T>(du, bd + k, jb.pstride, jb.parts);
    acc += ok ? v : 0.0;
  }
  if (jb.assign)
    jb.u[g] = acc;
  else
    jb.u[g] += acc;
}

__global__ void __launch_bounds__(256)
k_batch_scatter(const BScatterJob* __restrict__ jobs, int njobs) {
  const int j = job_of(jobs, njobs, (int)blockIdx.x);
  const BScatterJob& jb = jobs[j];
  const long long g = ((long long)blockIdx.x - jb.blk0) * 256 + threadIdx.x;
  if (g >= jb.total) return;
  if (jb.f32)
    batch_scatter_point<float>(jb, g);
  else
    batch_scatter_point<double>(jb, g);
}

// ---------------------------------------------------------------------------
// Multigrid transfer: one coarse (restriction) or fine (prolongation)
// element per workgroup, any N <= 9
// ---------------------------------------------------------------------------
constexpr int kBatchN3 = kBatchMaxN * kBatchMaxN * kBatchMaxN;

template <int N>
__device__ __forceinline__ void batch_restrict_element(double* lds, const BTransferJob& jb,
                                                       long long ec, const MgTables& T) {
  constexpr int N3 = N * N * N;
  double(*T1)[N3] = reinterpret_cast<double(*)[N3]>(lds);
  double(*T2)[N3] = reinterpret_cast<double(*)[N3]>(lds + 4 * N3);
  double* sPlo = lds + 6 * N3;
  double* sPhi = sPlo + N * N;
  PullEntry* sPull = reinterpret_cast<PullEntry*>(sPhi + N * N);
  restrict_element<N>(T1, T2, sPlo, sPhi, sPull, jb.src, jb.dst, jb.nf[0], jb.nf[1], jb.nc[0],
                      jb.nc[1], jb.split[0], jb.split[1], jb.split[2], T.Plo, T.Phi, jb.go, ec);
}

__global__ void __launch_bounds__(256)
k_batch_restrict(const BTransferJob* __restrict__ jobs, int njobs, const MgTables* __restrict__ tabs) {
  __shared__ double lds[6 * kBatchN3 + 2 * kBatchMaxN * kBatchMaxN + 14];
  const int j = job_of(jobs, njobs, (int)blockIdx.x);
  const BTransferJob& jb = jobs[j];
  const long long ec = (long long)blockIdx.x - jb.blk0;
  const MgTables& T = tabs[jb.N];
  switch (jb.N) {
    case 2: batch_restrict_element<2>(lds, jb, ec, T); break;
    case 3: batch_restrict_element<3>(lds, jb, ec, T); break;
    case 4: batch_restrict_element<4>(lds, jb, ec, T); break;
    case 5: batch_restrict_element<5>(lds, jb, ec, T); break;
    case 6: batch_restrict_element<6>(lds, jb, ec, T); break;
    case 7: batch_restrict_element<7>(lds, jb, ec, T); break;
    case 8: batch_restrict_element<8>(lds, jb, ec, T); break;
    case 9: batch_restrict_element<9>(lds, jb, ec, T); break;
    default: break;
  }
}

template <int N>
__device__ __forceinline__ void batch_prolongate_element(double* lds, const BTransferJob& jb,
                                                         long long ef, const MgTables& T) {
  constexpr int N3 = N * N * N;
  prolongate_element<N>(lds, lds + N3, lds + 2 * N3, lds + 2 * N3 + N * N, jb.src, jb.dst,
                        jb.nf[0], jb.nf[1], jb.nc[0], jb.nc[1], jb.split[0], jb.split[1],
                        jb.split[2], T.Plo, T.Phi, ef);
}

__global__ void __launch_bounds__(256)
k_batch_prolongate(const BTransferJob* __restrict__ jobs, int njobs,
                   const MgTables* __restrict__ tabs) {
  __shared__ double lds[2 * kBatchN3 + 2 * kBatchMaxN * kBatchMaxN];
  const int j = job_of(jobs, njobs, (int)blockIdx.x);
  const BTransferJob& jb = jobs[j];
  const long long ef = (long long)blockIdx.x - jb.blk0;
  const MgTables& T = tabs[jb.N];
  switch (jb.N) {
    case 2: batch_prolongate_element<2>(lds, jb, ef, T); break;
    case 3: batch_prolongate_element<3>(lds, jb, ef, T); break;
    case 4: batch_prolongate_element<4>(lds, jb, ef, T); break;
    case 5: batch_prolongate_element<5>(lds, jb, ef, T); break;
    case 6: batch_prolongate_element<6>(lds, jb, ef, T); break;
    case 7: batch_prolongate_element<7>(lds, jb, ef, T); break;
    case 8: batch_prolongate_element<8>(lds, jb, ef, T); break;
    case 9: batch_prolongate_element<9>(lds, jb, ef, T); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Krylov vector work: the solo kernels' chunks and summation orders per job
// ---------------------------------------------------------------------------
// partial sums: mode 0 dots of V_0..V_{m-1} with w; mode 1 w -= sum coef_i V_i
// then those dots; mode 2 w -= sum coef_i V_i then |w|^2
__global__ void __launch_bounds__(kDotThreads)
k_batch_dot_partial(const BDotJob* __restrict__ jobs, int njobs) {
  __shared__ double red[kDotGroup * (kDotThreads / 64)];
  const int j = job_of(jobs, njobs, (int)blockIdx.x);
  const BDotJob& jb = jobs[j];
  const int blk = (int)blockIdx.x - jb.blk0;
  const long long start = (long long)blk * jb.chunk;
  const long long end = start + jb.chunk < jb.n ? start + jb.chunk : jb.n;
  double* __restrict__ w = jb.w;
  if (jb.mode >= 1) {
    for (long long g = start + threadIdx.x; g < end; g += kDotThreads) {
      double acc = w[g];
      for (int i = 0; i < jb.m; ++i) acc -= jb.coef[i] * jb.V[(long long)i * jb.ldv + g];
      w[g] = acc;
    }
  }
  if (jb.mode == 2) {
    double acc[1] = {0.0};
    for (long long g = start + threadIdx.x; g < end; g += kDotThreads) acc[0] += w[g] * w[g];
    group_store<1>(acc, red, jb.partial + blk, 1);
  } else {
    // partial + blk * m + i, as chunk_dots writes it for a block index blk
    const int m = jb.m;
    for (int i0 = 0; i0 < m; i0 += kDotGroup) {
      double acc[kDotGroup];
#pragma unroll
      for (int q = 0; q < kDotGroup; ++q) acc[q] = 0.0;
      for (long long g = start + threadIdx.x; g < end; g += kDotThreads) {
        const double wg = w[g];
#pragma unroll
        for (int q = 0; q < kDotGroup; ++q)
          if (i0 + q < m) acc[q] += jb.V[(long long)(i0 + q) * jb.ldv + g] * wg;
      }
      group_store<kDotGroup>(acc, red, jb.partial + (long long)blk * m + i0,
                             m - i0 < kDotGroup ? m - i0 : kDotGroup);
    }
  }
}

// h[i] = sum_b partial[b * cnt + i] (cnt = m, or 1 for the norm), one workgroup
// per output, fixed order; the outputs of job j start at workgroup fblk0
__global__ void __launch_bounds__(kDotThreads)
k_batch_dot_final(const BDotJob* __restrict__ jobs, int njobs) {
  __shared__ double red[kDotThreads / 64];
  int j = 0;
  while (j + 1 < njobs && jobs[j + 1].fblk0 <= (int)blockIdx.x) ++j;
  const BDotJob& jb = jobs[j];
  const int i = (int)blockIdx.x - jb.fblk0;
  const int cnt = jb.mode == 2 ? 1 : jb.m;
  double s = 0.0;
  for (int b = threadIdx.x; b < jb.nblocks; b += kDotThreads) s += jb.partial[(long long)b * cnt + i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) jb.h[i] = s;
}

// y = x / sqrt(*nrm2) (also into y2, and into the finest level's subdomain
// rows when go.rs is set), or with Z set: y += sum_i coef_i Z_i
__global__ void __launch_bounds__(256)
k_batch_vec(const BVecJob* __restrict__ jobs, int njobs) {
  const int j = job_of(jobs, njobs, (int)blockIdx.x);
  const BVecJob& jb = jobs[j];
  const long long g = ((long long)blockIdx.x - jb.blk0) * 256 + threadIdx.x;
  if (g >= jb.n) return;
  if (jb.Z) {
    double acc = jb.y[g];
    for (int i = 0; i < jb.m; ++i) acc += jb.coef[i] * jb.Z[(long long)i * jb.ldz + g];
    jb.y[g] = acc;
    return;
  }
  const double v = jb.x[g] / sqrt(jb.nrm2[0]);
  jb.y[g] = v;
  if (jb.y2) jb.y2[g] = v;
  if (jb.go.rs) {
    const int N = jb.N, N3 = N * N * N;
    const long long e = g / N3;
    const int loc = (int)(g - e * N3);
    const int i = loc % N, jj = (loc / N) % N, k = loc / (N * N);
    if (jb.go.f32)
      gather_out_point<float>((float*)jb.go.rs, jb.go.pull + e * 7, N, jb.go.nov, i, jj, k, v);
    else
      gather_out_point<double>((double*)jb.go.rs, jb.go.pull + e * 7, N, jb.go.nov, i, jj, k, v);
  }
}

}  // namespace

hipError_t launch_batch_apply(int mode, bool rows, const BApplyJob* jobs, int njobs, int nblocks,
                              int threads, const DevTables* tabs, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  if (threads != 64 && threads != 128) return hipErrorInvalidValue;
  const dim3 grid((unsigned)nblocks), block((unsigned)threads);
  if (mode == kApply && !rows)
    hipLaunchKernelGGL((k_batch_apply<kApply, false>), grid, block, 0, s, jobs, njobs, tabs);
  else if (mode == kResidual && !rows)
    hipLaunchKernelGGL((k_batch_apply<kResidual, false>), grid, block, 0, s, jobs, njobs, tabs);
  else if (mode == kResidual && rows)
    hipLaunchKernelGGL((k_batch_apply<kResidual, true>), grid, block, 0, s, jobs, njobs, tabs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_batch_scatter(const BScatterJob* jobs, int njobs, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_scatter, dim3((unsigned)nblocks), dim3(256), 0, s, jobs, njobs);
  return hipGetLastError();
}

hipError_t launch_batch_restrict(const BTransferJob* jobs, int njobs, int nblocks,
                                 const MgTables* tabs, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_restrict, dim3((unsigned)nblocks), dim3(256), 0, s, jobs, njobs, tabs);
  return hipGetLastError();
}

hipError_t launch_batch_prolongate(const BTransferJob* jobs, int njobs, int nblocks,
                                   const MgTables* tabs, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_prolongate, dim3((unsigned)nblocks), dim3(256), 0, s, jobs, njobs,
                     tabs);
  return hipGetLastError();
}

hipError_t launch_batch_dots(const BDotJob* jobs, int njobs, int nblocks, int nfinal,
                             hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_dot_partial, dim3((unsigned)nblocks), dim3(kDotThreads), 0, s, jobs,
                     njobs);
  hipLaunchKernelGGL(k_batch_dot_final, dim3((unsigned)nfinal), dim3(kDotThreads), 0, s, jobs,
                     njobs);
  return hipGetLastError();
}

hipError_t launch_batch_vec(const BVecJob* jobs, int njobs, int nblocks, hipStream_t s) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_vec, dim3((unsigned)nblocks), dim3(256), 0, s, jobs, njobs);
  return hipGetLastError();
}

}  // namespace dgs
