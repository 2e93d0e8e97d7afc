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

// Subdomains are grouped by canonical boundary class: an element whose class
// is a mirror image and / or an exchange of equal-width axes of a canonical
// class uses the canonical class's inverse with its points mapped into the
// class frame.  elem_class[e] = group | (frame code << 24).
constexpr int kGroupMask = 0xFFFFFF;

// Pointers into device (global) memory.  Matrices whose addresses are read
// from a table (the class inverses, the per-class rows of the batched GEMM)
// would otherwise be generic pointers, whose loads are flat loads: these count
// against the LDS counter too, so every wait for an LDS read would also wait
// for the prefetch of the next K step.
#define DGS_GLOBAL __attribute__((address_space(1)))

// class-frame point (seg, loc) -> the element's own frame: seg 0 is the
// element itself, seg 1 + f the face neighbour across class-frame face f
__device__ __forceinline__ void frame_point(int& seg, int& loc, int code, int N) {
  if (!code) return;
  const int t = code >> 3;
  const int c0 = loc % N, c1 = (loc / N) % N, c2 = loc / (N * N);
  // the transposition is its own inverse
  int m0 = t == 1 ? c1 : (t == 2 ? c2 : c0);
  int m1 = t == 1 ? c0 : (t == 3 ? c2 : c1);
  int m2 = t == 2 ? c0 : (t == 3 ? c1 : c2);
  if (code & 1) m0 = N - 1 - m0;
  if (code & 2) m1 = N - 1 - m1;
  if (code & 4) m2 = N - 1 - m2;
  loc = (m2 * N + m1) * N + m0;
  if (seg > 0) {
    const int f = seg - 1;
    const int d = frame_axis(f >> 1, t);
    seg = 2 * d + ((f & 1) ^ ((code >> d) & 1)) + 1;
  }
}

// r_S = R_S r for the subdomain of element e (one workgroup per subdomain);
// row elem_row[e] of the class block receives the n_S gathered values.
template <typename T>
__global__ void __launch_bounds__(256)
k_gather_rows(const double* __restrict__ r, T* __restrict__ rs, const int* __restrict__ elem_class,
              const long long* __restrict__ elem_row, const int* __restrict__ nbr,
              const ClassInfo* __restrict__ cls, const int* __restrict__ seg_loc, int E, int N) {
  const int e = blockIdx.x;
  if (e >= E) return;
  const int N3 = N * N * N;
  const int cv = elem_class[e];
  const int code = cv >> 24;
  const ClassInfo ci = cls[cv & kGroupMask];
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
    int seg = sl / N3;
    int loc = sl - seg * N3;
    frame_point(seg, loc, code, N);
    out[k] = (T)r[src[seg] + loc];
  }
}

// Pull-based weighted scatter: every point adds its own subdomain's
// correction and the overlap corrections of the face neighbours' subdomains.
// The per-element pull table holds every offset, so each point issues its
// (at most 7 x PARTS) loads at once: absent or out-of-overlap terms read a
// valid address and are discarded by a select, not skipped by a branch.
template <typename T, int PARTS>
__device__ __forceinline__ double sum_parts(const T* __restrict__ du, long long idx,
                                            long long stride) {
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < PARTS; ++q) v += (double)du[q * stride + idx];
  return v;
}

template <typename T, int PARTS>
__global__ void __launch_bounds__(256)
k_scatter(double* __restrict__ u, const T* __restrict__ du, long long pstride,
          const double* __restrict__ weights, const PullEntry* __restrict__ pull, int N, int nov,
          long long total, int assign) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int N2 = N * N, N3 = N2 * N;
  const long long e = g / N3;
  const int loc = (int)(g - e * N3);
  const int idx[3] = {loc % N, (loc / N) % N, loc / N2};
  const PullEntry* pe = pull + e * 7;
  const PullEntry own = pe[0];
  const int lc = to_class_frame(idx[0], idx[1], idx[2], own.flip, N);
  double acc = weights[own.w + lc] * sum_parts<T, PARTS>(du, own.du + lc, pstride);
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const PullEntry q = pe[1 + f];
    const int d = f >> 1;
    const int layer = (f & 1) ? (N - 1 - idx[d]) : idx[d];
    int t0 = idx[d == 0 ? 1 : 0], t1 = idx[d == 2 ? 1 : 2];  // transverse coordinates
    strip_coords(t0, t1, q.flip, N);
    const bool ok = q.du >= 0 && layer < nov;
    const int k = ok ? layer * N2 + t1 * N + t0 : lc;
    const long long bd = ok ? q.du : own.du;
    const int bw = ok ? q.w : own.w;
    const double v = weights[bw + k] * sum_parts<T, PARTS>(du, bd + k, pstride);
    acc += ok ? v : 0.0;
  }
  if (assign)  // u starts from zero: write instead of add (no clearing pass)
    u[g] = acc;
  else
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

// Tiled grouped GEMM.  Four waves arranged WM x WN, each computing TM x TN
// MFMA tiles of 16 x 16; the block tile is BM = 16 WM TM rows by BN = 16 WN TN
// columns, the K loop steps by BK with the next tile prefetched into registers
// while the current one is multiplied out of LDS.
//
// BATCH: the classes come from several problems (the serving loop's batched
// sweeps): class c's subdomain rows and corrections are at ptrs[c].rs /
// ptrs[c].du, with its own part stride, instead of the shared rs / du.
template <typename T, int WM, int WN, int TM, int TN, int BK, bool BATCH = false>
__global__ void __launch_bounds__(256)
k_sub_gemm(const T* __restrict__ rs, T* __restrict__ du,
           long long pstride, const ClassInfo* __restrict__ cls,
           const GemmTile* __restrict__ tiles, int use_op,
           const GemmPtr* __restrict__ ptrs = nullptr) {
  constexpr int BM = 16 * WM * TM, BN = 16 * WN * TN;
  // LDS row paddings: the MFMA operand reads touch 16 lanes per row and 2 (FP32)
  // or 1 (FP64) rows per LDS cycle; row strides of 36 / 144 floats (FP32) and
  // 18 / 136 doubles (FP64) put those row groups on disjoint banks and keep
  // every row 16-byte aligned for vector stores
  constexpr int PA = sizeof(T) == 4 ? 4 : 2, PB = sizeof(T) == 4 ? 16 : 8;
  // tiles move as 16-byte vectors: the class blocks are padded (zero outside
  // the values) so that no load needs a bounds check
  constexpr int VW = 16 / (int)sizeof(T);
  typedef T vec __attribute__((ext_vector_type(VW)));
  constexpr int AV = BM * BK / VW, BV = BK * BN / VW;
  constexpr int NAV = (AV + 255) / 256, NBV = BV / 256;
  static_assert(BV % 256 == 0 && BK % VW == 0, "tile");
  typedef typename Mfma<T>::v4 v4;
  __shared__ __attribute__((aligned(16))) T As[BM][BK + PA];  // row-major like RS
  __shared__ __attribute__((aligned(16))) T Bs[BK][BN + PB];
  const GemmTile tl = tiles[blockIdx.x];
  const ClassInfo ci = cls[tl.cls];
  const int ld = ci.ld;
  const T DGS_GLOBAL* A;
  T DGS_GLOBAL* C;
  if constexpr (BATCH) {
    const GemmPtr gp = ptrs[tl.cls];
    A = (const T DGS_GLOBAL*)gp.rs + ci.rs_off;
    C = (T DGS_GLOBAL*)gp.du + tl.part * gp.pstride + ci.rs_off;
  } else {
    A = (const T DGS_GLOBAL*)rs + ci.rs_off;
    C = (T DGS_GLOBAL*)du + tl.part * pstride + ci.rs_off;
  }
  const T DGS_GLOBAL* B = (const T DGS_GLOBAL*)(use_op ? ci.op : ci.inv);
  const int m0 = tl.m0, n0 = tl.n0, kbeg = tl.k0, kend = tl.k1;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave / WN, wn = wave % WN;
  v4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = v4{0, 0, 0, 0};

  vec ra[NAV], rb[NBV];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NAV; ++q) {
      const int idx = tid + 256 * q;
      if (AV % 256 == 0 || idx < AV) {
        const int r = idx / (BK / VW), c = idx % (BK / VW);
        ra[q] = *(const vec DGS_GLOBAL*)(A + (long long)(m0 + r) * ld + k0 + c * VW);
      }
    }
#pragma unroll
    for (int q = 0; q < NBV; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / (BN / VW), c = idx % (BN / VW);
      rb[q] = *(const vec DGS_GLOBAL*)(B + (long long)(k0 + r) * ld + n0 + c * VW);
    }
  };
  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int q = 0; q < NAV; ++q) {
      const int idx = tid + 256 * q;
      if (AV % 256 == 0 || idx < AV) {
        const int r = idx / (BK / VW), c = idx % (BK / VW);
        *(vec*)&As[r][c * VW] = ra[q];
      }
    }
#pragma unroll
    for (int q = 0; q < NBV; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / (BN / VW), c = idx % (BN / VW);
      *(vec*)&Bs[r][c * VW] = rb[q];
    }
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[(wm * TM + a) * 16 + (lane & 15)][kr];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = Bs[kr][(wn * TN + b) * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = Mfma<T>::run(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  // the tile lies inside the padded class block: padding rows and columns
  // receive zeros (their operands are zero)
  const T sc = (T)(use_op ? ci.scale_op : ci.scale);
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + (wm * TM + a) * 16 + Mfma<T>::row(lane, r);
        const int col = n0 + (wn * TN + b) * 16 + (lane & 15);
        C[(long long)row * ld + col] = sc * acc[a][b][r];
      }
}

// Double-buffered form of the grouped GEMM: two LDS stages and two register
// stages.  The loads of K step k + 2 are issued before step k is multiplied,
// so they have two steps of MFMA work to land, and one barrier per step
// orders the LDS stages.  Same tiles, K ranges and summation order as
// k_sub_gemm.
template <typename T, int WM, int WN, int TM, int TN, int BK>
__global__ void __launch_bounds__(256)
k_sub_gemm_db(const T* __restrict__ rs, T* __restrict__ du, long long pstride,
              const ClassInfo* __restrict__ cls, const GemmTile* __restrict__ tiles, int use_op) {
  constexpr int BM = 16 * WM * TM, BN = 16 * WN * TN;
  constexpr int PA = sizeof(T) == 4 ? 4 : 2, PB = sizeof(T) == 4 ? 16 : 8;
  constexpr int VW = 16 / (int)sizeof(T);
  typedef T vec __attribute__((ext_vector_type(VW)));
  constexpr int AV = BM * BK / VW, BV = BK * BN / VW;
  constexpr int NAV = AV / 256, NBV = BV / 256;
  static_assert(AV % 256 == 0 && BV % 256 == 0 && BK % VW == 0, "tile");
  typedef typename Mfma<T>::v4 v4;
  __shared__ __attribute__((aligned(16))) T As[2][BM][BK + PA];
  __shared__ __attribute__((aligned(16))) T Bs[2][BK][BN + PB];
  const GemmTile tl = tiles[blockIdx.x];
  const ClassInfo ci = cls[tl.cls];
  const int ld = ci.ld;
  const T DGS_GLOBAL* A = (const T DGS_GLOBAL*)rs + ci.rs_off;
  T DGS_GLOBAL* C = (T DGS_GLOBAL*)du + tl.part * pstride + ci.rs_off;
  const T DGS_GLOBAL* B = (const T DGS_GLOBAL*)(use_op ? ci.op : ci.inv);
  const int m0 = tl.m0, n0 = tl.n0, kbeg = tl.k0;
  const int nk = (tl.k1 - tl.k0) / BK;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave / WN, wn = wave % WN;
  v4 acc[TM][TN];
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = v4{0, 0, 0, 0};

  vec ra0[NAV], rb0[NBV], ra1[NAV], rb1[NBV];
  auto load = [&](vec* ra, vec* rb, int step) {
    const int k0 = kbeg + step * BK;
#pragma unroll
    for (int q = 0; q < NAV; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / (BK / VW), c = idx % (BK / VW);
      ra[q] = *(const vec DGS_GLOBAL*)(A + (long long)(m0 + r) * ld + k0 + c * VW);
    }
#pragma unroll
    for (int q = 0; q < NBV; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / (BN / VW), c = idx % (BN / VW);
      rb[q] = *(const vec DGS_GLOBAL*)(B + (long long)(k0 + r) * ld + n0 + c * VW);
    }
  };
  auto store = [&](int buf, const vec* ra, const vec* rb) {
#pragma unroll
    for (int q = 0; q < NAV; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / (BK / VW), c = idx % (BK / VW);
      *(vec*)&As[buf][r][c * VW] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NBV; ++q) {
      const int idx = tid + 256 * q;
      const int r = idx / (BN / VW), c = idx % (BN / VW);
      *(vec*)&Bs[buf][r][c * VW] = rb[q];
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T av[TM], bv[TN];
#pragma unroll
      for (int a = 0; a < TM; ++a) av[a] = As[buf][(wm * TM + a) * 16 + (lane & 15)][kr];
#pragma unroll
      for (int b = 0; b < TN; ++b) bv[b] = Bs[buf][kr][(wn * TN + b) * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = Mfma<T>::run(av[a], bv[b], acc[a][b]);
    }
  };
  // at the top of step k, LDS stage k % 2 holds tile k and register stage
  // (k + 1) % 2 holds (or is still loading) tile k + 1
  if (nk > 0) load(ra0, rb0, 0);
  if (nk > 1) load(ra1, rb1, 1);
  if (nk > 0) store(0, ra0, rb0);
  __syncthreads();
  for (int k = 0; k < nk; k += 2) {
    if (k + 2 < nk) load(ra0, rb0, k + 2);
    compute(0);
    if (k + 1 < nk) store(1, ra1, rb1);
    __syncthreads();
    if (k + 1 < nk) {
      if (k + 3 < nk) load(ra1, rb1, k + 3);
      compute(1);
      if (k + 2 < nk) store(0, ra0, rb0);
      __syncthreads();
    }
  }
  const T sc = (T)(use_op ? ci.scale_op : ci.scale);
#pragma unroll
  for (int a = 0; a < TM; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + (wm * TM + a) * 16 + Mfma<T>::row(lane, r);
        const int col = n0 + (wn * TN + b) * 16 + (lane & 15);
        C[(long long)row * ld + col] = sc * acc[a][b][r];
      }
}

template <typename T>
__global__ void k_reduce_parts(T* __restrict__ out, const T* __restrict__ parts, int np,
                               long long stride, long long total) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  double v = 0.0;
  for (int p = 0; p < np; ++p) v += (double)parts[p * stride + g];
  out[g] = (T)v;
}

__device__ __forceinline__ double block_reduce_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();  // red may still be read from a previous reduction
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;  // every thread gets the same sum, in the same order
}

constexpr int kSubThreads = 256;
// points per thread of the Arnoldi step: n_S <= 2048 (p <= 8) or <= 4352
// (p <= 12, n_S <= 4225)
constexpr int kSubPerSmall = 8, kSubPerLarge = 17;

template <typename T>
__global__ void __launch_bounds__(kSubThreads)
k_sub_start(const T* __restrict__ rs, T* __restrict__ V0, double* __restrict__ beta,
            const int* __restrict__ elem_class, const long long* __restrict__ elem_row,
            const ClassInfo* __restrict__ cls, int E) {
  __shared__ double red[kSubThreads / 64];
  const int e = blockIdx.x;
  if (e >= E) return;
  const int n = cls[elem_class[e] & kGroupMask].n;
  const long long row = elem_row[e];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kSubThreads) {
    const double x = (double)rs[row + i];
    s += x * x;
  }
  const double b = sqrt(block_reduce_sum(s, red));
  if (threadIdx.x == 0) beta[e] = b;
  for (int i = threadIdx.x; i < n; i += kSubThreads)
    V0[row + i] = b > 0.0 ? (T)((double)rs[row + i] / b) : (T)0;
}

template <typename T, int kSubPer>
__global__ void __launch_bounds__(kSubThreads)
k_sub_arnoldi(int j, int kmax, const T* __restrict__ W, T* __restrict__ V, const T* __restrict__ Zj,
              long long stride, const double* __restrict__ diag, double* __restrict__ H,
              const int* __restrict__ elem_class, const long long* __restrict__ elem_row,
              const int* __restrict__ nbr, const ClassInfo* __restrict__ cls,
              const int* __restrict__ seg_loc, int E, int N) {
  __shared__ double red[kSubThreads / 64];
  __shared__ long long src[7];
  const int N3 = N * N * N;
  const int e = blockIdx.x;
  if (e >= E) return;
  const int cv = elem_class[e];
  const int code = cv >> 24;
  const ClassInfo ci = cls[cv & kGroupMask];
  const int n = ci.n;
  const long long row = elem_row[e];
  if (threadIdx.x < 7) {
    const int el = threadIdx.x == 0 ? e : nbr[(long long)e * 6 + threadIdx.x - 1];
    src[threadIdx.x] = (long long)el * N3;
  }
  __syncthreads();
  const int* lay = seg_loc + ci.layout_off;
  double w[kSubPer];
#pragma unroll
  for (int q = 0; q < kSubPer; ++q) {
    const int i = threadIdx.x + q * kSubThreads;
    w[q] = 0.0;
    if (i < n) {
      const int sl = lay[i];
      int seg = sl / N3;
      int loc = sl - seg * N3;
      frame_point(seg, loc, code, N);
      const double d = diag[src[seg] + loc];
      w[q] = (double)W[row + i] + d * (double)Zj[row + i];
    }
  }
  double* Hs = H + (long long)e * (kmax + 1) * kmax;  // column-major (kmax+1) x kmax
  for (int i = 0; i <= j; ++i) {
    const T* vi = V + i * stride + row;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kSubPer; ++q) {
      const int p = threadIdx.x + q * kSubThreads;
      if (p < n) s += w[q] * (double)vi[p];
    }
    const double h = block_reduce_sum(s, red);
#pragma unroll
    for (int q = 0; q < kSubPer; ++q) {
      const int p = threadIdx.x + q * kSubThreads;
      if (p < n) w[q] -= h * (double)vi[p];
    }
    if (threadIdx.x == 0) Hs[j * (kmax + 1) + i] = h;
  }
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kSubPer; ++q) s += w[q] * w[q];
  const double hn = sqrt(block_reduce_sum(s, red));
  if (threadIdx.x == 0) Hs[j * (kmax + 1) + j + 1] = hn;
  if (j + 1 <= kmax) {
    T* vn = V + (j + 1) * stride + row;
#pragma unroll
    for (int q = 0; q < kSubPer; ++q) {
      const int p = threadIdx.x + q * kSubThreads;
      if (p < n) vn[p] = hn > 0.0 ? (T)(w[q] / hn) : (T)0;
    }
  }
}

// Least squares min |beta e1 - H y| of one subdomain's (kmax+1) x kmax
// Hessenberg matrix Hs (column-major) by Givens rotations, stopping at a
// breakdown column (zero subdiagonal); returns the number of columns used
// (0 for beta = 0) and writes y.  One thread.
// h and g: LDS scratch of the calling workgroup (runtime-indexed arrays in
// private memory would live in scratch memory)
__device__ int small_lsq(const double* Hs, int kmax, double beta, double* y, double (*h)[8],
                         double* g) {
  int m = kmax;
  for (int jj = 0; jj < kmax; ++jj)
    if (Hs[jj * (kmax + 1) + jj + 1] == 0.0) {
      m = jj + 1;
      break;
    }
  for (int jj = 0; jj < m; ++jj)
    for (int ii = 0; ii <= m; ++ii) h[ii][jj] = (ii <= jj + 1) ? Hs[jj * (kmax + 1) + ii] : 0.0;
  for (int ii = 0; ii <= m; ++ii) g[ii] = 0.0;
  g[0] = beta;
  if (g[0] == 0.0) return 0;
  for (int jj = 0; jj < m; ++jj) {
    const double a = h[jj][jj], b = h[jj + 1][jj];
    const double r = sqrt(a * a + b * b);
    const double c = a / r, sn = b / r;
    for (int q = jj; q < m; ++q) {
      const double t0 = h[jj][q], t1 = h[jj + 1][q];
      h[jj][q] = c * t0 + sn * t1;
      h[jj + 1][q] = -sn * t0 + c * t1;
    }
    const double g0 = g[jj], g1 = g[jj + 1];
    g[jj] = c * g0 + sn * g1;
    g[jj + 1] = -sn * g0 + c * g1;
  }
  for (int ii = m - 1; ii >= 0; --ii) {
    double t = g[ii];
    for (int q = ii + 1; q < m; ++q) t -= h[ii][q] * y[q];
    y[ii] = t / h[ii][ii];
  }
  return m;
}

template <typename T>
__global__ void __launch_bounds__(kSubThreads)
k_sub_finish(int kmax, const T* __restrict__ Z, long long stride, const double* __restrict__ H,
             const double* __restrict__ beta, T* __restrict__ du,
             const int* __restrict__ elem_class, const long long* __restrict__ elem_row,
             const ClassInfo* __restrict__ cls, int E) {
  __shared__ double y[16];
  __shared__ double lsq_h[9][8], lsq_g[9];
  __shared__ int mm;
  const int e = blockIdx.x;
  if (e >= E) return;
  const int n = cls[elem_class[e] & kGroupMask].n;
  const long long row = elem_row[e];
  if (threadIdx.x == 0)
    mm = small_lsq(H + (long long)e * (kmax + 1) * kmax, kmax, beta[e], y, lsq_h, lsq_g);
  __syncthreads();
  const int m = mm;
  for (int i = threadIdx.x; i < n; i += kSubThreads) {
    double v = 0.0;
    for (int jj = 0; jj < m; ++jj) v += y[jj] * (double)Z[jj * stride + row + i];
    du[row + i] = (T)v;
  }
}

// ---------------------------------------------------------------------------
// Subdomain GMRES(k) of a system of nv variables (Sec. III.E.1): the
// subdomain vector stacks the variables' rows, variable a's at a * stride in
// every buffer (the variables share one class structure, so a subdomain's
// rows sit at the same offset for all of them).  The operator is
// blockdiag_a(A_S^(a)) + D_S with pointwise couplings D_ab; the GEMMs with
// each variable's Poisson inverse and subdomain operator run between the
// Arnoldi steps, like the scalar form above.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(kSubThreads)
k_sys_start(int nv, const T* __restrict__ rs, T* __restrict__ V0, double* __restrict__ beta,
            long long stride, const int* __restrict__ elem_class,
            const long long* __restrict__ elem_row, const ClassInfo* __restrict__ cls, int E) {
  __shared__ double red[kSubThreads / 64];
  const int e = blockIdx.x;
  if (e >= E) return;
  const int n = cls[elem_class[e] & kGroupMask].n;
  const long long row = elem_row[e];
  double s = 0.0;
  for (int a = 0; a < nv; ++a)
    for (int i = threadIdx.x; i < n; i += kSubThreads) {
      const double x = (double)rs[a * stride + row + i];
      s += x * x;
    }
  const double b = sqrt(block_reduce_sum(s, red));
  if (threadIdx.x == 0) beta[e] = b;
  for (int a = 0; a < nv; ++a)
    for (int i = threadIdx.x; i < n; i += kSubThreads)
      V0[a * stride + row + i] = b > 0.0 ? (T)((double)rs[a * stride + row + i] / b) : (T)0;
}

// One Arnoldi step j: w_a = W_a + sum_b D_ab z_b at every subdomain point
// (W_a = A_S^(a) z_a from the GEMM), classical Gram-Schmidt against the
// stacked basis vectors 0..j, the Hessenberg column, and v_{j+1}.  Basis slot
// i of V is at i * nv * stride.  Subdomains of at most kSubThreads *
// kSubPerSmall points and at most kSysMaxVars variables.
template <typename T>
__global__ void __launch_bounds__(kSubThreads)
k_sys_arnoldi(int j, int kmax, int nv, const T* __restrict__ W, T* __restrict__ V,
              const T* __restrict__ Zj, long long stride, const double* __restrict__ D,
              long long nd, double* __restrict__ H, const int* __restrict__ elem_class,
              const long long* __restrict__ elem_row, const int* __restrict__ nbr,
              const ClassInfo* __restrict__ cls, const int* __restrict__ seg_loc, int E, int N) {
  __shared__ double red[kSubThreads / 64];
  __shared__ long long src[7];
  const int N3 = N * N * N;
  const int e = blockIdx.x;
  if (e >= E) return;
  const int cv = elem_class[e];
  const int code = cv >> 24;
  const ClassInfo ci = cls[cv & kGroupMask];
  const int n = ci.n;
  const long long row = elem_row[e];
  if (threadIdx.x < 7) {
    const int el = threadIdx.x == 0 ? e : nbr[(long long)e * 6 + threadIdx.x - 1];
    src[threadIdx.x] = (long long)el * N3;
  }
  __syncthreads();
  const int* lay = seg_loc + ci.layout_off;
  double w[kSysMaxVars][kSubPerSmall];
#pragma unroll
  for (int q = 0; q < kSubPerSmall; ++q) {
    const int i = threadIdx.x + q * kSubThreads;
    long long g = 0;
    if (i < n) {
      const int sl = lay[i];
      int seg = sl / N3;
      int loc = sl - seg * N3;
      frame_point(seg, loc, code, N);
      g = src[seg] + loc;
    }
#pragma unroll
    for (int a = 0; a < kSysMaxVars; ++a) {
      double v = 0.0;
      if (a < nv && i < n) {
        v = (double)W[a * stride + row + i];
        for (int b = 0; b < nv; ++b)
          v += D[(long long)(a * nv + b) * nd + g] * (double)Zj[b * stride + row + i];
      }
      w[a][q] = v;
    }
  }
  const long long slot = (long long)nv * stride;
  double* Hs = H + (long long)e * (kmax + 1) * kmax;  // column-major (kmax+1) x kmax
  for (int ii = 0; ii <= j; ++ii) {
    const T* vi = V + ii * slot + row;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < kSysMaxVars; ++a)
#pragma unroll
      for (int q = 0; q < kSubPerSmall; ++q) {
        const int p = threadIdx.x + q * kSubThreads;
        if (a < nv && p < n) s += w[a][q] * (double)vi[a * stride + p];
      }
    const double h = block_reduce_sum(s, red);
#pragma unroll
    for (int a = 0; a < kSysMaxVars; ++a)
#pragma unroll
      for (int q = 0; q < kSubPerSmall; ++q) {
        const int p = threadIdx.x + q * kSubThreads;
        if (a < nv && p < n) w[a][q] -= h * (double)vi[a * stride + p];
      }
    if (threadIdx.x == 0) Hs[j * (kmax + 1) + ii] = h;
  }
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < kSysMaxVars; ++a)
#pragma unroll
    for (int q = 0; q < kSubPerSmall; ++q) s += w[a][q] * w[a][q];
  const double hn = sqrt(block_reduce_sum(s, red));
  if (threadIdx.x == 0) Hs[j * (kmax + 1) + j + 1] = hn;
  if (j + 1 <= kmax) {
    T* vn = V + (j + 1) * slot + row;
#pragma unroll
    for (int a = 0; a < kSysMaxVars; ++a)
#pragma unroll
      for (int q = 0; q < kSubPerSmall; ++q) {
        const int p = threadIdx.x + q * kSubThreads;
        if (a < nv && p < n) vn[a * stride + p] = hn > 0.0 ? (T)(w[a][q] / hn) : (T)0;
      }
  }
}

// du_a = sum_j y_j Z_j,a with y the least-squares coefficients (Z slot j at
// j * nv * stride); du is written as part 0 of each variable's block.
template <typename T>
__global__ void __launch_bounds__(kSubThreads)
k_sys_finish(int kmax, int nv, const T* __restrict__ Z, long long stride,
             const double* __restrict__ H, const double* __restrict__ beta, T* __restrict__ du,
             const int* __restrict__ elem_class, const long long* __restrict__ elem_row,
             const ClassInfo* __restrict__ cls, int E) {
  __shared__ double y[16];
  __shared__ double lsq_h[9][8], lsq_g[9];
  __shared__ int mm;
  const int e = blockIdx.x;
  if (e >= E) return;
  const int n = cls[elem_class[e] & kGroupMask].n;
  const long long row = elem_row[e];
  if (threadIdx.x == 0)
    mm = small_lsq(H + (long long)e * (kmax + 1) * kmax, kmax, beta[e], y, lsq_h, lsq_g);
  __syncthreads();
  const int m = mm;
  const long long slot = (long long)nv * stride;
  for (int a = 0; a < nv; ++a)
    for (int i = threadIdx.x; i < n; i += kSubThreads) {
      double v = 0.0;
      for (int jj = 0; jj < m; ++jj) v += y[jj] * (double)Z[jj * slot + a * stride + row + i];
      du[a * stride + row + i] = (T)v;
    }
}

// y_a += sign * sum_b D_ab u_b pointwise (the coupling of a system)
__global__ void k_sys_couple(double* __restrict__ y, const double* __restrict__ u,
                             const double* __restrict__ D, int nv, long long nd, double sign) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nd) return;
  for (int a = 0; a < nv; ++a) {
    double acc = 0.0;
    for (int b = 0; b < nv; ++b) acc += D[(long long)(a * nv + b) * nd + g] * u[b * nd + g];
    y[a * nd + g] += sign * acc;
  }
}

}  // namespace

hipError_t launch_reduce_parts(bool f32, void* out, const void* parts_base, int parts,
                               long long stride, long long total, hipStream_t s) {
  if (total <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  if (f32)
    hipLaunchKernelGGL(k_reduce_parts<float>, dim3(blocks), dim3(256), 0, s, (float*)out,
                       (const float*)parts_base, parts, stride, total);
  else
    hipLaunchKernelGGL(k_reduce_parts<double>, dim3(blocks), dim3(256), 0, s, (double*)out,
                       (const double*)parts_base, parts, stride, total);
  return hipGetLastError();
}

hipError_t launch_sub_start(bool f32, const void* rs, void* V0, double* beta,
                            const int* elem_class, const long long* elem_row, const ClassInfo* cls,
                            int E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_sub_start<float>, dim3(E), dim3(kSubThreads), 0, s, (const float*)rs,
                       (float*)V0, beta, elem_class, elem_row, cls, E);
  else
    hipLaunchKernelGGL(k_sub_start<double>, dim3(E), dim3(kSubThreads), 0, s, (const double*)rs,
                       (double*)V0, beta, elem_class, elem_row, cls, E);
  return hipGetLastError();
}

hipError_t launch_sub_arnoldi(int N, bool f32, int j, int kmax, const void* W, void* V, const void* Zj,
                              long long stride, const double* diag, double* H,
                              const int* elem_class, const long long* elem_row, const int* nbr,
                              const ClassInfo* cls, const int* seg_loc, int E, int max_n,
                              hipStream_t s) {
  if (E <= 0) return hipSuccess;
  if (max_n > kSubThreads * kSubPerLarge) return hipErrorInvalidValue;
  const bool large = max_n > kSubThreads * kSubPerSmall;
#define DGS_ARNOLDI(T, PER)                                                                     \
  hipLaunchKernelGGL((k_sub_arnoldi<T, PER>), dim3(E), dim3(kSubThreads), 0, s, j, kmax,         \
                     (const T*)W, (T*)V, (const T*)Zj, stride, diag, H, elem_class, elem_row, nbr, \
                     cls, seg_loc, E, N)
  if (f32) {
    if (large)
      DGS_ARNOLDI(float, kSubPerLarge);
    else
      DGS_ARNOLDI(float, kSubPerSmall);
  } else {
    if (large)
      DGS_ARNOLDI(double, kSubPerLarge);
    else
      DGS_ARNOLDI(double, kSubPerSmall);
  }
#undef DGS_ARNOLDI
  return hipGetLastError();
}

hipError_t launch_sub_finish(bool f32, int kmax, const void* Z, long long stride, const double* H,
                             const double* beta, void* du, const int* elem_class,
                             const long long* elem_row, const ClassInfo* cls, int E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_sub_finish<float>, dim3(E), dim3(kSubThreads), 0, s, kmax, (const float*)Z,
                       stride, H, beta, (float*)du, elem_class, elem_row, cls, E);
  else
    hipLaunchKernelGGL(k_sub_finish<double>, dim3(E), dim3(kSubThreads), 0, s, kmax,
                       (const double*)Z, stride, H, beta, (double*)du, elem_class, elem_row, cls, E);
  return hipGetLastError();
}

hipError_t launch_sys_start(bool f32, int nv, const void* rs, void* V0, double* beta,
                            long long stride, const int* elem_class, const long long* elem_row,
                            const ClassInfo* cls, int E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_sys_start<float>, dim3(E), dim3(kSubThreads), 0, s, nv, (const float*)rs,
                       (float*)V0, beta, stride, elem_class, elem_row, cls, E);
  else
    hipLaunchKernelGGL(k_sys_start<double>, dim3(E), dim3(kSubThreads), 0, s, nv,
                       (const double*)rs, (double*)V0, beta, stride, elem_class, elem_row, cls, E);
  return hipGetLastError();
}

hipError_t launch_sys_arnoldi(int N, bool f32, int j, int kmax, int nv, const void* W, void* V,
                              const void* Zj, long long stride, const double* D, long long nd,
                              double* H, const int* elem_class, const long long* elem_row,
                              const int* nbr, const ClassInfo* cls, const int* seg_loc, int E,
                              int max_n, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  if (max_n > kSubThreads * kSubPerSmall || nv < 1 || nv > kSysMaxVars) return hipErrorInvalidValue;
  if (f32)
    hipLaunchKernelGGL(k_sys_arnoldi<float>, dim3(E), dim3(kSubThreads), 0, s, j, kmax, nv,
                       (const float*)W, (float*)V, (const float*)Zj, stride, D, nd, H, elem_class,
                       elem_row, nbr, cls, seg_loc, E, N);
  else
    hipLaunchKernelGGL(k_sys_arnoldi<double>, dim3(E), dim3(kSubThreads), 0, s, j, kmax, nv,
                       (const double*)W, (double*)V, (const double*)Zj, stride, D, nd, H,
                       elem_class, elem_row, nbr, cls, seg_loc, E, N);
  return hipGetLastError();
}

hipError_t launch_sys_finish(bool f32, int kmax, int nv, const void* Z, long long stride,
                             const double* H, const double* beta, void* du, const int* elem_class,
                             const long long* elem_row, const ClassInfo* cls, int E,
                             hipStream_t s) {
  if (E <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_sys_finish<float>, dim3(E), dim3(kSubThreads), 0, s, kmax, nv,
                       (const float*)Z, stride, H, beta, (float*)du, elem_class, elem_row, cls, E);
  else
    hipLaunchKernelGGL(k_sys_finish<double>, dim3(E), dim3(kSubThreads), 0, s, kmax, nv,
                       (const double*)Z, stride, H, beta, (double*)du, elem_class, elem_row, cls,
                       E);
  return hipGetLastError();
}

hipError_t launch_sys_couple(double* y, const double* u, const double* D, int nv, long long nd,
                             double sign, hipStream_t s) {
  if (nd <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sys_couple, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, s, y, u, D,
                     nv, nd, sign);
  return hipGetLastError();
}

hipError_t launch_gather(int N, bool f32, const double* r, void* rs, const int* elem_class,
                         const long long* elem_row, const int* nbr, const ClassInfo* cls,
                         const int* seg_loc, int E, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_gather_rows<float>, dim3(E), dim3(256), 0, s, r, (float*)rs, elem_class,
                       elem_row, nbr, cls, seg_loc, E, N);
  else
    hipLaunchKernelGGL(k_gather_rows<double>, dim3(E), dim3(256), 0, s, r, (double*)rs, elem_class,
                       elem_row, nbr, cls, seg_loc, E, N);
  return hipGetLastError();
}

GemmPlan plan_subdomain_gemm(const std::vector<ClassInfo>& cls, int variant, int parts_cap) {
  GemmPlan plan;
  bool any_big = false;
  for (const ClassInfo& c : cls) any_big = any_big || c.count > kGemmSmallCount;
  // the few partly filled tiles of small classes run beside the large ones
  plan.small = !any_big;
  const int bm = plan.small ? 16 : ((variant == 1 || variant == 3) ? 64 : 32);
  // few-subdomain levels: 16 x 64 tiles, twice as many and half as long as
  // 16 x 128 ones (these launches are latency-bound); variant 2 of the large
  // levels: 32 x 64 tiles, for levels whose 32 x 128 tiles leave the compute
  // units short of work; variants 3 (64 x 64) and 4 (32 x 64): the
  // double-buffered kernel, which keeps two K steps of loads in flight
  const int bn = (plan.small || variant == 2 || variant >= 3) ? 64 : kGemmN;
  // split K until there are enough tiles to fill the 256 compute units; the
  // short K loops of few-subdomain levels are latency-bound, so they may
  // split further (up to 16 parts in variant 0, 4 in variant 1: more parts
  // shorten the GEMM and lengthen the scatter that sums them)
  int base = 0;
  for (const ClassInfo& c : cls) base += ((c.count + bm - 1) / bm) * ((c.n + bn - 1) / bn);
  static const int small_parts[kGemmVariants] = {kMaxParts, 4, 8, 2, 1};
  int max_parts = plan.small ? small_parts[variant] : 4;
  if (parts_cap > 0) max_parts = std::min(max_parts, parts_cap);
  plan.kparts = 1;
  while (plan.kparts < max_parts && base * plan.kparts < 1024) plan.kparts *= 2;
  for (int c = 0; c < (int)cls.size(); ++c) {
    const ClassInfo& I = cls[c];
    // K runs over the padded extent in chunks of whole 32-wide steps (FP32 and
    // FP64 tiles both stay aligned)
    const int chunk = ((I.kext + plan.kparts - 1) / plan.kparts + 31) / 32 * 32;
    for (int part = 0; part < plan.kparts; ++part) {
      const int k0 = part * chunk, k1 = std::min(I.kext, (part + 1) * chunk);
      for (int m0 = 0; m0 < I.count; m0 += bm)
        for (int n0 = 0; n0 < I.n; n0 += bn)
          // an empty K range still writes zeros so every part is defined
          plan.tiles.push_back(GemmTile{c, m0, n0, part, k0, std::max(k0, k1)});
    }
  }
  return plan;
}

hipError_t launch_subdomain_gemm(bool f32, const void* rs, void* du, long long ps,
                                 const ClassInfo* cls, const GemmTile* tiles, int ntiles,
                                 bool small, int use_op, hipStream_t s, int variant) {
  if (ntiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)ntiles), block(256);
  if (f32) {
    const float* a = (const float*)rs;
    float* c = (float*)du;
    if (small)
      hipLaunchKernelGGL((k_sub_gemm<float, 1, 4, 1, 1, 32>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
    else if (variant == 0)
      hipLaunchKernelGGL((k_sub_gemm<float, 2, 2, 1, 4, 32>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
    else if (variant == 2)
      hipLaunchKernelGGL((k_sub_gemm<float, 2, 2, 1, 2, 32>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
    else if (variant == 3)
      hipLaunchKernelGGL((k_sub_gemm_db<float, 2, 2, 2, 2, 32>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
    else if (variant == 4)
      hipLaunchKernelGGL((k_sub_gemm_db<float, 2, 2, 1, 2, 32>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
    else
      hipLaunchKernelGGL((k_sub_gemm<float, 2, 2, 2, 4, 32>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
  } else {
    const double* a = (const double*)rs;
    double* c = (double*)du;
    if (small)
      hipLaunchKernelGGL((k_sub_gemm<double, 1, 4, 1, 1, 16>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
    else if (variant == 0)
      hipLaunchKernelGGL((k_sub_gemm<double, 2, 2, 1, 4, 16>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
    else if (variant == 2)
      hipLaunchKernelGGL((k_sub_gemm<double, 2, 2, 1, 2, 16>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
    else if (variant == 3)
      hipLaunchKernelGGL((k_sub_gemm_db<double, 2, 2, 2, 2, 16>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
    else if (variant == 4)
      hipLaunchKernelGGL((k_sub_gemm_db<double, 2, 2, 1, 2, 16>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
    else
      hipLaunchKernelGGL((k_sub_gemm<double, 2, 2, 2, 4, 16>), grid, block, 0, s, a, c, ps, cls,
                         tiles, use_op);
  }
  return hipGetLastError();
}

hipError_t launch_subdomain_gemm_batched(bool f32, const ClassInfo* cls, const GemmPtr* ptrs,
                                         const GemmTile* tiles, int ntiles, bool small,
                                         hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)ntiles), block(256);
  if (f32) {
    if (small)
      hipLaunchKernelGGL((k_sub_gemm<float, 1, 4, 1, 1, 32, true>), grid, block, 0, s, nullptr,
                         nullptr, 0, cls, tiles, 0, ptrs);
    else
      hipLaunchKernelGGL((k_sub_gemm<float, 2, 2, 1, 2, 32, true>), grid, block, 0, s, nullptr,
                         nullptr, 0, cls, tiles, 0, ptrs);
  } else {
    if (small)
      hipLaunchKernelGGL((k_sub_gemm<double, 1, 4, 1, 1, 16, true>), grid, block, 0, s, nullptr,
                         nullptr, 0, cls, tiles, 0, ptrs);
    else
      hipLaunchKernelGGL((k_sub_gemm<double, 2, 2, 1, 2, 16, true>), grid, block, 0, s, nullptr,
                         nullptr, 0, cls, tiles, 0, ptrs);
  }
  return hipGetLastError();
}

template <typename T, int PARTS>
void scatter_launch(unsigned blocks, hipStream_t s, double* u, const void* du, long long pstride,
                    const double* weights, const PullEntry* pull, int N, int nov, long long total,
                    int assign) {
  hipLaunchKernelGGL((k_scatter<T, PARTS>), dim3(blocks), dim3(256), 0, s, u, (const T*)du, pstride,
                     weights, pull, N, nov, total, assign);
}

template <typename T>
hipError_t scatter_parts(int parts, unsigned blocks, hipStream_t s, double* u, const void* du,
                         long long pstride, const double* weights, const PullEntry* pull, int N,
                         int nov, long long total, int assign) {
  switch (parts) {
    case 1: scatter_launch<T, 1>(blocks, s, u, du, pstride, weights, pull, N, nov, total, assign); break;
    case 2: scatter_launch<T, 2>(blocks, s, u, du, pstride, weights, pull, N, nov, total, assign); break;
    case 3: scatter_launch<T, 3>(blocks, s, u, du, pstride, weights, pull, N, nov, total, assign); break;
    case 4: scatter_launch<T, 4>(blocks, s, u, du, pstride, weights, pull, N, nov, total, assign); break;
    case 8: scatter_launch<T, 8>(blocks, s, u, du, pstride, weights, pull, N, nov, total, assign); break;
    case 16: scatter_launch<T, 16>(blocks, s, u, du, pstride, weights, pull, N, nov, total, assign); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_scatter(int N, bool f32, double* u, const void* du, int parts,
                          long long pstride, const double* weights, const PullEntry* pull, int nov,
                          long long E, hipStream_t s, bool assign) {
  const long long total = E * N * N * N;
  if (total <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((total + 255) / 256);
  const int as = assign ? 1 : 0;
  return f32 ? scatter_parts<float>(parts, blocks, s, u, du, pstride, weights, pull, N, nov, total, as)
             : scatter_parts<double>(parts, blocks, s, u, du, pstride, weights, pull, N, nov, total,
                                     as);
}

}  // namespace dgs
