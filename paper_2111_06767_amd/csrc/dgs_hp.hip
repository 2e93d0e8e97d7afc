// Kernels of the hp-nonuniform path (Sec. II with mortars on nonconforming
// faces, Sec. III.C.1-2 transfers, Sec. III.D Schwarz gather and scatter).
//
// Operator: one workgroup per element, one thread per node (loops for more
// nodes than threads).  The element's values and its three unlifted
// derivatives sit in LDS.  Every face is a list of terms: a box-boundary term
// (the ghost state of eq. bc on the element's own face points), a conforming
// neighbour of equal points (the flux point by point), or a mortar shared
// with one neighbour, whose corrections reach the element's face points
// through the premultiplied interpolation-and-projection matrices.  The lift
// (eq. liftop) and the strong-form primal equation (eq. dg_op_primal) follow
// as on the uniform grid.
#include "dgs_hp.h"

namespace dgs {
namespace {

constexpr int kHpThreads = 256;
constexpr int kNodesPerThread = kHpMaxNodes / kHpThreads;
constexpr int kF = kHpMaxN * kHpMaxN;  // points of a face or mortar
static_assert(kF <= 64, "a face's points fit one wavefront");
// wavefronts that take mortar faces side by side (LDS: 3 KB each)
constexpr int kMortarWaves = 3;
static_assert(kMortarWaves <= kHpThreads / 64, "one wavefront per mortar face");

// Orders the LDS accesses of one wavefront: its lanes exchange data through
// LDS between the passes of a mortar term, with no other wave involved.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Select one of three values by a dimension index without a runtime-indexed
// private array (those go to scratch memory).
__device__ __forceinline__ int pick(int d, int a, int b, int c) { return d == 0 ? a : (d == 1 ? b : c); }
__device__ __forceinline__ double pick(int d, double a, double b, double c) {
  return d == 0 ? a : (d == 1 ? b : c);
}

// Node of an element with N0 x N1 (x N2) points at position od along d and
// (b0, b1) along the transverse dimensions t0 < t1.
__device__ __forceinline__ int face_node(int d, int od, int b0, int b1, int N0, int N1) {
  const int i = d == 0 ? od : b0;
  const int j = d == 0 ? b0 : (d == 1 ? od : b1);
  const int k = d == 2 ? od : b1;
  return (k * N1 + j) * N0 + i;
}

// PUSH (residual mode on a mesh): instead of out, every point's residual is
// written into the Schwarz subdomain rows that hold it (push_ptr / push_pos
// list the row positions of each point; rows in FP32 with rs_f32), the
// gather fused into the residual.
template <bool RES, bool PUSH = false>
__global__ void __launch_bounds__(kHpThreads)
    k_hp_apply(const double* __restrict__ u, double* __restrict__ out, const double* __restrict__ b,
               const HpElem* __restrict__ el, const HpTerm* __restrict__ terms,
               const double* __restrict__ pool, HpRule R, long long copy_stride,
               const int* __restrict__ order, const long long* __restrict__ push_ptr = nullptr,
               const long long* __restrict__ push_pos = nullptr, void* __restrict__ rs = nullptr,
               int rs_f32 = 0) {
  __shared__ double su[kHpMaxNodes];
  __shared__ double sg[3][kHpMaxNodes];
  __shared__ double scu[6][kF], scp[6][kF];
  __shared__ double wb[kMortarWaves][6][kF];  // per-wave mortar buffers
  const HpElem E = el[order ? order[blockIdx.x] : (int)blockIdx.x];
  const long long cbase = (long long)blockIdx.y * copy_stride;
  const long long base = cbase + E.off;
  const int N0 = E.N[0], N1 = E.N[1], N2 = E.N[2];
  const int n = N0 * N1 * N2;
  const int tid = threadIdx.x;
  // this thread's nodes (at most kNodesPerThread) and their indices
  int ni[kNodesPerThread], nj[kNodesPerThread], nk[kNodesPerThread];
#pragma unroll
  for (int r = 0; r < kNodesPerThread; ++r) {
    const int p = tid + r * kHpThreads;
    ni[r] = p % N0;
    nj[r] = (p / N0) % N1;
    nk[r] = p / (N0 * N1);
    if (p < n) su[p] = u[base + p];
  }
  __syncthreads();
  // unlifted derivatives D_d u = (2/h_d) D_xi u
#pragma unroll
  for (int r = 0; r < kNodesPerThread; ++r) {
    const int p = tid + r * kHpThreads;
    if (p >= n) continue;
    const int i = ni[r], j = nj[r], k = nk[r];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int Nd = pick(d, N0, N1, N2), id = pick(d, i, j, k), st = pick(d, 1, N0, N0 * N1);
      const double* D = R.D + (Nd - 2) * 64 + id * Nd;
      const int l0 = p - id * st;
      double acc = 0.0;
      for (int m = 0; m < Nd; ++m) acc += D[m] * su[l0 + m * st];
      sg[d][p] = E.rh[d] * acc;
    }
  }
  __syncthreads();
  // pass 1, without barriers: box faces and conforming faces of equal points
  // (a single term each), point by point from the ghost state (eq. bc) or the
  // neighbour's trace and normal derivative at the matching point; the points
  // of all such faces are spread over the workgroup together, so the
  // neighbours' loads are in flight at once
  int nd[6];  // points of each face handled here (0: a mortar face)
  bool any_mortar = false;
  {
    int t = E.term0;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1;
      const bool direct = terms[t].direct;
      nd[f] = direct ? pick(d, N1, N0, N0) * pick(d, N2, N2, N1) : 0;
      any_mortar = any_mortar || !direct;
      t += E.nterm[f];
    }
  }
  const int ndirect = nd[0] + nd[1] + nd[2] + nd[3] + nd[4] + nd[5];
  for (int g = tid; g < ndirect; g += blockDim.x) {
    int f = 0, q = g, t = E.term0;
#pragma unroll
    for (int k = 0; k < 6; ++k)
      if (f == k && q >= nd[k]) {
        q -= nd[k];
        t += E.nterm[k];
        f = k + 1;
      }
    const HpTerm T = terms[t];
    const int d = f >> 1;
    const double sgn = (f & 1) ? 1.0 : -1.0;
    const int n0 = d == 0 ? N1 : N0;
    const int b0 = q % n0, b1 = q / n0;
    const int Nd = pick(d, N0, N1, N2);
    const int p = face_node(d, (f & 1) ? Nd - 1 : 0, b0, b1, N0, N1);
    const double ui = su[p], dui = sg[d][p];
    double ue, due;
    if (T.nb >= 0) {
      const int FN = pick(d, T.fN[0], T.fN[1], T.fN[2]);
      const int fod = (f & 1) ? 0 : FN - 1;
      const double* D = R.D + (FN - 2) * 64 + fod * FN;
      const int strd = pick(d, 1, T.fN[0], T.fN[0] * T.fN[1]);
      const double* line = u + cbase + T.foff + face_node(d, 0, b0, b1, T.fN[0], T.fN[1]);
      double acc = 0.0;
      for (int m = 0; m < FN; ++m) acc += D[m] * line[m * strd];
      ue = line[fod * strd];
      due = T.frh * acc;
    } else if (T.nb == kHpZero) {  // a zero neighbour (set-up patches)
      ue = 0.0;
      due = 0.0;
    } else {
      const bool dir = T.nb == kHpDirichlet;
      ue = dir ? -ui : ui;
      due = dir ? dui : -dui;
    }
    scu[f][q] = 0.5 * (ue - ui);
    scp[f][q] = 0.5 * sgn * (dui + due) - T.sigma * (ui - ue);
  }
  // pass 2: mortars of nonconforming faces.  The terms of one face are taken
  // in sequence by one wavefront (a face writes only its own corrections), so
  // up to kMortarWaves faces proceed side by side; within the wave every lane
  // holds one face point (at most kF).  Per term, the premultiplied matrices
  // A = P I_own and B = P I_nb (read from the pool) carry the element's and
  // the neighbour's face data through the mortar and back to the element's
  // face points; the fluxes of eq. numflux combine them there.
  if (any_mortar) {
    const int wave = tid >> 6, q = tid & 63;
    int c = 0, t = E.term0;
#pragma unroll 1
    for (int f = 0; f < 6; ++f) {
      const int ntf = f < 3 ? pick(f, E.nterm[0], E.nterm[1], E.nterm[2])
                            : pick(f - 3, E.nterm[3], E.nterm[4], E.nterm[5]);
      const int tf = t;
      t += ntf;
      if (terms[tf].direct) continue;
      const bool mine = (c % kMortarWaves) == wave;
      ++c;
      if (!mine) continue;
      double* oa = wb[wave][0];
      double* ob = wb[wave][1];
      double* ma = wb[wave][2];
      double* mb = wb[wave][3];
      double* na = wb[wave][4];
      double* nbv = wb[wave][5];
      const int d = f >> 1;
      const double sgn = (f & 1) ? 1.0 : -1.0;
      const int n0 = d == 0 ? N1 : N0, n1 = d == 2 ? N1 : N2;
      const int Nd = pick(d, N0, N1, N2);
      const int od = (f & 1) ? Nd - 1 : 0;
      const bool qon = q < n0 * n1;
      const int qi = q % n0, qj = q / n0;
      double cu = 0.0, cp = 0.0;
      for (int k = 0; k < ntf; ++k) {
        const HpTerm T = terms[tf + k];
        int m0 = 0, m1 = 0, FN = 2, FN0 = 1, FN1 = 1;
        long long foff = 0;
        double frh = 0.0;
        if (T.nb >= 0) {
          m0 = d == 0 ? T.fN[1] : T.fN[0];
          m1 = d == 2 ? T.fN[1] : T.fN[2];
          FN = pick(d, T.fN[0], T.fN[1], T.fN[2]);
          FN0 = T.fN[0];
          FN1 = T.fN[1];
          foff = T.foff;
          frh = T.frh;
          // the neighbour's trace and normal derivative on its own face points
          if (q < m0 * m1) {
            const int fod = (f & 1) ? 0 : FN - 1;
            const double* D = R.D + (FN - 2) * 64 + fod * FN;
            const int strd = pick(d, 1, FN0, FN0 * FN1);
            const double* line = u + cbase + foff + face_node(d, 0, q % m0, q / m0, FN0, FN1);
            double acc = 0.0;
            for (int m = 0; m < FN; ++m) acc += D[m] * line[m * strd];
            oa[q] = line[fod * strd];
            ob[q] = frh * acc;
          }
        }
        wave_sync();
        const double* A0 = T.A0 >= 0 ? pool + T.A0 : nullptr;
        const double* A1 = T.A1 >= 0 ? pool + T.A1 : nullptr;
        const double* B0 = T.B0 >= 0 ? pool + T.B0 : nullptr;
        const double* B1 = T.B1 >= 0 ? pool + T.B1 : nullptr;
        // along t0: own data [n1][n0] -> [n1][n0] (read from the element's
        // trace and derivative in place), neighbour data [m1][m0] -> [m1][n0]
        if (qon) {
          double a = 0.0, cc = 0.0;
          if (A0) {
            for (int m = 0; m < n0; ++m) {
              const double w = A0[qi * n0 + m];
              const int p = face_node(d, od, m, qj, N0, N1);
              a += w * su[p];
              cc += w * sg[d][p];
            }
          } else {
            const int p = face_node(d, od, qi, qj, N0, N1);
            a = su[p];
            cc = sg[d][p];
          }
          ma[q] = a;
          mb[q] = cc;
        }
        if (T.nb >= 0 && q < m1 * n0) {
          const int j = q / n0, i = q - j * n0;
          double a = 0.0, cc = 0.0;
          if (B0) {
            for (int m = 0; m < m0; ++m) {
              const double w = B0[i * m0 + m];
              a += w * oa[j * m0 + m];
              cc += w * ob[j * m0 + m];
            }
          } else {
            a = oa[j * m0 + i];
            cc = ob[j * m0 + i];
          }
          na[q] = a;
          nbv[q] = cc;
        }
        wave_sync();
        // along t1, then the fluxes (a zero neighbour contributes nothing)
        if (qon) {
          double hu = 0.0, hd = 0.0, gu = 0.0, gd = 0.0;
          if (A1) {
            for (int m = 0; m < n1; ++m) {
              const double w = A1[qj * n1 + m];
              hu += w * ma[m * n0 + qi];
              hd += w * mb[m * n0 + qi];
            }
          } else {
            hu = ma[q];
            hd = mb[q];
          }
          if (T.nb >= 0) {
            if (B1) {
              for (int m = 0; m < m1; ++m) {
                const double w = B1[qj * m1 + m];
                gu += w * na[m * n0 + qi];
                gd += w * nbv[m * n0 + qi];
              }
            } else {
              gu = na[q];
              gd = nbv[q];
            }
          }
          cu += 0.5 * (gu - hu);
          cp += 0.5 * sgn * (hd + gd) - T.sigma * (hu - gu);
        }
        wave_sync();  // the next term overwrites this wave's buffers
      }
      if (qon) {
        scu[f][q] = cu;
        scp[f][q] = cp;
      }
    }
  }
  __syncthreads();
  // auxiliary variable (eq. dg_op_auxvars): v_d = D_d u + M^-1 ML n_d cu on
  // the faces normal to d, M^-1 ML = (2/h_d) / w_end
#pragma unroll
  for (int r = 0; r < kNodesPerThread; ++r) {
    const int p = tid + r * kHpThreads;
    if (p >= n) continue;
    const int i = ni[r], j = nj[r], k = nk[r];
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1;
      const int Nd = pick(d, N0, N1, N2), id = pick(d, i, j, k);
      if (id != ((f & 1) ? Nd - 1 : 0)) continue;
      const int q = d == 0 ? k * N1 + j : (d == 1 ? k * N0 + i : j * N0 + i);
      const double lift = E.rh[d] / R.w[(Nd - 2) * 8];
      sg[d][p] += lift * ((f & 1) ? 1.0 : -1.0) * scu[f][q];
    }
  }
  __syncthreads();
  // primal equation (eq. dg_op_primal): -M D_d v_d - ML ((n F_u)* - n_d v_d)
#pragma unroll
  for (int r = 0; r < kNodesPerThread; ++r) {
    const int p = tid + r * kHpThreads;
    if (p >= n) continue;
    const int i = ni[r], j = nj[r], k = nk[r];
    double acc = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int Nd = pick(d, N0, N1, N2), id = pick(d, i, j, k), st = pick(d, 1, N0, N0 * N1);
      const double* D = R.D + (Nd - 2) * 64 + id * Nd;
      const int l0 = p - id * st;
      double a = 0.0;
      for (int m = 0; m < Nd; ++m) a += D[m] * sg[d][l0 + m * st];
      acc += E.rh[d] * a;
    }
    const double wx = R.w[(N0 - 2) * 8 + i], wy = R.w[(N1 - 2) * 8 + j], wz = R.w[(N2 - 2) * 8 + k];
    double Au = -E.jac * wx * wy * wz * acc;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1;
      const int Nd = pick(d, N0, N1, N2), id = pick(d, i, j, k);
      if (id != ((f & 1) ? Nd - 1 : 0)) continue;
      const int q = d == 0 ? k * N1 + j : (d == 1 ? k * N0 + i : j * N0 + i);
      const double wt = d == 0 ? wy * wz : (d == 1 ? wx * wz : wx * wy);
      const double ML = E.jac * E.rh[d] * wt;
      Au -= ML * (scp[f][q] - ((f & 1) ? 1.0 : -1.0) * sg[d][p]);
    }
    const double val = RES ? b[base + p] - Au : Au;
    if constexpr (PUSH) {
      const long long g = base + p;
      const long long q1 = push_ptr[g + 1];
      for (long long q = push_ptr[g]; q < q1; ++q) {
        if (rs_f32)
          static_cast<float*>(rs)[push_pos[q]] = (float)val;
        else
          static_cast<double*>(rs)[push_pos[q]] = val;
      }
    } else {
      out[base + p] = val;
    }
  }
}

__global__ void k_hp_mass(const double* __restrict__ f, double* __restrict__ out,
                          const HpElem* __restrict__ el, HpRule R) {
  const HpElem E = el[blockIdx.x];
  const int N0 = E.N[0], N1 = E.N[1], N2 = E.N[2];
  for (int p = threadIdx.x; p < N0 * N1 * N2; p += blockDim.x) {
    const int i = p % N0, j = (p / N0) % N1, k = p / (N0 * N1);
    const double M = E.jac * R.w[(N0 - 2) * 8 + i] * R.w[(N1 - 2) * 8 + j] * R.w[(N2 - 2) * 8 + k];
    out[E.off + p] = M * f[E.off + p];
  }
}

__global__ void k_hp_coords(double* __restrict__ xyz, long long ndof, const HpElem* __restrict__ el,
                            const double* __restrict__ plo_h, HpRule R) {
  const HpElem E = el[blockIdx.x];
  const double* g = plo_h + 6 * (long long)blockIdx.x;
  const int N0 = E.N[0], N1 = E.N[1], N2 = E.N[2];
  for (int p = threadIdx.x; p < N0 * N1 * N2; p += blockDim.x) {
    const int idx[3] = {p % N0, (p / N0) % N1, p / (N0 * N1)};
    for (int d = 0; d < 3; ++d)
      xyz[d * ndof + E.off + p] = g[d] + g[3 + d] * 0.5 * (R.xi[(E.N[d] - 2) * 8 + idx[d]] + 1.0);
  }
}

template <typename TS>
__global__ void k_hp_gather(const double* __restrict__ r, TS* __restrict__ rs,
                            const HpSub* __restrict__ subs, const long long* __restrict__ gidx) {
  const HpSub S = subs[blockIdx.x];
  for (int q = threadIdx.x; q < S.n; q += blockDim.x) rs[S.rs + q] = (TS)r[gidx[S.start + q]];
}

template <typename TS>
__global__ void k_hp_scatter(double* __restrict__ u, const TS* __restrict__ du, int parts,
                             long long stride, const long long* __restrict__ ptr,
                             const HpPull* __restrict__ pull, long long ndof) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ndof) return;
  // entries four at a time, their loads issued together (the chain of
  // dependent loads, not the bytes, bounds this kernel)
  double acc = 0.0;
  const long long q1 = ptr[p + 1];
  for (long long q0 = ptr[p]; q0 < q1; q0 += 4) {
    HpPull e[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) e[k] = q0 + k < q1 ? pull[q0 + k] : HpPull{0, 0.0};
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int part = 0; part < parts; ++part)
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] += (double)du[part * stride + e[k].pos];
#pragma unroll
    for (int k = 0; k < 4; ++k) acc += e[k].w * v[k];
  }
  u[p] += acc;
}

// One 1D pass of a tensor-product transfer in LDS: out = (A along dimension
// d) in, with A row-major R x C and `in` of extents n[3] (n[d] = C before,
// R after).  trans: use A^T (C x R view) instead.
__device__ void pass1d(const double* A, int Rr, int Cc, bool trans, int d, const int nin[3],
                       const double* in, double* outv) {
  int nout[3] = {nin[0], nin[1], nin[2]};
  nout[d] = trans ? Cc : Rr;
  const int total = nout[0] * nout[1] * nout[2];
  for (int q = threadIdx.x; q < total; q += blockDim.x) {
    int idx[3] = {q % nout[0], (q / nout[0]) % nout[1], q / (nout[0] * nout[1])};
    const int o = idx[d];
    double acc = 0.0;
    const int K = nin[d];
    for (int m = 0; m < K; ++m) {
      idx[d] = m;
      const double a = trans ? A[m * Cc + o] : A[o * Cc + m];
      acc += a * in[(idx[2] * nin[1] + idx[1]) * nin[0] + idx[0]];
    }
    outv[q] = acc;
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kHpThreads)
    k_hp_prolongate_add(const double* __restrict__ coarse, double* __restrict__ fine,
                        const HpElem* __restrict__ fel, const HpElem* __restrict__ cel,
                        const HpChild* __restrict__ ch, const double* __restrict__ pool) {
  __shared__ double s0[kHpMaxNodes], s1[kHpMaxNodes];
  const HpChild C = ch[blockIdx.x];
  const HpElem F = fel[blockIdx.x], P = cel[C.parent];
  const int nc = P.N[0] * P.N[1] * P.N[2];
  for (int p = threadIdx.x; p < nc; p += blockDim.x) s0[p] = coarse[P.off + p];
  __syncthreads();
  int n[3] = {P.N[0], P.N[1], P.N[2]};
  pass1d(pool + C.P[0], F.N[0], P.N[0], false, 0, n, s0, s1);
  n[0] = F.N[0];
  pass1d(pool + C.P[1], F.N[1], P.N[1], false, 1, n, s1, s0);
  n[1] = F.N[1];
  pass1d(pool + C.P[2], F.N[2], P.N[2], false, 2, n, s0, s1);
  for (int p = threadIdx.x; p < F.N[0] * F.N[1] * F.N[2]; p += blockDim.x) fine[F.off + p] += s1[p];
}

__global__ void __launch_bounds__(kHpThreads)
    k_hp_restrict(const double* __restrict__ fine, double* __restrict__ coarse,
                  const HpElem* __restrict__ fel, const HpElem* __restrict__ cel,
                  const HpChild* __restrict__ ch, const int* __restrict__ kid_ptr,
                  const int* __restrict__ kids, const double* __restrict__ pool) {
  __shared__ double s0[kHpMaxNodes], s1[kHpMaxNodes], acc[kHpMaxNodes];
  const HpElem P = cel[blockIdx.x];
  const int nc = P.N[0] * P.N[1] * P.N[2];
  for (int p = threadIdx.x; p < nc; p += blockDim.x) acc[p] = 0.0;
  for (int k = kid_ptr[blockIdx.x]; k < kid_ptr[blockIdx.x + 1]; ++k) {
    const int e = kids[k];
    const HpElem F = fel[e];
    const HpChild C = ch[e];
    __syncthreads();
    for (int p = threadIdx.x; p < F.N[0] * F.N[1] * F.N[2]; p += blockDim.x) s0[p] = fine[F.off + p];
    __syncthreads();
    int n[3] = {F.N[0], F.N[1], F.N[2]};
    pass1d(pool + C.P[0], F.N[0], P.N[0], true, 0, n, s0, s1);
    n[0] = P.N[0];
    pass1d(pool + C.P[1], F.N[1], P.N[1], true, 1, n, s1, s0);
    n[1] = P.N[1];
    pass1d(pool + C.P[2], F.N[2], P.N[2], true, 2, n, s0, s1);
    for (int p = threadIdx.x; p < nc; p += blockDim.x) acc[p] += s1[p];
  }
  __syncthreads();
  for (int p = threadIdx.x; p < nc; p += blockDim.x) coarse[P.off + p] = acc[p];
}

unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_hp_apply(bool residual, const double* u, double* out, const double* b,
                           const HpElem* el, int E, const HpTerm* terms, const double* pool,
                           const HpRule& R, int copies, long long copy_stride, hipStream_t s,
                           const int* order) {
  if (E <= 0 || copies <= 0) return hipSuccess;
  const dim3 grid((unsigned)E, (unsigned)copies);
  if (residual)
    hipLaunchKernelGGL(k_hp_apply<true>, grid, dim3(kHpThreads), 0, s, u, out, b, el, terms, pool, R,
                       copy_stride, order);
  else
    hipLaunchKernelGGL(k_hp_apply<false>, grid, dim3(kHpThreads), 0, s, u, out, b, el, terms, pool, R,
                       copy_stride, order);
  return hipGetLastError();
}

hipError_t launch_hp_residual_gather(const double* u, const double* b, const HpElem* el, int E,
                                     const HpTerm* terms, const double* pool, const HpRule& R,
                                     const int* order, const long long* push_ptr,
                                     const long long* push_pos, bool f32, void* rs, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_hp_apply<true, true>), dim3((unsigned)E), dim3(kHpThreads), 0, s, u, nullptr, b,
                     el, terms, pool, R, 0LL, order, push_ptr, push_pos, rs, f32 ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_hp_mass(const double* f, double* out, const HpElem* el, int E, const HpRule& R,
                          hipStream_t s) {
  if (E <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hp_mass, dim3((unsigned)E), dim3(kHpThreads), 0, s, f, out, el, R);
  return hipGetLastError();
}

hipError_t launch_hp_coords(double* xyz, long long ndof, const HpElem* el, const double* plo_h,
                            int E, const HpRule& R, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hp_coords, dim3((unsigned)E), dim3(kHpThreads), 0, s, xyz, ndof, el, plo_h, R);
  return hipGetLastError();
}

hipError_t launch_hp_gather(bool f32, const double* r, void* rs, const HpSub* subs, int nsub,
                            const long long* gidx, hipStream_t s) {
  if (nsub <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_hp_gather<float>, dim3((unsigned)nsub), dim3(256), 0, s, r, (float*)rs, subs, gidx);
  else
    hipLaunchKernelGGL(k_hp_gather<double>, dim3((unsigned)nsub), dim3(256), 0, s, r, (double*)rs, subs,
                       gidx);
  return hipGetLastError();
}

hipError_t launch_hp_scatter(bool f32, double* u, const void* du, int parts, long long part_stride,
                             const long long* ptr, const HpPull* pull, long long ndof,
                             hipStream_t s) {
  if (ndof <= 0) return hipSuccess;
  if (f32)
    hipLaunchKernelGGL(k_hp_scatter<float>, dim3(nblk(ndof)), dim3(256), 0, s, u, (const float*)du, parts,
                       part_stride, ptr, pull, ndof);
  else
    hipLaunchKernelGGL(k_hp_scatter<double>, dim3(nblk(ndof)), dim3(256), 0, s, u, (const double*)du,
                       parts, part_stride, ptr, pull, ndof);
  return hipGetLastError();
}

hipError_t launch_hp_prolongate_add(const double* coarse, double* fine, const HpElem* fel,
                                    const HpElem* cel, const HpChild* ch, int Ef,
                                    const double* pool, hipStream_t s) {
  if (Ef <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hp_prolongate_add, dim3((unsigned)Ef), dim3(kHpThreads), 0, s, coarse, fine,
                     fel, cel, ch, pool);
  return hipGetLastError();
}

hipError_t launch_hp_restrict(const double* fine, double* coarse, const HpElem* fel,
                              const HpElem* cel, const HpChild* ch, const int* kid_ptr,
                              const int* kids, int Ec, const double* pool, hipStream_t s) {
  if (Ec <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_hp_restrict, dim3((unsigned)Ec), dim3(kHpThreads), 0, s, fine, coarse, fel,
                     cel, ch, kid_ptr, kids, pool);
  return hipGetLastError();
}

}  // namespace dgs
