// DG operator apply on gfx950 (Sec. II, eqs. dg_op_auxvars, dg_op_primal,
// massmat, stiffmat, liftop, numflux, penalty, bc).
//
// One kernel computes A u for a batch of elements with line-based sum
// factorisation.  Each element is handled by N^2 lanes; lane t = a + N b
// plays three roles: it owns the x-line (j, k) = (a, b), the y-line
// (i, k) = (a, b) and the z-line (i, j) = (a, b).  The z-line lives in
// registers; x- and y-lines are read from one LDS copy of the element.  Each
// role applies the 1D derivative to its whole line, adds the lift and the
// numerical flux at the line's two face points (the neighbour's trace and its
// own normal derivative come from the neighbour's line, read straight from
// global memory), and applies the transposed derivative.  The three partial
// results meet in LDS.  The derivative matrix entries are compile-time
// indexed, so they are uniform across the wave (scalar loads), and every LDS
// access is one read or write per point.  The whole apply is one pass: read u,
// write A u.
//
// With LGL quadrature the strong form is evaluated through summation by parts,
//   -M D_d v_d + ML_d n_d v_d = D_d^T M v_d      (exact for LGL points),
// so that
//   A u = sum_d D_d^T (M v_d) - sum_faces ML_f (n F_u)*,
//   v_d = D_d u + L_d (1/2) n_d (u_ext - u_int)  on the faces normal to d,
//   (n F_u)* = 1/2 n.(grad u_int + grad u_ext) - sigma (u_int - u_ext).
// Dirichlet faces use the ghost state u_ext = -u_int, grad u_ext = grad u_int;
// homogeneous Neumann faces (P.neumann) u_ext = u_int and the normal
// derivative negated, so that no flux crosses them.
#include "dgs_internal.h"
#include "dgs_elem.h"

namespace dgs {
namespace {

// MODE is an ApplyMode; GO = 0 writes out, GO = 1 / 2 writes r_S into FP32 /
// FP64 subdomain rows (residual modes only).  Each combination is compiled
// separately so that it carries only its own loads, stores and registers.
//
// BR = true (N = 8): a workgroup takes a 2 x 2 x 2 brick of elements of a box grid
// (EPB = 8, slot s at offset (s & 1, (s >> 1) & 1, s >> 2) in the brick;
// order[] lists the bricks).  Each element then has one face neighbour per
// direction inside the brick, whose lines are read from that element's LDS
// copy, and only the three outside neighbours come from global memory: four
// element reads per element instead of seven.
template <int N, int EPB, int MODE, int GO, bool BR, bool NT = false>
__global__ void __launch_bounds__(((EPB * N * N + 63) / 64) * 64)
k_apply(const double* __restrict__ u, double* __restrict__ out, const double* __restrict__ bvec,
        const double* __restrict__ aux0, const double* __restrict__ aux1,
        const int* __restrict__ nbr, OpParams P, DevTables T,
        const int* __restrict__ order, GatherOut go, double* __restrict__ ucopy) {
  static_assert(GO == 0 || MODE == kResidual || MODE == kResidualDiag, "gather-out mode");
  static_assert(!BR || EPB == 8, "a brick holds 8 elements");
  constexpr int N2 = N * N, N3 = N2 * N;
  constexpr int PIT = N + 1;  // padded row pitch (bank spread for line reads)
  constexpr int S3 = N * N * PIT;
  // sU: the element (its x- and y-lines for the forward phase); after the
  // forward phase sA and sU take the transposed x and y contributions
  __shared__ double sU[EPB][S3], sA[EPB][S3];
  __shared__ double sw[N];
  __shared__ PullEntry sPull[GO ? EPB : 1][7];  // gather-out only

  const int tid = threadIdx.x;
  if (tid < N) sw[tid] = T.w[tid];
  // with N^2 = 64 a slot is one wavefront: say so, so that everything derived
  // from the element index stays in scalar registers
  const int slot = (N2 % 64 == 0) ? __builtin_amdgcn_readfirstlane(tid / N2) : tid / N2;
  const int t = tid - slot * N2;
  const int a = t % N, b = t / N;
  // XCD-aware block order: the hardware deals workgroups round-robin to the
  // 8 XCDs, so hand each XCD a contiguous run of elements (neighbours then
  // share that XCD's L2).
  const unsigned G = gridDim.x, per = G / 8u;
  const unsigned blk = (blockIdx.x % 8u) * per + blockIdx.x / 8u;
  // element of slot s of this block, -1 for none; with one element per
  // block it is derived from blockIdx alone (uniform across the wave)
  auto element_of = [&](int s) -> long long {
    if constexpr (BR) {
      const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
      const int nbx = (nx + 1) >> 1, nby = (ny + 1) >> 1, nbz = (nz + 1) >> 1;
      if (blk >= (unsigned)(nbx * nby * nbz)) return -1;
      const int bl = order[blk];
      const int bx = bl % nbx, by = (bl / nbx) % nby, bz = bl / (nbx * nby);
      const int ex = 2 * bx + (s & 1), ey = 2 * by + ((s >> 1) & 1), ez = 2 * bz + (s >> 2);
      if (ex >= nx || ey >= ny || ez >= nz) return -1;
      return ((long long)ez * ny + ey) * nx + ex;
    } else {
      const long long ps = EPB == 1 ? (long long)blk : (long long)blk * EPB + s;
      if (ps >= P.E) return -1;
      return order ? (long long)order[ps] : ps;
    }
  };
  const long long e0 = slot < EPB ? element_of(EPB == 1 ? 0 : slot) : -1;
  const bool active = e0 >= 0;
  const long long e = active ? e0 : 0;
  const double J = P.J;
  auto L = [](int k, int j, int i) { return (k * N + j) * PIT + i; };
  if constexpr (GO != 0) {
    for (int q = tid; q < EPB * 7; q += blockDim.x) {
      const int s7 = q / 7, j7 = q - s7 * 7;
      const long long es = element_of(s7);
      if (es >= 0) sPull[s7][j7] = go.pull[es * 7 + j7];
    }
  }

  // uz: the lane's z-line; xf / yf / zf: trace and normal derivative of the
  // x / y / z neighbours on the shared faces (index side * 2 + {trace, derivative}),
  // reduced from their lines as soon as they arrive so the lines do not stay
  // in registers through the forward phase
  double uz[N], xf[4], yf[4], zf[4];
  int nb[6];
  if (active) {
    const double* ue = u + e * N3;
    if (P.n[0] > 0) {  // box grid: no table lookup on the critical path
      const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
      const int ie = (int)e, ex = ie % nx, ey = (ie / nx) % ny, ez = ie / (nx * ny);
      nb[0] = ex > 0 ? ie - 1 : -1;
      nb[1] = ex < nx - 1 ? ie + 1 : -1;
      nb[2] = ey > 0 ? ie - nx : -1;
      nb[3] = ey < ny - 1 ? ie + nx : -1;
      nb[4] = ez > 0 ? ie - nx * ny : -1;
      nb[5] = ez < nz - 1 ? ie + nx * ny : -1;
    } else {
#pragma unroll
      for (int f = 0; f < 6; ++f) nb[f] = nbr[e * 6 + f];
    }
#pragma unroll
    for (int k = 0; k < N; ++k) {
      uz[k] = ue[k * N2 + t];
      sU[slot][L(k, b, a)] = uz[k];
    }
    // every neighbour line this lane reads from global memory, issued before
    // the first barrier (a missing neighbour reads the element itself; its
    // result is replaced by the Dirichlet ghost state)
    auto nbi = [&](int f) -> long long { return nb[f] >= 0 ? (long long)nb[f] : e; };
    if constexpr (BR) {
      // the neighbour on side o_d of direction d is outside the brick
      const int ox = slot & 1, oy = (slot >> 1) & 1, oz = slot >> 2;
      const long long xo = nbi(ox), yo = nbi(2 + oy), zo = nbi(4 + oz);
      double xl[N], yl[N], zl[N];
#pragma unroll
      for (int m = 0; m < N; ++m) {
        xl[m] = u[xo * N3 + b * N2 + a * N + m];
        yl[m] = u[yo * N3 + b * N2 + m * N + a];
        zl[m] = u[zo * N3 + m * N2 + t];
      }
      // parked in the high / low pair of the outside side; the inside side
      // is filled after the barrier
      face_from_line<N>(xl, ox, P.rh[0], T, xf[0], xf[1]);
      face_from_line<N>(yl, oy, P.rh[1], T, yf[0], yf[1]);
      face_from_line<N>(zl, oz, P.rh[2], T, zf[0], zf[1]);
    } else {
      const long long xl0 = nbi(0), xh0 = nbi(1), yl = nbi(2), yh = nbi(3), zl = nbi(4),
                      zh = nbi(5);
      double xlo[N], xhi[N], ylo[N], yhi[N], zlo[N], zhi[N];
#pragma unroll
      for (int m = 0; m < N; ++m) {  // x-lines: N contiguous values per lane
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
  } else if (BR && slot < EPB) {
    // an empty brick slot: defined values for its neighbours' reads (they
    // are discarded, the face is a domain boundary)
#pragma unroll
    for (int k = 0; k < N; ++k) sU[slot][L(k, b, a)] = 0.0;
  }
  __syncthreads();
  if constexpr (BR) {
    if (active) {  // the inside neighbours' lines, from their LDS copies
      const int ox = slot & 1, oy = (slot >> 1) & 1, oz = slot >> 2;
      double xl[N], yl[N], zl[N];
#pragma unroll
      for (int m = 0; m < N; ++m) {
        xl[m] = sU[slot ^ 1][L(b, a, m)];
        yl[m] = sU[slot ^ 2][L(b, m, a)];
        zl[m] = sU[slot ^ 4][L(m, b, a)];
      }
      double xu, xg, yu, yg, zu, zg;
      face_from_line<N>(xl, 1 - ox, P.rh[0], T, xu, xg);
      face_from_line<N>(yl, 1 - oy, P.rh[1], T, yu, yg);
      face_from_line<N>(zl, 1 - oz, P.rh[2], T, zu, zg);
      // low side outside (o_d = 0): outside pair low, inside pair high
      xf[2] = ox ? xf[0] : xu;
      xf[3] = ox ? xf[1] : xg;
      xf[0] = ox ? xu : xf[0];
      xf[1] = ox ? xg : xf[1];
      yf[2] = oy ? yf[0] : yu;
      yf[3] = oy ? yf[1] : yg;
      yf[0] = oy ? yu : yf[0];
      yf[1] = oy ? yg : yf[1];
      zf[2] = oz ? zf[0] : zu;
      zf[3] = oz ? zf[1] : zg;
      zf[0] = oz ? zu : zf[0];
      zf[1] = oz ? zg : zf[1];
    }
  }

  // forward phase: q_d = M (grad_d u + lift) on every line, flux at line
  // ends, each role followed as early as possible by its transposed product
  // D_d^T q_d: the x role's goes straight to sA (which the forward phase does
  // not read), the z role's stays in registers, and only the y role's q waits
  // for the barrier (its result overwrites sU, which other lanes still read)
  double qy[N], cz[N];
  double fy[2], fz[2];
  if (active) {
    const double wa = sw[a], wb = sw[b];
    const double jwab = J * wa * wb;
    // ---- x role: line (j, k) = (a, b) ----
    {
      double line[N], g[N];
#pragma unroll
      for (int m = 0; m < N; ++m) line[m] = sU[slot][L(b, a, m)];
      eo_apply<N>(line, g, T.fwd);
#pragma unroll
      for (int m = 0; m < N; ++m) g[m] *= P.rh[0];
      double fx[2];
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int ie = side ? N - 1 : 0;
        const double sg = side ? 1.0 : -1.0;
        // branch-free: a missing neighbour reads the element itself and the
        // result is replaced by the boundary's ghost state
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
        sA[slot][L(b, a, i)] = v;
      }
    }
    // ---- y role: line (i, k) = (a, b) ----
    {
      double line[N], g[N];
#pragma unroll
      for (int m = 0; m < N; ++m) line[m] = sU[slot][L(b, m, a)];
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
      sU[slot][L(b, j, a)] = v;
    }
  }
  // the right-hand side and diagonal of this lane's z-line, loaded before the
  // barrier and before any store (the gather-out stores may not be reordered
  // ahead of later loads, so loads inside the store loop would serialise)
  constexpr bool need_b = MODE == kResidual || MODE == kResidualDiag || MODE == kPuncture;
  constexpr bool need_d = MODE == kApplyDiag || MODE == kResidualDiag || MODE == kPuncture;
  double bz[need_b ? N : 1], dz[need_d ? N : 1];
  if (active) {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const long long gi = e * N3 + k * N2 + t;
      if constexpr (need_b) bz[k] = bvec[gi];
      if constexpr (need_d) dz[k] = aux0[gi];
    }
  }
  __syncthreads();
  if (active) {
    const double jwab = J * sw[a] * sw[b];
    double rz[N];
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double r = cz[k] * P.rh[2] + sA[slot][L(k, b, a)] + sU[slot][L(k, b, a)];
      if (k == 0) r -= fz[0];
      if (k == N - 1) r -= fz[1];
      const long long gi = e * N3 + k * N2 + t;
      if constexpr (MODE == kResidual) {
        r = bz[k] - r;
      } else if constexpr (MODE == kApplyDiag) {
        r += dz[k] * uz[k];
      } else if constexpr (MODE == kResidualDiag) {
        r = bz[k] - (r + dz[k] * uz[k]);
      } else if constexpr (MODE == kPuncture) {
        const double tt = dz[k] * (1.0 + uz[k]) + 1.0;
        const double t2 = tt * tt, t4 = t2 * t2;
        const double S = -aux1[gi] / (t4 * t2 * tt);
        r += jwab * T.w[k] * S - bz[k];
      }
      rz[k] = r;
    }
    if (ucopy) {
#pragma unroll
      for (int k = 0; k < N; ++k) ucopy[e * N3 + k * N2 + t] = uz[k];
    }
    if constexpr (GO == 0) {
      // NT: streamed out with non-temporal stores, which leave the cached
      // input lines (the neighbours' lines read by later workgroups) in place
      // (a compile-time choice: a runtime branch lets the compiler merge the
      // two stores and drop the non-temporal hint)
      if constexpr (NT) {
#pragma unroll
        for (int k = 0; k < N; ++k) __builtin_nontemporal_store(rz[k], &out[e * N3 + k * N2 + t]);
      } else {
#pragma unroll
        for (int k = 0; k < N; ++k) out[e * N3 + k * N2 + t] = rz[k];
      }
    } else if constexpr (GO == 1) {
      store_subdomain_rows<float, N>(rz, (float*)go.rs, sPull[slot], a, b, go.nov);
    } else {
      store_subdomain_rows<double, N>(rz, (double*)go.rs, sPull[slot], a, b, go.nov);
    }
  }
}

template <int N, int EPB, int MODE, int GO, bool BR>
hipError_t launch_apply_k(const double* u, double* out, const double* b, const double* aux0,
                          const double* aux1, const int* nbr, const OpParams& P, const DevTables& T,
                          hipStream_t s, const int* order, const GatherOut& go, double* ucopy) {
  const int threads = ((EPB * N * N + 63) / 64) * 64;
  long long need = ((long long)P.E + EPB - 1) / EPB;
  if (BR)
    need = (long long)((P.n[0] + 1) / 2) * ((P.n[1] + 1) / 2) * ((P.n[2] + 1) / 2);
  const long long blocks = ((need + 7) / 8) * 8;  // whole rounds over the 8 XCDs
  // when u and A u together exceed the 256 MB Infinity Cache, the output
  // would only push out input lines that neighbouring workgroups still read:
  // it is then written with non-temporal stores (measured at 40^3, p = 7:
  // 12-18 % faster; on cache-resident sizes the solves that read the output
  // next lose 0.3-1.4 % with them, so those keep ordinary stores)
  const long long vec_bytes = (long long)P.E * N * N * N * (long long)sizeof(double);
  if constexpr (GO == 0) {
    if (2 * vec_bytes > (256LL << 20)) {
      hipLaunchKernelGGL((k_apply<N, EPB, MODE, GO, BR, true>), dim3((unsigned)blocks), dim3(threads), 0,
                         s, u, out, b, aux0, aux1, nbr, P, T, order, go, ucopy);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((k_apply<N, EPB, MODE, GO, BR>), dim3((unsigned)blocks), dim3(threads), 0, s,
                     u, out, b, aux0, aux1, nbr, P, T, order, go, ucopy);
  return hipGetLastError();
}

template <int N, int EPB, bool BR>
hipError_t launch_apply_t(int mode, const double* u, double* out, const double* b,
                          const double* aux0, const double* aux1, const int* nbr,
                          const OpParams& P, const DevTables& T, hipStream_t s, const int* order,
                          const GatherOut& go, double* ucopy) {
  if (P.E <= 0) return hipSuccess;
  const int gox = go.rs ? (go.f32 ? 1 : 2) : 0;
#define DGS_APPLY(M, G) \
  launch_apply_k<N, EPB, M, G, BR>(u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy)
  switch (mode) {
    case kApply: return DGS_APPLY(kApply, 0);
    case kApplyDiag: return DGS_APPLY(kApplyDiag, 0);
    case kPuncture: return DGS_APPLY(kPuncture, 0);
    case kResidual:
      return gox == 0 ? DGS_APPLY(kResidual, 0)
                      : (gox == 1 ? DGS_APPLY(kResidual, 1) : DGS_APPLY(kResidual, 2));
    case kResidualDiag:
      return gox == 0 ? DGS_APPLY(kResidualDiag, 0)
                      : (gox == 1 ? DGS_APPLY(kResidualDiag, 1) : DGS_APPLY(kResidualDiag, 2));
    default: return hipErrorInvalidValue;
  }
#undef DGS_APPLY
}

template <int N>
hipError_t launch_apply_n(const ApplyConfig& cfg, int mode, const double* u, double* out,
                          const double* b, const double* aux0, const double* aux1, const int* nbr,
                          const OpParams& P, const DevTables& T, hipStream_t s, const int* order,
                          const GatherOut& go, double* ucopy) {
  constexpr int def = (N == 2) ? 64 : (256 / (N * N));  // >= 3 for N <= 9, 1 or 2 beyond
  if (cfg.bricks) {
    // bricks pay off only where one element fills a wavefront (N^2 = 64):
    // then every brick decision is wave-uniform
    if constexpr (N == 8) {
      if (P.n[0] <= 0) return hipErrorInvalidValue;  // bricks need the box grid
      return launch_apply_t<N, 8, true>(mode, u, out, b, aux0, aux1, nbr, P, T, s, cfg.bricks, go,
                                        ucopy);
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (cfg.epb == 1)
    return launch_apply_t<N, 1, false>(mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
  if (cfg.epb == 2)
    return launch_apply_t<N, 2, false>(mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
  return launch_apply_t<N, def, false>(mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
}

// b = M f, M = J w_i w_j w_k
__global__ void k_mass(const double* __restrict__ f, double* __restrict__ out, long long total,
                       int N, double J, DevTables T) {
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int N3 = N * N * N;
  const int loc = (int)(g % N3);
  const int i = loc % N, j = (loc / N) % N, k = loc / (N * N);
  out[g] = J * T.w[i] * T.w[j] * T.w[k] * f[g];
}

__global__ void k_coords(double* __restrict__ xyz, long long total, int N, int nx, int ny,
                         double lx, double ly, double lz, double hx, double hy, double hz,
                         DevTables T) {
  const double* xi = T.xi;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= total) return;
  const int N3 = N * N * N;
  const long long e = g / N3;
  const int loc = (int)(g % N3);
  const int i = loc % N, j = (loc / N) % N, k = loc / (N * N);
  const int ex = (int)(e % nx), ey = (int)((e / nx) % ny), ez = (int)(e / ((long long)nx * ny));
  xyz[g] = lx + hx * (ex + 0.5 * (xi[i] + 1.0));
  xyz[total + g] = ly + hy * (ey + 0.5 * (xi[j] + 1.0));
  xyz[2 * total + g] = lz + hz * (ez + 0.5 * (xi[k] + 1.0));
}

}  // namespace

hipError_t launch_apply(int N, int mode, const double* u, double* out, const double* b,
                        const double* aux0, const double* aux1, const int* nbr, const OpParams& P,
                        const DevTables& T, const ApplyConfig& cfg, hipStream_t s,
                        const int* order, const GatherOut& go, double* ucopy) {
  if (go.rs && (mode != kResidual && mode != kResidualDiag)) return hipErrorInvalidValue;
  switch (N) {
    case 2: return launch_apply_n<2>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    case 3: return launch_apply_n<3>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    case 4: return launch_apply_n<4>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    case 5: return launch_apply_n<5>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    case 6: return launch_apply_n<6>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    case 7: return launch_apply_n<7>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    case 8: return launch_apply_n<8>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    case 9: return launch_apply_n<9>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    case 10: return launch_apply_n<10>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    case 11: return launch_apply_n<11>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    case 12: return launch_apply_n<12>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    case 13: return launch_apply_n<13>(cfg, mode, u, out, b, aux0, aux1, nbr, P, T, s, order, go, ucopy);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_mass(int N, const double* f, double* out, long long E, const double h[3],
                       const DevTables& T, hipStream_t s) {
  const long long total = E * N * N * N;
  if (total <= 0) return hipSuccess;
  const double J = h[0] * h[1] * h[2] * 0.125;
  hipLaunchKernelGGL(k_mass, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, f, out, total,
                     N, J, T);
  return hipGetLastError();
}

hipError_t launch_coords(int N, double* xyz, const int n[3], const double lower[3],
                         const double h[3], const DevTables& T, hipStream_t s) {
  const long long total = (long long)n[0] * n[1] * n[2] * N * N * N;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coords, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, xyz, total,
                     N, n[0], n[1], lower[0], lower[1], lower[2], h[0], h[1], h[2], T);
  return hipGetLastError();
}

}  // namespace dgs
