// Internal declarations of the gfx950 DG multigrid-Schwarz solver library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace dgs {

constexpr int kMaxN = 13;  // p <= 12

// ---------------------------------------------------------------------------
// Host tables (LGL nodes/weights, derivative and child interpolation)
// ---------------------------------------------------------------------------
struct HostTables {
  int N = 0;
  std::vector<double> xi, w, D, Plo, Phi;  // D, Plo, Phi row-major N x N
};
HostTables make_tables(int N);

// Even-odd split of a centro-antisymmetric N x N matrix M (M[N-1-i][N-1-j] =
// -M[i][j], true of the LGL derivative and its transpose): with H = N/2,
// e_m = x_m + x_{N-1-m}, o_m = x_m - x_{N-1-m},
//   a_i = sum_m P[i][m] e_m (+ cf[i] x_c for odd N), c_i = sum_m Q[i][m] o_m,
//   (M x)_i = a_i + c_i, (M x)_{N-1-i} = c_i - a_i, (M x)_c = sum_m rc[m] o_m,
// where P = (M[i][m] + M[i][N-1-m]) / 2, Q = (M[i][m] - M[i][N-1-m]) / 2,
// cf[i] = M[i][c], rc[m] = M[c][m] and c = H is the middle index of odd N.
struct EvenOdd {
  double P[(kMaxN / 2) * (kMaxN / 2)];
  double Q[(kMaxN / 2) * (kMaxN / 2)];
  double cf[kMaxN / 2];
  double rc[kMaxN / 2];
};

// Kernel-argument copy of the tables the operator kernels read (fixed size
// so one struct serves every N): nodes, weights, the first and last rows of
// the derivative matrix (normal derivatives on the faces) and the even-odd
// splits of D and D^T.
struct DevTables {
  double xi[kMaxN];
  double w[kMaxN];
  double D0[kMaxN];  // D[0][m]
  double DN[kMaxN];  // D[N-1][m]
  EvenOdd fwd;  // D
  EvenOdd bwd;  // D^T
};
DevTables to_dev(const HostTables& t);
// Kernel-argument copy of the child interpolation matrices (multigrid
// transfer kernels only).
struct MgTables {
  double Plo[kMaxN * kMaxN];
  double Phi[kMaxN * kMaxN];
};
MgTables to_dev_mg(const HostTables& t);

// Geometry of one uniform box level.
struct OpParams {
  double h[3];
  double penalty;
  int E;
  // element grid n_x, n_y, n_z of a box (face neighbours follow from an
  // element's position); n[0] = 0: take them from the neighbour table instead
  int n[3];
  // derived on the host (set_derived): 2/h_d, sigma_d, lift factor 1/(h_d w_end),
  // J = h_x h_y h_z / 8
  double rh[3], sig[3], lf[3], J;
  // bit f = 2 d + side set: a missing neighbour across face f is a homogeneous
  // Neumann boundary (ghost u_ext = u_int, normal derivative negated), else
  // homogeneous Dirichlet (u_ext = -u_int, normal derivative kept); eq. bc
  int neumann;
};
void set_derived(OpParams& P, int N, double w_end);

// Operator modes of the fused apply kernel.
enum ApplyMode : int {
  kApply = 0,         // out = A u
  kResidual = 1,      // out = b - A u
  kApplyDiag = 2,     // out = A u + d .* u
  kResidualDiag = 3,  // out = b - (A u + d .* u)
  kPuncture = 4,      // out = A u + M S(u) - b,  S = -beta (alpha (1+u) + 1)^-7
};

// Launch configuration of the operator kernel: elements per workgroup, or
// 2 x 2 x 2 bricks of a box grid taken in the order of the brick table.
struct ApplyConfig {
  int epb = 0;                   // 0 = default for N
  const int* bricks = nullptr;   // device table of brick indices (N = 8)
};

constexpr int kGemmLd = 128, kGemmRows = 64;

// Class frames.  A subdomain is stored in the frame of its canonical boundary
// class: the element's own axes are first mirrored (bit d of a 3-bit mask
// reverses axis d), then two axes of equal element width may be exchanged
// (transposition t: 0 none, 1 axes 0 / 1, 2 axes 0 / 2, 3 axes 1 / 2), so that
// the face, edge and corner subdomains of all orientations share one class.
// A frame code is mask | t << 3.
__host__ __device__ __forceinline__ int frame_axis(int d, int t) {
  // the axis that holds axis d after transposition t (t is an involution)
  if (t == 1) return d == 0 ? 1 : (d == 1 ? 0 : 2);
  if (t == 2) return d == 0 ? 2 : (d == 2 ? 0 : 1);
  if (t == 3) return d == 1 ? 2 : (d == 2 ? 1 : 0);
  return d;
}

// Offsets of a point's three own-axis coordinates in its class frame: a point
// (i, j, k) lies at mi * s0 + mj * s1 + mk * s2, m the mirrored coordinates.
__device__ __forceinline__ void frame_strides(int code, int N, int& s0, int& s1, int& s2) {
  const int t = code >> 3, N2 = N * N;
  s0 = t == 1 ? N : (t == 2 ? N2 : 1);
  s1 = t == 1 ? 1 : (t == 3 ? N2 : N);
  s2 = t == 2 ? 1 : (t == 3 ? N : N2);
}

// own point (i, j, k) -> its offset in the class frame
__device__ __forceinline__ int to_class_frame(int i, int j, int k, int code, int N) {
  int s0, s1, s2;
  frame_strides(code, N, s0, s1, s2);
  const int mi = (code & 1) ? N - 1 - i : i;
  const int mj = (code & 2) ? N - 1 - j : j;
  const int mk = (code & 4) ? N - 1 - k : k;
  return mi * s0 + mj * s1 + mk * s2;
}

// Overlap strips: (t0, t1) are the point's coordinates along the two own
// axes transverse to the shared face, in ascending axis order; the flip bits
// of the neighbour's pull entry map them into the neighbour's class frame.
__device__ __forceinline__ void strip_coords(int& t0, int& t1, int flip, int N) {
  if (flip & 4) {
    const int t = t0;
    t0 = t1;
    t1 = t;
  }
  if (flip & 1) t0 = N - 1 - t0;
  if (flip & 2) t1 = N - 1 - t1;
}

// Pull table of the weighted scatter, 7 entries per element: entry 0 is the
// element's own subdomain, entry 1 + f the subdomain of its face-f neighbour.
struct PullEntry {
  long long du;  // entry 0: the element's row in the correction block;
                 // faces: start of the neighbour's strip toward the element (-1: none)
  int w;         // matching offset in the weight table
  int flip;      // entry 0: frame code of the element; faces: bit 2 exchanges the two
                 // transverse coordinates, then bits 0 / 1 reverse the first / second
                 // (the neighbour's class frame there)
};

// Write the value v of point (i, j, k) of an element into the subdomain rows
// that hold it: the element's own row (pe[0], in its class frame) and the
// overlap strips of its face neighbours' subdomains (pe[1 + f]), at the
// offsets of the scatter's pull table (the transpose of its reads).
template <typename TS>
__device__ __forceinline__ void gather_out_point(TS* rs, const PullEntry* pe, int N, int nov,
                                                 int i, int j, int k, double v) {
  const int N2 = N * N;
  const PullEntry own = pe[0];
  rs[own.du + to_class_frame(i, j, k, own.flip, N)] = (TS)v;
  const int idx[3] = {i, j, k};
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const PullEntry q = pe[1 + f];
    const int d = f >> 1;
    const int layer = (f & 1) ? N - 1 - idx[d] : idx[d];
    if (q.du < 0 || layer >= nov) continue;
    int t0 = d == 0 ? j : i, t1 = d == 2 ? j : k;
    strip_coords(t0, t1, q.flip, N);
    rs[q.du + layer * N2 + t1 * N + t0] = (TS)v;
  }
}

// Residual modes only: instead of r, write r_S = R_S r for every subdomain
// (the element's own row and its points in the face neighbours' overlap
// strips, located through the scatter's pull table) into the gather block rs.
struct GatherOut {
  void* rs = nullptr;  // nullptr: write r to `out` as usual
  bool f32 = false;    // rs holds FP32 (mixed-precision level) or FP64 values
  const PullEntry* pull = nullptr;
  int nov = 0;         // overlap layers
};

// order (optional, may be NULL): processing order of the elements, a
// permutation of 0..E-1 that keeps face neighbours close in time.
hipError_t launch_apply(int N, int mode, const double* u, double* out, const double* b,
                        const double* aux0, const double* aux1, const int* nbr, const OpParams& P,
                        const DevTables& T, const ApplyConfig& cfg, hipStream_t s,
                        const int* order = nullptr, const GatherOut& go = GatherOut{},
                        double* ucopy = nullptr);  // ucopy: optional copy of u
hipError_t launch_mass(int N, const double* f, double* out, long long E, const double h[3],
                       const DevTables& T, hipStream_t s);
hipError_t launch_coords(int N, double* xyz, const int n[3], const double lower[3],
                         const double h[3], const DevTables& T, hipStream_t s);

// Schwarz subdomain data of one level.
struct ClassInfo {
  int n;            // subdomain size n_S
  int count;        // number of subdomains (elements) in the class
  // Padded storage, zero outside the n x n / count x n values, so that the
  // class GEMM reads whole 16-byte vectors without bounds checks:
  int ld;           // row stride of the class's RS / DU rows and of its stored
                    // matrices: n rounded up to a multiple of kGemmLd
  int rows;         // RS / DU rows reserved: count rounded up to kGemmRows
  int kext;         // K extent of the products: n rounded up to 32
  const void* inv;    // stored transposed inverse (n x n, level precision)
  const void* op;     // stored transposed subdomain operator A_S (level precision)
  double scale;       // factor applied to the stored inverse for this level
  double scale_op;    // factor applied to the stored A_S for this level
  long long rs_off;   // offset of this class's [rows][ld] block in RS / DU
  int layout_off;     // offset into seg_loc / weights
  int strip_off[6];   // offset of each face strip in the layout, -1 if absent
};

// One output tile of a class GEMM over the K range [k0, k1); split-K part
// `part` writes its partial product to part * part_stride + rs_off.
struct GemmTile {
  int cls, m0, n0, part, k0, k1;
};

// r_S = R_S r for every subdomain (one per element) into row elem_row[e].
hipError_t launch_gather(int N, bool f32, const double* r, void* rs, const int* elem_class,
                         const long long* elem_row, const int* nbr, const ClassInfo* cls,
                         const int* seg_loc, int E, hipStream_t s);
// Grouped subdomain GEMM of one level, one launch: DU_c = scale * RS_c * B_c
// for every class c (B_c the stored transposed inverse, or with use_op the
// stored A_S and factor scale_op).  Output tiles of BM rows (subdomains) by
// BN columns: BM = 16, BN = 64 when no class has more than kGemmSmallCount
// subdomains, with the K range split into up to 16 (variant 0), 4 (variant 1),
// 8 (variant 2), 2 (variant 3) or 1 (variant 4) partial products; else
// BM x BN = 32 x kGemmN (variant 0), 64 x kGemmN (variant 1), 32 x 64
// (variant 2), 64 x 64 (variant 3) or 64 x 64 with twice the K step in FP64
// (variant 4), and up to 4 parts.  The set-up autotuner picks one per level.
constexpr int kGemmN = 128, kGemmSmallCount = 32;
constexpr int kMaxParts = 16;  // split-K partial products (1, 2, 4, 8 or 16)
constexpr int kGemmVariants = 5;
struct GemmPlan {
  std::vector<GemmTile> tiles;
  bool small = false;
  int kparts = 1;
};
// parts_cap > 0: at most that many split-K parts (the partial-product
// buffers of the classes hold no more)
GemmPlan plan_subdomain_gemm(const std::vector<ClassInfo>& cls, int variant, int parts_cap = 0);
// The grouped GEMM over classes of several problems (the serving loop's
// batched sweeps): class c reads its rows at ptrs[c].rs and writes part p of
// its corrections at ptrs[c].du + p * ptrs[c].pstride (offsets rs_off within);
// tiles from plan_subdomain_gemm over the joined class list, variant 2 (or
// the small-tile form).
struct GemmPtr {
  const void* rs;
  void* du;
  long long pstride;
};
hipError_t launch_subdomain_gemm_batched(bool f32, const ClassInfo* cls, const GemmPtr* ptrs,
                                         const GemmTile* tiles, int ntiles, bool small,
                                         hipStream_t s);
hipError_t launch_subdomain_gemm(bool f32, const void* rs, void* du, long long part_stride,
                                 const ClassInfo* cls, const GemmTile* tiles, int ntiles,
                                 bool small, int use_op, hipStream_t s, int variant);
// out[i] = sum over parts of part_base[p * stride + i]
hipError_t launch_reduce_parts(bool f32, void* out, const void* parts_base, int parts,
                               long long stride, long long total, hipStream_t s);
// Batched subdomain GMRES(k) pieces (one workgroup per subdomain):
//   start:   beta = |r_S|, V_0 = r_S / beta
//   arnoldi: w = W + d_S .* Z_j, modified Gram-Schmidt against V_0..V_j,
//            H[:, j], V_{j+1} = w / |w|
//   finish:  least-squares solve of the Hessenberg system, du_S = sum y_j Z_j
hipError_t launch_sub_start(bool f32, const void* rs, void* V0, double* beta,
                            const int* elem_class, const long long* elem_row, const ClassInfo* cls,
                            int E, hipStream_t s);
// (max_n: the largest subdomain of the level, at most 4352 points)
hipError_t launch_sub_arnoldi(int N, bool f32, int j, int kmax, const void* W, void* V, const void* Zj,
                              long long stride, const double* diag, double* H,
                              const int* elem_class, const long long* elem_row, const int* nbr,
                              const ClassInfo* cls, const int* seg_loc, int E, int max_n,
                              hipStream_t s);
hipError_t launch_sub_finish(bool f32, int kmax, const void* Z, long long stride, const double* H,
                             const double* beta, void* du, const int* elem_class,
                             const long long* elem_row, const ClassInfo* cls, int E, hipStream_t s);
// u += sum_S R_S^T (w_S du_S), pulled per point; du is the sum of `parts`
// split-K partial products spaced part_stride apart.

// u += sum_S R_S^T (w_S du_S), summing `parts` split-K partials (1, 2, 4, 8, 16) of du.
// assign: u = (the sum) instead of u += (the sum), for a u that starts at zero.
// Subdomain GMRES of a system of nv <= kSysMaxVars variables whose rows sit
// at a * stride (see k_sys_arnoldi); D holds the pointwise couplings D_ab as
// nv * nv fields of nd points.  Subdomains of at most 2048 points.
constexpr int kSysMaxVars = 5;
constexpr int kSysMaxRows = 2048;  // subdomain points of the system Arnoldi step (256 x 8)
hipError_t launch_sys_start(bool f32, int nv, const void* rs, void* V0, double* beta,
                            long long stride, const int* elem_class, const long long* elem_row,
                            const ClassInfo* cls, int E, hipStream_t s);
hipError_t launch_sys_arnoldi(int N, bool f32, int j, int kmax, int nv, const void* W, void* V,
                              const void* Zj, long long stride, const double* D, long long nd,
                              double* H, const int* elem_class, const long long* elem_row,
                              const int* nbr, const ClassInfo* cls, const int* seg_loc, int E,
                              int max_n, hipStream_t s);
hipError_t launch_sys_finish(bool f32, int kmax, int nv, const void* Z, long long stride,
                             const double* H, const double* beta, void* du, const int* elem_class,
                             const long long* elem_row, const ClassInfo* cls, int E,
                             hipStream_t s);
// y_a += sign * sum_b D_ab u_b at every point (nv fields of nd points each)
hipError_t launch_sys_couple(double* y, const double* u, const double* D, int nv, long long nd,
                             double sign, hipStream_t s);

hipError_t launch_scatter(int N, bool f32, double* u, const void* du, int parts,
                          long long part_stride, const double* weights, const PullEntry* pull,
                          int nov, long long E, hipStream_t s, bool assign = false);

// Multigrid transfer (per-dimension split flags).
hipError_t launch_restrict(int N, const double* fine, double* coarse, const int nf[3],
                           const int nc[3], const int split[3], const MgTables& T, hipStream_t s,
                           const GatherOut& go = GatherOut{});  // go: also the coarse r_S rows
hipError_t launch_prolongate_add(int N, const double* coarse, double* fine, const int nf[3],
                                 const int nc[3], const int split[3], const MgTables& T,
                                 hipStream_t s);

// Curved (isoparametric) elements: per-node metric of the finest level, set
// from caller-given node coordinates.  inv holds invJ^d_c = dxi^d/dx^c as 9
// fields (field 3 d + c), det the Jacobian determinant, grad 3 work fields
// (the physical gradient of the operand), D the N x N LGL derivative and w
// the N LGL weights (device copies).  Elements of 2..8 points per dimension.
struct CurvedGeometry {
  double* inv = nullptr;
  double* det = nullptr;
  double* grad = nullptr;
  double* D = nullptr;
  double* w = nullptr;
};
hipError_t launch_curved_geometry(int N, const double* xyz, long long E, const double* D,
                                  double* inv, double* det, hipStream_t s);
// out = A u (+ diag u) or, with residual, out = b - (A u + diag u) (diag may be NULL)
hipError_t launch_curved_apply(int N, bool residual, const double* u, double* out, const double* b,
                               const double* diag, const CurvedGeometry& G, const int* nbr, double C,
                               int neumann, long long E, hipStream_t s);
hipError_t launch_curved_mass(int N, const double* f, double* out, const CurvedGeometry& G,
                              long long E, hipStream_t s);

// Vector kernels.
hipError_t launch_fill(double* x, double v, long long n, hipStream_t s);
// FP32 or FP64 pseudo-random values in [-0.5, 0.5) (timing operands)
hipError_t launch_fill_pattern(void* x, bool f32, long long n, hipStream_t s);
hipError_t launch_copy(double* y, const double* x, long long n, hipStream_t s);
hipError_t launch_axpy(double* y, double a, const double* x, long long n, hipStream_t s);
// Multi-dot: h[i] = <V_i, w> for i < m (V_i = V + i * ldv); partial sums in
// `partial` (blocks x m), final reduction into h (device).  Deterministic.
int multidot_blocks(long long n);
hipError_t launch_multidot(const double* V, long long ldv, int m, const double* w, long long n,
                           double* partial, double* h, hipStream_t s);
// w -= sum_{i < m} coef_i V_i (coef on the device), then h_i = V_i . w for
// i < m, or h_0 = w . w when norm_only; the same fixed-order reductions.
hipError_t launch_axpy_multidot(const double* V, long long ldv, int m, const double* coef, double* w,
                                long long n, bool norm_only, double* partial, double* h,
                                hipStream_t s);
// w -= sum_i coef[i] * V_i  (coef on the device, scaled by `sign`)
hipError_t launch_multi_axpy(double* w, const double* V, long long ldv, int m, const double* coef,
                             long long n, hipStream_t s);
// y = x / sqrt(*nrm2); y2 (optional) receives a copy; with go.rs the values
// are also written into the finest level's subdomain rows (N points per
// dimension, go.pull of that level).
hipError_t launch_scale_by_inv_norm(double* y, const double* x, const double* nrm2, long long n,
                                    hipStream_t s, double* y2 = nullptr, int N = 0,
                                    const GatherOut& go = GatherOut{});  // y2: optional copy
// x += sum_i y[i] Z_i (y on the device)
hipError_t launch_combine(double* x, const double* Z, long long ldz, int m, const double* y,
                          long long n, hipStream_t s);
// d = M * 7 alpha beta (alpha (1+u) + 1)^-8 (puncture linearisation diagonal)
hipError_t launch_puncture_diag(int N, const double* alpha, const double* beta, const double* u,
                                double* d, long long E, const double h[3], const DevTables& T,
                                hipStream_t s);
// y = x + lam * dx
hipError_t launch_waxpy(double* y, const double* x, double lam, const double* dx, long long n,
                        hipStream_t s);
// Conjugate-gradient update: alpha = rz / *pq (0 if *pq <= 0; pq on the
// device), x += alpha p, r_next = r - alpha q.
hipError_t launch_cg_step(double* x, double* r_next, const double* r, const double* p,
                          const double* q, double rz, const double* pq, long long n, hipStream_t s);

// ---------------------------------------------------------------------------
// Cross-request batched launches (the serving loop): each problem's share of
// a launch is a job; the jobs of a launch are listed by their first
// workgroup blk0 (ascending), and the last job ends at the launch's block
// count.  Degrees N <= 9 may mix in one launch.
// ---------------------------------------------------------------------------
struct BApplyJob {       // one element per workgroup: blk0 + e for element e
  const double* u;
  double* out;           // vector output (when the launch does not write rows)
  const double* b;       // right-hand side (residual)
  double* ucopy;         // optional copy of u
  GatherOut go;          // rows output (rs, f32, pull, nov)
  OpParams P;            // box grid (P.n set)
  int N;
  int blk0;
};
struct BScatterJob {     // 256 points per workgroup
  double* u;
  const void* du;        // partial products, FP32 (f32) or FP64
  const double* weights;
  const PullEntry* pull;
  long long pstride;     // distance between split-K parts
  long long total;       // E N^3
  int N, nov, parts, f32, assign;
  int blk0;
};
struct BTransferJob {    // one coarse (restriction) / fine (prolongation) element per workgroup
  const double* src;
  double* dst;
  GatherOut go;          // restriction: the coarse level's first rows
  int nf[3], nc[3], split[3];
  int N;
  int blk0;
};
struct BDotJob {         // multidot_blocks(n) workgroups from blk0, outputs from fblk0
  const double* V;
  long long ldv;
  int m;                 // vectors V_0..V_{m-1}
  int mode;              // 0 dots with w; 1 w -= V coef, then dots; 2 w -= V coef, then |w|^2
  const double* coef;
  double* w;
  long long n, chunk;
  double* partial;
  int nblocks;
  double* h;             // m results (1 for mode 2)
  int blk0, fblk0;
};
struct BVecJob {         // 256 points per workgroup
  double* y;             // Z null: y = x / sqrt(*nrm2) (and y2, rows); else y += sum coef_i Z_i
  const double* x;
  const double* nrm2;
  double* y2;
  GatherOut go;
  long long n;
  int N;
  const double* coef;
  const double* Z;
  long long ldz;
  int m;
  int blk0;
};
// mode kApply (rows = false, with ucopy) or kResidual (rows: write r_S);
// threads 64 (every N^2 <= 64) or 128; tabs[N] the device tables of degree N-1
hipError_t launch_batch_apply(int mode, bool rows, const BApplyJob* jobs, int njobs, int nblocks,
                              int threads, const DevTables* tabs, hipStream_t s);
hipError_t launch_batch_scatter(const BScatterJob* jobs, int njobs, int nblocks, hipStream_t s);
hipError_t launch_batch_restrict(const BTransferJob* jobs, int njobs, int nblocks,
                                 const MgTables* tabs, hipStream_t s);
hipError_t launch_batch_prolongate(const BTransferJob* jobs, int njobs, int nblocks,
                                   const MgTables* tabs, hipStream_t s);
hipError_t launch_batch_dots(const BDotJob* jobs, int njobs, int nblocks, int nfinal,
                             hipStream_t s);
hipError_t launch_batch_vec(const BVecJob* jobs, int njobs, int nblocks, hipStream_t s);

// Set-up kernels: unit-vector fill and column gather for the patch apply, the
// blocked inversion, and the transposed copies of the results.
// Blocked Gauss-Jordan inversion in place of a batch of n x n SPD matrices,
// n a multiple of 64; work buffers P (batch*64*64), R and C (batch*64*n each).
hipError_t launch_block_inverse(double* A, int n, int batch, double* Pbuf, double* Rbuf,
                                double* Cbuf, hipStream_t s);
hipError_t launch_unit_columns(double* X, long long copy_stride, const int* idx, int ncols,
                               hipStream_t s);
hipError_t launch_gather_columns(const double* AX, long long copy_stride, const int* idx, int n,
                                 double* A, int n_pad, hipStream_t s);
// out[k * ld + row] = scale * Ainv[row * n_pad + k] for row, k < n (the
// transposed matrix, in a caller-zeroed ld x ld array)
hipError_t launch_finish_inverse(const double* Ainv, int n_pad, int n, int ld, double scale,
                                 double* out64, float* out32, hipStream_t s);
hipError_t launch_scale_copy(const double* A, int n_pad, int n, double scale, double* out64,
                             float* out32, hipStream_t s);

}  // namespace dgs
