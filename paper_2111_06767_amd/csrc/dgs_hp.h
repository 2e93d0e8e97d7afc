// Internal declarations of the hp-nonuniform path: elements of their own
// degree per dimension (2..8 points) and refinement level, joined by mortars
// on nonconforming faces (Sec. II), with per-subdomain Schwarz inverses and a
// multigrid hierarchy that keeps the smaller degree when it merges elements
// (Sec. III.C.1).
#pragma once

#include "dgs_internal.h"

namespace dgs {

constexpr int kHpMaxN = 8;  // points per dimension
constexpr int kHpMaxNodes = kHpMaxN * kHpMaxN * kHpMaxN;

// Neighbour codes of a face term that has no neighbour data.
constexpr int kHpDirichlet = -1;  // box face, homogeneous Dirichlet ghost (eq. bc)
constexpr int kHpNeumann = -2;    // box face, homogeneous Neumann ghost (eq. bc)
constexpr int kHpZero = -3;       // a neighbour whose values are zero (set-up patches)

// One mortar of an element face: the part shared with one neighbour.  The
// face's transverse dimensions are t0 < t1; face arrays are [t1][t0].  The
// mortar's interpolations I (face points -> mortar points) and its exact L2
// projection P back to the element's face points are stored premultiplied
// per dimension: A_t = P_t I_own,t (N_own x N_own) and B_t = P_t I_nb,t
// (N_own x N_nb), so that the projected corrections are
//   cu = 1/2 (B u_nb - A u_own),
//   cp = 1/2 s (A du_own + B du_nb) - sigma (A u_own - B u_nb)
// with A = A_t1 (x) A_t0 and B = B_t1 (x) B_t0.  Matrices live in a pool of
// doubles (row-major); offset -1 is the identity.
struct HpTerm {
  int nb;        // neighbour element (>= 0) or one of the codes above
  int direct;    // 1: a box face, or a conforming face of equal points (every
                 //    matrix the identity): the flux is formed point by point
  int A0, A1;    // P I_own per transverse dimension
  int B0, B1;    // P I_nb per transverse dimension
  double sigma;  // penalty (eq. penalty)
  // the neighbour's first node, points per dimension and 2 / h along the
  // face normal (copies of its HpElem fields, so that its face data can be
  // read without first loading its element record)
  long long foff;
  int fN[3];
  double frh;
};

struct HpElem {
  long long off;      // first node; nodes [k][j][i] with i fastest
  int N[3];           // points per dimension
  int term0;          // first term of face 0; faces' terms follow in face order
  int nterm[6];       // terms per face (>= 1)
  double rh[3];       // 2 / h_d
  double jac;         // h_x h_y h_z / 8
};

// Device tables of the LGL rule for N = 2..kHpMaxN: D at (N - 2) * 64
// (row-major N x N), weights and nodes at (N - 2) * 8.
struct HpRule {
  const double* D;
  const double* w;
  const double* xi;
};

// Subdomain rows of one Schwarz subdomain in the gather block.
struct HpSub {
  long long rs;  // first row entry in RS / DU
  int start;     // first entry in the global-index table
  int n;         // rows
};

// One entry of the pull scatter: point p adds w * DU[pos] (summed over parts).
struct HpPull {
  long long pos;
  double w;
};

// Multigrid transfer of one fine element: its parent and the 1D child
// interpolation matrices (pool offsets, N_fine x N_coarse per dimension).
struct HpChild {
  int parent;
  int P[3];
};

// out = A u (residual: b - A u) for elements [0, E) of a mesh or of
// `copies` copies of a set-up patch (copy c reads and writes at c * copy_stride).
// order (optional): workgroup w takes element order[w] (the most expensive
// elements first, so that their longer chains of face terms start early).
hipError_t launch_hp_apply(bool residual, const double* u, double* out, const double* b,
                           const HpElem* el, int E, const HpTerm* terms, const double* pool,
                           const HpRule& R, int copies, long long copy_stride, hipStream_t s,
                           const int* order = nullptr);
// RS[pos] = (b - A u)[p] for every row position pos that push_ptr / push_pos
// list for point p (the Schwarz gather fused into the residual; RS in FP32
// with f32); the residual vector itself is not written
hipError_t launch_hp_residual_gather(const double* u, const double* b, const HpElem* el, int E,
                                     const HpTerm* terms, const double* pool, const HpRule& R,
                                     const int* order, const long long* push_ptr,
                                     const long long* push_pos, bool f32, void* rs, hipStream_t s);
hipError_t launch_hp_mass(const double* f, double* out, const HpElem* el, int E, const HpRule& R,
                          hipStream_t s);
// node coordinates: plo (3 per element, the lower corner) and h (3 per element)
hipError_t launch_hp_coords(double* xyz, long long ndof, const HpElem* el, const double* plo_h,
                            int E, const HpRule& R, hipStream_t s);
// RS[sub.rs + q] = r[gidx[sub.start + q]] for every subdomain (RS in FP32
// with f32, else FP64)
hipError_t launch_hp_gather(bool f32, const double* r, void* rs, const HpSub* subs, int nsub,
                            const long long* gidx, hipStream_t s);
// u[p] += sum over the pull entries of p of w * sum_parts DU[part * stride + pos]
// (DU in FP32 with f32), summed in FP64
hipError_t launch_hp_scatter(bool f32, double* u, const void* du, int parts, long long part_stride,
                             const long long* ptr, const HpPull* pull, long long ndof,
                             hipStream_t s);
// fine[e] += P_e coarse[parent]
hipError_t launch_hp_prolongate_add(const double* coarse, double* fine, const HpElem* fel,
                                    const HpElem* cel, const HpChild* ch, int Ef,
                                    const double* pool, hipStream_t s);
// coarse[c] = sum over children e of P_e^T fine[e]; children of c listed at
// kids[kid_ptr[c] .. kid_ptr[c + 1])
hipError_t launch_hp_restrict(const double* fine, double* coarse, const HpElem* fel,
                              const HpElem* cel, const HpChild* ch, const int* kid_ptr,
                              const int* kids, int Ec, const double* pool, hipStream_t s);

}  // namespace dgs
