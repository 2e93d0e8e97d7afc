// Host set-up and C ABI of the hp-nonuniform path.
//
//   mesh        a box of equal blocks, each split 2^L_d times along every
//               dimension d (levels free from block to block, two-to-one
//               balanced across block faces), every element with its own
//               degree per dimension (Sec. II)
//   mortars     one term per (element face, neighbour): interpolation of both
//               sides' face data to the mortar points (the larger degree per
//               face dimension) and the exact L2 projection back
//   Schwarz     element-centred subdomains reaching N_ov points into every
//               face neighbour (Sec. III.D.1), weights from each point's own
//               element so that they sum to one, subdomains of equal
//               structure sharing one explicit inverse built on the device
//   multigrid   each coarser level halves every block along its split
//               dimensions and keeps the smaller degree (Sec. III.C.1)
//   solve       FGMRES preconditioned by one V-cycle (Sec. III.B, III.C.3)
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/dgsolve.h"
#include "dgs_host.h"
#include "dgs_hp.h"

using namespace dgs;

namespace {

// ---------------------------------------------------------------------------
// 1D polynomial tools
// ---------------------------------------------------------------------------
// Gauss-Legendre rule of n points (Newton on the three-term recurrence).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// L[a][b] = l_b(t_a), the Lagrange basis of `nodes` at the targets (rows).
std::vector<double> lagrange(const std::vector<double>& nodes, const std::vector<double>& t) {
  const int n = (int)nodes.size();
  std::vector<double> L(t.size() * n, 1.0);
  for (size_t a = 0; a < t.size(); ++a)
    for (int b = 0; b < n; ++b)
      for (int m = 0; m < n; ++m)
        if (m != b) L[a * n + b] *= (t[a] - nodes[m]) / (nodes[b] - nodes[m]);
  return L;
}

const std::vector<double>& lgl(int N) {
  static std::map<int, std::vector<double>> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(N);
  if (it == cache.end()) it = cache.emplace(N, make_tables(N).xi).first;
  return it->second;
}

// Exact mass matrix of the N-point LGL Lagrange basis on [-1, 1].
std::vector<double> exact_mass(int N) {
  std::vector<double> xg, wg;
  gauss_legendre(N + 1, xg, wg);
  const std::vector<double> B = lagrange(lgl(N), xg);
  std::vector<double> M(N * N, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j)
      for (int g = 0; g < N + 1; ++g) M[i * N + j] += wg[g] * B[g * N + i] * B[g * N + j];
  return M;
}

// X = A^-1 B for A n x n and B n x m (partial pivoting).
std::vector<double> solve_dense(std::vector<double> A, std::vector<double> B, int n, int m) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i * n + k]) > std::fabs(A[piv * n + k])) piv = i;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
      for (int j = 0; j < m; ++j) std::swap(B[k * m + j], B[piv * m + j]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      for (int j = 0; j < m; ++j) B[i * m + j] -= f * B[k * m + j];
    }
  }
  for (int k = n - 1; k >= 0; --k)
    for (int j = 0; j < m; ++j) {
      double v = B[k * m + j];
      for (int q = k + 1; q < n; ++q) v -= A[k * n + q] * B[q * m + j];
      B[k * m + j] = v / A[k * n + k];
    }
  return B;
}

// Pool of small matrices shared by the kernels; identical contents share one
// slot.
struct MatPool {
  std::vector<double> data;
  std::map<std::vector<double>, int> index;
  int add(const std::vector<double>& m) {
    auto it = index.find(m);
    if (it != index.end()) return it->second;
    const int off = (int)data.size();
    data.insert(data.end(), m.begin(), m.end());
    index.emplace(m, off);
    return off;
  }
};

// ---------------------------------------------------------------------------
// Mesh
// ---------------------------------------------------------------------------
struct HElem {
  int block = 0;
  int L[3] = {0, 0, 0};
  long long lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // integer coordinates (see HMesh::R)
  double h[3] = {0, 0, 0}, plo[3] = {0, 0, 0};
  int N[3] = {0, 0, 0};
  long long off = 0;
};

const int kFaceDim[6] = {0, 0, 1, 1, 2, 2};
int face_sign(int f) { return (f & 1) ? 1 : -1; }
int tdim0(int d) { return d == 0 ? 1 : 0; }
int tdim1(int d) { return d == 2 ? 1 : 2; }

struct HMesh {
  double lower[3], upper[3];
  int blocks[3];
  std::vector<std::array<int, 3>> blev;
  std::vector<int> bstart;  // first element of every block
  long long R[3];           // integer units per block: 2^(max level + 2)
  int neumann = 0;
  std::vector<HElem> el;
  long long ndof = 0;
  std::vector<std::array<std::vector<int>, 6>> nbr;

  int E() const { return (int)el.size(); }

  int find(const long long x[3]) const {
    int bc[3];
    for (int d = 0; d < 3; ++d) {
      if (x[d] < 0 || x[d] >= blocks[d] * R[d]) return -1;
      bc[d] = (int)(x[d] / R[d]);
    }
    const int b = (bc[2] * blocks[1] + bc[1]) * blocks[0] + bc[0];
    int idx[3], n[3];
    for (int d = 0; d < 3; ++d) {
      n[d] = 1 << blev[b][d];
      idx[d] = (int)((x[d] - bc[d] * R[d]) / (R[d] >> blev[b][d]));
    }
    return bstart[b] + (idx[2] * n[1] + idx[1]) * n[0] + idx[0];
  }
};

HMesh make_mesh(const double lower[3], const double upper[3], const int blocks[3],
                const std::vector<std::array<int, 3>>& blev, const std::vector<std::array<int, 3>>& deg,
                int neumann) {
  HMesh m;
  for (int d = 0; d < 3; ++d) {
    m.lower[d] = lower[d];
    m.upper[d] = upper[d];
    m.blocks[d] = blocks[d];
  }
  m.blev = blev;
  m.neumann = neumann;
  int Lmax[3] = {0, 0, 0};
  for (auto& L : blev)
    for (int d = 0; d < 3; ++d) Lmax[d] = std::max(Lmax[d], L[d]);
  for (int d = 0; d < 3; ++d) m.R[d] = 1LL << (Lmax[d] + 2);
  const int nb = blocks[0] * blocks[1] * blocks[2];
  for (int b = 0; b < nb; ++b) {
    const int bpos[3] = {b % blocks[0], (b / blocks[0]) % blocks[1], b / (blocks[0] * blocks[1])};
    m.bstart.push_back(m.E());
    const int n[3] = {1 << blev[b][0], 1 << blev[b][1], 1 << blev[b][2]};
    for (int iz = 0; iz < n[2]; ++iz)
      for (int iy = 0; iy < n[1]; ++iy)
        for (int ix = 0; ix < n[0]; ++ix) {
          const int idx[3] = {ix, iy, iz};
          HElem e;
          e.block = b;
          for (int d = 0; d < 3; ++d) {
            e.L[d] = blev[b][d];
            const long long w = m.R[d] >> e.L[d];
            e.lo[d] = bpos[d] * m.R[d] + idx[d] * w;
            e.hi[d] = e.lo[d] + w;
            const double bs = (upper[d] - lower[d]) / blocks[d];
            e.h[d] = bs / n[d];
            e.plo[d] = lower[d] + bs * bpos[d] + e.h[d] * idx[d];
          }
          m.el.push_back(e);
        }
  }
  if ((int)deg.size() != m.E()) throw DgsError(DGS_ERR_INVALID, "num_elements does not match the block levels");
  for (int e = 0; e < m.E(); ++e) {
    for (int d = 0; d < 3; ++d) {
      if (deg[e][d] < 1 || deg[e][d] > kHpMaxN - 1)
        throw DgsError(DGS_ERR_INVALID, "hp degrees must be in [1, 7]");
      m.el[e].N[d] = deg[e][d] + 1;
    }
    m.el[e].off = m.ndof;
    m.ndof += (long long)m.el[e].N[0] * m.el[e].N[1] * m.el[e].N[2];
  }
  // face neighbours: probe the four quarter points of every face just
  // outside it (two-to-one balance allows at most two neighbours per face
  // dimension)
  m.nbr.resize(m.E());
  for (int e = 0; e < m.E(); ++e) {
    const HElem& E = m.el[e];
    for (int f = 0; f < 6; ++f) {
      const int d = kFaceDim[f], s = face_sign(f);
      std::vector<int>& out = m.nbr[e][f];
      if ((s > 0 && E.hi[d] == m.blocks[d] * m.R[d]) || (s < 0 && E.lo[d] == 0)) continue;
      const int t0 = tdim0(d), t1 = tdim1(d);
      for (int q0 = 0; q0 < 2; ++q0)
        for (int q1 = 0; q1 < 2; ++q1) {
          long long x[3];
          x[d] = s > 0 ? E.hi[d] : E.lo[d] - 1;
          x[t0] = E.lo[t0] + (2 * q0 + 1) * (E.hi[t0] - E.lo[t0]) / 4;
          x[t1] = E.lo[t1] + (2 * q1 + 1) * (E.hi[t1] - E.lo[t1]) / 4;
          const int g = m.find(x);
          if (g < 0) throw DgsError(DGS_ERR_INVALID, "hp mesh: face neighbour not found");
          if (std::find(out.begin(), out.end(), g) == out.end()) out.push_back(g);
        }
      std::sort(out.begin(), out.end());
      for (int g : out)
        for (int t : {t0, t1})
          if (std::abs(m.el[g].L[t] - E.L[t]) > 1)
            throw DgsError(DGS_ERR_INVALID, "hp mesh is not two-to-one balanced");
    }
  }
  return m;
}

// ---------------------------------------------------------------------------
// Face terms (mortars)
// ---------------------------------------------------------------------------
void build_terms(const HMesh& m, double C, MatPool& pool, std::vector<HpElem>& hel,
                 std::vector<HpTerm>& terms) {
  hel.assign(m.E(), HpElem{});
  terms.clear();
  for (int e = 0; e < m.E(); ++e) {
    const HElem& E = m.el[e];
    HpElem& H = hel[e];
    H.off = E.off;
    for (int d = 0; d < 3; ++d) {
      H.N[d] = E.N[d];
      H.rh[d] = 2.0 / E.h[d];
    }
    H.jac = E.h[0] * E.h[1] * E.h[2] / 8.0;
    H.term0 = (int)terms.size();
    for (int f = 0; f < 6; ++f) {
      const int d = kFaceDim[f];
      const int t0 = tdim0(d), t1 = tdim1(d);
      const auto& nb = m.nbr[e][f];
      if (nb.empty()) {
        HpTerm T{};
        T.nb = ((m.neumann >> f) & 1) ? kHpNeumann : kHpDirichlet;
        T.A0 = T.A1 = T.B0 = T.B1 = -1;
        T.sigma = C * E.N[d] * E.N[d] / E.h[d];
        T.direct = 1;
        terms.push_back(T);
        H.nterm[f] = 1;
        continue;
      }
      H.nterm[f] = (int)nb.size();
      for (int g : nb) {
        const HElem& F = m.el[g];
        HpTerm T{};
        T.nb = g;
        T.sigma = C * std::pow((double)std::max(E.N[d], F.N[d]), 2) / std::min(E.h[d], F.h[d]);
        T.foff = F.off;
        for (int q = 0; q < 3; ++q) T.fN[q] = F.N[q];
        T.frh = 2.0 / F.h[d];
        int* As[2] = {&T.A0, &T.A1};
        int* Bs[2] = {&T.B0, &T.B1};
        const int ts[2] = {t0, t1};
        bool identity = true;
        for (int k = 0; k < 2; ++k) {
          const int t = ts[k];
          const long long a = std::max(E.lo[t], F.lo[t]), b = std::min(E.hi[t], F.hi[t]);
          const int M = std::max(E.N[t], F.N[t]);
          const std::vector<double>& eta = lgl(M);
          // interpolation of side G's face points to the mortar points (M x N_G),
          // empty for the identity
          auto interp = [&](const HElem& G, double& al, double& be) {
            const double w = (double)(G.hi[t] - G.lo[t]);
            al = -1.0 + 2.0 * (a - G.lo[t]) / w;
            be = -1.0 + 2.0 * (b - G.lo[t]) / w;
            if (M == G.N[t] && al == -1.0 && be == 1.0) return std::vector<double>();
            std::vector<double> x(M);
            for (int q = 0; q < M; ++q) x[q] = al + (be - al) * (eta[q] + 1.0) / 2.0;
            return lagrange(lgl(G.N[t]), x);
          };
          double ale, bee, alf, bef;
          const std::vector<double> Ie = interp(E, ale, bee), If = interp(F, alf, bef);
          const int NE = E.N[t], NF = F.N[t];
          if (Ie.empty() && If.empty()) {
            *As[k] = *Bs[k] = -1;
            continue;
          }
          identity = false;
          // P = Mex(N_E)^-1 Ie^T Mex(M) (be - al) / 2, N_E x M (Ie empty: M = N_E, Ie = I)
          const std::vector<double> Mm = exact_mass(M);
          std::vector<double> rhs(NE * M, 0.0);
          for (int i = 0; i < NE; ++i)
            for (int j = 0; j < M; ++j) {
              double v = 0.0;
              for (int q = 0; q < M; ++q) v += (Ie.empty() ? (q == i ? 1.0 : 0.0) : Ie[q * NE + i]) * Mm[q * M + j];
              rhs[i * M + j] = v * (bee - ale) / 2.0;
            }
          const std::vector<double> P = solve_dense(exact_mass(NE), rhs, NE, M);
          auto times = [&](const std::vector<double>& I, int NG) {
            std::vector<double> out(NE * NG, 0.0);
            for (int i = 0; i < NE; ++i)
              for (int j = 0; j < NG; ++j) {
                double v = 0.0;
                for (int q = 0; q < M; ++q) v += P[i * M + q] * (I.empty() ? (q == j ? 1.0 : 0.0) : I[q * NG + j]);
                out[i * NG + j] = v;
              }
            return out;
          };
          *As[k] = pool.add(times(Ie, NE));
          *Bs[k] = pool.add(times(If, NF));
        }
        T.direct = identity ? 1 : 0;
        terms.push_back(T);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Levels
// ---------------------------------------------------------------------------
struct HpLevel {
  HMesh mesh;
  std::vector<HpElem> hel;
  std::vector<HpTerm> terms;
  HpElem* d_el = nullptr;
  HpTerm* d_terms = nullptr;
  std::vector<int> order;  // launch order of the operator: most mortar terms first
  int* d_order = nullptr;
  double *r = nullptr, *b = nullptr, *u = nullptr;
  // Schwarz
  std::vector<ClassInfo> cls;
  ClassInfo* d_cls = nullptr;
  std::vector<HpSub> subs;
  HpSub* d_subs = nullptr;
  long long* d_gidx = nullptr;
  // per point, the subdomain row positions that hold it (the gather pushed
  // from the residual kernel)
  long long* d_push_ptr = nullptr;
  long long* d_push_pos = nullptr;
  long long* d_pull_ptr = nullptr;
  HpPull* d_pull = nullptr;
  bool f32 = false;  // FP32 subdomain rows, inverses and GEMM (mixed precision)
  void *rs = nullptr, *du = nullptr;
  long long rs_total = 0;
  GemmTile* d_tiles = nullptr;
  int ntiles = 0, kparts = 1, variant = 2;
  bool small = false;
  // transfer to the next coarser level
  HpChild* d_child = nullptr;
  int* d_kid_ptr = nullptr;
  int* d_kids = nullptr;
};

int overlap_layers(int N, int overlap) { return std::max(1, std::min(overlap, N - 1)); }

double smoothstep(double x) {
  if (x > 1.0) return 1.0;
  if (x < -1.0) return -1.0;
  const double x2 = x * x;
  return x * (15.0 - 10.0 * x2 + 3.0 * x2 * x2) / 8.0;
}

// A point's own Schwarz weight factor along d (eq. schwarz_weight_function)
// and the parts of the remainder on its low and high sides.
struct Factor {
  std::vector<double> a, low, high;
};
Factor own_factor(const HMesh& m, int e, int d, int overlap) {
  const int N = m.el[e].N[d];
  const std::vector<double>& xi = lgl(N);
  const double delta = 1.0 + xi[overlap_layers(N, overlap)];
  const bool lo_ext = m.nbr[e][2 * d].empty(), hi_ext = m.nbr[e][2 * d + 1].empty();
  Factor F;
  for (int i = 0; i < N; ++i) {
    const double lo = lo_ext ? 1.0 : smoothstep((xi[i] + 1.0) / delta);
    const double hi = hi_ext ? -1.0 : smoothstep((xi[i] - 1.0) / delta);
    F.a.push_back(0.5 * (lo - hi));
    F.low.push_back(0.5 * (1.0 - lo));
    F.high.push_back(0.5 * (1.0 + hi));
  }
  return F;
}
double edge_share(double aj, double ak) {
  const double bj = 1.0 - aj, bk = 1.0 - ak;
  return aj * ak + 0.5 * bj * ak + 0.5 * aj * bk + bj * bk / 3.0;
}

int node_of(int d, int od, int b0, int b1, const int N[3]) {
  int idx[3];
  idx[d] = od;
  idx[tdim0(d)] = b0;
  idx[tdim1(d)] = b1;
  return (idx[2] * N[1] + idx[1]) * N[0] + idx[0];
}

// Subdomain of element e: (element, node) per row and the weights.
struct SubLayout {
  std::vector<int> elem, node;
  std::vector<double> w;
};
SubLayout sub_layout(const HMesh& m, int e, int overlap, std::vector<std::array<Factor, 3>>& fac) {
  SubLayout S;
  const HElem& E = m.el[e];
  for (int k = 0; k < E.N[2]; ++k)
    for (int j = 0; j < E.N[1]; ++j)
      for (int i = 0; i < E.N[0]; ++i) {
        S.elem.push_back(e);
        S.node.push_back((k * E.N[1] + j) * E.N[0] + i);
        S.w.push_back(fac[e][0].a[i] * fac[e][1].a[j] * fac[e][2].a[k]);
      }
  for (int f = 0; f < 6; ++f) {
    const int d = kFaceDim[f], s = face_sign(f);
    const int t0 = tdim0(d), t1 = tdim1(d);
    for (int g : m.nbr[e][f]) {
      const HElem& G = m.el[g];
      const int nov = overlap_layers(G.N[d], overlap);
      const double cnt = (double)m.nbr[g][f ^ 1].size();
      for (int layer = 0; layer < nov; ++layer) {
        const int od = s > 0 ? layer : G.N[d] - 1 - layer;
        const double part = s > 0 ? fac[g][d].low[od] : fac[g][d].high[od];
        for (int b1 = 0; b1 < G.N[t1]; ++b1)
          for (int b0 = 0; b0 < G.N[t0]; ++b0) {
            S.elem.push_back(g);
            S.node.push_back(node_of(d, od, b0, b1, G.N));
            S.w.push_back(part * edge_share(fac[g][t0].a[b0], fac[g][t1].a[b1]) / cnt);
          }
      }
    }
  }
  return S;
}

// Patch of subdomain e: the element and its face neighbours, with their face
// terms pointing at patch-local elements (others become zero neighbours).
struct Patch {
  std::vector<int> elems;
  std::vector<HpElem> hel;
  std::vector<HpTerm> terms;
  long long ndof = 0;
};
Patch make_patch(const HMesh& m, const std::vector<HpElem>& hel, const std::vector<HpTerm>& terms, int e) {
  Patch P;
  P.elems.push_back(e);
  for (int f = 0; f < 6; ++f)
    for (int g : m.nbr[e][f]) P.elems.push_back(g);
  std::map<int, int> local;
  for (int i = 0; i < (int)P.elems.size(); ++i) local[P.elems[i]] = i;
  std::vector<long long> loff(P.elems.size());  // patch-local first nodes
  {
    long long o = 0;
    for (size_t i = 0; i < P.elems.size(); ++i) {
      const HpElem& H = hel[P.elems[i]];
      loff[i] = o;
      o += (long long)H.N[0] * H.N[1] * H.N[2];
    }
  }
  for (int g : P.elems) {
    HpElem H = hel[g];
    H.off = P.ndof;
    P.ndof += (long long)H.N[0] * H.N[1] * H.N[2];
    const int t0 = H.term0;
    int nt = 0;
    for (int f = 0; f < 6; ++f) nt += H.nterm[f];
    H.term0 = (int)P.terms.size();
    for (int q = 0; q < nt; ++q) {
      HpTerm T = terms[t0 + q];
      if (T.nb >= 0) {
        auto it = local.find(T.nb);
        T.nb = it == local.end() ? kHpZero : it->second;
        T.foff = T.nb >= 0 ? loff[T.nb] : 0;
      }
      P.terms.push_back(T);
    }
    P.hel.push_back(H);
  }
  return P;
}



// Frames of the symmetry group of axis-aligned boxes: new axis a is old axis
// perm[a], reversed when mir[a].  The DG operator, the LGL points, the
// weights and the mortar rules are invariant under these maps, so subdomains
// that coincide after one of them share A_S up to the order of their rows.
struct Frame {
  int perm[3];
  int mir[3];
};
std::vector<Frame> all_frames() {
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  std::vector<Frame> out;
  for (auto& p : perms)
    for (int mm = 0; mm < 8; ++mm) {
      Frame T;
      for (int a = 0; a < 3; ++a) {
        T.perm[a] = p[a];
        T.mir[a] = (mm >> a) & 1;
      }
      out.push_back(T);
    }
  return out;
}
// the old face that new face fn of a frame is
int old_face(const Frame& T, int fn) {
  const int a = fn >> 1;
  const int s = (fn & 1) ? 1 : -1;
  const int so = T.mir[a] ? -s : s;
  return 2 * T.perm[a] + (so > 0 ? 1 : 0);
}
// old node of the node with new indices inew of an element with old extents N
int old_node(const Frame& T, const int N[3], const int inew[3]) {
  int io[3];
  for (int a = 0; a < 3; ++a) {
    const int d = T.perm[a];
    io[d] = T.mir[a] ? N[d] - 1 - inew[a] : inew[a];
  }
  return (io[2] * N[1] + io[1]) * N[0] + io[0];
}

struct FrameView {
  const HMesh& m;
  int e;
  Frame T;
  double unit[3];  // physical length of one integer unit per old axis (halved)
  // box of g relative to the centre of e, in the new frame (physical units)
  void box(int g, double lo[3], double hi[3]) const {
    const HElem &E = m.el[e], &G = m.el[g];
    for (int a = 0; a < 3; ++a) {
      const int d = T.perm[a];
      const long long c2 = E.lo[d] + E.hi[d];
      long long l = 2 * G.lo[d] - c2, h = 2 * G.hi[d] - c2;
      if (T.mir[a]) {
        const long long t = -l;
        l = -h;
        h = t;
      }
      lo[a] = l * unit[d];
      hi[a] = h * unit[d];
    }
  }
  int Nn(int g, int a) const { return m.el[g].N[T.perm[a]]; }
  // neighbours of g across new face fn, ordered by their boxes in the new frame
  std::vector<int> nbrs(int g, int fn) const {
    std::vector<int> v = m.nbr[g][old_face(T, fn)];
    std::vector<std::array<double, 3>> key(v.size());
    for (size_t i = 0; i < v.size(); ++i) {
      double lo[3], hi[3];
      box(v[i], lo, hi);
      key[i] = {lo[2], lo[1], lo[0]};
    }
    std::vector<size_t> idx(v.size());
    for (size_t i = 0; i < v.size(); ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return key[a] < key[b]; });
    std::vector<int> out;
    for (size_t i : idx) out.push_back(v[i]);
    return out;
  }
};

// The structure of subdomain e seen in frame T (everything that decides A_S
// in that frame's row order): the patch (the centre and its face
// neighbours) with boxes, points and the face data of each patch element,
// except the faces of the neighbours that point away from the centre (the
// subdomain's values vanish on them and beyond, so they reach no row).
std::vector<double> frame_signature(const FrameView& V, std::vector<int>& patch) {
  const HMesh& m = V.m;
  patch.assign(1, V.e);
  std::vector<int> via(1, -1);
  for (int fn = 0; fn < 6; ++fn)
    for (int g : V.nbrs(V.e, fn)) {
      patch.push_back(g);
      via.push_back(fn);
    }
  std::vector<double> v;
  auto put_elem = [&](int g) {
    double lo[3], hi[3];
    V.box(g, lo, hi);
    for (int a = 0; a < 3; ++a) v.push_back(lo[a]), v.push_back(hi[a]), v.push_back(V.Nn(g, a));
  };
  for (size_t i = 0; i < patch.size(); ++i) {
    const int g = patch[i];
    put_elem(g);
    for (int fn = 0; fn < 6; ++fn) {
      if (via[i] == fn) {
        v.push_back(-7.0);
        continue;
      }
      const std::vector<int> nb = V.nbrs(g, fn);
      if (nb.empty()) {
        v.push_back(((m.neumann >> old_face(V.T, fn)) & 1) ? -2.0 : -1.0);
        continue;
      }
      v.push_back((double)nb.size());
      for (int k : nb) {
        const auto it = std::find(patch.begin(), patch.end(), k);
        if (it != patch.end() && (size_t)(it - patch.begin()) < patch.size()) {
          v.push_back(-1000.0 - (double)(it - patch.begin()));
        } else {
          v.push_back(-3.0);
          put_elem(k);
        }
      }
    }
  }
  return v;
}

// Rows of subdomain e in frame T: the centre's points in the new [k][j][i]
// order, then per new face the neighbours in frame order, N_ov layers each,
// layer 0 nearest the face, the lower new transverse dimension fastest.
void frame_rows(const FrameView& V, int overlap, std::vector<int>& elem, std::vector<int>& node) {
  const HMesh& m = V.m;
  const int e = V.e;
  elem.clear();
  node.clear();
  int n[3] = {V.Nn(e, 0), V.Nn(e, 1), V.Nn(e, 2)};
  for (int k = 0; k < n[2]; ++k)
    for (int j = 0; j < n[1]; ++j)
      for (int i = 0; i < n[0]; ++i) {
        const int inew[3] = {i, j, k};
        elem.push_back(e);
        node.push_back(old_node(V.T, m.el[e].N, inew));
      }
  for (int fn = 0; fn < 6; ++fn) {
    const int a = fn >> 1, s = (fn & 1) ? 1 : -1;
    const int t0 = a == 0 ? 1 : 0, t1 = a == 2 ? 1 : 2;
    for (int g : V.nbrs(e, fn)) {
      const int Na = V.Nn(g, a);
      const int nov = overlap_layers(Na, overlap);
      for (int layer = 0; layer < nov; ++layer)
        for (int b1 = 0; b1 < V.Nn(g, t1); ++b1)
          for (int b0 = 0; b0 < V.Nn(g, t0); ++b0) {
            int inew[3];
            inew[a] = s > 0 ? layer : Na - 1 - layer;
            inew[t0] = b0;
            inew[t1] = b1;
            elem.push_back(g);
            node.push_back(old_node(V.T, m.el[g].N, inew));
          }
    }
  }
}

// Canonical form of subdomain e: the smallest signature over the frames (a
// cheap key of the centre alone selects the candidate frames first), its
// rows in that frame with their weights, and the patch elements.
std::string canonical_subdomain(const HMesh& m, int e, int overlap, const SubLayout& own,
                                SubLayout& rows, std::vector<int>& patch) {
  static const std::vector<Frame> frames = all_frames();
  double unit[3];
  for (int d = 0; d < 3; ++d) unit[d] = 0.5 * (m.upper[d] - m.lower[d]) / m.blocks[d] / (double)m.R[d];
  std::vector<std::vector<double>> small(frames.size());
  for (size_t f = 0; f < frames.size(); ++f) {
    FrameView V{m, e, frames[f], {unit[0], unit[1], unit[2]}};
    std::vector<double>& k = small[f];
    for (int a = 0; a < 3; ++a) k.push_back(V.Nn(e, a)), k.push_back(m.el[e].h[frames[f].perm[a]]);
    for (int fn = 0; fn < 6; ++fn) {
      const auto& nb = m.nbr[e][old_face(frames[f], fn)];
      k.push_back(nb.empty() ? (((m.neumann >> old_face(frames[f], fn)) & 1) ? -2.0 : -1.0) : (double)nb.size());
      for (int g : nb) k.push_back(m.el[g].N[frames[f].perm[fn >> 1]]);
    }
  }
  const std::vector<double> kmin = *std::min_element(small.begin(), small.end());
  std::vector<double> best;
  int bestf = -1;
  std::vector<int> bestpatch;
  for (size_t f = 0; f < frames.size(); ++f) {
    if (small[f] != kmin) continue;
    FrameView V{m, e, frames[f], {unit[0], unit[1], unit[2]}};
    std::vector<int> pt;
    std::vector<double> sig = frame_signature(V, pt);
    if (bestf < 0 || sig < best) {
      best = std::move(sig);
      bestf = (int)f;
      bestpatch = std::move(pt);
    }
  }
  FrameView V{m, e, frames[bestf], {unit[0], unit[1], unit[2]}};
  frame_rows(V, overlap, rows.elem, rows.node);
  // weights of the points, from the subdomain's own layout
  std::map<std::pair<int, int>, double> w;
  for (size_t r = 0; r < own.elem.size(); ++r) w[{own.elem[r], own.node[r]}] = own.w[r];
  rows.w.resize(rows.elem.size());
  for (size_t r = 0; r < rows.elem.size(); ++r) {
    const auto it = w.find({rows.elem[r], rows.node[r]});
    if (it == w.end()) throw DgsError(DGS_ERR_HIP, "hp subdomain rows do not match their layout");
    rows.w[r] = it->second;
  }
  patch = std::move(bestpatch);
  return std::string(reinterpret_cast<const char*>(best.data()), best.size() * sizeof(double));
}
}  // namespace

struct dgs_hp_problem {
  dgs_options opt{};
  double penalty = 0;
  std::vector<std::unique_ptr<HpLevel>> lv;
  MatPool pool;
  double* d_pool = nullptr;
  HpRule rule{};
  std::vector<void*> allocations;
  KrylovSpace K;
  double t_setup = 0;
  // the V-cycle captured at set-up (input in the finest level's b, output in
  // its u) and the capture stream
  hipGraphExec_t vgraph = nullptr;
  hipStream_t cap_stream = nullptr;

  template <typename T>
  T* alloc(size_t count) {
    T* p = dalloc<T>(count);
    allocations.push_back(p);
    return p;
  }
  ~dgs_hp_problem() {
    std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
    if (vgraph) (void)hipGraphExecDestroy(vgraph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (void* p : allocations) (void)hipFree(p);
    if (K.pinned) (void)hipHostFree(K.pinned);
  }
};

namespace {

void upload_level_mesh(dgs_hp_problem* P, HpLevel& L, hipStream_t s) {
  L.d_el = P->alloc<HpElem>(L.hel.size());
  upload(L.d_el, L.hel, s);
  L.d_terms = P->alloc<HpTerm>(L.terms.size());
  upload(L.d_terms, L.terms, s);
  // an element's work grows with its mortar terms (each a serial chain of
  // tensor passes) and its points: the costly ones are launched first
  const int E = (int)L.hel.size();
  std::vector<int>& order = L.order;  // kept: the upload may still read it
  order.resize(E);
  std::vector<long long> cost(E);
  for (int e = 0; e < E; ++e) {
    const HpElem& H = L.hel[e];
    long long c = (long long)H.N[0] * H.N[1] * H.N[2];
    for (int f = 0, t = H.term0; f < 6; t += H.nterm[f], ++f)
      if (!L.terms[t].direct) c += 512LL * H.nterm[f];
    order[e] = e;
    cost[e] = c;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  L.d_order = P->alloc<int>(E);
  upload(L.d_order, order, s);
  L.r = P->alloc<double>(L.mesh.ndof);
  L.b = P->alloc<double>(L.mesh.ndof);
  L.u = P->alloc<double>(L.mesh.ndof);
}

// Subdomain classes, gather/scatter tables and the explicit inverses of one
// level (Sec. III.D.1-4, III.E.2).
void build_schwarz(dgs_hp_problem* P, HpLevel& L, hipStream_t s) {
  const HMesh& m = L.mesh;
  const int overlap = P->opt.overlap;
  std::vector<std::array<Factor, 3>> fac(m.E());
  for (int e = 0; e < m.E(); ++e)
    for (int d = 0; d < 3; ++d) fac[e][d] = own_factor(m, e, d, overlap);
  std::vector<SubLayout> lay(m.E());
  std::map<std::string, int> class_of;
  std::vector<std::vector<int>> members;
  std::vector<Patch> rep;
  for (int e = 0; e < m.E(); ++e) {
    const SubLayout own = sub_layout(m, e, overlap, fac);
    std::vector<int> pe;
    const std::string key = canonical_subdomain(m, e, overlap, own, lay[e], pe);
    auto it = class_of.find(key);
    if (it == class_of.end()) {
      it = class_of.emplace(key, (int)members.size()).first;
      members.emplace_back();
      rep.push_back(make_patch(m, L.hel, L.terms, e));
    }
    members[it->second].push_back(e);
  }
  const int nc = (int)members.size();
  // gather block: class-major, one row of ld entries per subdomain
  L.cls.assign(nc, ClassInfo{});
  long long rs_off = 0;
  for (int c = 0; c < nc; ++c) {
    ClassInfo& I = L.cls[c];
    I.n = (int)lay[members[c][0]].elem.size();
    I.count = (int)members[c].size();
    I.ld = (I.n + kGemmLd - 1) / kGemmLd * kGemmLd;
    I.rows = (I.count + kGemmRows - 1) / kGemmRows * kGemmRows;
    I.kext = (I.n + 31) / 32 * 32;
    I.scale = I.scale_op = 1.0;
    I.rs_off = rs_off;
    for (int& so : I.strip_off) so = -1;
    rs_off += (long long)I.rows * I.ld;
  }
  L.rs_total = rs_off;
  std::vector<long long> gidx;
  std::vector<std::vector<HpPull>> pulls(m.ndof);
  L.subs.clear();
  for (int c = 0; c < nc; ++c)
    for (int i = 0; i < (int)members[c].size(); ++i) {
      const int e = members[c][i];
      const SubLayout& S = lay[e];
      HpSub sub;
      sub.rs = L.cls[c].rs_off + (long long)i * L.cls[c].ld;
      sub.start = (int)gidx.size();
      sub.n = (int)S.elem.size();
      for (int q = 0; q < sub.n; ++q) {
        const long long g = m.el[S.elem[q]].off + S.node[q];
        gidx.push_back(g);
        pulls[g].push_back(HpPull{sub.rs + q, S.w[q]});
      }
      L.subs.push_back(sub);
    }
  std::vector<long long> ptr(m.ndof + 1, 0);
  std::vector<HpPull> flat;
  for (long long p = 0; p < m.ndof; ++p) {
    ptr[p + 1] = ptr[p] + (long long)pulls[p].size();
    flat.insert(flat.end(), pulls[p].begin(), pulls[p].end());
  }
  L.d_subs = P->alloc<HpSub>(L.subs.size());
  upload(L.d_subs, L.subs, s);
  L.d_gidx = P->alloc<long long>(gidx.size());
  upload(L.d_gidx, gidx, s);
  L.d_pull_ptr = P->alloc<long long>(ptr.size());
  upload(L.d_pull_ptr, ptr, s);
  L.d_pull = P->alloc<HpPull>(flat.size());
  upload(L.d_pull, flat, s);
  // the same row positions grouped by point: pos = sub.rs + q for point gidx
  std::vector<long long> pptr(m.ndof + 1, 0), ppos(gidx.size());
  for (long long g : gidx) ++pptr[g + 1];
  for (long long p = 0; p < m.ndof; ++p) pptr[p + 1] += pptr[p];
  {
    std::vector<long long> fill(pptr.begin(), pptr.end() - 1);
    for (const HpSub& sub : L.subs)
      for (int q = 0; q < sub.n; ++q) ppos[fill[gidx[sub.start + q]]++] = sub.rs + q;
  }
  L.d_push_ptr = P->alloc<long long>(pptr.size());
  upload(L.d_push_ptr, pptr, s);
  L.d_push_pos = P->alloc<long long>(ppos.size());
  upload(L.d_push_pos, ppos, s);
  HIP_OK(hipStreamSynchronize(s));

  // explicit inverses: A_S assembled column by column by the operator kernel
  // on copies of the class patch, then blocked Gauss-Jordan elimination
  // (no pivoting; the symmetric part of A_S dominates)
  std::vector<void*> inv(nc, nullptr);
  std::vector<int> order(nc);
  for (int c = 0; c < nc; ++c) order[c] = c;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return L.cls[a].n < L.cls[b].n; });
  size_t pos = 0;
  while (pos < order.size()) {
    const int n_pad = (L.cls[order[pos]].n + 63) / 64 * 64;
    std::vector<int> group;
    const size_t cap = std::max<size_t>(1, (size_t)(1u << 30) / ((size_t)n_pad * n_pad * 8));
    while (pos < order.size() && (L.cls[order[pos]].n + 63) / 64 * 64 == n_pad && group.size() < cap)
      group.push_back(order[pos++]);
    const int nk = (int)group.size();
    double* batch = dalloc<double>((size_t)nk * n_pad * n_pad);
    std::unique_ptr<void, void (*)(void*)> g1(batch, dfree);
    HIP_OK(hipMemsetAsync(batch, 0, (size_t)nk * n_pad * n_pad * sizeof(double), s));
    {
      std::vector<int> iota(n_pad);
      for (int i = 0; i < n_pad; ++i) iota[i] = i;
      int* d_iota = dalloc<int>(n_pad);
      std::unique_ptr<void, void (*)(void*)> g2(d_iota, dfree);
      upload(d_iota, iota, s);
      for (int k = 0; k < nk; ++k)
        HIP_OK(launch_unit_columns(batch + (size_t)k * n_pad * n_pad, n_pad, d_iota, n_pad, s));
      HIP_OK(hipStreamSynchronize(s));
    }
    for (int k = 0; k < nk; ++k) {
      const int c = group[k];
      const Patch& Pt = rep[c];
      const SubLayout& S = lay[members[c][0]];
      const int n = L.cls[c].n;
      std::map<int, long long> loff;
      for (size_t i = 0; i < Pt.elems.size(); ++i) loff[Pt.elems[i]] = Pt.hel[i].off;
      std::vector<int> idx(n);
      for (int r = 0; r < n; ++r) idx[r] = (int)(loff[S.elem[r]] + S.node[r]);
      HpElem* d_pel = dalloc<HpElem>(Pt.hel.size());
      std::unique_ptr<void, void (*)(void*)> g3(d_pel, dfree);
      HpTerm* d_pt = dalloc<HpTerm>(Pt.terms.size());
      std::unique_ptr<void, void (*)(void*)> g4(d_pt, dfree);
      int* d_idx = dalloc<int>(n);
      std::unique_ptr<void, void (*)(void*)> g5(d_idx, dfree);
      const long long tot = Pt.ndof * n;
      double* X = dalloc<double>(tot);
      std::unique_ptr<void, void (*)(void*)> g6(X, dfree);
      double* AX = dalloc<double>(tot);
      std::unique_ptr<void, void (*)(void*)> g7(AX, dfree);
      upload(d_pel, Pt.hel, s);
      upload(d_pt, Pt.terms, s);
      upload(d_idx, idx, s);
      HIP_OK(launch_fill(X, 0.0, tot, s));
      HIP_OK(launch_unit_columns(X, Pt.ndof, d_idx, n, s));
      HIP_OK(launch_hp_apply(false, X, AX, nullptr, d_pel, (int)Pt.hel.size(), d_pt, P->d_pool, P->rule,
                             n, Pt.ndof, s));
      HIP_OK(launch_gather_columns(AX, Pt.ndof, d_idx, n, batch + (size_t)k * n_pad * n_pad, n_pad, s));
      HIP_OK(hipStreamSynchronize(s));
    }
    double* dP = dalloc<double>((size_t)nk * 64 * 64);
    std::unique_ptr<void, void (*)(void*)> g8(dP, dfree);
    double* dR = dalloc<double>((size_t)nk * 64 * n_pad);
    std::unique_ptr<void, void (*)(void*)> g9(dR, dfree);
    double* dC = dalloc<double>((size_t)nk * 64 * n_pad);
    std::unique_ptr<void, void (*)(void*)> g10(dC, dfree);
    HIP_OK(launch_block_inverse(batch, n_pad, nk, dP, dR, dC, s));
    for (int k = 0; k < nk; ++k) {
      const int c = group[k];
      const size_t nn = (size_t)L.cls[c].ld * L.cls[c].ld;
      const size_t es = L.f32 ? sizeof(float) : sizeof(double);
      inv[c] = P->alloc<char>(nn * es);
      HIP_OK(hipMemsetAsync(inv[c], 0, nn * es, s));
      HIP_OK(launch_finish_inverse(batch + (size_t)k * n_pad * n_pad, n_pad, L.cls[c].n, L.cls[c].ld, 1.0,
                                   L.f32 ? nullptr : (double*)inv[c], L.f32 ? (float*)inv[c] : nullptr,
                                   s));
    }
    HIP_OK(hipStreamSynchronize(s));
  }
  for (int c = 0; c < nc; ++c) L.cls[c].inv = inv[c];
  L.d_cls = P->alloc<ClassInfo>(nc);
  upload(L.d_cls, L.cls, s);
  // at most 4 split-K parts: the scatter sums every part of every entry
  GemmPlan plan = plan_subdomain_gemm(L.cls, L.variant, 4);
  L.small = plan.small;
  L.kparts = plan.kparts;
  L.ntiles = (int)plan.tiles.size();
  L.d_tiles = P->alloc<GemmTile>(plan.tiles.size());
  upload(L.d_tiles, plan.tiles, s);
  const size_t es = L.f32 ? sizeof(float) : sizeof(double);
  L.rs = P->alloc<char>(L.rs_total * es);
  L.du = P->alloc<char>(L.rs_total * L.kparts * es);
  HIP_OK(hipMemsetAsync(L.rs, 0, L.rs_total * es, s));
  HIP_OK(hipMemsetAsync(L.du, 0, L.rs_total * L.kparts * es, s));
  HIP_OK(hipStreamSynchronize(s));
}

// Coarser mesh (Sec. III.C.1): every block halved along its split
// dimensions, merged elements keeping the smaller degree per dimension.
bool coarsen(const HMesh& fine, HMesh& coarse, std::vector<int>& parent, std::vector<std::array<int, 3>>& pos) {
  bool any = false;
  std::vector<std::array<int, 3>> cl = fine.blev;
  for (auto& L : cl)
    for (int d = 0; d < 3; ++d)
      if (L[d] > 0) {
        --L[d];
        any = true;
      }
  if (!any) return false;
  // coarse element numbering: block by block, x fastest
  std::vector<int> cstart;
  int Ec = 0;
  for (auto& L : cl) {
    cstart.push_back(Ec);
    Ec += 1 << (L[0] + L[1] + L[2]);
  }
  std::vector<std::array<int, 3>> deg(Ec, std::array<int, 3>{1 << 20, 1 << 20, 1 << 20});
  parent.assign(fine.E(), 0);
  pos.assign(fine.E(), std::array<int, 3>{-1, -1, -1});
  for (int e = 0; e < fine.E(); ++e) {
    const HElem& E = fine.el[e];
    const int b = E.block;
    int idx[3], cidx[3];
    const int n[3] = {1 << fine.blev[b][0], 1 << fine.blev[b][1], 1 << fine.blev[b][2]};
    const int local = e - fine.bstart[b];
    idx[0] = local % n[0];
    idx[1] = (local / n[0]) % n[1];
    idx[2] = local / (n[0] * n[1]);
    for (int d = 0; d < 3; ++d) {
      const bool split = fine.blev[b][d] > 0;
      cidx[d] = split ? idx[d] / 2 : idx[d];
      pos[e][d] = split ? idx[d] % 2 : -1;
    }
    const int cn[3] = {1 << cl[b][0], 1 << cl[b][1], 1 << cl[b][2]};
    const int c = cstart[b] + (cidx[2] * cn[1] + cidx[1]) * cn[0] + cidx[0];
    parent[e] = c;
    for (int d = 0; d < 3; ++d) deg[c][d] = std::min(deg[c][d], E.N[d] - 1);
  }
  coarse = make_mesh(fine.lower, fine.upper, fine.blocks, cl, deg, fine.neumann);
  return true;
}

void build_transfer(dgs_hp_problem* P, HpLevel& F, const HpLevel& Cl, const std::vector<int>& parent,
                    const std::vector<std::array<int, 3>>& pos, hipStream_t s) {
  std::vector<HpChild> ch(F.mesh.E());
  std::vector<std::vector<int>> kids(Cl.mesh.E());
  for (int e = 0; e < F.mesh.E(); ++e) {
    ch[e].parent = parent[e];
    kids[parent[e]].push_back(e);
    for (int d = 0; d < 3; ++d) {
      const int Nf = F.mesh.el[e].N[d], Nc = Cl.mesh.el[parent[e]].N[d];
      const std::vector<double>& x = lgl(Nf);
      std::vector<double> t(Nf);
      for (int a = 0; a < Nf; ++a)
        t[a] = pos[e][d] < 0 ? x[a] : (pos[e][d] == 0 ? 0.5 * (x[a] - 1.0) : 0.5 * (x[a] + 1.0));
      ch[e].P[d] = P->pool.add(lagrange(lgl(Nc), t));  // Nf x Nc
    }
  }
  std::vector<int> kp(Cl.mesh.E() + 1, 0), kl;
  for (int c = 0; c < Cl.mesh.E(); ++c) {
    kp[c + 1] = kp[c] + (int)kids[c].size();
    kl.insert(kl.end(), kids[c].begin(), kids[c].end());
  }
  F.d_child = P->alloc<HpChild>(ch.size());
  upload(F.d_child, ch, s);
  F.d_kid_ptr = P->alloc<int>(kp.size());
  upload(F.d_kid_ptr, kp, s);
  F.d_kids = P->alloc<int>(kl.size());
  upload(F.d_kids, kl, s);
  HIP_OK(hipStreamSynchronize(s));
}

void hp_residual(dgs_hp_problem* P, int l, const double* u, const double* b, double* r, hipStream_t s) {
  HpLevel& L = *P->lv[l];
  HIP_OK(launch_hp_apply(true, u, r, b, L.d_el, L.mesh.E(), L.d_terms, P->d_pool, P->rule, 1, 0, s,
                         L.d_order));
}

void hp_apply(dgs_hp_problem* P, int l, const double* u, double* y, hipStream_t s) {
  HpLevel& L = *P->lv[l];
  HIP_OK(launch_hp_apply(false, u, y, nullptr, L.d_el, L.mesh.E(), L.d_terms, P->d_pool, P->rule, 1, 0, s,
                         L.d_order));
}

// Additive Schwarz steps (Sec. III.D.5) on level l: residual, gather into
// the subdomain rows, grouped GEMM with the inverses, weighted scatter.
void hp_schwarz(dgs_hp_problem* P, int l, const double* b, double* u, int steps, bool u_zero,
                hipStream_t s) {
  HpLevel& L = *P->lv[l];
  const long long n = L.mesh.ndof;
  if (u_zero) HIP_OK(launch_fill(u, 0.0, n, s));
  for (int k = 0; k < steps; ++k) {
    if (u_zero && k == 0)  // the residual is b itself
      HIP_OK(launch_hp_gather(L.f32, b, L.rs, L.d_subs, (int)L.subs.size(), L.d_gidx, s));
    else  // the residual written straight into the subdomain rows
      HIP_OK(launch_hp_residual_gather(u, b, L.d_el, L.mesh.E(), L.d_terms, P->d_pool, P->rule,
                                       L.d_order, L.d_push_ptr, L.d_push_pos, L.f32, L.rs, s));
    HIP_OK(launch_subdomain_gemm(L.f32, L.rs, L.du, L.rs_total, L.d_cls, L.d_tiles, L.ntiles, L.small, 0, s,
                                 L.variant));
    HIP_OK(launch_hp_scatter(L.f32, u, L.du, L.kparts, L.rs_total, L.d_pull_ptr, L.d_pull, n, s));
  }
}

// One V-cycle visit of level l (Sec. III.C.3).
void hp_visit(dgs_hp_problem* P, int l, const double* b, double* u, hipStream_t s) {
  const int nl = (int)P->lv.size();
  const int pre = P->opt.pre_smooth, post = P->opt.post_smooth;
  if (l == nl - 1) {
    hp_schwarz(P, l, b, u, pre + post, true, s);
    return;
  }
  hp_schwarz(P, l, b, u, pre, true, s);
  HpLevel& L = *P->lv[l];
  HpLevel& C = *P->lv[l + 1];
  hp_residual(P, l, u, b, L.r, s);
  HIP_OK(launch_hp_restrict(L.r, C.b, L.d_el, C.d_el, L.d_child, L.d_kid_ptr, L.d_kids, C.mesh.E(),
                            P->d_pool, s));
  hp_visit(P, l + 1, C.b, C.u, s);
  HIP_OK(launch_hp_prolongate_add(C.u, u, L.d_el, C.d_el, L.d_child, L.mesh.E(), P->d_pool, s));
  hp_schwarz(P, l, b, u, post, false, s);
}

// Capture one V-cycle from the finest level's b into its u as a hipGraph
// (the launches of a cycle depend only on the problem, so the graph is
// replayed by every preconditioner application).
void hp_capture(dgs_hp_problem* P) {
  std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
  HpLevel& L0 = *P->lv[0];
  if (!P->cap_stream) HIP_OK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
  HIP_OK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
  hipGraph_t graph = nullptr;
  try {
    hp_visit(P, 0, L0.b, L0.u, P->cap_stream);
  } catch (...) {
    (void)hipStreamEndCapture(P->cap_stream, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  HIP_OK(hipStreamEndCapture(P->cap_stream, &graph));
  const hipError_t e = hipGraphInstantiate(&P->vgraph, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIP_OK(e);
}

// z = one V-cycle applied to r: the captured cycle between two copies, or
// the launches themselves without graphs
void hp_precondition(dgs_hp_problem* P, const double* r, double* z, hipStream_t s) {
  if (!P->vgraph) {
    hp_visit(P, 0, r, z, s);
    return;
  }
  HpLevel& L0 = *P->lv[0];
  HIP_OK(launch_copy(L0.b, r, L0.mesh.ndof, s));
  HIP_OK(hipGraphLaunch(P->vgraph, s));
  HIP_OK(launch_copy(z, L0.u, L0.mesh.ndof, s));
}

void hp_ensure_krylov(dgs_hp_problem* P, int m) {
  if (P->K.m >= m) return;
  const long long n = P->lv[0]->mesh.ndof;
  KrylovSpace& K = P->K;
  K.m = m;
  K.n = n;
  K.V = P->alloc<double>((size_t)(m + 1) * n);
  K.Z = P->alloc<double>((size_t)m * n);
  K.partial = P->alloc<double>((size_t)multidot_blocks(n) * (m + 2));
  K.h = P->alloc<double>(3 * (m + 2));
  K.y = P->alloc<double>(m + 1);
  K.tmp = P->alloc<double>(n);
  std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
  if (K.pinned) (void)hipHostFree(K.pinned);
  K.pinned = nullptr;
  HIP_OK(hipHostMalloc((void**)&K.pinned, sizeof(double) * 4 * (m + 2), hipHostMallocDefault));
}

}  // namespace

extern "C" {

int dgs_create_hp_problem(const dgs_domain* domain, const int blocks[3], const int* block_levels,
                          const int* degrees, int num_elements, double penalty, const dgs_options* opt,
                          void* stream, dgs_hp_problem** out) {
  return guarded([&]() -> int {
    if (!domain || !blocks || !block_levels || !degrees || !out) return fail(DGS_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (!(penalty > 0)) return fail(DGS_ERR_INVALID, "penalty must be positive");
    for (int d = 0; d < 3; ++d) {
      if (blocks[d] < 1) return fail(DGS_ERR_INVALID, "block counts must be at least 1");
      if (!(domain->upper[d] > domain->lower[d])) return fail(DGS_ERR_INVALID, "empty box");
    }
    dgs_options o;
    dgs_default_options(&o);
    if (opt) o = *opt;
    if (o.precision != DGS_FP64 && o.precision != DGS_MIXED) return fail(DGS_ERR_INVALID, "unknown precision");
    if (o.cycle != 1 || o.additive != 0) return fail(DGS_ERR_INVALID, "hp meshes use the V-cycle");
    if (o.neumann_faces < 0 || o.neumann_faces >= 63)
      return fail(DGS_ERR_INVALID, "Neumann faces must leave one face Dirichlet");
    if (o.overlap < 1 || o.pre_smooth < 0 || o.post_smooth < 0 || o.max_iter < 1 || !(o.rtol > 0) ||
        o.mg_levels < 0 || o.restart < 0)
      return fail(DGS_ERR_INVALID, "bad options");
    const int nb = blocks[0] * blocks[1] * blocks[2];
    std::vector<std::array<int, 3>> blev(nb);
    long long E = 0;
    for (int b = 0; b < nb; ++b) {
      for (int d = 0; d < 3; ++d) {
        blev[b][d] = block_levels[3 * b + d];
        if (blev[b][d] < 0 || blev[b][d] > 10) return fail(DGS_ERR_INVALID, "block levels must be in [0, 10]");
      }
      E += 1LL << (blev[b][0] + blev[b][1] + blev[b][2]);
    }
    if (E != num_elements) return fail(DGS_ERR_INVALID, "num_elements does not match the block levels");
    std::vector<std::array<int, 3>> deg(E);
    for (long long e = 0; e < E; ++e)
      for (int d = 0; d < 3; ++d) deg[e][d] = degrees[3 * e + d];
    if (E > (1LL << 22)) return fail(DGS_ERR_INVALID, "more than 2^22 hp elements");
    const double t0 = now_s();
    hipStream_t s = as_stream(stream);
    std::unique_ptr<dgs_hp_problem> P(new dgs_hp_problem());
    P->opt = o;
    P->penalty = penalty;
    // host set-up first (meshes, hierarchy, mortars), so that an invalid mesh
    // is refused before any device work
    std::vector<std::vector<int>> parents;
    std::vector<std::vector<std::array<int, 3>>> poss;
    {
      auto L0 = std::make_unique<HpLevel>();
      L0->mesh = make_mesh(domain->lower, domain->upper, blocks, blev, deg, o.neumann_faces);
      P->lv.push_back(std::move(L0));
      const int cap = o.mg_levels > 0 ? o.mg_levels : 64;
      while ((int)P->lv.size() < cap) {
        auto C = std::make_unique<HpLevel>();
        std::vector<int> parent;
        std::vector<std::array<int, 3>> pos;
        if (!coarsen(P->lv.back()->mesh, C->mesh, parent, pos)) break;
        parents.push_back(parent);
        poss.push_back(pos);
        P->lv.push_back(std::move(C));
      }
    }
    for (auto& L : P->lv) build_terms(L->mesh, penalty, P->pool, L->hel, L->terms);
    // the LGL rules for 2..8 points
    {
      std::vector<double> D(7 * 64, 0.0), w(7 * 8, 0.0), xi(7 * 8, 0.0);
      for (int N = 2; N <= kHpMaxN; ++N) {
        const HostTables t = make_tables(N);
        for (int i = 0; i < N * N; ++i) D[(N - 2) * 64 + i] = t.D[i];
        for (int i = 0; i < N; ++i) {
          w[(N - 2) * 8 + i] = t.w[i];
          xi[(N - 2) * 8 + i] = t.xi[i];
        }
      }
      double* dD = P->alloc<double>(D.size());
      double* dw = P->alloc<double>(w.size());
      double* dx = P->alloc<double>(xi.size());
      upload(dD, D, s);
      upload(dw, w, s);
      upload(dx, xi, s);
      P->rule = HpRule{dD, dw, dx};
      HIP_OK(hipStreamSynchronize(s));
    }
    for (size_t l = 0; l + 1 < P->lv.size(); ++l)
      build_transfer(P.get(), *P->lv[l], *P->lv[l + 1], parents[l], poss[l], s);
    P->d_pool = P->alloc<double>(std::max<size_t>(1, P->pool.data.size()));
    upload(P->d_pool, P->pool.data, s);
    for (auto& L : P->lv) upload_level_mesh(P.get(), *L, s);
    HIP_OK(hipStreamSynchronize(s));
    // mixed precision: FP32 subdomain solves on every level but the coarsest
    for (size_t l = 0; l + 1 < P->lv.size(); ++l) P->lv[l]->f32 = o.precision == DGS_MIXED;
    for (auto& L : P->lv) build_schwarz(P.get(), *L, s);
    if (o.use_graphs) hp_capture(P.get());
    P->t_setup = now_s() - t0;
    *out = P.release();
    return DGS_OK;
  });
}

int dgs_destroy_hp_problem(dgs_hp_problem* prob) {
  return guarded([&]() -> int {
    delete prob;
    return DGS_OK;
  });
}

long long dgs_hp_num_dofs(const dgs_hp_problem* prob) { return prob ? prob->lv[0]->mesh.ndof : -1; }

int dgs_hp_num_levels(const dgs_hp_problem* prob) { return prob ? (int)prob->lv.size() : -1; }

int dgs_hp_num_classes(const dgs_hp_problem* prob, int level) {
  if (!prob || level < 0 || level >= (int)prob->lv.size()) return -1;
  return (int)prob->lv[level]->cls.size();
}

int dgs_hp_node_coordinates(dgs_hp_problem* prob, double* xyz, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !xyz) return fail(DGS_ERR_INVALID, "NULL argument");
    hipStream_t s = as_stream(stream);
    HpLevel& L = *prob->lv[0];
    std::vector<double> g;
    for (const HElem& E : L.mesh.el)
      for (double v : {E.plo[0], E.plo[1], E.plo[2], E.h[0], E.h[1], E.h[2]}) g.push_back(v);
    double* d_g = dalloc<double>(g.size());
    std::unique_ptr<void, void (*)(void*)> guard(d_g, dfree);
    upload(d_g, g, s);
    HIP_OK(launch_hp_coords(xyz, L.mesh.ndof, L.d_el, d_g, L.mesh.E(), prob->rule, s));
    HIP_OK(hipStreamSynchronize(s));
    return DGS_OK;
  });
}

int dgs_hp_apply_operator(dgs_hp_problem* prob, const double* u, double* Au, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !u || !Au) return fail(DGS_ERR_INVALID, "NULL argument");
    hp_apply(prob, 0, u, Au, as_stream(stream));
    return DGS_OK;
  });
}

int dgs_hp_apply_mass(dgs_hp_problem* prob, const double* f, double* Mf, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !f || !Mf) return fail(DGS_ERR_INVALID, "NULL argument");
    HpLevel& L = *prob->lv[0];
    HIP_OK(launch_hp_mass(f, Mf, L.d_el, L.mesh.E(), prob->rule, as_stream(stream)));
    return DGS_OK;
  });
}

int dgs_hp_smooth(dgs_hp_problem* prob, const double* b, double* u, int steps, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !b || !u || steps < 0) return fail(DGS_ERR_INVALID, "bad argument");
    hp_schwarz(prob, 0, b, u, steps, false, as_stream(stream));
    return DGS_OK;
  });
}

int dgs_hp_precondition(dgs_hp_problem* prob, const double* r, double* z, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !r || !z) return fail(DGS_ERR_INVALID, "NULL argument");
    hp_precondition(prob, r, z, as_stream(stream));
    return DGS_OK;
  });
}

int dgs_hp_solve(dgs_hp_problem* prob, const double* b, double* u, dgs_stats* stats, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !b || !u) return fail(DGS_ERR_INVALID, "NULL argument");
    const double t0 = now_s();
    hipStream_t s = as_stream(stream);
    const int max_total = prob->opt.max_iter;
    const int m = prob->opt.restart > 0 ? std::min(prob->opt.restart, max_total) : max_total;
    hp_ensure_krylov(prob, m);
    KrylovSpace K = prob->K;
    K.m = m;
    const FgmresResult R = fgmres_run(
        K, prob->opt.rtol, max_total,
        [&](const double* x, const double* bb, double* out) { hp_residual(prob, 0, x, bb, out, s); },
        [&](const double* z, double* w) { hp_apply(prob, 0, z, w, s); },
        [&](const double* v, double* z) { hp_precondition(prob, v, z, s); }, b, u, s);
    if (stats) {
      stats->iterations = R.iterations;
      stats->newton_steps = 0;
      stats->backtracks = 0;
      stats->rel_residual = R.rel_residual;
      stats->t_setup_s = prob->t_setup;
      stats->t_solve_s = now_s() - t0;
      stats->history_len = 0;
      if (stats->history && stats->history_capacity > 0) {
        const int nh = std::min<int>(stats->history_capacity, (int)R.history.size());
        for (int i = 0; i < nh; ++i) stats->history[i] = R.history[i];
        stats->history_len = nh;
      }
    }
    return R.converged ? DGS_OK : DGS_NOT_CONVERGED;
  });
}

}  // extern "C"
