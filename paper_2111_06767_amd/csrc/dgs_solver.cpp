// Host orchestration and C ABI of the gfx950 DG multigrid-Schwarz solver.
//
//   set-up       mesh levels (Sec. III.C.1), Schwarz subdomain classes and
//                layouts (Sec. III.D.1-4), explicit subdomain inverses built on
//                the device column by column (Sec. III.E.2)
//   apply        A u (Sec. II)
//   smooth       additive Schwarz steps (Sec. III.D.5)
//   precondition one multigrid V-cycle (Sec. III.C.3)
//   solve        flexible GMRES (Sec. III.B; Saad Alg. 9.6) with classical
//                Gram-Schmidt applied twice, one host synchronisation per
//                iteration for the Hessenberg column
//   newton_solve Newton-Raphson with backtracking line search (Sec. III.A)
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <condition_variable>
#include <cstring>
#include <exception>
#include <functional>
#include <limits>
#include <map>
#include <unordered_map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/dgsolve.h"
#include "dgs_internal.h"
#include "dgs_curved.h"
#include "dgs_host.h"

using namespace dgs;

namespace {


const int kFace[6][2] = {{0, -1}, {0, 1}, {1, -1}, {1, 1}, {2, -1}, {2, 1}};

// Boundary class: bit f (f = 2 d + side) set when face f of the element is
// external, bit 6 + f when that external face is a Neumann boundary.
int class_flags(const int c[3], const int n[3], int neumann) {
  int fl = 0;
  for (int d = 0; d < 3; ++d) {
    if (c[d] == 0) fl |= 1 << (2 * d);
    if (c[d] == n[d] - 1) fl |= 1 << (2 * d + 1);
  }
  return fl | ((fl & neumann) << 6);
}

struct ClassLayout {
  int flags = 0;
  int n = 0;
  std::vector<int> seg_loc;     // seg * N^3 + local point
  std::vector<double> weights;  // w_S at every subdomain point
  int strip_off[6];
};

// 1D Schwarz weight (eq. schwarz_weight_function) extended to 1 toward
// external faces.
double smoothstep(double x) {
  if (x > 1.0) return 1.0;
  if (x < -1.0) return -1.0;
  const double x2 = x * x;
  return x * (15.0 - 10.0 * x2 + 3.0 * x2 * x2) / 8.0;
}
double weight1d(double xi, double delta, bool lo_ext, bool hi_ext) {
  const double a = lo_ext ? 1.0 : smoothstep((xi + 1.0) / delta);
  const double b = hi_ext ? -1.0 : smoothstep((xi - 1.0) / delta);
  return 0.5 * (a - b);
}

ClassLayout make_layout(int flags, int N, int nov, const std::vector<double>& xi) {
  ClassLayout L;
  L.flags = flags;
  const int N2 = N * N, N3 = N2 * N;
  const double delta = 1.0 + xi[nov];
  bool ext[3][2];
  for (int d = 0; d < 3; ++d) {
    ext[d][0] = (flags >> (2 * d)) & 1;
    ext[d][1] = (flags >> (2 * d + 1)) & 1;
  }
  auto w1 = [&](int d, double x) { return weight1d(x, delta, ext[d][0], ext[d][1]); };
  // central element
  for (int k = 0; k < N; ++k)
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i) {
        L.seg_loc.push_back((k * N + j) * N + i);
        L.weights.push_back(w1(0, xi[i]) * w1(1, xi[j]) * w1(2, xi[k]));
      }
  for (int f = 0; f < 6; ++f) {
    const int d = kFace[f][0], s = kFace[f][1];
    if (ext[d][s > 0 ? 1 : 0]) {
      L.strip_off[f] = -1;
      continue;
    }
    L.strip_off[f] = (int)L.seg_loc.size();
    const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
    for (int layer = 0; layer < nov; ++layer) {
      const int m = s > 0 ? layer : N - 1 - layer;
      const double xs = 2.0 * s + xi[m];
      for (int b1 = 0; b1 < N; ++b1)
        for (int b0 = 0; b0 < N; ++b0) {
          int node[3];
          node[d] = m;
          node[t0] = b0;
          node[t1] = b1;
          L.seg_loc.push_back((f + 1) * N3 + (node[2] * N + node[1]) * N + node[0]);
          const double aj = w1(t0, xi[b0]), ak = w1(t1, xi[b1]);
          const double T = aj * ak + 0.5 * (1 - aj) * ak + 0.5 * aj * (1 - ak) +
                           (1 - aj) * (1 - ak) / 3.0;
          L.weights.push_back(w1(d, xs) * T);
        }
    }
  }
  L.n = (int)L.seg_loc.size();
  return L;
}

struct Level {
  int n[3] = {0, 0, 0};
  long long E = 0;
  double h[3] = {0, 0, 0};
  int split[3] = {0, 0, 0};
  bool has_coarser = false;
  bool f32 = false;
  OpParams op{};
  int* d_nbr = nullptr;
  int* d_order = nullptr;  // element processing order of the operator kernel
  int* d_bricks = nullptr;  // the same order over 2 x 2 x 2 bricks (N = 8)
  // Schwarz
  std::vector<ClassLayout> layouts;
  std::vector<ClassInfo> cls;
  ClassInfo* d_cls = nullptr;
  int* d_seg_loc = nullptr;
  double* d_weights = nullptr;
  int* d_elem_class = nullptr;
  long long* d_elem_row = nullptr;
  PullEntry* d_pull = nullptr;  // scatter pull table, 7 entries per element
  // grouped subdomain GEMM: one work list per tile variant
  GemmTile* d_tiles[kGemmVariants] = {};
  int ntiles[kGemmVariants] = {};
  int kparts_of[kGemmVariants] = {};
  bool gemm_small = false;
  int kparts = 1;  // split-K factor of the class GEMMs
  int gemm_variant = 0;  // large-tile GEMM variant chosen by the autotuner
  // operator-kernel launch shapes chosen by the autotuner: acfg for the
  // Schwarz residuals that write subdomain rows, acfg_out for the launches
  // that write a vector (A u, residuals, the puncture residual)
  ApplyConfig acfg, acfg_out;
  long long rs_total = 0;
  void* d_rs = nullptr;
  void* d_du = nullptr;
  // level vectors
  double *d_u = nullptr, *d_b = nullptr, *d_r = nullptr, *d_diag = nullptr;
  // batched subdomain GMRES(k) work space (level precision)
  void *d_gV = nullptr, *d_gZ = nullptr, *d_gW = nullptr;
  double *d_gH = nullptr, *d_gbeta = nullptr;
  int gk = 0;
  int max_n = 0;
};

}  // namespace

struct dgs_problem {
  dgs_options opt{};
  int p = 0, N = 0;
  double penalty = 0;
  dgs_domain dom{};
  HostTables ht;
  DevTables dt{};
  MgTables mt{};
  std::vector<Level> levels;
  std::vector<void*> allocations;
  // the caller's device allocator (null: hipMalloc / hipFree)
  dgs_alloc_fn alloc_fn = nullptr;
  dgs_free_fn free_fn = nullptr;
  void* alloc_ctx = nullptr;
  // Krylov workspace
  int kry_m = 0;
  double *d_V = nullptr, *d_Z = nullptr, *d_partial = nullptr, *d_h = nullptr, *d_y = nullptr;
  double* d_tmp = nullptr;  // one full vector
  double* d_tmp2 = nullptr;
  double* h_pinned = nullptr;  // pinned host staging for reduction results
  int h_pinned_len = 0;
  bool diag_active = false;
  double t_setup = 0;
  double* d_newton = nullptr;  // Newton work vectors
  // the diagonal mass of the curved elements (power-source Newton solves);
  // invalidated when the geometry or the metric changes
  double* d_mdiag = nullptr;
  // a variable of a system: the Neumann faces of all its variables, which
  // decide the classes and frames (empty for a scalar problem)
  std::vector<int> class_masks;
  // curved elements on the finest level (dgs_set_geometry): the operator,
  // the mass and the Krylov solves use this metric; the multigrid
  // preconditioner keeps the box hierarchy
  bool curved_on = false;
  CurvedGeometry curved;
  // a curved background metric on those elements (dgs_set_metric)
  bool metric_on = false;
  CurvedMetric metric;
  // captured V-cycles (index: linearised operator or not) and the capture stream
  hipGraphExec_t vgraph[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;

  long long nd(int l) const { return levels[l].E * (long long)N * N * N; }

  template <typename T>
  T* alloc(size_t count) {
    T* p = nullptr;
    std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
    if (alloc_fn) {
      const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
      p = static_cast<T*>(alloc_fn(bytes, alloc_ctx));
      if (!p) throw DgsError(DGS_ERR_OOM, "the caller's allocator returned NULL");
      if (reinterpret_cast<uintptr_t>(p) % 256 != 0) {
        free_fn(p, alloc_ctx);
        throw DgsError(DGS_ERR_INVALID, "the caller's allocator returned a pointer not 256-byte aligned");
      }
    } else {
      p = dalloc<T>(count);
    }
    allocations.push_back(p);
    return p;
  }
  // p must be one of `allocations` and no longer in use on the device
  void release(void* p) {
    std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
    auto it = std::find(allocations.begin(), allocations.end(), p);
    if (it != allocations.end()) allocations.erase(it);
    if (free_fn)
      free_fn(p, alloc_ctx);
    else
      (void)hipFree(p);
  }
  // false when the allocator is the server's block pool and the problem is
  // deleted only after its work has finished
  bool sync_before_free = true;
  // host arrays of set-up uploads that may still be in flight, kept until
  // the set-up's final synchronisation (one wait instead of one per table)
  std::vector<std::shared_ptr<void>> setup_keep;
  template <typename T>
  void upload_kept(T* dst, std::vector<T>&& src, hipStream_t s) {
    auto h = std::make_shared<std::vector<T>>(std::move(src));
    upload(dst, *h, s);
    setup_keep.push_back(h);
  }
  ~dgs_problem() {
    std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
    if (!setup_keep.empty()) (void)hipDeviceSynchronize();  // a failed set-up
    // a caller's allocator may hand the memory out again at once: let the
    // device finish with it first (also when set-up failed half-way)
    if (free_fn && sync_before_free && !allocations.empty()) (void)hipDeviceSynchronize();
    for (void* p : allocations) {
      if (free_fn)
        free_fn(p, alloc_ctx);
      else
        (void)hipFree(p);
    }
    if (h_pinned) (void)hipHostFree(h_pinned);
    for (auto& g : vgraph)
      if (g) (void)hipGraphExecDestroy(g);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace {

int nov_of(const dgs_problem* P) { return std::max(1, std::min(P->opt.overlap, P->N - 1)); }

// Face neighbours of every element (-1 at the boundary), faces ordered
// -x, +x, -y, +y, -z, +z.
std::vector<int> host_neighbors(const Level& L) {
  std::vector<int> nbr(L.E * 6);
  for (long long e = 0; e < L.E; ++e) {
    const int c[3] = {(int)(e % L.n[0]), (int)((e / L.n[0]) % L.n[1]),
                      (int)(e / ((long long)L.n[0] * L.n[1]))};
    for (int f = 0; f < 6; ++f) {
      int cc[3] = {c[0], c[1], c[2]};
      cc[kFace[f][0]] += kFace[f][1];
      const int d = kFace[f][0];
      nbr[e * 6 + f] = (cc[d] < 0 || cc[d] >= L.n[d])
                           ? -1
                           : (int)(((long long)cc[2] * L.n[1] + cc[1]) * L.n[0] + cc[0]);
    }
  }
  return nbr;
}

void build_level_mesh(dgs_problem* P, Level& L, hipStream_t s) {
  L.E = (long long)L.n[0] * L.n[1] * L.n[2];
  for (int d = 0; d < 3; ++d) L.h[d] = (P->dom.upper[d] - P->dom.lower[d]) / L.n[d];
  L.op.h[0] = L.h[0];
  L.op.h[1] = L.h[1];
  L.op.h[2] = L.h[2];
  L.op.penalty = P->penalty;
  L.op.E = (int)L.E;
  L.op.n[0] = L.n[0];
  L.op.n[1] = L.n[1];
  L.op.n[2] = L.n[2];
  L.op.neumann = P->opt.neumann_faces;
  set_derived(L.op, P->N, P->ht.w[0]);
  std::vector<int> nbr = host_neighbors(L);
  L.d_nbr = P->alloc<int>(nbr.size());
  P->upload_kept(L.d_nbr, std::move(nbr), s);
  // processing order: columns of 8 x 8 elements in x-y, each swept through z
  // (x fastest inside a layer), so that every face neighbour of an element is
  // processed within about one column layer of it and is still in L2
  std::vector<int> order;
  order.reserve(L.E);
  const int T = 8;
  for (int ty = 0; ty < L.n[1]; ty += T)
    for (int tx = 0; tx < L.n[0]; tx += T)
      for (int z = 0; z < L.n[2]; ++z)
        for (int y = ty; y < std::min(ty + T, L.n[1]); ++y)
          for (int x = tx; x < std::min(tx + T, L.n[0]); ++x)
            order.push_back((int)(((long long)z * L.n[1] + y) * L.n[0] + x));
  bool identity = true;
  for (size_t i = 0; i < order.size() && identity; ++i) identity = order[i] == (int)i;
  if (!identity) {  // the identity order needs no table (and no load)
    L.d_order = P->alloc<int>(order.size());
    P->upload_kept(L.d_order, std::move(order), s);
  }
  if (P->N == 8) {  // bricks (p = 7): the same column order at brick granularity
    const int bn[3] = {(L.n[0] + 1) / 2, (L.n[1] + 1) / 2, (L.n[2] + 1) / 2};
    const int TB = T / 2;
    std::vector<int> border;
    border.reserve((size_t)bn[0] * bn[1] * bn[2]);
    for (int ty = 0; ty < bn[1]; ty += TB)
      for (int tx = 0; tx < bn[0]; tx += TB)
        for (int z = 0; z < bn[2]; ++z)
          for (int y = ty; y < std::min(ty + TB, bn[1]); ++y)
            for (int x = tx; x < std::min(tx + TB, bn[0]); ++x)
              border.push_back((z * bn[1] + y) * bn[0] + x);
    L.d_bricks = P->alloc<int>(border.size());
    P->upload_kept(L.d_bricks, std::move(border), s);
  }
  const long long nd = L.E * (long long)P->N * P->N * P->N;
  L.d_u = P->alloc<double>(nd);
  L.d_b = P->alloc<double>(nd);
  L.d_r = P->alloc<double>(nd);
}

// Schwarz classes, layouts, tiles and work buffers of a level.
void build_level_schwarz(dgs_problem* P, Level& L, hipStream_t s) {
  const int N = P->N, nov = nov_of(P);
  // canonical class: a dimension with only its high face external is mirrored
  // so that the low face is the external one (the DG operator, the subdomain
  // geometry and the weights are all symmetric under the mirror); then, of the
  // exchanges of two axes with equal element widths (under which they are
  // symmetric too), the one that gives the largest flags is taken, so that
  // faces, edges and corners of every orientation share a class.  A variable
  // of a system (class_masks: the Neumann faces of all its variables) takes
  // the frame and the classes from the flags of all variables together, so
  // that every variable has the same classes, frames and row layout, and
  // only its own boundary types in the inverses.
  const std::vector<int> key_masks =
      P->class_masks.empty() ? std::vector<int>{P->opt.neumann_faces} : P->class_masks;
  const int nk = (int)key_masks.size();
  auto mirror = [](int fl, int d) {  // the face and its boundary type move to the low side
    const int nh = (fl >> (6 + 2 * d + 1)) & 1;
    return (fl & ~(3 << (2 * d)) & ~(3 << (6 + 2 * d))) | (1 << (2 * d)) | (nh << (6 + 2 * d));
  };
  auto exchange = [](int fl, int t) {
    int ft = 0;
    for (int d = 0; d < 3; ++d) {
      const int from = frame_axis(d, t);
      ft |= ((fl >> (2 * from)) & 3) << (2 * d);
      ft |= ((fl >> (6 + 2 * from)) & 3) << (6 + 2 * d);
    }
    return ft;
  };
  auto combine = [&](const int* f) {
    uint64_t k = 0;
    for (int v = 0; v < nk; ++v) k |= (uint64_t)f[v] << (12 * v);
    return k;
  };
  std::map<uint64_t, int> cls_of_key;
  std::vector<uint64_t> elem_key(L.E);
  std::vector<int> elem_flags(L.E), elem_code(L.E);
  for (long long e = 0; e < L.E; ++e) {
    const int c[3] = {(int)(e % L.n[0]), (int)((e / L.n[0]) % L.n[1]),
                      (int)(e / ((long long)L.n[0] * L.n[1]))};
    int own = class_flags(c, L.n, P->opt.neumann_faces), mask = 0;
    int kf[kSysMaxVars], tf[kSysMaxVars];
    for (int v = 0; v < nk; ++v) kf[v] = class_flags(c, L.n, key_masks[v]);
    for (int d = 0; d < 3; ++d) {
      const int lo = (own >> (2 * d)) & 1, hi = (own >> (2 * d + 1)) & 1;
      if (!lo && hi) {
        mask |= 1 << d;
        own = mirror(own, d);
        for (int v = 0; v < nk; ++v) kf[v] = mirror(kf[v], d);
      }
    }
    uint64_t best = combine(kf);
    int best_t = 0, best_own = own;
    for (int t = 1; t <= 3; ++t) {
      const int a = t == 3 ? 1 : 0, b = t == 1 ? 1 : 2;
      if (L.h[a] != L.h[b]) continue;
      for (int v = 0; v < nk; ++v) tf[v] = exchange(kf[v], t);
      const uint64_t kt = combine(tf);
      if (kt > best) {
        best = kt;
        best_t = t;
        best_own = exchange(own, t);
      }
    }
    elem_flags[e] = best_own;
    elem_key[e] = best;
    elem_code[e] = mask | best_t << 3;
    cls_of_key.emplace(best, 0);
  }
  int ci = 0;
  for (auto& kv : cls_of_key) kv.second = ci++;
  // a class's own flags (the same for all its elements: the own boundary
  // types are part of the key)
  std::vector<int> own_of_class(ci, 0);
  std::vector<int> elem_class(L.E), count(ci, 0), pos(L.E);
  for (long long e = 0; e < L.E; ++e) {
    elem_class[e] = cls_of_key[elem_key[e]];
    own_of_class[elem_class[e]] = elem_flags[e];
    pos[e] = count[elem_class[e]]++;
  }
  L.layouts.clear();
  L.cls.assign(ci, ClassInfo{});
  for (int c = 0; c < ci; ++c) L.layouts.push_back(make_layout(own_of_class[c], N, nov, P->ht.xi));
  std::vector<int> seg_loc;
  std::vector<double> weights;
  long long rs_off = 0;
  for (int c = 0; c < ci; ++c) {
    ClassInfo& I = L.cls[c];
    const ClassLayout& lay = L.layouts[c];
    I.n = lay.n;
    I.count = count[c];
    I.ld = (lay.n + kGemmLd - 1) / kGemmLd * kGemmLd;
    I.rows = (count[c] + kGemmRows - 1) / kGemmRows * kGemmRows;
    I.kext = (lay.n + 31) / 32 * 32;
    I.inv = nullptr;  // set once the inverses exist
    I.op = nullptr;
    I.scale = 1.0;
    I.scale_op = 1.0;
    I.rs_off = rs_off;
    I.layout_off = (int)seg_loc.size();
    for (int f = 0; f < 6; ++f) I.strip_off[f] = lay.strip_off[f];
    seg_loc.insert(seg_loc.end(), lay.seg_loc.begin(), lay.seg_loc.end());
    weights.insert(weights.end(), lay.weights.begin(), lay.weights.end());
    rs_off += (long long)I.ld * I.rows;
  }
  L.rs_total = rs_off;
  L.max_n = 0;
  for (int c = 0; c < ci; ++c) L.max_n = std::max(L.max_n, L.cls[c].n);
  int max_parts = 1;
  for (int v = 0; v < kGemmVariants; ++v) {
    GemmPlan plan = plan_subdomain_gemm(L.cls, v);
    L.gemm_small = plan.small;
    L.kparts_of[v] = plan.kparts;
    L.ntiles[v] = (int)plan.tiles.size();
    L.d_tiles[v] = P->alloc<GemmTile>(plan.tiles.size());
    max_parts = std::max(max_parts, plan.kparts);
    P->upload_kept(L.d_tiles[v], std::move(plan.tiles), s);
  }
  L.gemm_variant = 0;
  L.kparts = L.kparts_of[0];
  std::vector<long long> elem_row(L.E);
  for (long long e = 0; e < L.E; ++e)
    elem_row[e] = L.cls[elem_class[e]].rs_off + (long long)pos[e] * L.cls[elem_class[e]].ld;
  L.d_cls = P->alloc<ClassInfo>(ci);
  upload(L.d_cls, L.cls, s);
  L.d_seg_loc = P->alloc<int>(seg_loc.size());
  P->upload_kept(L.d_seg_loc, std::move(seg_loc), s);
  L.d_weights = P->alloc<double>(weights.size());
  P->upload_kept(L.d_weights, std::move(weights), s);
  std::vector<int> elem_cv(L.E);
  for (long long e = 0; e < L.E; ++e) elem_cv[e] = elem_class[e] | (elem_code[e] << 24);
  L.d_elem_class = P->alloc<int>(L.E);
  P->upload_kept(L.d_elem_class, std::move(elem_cv), s);
  // scatter pull table: the element's own row, and for every face neighbour b
  // the start of b's strip toward the element (in b's class frame)
  const std::vector<int> nbr = host_neighbors(L);
  std::vector<PullEntry> pull(L.E * 7);
  for (long long e = 0; e < L.E; ++e) {
    const ClassInfo& ce = L.cls[elem_class[e]];
    pull[e * 7] = PullEntry{elem_row[e], ce.layout_off, elem_code[e]};
    for (int f = 0; f < 6; ++f) {
      const int b = nbr[e * 6 + f];
      if (b < 0) {
        pull[e * 7 + 1 + f] = PullEntry{-1, 0, 0};
        continue;
      }
      const int d = f >> 1, d0 = d == 0 ? 1 : 0;
      const int mb = elem_code[b] & 7, tb = elem_code[b] >> 3;
      // b's face toward e (own side (f ^ 1) & 1 along axis d) in b's class frame
      const int dc = frame_axis(d, tb);
      const int g = 2 * dc + (((f ^ 1) & 1) ^ ((mb >> d) & 1));
      // the own axes that b's class-frame transverse axes (ascending) hold
      const int x0 = frame_axis(dc == 0 ? 1 : 0, tb), x1 = frame_axis(dc == 2 ? 1 : 2, tb);
      const ClassInfo& cb = L.cls[elem_class[b]];
      if (cb.strip_off[g] < 0) throw DgsError(DGS_ERR_HIP, "subdomain strip missing");
      pull[e * 7 + 1 + f] = PullEntry{elem_row[b] + cb.strip_off[g], cb.layout_off + cb.strip_off[g],
                                      ((mb >> x0) & 1) | (((mb >> x1) & 1) << 1) |
                                          ((x0 != d0 ? 1 : 0) << 2)};
    }
  }
  L.d_pull = P->alloc<PullEntry>(pull.size());
  P->upload_kept(L.d_pull, std::move(pull), s);
  L.d_elem_row = P->alloc<long long>(L.E);
  P->upload_kept(L.d_elem_row, std::move(elem_row), s);
  // the padding of the subdomain rows is never written and must read as zero
  const size_t es = L.f32 ? sizeof(float) : sizeof(double);
  L.d_rs = P->alloc<char>(es * (size_t)L.rs_total);
  L.d_du = P->alloc<char>(es * (size_t)L.rs_total * max_parts);
  HIP_OK(hipMemsetAsync(L.d_rs, 0, es * (size_t)L.rs_total, s));
  HIP_OK(hipMemsetAsync(L.d_du, 0, es * (size_t)L.rs_total * max_parts, s));
}

// Explicit inverses of A_S for every (class flags, element aspect) key, built
// on the device: the subdomain operator is assembled column by column by
// applying the DG operator to unit vectors on a small patch (the central
// element, its face neighbours and one all-zero element standing for every
// element outside the subdomain), then inverted by Gauss-Jordan elimination
// (A_S is symmetric positive definite, so no pivoting is needed).  Uniform
// scaling of all element widths by lambda scales A_S by lambda, so one inverse
// per key serves every level and every problem with the same aspect ratio.
// Keys live in a process-wide cache shared by all problems on a device (a
// serving process reuses them across requests); cache memory is held until
// the process ends.
struct CacheEntry {
  int device, N, nov, flags;
  double ry, rz, penalty, hx;  // key and the reference width along x
  int n, ld;
  double* inv64 = nullptr;
  float* inv32 = nullptr;
  double* op64 = nullptr;
  float* op32 = nullptr;
  // an entry is listed as soon as one problem starts building it; others
  // that need it wait until it is ready (or drop it when its build failed)
  bool ready = false, failed = false;
};
std::mutex g_cache_mutex;
std::condition_variable g_cache_cv;
std::vector<std::unique_ptr<CacheEntry>> g_cache;

CacheEntry* cache_find(int device, int N, int nov, int flags, double ry, double rz, double penalty) {
  for (auto& c : g_cache)
    if (!c->failed && c->device == device && c->N == N && c->nov == nov && c->flags == flags &&
        c->penalty == penalty && std::fabs(c->ry - ry) <= 1e-12 * ry &&
        std::fabs(c->rz - rz) <= 1e-12 * rz)
      return c.get();
  return nullptr;
}

void build_keys(dgs_problem* P, const std::vector<CacheEntry*>& todo,
                const std::vector<const Level*>& ref, hipStream_t s) {
  const int N = P->N, N3 = N * N * N;
  const int nk = (int)todo.size();
  if (nk == 0) return;
  std::vector<ClassLayout> klay;
  int n_pad = 0;
  for (auto& k : todo) {
    klay.push_back(make_layout(k->flags, N, k->nov, P->ht.xi));
    n_pad = std::max(n_pad, klay.back().n);
  }
  n_pad = (n_pad + 63) / 64 * 64;  // the blocked inversion works on 64-wide blocks
  double* d_batch = dalloc<double>((size_t)nk * n_pad * n_pad);
  std::unique_ptr<void, void (*)(void*)> g1(d_batch, dfree);
  {
    std::vector<double> eye((size_t)n_pad * n_pad, 0.0);
    for (int i = 0; i < n_pad; ++i) eye[(size_t)i * n_pad + i] = 1.0;
    for (int k = 0; k < nk; ++k)
      HIP_OK(hipMemcpyAsync(d_batch + (size_t)k * n_pad * n_pad, eye.data(),
                            eye.size() * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  for (int k = 0; k < nk; ++k) {
    const ClassLayout& lay = klay[k];
    // patch: 0 = central, 1.. = existing face neighbours, last = zero element
    int face_elem[6];
    int Ep = 1;
    for (int f = 0; f < 6; ++f) face_elem[f] = lay.strip_off[f] >= 0 ? Ep++ : -1;
    const int zero = Ep++;
    std::vector<int> pn(Ep * 6, -1);
    for (int f = 0; f < 6; ++f) pn[0 * 6 + f] = face_elem[f];  // -1 = Dirichlet
    for (int f = 0; f < 6; ++f) {
      if (face_elem[f] < 0) continue;
      const int b = face_elem[f];
      for (int g = 0; g < 6; ++g) {
        if (g == (f ^ 1)) {
          pn[b * 6 + g] = 0;  // back to the central element
        } else if (g == f) {
          pn[b * 6 + g] = zero;  // far face: never reaches a subdomain row
        } else {
          const bool ext = (lay.flags >> g) & 1;  // same row of elements as the centre
          pn[b * 6 + g] = ext ? -1 : zero;
        }
      }
    }
    const int n = lay.n;
    std::vector<int> nb((size_t)n * Ep * 6);
    for (int c = 0; c < n; ++c)
      for (int q = 0; q < Ep * 6; ++q) nb[(size_t)c * Ep * 6 + q] = pn[q] < 0 ? -1 : pn[q] + c * Ep;
    std::vector<int> idx(n);
    for (int r = 0; r < n; ++r) {
      const int seg = lay.seg_loc[r] / N3, loc = lay.seg_loc[r] % N3;
      const int el = seg == 0 ? 0 : face_elem[seg - 1];
      idx[r] = el * N3 + loc;
    }
    const long long stride = (long long)Ep * N3;
    const long long tot = stride * n;
    int* d_nb = dalloc<int>(nb.size());
    std::unique_ptr<void, void (*)(void*)> g2(d_nb, dfree);
    int* d_idx = dalloc<int>(n);
    std::unique_ptr<void, void (*)(void*)> g3(d_idx, dfree);
    double* d_X = dalloc<double>(tot);
    std::unique_ptr<void, void (*)(void*)> g4(d_X, dfree);
    double* d_AX = dalloc<double>(tot);
    std::unique_ptr<void, void (*)(void*)> g5(d_AX, dfree);
    upload(d_nb, nb, s);
    upload(d_idx, idx, s);
    HIP_OK(launch_fill(d_X, 0.0, tot, s));
    HIP_OK(launch_unit_columns(d_X, stride, d_idx, n, s));
    OpParams op = ref[k]->op;
    op.neumann = (lay.flags >> 6) & 63;  // the class's Neumann faces, in its frame
    set_derived(op, N, P->ht.w[0]);
    op.E = (int)(Ep * (long long)n);
    op.n[0] = op.n[1] = op.n[2] = 0;  // patch elements: neighbours from the table
    HIP_OK(launch_apply(N, kApply, d_X, d_AX, nullptr, nullptr, nullptr, d_nb, op, P->dt,
                        ApplyConfig{}, s));
    HIP_OK(launch_gather_columns(d_AX, stride, d_idx, n, d_batch + (size_t)k * n_pad * n_pad, n_pad, s));
    HIP_OK(hipStreamSynchronize(s));
  }
  // keep A_S itself (transposed) for the linearised subdomain solver
  for (int k = 0; k < nk; ++k) {
    CacheEntry& c = *todo[k];
    c.n = klay[k].n;
    c.ld = (c.n + kGemmLd - 1) / kGemmLd * kGemmLd;
    const size_t nn = (size_t)c.ld * c.ld;  // zero-padded to ld x ld
    c.op64 = dalloc<double>(nn);
    c.op32 = dalloc<float>(nn);
    c.inv64 = dalloc<double>(nn);
    c.inv32 = dalloc<float>(nn);
    HIP_OK(hipMemsetAsync(c.op64, 0, nn * sizeof(double), s));
    HIP_OK(hipMemsetAsync(c.op32, 0, nn * sizeof(float), s));
    HIP_OK(hipMemsetAsync(c.inv64, 0, nn * sizeof(double), s));
    HIP_OK(hipMemsetAsync(c.inv32, 0, nn * sizeof(float), s));
    HIP_OK(launch_finish_inverse(d_batch + (size_t)k * n_pad * n_pad, n_pad, c.n, c.ld, 1.0,
                                 c.op64, c.op32, s));
  }
  double* d_P = dalloc<double>((size_t)nk * 64 * 64);
  std::unique_ptr<void, void (*)(void*)> g6(d_P, dfree);
  double* d_R = dalloc<double>((size_t)nk * 64 * n_pad);
  std::unique_ptr<void, void (*)(void*)> g7(d_R, dfree);
  double* d_C = dalloc<double>((size_t)nk * 64 * n_pad);
  std::unique_ptr<void, void (*)(void*)> g8(d_C, dfree);
  HIP_OK(launch_block_inverse(d_batch, n_pad, nk, d_P, d_R, d_C, s));
  for (int k = 0; k < nk; ++k) {
    CacheEntry& c = *todo[k];
    HIP_OK(launch_finish_inverse(d_batch + (size_t)k * n_pad * n_pad, n_pad, c.n, c.ld, 1.0,
                                 c.inv64, c.inv32, s));
  }
  HIP_OK(hipStreamSynchronize(s));
}

void build_inverses(dgs_problem* P, hipStream_t s) {
  int device = 0;
  HIP_OK(hipGetDevice(&device));
  const int nov = nov_of(P);
  // the keys this problem needs: found in the cache (ready or being built by
  // another problem) or listed now and built here, outside the lock, so that
  // problems of different shapes build their inverses concurrently
  std::unique_lock<std::mutex> lk(g_cache_mutex);
  std::vector<CacheEntry*> todo;
  std::vector<const Level*> ref;
  struct Use {
    int level, cls;
    CacheEntry* entry;
  };
  std::vector<Use> uses;
  for (int l = 0; l < (int)P->levels.size(); ++l) {
    const Level& L = P->levels[l];
    const double ry = L.h[1] / L.h[0], rz = L.h[2] / L.h[0];
    for (int c = 0; c < (int)L.layouts.size(); ++c) {
      const int flags = L.layouts[c].flags;
      CacheEntry* e = cache_find(device, P->N, nov, flags, ry, rz, P->penalty);
      if (!e) {
        std::unique_ptr<CacheEntry> ne(new CacheEntry());
        ne->device = device;
        ne->N = P->N;
        ne->nov = nov;
        ne->flags = flags;
        ne->ry = ry;
        ne->rz = rz;
        ne->penalty = P->penalty;
        ne->hx = L.h[0];
        e = ne.get();
        g_cache.push_back(std::move(ne));
        todo.push_back(e);
        ref.push_back(&L);
      }
      uses.push_back(Use{l, c, e});
    }
  }
  lk.unlock();
  try {
    build_keys(P, todo, ref, s);
  } catch (...) {
    lk.lock();
    for (CacheEntry* e : todo) e->failed = true;
    g_cache_cv.notify_all();
    throw;
  }
  lk.lock();
  for (CacheEntry* e : todo) e->ready = true;
  g_cache_cv.notify_all();
  g_cache_cv.wait(lk, [&]() {
    for (const Use& u : uses)
      if (!u.entry->ready && !u.entry->failed) return false;
    return true;
  });
  for (const Use& u : uses)
    if (u.entry->failed) throw DgsError(DGS_ERR_HIP, "building a subdomain inverse failed");
  lk.unlock();
  for (const Use& u : uses) {
    Level& L = P->levels[u.level];
    ClassInfo& I = L.cls[u.cls];
    I.inv = L.f32 ? (const void*)u.entry->inv32 : (const void*)u.entry->inv64;
    I.op = L.f32 ? (const void*)u.entry->op32 : (const void*)u.entry->op64;
    I.scale = u.entry->hx / L.h[0];  // A_S(lambda h) = lambda A_S(h)
    I.scale_op = L.h[0] / u.entry->hx;
  }
  for (Level& L : P->levels) upload(L.d_cls, L.cls, s);
  HIP_OK(hipStreamSynchronize(s));
}


// Per-degree launch-shape autotuner of the operator kernel: time every
// candidate elements-per-workgroup value on the finest mesh and keep the
// fastest.  Results are cached per (N, element count) for the process.
// The level's grouped subdomain GEMM in its tuned variant; part_stride is the
// distance between the split-K partial products in DU.
hipError_t gemm_level(Level& L, const void* rs, long long part_stride, int use_op, hipStream_t s) {
  const int v = L.gemm_variant;
  return launch_subdomain_gemm(L.f32, rs, L.d_du, part_stride, L.d_cls, L.d_tiles[v], L.ntiles[v],
                               L.gemm_small, use_op, s, v);
}

std::mutex g_tune_mutex;
// Elements per workgroup of the operator kernel, timed per level in the mode
// the Schwarz steps launch most (residual with the gather written out) and
// cached per level shape.  Each candidate's time is the best of 3 trials; a
// later candidate must win by 3 % so near ties resolve the same way.
std::map<std::tuple<int, long long, int, int, int, int>, int> g_tuned_epb;

ApplyConfig shape_config(const Level& L, int shape) {
  ApplyConfig c;
  c.epb = shape;
  c.bricks = shape == -1 ? L.d_bricks : nullptr;
  return c;
}

// Time `launch` (kernel launches on s): the minimum over `trials` trials of
// a repetition count sized so that a trial lasts about `trial_ms`.
template <typename F>
float time_launches(F&& launch, hipStream_t s, hipEvent_t e0, hipEvent_t e1, float trial_ms,
                    int trials) {
  launch();  // warm-up
  HIP_OK(hipEventRecord(e0, s));
  launch();
  HIP_OK(hipEventRecord(e1, s));
  HIP_OK(hipEventSynchronize(e1));
  float one = 0;
  HIP_OK(hipEventElapsedTime(&one, e0, e1));
  const int reps = std::max(3, std::min(200, (int)(trial_ms / std::max(one, 1e-4f))));
  float tmin = 1e30f;
  for (int trial = 0; trial < trials; ++trial) {
    HIP_OK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) launch();
    HIP_OK(hipEventRecord(e1, s));
    HIP_OK(hipEventSynchronize(e1));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    tmin = std::min(tmin, ms / reps);
  }
  return tmin;
}

// Per-level launch-shape autotuner of the operator kernel, once for each use:
// the Schwarz residual with its subdomain-row stores (acfg) and the plain
// apply that writes a vector (acfg_out).  Candidates are timed in order and
// a later one must win by 3 %, so near ties resolve the same way every time.
void autotune_apply(dgs_problem* P, hipStream_t s) {
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  const int N = P->N;
  for (Level& L : P->levels) {
    const long long n = L.E * (long long)N * N * N;
    bool filled = false;
    for (int use = 0; use < 2; ++use) {
      ApplyConfig& target = use == 0 ? L.acfg : L.acfg_out;
      const auto key = std::make_tuple(N, L.E, L.n[0], L.n[1], (int)L.f32, use);
      {
        std::lock_guard<std::mutex> lk(g_tune_mutex);
        auto it = g_tuned_epb.find(key);
        if (it != g_tuned_epb.end()) {
          target = shape_config(L, it->second);
          continue;
        }
      }
      if (!filled) {
        HIP_OK(launch_fill(L.d_u, 1.0, n, s));
        HIP_OK(launch_fill(L.d_b, 0.0, n, s));
        filled = true;
      }
      GatherOut go;
      go.rs = L.d_rs;
      go.f32 = L.f32;
      go.pull = L.d_pull;
      go.nov = nov_of(P);
      // large levels are timed for longer: their choice matters and is
      // made once per shape, while the small shapes of a serving stream are
      // many and latency-bound
      const float tune_ms = L.E >= 512 ? 0.5f : 0.1f;
      const int tune_trials = L.E >= 512 ? 5 : 3;
      // elements per workgroup; -1: 2 x 2 x 2 bricks
      int cands[4] = {1, 2, 0}, ncand = 3;
      if (L.d_bricks) cands[ncand++] = -1;
      int best = cands[0];
      float best_ms = 1e30f;
      for (int ci = 0; ci < ncand; ++ci) {
        const ApplyConfig cfg = shape_config(L, cands[ci]);
        const float t = time_launches(
            [&]() {
              if (use == 0)
                HIP_OK(launch_apply(N, kResidual, L.d_u, nullptr, L.d_b, nullptr, nullptr,
                                    L.d_nbr, L.op, P->dt, cfg, s, L.d_order, go));
              else
                HIP_OK(launch_apply(N, kApply, L.d_u, L.d_r, nullptr, nullptr, nullptr, L.d_nbr,
                                    L.op, P->dt, cfg, s, L.d_order));
            },
            s, e0, e1, tune_ms, tune_trials);
        if (t < 0.97f * best_ms) {
          best_ms = t;
          best = cands[ci];
        }
      }
      target = shape_config(L, best);
      std::lock_guard<std::mutex> lk(g_tune_mutex);
      g_tuned_epb[key] = best;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// Tile variant of the grouped subdomain GEMM (row-tile height and K split),
// timed together with the scatter that sums its partial products, on every
// level with large tiles; cached per level shape.
std::map<std::tuple<int, int, int, int, int, int>, int> g_tuned_gemm;

void autotune_gemm(dgs_problem* P, hipStream_t s) {
  hipEvent_t e0, e1;
  HIP_OK(hipEventCreate(&e0));
  HIP_OK(hipEventCreate(&e1));
  const int N = P->N;
  for (Level& L : P->levels) {
    if (L.ntiles[0] == 0) continue;
    const auto key = std::make_tuple(N, L.n[0], L.n[1], L.n[2], (int)L.f32, nov_of(P));
    int best = 0;
    bool cached = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mutex);
      auto it = g_tuned_gemm.find(key);
      if (it != g_tuned_gemm.end()) {
        best = it->second;
        cached = true;
      }
    }
    if (!cached) {
      const size_t es = L.f32 ? sizeof(float) : sizeof(double);
      // pseudo-random operands: the MFMA clock under load depends on the data,
      // and zeros would favour tiles that run hotter on real residuals
      HIP_OK(launch_fill_pattern(L.d_rs, L.f32, L.rs_total, s));
      HIP_OK(launch_fill(L.d_u, 0.0, L.E * (long long)N * N * N, s));
      float best_ms = 1e30f;
      for (int v = 0; v < kGemmVariants; ++v) {
        L.gemm_variant = v;
        L.kparts = L.kparts_of[v];
        const float t = time_launches(
            [&]() {
              HIP_OK(gemm_level(L, L.d_rs, L.rs_total, 0, s));
              HIP_OK(launch_scatter(N, L.f32, L.d_u, L.d_du, L.kparts, L.rs_total, L.d_weights,
                                    L.d_pull, nov_of(P), L.E, s));
            },
            s, e0, e1, L.E >= 512 ? 0.5f : 0.1f, L.E >= 512 ? 5 : 3);
        // a later variant must win by 3 % so near ties resolve the same way
        if (t < 0.97f * best_ms) {
          best_ms = t;
          best = v;
        }
      }
      // the class blocks' padding must read as zeros again, and nothing
      // later expects what the timing runs left in u or the products
      HIP_OK(hipMemsetAsync(L.d_rs, 0, es * (size_t)L.rs_total, s));
      int mp = 1;
      for (int v = 0; v < kGemmVariants; ++v) mp = std::max(mp, L.kparts_of[v]);
      HIP_OK(hipMemsetAsync(L.d_du, 0, es * (size_t)L.rs_total * mp, s));
      HIP_OK(launch_fill(L.d_u, 0.0, L.E * (long long)N * N * N, s));
      std::lock_guard<std::mutex> lk(g_tune_mutex);
      g_tuned_gemm[key] = best;
    }
    L.gemm_variant = best;
    L.kparts = L.kparts_of[best];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// ---------------------------------------------------------------------------
// Schwarz smoothing and the V-cycle
// ---------------------------------------------------------------------------

// Subdomain problems of the linearised operator, (A_S + diag(R_S d)) du_S = r_S,
// solved for every subdomain at once by k iterations of right-preconditioned
// GMRES with the Poisson inverse as preconditioner (Laplacian approximation,
// Sec. III.E.1).  Input: the gathered residuals in L.d_rs; output: du_S in
// part 0 of L.d_du.
void subdomain_gmres(dgs_problem* P, Level& L, hipStream_t s) {
  const int k = P->opt.subdomain_iters;
  const int N = P->N;
  const size_t es = L.f32 ? sizeof(float) : sizeof(double);
  const long long st = L.rs_total;
  auto slot = [&](void* base, int i) { return (void*)((char*)base + es * (size_t)st * i); };
  HIP_OK(launch_sub_start(L.f32, L.d_rs, L.d_gV, L.d_gbeta, L.d_elem_class, L.d_elem_row, L.d_cls,
                          (int)L.E, s));
  for (int j = 0; j < k; ++j) {
    void* Vj = slot(L.d_gV, j);
    void* Zj = slot(L.d_gZ, j);
    HIP_OK(gemm_level(L, Vj, st, 0, s));
    HIP_OK(launch_reduce_parts(L.f32, Zj, L.d_du, L.kparts, st, st, s));
    HIP_OK(gemm_level(L, Zj, st, 1, s));
    HIP_OK(launch_reduce_parts(L.f32, L.d_gW, L.d_du, L.kparts, st, st, s));
    HIP_OK(launch_sub_arnoldi(N, L.f32, j, k, L.d_gW, L.d_gV, Zj, st, L.d_diag, L.d_gH,
                              L.d_elem_class, L.d_elem_row, L.d_nbr, L.d_cls, L.d_seg_loc, (int)L.E,
                              L.max_n, s));
  }
  HIP_OK(launch_sub_finish(L.f32, k, L.d_gZ, st, L.d_gH, L.d_gbeta, L.d_du, L.d_elem_class,
                           L.d_elem_row, L.d_cls, (int)L.E, s));
}
// The level's gather-out target: its subdomain rows and pull table.
GatherOut level_gather(const dgs_problem* P, const Level& L) {
  GatherOut go;
  go.rs = L.d_rs;
  go.f32 = L.f32;
  go.pull = L.d_pull;
  go.nov = nov_of(P);
  return go;
}

// rs_ready: the first step's r_S = R_S b is already in the level's rows
// (written by the kernel that produced b).
void schwarz_steps(dgs_problem* P, int l, const double* b, double* u, int steps, bool u_zero,
                   hipStream_t s, bool rs_ready = false) {
  Level& L = P->levels[l];
  const int N = P->N;
  const bool diag = P->diag_active && L.d_diag != nullptr;
  const GatherOut go = level_gather(P, L);
  for (int it = 0; it < steps; ++it) {
    if (it == 0 && u_zero) {
      // r = b: gather it (unless its producer already did)
      if (!rs_ready)
        HIP_OK(launch_gather(N, L.f32, b, L.d_rs, L.d_elem_class, L.d_elem_row, L.d_nbr, L.d_cls,
                             L.d_seg_loc, (int)L.E, s));
    } else {
      // the residual kernel writes r_S = R_S (b - A u) straight into the rows
      HIP_OK(launch_apply(N, diag ? kResidualDiag : kResidual, u, nullptr, b, L.d_diag, nullptr,
                          L.d_nbr, L.op, P->dt, L.acfg, s, L.d_order, go));
    }
    if (diag && P->opt.subdomain_iters > 0) {
      subdomain_gmres(P, L, s);
      HIP_OK(launch_scatter(N, L.f32, u, L.d_du, 1, L.rs_total, L.d_weights, L.d_pull, nov_of(P),
                            L.E, s, it == 0 && u_zero));
      continue;
    }
    HIP_OK(gemm_level(L, L.d_rs, L.rs_total, 0, s));
    // the scatter sums the split-K partials itself
    HIP_OK(launch_scatter(N, L.f32, u, L.d_du, L.kparts, L.rs_total, L.d_weights, L.d_pull,
                          nov_of(P), L.E, s, it == 0 && u_zero));
  }
}

// rs0_ready: the finest level's rows already hold R_S r.
// One visit of level l in a multigrid cycle (Sec. III.C.3): presmoothing,
// the residual restricted to the next coarser level, the visits of that level
// (kind 1, V: one; kind 2, W: two W-visits; kind 3, F: an F-visit and then a
// V-visit; every second visit starts from the first one's result),
// prolongation, postsmoothing; the coarsest level smooths only.
// u_zero: u[l] starts from zero (its first smoothing step writes u);
// rs_ready: the first step's subdomain rows r_S = R_S b are already gathered.
void mg_visit(dgs_problem* P, int l, const std::vector<const double*>& b,
              const std::vector<double*>& u, bool u_zero, bool rs_ready, int coarse_steps,
              int kind, hipStream_t s) {
  const int nl = (int)P->levels.size();
  const int N = P->N;
  Level& L = P->levels[l];
  const int pre = l < nl - 1 ? P->opt.pre_smooth : coarse_steps;
  // a level without smoothing steps still needs its zero start
  if (u_zero && pre == 0) HIP_OK(launch_fill(u[l], 0.0, P->nd(l), s));
  schwarz_steps(P, l, b[l], u[l], pre, u_zero, s, rs_ready);
  if (l == nl - 1) return;
  const bool diag = P->diag_active && L.d_diag != nullptr;
  HIP_OK(launch_apply(N, diag ? kResidualDiag : kResidual, u[l], L.d_r, b[l], L.d_diag, nullptr,
                      L.d_nbr, L.op, P->dt, L.acfg_out, s, L.d_order));
  Level& C = P->levels[l + 1];
  // the restriction also writes the coarse level's first r_S rows
  HIP_OK(launch_restrict(N, L.d_r, C.d_b, L.n, C.n, L.split, P->mt, s, level_gather(P, C)));
  // V: one V-visit; W: two W-visits; F: an F-visit, then a V-visit
  const int visits[2] = {kind, kind == 3 ? 1 : kind};
  const int nvisits = kind == 1 ? 1 : 2;
  for (int visit = 0; visit < nvisits; ++visit)
    mg_visit(P, l + 1, b, u, visit == 0, visit == 0, coarse_steps, visits[visit], s);
  HIP_OK(launch_prolongate_add(N, u[l + 1], u[l], L.n, C.n, L.split, P->mt, s));
  schwarz_steps(P, l, b[l], u[l], P->opt.post_smooth, false, s);
}

void vcycle_eager(dgs_problem* P, const double* r, double* z, hipStream_t s,
                  bool rs0_ready = false) {
  const int nl = (int)P->levels.size();
  std::vector<const double*> b(nl);
  std::vector<double*> u(nl);
  b[0] = r;
  u[0] = z;
  for (int l = 1; l < nl; ++l) {
    b[l] = P->levels[l].d_b;
    u[l] = P->levels[l].d_u;
  }
  // the coarsest level takes pre- and postsmoothing (Sec. III.C.3); when it
  // is a single element with the plain operator, its one subdomain is the
  // whole level and the subdomain solve is exact, so the first step already
  // gives the solution and further steps would change it only by rounding
  const Level& Lc = P->levels[nl - 1];
  int coarse_steps = P->opt.pre_smooth + P->opt.post_smooth;
  if (Lc.E == 1 && !(P->diag_active && Lc.d_diag != nullptr))
    coarse_steps = std::min(coarse_steps, 1);
  if (!P->opt.additive) {
    mg_visit(P, 0, b, u, true, rs0_ready, coarse_steps, P->opt.cycle, s);
    return;
  }
  // additive multigrid: the residual restricted to every level (each
  // restriction also writes that level's first r_S rows), every level
  // smoothed from zero, the corrections prolongated and summed coarsest first
  const int N = P->N;
  for (int l = 0; l + 1 < nl; ++l) {
    Level& L = P->levels[l];
    Level& C = P->levels[l + 1];
    HIP_OK(launch_restrict(N, b[l], C.d_b, L.n, C.n, L.split, P->mt, s, level_gather(P, C)));
  }
  for (int l = 0; l < nl; ++l) {
    const int steps = l < nl - 1 ? P->opt.pre_smooth + P->opt.post_smooth : coarse_steps;
    if (steps == 0) HIP_OK(launch_fill(u[l], 0.0, P->nd(l), s));
    schwarz_steps(P, l, b[l], u[l], steps, true, s, l == 0 ? rs0_ready : true);
  }
  for (int l = nl - 2; l >= 0; --l) {
    Level& L = P->levels[l];
    Level& C = P->levels[l + 1];
    HIP_OK(launch_prolongate_add(N, u[l + 1], u[l], L.n, C.n, L.split, P->mt, s));
  }
}

// Capture the multigrid cycle of operator kind gi (0: A; 1: A + diag(d)) as a
// hipGraph that reads the finest level's d_b (with its first subdomain rows
// already gathered) and writes its d_u.  Called at set-up: kind 0 by
// dgs_create_problem, kind 1 by the first dgs_set_diagonal, and again after
// a tuning override changes the launches; never inside a solve, so
// dgs_precondition and the Krylov iterations only replay.  Capture touches no
// device memory, so it needs no synchronisation with earlier work.
void capture_vgraph(dgs_problem* P, int gi) {
  std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
  Level& L0 = P->levels[0];
  if (P->vgraph[gi]) {
    HIP_OK(hipGraphExecDestroy(P->vgraph[gi]));
    P->vgraph[gi] = nullptr;
  }
  if (!P->cap_stream) HIP_OK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
  const bool saved = P->diag_active;
  P->diag_active = gi == 1;
  HIP_OK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
  hipGraph_t graph = nullptr;
  try {
    vcycle_eager(P, L0.d_b, L0.d_u, P->cap_stream, /*rs0_ready=*/true);
  } catch (...) {
    (void)hipStreamEndCapture(P->cap_stream, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    P->diag_active = saved;
    throw;
  }
  P->diag_active = saved;
  HIP_OK(hipStreamEndCapture(P->cap_stream, &graph));
  hipError_t e = hipGraphInstantiate(&P->vgraph[gi], graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIP_OK(e);
}

// Re-capture the cycles that exist after a change of the launches they hold
// (launch shape, GEMM variant); earlier replays may still be in flight.
void recapture_vgraphs(dgs_problem* P) {
  if (!P->opt.use_graphs) return;
  HIP_OK(hipDeviceSynchronize());
  for (int gi = 0; gi < 2; ++gi)
    if (P->vgraph[gi]) capture_vgraph(P, gi);
}

// Replay the captured cycle of the current operator kind on s.
void vcycle_graph(dgs_problem* P, hipStream_t s) {
  Level& L0 = P->levels[0];
  const int gi = (P->diag_active && L0.d_diag) ? 1 : 0;
  if (!P->vgraph[gi]) throw DgsError(DGS_ERR_HIP, "multigrid cycle was not captured at set-up");
  HIP_OK(hipGraphLaunch(P->vgraph[gi], s));
}

void vcycle(dgs_problem* P, const double* r, double* z, hipStream_t s) {
  if (!P->opt.use_graphs) {
    vcycle_eager(P, r, z, s);
    return;
  }
  Level& L0 = P->levels[0];
  const long long n = P->nd(0);
  HIP_OK(launch_copy(L0.d_b, r, n, s));
  HIP_OK(launch_gather(P->N, L0.f32, L0.d_b, L0.d_rs, L0.d_elem_class, L0.d_elem_row, L0.d_nbr,
                       L0.d_cls, L0.d_seg_loc, (int)L0.E, s));
  vcycle_graph(P, s);
  HIP_OK(launch_copy(z, L0.d_u, n, s));
}

void ensure_krylov(dgs_problem* P, int m) {
  if (P->kry_m >= m) return;
  // the old basis may still be read by work in flight (hipFree would wait
  // for the device by itself; a caller's allocator may not)
  if (P->kry_m > 0 && P->free_fn) HIP_OK(hipDeviceSynchronize());
  for (double* p : {P->d_V, P->d_Z, P->d_partial, P->d_h, P->d_y, P->d_tmp, P->d_tmp2})
    if (p) P->release(p);
  const long long n = P->nd(0);
  P->d_V = P->alloc<double>((size_t)(m + 1) * n);
  P->d_Z = P->alloc<double>((size_t)m * n);
  P->d_partial = P->alloc<double>((size_t)multidot_blocks(n) * (m + 2));
  P->d_h = P->alloc<double>(3 * (m + 2));
  P->d_y = P->alloc<double>(m + 1);
  P->d_tmp = P->alloc<double>(n);
  P->d_tmp2 = P->alloc<double>(n);
  std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
  if (P->h_pinned) (void)hipHostFree(P->h_pinned);
  P->h_pinned = nullptr;
  HIP_OK(hipHostMalloc((void**)&P->h_pinned, sizeof(double) * 4 * (m + 2), hipHostMallocDefault));
  P->h_pinned_len = 4 * (m + 2);
  P->kry_m = m;
}

double device_norm2(dgs_problem* P, const double* x, long long n, hipStream_t s) {
  HIP_OK(launch_multidot(x, n, 1, x, n, P->d_partial, P->d_h, s));
  HIP_OK(hipMemcpyAsync(P->h_pinned, P->d_h, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return P->h_pinned[0];
}

// Apply either A or the linearised operator A + diag(d) on the finest level.
// xcopy (optional) receives a copy of x.
void apply_fine(dgs_problem* P, const double* x, double* y, hipStream_t s,
                double* xcopy = nullptr) {
  Level& L = P->levels[0];
  const bool diag = P->diag_active && L.d_diag != nullptr;
  if (P->curved_on) {
    if (xcopy) HIP_OK(launch_copy(xcopy, x, P->nd(0), s));
    if (P->metric_on)
      HIP_OK(launch_curved_apply_metric(P->N, false, x, y, nullptr, diag ? L.d_diag : nullptr,
                                        P->curved, P->metric, L.d_nbr, P->penalty, L.op.neumann,
                                        L.E, s));
    else
      HIP_OK(launch_curved_apply(P->N, false, x, y, nullptr, diag ? L.d_diag : nullptr, P->curved,
                                 L.d_nbr, P->penalty, L.op.neumann, L.E, s));
    return;
  }
  HIP_OK(launch_apply(P->N, diag ? kApplyDiag : kApply, x, y, nullptr, L.d_diag, nullptr, L.d_nbr,
                      L.op, P->dt, L.acfg_out, s, L.d_order, GatherOut{}, xcopy));
}

void residual_fine(dgs_problem* P, const double* x, const double* b, double* r, hipStream_t s) {
  Level& L = P->levels[0];
  const bool diag = P->diag_active && L.d_diag != nullptr;
  if (P->curved_on) {
    if (P->metric_on)
      HIP_OK(launch_curved_apply_metric(P->N, true, x, r, b, diag ? L.d_diag : nullptr, P->curved,
                                        P->metric, L.d_nbr, P->penalty, L.op.neumann, L.E, s));
    else
      HIP_OK(launch_curved_apply(P->N, true, x, r, b, diag ? L.d_diag : nullptr, P->curved,
                                 L.d_nbr, P->penalty, L.op.neumann, L.E, s));
    return;
  }
  HIP_OK(launch_apply(P->N, diag ? kResidualDiag : kResidual, x, r, b, L.d_diag, nullptr, L.d_nbr,
                      L.op, P->dt, L.acfg_out, s, L.d_order));
}

// Make subsequent smoothing, V-cycles and solves act on A + diag(d): copy d
// to the finest level and restrict it down the hierarchy (d_{l+1} = R d_l).
void set_diagonal(dgs_problem* P, const double* d, hipStream_t s) {
  if (!d) {
    P->diag_active = false;
    return;
  }
  const int k = P->opt.subdomain_iters;
  for (Level& L : P->levels) {
    if (!L.d_diag) L.d_diag = P->alloc<double>(L.E * (long long)P->N * P->N * P->N);
    if (k > 0 && L.gk < k) {
      if (L.max_n > 4352)
        throw DgsError(DGS_ERR_INVALID, "subdomain GMRES supports subdomains of at most 4352 points");
      const size_t es = L.f32 ? sizeof(float) : sizeof(double);
      L.d_gV = P->alloc<char>(es * (size_t)L.rs_total * (k + 1));
      L.d_gZ = P->alloc<char>(es * (size_t)L.rs_total * k);
      L.d_gW = P->alloc<char>(es * (size_t)L.rs_total);
      // the GEMMs read the row padding of the bases: it must be zero
      HIP_OK(hipMemsetAsync(L.d_gV, 0, es * (size_t)L.rs_total * (k + 1), s));
      HIP_OK(hipMemsetAsync(L.d_gZ, 0, es * (size_t)L.rs_total * k, s));
      L.d_gH = P->alloc<double>((size_t)L.E * (k + 1) * k);
      L.d_gbeta = P->alloc<double>(L.E);
      L.gk = k;
    }
  }
  HIP_OK(launch_copy(P->levels[0].d_diag, d, P->nd(0), s));
  for (size_t l = 0; l + 1 < P->levels.size(); ++l) {
    Level& L = P->levels[l];
    Level& C = P->levels[l + 1];
    HIP_OK(launch_restrict(P->N, L.d_diag, C.d_diag, L.n, C.n, L.split, P->mt, s));
  }
  P->diag_active = true;
  if (P->opt.use_graphs && !P->vgraph[1]) capture_vgraph(P, 1);
}


// Flexible GMRES (Saad Alg. 9.6) on the fine level as a resumable state
// machine: issue() enqueues the device work of the current stage on the
// stream without waiting, complete() runs the host part once the stream has
// been synchronised.  Stages: start (r0 = b - A x0 and its norm), one stage
// per iteration (V-cycle, operator, classical Gram-Schmidt twice, norm, the
// Hessenberg column to pinned memory), finish (x = x0 + Z y, true residual).
// dgs_solve runs the stages back to back; the server interleaves the stages
// of many requests, so a request computes the same numbers alone or in a mix.
struct FgmresRun {
  dgs_problem* P = nullptr;
  const double* b = nullptr;
  double* x = nullptr;
  double rtol = 0;
  int m = 0;          // iterations of one cycle (the Krylov basis size)
  int max_total = 0;  // iterations of all cycles together
  hipStream_t s = nullptr;
  enum Stage { kStart, kIter, kFinish, kDone } stage = kStart;
  int j = 0;          // iteration within the cycle
  int cycles = 0;
  double beta = 0;    // |r_0| of the cycle
  double beta0 = 0;   // |r_0| of the first cycle: the reference of rtol and the history
  std::vector<double> H, cs, sn, g;
  FgmresResult R;

  void init(dgs_problem* p, const double* bb, double* xx, double rt, int mi, hipStream_t st) {
    P = p;
    b = bb;
    x = xx;
    rtol = rt;
    max_total = mi;
    // restarted FGMRES(m): cycles of at most m iterations, each started from
    // the true residual of the previous cycle's solution
    m = P->opt.restart > 0 ? std::min(P->opt.restart, mi) : mi;
    s = st;
    ensure_krylov(P, m);
    cycles = 0;
    R = FgmresResult();
    new_cycle();
  }
  void new_cycle() {
    stage = kStart;
    j = 0;
    H.assign((size_t)(m + 1) * m, 0.0);
    cs.assign(m, 0.0);
    sn.assign(m, 0.0);
    g.assign(m + 1, 0.0);
  }
  bool done() const { return stage == kDone; }

  void issue() {
    const long long n = P->nd(0);
    double* V = P->d_V;
    double* Z = P->d_Z;
    double* hp = P->h_pinned;
    if (stage == kStart) {
      residual_fine(P, x, b, V, s);
      HIP_OK(launch_multidot(V, n, 1, V, n, P->d_partial, P->d_h, s));
      HIP_OK(hipMemcpyAsync(hp, P->d_h, sizeof(double), hipMemcpyDeviceToHost, s));
    } else if (stage == kIter) {
      double* vj = V + (size_t)j * n;
      double* zj = Z + (size_t)j * n;
      double* w = V + (size_t)(j + 1) * n;
      if (P->opt.use_graphs) {
        // v_j is already in the V-cycle's input (written when it was
        // normalised); the operator kernel copies the output z_j out
        vcycle_graph(P, s);
        apply_fine(P, P->levels[0].d_u, w, s, zj);
      } else {
        vcycle(P, vj, zj, s);
        apply_fine(P, zj, w, s);
      }
      double* h1 = P->d_h;
      double* h2 = P->d_h + (m + 2);
      double* hn = P->d_h + 2 * (m + 2);
      // classical Gram-Schmidt twice; each correction is fused with the
      // reduction that follows it
      HIP_OK(launch_multidot(V, n, j + 1, w, n, P->d_partial, h1, s));
      HIP_OK(launch_axpy_multidot(V, n, j + 1, h1, w, n, false, P->d_partial, h2, s));
      HIP_OK(launch_axpy_multidot(V, n, j + 1, h2, w, n, true, P->d_partial, hn, s));
      // h1, h2 and |w|^2 are contiguous on the device: one copy
      HIP_OK(hipMemcpyAsync(hp, P->d_h, sizeof(double) * (2 * (m + 2) + 1), hipMemcpyDeviceToHost, s));
      // v_{j+1} = w / |w| (unused if |w| = 0: the run stops), also into the
      // V-cycle's input for the next iteration
      if (P->opt.use_graphs)
        HIP_OK(launch_scale_by_inv_norm(w, w, hn, n, s, P->levels[0].d_b, P->N,
                                        level_gather(P, P->levels[0])));
      else
        HIP_OK(launch_scale_by_inv_norm(w, w, hn, n, s));
    } else if (stage == kFinish) {
      const int k = j;
      std::vector<double> y(k, 0.0);
      for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int q = i + 1; q < k; ++q) t -= H[(size_t)q * (m + 1) + i] * y[q];
        y[i] = t / H[(size_t)i * (m + 1) + i];
      }
      double* ypin = hp + 3 * (m + 2);
      for (int i = 0; i < k; ++i) ypin[i] = y[i];
      if (k > 0) {
        HIP_OK(hipMemcpyAsync(P->d_y, ypin, sizeof(double) * k, hipMemcpyHostToDevice, s));
        HIP_OK(launch_combine(x, Z, n, k, P->d_y, n, s));
      }
      residual_fine(P, x, b, P->d_tmp, s);
      HIP_OK(launch_multidot(P->d_tmp, n, 1, P->d_tmp, n, P->d_partial, P->d_h, s));
      HIP_OK(hipMemcpyAsync(hp, P->d_h, sizeof(double), hipMemcpyDeviceToHost, s));
    }
  }

  void complete() {
    const double* hp = P->h_pinned;
    if (stage == kStart) {
      const double beta2 = hp[0];
      if (!std::isfinite(beta2)) throw DgsError(DGS_ERR_NONFINITE, "non-finite initial residual");
      beta = std::sqrt(beta2);
      if (cycles++ == 0) {
        beta0 = beta;
        R.history.push_back(1.0);
      }
      if (beta == 0.0) {
        R.converged = true;
        stage = kDone;
        return;
      }
      g[0] = beta;
      if (P->opt.use_graphs)
        HIP_OK(launch_scale_by_inv_norm(P->d_V, P->d_V, P->d_h, P->nd(0), s, P->levels[0].d_b, P->N,
                                        level_gather(P, P->levels[0])));
      else
        HIP_OK(launch_scale_by_inv_norm(P->d_V, P->d_V, P->d_h, P->nd(0), s));
      stage = kIter;
    } else if (stage == kIter) {
      double* col = &H[(size_t)j * (m + 1)];  // column j, rows 0..j+1
      for (int i = 0; i <= j; ++i) col[i] = hp[i] + hp[(m + 2) + i];
      const double hn2 = hp[2 * (m + 2)];
      col[j + 1] = std::sqrt(hn2);
      for (int i = 0; i <= j + 1; ++i)
        if (!std::isfinite(col[i])) throw DgsError(DGS_ERR_NONFINITE, "non-finite Hessenberg entry");
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * col[i] + sn[i] * col[i + 1];
        col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
        col[i] = t;
      }
      const double den = std::hypot(col[j], col[j + 1]);
      cs[j] = col[j] / den;
      sn[j] = col[j + 1] / den;
      col[j] = den;
      col[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      R.history.push_back(std::fabs(g[j + 1]) / beta0);
      ++j;
      ++R.iterations;
      if (std::fabs(g[j]) <= rtol * beta0 || hn2 == 0.0) {
        R.converged = true;
        stage = kFinish;
      } else if (j >= m || R.iterations >= max_total) {
        stage = kFinish;
      }
    } else if (stage == kFinish) {
      R.rel_residual = std::sqrt(hp[0]) / beta0;
      if (!std::isfinite(R.rel_residual)) throw DgsError(DGS_ERR_NONFINITE, "non-finite residual");
      // the Givens estimate stopped the cycle; the true residual decides:
      // short of rtol, the next cycle starts from the true residual of x
      R.converged = R.rel_residual <= rtol;
      if (!R.converged && R.iterations < max_total)
        new_cycle();
      else
        stage = kDone;
    }
  }
};

FgmresResult fgmres(dgs_problem* P, const double* b, double* x, double rtol, int max_iter,
                    hipStream_t s) {
  FgmresRun run;
  run.init(P, b, x, rtol, max_iter, s);
  while (!run.done()) {
    run.issue();
    HIP_OK(hipStreamSynchronize(s));
    run.complete();
  }
  return run.R;
}

// Preconditioned conjugate gradients for symmetric positive definite
// problems (Sec. III.B; Saad Alg. 9.1) on the fine level, with the direction
// update beta = (z_{k+1}, r_{k+1} - r_k) / (z_k, r_k), which equals the
// textbook (z_{k+1}, r_{k+1}) / (z_k, r_k) for a fixed symmetric positive
// definite preconditioner and stays usable with the V-cycle, which is not.
// Per iteration: one operator application, one V-cycle, and one host round
// trip (p.Ap, the dot products of z_{k+1} with both residuals and |r_{k+1}|^2
// in one copy); alpha is formed on the device.  A run stops when the
// recursively updated residual drops to rtol |r_0|; the true residual then
// decides: short of rtol (and with iterations left) CG starts again from the
// true residual of x.  The returned residual is the true one.
// ws: the work vectors (4 vectors of the fine level, reduction partials, the
// device scalars and pinned host staging).
struct CgWork {
  double *R, *z, *p0, *p1, *q, *t, *partial, *h, *hp;
};

FgmresResult cg(dgs_problem* P, const double* b, double* x, double rtol, int max_iter,
                hipStream_t s, const CgWork& ws) {
  const long long n = P->nd(0);
  double* R = ws.R;  // rows 0 and 1: r_k and r_{k+1}, alternating
  double* z = ws.z;
  double* pdir[2] = {ws.p0, ws.p1};  // p_k and p_{k+1}, alternating
  double* q = ws.q;
  double* h = ws.h;
  double* hp = ws.hp;
  FgmresResult res;
  res.history.push_back(1.0);
  auto fetch = [&](int count) {
    HIP_OK(hipMemcpyAsync(hp, h, sizeof(double) * count, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int i = 0; i < count; ++i)
      if (!std::isfinite(hp[i])) throw DgsError(DGS_ERR_NONFINITE, "non-finite value in CG");
  };
  double nr0 = -1.0;  // |r_0| of the first run: the reference of rtol
  int k = 0;
  for (;;) {  // runs, each from the true residual of x
    int cur = 0, pc = 0;
    residual_fine(P, x, b, R, s);
    vcycle(P, R, z, s);
    HIP_OK(launch_copy(pdir[0], z, n, s));
    HIP_OK(launch_multidot(R, n, 1, R, n, ws.partial, h, s));
    HIP_OK(launch_multidot(R, n, 1, z, n, ws.partial, h + 1, s));
    fetch(2);
    const double nr_start = std::sqrt(hp[0]);
    if (nr0 < 0.0) nr0 = nr_start;
    if (nr0 == 0.0) {
      res.converged = true;
      return res;
    }
    if (nr_start <= rtol * nr0) {  // the true residual of x already meets rtol
      res.rel_residual = nr_start / nr0;
      res.converged = true;
      return res;
    }
    double rz = hp[1];
    bool stopped = false, hit = false;
    while (k < max_iter) {
      ++k;
      double* pv = pdir[pc];
      double* r = R + (size_t)cur * n;
      double* r_next = R + (size_t)(1 - cur) * n;
      apply_fine(P, pv, q, s);
      // p.Ap stays on the device: the update kernel forms alpha from it
      HIP_OK(launch_multidot(pv, n, 1, q, n, ws.partial, h + 3, s));
      HIP_OK(launch_cg_step(x, r_next, r, pv, q, rz, h + 3, n, s));
      res.iterations = k;
      // z_{k+1} is computed before |r_{k+1}| is known: one V-cycle more than
      // needed at the end, one host round trip per iteration
      vcycle(P, r_next, z, s);
      HIP_OK(launch_multidot(R, n, 2, z, n, ws.partial, h, s));  // (r_0 row, z), (r_1 row, z)
      HIP_OK(launch_multidot(r_next, n, 1, r_next, n, ws.partial, h + 2, s));
      fetch(4);
      if (!(hp[3] > 0.0)) {  // A is not positive definite on p: stopped, not converged
        res.iterations = --k;
        stopped = true;
        break;
      }
      const double nr = std::sqrt(hp[2]);
      res.history.push_back(nr / nr0);
      if (nr <= rtol * nr0) {
        hit = true;
        break;
      }
      const double rz_next = hp[1 - cur], zr_old = hp[cur];
      const double beta = (rz_next - zr_old) / rz;
      HIP_OK(launch_waxpy(pdir[1 - pc], z, beta, pv, n, s));
      rz = rz_next;
      cur = 1 - cur;
      pc = 1 - pc;
    }
    residual_fine(P, x, b, ws.t, s);
    HIP_OK(launch_multidot(ws.t, n, 1, ws.t, n, ws.partial, h, s));
    fetch(1);
    res.rel_residual = std::sqrt(hp[0]) / nr0;
    res.converged = res.rel_residual <= rtol;
    if (res.converged || stopped || !hit || k >= max_iter) return res;
  }
}

// Static device workspace of dgs_cg_solve_noalloc: the CG work vectors of
// a fine level of at most kNoAllocMaxDofs points (6 vectors, each starting on
// a 256-byte boundary), the reduction partials and the device scalars.
// Every GPU the library runs on holds its own copy until the process ends.
constexpr long long kNoAllocMaxDofs = 1LL << 20;
constexpr long long kNoAllocPartials = 2048;  // multidot_blocks(n) <= 1024, two dots
constexpr long long kNoAllocDoubles = 7 * kNoAllocMaxDofs + kNoAllocPartials + 64;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};     // device address of `scratch`, per device
double g_scratch_host[kMaxDevices][8] = {};  // host staging of the reduction results

// The current device's address of `scratch` (looked up once per device).
double* scratch_for_current_device(int* device) {
  HIP_OK(hipGetDevice(device));
  if (*device < 0 || *device >= kMaxDevices) throw DgsError(DGS_ERR_INVALID, "device id out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mutex);
  if (!g_scratch_ptr[*device]) {
    void* ptr = nullptr;
    HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[*device] = static_cast<double*>(ptr);
  }
  return g_scratch_ptr[*device];
}

CgWork problem_cg_work(dgs_problem* P) {
  ensure_krylov(P, 4);
  const long long n = P->nd(0);
  return CgWork{P->d_V, P->d_Z, P->d_Z + n, P->d_Z + 2 * n, P->d_tmp, P->d_tmp2,
                P->d_partial, P->d_h, P->h_pinned};
}

// Backtracking line search on f = |F|^2 / 2 with the linear model's slope
// -|F|^2 (Dennis & Schnabel: quadratic interpolation first, cubic after,
// each new step in [0.1, 0.5] times the previous, at most 10 backtracks).
// trial(lam) evaluates the residual at u + lam du and returns its f; the
// return value is the accepted trial's f.
template <class Trial>
double backtracking_line_search(double nrm2, Trial&& trial, int& backtracks) {
  const double alpha_sd = 1e-4;  // sufficient-decrease parameter
  const int max_bt = 10;
  const double f0 = 0.5 * nrm2, slope = -nrm2;
  double lam = 1.0, lam_prev = 0.0, f_prev = 0.0, ft = 0.0;
  for (int bt = 0; bt <= max_bt; ++bt) {
    ft = trial(lam);
    if (!std::isfinite(ft)) throw DgsError(DGS_ERR_NONFINITE, "non-finite trial residual");
    if (ft <= f0 + alpha_sd * lam * slope || bt == max_bt) break;
    double next;
    if (bt == 0) {
      next = -slope * lam * lam / (2.0 * (ft - f0 - slope * lam));
    } else {
      const double r1 = ft - f0 - lam * slope, r2 = f_prev - f0 - lam_prev * slope;
      const double ca = (r1 / (lam * lam) - r2 / (lam_prev * lam_prev)) / (lam - lam_prev);
      const double cb = (-lam_prev * r1 / (lam * lam) + lam * r2 / (lam_prev * lam_prev)) /
                        (lam - lam_prev);
      if (ca == 0.0) {
        next = -slope / (2.0 * cb);
      } else {
        const double disc = std::max(cb * cb - 3.0 * ca * slope, 0.0);
        next = (-cb + std::sqrt(disc)) / (3.0 * ca);
      }
    }
    next = std::min(next, 0.5 * lam);
    next = std::max(next, 0.1 * lam);
    lam_prev = lam;
    f_prev = ft;
    lam = next;
    ++backtracks;
  }
  return ft;
}

// The diagonal mass of a problem's curved elements (and metric), formed once
// per geometry
const double* ensure_mdiag(dgs_problem* p, hipStream_t st) {
  if (!p->d_mdiag) {
    const long long nn = p->nd(0);
    p->d_mdiag = p->alloc<double>(nn);
    HIP_OK(launch_fill(p->d_mdiag, 1.0, nn, st));
    if (p->metric_on)
      HIP_OK(launch_curved_mass_metric(p->N, p->d_mdiag, p->d_mdiag, p->curved, p->metric,
                                       p->levels[0].E, st));
    else
      HIP_OK(launch_curved_mass(p->N, p->d_mdiag, p->d_mdiag, p->curved, p->levels[0].E, st));
  }
  return p->d_mdiag;
}

// Newton-Raphson with a backtracking line search (Sec. III.A) as a resumable
// run: init() evaluates the first residual, each step() performs one Newton
// step (linearise, solve the linear system with FGMRES to linear_rtol, line
// search) and waits for it; done() once converged or after max_newton steps.
struct NewtonRun {
  dgs_problem* P = nullptr;
  // kind 0: the puncture source on the box grid (alpha, beta); kind 1: a
  // power-law source S(u) = sum_t c_t u^k_t on curved elements, with
  // Dirichlet data bvals (NULL: homogeneous) and the diagonal mass mdiag
  int kind = 0;
  PowerSource ps;
  const double *bvals = nullptr, *mdiag = nullptr;
  const double *alpha = nullptr, *beta = nullptr, *b = nullptr;
  double* u = nullptr;
  double newton_rtol = 0, linear_rtol = 0;
  int max_newton = 0;
  hipStream_t s = nullptr;
  long long n = 0;
  double *F = nullptr, *Ft = nullptr, *du = nullptr, *ut = nullptr, *work = nullptr;
  double nrm2 = 0, norm0 = 0;
  std::vector<double> hist;
  int its = 0, steps = 0, backtracks = 0;
  bool converged = false;

  void residual(const double* x, double* out) {  // A x + M S(x) - b
    const Level& L0 = P->levels[0];
    if (kind == 1) {
      HIP_OK(launch_curved_apply_bc(P->N, x, out, bvals, P->curved,
                                    P->metric_on ? &P->metric : nullptr, L0.d_nbr, P->penalty,
                                    L0.op.neumann, L0.E, s));
      HIP_OK(launch_power_source(ps, x, mdiag, b, out, nullptr, n, s));
      return;
    }
    HIP_OK(launch_apply(P->N, kPuncture, x, out, b, alpha, beta, L0.d_nbr, L0.op, P->dt,
                        L0.acfg_out, s, L0.d_order));
  }
  void init_powers(dgs_problem* p, const PowerSource& src, const double* bv, const double* bb,
                   double* uu, double nrt, double lrt, int mn, hipStream_t st) {
    kind = 1;
    ps = src;
    bvals = bv;
    mdiag = ensure_mdiag(p, st);
    start(p, bb, uu, nrt, lrt, mn, st);
  }
  void init(dgs_problem* p, const double* a, const double* be, const double* bb, double* uu,
            double nrt, double lrt, int mn, hipStream_t st) {
    kind = 0;
    alpha = a;
    beta = be;
    start(p, bb, uu, nrt, lrt, mn, st);
  }
  void start(dgs_problem* p, const double* bb, double* uu, double nrt, double lrt, int mn,
             hipStream_t st) {
    P = p;
    b = bb;
    u = uu;
    newton_rtol = nrt;
    linear_rtol = lrt;
    max_newton = mn;
    s = st;
    n = P->nd(0);
    ensure_krylov(P, P->opt.max_iter);
    if (!P->d_newton) P->d_newton = P->alloc<double>((size_t)5 * n);
    F = P->d_newton;
    Ft = F + n;
    du = F + 2 * n;
    ut = F + 3 * n;
    work = F + 4 * n;
    P->diag_active = false;
    residual(u, F);
    nrm2 = device_norm2(P, F, n, s);
    if (!std::isfinite(nrm2)) throw DgsError(DGS_ERR_NONFINITE, "non-finite nonlinear residual");
    norm0 = std::sqrt(nrm2);
    hist.assign(1, 1.0);
    its = steps = backtracks = 0;
    converged = norm0 == 0.0;
  }
  bool done() const { return converged || steps >= max_newton; }
  double rel_residual() const { return std::sqrt(nrm2) / (norm0 > 0 ? norm0 : 1.0); }

  void step() {
    // linearisation A + diag(M dS/du(u)) and the linear solve for du
    const Level& L0 = P->levels[0];
    if (kind == 1)
      HIP_OK(launch_power_source(ps, u, mdiag, nullptr, nullptr, work, n, s));
    else
      HIP_OK(launch_puncture_diag(P->N, alpha, beta, u, work, L0.E, L0.h, P->dt, s));
    set_diagonal(P, work, s);
    HIP_OK(launch_fill(work, 0.0, n, s));
    HIP_OK(launch_axpy(work, -1.0, F, n, s));  // right-hand side -F
    HIP_OK(launch_fill(du, 0.0, n, s));
    FgmresResult R = fgmres(P, work, du, linear_rtol, P->opt.max_iter, s);
    its += R.iterations;
    P->diag_active = false;
    const double ft = backtracking_line_search(
        nrm2,
        [&](double lam) {
          HIP_OK(launch_waxpy(ut, u, lam, du, n, s));
          residual(ut, Ft);
          return 0.5 * device_norm2(P, Ft, n, s);
        },
        backtracks);
    HIP_OK(launch_copy(u, ut, n, s));
    std::swap(F, Ft);
    nrm2 = 2.0 * ft;
    ++steps;
    hist.push_back(std::sqrt(nrm2) / norm0);
    converged = std::sqrt(nrm2) <= newton_rtol * norm0;
    HIP_OK(hipStreamSynchronize(s));
  }
};


void fill_stats(dgs_stats* st, const FgmresResult& R, double t0, double t_setup) {
  if (!st) return;
  st->iterations = R.iterations;
  st->rel_residual = R.rel_residual;
  st->t_solve_s = now_s() - t0;
  st->t_setup_s = t_setup;
  st->history_len = 0;
  if (st->history && st->history_capacity > 0) {
    const int n = std::min<int>(st->history_capacity, (int)R.history.size());
    for (int i = 0; i < n; ++i) st->history[i] = R.history[i];
    st->history_len = n;
  }
}

}  // namespace

// ===========================================================================
// Serving: continuous batching of many solves on one device
// ===========================================================================
// Requests wait in a FIFO queue until their estimated device footprint fits in
// the budget and a slot is free.  Every active request owns a problem (mesh,
// hierarchy, Krylov basis, all resident until it finishes) and a stream; the
// subdomain inverses come from the shared process-wide cache.  Each step
// enqueues the next FGMRES stage of every active request on its stream, so the
// requests' kernels overlap on the device, then completes all of them on the
// host; finished requests free their memory and queued ones are admitted.
namespace {

struct ServerRequest {
  long long id = 0;
  dgs_domain dom{};
  int elements[3] = {0, 0, 0};
  int p = 0;
  std::vector<double> f;  // host copy of f at the points
  size_t footprint = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  dgs_problem* prob = nullptr;
  hipStream_t stream = nullptr;
  double *d_b = nullptr, *d_u = nullptr;
  FgmresRun run;
  bool in_flight = false;  // a stage is issued on the stream and not yet completed
  // puncture requests (kind 1): Newton steps are the stages
  int kind = 0;
  std::vector<double> alpha, beta;  // host copies of the fields (b stays in f)
  bool has_b = false;
  double *d_alpha = nullptr, *d_beta = nullptr;
  double newton_rtol = 0, linear_rtol = 0;
  int max_newton = 0;
  NewtonRun nrun;
  int newton_steps = 0, backtracks = 0;
  bool reused = false;  // set up on a finished request's problem of the same shape
  bool done() const { return kind == 0 ? run.done() : nrun.done(); }
  std::vector<double> u;  // result
  FgmresResult result;
  double t_setup = 0;
  int status = 0;
  bool batched = false;  // advanced by the cross-request batch engine
};

}  // namespace

// ===========================================================================
// Cross-request batched engine of the serving loop
// ===========================================================================
// The active Poisson requests of degree p <= 8 advance together, one FGMRES
// iteration per step, through launches that each cover every request: one
// operator launch, one or two grouped GEMM launches (FP32 and FP64 classes)
// and one scatter launch per Schwarz step of the multigrid cycle, one launch
// per transfer, and one per Krylov vector operation.  The launches' job
// tables (the V-cycle's schedule over the requests' levels, the tiles of the
// GEMMs grouped across requests) are rebuilt when a request joins or leaves;
// the few per-step tables (Krylov vectors at the current iteration index)
// are staged in one host-to-device copy, and the scalars of every request
// come back in one device-to-host copy, one synchronisation per step.
namespace {

// A device buffer grown on demand (library memory).
struct DevBuf {
  char* p = nullptr;
  size_t cap = 0;
  void ensure(size_t n) {
    if (n <= cap) return;
    if (p) dfree(p);
    cap = std::max(n, 2 * cap);
    p = dalloc<char>(cap);
  }
  ~DevBuf() {
    if (p) dfree(p);
  }
};

// Job tables appended to one host byte image (16-byte aligned entries).
struct JobImage {
  std::vector<char> bytes;
  template <typename J>
  size_t put(const std::vector<J>& v) {
    const size_t off = (bytes.size() + 15) / 16 * 16;
    bytes.resize(off + v.size() * sizeof(J));
    if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(J));
    return off;
  }
};

enum BatchOpKind { kOpApplyRows, kOpApplyVec, kOpGemm, kOpScatter, kOpRestrict, kOpProlong };

struct BatchOp {
  int kind = 0;
  size_t off = 0;             // the job table (GEMM: the class list)
  size_t off_ptrs = 0, off_tiles = 0;  // GEMM: per-class pointers, tiles
  int njobs = 0, nblocks = 0, threads = 64;
  bool f32 = false, small = false;
};

// The engine's per-request state: the host side of FGMRES (Saad Alg. 9.6) as
// the solo solver keeps it, and the request's slot in the scalar pack.
struct BatchReq {
  ServerRequest* r = nullptr;
  int slot = 0;
  enum Stage { kStart, kIter, kFinish, kDone } stage = kStart;
  int m = 0, j = 0, cycles = 0, iterations = 0, max_total = 0;
  double rtol = 0, beta = 0, beta0 = 0;
  std::vector<double> H, cs, sn, g, y;
  bool converged = false;
};

class BatchEngine {
 public:
  BatchEngine(int max_active, int max_iter, int restart)
      : max_active_(max_active), kmax_(max_iter), restart_(restart) {
    std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
    HIP_OK(hipStreamCreateWithFlags(&s_, hipStreamNonBlocking));
    stride_ = 4 * (kmax_ + 2);
    pack_.ensure(sizeof(double) * (size_t)stride_ * max_active_);
    HIP_OK(hipHostMalloc((void**)&h_pack_, sizeof(double) * (size_t)stride_ * max_active_,
                         hipHostMallocDefault));
    // the operator and transfer tables of every degree p <= 8
    std::vector<DevTables> dt(kMaxN + 1);
    std::vector<MgTables> mt(kMaxN + 1);
    std::memset(dt.data(), 0, dt.size() * sizeof(DevTables));
    std::memset(mt.data(), 0, mt.size() * sizeof(MgTables));
    for (int N = 2; N <= 9; ++N) {
      const HostTables ht = make_tables(N);
      dt[N] = to_dev(ht);
      mt[N] = to_dev_mg(ht);
    }
    tabs_.ensure(dt.size() * sizeof(DevTables) + mt.size() * sizeof(MgTables) + 16);
    HIP_OK(hipMemcpy(tabs_.p, dt.data(), dt.size() * sizeof(DevTables), hipMemcpyHostToDevice));
    mt_off_ = (dt.size() * sizeof(DevTables) + 15) / 16 * 16;
    HIP_OK(hipMemcpy(tabs_.p + mt_off_, mt.data(), mt.size() * sizeof(MgTables),
                     hipMemcpyHostToDevice));
    free_slots_.clear();
    for (int i = max_active_ - 1; i >= 0; --i) free_slots_.push_back(i);
  }
  ~BatchEngine() {
    if (s_) (void)hipStreamSynchronize(s_);
    std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
    if (h_pack_) (void)hipHostFree(h_pack_);
    if (h_stage_) (void)hipHostFree(h_stage_);
    if (s_) (void)hipStreamDestroy(s_);
  }
  hipStream_t stream() const { return s_; }
  bool empty() const { return reqs_.empty(); }
  int size() const { return (int)reqs_.size(); }
  int launches_last_step() const { return launches_; }
  bool issued() const { return issued_; }

  // A request whose problem, b and u = 0 are set up (on its own stream, which
  // the caller has synchronised) joins at the next step.
  void add(ServerRequest* r) {
    if (free_slots_.empty()) throw DgsError(DGS_ERR_INVALID, "batch engine: no free slot");
    BatchReq q;
    q.r = r;
    q.slot = free_slots_.back();
    free_slots_.pop_back();
    q.max_total = r->run.max_total;
    q.rtol = r->run.rtol;
    // restarted FGMRES(m): cycles of at most m iterations (the basis size)
    q.m = std::min(restart_ > 0 ? restart_ : kmax_, q.max_total);
    ensure_krylov(r->prob, q.m);
    new_cycle(q);
    r->run.R = FgmresResult();
    reqs_.push_back(std::move(q));
    dirty_ = true;
  }

  // One lockstep step; returns the requests that finished (their results in
  // r->run.R, r->run.stage = done).
  // One step of every member: issue() enqueues the tables, the launches and
  // the copy of the pack back to the host; finish() waits for them and runs
  // the host part.  Host work between the two (the set-up of newly admitted
  // requests) overlaps the step on the device.
  void issue() {
    issued_ = false;
    if (reqs_.empty()) return;
    if (dirty_) rebuild();
    launches_ = 0;
    JobImage img;
    // ---- per-step job lists ----
    std::vector<BApplyJob> a_start, a_iter, a_fin;
    std::vector<BDotJob> d_start, d1, d2, d3, d_fin;
    std::vector<BVecJob> v_start, v_iter, v_comb;
    int thr_start = 64, thr_iter = 64, thr_fin = 64;
    for (BatchReq& q : reqs_) {
      dgs_problem* P = q.r->prob;
      Level& L0 = P->levels[0];
      const long long n = P->nd(0);
      double* pk = (double*)pack_.p + (size_t)q.slot * stride_;
      const int m2 = q.m + 2;
      double* h1 = pk;
      double* h2 = pk + m2;
      double* hn = pk + 2 * m2;
      double* beta2 = pk + 2 * m2 + 1;
      double* res2 = pk + 2 * m2 + 2;
      double* yv = pk + 3 * m2;
      double* V = P->d_V;
      double* Z = P->d_Z;
      if (q.stage == BatchReq::kStart || q.stage == BatchReq::kIter) {
        if (q.stage == BatchReq::kStart) {
          // r0 = b - A x (x = 0 at first: r0 = b exactly), |r0|^2, v_0 = r0 / |r0|
          a_start.push_back(apply_job(P, 0, q.r->d_u, V, q.r->d_b, nullptr, false));
          thr_start = std::max(thr_start, P->N * P->N > 64 ? 128 : 64);
          d_start.push_back(dot_job(V, n, 1, 0, nullptr, V, n, P->d_partial, beta2));
          v_start.push_back(norm_job(P, V, beta2));
        }
        const int j = q.j;
        // w = A z_j (z_j = the cycle's output, copied to Z_j), CGS2, v_{j+1}
        a_iter.push_back(apply_job(P, 0, L0.d_u, V + (size_t)(j + 1) * n, nullptr,
                                   Z + (size_t)j * n, false));
        thr_iter = std::max(thr_iter, P->N * P->N > 64 ? 128 : 64);
        double* w = V + (size_t)(j + 1) * n;
        d1.push_back(dot_job(V, n, j + 1, 0, nullptr, w, n, P->d_partial, h1));
        d2.push_back(dot_job(V, n, j + 1, 1, h1, w, n, P->d_partial, h2));
        d3.push_back(dot_job(V, n, j + 1, 2, h2, w, n, P->d_partial, hn));
        v_iter.push_back(norm_job(P, w, hn));
      } else if (q.stage == BatchReq::kFinish) {
        const int k = q.j;
        double* hp = h_pack_ + (size_t)q.slot * stride_;
        for (int i = 0; i < k; ++i) hp[3 * m2 + i] = q.y[i];
        if (k > 0) {
          BVecJob c{};
          c.y = q.r->d_u;
          c.n = n;
          c.coef = yv;
          c.Z = Z;
          c.ldz = n;
          c.m = k;
          v_comb.push_back(c);
        }
        a_fin.push_back(apply_job(P, 0, q.r->d_u, P->d_tmp, q.r->d_b, nullptr, false));
        thr_fin = std::max(thr_fin, P->N * P->N > 64 ? 128 : 64);
        d_fin.push_back(dot_job(P->d_tmp, n, 1, 0, nullptr, P->d_tmp, n, P->d_partial, res2));
      }
    }
    // block offsets
    auto apply_blocks = [](std::vector<BApplyJob>& v) {
      int nb = 0;
      for (auto& jb : v) {
        jb.blk0 = nb;
        nb += jb.P.E;
      }
      return nb;
    };
    auto dot_blocks = [](std::vector<BDotJob>& v, int& nfinal) {
      int nb = 0;
      nfinal = 0;
      for (auto& jb : v) {
        jb.blk0 = nb;
        nb += jb.nblocks;
        jb.fblk0 = nfinal;
        nfinal += jb.mode == 2 ? 1 : jb.m;
      }
      return nb;
    };
    auto vec_blocks = [](std::vector<BVecJob>& v) {
      int nb = 0;
      for (auto& jb : v) {
        jb.blk0 = nb;
        nb += (int)((jb.n + 255) / 256);
      }
      return nb;
    };
    int fs = 0, f1 = 0, f2 = 0, f3 = 0, ff = 0;
    const int nb_as = apply_blocks(a_start), nb_ai = apply_blocks(a_iter), nb_af = apply_blocks(a_fin);
    // the residual of a starting request writes r0 into V_0
    const int nb_ds = dot_blocks(d_start, fs), nb_d1 = dot_blocks(d1, f1), nb_d2 = dot_blocks(d2, f2),
              nb_d3 = dot_blocks(d3, f3), nb_df = dot_blocks(d_fin, ff);
    const int nb_vs = vec_blocks(v_start), nb_vi = vec_blocks(v_iter), nb_vc = vec_blocks(v_comb);
    const size_t o_as = img.put(a_start), o_ai = img.put(a_iter), o_af = img.put(a_fin);
    const size_t o_ds = img.put(d_start), o_d1 = img.put(d1), o_d2 = img.put(d2), o_d3 = img.put(d3),
                 o_df = img.put(d_fin);
    const size_t o_vs = img.put(v_start), o_vi = img.put(v_iter), o_vc = img.put(v_comb);
    // ---- upload the per-step tables and the pack (the combine reads y) ----
    stage_buf_.ensure(img.bytes.size() + 16);
    if (h_stage_cap_ < img.bytes.size()) {
      std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
      if (h_stage_) (void)hipHostFree(h_stage_);
      h_stage_cap_ = std::max(img.bytes.size(), 2 * h_stage_cap_);
      HIP_OK(hipHostMalloc((void**)&h_stage_, h_stage_cap_, hipHostMallocDefault));
    }
    if (!img.bytes.empty()) {
      std::memcpy(h_stage_, img.bytes.data(), img.bytes.size());
      HIP_OK(hipMemcpyAsync(stage_buf_.p, h_stage_, img.bytes.size(), hipMemcpyHostToDevice, s_));
    }
    if (!v_comb.empty())
      HIP_OK(hipMemcpyAsync(pack_.p, h_pack_, sizeof(double) * (size_t)stride_ * max_active_,
                            hipMemcpyHostToDevice, s_));
    const DevTables* dtabs = (const DevTables*)tabs_.p;
    auto sp = [&](size_t off) { return stage_buf_.p + off; };
    // ---- starts ----
    if (nb_as) {
      HIP_OK(launch_batch_apply(kResidual, false, (const BApplyJob*)sp(o_as), (int)a_start.size(),
                                nb_as, thr_start, dtabs, s_));
      HIP_OK(launch_batch_dots((const BDotJob*)sp(o_ds), (int)d_start.size(), nb_ds, fs, s_));
      HIP_OK(launch_batch_vec((const BVecJob*)sp(o_vs), (int)v_start.size(), nb_vs, s_));
      launches_ += 4;
    }
    // ---- the multigrid cycle of every request, then the Krylov step ----
    if (nb_ai) {
      run_vcycle();
      HIP_OK(launch_batch_apply(kApply, false, (const BApplyJob*)sp(o_ai), (int)a_iter.size(), nb_ai,
                                thr_iter, dtabs, s_));
      HIP_OK(launch_batch_dots((const BDotJob*)sp(o_d1), (int)d1.size(), nb_d1, f1, s_));
      HIP_OK(launch_batch_dots((const BDotJob*)sp(o_d2), (int)d2.size(), nb_d2, f2, s_));
      HIP_OK(launch_batch_dots((const BDotJob*)sp(o_d3), (int)d3.size(), nb_d3, f3, s_));
      HIP_OK(launch_batch_vec((const BVecJob*)sp(o_vi), (int)v_iter.size(), nb_vi, s_));
      launches_ += 8;
    }
    // ---- finishes: x += Z y, the true residual ----
    if (nb_af) {
      if (nb_vc) {
        HIP_OK(launch_batch_vec((const BVecJob*)sp(o_vc), (int)v_comb.size(), nb_vc, s_));
        ++launches_;
      }
      HIP_OK(launch_batch_apply(kResidual, false, (const BApplyJob*)sp(o_af), (int)a_fin.size(),
                                nb_af, thr_fin, dtabs, s_));
      HIP_OK(launch_batch_dots((const BDotJob*)sp(o_df), (int)d_fin.size(), nb_df, ff, s_));
      launches_ += 3;
    }
    HIP_OK(hipMemcpyAsync(h_pack_, pack_.p, sizeof(double) * (size_t)stride_ * max_active_,
                          hipMemcpyDeviceToHost, s_));
    issued_ = true;
  }

  // t_wait, t_host (optional): seconds spent waiting and in the host part
  std::vector<ServerRequest*> finish(double* t_wait = nullptr, double* t_host = nullptr) {
    std::vector<ServerRequest*> finished;
    if (!issued_) return finished;
    issued_ = false;
    const double t0 = now_s();
    HIP_OK(hipStreamSynchronize(s_));
    const double t1 = now_s();
    if (t_wait) *t_wait += t1 - t0;
    struct HostClock {
      double t1;
      double* out;
      ~HostClock() {
        if (out) *out += now_s() - t1;
      }
    } clock{t1, t_host};
    // ---- host part ----
    std::vector<BatchReq> keep;
    for (BatchReq& q : reqs_) {
      complete(q);
      if (q.stage == BatchReq::kDone) {
        q.r->run.stage = FgmresRun::kDone;
        free_slots_.push_back(q.slot);
        finished.push_back(q.r);
        dirty_ = true;
      } else {
        keep.push_back(std::move(q));
      }
    }
    reqs_ = std::move(keep);
    return finished;
  }

 private:
  BApplyJob apply_job(dgs_problem* P, int l, const double* u, double* out, const double* b,
                      double* ucopy, bool rows) {
    Level& L = P->levels[l];
    BApplyJob jb{};
    jb.u = u;
    jb.out = out;
    jb.b = b;
    jb.ucopy = ucopy;
    if (rows) jb.go = level_gather(P, L);
    jb.P = L.op;
    jb.N = P->N;
    return jb;
  }
  static BDotJob dot_job(const double* V, long long ldv, int m, int mode, const double* coef,
                         double* w, long long n, double* partial, double* h) {
    BDotJob jb{};
    jb.V = V;
    jb.ldv = ldv;
    jb.m = m;
    jb.mode = mode;
    jb.coef = coef;
    jb.w = w;
    jb.n = n;
    jb.nblocks = multidot_blocks(n);
    jb.chunk = (n + jb.nblocks - 1) / jb.nblocks;
    jb.partial = partial;
    jb.h = h;
    return jb;
  }
  // v = w / sqrt(*nrm2), also into the finest level's b and subdomain rows
  // (the cycle's input)
  static BVecJob norm_job(dgs_problem* P, double* w, const double* nrm2) {
    Level& L0 = P->levels[0];
    BVecJob jb{};
    jb.y = w;
    jb.x = w;
    jb.nrm2 = nrm2;
    jb.y2 = L0.d_b;
    jb.go = level_gather(P, L0);
    jb.n = P->nd(0);
    jb.N = P->N;
    return jb;
  }

  void new_cycle(BatchReq& q) {
    q.stage = BatchReq::kStart;
    q.j = 0;
    q.H.assign((size_t)(q.m + 1) * q.m, 0.0);
    q.cs.assign(q.m, 0.0);
    q.sn.assign(q.m, 0.0);
    q.g.assign(q.m + 1, 0.0);
  }

  // The host part of a request's step: the scalars of the pack.
  void complete(BatchReq& q) {
    FgmresResult& R = q.r->run.R;
    const double* hp = h_pack_ + (size_t)q.slot * stride_;
    const int m2 = q.m + 2;
    auto fail_nonfinite = [&]() {
      R.converged = false;
      R.rel_residual = std::numeric_limits<double>::quiet_NaN();
      q.r->status = DGS_ERR_NONFINITE;
      q.stage = BatchReq::kDone;
    };
    if (q.stage == BatchReq::kFinish) {
      R.rel_residual = std::sqrt(hp[2 * m2 + 2]) / q.beta0;
      if (!std::isfinite(R.rel_residual)) return fail_nonfinite();
      // the Givens estimate ended the cycle; the true residual decides
      R.converged = R.rel_residual <= q.rtol;
      if (!R.converged && q.iterations < q.max_total)
        new_cycle(q);  // the next cycle starts from the true residual of x
      else
        q.stage = BatchReq::kDone;
      return;
    }
    if (q.stage == BatchReq::kStart) {
      const double beta2 = hp[2 * m2 + 1];
      if (!std::isfinite(beta2)) return fail_nonfinite();
      q.beta = std::sqrt(beta2);
      if (q.cycles++ == 0) {
        q.beta0 = q.beta;
        R.history.push_back(1.0);
      }
      if (q.beta == 0.0) {  // b = A x already: nothing to iterate
        R.converged = true;
        R.rel_residual = 0.0;
        q.stage = BatchReq::kDone;
        return;
      }
      q.g[0] = q.beta;
      q.stage = BatchReq::kIter;
    }
    // the iteration this step ran: Hessenberg column j, Givens rotations
    const int j = q.j;
    double* col = &q.H[(size_t)j * (q.m + 1)];
    for (int i = 0; i <= j; ++i) col[i] = hp[i] + hp[m2 + i];
    const double hn2 = hp[2 * m2];
    col[j + 1] = std::sqrt(hn2);
    for (int i = 0; i <= j + 1; ++i)
      if (!std::isfinite(col[i])) return fail_nonfinite();
    for (int i = 0; i < j; ++i) {
      const double t = q.cs[i] * col[i] + q.sn[i] * col[i + 1];
      col[i + 1] = -q.sn[i] * col[i] + q.cs[i] * col[i + 1];
      col[i] = t;
    }
    const double den = std::hypot(col[j], col[j + 1]);
    q.cs[j] = col[j] / den;
    q.sn[j] = col[j + 1] / den;
    col[j] = den;
    col[j + 1] = 0.0;
    q.g[j + 1] = -q.sn[j] * q.g[j];
    q.g[j] = q.cs[j] * q.g[j];
    R.history.push_back(std::fabs(q.g[j + 1]) / q.beta0);
    ++q.j;
    ++q.iterations;
    R.iterations = q.iterations;
    if (std::fabs(q.g[q.j]) <= q.rtol * q.beta0 || hn2 == 0.0 || q.j >= q.m ||
        q.iterations >= q.max_total) {
      // y from the triangular system; the next step forms x += Z y and the
      // true residual
      const int k = q.j;
      q.y.assign(k, 0.0);
      for (int i = k - 1; i >= 0; --i) {
        double t = q.g[i];
        for (int c = i + 1; c < k; ++c) t -= q.H[(size_t)c * (q.m + 1) + i] * q.y[c];
        q.y[i] = t / q.H[(size_t)i * (q.m + 1) + i];
      }
      q.stage = BatchReq::kFinish;
    }
  }

  // ---- the multigrid cycle over every request (Sec. III.C.3) ----
  // The schedule by level index: on level l every request that has it runs
  // its smoothing steps (presmoothing, or on its coarsest level the coarse
  // steps), the requests with a coarser level restrict their residual; on the
  // way back the requests prolongate and postsmooth.  Step s of a level
  // covers the requests that take more than s steps there.
  void rebuild() {
    ops_.clear();
    JobImage img;
    int Lmax = 0;
    for (BatchReq& q : reqs_) Lmax = std::max(Lmax, (int)q.r->prob->levels.size());
    auto depth = [](const BatchReq& q) { return (int)q.r->prob->levels.size(); };
    auto coarse_steps = [](const dgs_problem* P) {
      const Level& Lc = P->levels.back();
      int c = P->opt.pre_smooth + P->opt.post_smooth;
      if (Lc.E == 1) c = std::min(c, 1);  // one subdomain: the first step is exact
      return c;
    };
    auto smoothing_ops = [&](int l, const std::vector<BatchReq*>& S, bool first) {
      // residual + gather (not in a first step from zero: r = b is gathered)
      if (!first) {
        std::vector<BApplyJob> aj;
        int threads = 64;
        for (BatchReq* q : S) {
          dgs_problem* P = q->r->prob;
          Level& L = P->levels[l];
          aj.push_back(apply_job(P, l, L.d_u, nullptr, L.d_b, nullptr, true));
          threads = std::max(threads, P->N * P->N > 64 ? 128 : 64);
        }
        BatchOp op;
        op.kind = kOpApplyRows;
        int nb = 0;
        for (auto& jb : aj) {
          jb.blk0 = nb;
          nb += jb.P.E;
        }
        op.nblocks = nb;
        op.njobs = (int)aj.size();
        op.threads = threads;
        op.off = img.put(aj);
        ops_.push_back(op);
      }
      // the subdomain solves: one grouped GEMM per precision over all classes
      std::vector<BScatterJob> sj;
      for (int prec = 0; prec < 2; ++prec) {
        std::vector<ClassInfo> cls;
        std::vector<GemmPtr> ptrs;
        std::vector<BatchReq*> who;
        int cap = kMaxParts;
        for (BatchReq* q : S) {
          Level& L = q->r->prob->levels[l];
          if ((int)L.f32 != prec) continue;
          int lp = 1;
          for (int v = 0; v < kGemmVariants; ++v) lp = std::max(lp, L.kparts_of[v]);
          cap = std::min(cap, lp);
          for (const ClassInfo& c : L.cls) {
            cls.push_back(c);
            ptrs.push_back(GemmPtr{L.d_rs, L.d_du, L.rs_total});
          }
          who.push_back(q);
        }
        if (cls.empty()) continue;
        const GemmPlan plan = plan_subdomain_gemm(cls, 2, cap);
        BatchOp op;
        op.kind = kOpGemm;
        op.f32 = prec == 1;
        op.small = plan.small;
        op.njobs = (int)plan.tiles.size();
        op.off = img.put(cls);
        op.off_ptrs = img.put(ptrs);
        op.off_tiles = img.put(plan.tiles);
        ops_.push_back(op);
        for (BatchReq* q : who) {
          dgs_problem* P = q->r->prob;
          Level& L = P->levels[l];
          BScatterJob s{};
          s.u = L.d_u;
          s.du = L.d_du;
          s.weights = L.d_weights;
          s.pull = L.d_pull;
          s.pstride = L.rs_total;
          s.total = L.E * (long long)P->N * P->N * P->N;
          s.N = P->N;
          s.nov = nov_of(P);
          s.parts = plan.kparts;
          s.f32 = L.f32 ? 1 : 0;
          s.assign = first ? 1 : 0;
          sj.push_back(s);
        }
      }
      BatchOp op;
      op.kind = kOpScatter;
      int nb = 0;
      for (auto& jb : sj) {
        jb.blk0 = nb;
        nb += (int)((jb.total + 255) / 256);
      }
      op.nblocks = nb;
      op.njobs = (int)sj.size();
      op.off = img.put(sj);
      ops_.push_back(op);
    };
    // descent
    for (int l = 0; l < Lmax; ++l) {
      std::vector<BatchReq*> part;
      for (BatchReq& q : reqs_)
        if (depth(q) > l) part.push_back(&q);
      auto steps_of = [&](BatchReq* q) {
        const dgs_problem* P = q->r->prob;
        return l < depth(*q) - 1 ? P->opt.pre_smooth : coarse_steps(P);
      };
      int smax = 0;
      for (BatchReq* q : part) smax = std::max(smax, steps_of(q));
      for (int st = 0; st < smax; ++st) {
        std::vector<BatchReq*> S;
        for (BatchReq* q : part)
          if (steps_of(q) > st) S.push_back(q);
        smoothing_ops(l, S, st == 0);
      }
      // residual and restriction of the requests with a coarser level
      std::vector<BApplyJob> aj;
      std::vector<BTransferJob> tj;
      int threads = 64;
      for (BatchReq* q : part) {
        if (l >= depth(*q) - 1) continue;
        dgs_problem* P = q->r->prob;
        Level& L = P->levels[l];
        Level& C = P->levels[l + 1];
        aj.push_back(apply_job(P, l, L.d_u, L.d_r, L.d_b, nullptr, false));
        threads = std::max(threads, P->N * P->N > 64 ? 128 : 64);
        BTransferJob t{};
        t.src = L.d_r;
        t.dst = C.d_b;
        t.go = level_gather(P, C);
        for (int d = 0; d < 3; ++d) {
          t.nf[d] = L.n[d];
          t.nc[d] = C.n[d];
          t.split[d] = L.split[d];
        }
        t.N = P->N;
        tj.push_back(t);
      }
      if (!aj.empty()) {
        BatchOp a;
        a.kind = kOpApplyVec;
        int nb = 0;
        for (auto& jb : aj) {
          jb.blk0 = nb;
          nb += jb.P.E;
        }
        a.nblocks = nb;
        a.njobs = (int)aj.size();
        a.threads = threads;
        a.off = img.put(aj);
        ops_.push_back(a);
        BatchOp r;
        r.kind = kOpRestrict;
        nb = 0;
        for (auto& jb : tj) {
          jb.blk0 = nb;
          nb += jb.nc[0] * jb.nc[1] * jb.nc[2];
        }
        r.nblocks = nb;
        r.njobs = (int)tj.size();
        r.off = img.put(tj);
        ops_.push_back(r);
      }
    }
    // ascent
    for (int l = Lmax - 2; l >= 0; --l) {
      std::vector<BatchReq*> Q;
      for (BatchReq& q : reqs_)
        if (l < depth(q) - 1) Q.push_back(&q);
      if (Q.empty()) continue;
      std::vector<BTransferJob> tj;
      for (BatchReq* q : Q) {
        dgs_problem* P = q->r->prob;
        Level& L = P->levels[l];
        Level& C = P->levels[l + 1];
        BTransferJob t{};
        t.src = C.d_u;
        t.dst = L.d_u;
        for (int d = 0; d < 3; ++d) {
          t.nf[d] = L.n[d];
          t.nc[d] = C.n[d];
          t.split[d] = L.split[d];
        }
        t.N = P->N;
        tj.push_back(t);
      }
      BatchOp pr;
      pr.kind = kOpProlong;
      int nb = 0;
      for (auto& jb : tj) {
        jb.blk0 = nb;
        nb += jb.nf[0] * jb.nf[1] * jb.nf[2];
      }
      pr.nblocks = nb;
      pr.njobs = (int)tj.size();
      pr.off = img.put(tj);
      ops_.push_back(pr);
      int post = 0;
      for (BatchReq* q : Q) post = std::max(post, q->r->prob->opt.post_smooth);
      for (int st = 0; st < post; ++st) {
        std::vector<BatchReq*> S;
        for (BatchReq* q : Q)
          if (q->r->prob->opt.post_smooth > st) S.push_back(q);
        smoothing_ops(l, S, false);
      }
    }
    vbuf_.ensure(img.bytes.size() + 16);
    HIP_OK(hipMemcpyAsync(vbuf_.p, img.bytes.data(), img.bytes.size(), hipMemcpyHostToDevice, s_));
    HIP_OK(hipStreamSynchronize(s_));  // img goes out of scope
    dirty_ = false;
  }

  void run_vcycle() {
    const DevTables* dtabs = (const DevTables*)tabs_.p;
    const MgTables* mtabs = (const MgTables*)(tabs_.p + mt_off_);
    for (const BatchOp& op : ops_) {
      char* base = vbuf_.p;
      switch (op.kind) {
        case kOpApplyRows:
          HIP_OK(launch_batch_apply(kResidual, true, (const BApplyJob*)(base + op.off), op.njobs,
                                    op.nblocks, op.threads, dtabs, s_));
          break;
        case kOpApplyVec:
          HIP_OK(launch_batch_apply(kResidual, false, (const BApplyJob*)(base + op.off), op.njobs,
                                    op.nblocks, op.threads, dtabs, s_));
          break;
        case kOpGemm:
          HIP_OK(launch_subdomain_gemm_batched(op.f32, (const ClassInfo*)(base + op.off),
                                               (const GemmPtr*)(base + op.off_ptrs),
                                               (const GemmTile*)(base + op.off_tiles), op.njobs,
                                               op.small, s_));
          break;
        case kOpScatter:
          HIP_OK(launch_batch_scatter((const BScatterJob*)(base + op.off), op.njobs, op.nblocks, s_));
          break;
        case kOpRestrict:
          HIP_OK(launch_batch_restrict((const BTransferJob*)(base + op.off), op.njobs, op.nblocks,
                                       mtabs, s_));
          break;
        case kOpProlong:
          HIP_OK(launch_batch_prolongate((const BTransferJob*)(base + op.off), op.njobs, op.nblocks,
                                         mtabs, s_));
          break;
      }
      ++launches_;
    }
  }

  int max_active_ = 0, kmax_ = 0, restart_ = 0, stride_ = 0;
  hipStream_t s_ = nullptr;
  DevBuf pack_, tabs_, vbuf_, stage_buf_;
  size_t mt_off_ = 0;
  double* h_pack_ = nullptr;
  char* h_stage_ = nullptr;
  size_t h_stage_cap_ = 0;
  std::vector<int> free_slots_;
  std::vector<BatchReq> reqs_;
  std::vector<BatchOp> ops_;
  bool dirty_ = true;
  bool issued_ = false;  // a step is on the device and finish() has not run
  int launches_ = 0;
};

}  // namespace


namespace {

// Persistent worker threads bound to one device: run(f) calls f(w) on every
// worker w = 0..n-1 in parallel and returns when all are done, rethrowing the
// first exception a worker raised.
class WorkerPool {
 public:
  WorkerPool(int n, int device) : errors_(n) {
    for (int w = 0; w < n; ++w) threads_.emplace_back([this, w, device] { loop(w, device); });
  }
  ~WorkerPool() {
    {
      std::lock_guard<std::mutex> lk(m_);
      quit_ = true;
    }
    cv_start_.notify_all();
    for (auto& t : threads_) t.join();
  }
  int size() const { return (int)threads_.size(); }
  void run(const std::function<void(int)>& f) {
    {
      std::lock_guard<std::mutex> lk(m_);
      task_ = f;
      pending_ = (int)threads_.size();
      ++generation_;
    }
    cv_start_.notify_all();
    std::unique_lock<std::mutex> lk(m_);
    cv_done_.wait(lk, [this] { return pending_ == 0; });
    for (auto& e : errors_)
      if (e) {
        std::exception_ptr first = e;
        for (auto& x : errors_) x = nullptr;
        std::rethrow_exception(first);
      }
  }

 private:
  void loop(int w, int device) {
    (void)hipSetDevice(device);
    long long seen = 0;
    for (;;) {
      std::function<void(int)> f;
      {
        std::unique_lock<std::mutex> lk(m_);
        cv_start_.wait(lk, [&] { return quit_ || generation_ != seen; });
        if (quit_) return;
        seen = generation_;
        f = task_;
      }
      try {
        f(w);
      } catch (...) {
        errors_[w] = std::current_exception();
      }
      std::lock_guard<std::mutex> lk(m_);
      if (--pending_ == 0) cv_done_.notify_one();
    }
  }
  std::vector<std::thread> threads_;
  std::vector<std::exception_ptr> errors_;
  std::mutex m_;
  std::condition_variable cv_start_, cv_done_;
  std::function<void(int)> task_;
  long long generation_ = 0;
  int pending_ = 0;
  bool quit_ = false;
};

}  // namespace

namespace {
int create_problem(const dgs_domain* domain, const int elements[3], int p, double penalty,
                   const dgs_options* opt, dgs_alloc_fn alloc_fn, dgs_free_fn free_fn,
                   void* alloc_ctx, void* stream, dgs_problem** out, bool light,
                   const std::vector<int>* class_masks = nullptr);
}  // namespace

// Device blocks of a server's requests when the caller gives no allocator.
// A freed block is kept by its size class (the next power of two) and handed
// out again, so that retiring a request costs no hipFree, which waits for
// the whole device; blocks are freed only once their request's work has
// finished.  Held blocks beyond `cap` bytes, and all of them when the server
// is destroyed, go back with hipFree.
struct BlockPool {
  std::mutex m;
  std::map<size_t, std::vector<void*>> free;  // by size class
  std::unordered_map<void*, size_t> size_of;   // every block handed out
  size_t held = 0, cap = 0;
  static size_t size_class(size_t bytes) {
    size_t c = 256;
    while (c < bytes) c <<= 1;
    return c;
  }
  void* get(size_t bytes) {
    const size_t c = size_class(bytes);
    {
      std::lock_guard<std::mutex> lk(m);
      auto it = free.find(c);
      if (it != free.end() && !it->second.empty()) {
        void* p = it->second.back();
        it->second.pop_back();
        held -= c;
        size_of[p] = c;
        return p;
      }
    }
    void* p = dalloc<char>(c);
    std::lock_guard<std::mutex> lk(m);
    size_of[p] = c;
    return p;
  }
  void put(void* p) {
    std::lock_guard<std::mutex> lk(m);
    auto it = size_of.find(p);
    if (it == size_of.end()) return;
    const size_t c = it->second;
    size_of.erase(it);
    if (held + c > cap) {
      dfree(p);
      return;
    }
    free[c].push_back(p);
    held += c;
  }
  ~BlockPool() {
    for (auto& kv : free)
      for (void* p : kv.second) (void)hipFree(p);
  }
  static void* alloc_cb(size_t bytes, void* ctx) { return static_cast<BlockPool*>(ctx)->get(bytes); }
  static void free_cb(void* p, void* ctx) { static_cast<BlockPool*>(ctx)->put(p); }
};

// Device memory of a retired request, freed later in a batch: freeing waits
// for the whole device, which would drain the other requests' stages.
struct RetiredMemory {
  dgs_problem* prob;
  double *d_b, *d_u, *d_alpha, *d_beta;
  size_t footprint;
};

struct dgs_server {
  dgs_server_options opt{};
  // the library's block pool, used when the caller gives no allocator
  BlockPool blocks;
  dgs_alloc_fn alloc_fn() const { return opt.alloc_fn ? opt.alloc_fn : &BlockPool::alloc_cb; }
  dgs_free_fn free_fn() const { return opt.alloc_fn ? opt.free_fn : &BlockPool::free_cb; }
  void* alloc_ctx() { return opt.alloc_fn ? opt.alloc_ctx : (void*)&blocks; }
  // the requests' own vectors (b, u, puncture fields) from the caller's
  // allocator when one is given, else from the block pool
  double* vec(size_t n) {
    std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
    void* p = alloc_fn()(std::max<size_t>(n, 1) * sizeof(double), alloc_ctx());
    if (!p) throw DgsError(DGS_ERR_OOM, "the caller's allocator returned NULL");
    return static_cast<double*>(p);
  }
  // released only after the device has finished with it
  void vec_free(double* p) {
    if (!p) return;
    std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
    free_fn()(p, alloc_ctx());
  }
  int device = 0;
  std::unique_ptr<WorkerPool> pool;  // launching is host-bound: stages run in parallel
  long long next_id = 1;
  size_t used = 0;  // footprints of the active requests and of the unfreed retired ones
  std::vector<std::unique_ptr<ServerRequest>> queue, active;
  std::map<long long, std::unique_ptr<ServerRequest>> finished;
  std::vector<hipStream_t> free_streams;
  std::vector<RetiredMemory> retired;
  // finished requests' problems (hierarchy, inverses' class tables, Krylov
  // basis, captured V-cycle graphs) kept for the next request of the same
  // box, grid and degree; most recently used last.  Their footprints stay in
  // `used` until they are freed.
  struct Idle {
    std::array<double, 6> box;
    std::array<int, 4> grid;  // elements, p
    dgs_problem* prob;
    double *d_b, *d_u;
    size_t footprint;
    bool batched;  // a light problem of the batch engine
  };
  // the cross-request batch engine (created with the first batched request)
  std::unique_ptr<BatchEngine> engine;
  long long steps = 0, batch_steps = 0, batch_launches = 0, batch_peak = 0;
  // host seconds spent in: admission and the per-request work of the workers
  // (set-up included), issuing the engine's steps, waiting for them, and the
  // engine's host part
  double t_workers = 0, t_issue = 0, t_wait = 0, t_engine_host = 0, t_retire = 0;
  std::vector<Idle> idle;
  double t0 = 0;
  void evict_idle(size_t keep) {  // oldest first, into the batch of frees
    while (idle.size() > keep) {
      Idle& m = idle.front();
      retired.push_back(RetiredMemory{m.prob, m.d_b, m.d_u, nullptr, nullptr, m.footprint});
      idle.erase(idle.begin());
    }
  }
  void free_retired() {
    // a caller's allocator may hand the memory out at once (hipFree waits by itself)
    if (opt.alloc_fn && !retired.empty()) (void)hipDeviceSynchronize();
    for (RetiredMemory& m : retired) {
      if (m.prob) delete m.prob;
      for (double* d : {m.d_b, m.d_u, m.d_alpha, m.d_beta}) vec_free(d);
      used -= m.footprint;
    }
    retired.clear();
  }
  ~dgs_server() {
    pool.reset();
    engine.reset();
    for (auto& r : active) {
      if (r->stream) (void)hipStreamSynchronize(r->stream);  // a stage may be in flight
      if (r->prob) delete r->prob;
      for (double* d : {r->d_b, r->d_u, r->d_alpha, r->d_beta}) vec_free(d);
      if (r->stream) (void)hipStreamDestroy(r->stream);
    }
    evict_idle(0);
    free_retired();
    for (hipStream_t st : free_streams) (void)hipStreamDestroy(st);
  }
};

namespace {

size_t request_footprint(const dgs_server* S, const int el[3], int p) {
  const double ndof = (double)el[0] * el[1] * el[2] * (p + 1.0) * (p + 1.0) * (p + 1.0);
  // Krylov basis (2m+1 vectors), b and u, Newton-free work vectors, level
  // vectors and Schwarz buffers (about 16 vectors' worth, all levels together)
  const double vecs = 2.0 * S->opt.solver.max_iter + 1 + 2 + 4 + 16;
  return (size_t)(ndof * 8.0 * vecs);
}

// Retired requests' memory is released in batches of this many, or sooner
// when a queued request would otherwise not fit the budget.
constexpr size_t kRetiredBatch = 16;
// finished requests' problems kept resident for reuse
constexpr size_t kIdleMax = 32;

// Set-up of one admitted request on its stream: problem (hierarchy, classes,
// inverses from the cache), b = M f, u = 0, and the FGMRES state.
void server_setup(dgs_server* S, ServerRequest& r) {
  const double ta = now_s();
  if (!r.reused) {
    dgs_problem* created = nullptr;
    const int code = create_problem(&r.dom, r.elements, r.p, S->opt.penalty, &S->opt.solver,
                                    S->alloc_fn(), S->free_fn(), S->alloc_ctx(), r.stream,
                                    &created, r.batched);
    if (code != DGS_OK) throw DgsError(code, g_last_error);
    // a server deletes a problem only once its work has finished
    if (!S->opt.alloc_fn) created->sync_before_free = false;
    r.prob = created;
    r.d_b = S->vec(created->nd(0));
    r.d_u = S->vec(created->nd(0));
  }
  dgs_problem* prob = r.prob;
  const long long n = prob->nd(0);
  if (r.kind == 0) {
    // f to the device (pinned staging is not needed: a one-off copy), b = M f
    HIP_OK(hipMemcpyAsync(r.d_u, r.f.data(), sizeof(double) * n, hipMemcpyHostToDevice, r.stream));
    const Level& L0 = prob->levels[0];
    HIP_OK(launch_mass(prob->N, r.d_u, r.d_b, L0.E, L0.h, prob->dt, r.stream));
    HIP_OK(launch_fill(r.d_u, 0.0, n, r.stream));
    if (r.batched) {  // the batch engine takes it from here, on its own stream
      r.run.P = prob;
      r.run.b = r.d_b;
      r.run.x = r.d_u;
      r.run.rtol = S->opt.solver.rtol;
      r.run.max_total = S->opt.solver.max_iter;
      r.run.stage = FgmresRun::kStart;
      HIP_OK(hipStreamSynchronize(r.stream));
    } else {
      r.run.init(prob, r.d_b, r.d_u, S->opt.solver.rtol, S->opt.solver.max_iter, r.stream);
    }
  } else {
    // the puncture equation: alpha, beta and b (zero when not given) to the
    // device, u0 = 0, and the first nonlinear residual
    r.d_alpha = S->vec(n);
    r.d_beta = S->vec(n);
    HIP_OK(hipMemcpyAsync(r.d_alpha, r.alpha.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                          r.stream));
    HIP_OK(hipMemcpyAsync(r.d_beta, r.beta.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                          r.stream));
    if (r.has_b)
      HIP_OK(hipMemcpyAsync(r.d_b, r.f.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                            r.stream));
    else
      HIP_OK(launch_fill(r.d_b, 0.0, n, r.stream));
    HIP_OK(launch_fill(r.d_u, 0.0, n, r.stream));
    r.nrun.init(prob, r.d_alpha, r.d_beta, r.d_b, r.d_u, r.newton_rtol, r.linear_rtol,
                r.max_newton, r.stream);
  }
  r.t_setup = now_s() - ta;
  r.t_admit = ta - S->t0;
}

// Admission: the queued requests that fit (slots, budget), in order, with a
// stream and, where one of the same shape is idle, a resident problem; their
// set-up is left to the workers.
std::vector<std::unique_ptr<ServerRequest>> server_select(dgs_server* S) {
  if (S->retired.size() >= kRetiredBatch) S->free_retired();
  std::vector<std::unique_ptr<ServerRequest>> admitted;
  while (!S->queue.empty() && (int)(S->active.size() + admitted.size()) < S->opt.max_active) {
    ServerRequest& r = *S->queue.front();
    const std::array<double, 6> box = {r.dom.lower[0], r.dom.lower[1], r.dom.lower[2],
                                       r.dom.upper[0], r.dom.upper[1], r.dom.upper[2]};
    const std::array<int, 4> grid = {r.elements[0], r.elements[1], r.elements[2], r.p};
    int match = -1;  // most recently used idle problem of this shape
    for (int i = (int)S->idle.size() - 1; i >= 0 && match < 0; --i)
      if (S->idle[i].box == box && S->idle[i].grid == grid && S->idle[i].batched == r.batched)
        match = i;
    // a reused problem's footprint is already counted; only what this request
    // needs beyond it (a puncture request on a Poisson request's problem) is new
    auto extra = [&](int i) -> size_t {
      return r.footprint > S->idle[i].footprint ? r.footprint - S->idle[i].footprint : 0;
    };
    const size_t need = match >= 0 ? extra(match) : r.footprint;
    const size_t budget = (size_t)S->opt.hbm_budget_bytes;
    if (S->used + need > budget) {
      S->evict_idle(0);
      match = -1;
      S->free_retired();
    }
    const size_t need2 = match >= 0 ? extra(match) : r.footprint;
    const bool none_running = S->active.empty() && admitted.empty();
    if (S->used + need2 > budget && !none_running) break;
    if (S->used + need2 > budget && none_running && r.footprint > budget) {
      // can never fit: reject
      std::unique_ptr<ServerRequest> rq = std::move(S->queue.front());
      S->queue.erase(S->queue.begin());
      rq->status = DGS_ERR_OOM;
      rq->t_done = now_s() - S->t0;
      S->finished[rq->id] = std::move(rq);
      continue;
    }
    std::unique_ptr<ServerRequest> rq = std::move(S->queue.front());
    S->queue.erase(S->queue.begin());
    if (!S->free_streams.empty()) {
      rq->stream = S->free_streams.back();
      S->free_streams.pop_back();
    } else {
      std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
      HIP_OK(hipStreamCreateWithFlags(&rq->stream, hipStreamNonBlocking));
    }
    if (match >= 0) {
      const dgs_server::Idle m = S->idle[match];
      S->idle.erase(S->idle.begin() + match);
      rq->prob = m.prob;
      rq->d_b = m.d_b;
      rq->d_u = m.d_u;
      S->used += need2;
      rq->footprint = m.footprint + need2;
      rq->reused = true;
    } else {
      S->used += rq->footprint;
    }
    admitted.push_back(std::move(rq));
  }
  return admitted;
}

void server_retire(dgs_server* S, std::unique_ptr<ServerRequest> rq) {
  const long long n = rq->prob->nd(0);
  rq->u.resize(n);
  HIP_OK(hipMemcpyAsync(rq->u.data(), rq->d_u, sizeof(double) * n, hipMemcpyDeviceToHost, rq->stream));
  HIP_OK(hipStreamSynchronize(rq->stream));
  if (rq->kind == 0) {
    rq->result = rq->run.R;
  } else {
    rq->result.iterations = rq->nrun.its;
    rq->result.rel_residual = rq->nrun.rel_residual();
    rq->result.converged = rq->nrun.converged;
    rq->result.history = rq->nrun.hist;
    rq->newton_steps = rq->nrun.steps;
    rq->backtracks = rq->nrun.backtracks;
  }
  if (rq->status >= 0) rq->status = rq->result.converged ? DGS_OK : DGS_NOT_CONVERGED;
  rq->t_done = now_s() - S->t0;
  // the problem stays resident for the next request of its shape; the
  // puncture fields go with the next batch of frees
  S->idle.push_back(dgs_server::Idle{
      {rq->dom.lower[0], rq->dom.lower[1], rq->dom.lower[2], rq->dom.upper[0], rq->dom.upper[1],
       rq->dom.upper[2]},
      {rq->elements[0], rq->elements[1], rq->elements[2], rq->p},
      rq->prob, rq->d_b, rq->d_u, rq->footprint, rq->batched});
  if (rq->d_alpha || rq->d_beta)
    S->retired.push_back(RetiredMemory{nullptr, nullptr, nullptr, rq->d_alpha, rq->d_beta, 0});
  S->evict_idle(kIdleMax);
  rq->prob = nullptr;
  rq->d_b = rq->d_u = rq->d_alpha = rq->d_beta = nullptr;
  rq->alpha.clear();
  rq->alpha.shrink_to_fit();
  rq->beta.clear();
  rq->beta.shrink_to_fit();
  S->free_streams.push_back(rq->stream);
  rq->stream = nullptr;
  rq->f.clear();
  rq->f.shrink_to_fit();
  S->finished[rq->id] = std::move(rq);
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void dgs_default_options(dgs_options* o) {
  if (!o) return;
  o->overlap = 2;
  o->mg_levels = 0;
  o->pre_smooth = 3;
  o->post_smooth = 3;
  o->precision = DGS_FP64;
  o->subdomain_iters = 3;
  o->max_iter = 200;
  o->rtol = 1e-10;
  o->use_graphs = 1;
  o->restart = 0;
  o->cycle = 1;
  o->additive = 0;
  o->neumann_faces = 0;
}

const char* dgs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {
// light: no launch-shape / GEMM-variant autotuning and no captured cycles
// (problems of the serving loop's batch engine use neither)
int create_problem(const dgs_domain* domain, const int elements[3], int p, double penalty,
                   const dgs_options* opt, dgs_alloc_fn alloc_fn, dgs_free_fn free_fn,
                   void* alloc_ctx, void* stream, dgs_problem** out, bool light,
                   const std::vector<int>* class_masks) {
  return guarded([&]() -> int {
    if (!domain || !elements || !out) return fail(DGS_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (!alloc_fn != !free_fn) return fail(DGS_ERR_INVALID, "alloc_fn and free_fn go together");
    if (p < 1 || p > kMaxN - 1) return fail(DGS_ERR_INVALID, "p must be in [1, 12]");
    if (!(penalty > 0.0) || !std::isfinite(penalty)) return fail(DGS_ERR_INVALID, "penalty must be > 0");
    for (int d = 0; d < 3; ++d) {
      if (elements[d] < 1) return fail(DGS_ERR_INVALID, "element counts must be >= 1");
      if (!(domain->upper[d] > domain->lower[d]) || !std::isfinite(domain->upper[d] - domain->lower[d]))
        return fail(DGS_ERR_INVALID, "domain upper must exceed lower");
    }
    dgs_options o;
    dgs_default_options(&o);
    if (opt) o = *opt;
    if (o.overlap < 1 || o.pre_smooth < 0 || o.post_smooth < 0 || o.mg_levels < 0 ||
        o.max_iter < 1 || !(o.rtol > 0.0) || o.subdomain_iters < 0 || o.subdomain_iters > 8 ||
        o.restart < 0 || o.cycle < 1 || o.cycle > 3 || o.additive < 0 || o.additive > 1 ||
        o.neumann_faces < 0 || o.neumann_faces >= 63 ||
        (o.precision != DGS_FP64 && o.precision != DGS_MIXED))
      return fail(DGS_ERR_INVALID, "invalid options");
    const long long E0 = (long long)elements[0] * elements[1] * elements[2];
    const long long N3 = (long long)(p + 1) * (p + 1) * (p + 1);
    if (E0 > (1LL << 30) / 8 || E0 * N3 > (1LL << 31) - 1)
      return fail(DGS_ERR_INVALID, "mesh too large for 32-bit element indexing");
    const double t0 = now_s();
    hipStream_t s = as_stream(stream);
    std::unique_ptr<dgs_problem> P(new dgs_problem());
    P->alloc_fn = alloc_fn;
    P->free_fn = free_fn;
    P->alloc_ctx = alloc_ctx;
    P->opt = o;
    P->p = p;
    P->N = p + 1;
    P->penalty = penalty;
    P->dom = *domain;
    if (class_masks) P->class_masks = *class_masks;
    P->ht = make_tables(P->N);
    P->dt = to_dev(P->ht);
    P->mt = to_dev_mg(P->ht);
    // hierarchy (Sec. III.C.1): halve every even element count > 1
    int n[3] = {elements[0], elements[1], elements[2]};
    const int max_levels = o.mg_levels > 0 ? o.mg_levels : 64;
    for (int l = 0; l < max_levels; ++l) {
      Level L;
      L.n[0] = n[0];
      L.n[1] = n[1];
      L.n[2] = n[2];
      bool any = false;
      for (int d = 0; d < 3; ++d) {
        L.split[d] = (n[d] > 1 && n[d] % 2 == 0) ? 1 : 0;
        any = any || L.split[d];
      }
      P->levels.push_back(L);
      if (!any || l == max_levels - 1) break;
      for (int d = 0; d < 3; ++d)
        if (L.split[d]) n[d] /= 2;
    }
    const int nl = (int)P->levels.size();
    for (int l = 0; l < nl; ++l) {
      Level& L = P->levels[l];
      L.has_coarser = l < nl - 1;
      if (!L.has_coarser) L.split[0] = L.split[1] = L.split[2] = 0;
      // mixed precision: FP32 subdomain solves everywhere except the coarsest grid
      L.f32 = (o.precision == DGS_MIXED) && L.has_coarser;
      build_level_mesh(P.get(), L, s);
      build_level_schwarz(P.get(), L, s);
    }
    build_inverses(P.get(), s);
    if (!light) {
      autotune_apply(P.get(), s);
      autotune_gemm(P.get(), s);
      if (o.use_graphs) capture_vgraph(P.get(), 0);
    }
    HIP_OK(hipStreamSynchronize(s));
    P->setup_keep.clear();
    P->t_setup = now_s() - t0;
    *out = P.release();
    return DGS_OK;
  });
}
}  // namespace

extern "C" {

int dgs_create_problem(const dgs_domain* domain, const int elements[3], int p, double penalty,
                       const dgs_options* opt, dgs_alloc_fn alloc_fn, dgs_free_fn free_fn,
                       void* alloc_ctx, void* stream, dgs_problem** out) {
  return create_problem(domain, elements, p, penalty, opt, alloc_fn, free_fn, alloc_ctx, stream,
                        out, false);
}

int dgs_destroy_problem(dgs_problem* prob) {
  return guarded([&]() -> int {
    if (!prob) return DGS_OK;
    (void)hipDeviceSynchronize();
    delete prob;
    return DGS_OK;
  });
}

int dgs_num_dofs(const dgs_problem* prob, long long* n) {
  if (!prob || !n) return fail(DGS_ERR_INVALID, "NULL argument");
  *n = prob->nd(0);
  return DGS_OK;
}

int dgs_node_coordinates(const dgs_problem* prob, double* xyz, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !xyz) return fail(DGS_ERR_INVALID, "NULL argument");
    const Level& L = prob->levels[0];
    HIP_OK(launch_coords(prob->N, xyz, L.n, prob->dom.lower, L.h, prob->dt, as_stream(stream)));
    return DGS_OK;
  });
}

int dgs_apply_mass(const dgs_problem* prob, const double* f, double* b, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !f || !b) return fail(DGS_ERR_INVALID, "NULL argument");
    const Level& L = prob->levels[0];
    if (prob->metric_on)
      HIP_OK(launch_curved_mass_metric(prob->N, f, b, prob->curved, prob->metric, L.E,
                                       as_stream(stream)));
    else if (prob->curved_on)
      HIP_OK(launch_curved_mass(prob->N, f, b, prob->curved, L.E, as_stream(stream)));
    else
      HIP_OK(launch_mass(prob->N, f, b, L.E, L.h, prob->dt, as_stream(stream)));
    return DGS_OK;
  });
}

int dgs_apply_operator(dgs_problem* prob, const double* u, double* Au, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !u || !Au) return fail(DGS_ERR_INVALID, "NULL argument");
    if (u == Au) return fail(DGS_ERR_INVALID, "u and Au must not overlap");
    Level& L = prob->levels[0];
    if (prob->metric_on)
      HIP_OK(launch_curved_apply_metric(prob->N, false, u, Au, nullptr, nullptr, prob->curved,
                                        prob->metric, L.d_nbr, prob->penalty, L.op.neumann, L.E,
                                        as_stream(stream)));
    else if (prob->curved_on)
      HIP_OK(launch_curved_apply(prob->N, false, u, Au, nullptr, nullptr, prob->curved, L.d_nbr,
                                 prob->penalty, L.op.neumann, L.E, as_stream(stream)));
    else
      HIP_OK(launch_apply(prob->N, kApply, u, Au, nullptr, nullptr, nullptr, L.d_nbr, L.op, prob->dt,
                          L.acfg_out, as_stream(stream), L.d_order));
    return DGS_OK;
  });
}

int dgs_set_geometry(dgs_problem* prob, const double* xyz, void* stream) {
  return guarded([&]() -> int {
    if (!prob) return fail(DGS_ERR_INVALID, "NULL argument");
    hipStream_t s = as_stream(stream);
    if (!xyz) {
      prob->curved_on = false;
      prob->metric_on = false;
      return DGS_OK;
    }
    const int N = prob->N;
    if (N > 8) return fail(DGS_ERR_INVALID, "curved elements are limited to p <= 7");
    Level& L = prob->levels[0];
    const long long nd = prob->nd(0);
    CurvedGeometry& G = prob->curved;
    if (!G.inv) {
      G.inv = prob->alloc<double>((size_t)9 * nd);
      G.det = prob->alloc<double>(nd);
      G.grad = prob->alloc<double>((size_t)3 * nd);
      G.D = prob->alloc<double>((size_t)N * N);
      G.w = prob->alloc<double>(N);
      upload(G.D, prob->ht.D, s);
      upload(G.w, prob->ht.w, s);
    }
    if (prob->d_mdiag) {  // formed again from the new geometry when needed
      HIP_OK(hipStreamSynchronize(s));
      prob->release(prob->d_mdiag);
      prob->d_mdiag = nullptr;
    }
    HIP_OK(launch_curved_geometry(N, xyz, L.E, G.D, G.inv, G.det, s));
    // every element map must preserve orientation
    std::vector<double> det(nd);
    HIP_OK(hipMemcpyAsync(det.data(), G.det, sizeof(double) * nd, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (double v : det)
      if (!(v > 0.0) || !std::isfinite(v)) {
        prob->curved_on = false;
        prob->metric_on = false;
        return fail(DGS_ERR_INVALID, "the node coordinates give a Jacobian determinant <= 0");
      }
    prob->curved_on = true;
    if (prob->metric_on)  // the Christoffel contraction depends on the element maps
      HIP_OK(launch_curved_metric_source(N, G, prob->metric, L.E, s));
    return DGS_OK;
  });
}

int dgs_set_metric(dgs_problem* prob, const double* ginv, const double* sqrtg, void* stream) {
  return guarded([&]() -> int {
    if (!prob) return fail(DGS_ERR_INVALID, "NULL argument");
    if (!ginv != !sqrtg) return fail(DGS_ERR_INVALID, "ginv and sqrtg are given together");
    hipStream_t s = as_stream(stream);
    if (!ginv) {
      if (prob->metric_on && prob->d_mdiag) {
        HIP_OK(hipStreamSynchronize(s));
        prob->release(prob->d_mdiag);
        prob->d_mdiag = nullptr;
      }
      prob->metric_on = false;
      return DGS_OK;
    }
    const int N = prob->N;
    if (N > 8) return fail(DGS_ERR_INVALID, "curved elements are limited to p <= 7");
    const Level& L = prob->levels[0];
    const long long nd = prob->nd(0);
    // the metric must be positive definite with a positive root of its
    // determinant at every node: check on the host before any use
    std::vector<double> hg((size_t)6 * nd), hs(nd);
    HIP_OK(hipMemcpyAsync(hg.data(), ginv, sizeof(double) * 6 * nd, hipMemcpyDeviceToHost, s));
    HIP_OK(hipMemcpyAsync(hs.data(), sqrtg, sizeof(double) * nd, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (long long i = 0; i < nd; ++i) {
      const double a = hg[i], b = hg[nd + i], c = hg[2 * nd + i], d = hg[3 * nd + i],
                   e = hg[4 * nd + i], f = hg[5 * nd + i];
      const double m2 = a * d - b * b;
      const double m3 = a * (d * f - e * e) - b * (b * f - e * c) + c * (b * e - d * c);
      if (!(a > 0.0) || !(m2 > 0.0) || !(m3 > 0.0) || !std::isfinite(m3))
        return fail(DGS_ERR_INVALID, "g^ij is not positive definite at every node");
      if (!(hs[i] > 0.0) || !std::isfinite(hs[i]))
        return fail(DGS_ERR_INVALID, "sqrt(g) must be positive and finite at every node");
    }
    if (!prob->curved_on) {  // the box grid's own coordinates as the element maps
      double* xyz = prob->alloc<double>((size_t)3 * nd);
      HIP_OK(launch_coords(N, xyz, L.n, prob->dom.lower, L.h, prob->dt, s));
      const int rc = dgs_set_geometry(prob, xyz, stream);
      HIP_OK(hipStreamSynchronize(s));
      prob->release(xyz);
      if (rc != DGS_OK) return rc;
    }
    if (prob->d_mdiag) {
      HIP_OK(hipStreamSynchronize(s));
      prob->release(prob->d_mdiag);
      prob->d_mdiag = nullptr;
    }
    CurvedMetric& Mt = prob->metric;
    if (!Mt.ginv) {
      Mt.ginv = prob->alloc<double>((size_t)6 * nd);
      Mt.sqrtg = prob->alloc<double>(nd);
      Mt.dlsg = prob->alloc<double>((size_t)3 * nd);
    }
    HIP_OK(hipMemcpyAsync(Mt.ginv, ginv, sizeof(double) * 6 * nd, hipMemcpyDeviceToDevice, s));
    HIP_OK(hipMemcpyAsync(Mt.sqrtg, sqrtg, sizeof(double) * nd, hipMemcpyDeviceToDevice, s));
    HIP_OK(launch_curved_metric_source(N, prob->curved, Mt, L.E, s));
    prob->metric_on = true;
    return DGS_OK;
  });
}

int dgs_schwarz_smooth(dgs_problem* prob, const double* b, double* u, int steps, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !b || !u) return fail(DGS_ERR_INVALID, "NULL argument");
    if (steps < 0) return fail(DGS_ERR_INVALID, "steps must be >= 0");
    schwarz_steps(prob, 0, b, u, steps, false, as_stream(stream));
    return DGS_OK;
  });
}

int dgs_subdomain_solves(dgs_problem* prob, int level, int reps, double* flops, void* stream) {
  return guarded([&]() -> int {
    if (!prob) return fail(DGS_ERR_INVALID, "NULL argument");
    if (level < 0 || level >= (int)prob->levels.size())
      return fail(DGS_ERR_INVALID, "level out of range");
    if (reps < 0) return fail(DGS_ERR_INVALID, "reps must be >= 0");
    Level& L = prob->levels[level];
    if (flops) {
      double f = 0.0;
      for (const ClassInfo& c : L.cls) f += 2.0 * (double)c.n * (double)c.n * (double)c.count;
      *flops = f;
    }
    const hipStream_t s = as_stream(stream);
    for (int r = 0; r < reps; ++r)
      HIP_OK(gemm_level(L, L.d_rs, L.rs_total, 0, s));
    return DGS_OK;
  });
}

int dgs_set_apply_shape(dgs_problem* prob, int level, int shape) {
  return guarded([&]() -> int {
    if (!prob) return fail(DGS_ERR_INVALID, "NULL argument");
    if (level < 0 || level >= (int)prob->levels.size())
      return fail(DGS_ERR_INVALID, "level out of range");
    Level& L = prob->levels[level];
    if (shape < -1 || shape > 2) return fail(DGS_ERR_INVALID, "unknown apply shape");
    if (shape == -1 && !L.d_bricks) return fail(DGS_ERR_INVALID, "bricks need p = 7");
    L.acfg = L.acfg_out = shape_config(L, shape);
    recapture_vgraphs(prob);
    return DGS_OK;
  });
}

int dgs_set_gemm_variant(dgs_problem* prob, int level, int variant) {
  return guarded([&]() -> int {
    if (!prob) return fail(DGS_ERR_INVALID, "NULL argument");
    if (level < 0 || level >= (int)prob->levels.size())
      return fail(DGS_ERR_INVALID, "level out of range");
    if (variant < 0 || variant >= kGemmVariants) return fail(DGS_ERR_INVALID, "unknown variant");
    Level& L = prob->levels[level];
    L.gemm_variant = variant;
    L.kparts = L.kparts_of[variant];
    recapture_vgraphs(prob);
    return DGS_OK;
  });
}

int dgs_get_gemm_variant(const dgs_problem* prob, int level, int* variant) {
  if (!prob || !variant) return fail(DGS_ERR_INVALID, "NULL argument");
  if (level < 0 || level >= (int)prob->levels.size())
    return fail(DGS_ERR_INVALID, "level out of range");
  *variant = prob->levels[level].gemm_variant;
  return DGS_OK;
}

int dgs_get_apply_shape(const dgs_problem* prob, int level, int* shape) {
  if (!prob || !shape) return fail(DGS_ERR_INVALID, "NULL argument");
  if (level < 0 || level >= (int)prob->levels.size())
    return fail(DGS_ERR_INVALID, "level out of range");
  *shape = prob->levels[level].acfg_out.epb;
  return DGS_OK;
}

int dgs_precondition(dgs_problem* prob, const double* r, double* z, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !r || !z) return fail(DGS_ERR_INVALID, "NULL argument");
    if (r == z) return fail(DGS_ERR_INVALID, "r and z must not overlap");
    vcycle(prob, r, z, as_stream(stream));
    return DGS_OK;
  });
}

int dgs_solve(dgs_problem* prob, const double* b, double* u, dgs_stats* stats, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !b || !u) return fail(DGS_ERR_INVALID, "NULL argument");
    const double t0 = now_s();
    FgmresResult R = fgmres(prob, b, u, prob->opt.rtol, prob->opt.max_iter, as_stream(stream));
    fill_stats(stats, R, t0, prob->t_setup);
    if (stats) {
      stats->newton_steps = 0;
      stats->backtracks = 0;
    }
    if (!std::isfinite(R.rel_residual)) return fail(DGS_ERR_NONFINITE, "non-finite residual");
    return R.converged ? DGS_OK : DGS_NOT_CONVERGED;
  });
}

int dgs_cg_solve(dgs_problem* prob, const double* b, double* u, dgs_stats* stats, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !b || !u) return fail(DGS_ERR_INVALID, "NULL argument");
    if (b == u) return fail(DGS_ERR_INVALID, "b and u must not overlap");
    const double t0 = now_s();
    FgmresResult R = cg(prob, b, u, prob->opt.rtol, prob->opt.max_iter, as_stream(stream),
                        problem_cg_work(prob));
    fill_stats(stats, R, t0, prob->t_setup);
    if (stats) {
      stats->newton_steps = 0;
      stats->backtracks = 0;
    }
    if (!std::isfinite(R.rel_residual)) return fail(DGS_ERR_NONFINITE, "non-finite residual");
    return R.converged ? DGS_OK : DGS_NOT_CONVERGED;
  });
}

int dgs_cg_solve_noalloc(dgs_problem* prob, const double* b, double* u, dgs_stats* stats,
                         void* stream) {
  return guarded([&]() -> int {
    if (!prob || !b || !u) return fail(DGS_ERR_INVALID, "NULL argument");
    if (b == u) return fail(DGS_ERR_INVALID, "b and u must not overlap");
    const long long n = prob->nd(0);
    if (n > kNoAllocMaxDofs)
      return fail(DGS_ERR_INVALID, "dgs_cg_solve_noalloc: the problem has " + std::to_string(n) +
                                       " points, more than its static workspace holds (" +
                                       std::to_string(kNoAllocMaxDofs) + ")");
    int device = 0;
    double* base = scratch_for_current_device(&device);
    const long long ld = (n + 31) / 32 * 32;  // each vector on a 256-byte boundary
    CgWork w;
    w.R = base;  // two rows
    w.z = base + 2 * ld;
    w.p0 = base + 3 * ld;
    w.p1 = base + 4 * ld;
    w.q = base + 5 * ld;
    w.t = base + 6 * ld;
    w.partial = base + 7 * kNoAllocMaxDofs;
    w.h = w.partial + kNoAllocPartials;
    w.hp = g_scratch_host[device];
    const double t0 = now_s();
    FgmresResult R = cg(prob, b, u, prob->opt.rtol, prob->opt.max_iter, as_stream(stream), w);
    fill_stats(stats, R, t0, prob->t_setup);
    if (stats) {
      stats->newton_steps = 0;
      stats->backtracks = 0;
    }
    if (!std::isfinite(R.rel_residual)) return fail(DGS_ERR_NONFINITE, "non-finite residual");
    return R.converged ? DGS_OK : DGS_NOT_CONVERGED;
  });
}

int dgs_set_diagonal(dgs_problem* prob, const double* d, void* stream) {
  return guarded([&]() -> int {
    if (!prob) return fail(DGS_ERR_INVALID, "NULL argument");
    set_diagonal(prob, d, as_stream(stream));
    return DGS_OK;
  });
}

int dgs_newton_solve(dgs_problem* prob, const double* alpha, const double* beta, const double* b,
                     double* u, double newton_rtol, double linear_rtol, int max_newton,
                     dgs_stats* stats, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !alpha || !beta || !b || !u) return fail(DGS_ERR_INVALID, "NULL argument");
    if (!(newton_rtol > 0.0) || !(linear_rtol > 0.0) || max_newton < 1)
      return fail(DGS_ERR_INVALID, "invalid Newton tolerances");
    if (prob->curved_on) return fail(DGS_ERR_INVALID, "the puncture problem is set on the box grid");
    hipStream_t s = as_stream(stream);
    const double t0 = now_s();
    NewtonRun nr;
    nr.init(prob, alpha, beta, b, u, newton_rtol, linear_rtol, max_newton, s);
    while (!nr.done()) nr.step();
    prob->diag_active = false;
    HIP_OK(hipStreamSynchronize(s));
    const bool converged = nr.converged;
    if (stats) {
      stats->iterations = nr.its;
      stats->newton_steps = nr.steps;
      stats->backtracks = nr.backtracks;
      stats->rel_residual = nr.rel_residual();
      stats->t_solve_s = now_s() - t0;
      stats->t_setup_s = prob->t_setup;
      stats->history_len = 0;
      if (stats->history && stats->history_capacity > 0) {
        const int m = std::min<int>(stats->history_capacity, (int)nr.hist.size());
        for (int i = 0; i < m; ++i) stats->history[i] = nr.hist[i];
        stats->history_len = m;
      }
    }
    return converged ? DGS_OK : DGS_NOT_CONVERGED;
  });
}

int dgs_newton_solve_powers(dgs_problem* prob, int nterms, const int* powers, const double* coef,
                            const double* dirichlet, const double* b, double* u, double newton_rtol,
                            double linear_rtol, int max_newton, dgs_stats* stats, void* stream) {
  return guarded([&]() -> int {
    if (!prob || !powers || !coef || !u) return fail(DGS_ERR_INVALID, "NULL argument");
    if (nterms < 1 || nterms > kMaxPowerTerms)
      return fail(DGS_ERR_INVALID, "the source takes 1 to 8 terms");
    for (int t = 0; t < nterms; ++t)
      if (powers[t] < -kMaxPower || powers[t] > kMaxPower)
        return fail(DGS_ERR_INVALID, "powers must lie in [-12, 12]");
    if (!(newton_rtol > 0.0) || !(linear_rtol > 0.0) || max_newton < 1)
      return fail(DGS_ERR_INVALID, "invalid Newton tolerances");
    if (!prob->curved_on)
      return fail(DGS_ERR_INVALID, "set node coordinates (dgs_set_geometry) or a metric first");
    hipStream_t s = as_stream(stream);
    const double t0 = now_s();
    PowerSource src;
    src.nterms = nterms;
    for (int t = 0; t < nterms; ++t) src.power[t] = powers[t];
    src.coef = coef;
    NewtonRun nr;
    nr.init_powers(prob, src, dirichlet, b, u, newton_rtol, linear_rtol, max_newton, s);
    while (!nr.done()) nr.step();
    prob->diag_active = false;
    HIP_OK(hipStreamSynchronize(s));
    if (stats) {
      stats->iterations = nr.its;
      stats->newton_steps = nr.steps;
      stats->backtracks = nr.backtracks;
      stats->rel_residual = nr.rel_residual();
      stats->t_solve_s = now_s() - t0;
      stats->t_setup_s = prob->t_setup;
      stats->history_len = 0;
      if (stats->history && stats->history_capacity > 0) {
        const int m = std::min<int>(stats->history_capacity, (int)nr.hist.size());
        for (int i = 0; i < m; ++i) stats->history[i] = nr.hist[i];
        stats->history_len = m;
      }
    }
    return nr.converged ? DGS_OK : DGS_NOT_CONVERGED;
  });
}

int dgs_lgl_nodes(int p, double* xi) {
  return guarded([&]() -> int {
    if (!xi || p < 1 || p > kMaxN - 1) return fail(DGS_ERR_INVALID, "need p in [1, 12] and xi");
    HostTables t = make_tables(p + 1);
    for (int i = 0; i <= p; ++i) xi[i] = t.xi[i];
    return DGS_OK;
  });
}

int dgs_grid_coordinates(const dgs_domain* domain, const int elements[3], int p, double* xyz,
                         long long n) {
  return guarded([&]() -> int {
    if (!domain || !elements || !xyz) return fail(DGS_ERR_INVALID, "NULL argument");
    if (p < 1 || p > kMaxN - 1) return fail(DGS_ERR_INVALID, "p out of range");
    for (int d = 0; d < 3; ++d)
      if (elements[d] < 1 || !(domain->upper[d] > domain->lower[d]))
        return fail(DGS_ERR_INVALID, "bad mesh");
    const int N = p + 1;
    const long long E = (long long)elements[0] * elements[1] * elements[2];
    const long long nd = E * N * N * N;
    if (n != nd) return fail(DGS_ERR_INVALID, "n must be the number of points E (p+1)^3");
    const HostTables t = make_tables(N);
    double h[3];
    for (int d = 0; d < 3; ++d) h[d] = (domain->upper[d] - domain->lower[d]) / elements[d];
    for (long long e = 0; e < E; ++e) {
      const long long c[3] = {e % elements[0], (e / elements[0]) % elements[1],
                              e / ((long long)elements[0] * elements[1])};
      for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
          for (int i = 0; i < N; ++i) {
            const long long idx = ((e * N + k) * N + j) * N + i;
            const int node[3] = {i, j, k};
            for (int d = 0; d < 3; ++d)
              xyz[d * nd + idx] = domain->lower[d] + h[d] * ((double)c[d] + 0.5 * (t.xi[node[d]] + 1.0));
          }
    }
    return DGS_OK;
  });
}

int dgs_server_create(const dgs_server_options* opt, dgs_server** out) {
  return guarded([&]() -> int {
    if (!opt || !out) return fail(DGS_ERR_INVALID, "NULL argument");
    if (opt->max_active < 1 || !(opt->hbm_budget_bytes > 0) || !(opt->penalty > 0))
      return fail(DGS_ERR_INVALID, "invalid server options");
    if (opt->host_threads < 0) return fail(DGS_ERR_INVALID, "host_threads must be >= 0");
    if (!opt->alloc_fn != !opt->free_fn)
      return fail(DGS_ERR_INVALID, "alloc_fn and free_fn go together");
    std::unique_ptr<dgs_server> S(new dgs_server());
    S->opt = *opt;
    S->t0 = now_s();
    // free blocks kept for reuse: at most half the budget on top of it
    S->blocks.cap = (size_t)(opt->hbm_budget_bytes / 2);
    HIP_OK(hipGetDevice(&S->device));
    const int threads = std::min(opt->host_threads > 0 ? opt->host_threads : 4, opt->max_active);
    if (threads > 1) S->pool.reset(new WorkerPool(threads, S->device));
    *out = S.release();
    return DGS_OK;
  });
}

int dgs_server_destroy(dgs_server* S) {
  return guarded([&]() -> int {
    if (S) {
      (void)hipDeviceSynchronize();
      delete S;
    }
    return DGS_OK;
  });
}

int dgs_server_submit(dgs_server* S, const dgs_domain* domain, const int elements[3], int p,
                      const double* f, long long n, long long* id) {
  return guarded([&]() -> int {
    if (!S || !domain || !elements || !f || !id) return fail(DGS_ERR_INVALID, "NULL argument");
    if (p < 1 || p > kMaxN - 1) return fail(DGS_ERR_INVALID, "p must be in [1, 12]");
    for (int d = 0; d < 3; ++d)
      if (elements[d] < 1 || !(domain->upper[d] > domain->lower[d]))
        return fail(DGS_ERR_INVALID, "bad mesh");
    const long long nd = (long long)elements[0] * elements[1] * elements[2] * (p + 1) * (p + 1) * (p + 1);
    if (n != nd) return fail(DGS_ERR_INVALID, "f has the wrong length");
    std::unique_ptr<ServerRequest> r(new ServerRequest());
    r->id = S->next_id++;
    r->dom = *domain;
    for (int d = 0; d < 3; ++d) r->elements[d] = elements[d];
    r->p = p;
    r->f.assign(f, f + n);
    r->footprint = request_footprint(S, elements, p);
    // the batch engine: Poisson requests of degree <= 8 with the V-cycle
    const dgs_options& so = S->opt.solver;
    r->batched = S->opt.batched && p <= 8 && so.cycle == 1 && !so.additive &&
                 so.pre_smooth >= 1 && so.post_smooth >= 1;
    r->t_submit = now_s() - S->t0;
    *id = r->id;
    S->queue.push_back(std::move(r));
    return DGS_OK;
  });
}

int dgs_server_submit_puncture(dgs_server* S, const dgs_domain* domain, const int elements[3],
                               int p, const double* alpha, const double* beta, const double* b,
                               long long n, double newton_rtol, double linear_rtol,
                               int max_newton, long long* id) {
  return guarded([&]() -> int {
    if (!S || !domain || !elements || !alpha || !beta || !id)
      return fail(DGS_ERR_INVALID, "NULL argument");
    if (p < 1 || p > kMaxN - 1) return fail(DGS_ERR_INVALID, "p must be in [1, 12]");
    for (int d = 0; d < 3; ++d)
      if (elements[d] < 1 || !(domain->upper[d] > domain->lower[d]))
        return fail(DGS_ERR_INVALID, "bad mesh");
    if (!(newton_rtol > 0.0) || !(linear_rtol > 0.0) || max_newton < 1)
      return fail(DGS_ERR_INVALID, "invalid Newton tolerances");
    const long long nd = (long long)elements[0] * elements[1] * elements[2] * (p + 1) * (p + 1) * (p + 1);
    if (n != nd) return fail(DGS_ERR_INVALID, "fields have the wrong length");
    std::unique_ptr<ServerRequest> r(new ServerRequest());
    r->id = S->next_id++;
    r->kind = 1;
    r->dom = *domain;
    for (int d = 0; d < 3; ++d) r->elements[d] = elements[d];
    r->p = p;
    r->alpha.assign(alpha, alpha + n);
    r->beta.assign(beta, beta + n);
    r->has_b = b != nullptr;
    if (b) r->f.assign(b, b + n);
    r->newton_rtol = newton_rtol;
    r->linear_rtol = linear_rtol;
    r->max_newton = max_newton;
    // the Poisson footprint plus alpha, beta and the Newton work vectors
    r->footprint = request_footprint(S, elements, p) + (size_t)(7.0 * 8.0 * (double)n);
    r->t_submit = now_s() - S->t0;
    *id = r->id;
    S->queue.push_back(std::move(r));
    return DGS_OK;
  });
}

int dgs_server_step(dgs_server* S, int* n_active, int* n_queued) {
  return guarded([&]() -> int {
    if (!S) return fail(DGS_ERR_INVALID, "NULL argument");
    const double t_begin = now_s();
    std::vector<std::unique_ptr<ServerRequest>> admitted = server_select(S);
    S->t_workers += now_s() - t_begin;
    // the batch engine's step goes to the device first, so that the set-up
    // of the newly admitted requests and the per-request work below overlap
    // it; the requests set up here join the engine after its step
    double t = now_s();
    if (S->engine && !S->engine->empty()) {
      S->batch_peak = std::max<long long>(S->batch_peak, S->engine->size());
      S->engine->issue();
    }
    S->t_issue += now_s() - t;
    t = now_s();
    // each worker first sets up every W-th newly admitted request (host work
    // that overlaps the stages already on the device), then takes every W-th
    // active request: a request whose stage has finished is completed on the
    // host and its next stage issued at once; one whose stage is still on the
    // device is left to run, so a small request does not wait for a large
    // one.  If none of the worker's requests has finished, it waits for the
    // first one that is in flight, so every call makes progress.  Every
    // unfinished request leaves this call with a stage on the device
    // (requests never share state).
    auto work = [S, &admitted](size_t first, size_t stride) {
      for (size_t i = first; i < admitted.size(); i += stride) server_setup(S, *admitted[i]);
      auto advance = [](ServerRequest& r) {
        r.in_flight = false;
        r.run.complete();
        if (!r.run.done()) {
          r.run.issue();
          r.in_flight = true;
        }
      };
      bool progressed = false;
      ServerRequest* waiting = nullptr;
      for (size_t i = first; i < S->active.size(); i += stride) {
        ServerRequest& r = *S->active[i];
        if (r.batched) continue;  // advanced by the batch engine below
        if (r.kind == 1) {  // a Newton step runs to its end on the worker
          if (!r.nrun.done()) r.nrun.step();
          progressed = true;
          continue;
        }
        if (!r.in_flight) {
          if (!r.run.done()) {
            r.run.issue();
            r.in_flight = true;
          }
          progressed = true;
          continue;
        }
        const hipError_t q = hipStreamQuery(r.stream);
        if (q == hipErrorNotReady) {
          if (!waiting) waiting = &r;
          continue;
        }
        HIP_OK(q);
        advance(r);
        progressed = true;
      }
      if (!progressed && waiting) {
        HIP_OK(hipStreamSynchronize(waiting->stream));
        advance(*waiting);
      }
      for (size_t i = first; i < admitted.size(); i += stride) {  // their first stages
        ServerRequest& r = *admitted[i];
        if (r.kind == 0 && !r.batched && !r.run.done()) {
          r.run.issue();
          r.in_flight = true;
        }
      }
    };
    if (S->pool && S->active.size() + admitted.size() > 1) {
      const size_t W = (size_t)S->pool->size();
      S->pool->run([&work, W](int w) { work((size_t)w, W); });
    } else {
      work(0, 1);
    }
    ++S->steps;
    S->t_workers += now_s() - t;
    // the batch engine: every member advanced by one FGMRES iteration in
    // shared launches; then the newly set-up requests join for the next step
    if (S->engine && S->engine->issued()) {
      S->engine->finish(&S->t_wait, &S->t_engine_host);
      ++S->batch_steps;
      S->batch_launches += S->engine->launches_last_step();
    }
    for (auto& rq : admitted) {
      if (!rq->batched) continue;
      if (!S->engine)
        S->engine.reset(new BatchEngine(S->opt.max_active, S->opt.solver.max_iter,
                                        S->opt.solver.restart));
      S->engine->add(rq.get());
    }
    for (auto& rq : admitted) S->active.push_back(std::move(rq));
    const double t_ret = now_s();
    std::vector<std::unique_ptr<ServerRequest>> still;
    for (auto& r : S->active) {
      if (r->done())
        server_retire(S, std::move(r));
      else
        still.push_back(std::move(r));
    }
    S->active = std::move(still);
    if (S->active.empty() && S->queue.empty()) S->free_retired();  // idle: return the memory
    S->t_retire += now_s() - t_ret;
    if (n_active) *n_active = (int)S->active.size();
    if (n_queued) *n_queued = (int)S->queue.size();
    return DGS_OK;
  });
}

int dgs_server_counters(const dgs_server* S, long long counters[4]) {
  if (!S || !counters) return fail(DGS_ERR_INVALID, "NULL argument");
  counters[0] = S->steps;
  counters[1] = S->batch_steps;
  counters[2] = S->batch_launches;
  counters[3] = S->batch_peak;
  return DGS_OK;
}

int dgs_server_timings(const dgs_server* S, double seconds[5]) {
  if (!S || !seconds) return fail(DGS_ERR_INVALID, "NULL argument");
  seconds[0] = S->t_workers;
  seconds[1] = S->t_issue;
  seconds[2] = S->t_wait;
  seconds[3] = S->t_engine_host;
  seconds[4] = S->t_retire;
  return DGS_OK;
}

int dgs_server_finished(dgs_server* S, long long* ids, int capacity, int* count) {
  return guarded([&]() -> int {
    if (!S || !count) return fail(DGS_ERR_INVALID, "NULL argument");
    int c = 0;
    for (auto& kv : S->finished) {
      if (ids && c < capacity) ids[c] = kv.first;
      ++c;
    }
    *count = c;
    return DGS_OK;
  });
}

int dgs_server_fetch(dgs_server* S, long long id, double* u, long long n, dgs_stats* stats,
                     double times[4]) {
  return guarded([&]() -> int {
    if (!S) return fail(DGS_ERR_INVALID, "NULL argument");
    auto it = S->finished.find(id);
    if (it == S->finished.end()) return fail(DGS_ERR_INVALID, "request not finished or unknown");
    ServerRequest& r = *it->second;
    if (r.status < 0) {
      const int st = r.status;
      S->finished.erase(it);
      return fail(st, st == DGS_ERR_OOM ? "request rejected: its footprint exceeds the device budget"
                                        : "request failed: non-finite values in its solve");
    }
    if (u) {
      if (n != (long long)r.u.size()) return fail(DGS_ERR_INVALID, "u has the wrong length");
      std::copy(r.u.begin(), r.u.end(), u);
    }
    if (stats) {
      stats->iterations = r.result.iterations;
      stats->newton_steps = r.newton_steps;
      stats->backtracks = r.backtracks;
      stats->rel_residual = r.result.rel_residual;
      stats->t_setup_s = r.t_setup;
      stats->t_solve_s = r.t_done - r.t_admit;
      stats->history_len = 0;
      if (stats->history && stats->history_capacity > 0) {
        const int m = std::min<int>(stats->history_capacity, (int)r.result.history.size());
        for (int i = 0; i < m; ++i) stats->history[i] = r.result.history[i];
        stats->history_len = m;
      }
    }
    if (times) {
      times[0] = r.t_submit;
      times[1] = r.t_admit;
      times[2] = r.t_done;
      times[3] = (double)r.footprint;
    }
    const int status = r.status;
    S->finished.erase(it);
    return status;
  });
}

}  // extern "C"

// ===========================================================================
// Systems of several variables (Sec. III.E.1): each variable has its own
// boundary types; the Schwarz subdomain problem of the whole system is
// solved by k iterations of right-preconditioned GMRES whose preconditioner
// is the Laplacian approximation (eq. lapl_approx), one Poisson inverse per
// variable with that variable's boundary types (or, for comparison, the
// Dirichlet one for every variable).
//
// A system is one scalar problem per variable, all built with the Neumann
// faces of every variable in their class key, so that they share classes,
// element frames, row layouts, tiles and tables; each holds the inverses and
// subdomain operators of its own boundary types (the process-wide inverse
// cache stores a class's inverse once however many variables use it, so a
// subdomain with only internal faces has one inverse for all variables).
// ===========================================================================
namespace {

struct SysLevel {
  long long nd = 0;       // points per variable
  long long st = 0;       // subdomain rows per variable (shared by all variables)
  double* D = nullptr;    // couplings D_ab, nv * nv fields of nd points
  double* b = nullptr;    // coarse levels: restricted residual, nv * nd
  double* u = nullptr;    // coarse levels: correction, nv * nd
  double* r = nullptr;    // residual, nv * nd
  void* rs = nullptr;     // gathered rows, nv * st (level precision)
  void* du = nullptr;     // subdomain corrections, nv * st
  void* parts = nullptr;  // split-K partial products of one GEMM
  void *gV = nullptr, *gZ = nullptr, *gW = nullptr;  // subdomain GMRES bases
  double *H = nullptr, *beta = nullptr;
  // one grouped GEMM over the classes of all variables: class a * ncls + c
  // is variable a's class c (its Laplacian-approximation inverse in cls_inv,
  // its A_S in cls_op); the rows of slot j (ptr_inv[j]: V_j, ptr_op[j]: Z_j)
  // and the split-K partials, [part][variable][row]
  int ncls = 0;
  ClassInfo* cls_inv = nullptr;
  ClassInfo* cls_op = nullptr;
  std::vector<GemmPtr*> ptr_inv, ptr_op;
  GemmPtr* ptr_rs = nullptr;  // the gathered rows (k = 0)
  GemmTile* tiles = nullptr;
  int ntiles = 0, kparts = 1;
  bool small = false;
};

}  // namespace

struct dgs_system {
  int nv = 0;
  int matched = 1;
  bool coupled = false;
  std::vector<dgs_problem*> var;  // one scalar problem per variable
  dgs_problem* dir = nullptr;     // all-Dirichlet problem of the naive approximation
  std::vector<SysLevel> lv;
  int kry_m = 0;
  double *V = nullptr, *Z = nullptr, *partial = nullptr, *h = nullptr, *y = nullptr, *tmp = nullptr;
  double* h_pinned = nullptr;
  double* d_newton = nullptr;  // Newton work vectors (5 system vectors)
  double t_setup = 0;

  dgs_problem* base() const { return var[0]; }
  // the system's buffers are allocations of the first variable's problem
  template <typename T>
  T* alloc(size_t n) { return var[0]->alloc<T>(n); }
  ~dgs_system() {
    (void)hipDeviceSynchronize();
    std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
    if (h_pinned) (void)hipHostFree(h_pinned);
    for (dgs_problem* p : var) delete p;
    delete dir;
  }
};

namespace {

// One grouped GEMM over all variables on level l: every variable's inverse
// (the Laplacian approximation, cls_inv) or A_S (cls_op) times its rows as
// listed in ptrs, split-K partials into the level's parts buffer.
void sys_gemm(dgs_system* S, int l, const ClassInfo* cls, const GemmPtr* ptrs, hipStream_t s) {
  SysLevel& SL = S->lv[l];
  const Level& L0 = S->base()->levels[l];
  HIP_OK(launch_subdomain_gemm_batched(L0.f32, cls, ptrs, SL.tiles, SL.ntiles, SL.small, s));
}

// r = b - A_sys u on level l (vectors of nv * nd)
void sys_residual(dgs_system* S, int l, const double* u, const double* b, double* r, hipStream_t s) {
  const dgs_problem* P = S->base();
  const long long nd = S->lv[l].nd;
  for (int a = 0; a < S->nv; ++a) {
    const dgs_problem* Pa = S->var[a];
    const Level& L = Pa->levels[l];
    HIP_OK(launch_apply(P->N, kResidual, u + a * nd, r + a * nd, b + a * nd, nullptr, nullptr,
                        L.d_nbr, L.op, Pa->dt, L.acfg_out, s, L.d_order));
  }
  if (S->coupled) HIP_OK(launch_sys_couple(r, u, S->lv[l].D, S->nv, nd, -1.0, s));
}

// y = A_sys u on the finest level: each variable's own operator (the curved
// one when its problem has curved elements), then the couplings
void sys_apply(dgs_system* S, const double* u, double* y, hipStream_t s) {
  const long long nd = S->lv[0].nd;
  for (int a = 0; a < S->nv; ++a) apply_fine(S->var[a], u + a * nd, y + a * nd, s);
  if (S->coupled) HIP_OK(launch_sys_couple(y, u, S->lv[0].D, S->nv, nd, 1.0, s));
}

// r = b - A_sys u on the finest level with the operators of sys_apply (the
// V-cycle's residuals stay those of the box grids, sys_residual)
void sys_residual_fine(dgs_system* S, const double* u, const double* b, double* r, hipStream_t s) {
  const long long nd = S->lv[0].nd;
  for (int a = 0; a < S->nv; ++a) residual_fine(S->var[a], u + a * nd, b + a * nd, r + a * nd, s);
  if (S->coupled) HIP_OK(launch_sys_couple(r, u, S->lv[0].D, S->nv, nd, -1.0, s));
}

// Subdomain GMRES(k) of the system on level l: rows in SL.rs, corrections
// into SL.du (one block per variable).
void sys_subdomain_gmres(dgs_system* S, int l, hipStream_t s) {
  const dgs_problem* P = S->base();
  SysLevel& SL = S->lv[l];
  const Level& L0 = P->levels[l];
  const int k = P->opt.subdomain_iters, nv = S->nv;
  const size_t es = L0.f32 ? sizeof(float) : sizeof(double);
  auto at = [&](void* base, long long blocks) { return (void*)((char*)base + es * (size_t)(SL.st * blocks)); };
  HIP_OK(launch_sys_start(L0.f32, nv, SL.rs, SL.gV, SL.beta, SL.st, L0.d_elem_class, L0.d_elem_row,
                          L0.d_cls, (int)L0.E, s));
  const long long all = (long long)nv * SL.st;
  for (int j = 0; j < k; ++j) {
    void* Vj = at(SL.gV, (long long)j * nv);
    void* Zj = at(SL.gZ, (long long)j * nv);
    // z_a = M_a v_a (Laplacian approximation), then w_a = A_S^(a) z_a, each
    // one launch over all variables and one reduction of its partials
    sys_gemm(S, l, SL.cls_inv, SL.ptr_inv[j], s);
    HIP_OK(launch_reduce_parts(L0.f32, Zj, SL.parts, SL.kparts, all, all, s));
    sys_gemm(S, l, SL.cls_op, SL.ptr_op[j], s);
    HIP_OK(launch_reduce_parts(L0.f32, SL.gW, SL.parts, SL.kparts, all, all, s));
    HIP_OK(launch_sys_arnoldi(P->N, L0.f32, j, k, nv, SL.gW, SL.gV, Zj, SL.st, SL.D, SL.nd, SL.H,
                              L0.d_elem_class, L0.d_elem_row, L0.d_nbr, L0.d_cls, L0.d_seg_loc,
                              (int)L0.E, L0.max_n, s));
  }
  HIP_OK(launch_sys_finish(L0.f32, k, nv, SL.gZ, SL.st, SL.H, SL.beta, SL.du, L0.d_elem_class,
                           L0.d_elem_row, L0.d_cls, (int)L0.E, s));
}

// `steps` additive Schwarz steps on A_sys u = b, level l (u_zero: u starts
// at zero and the first step writes it)
void sys_schwarz_steps(dgs_system* S, int l, const double* b, double* u, int steps, bool u_zero,
                       hipStream_t s) {
  const dgs_problem* P = S->base();
  SysLevel& SL = S->lv[l];
  const Level& L0 = P->levels[l];
  const int N = P->N, nv = S->nv;
  const size_t es = L0.f32 ? sizeof(float) : sizeof(double);
  auto at = [&](void* base, long long blocks) { return (void*)((char*)base + es * (size_t)(SL.st * blocks)); };
  for (int it = 0; it < steps; ++it) {
    const bool first = it == 0 && u_zero;
    const double* src = b;
    if (!first) {
      sys_residual(S, l, u, b, SL.r, s);
      src = SL.r;
    }
    for (int a = 0; a < nv; ++a)
      HIP_OK(launch_gather(N, L0.f32, src + a * SL.nd, at(SL.rs, a), L0.d_elem_class,
                           L0.d_elem_row, L0.d_nbr, L0.d_cls, L0.d_seg_loc, (int)L0.E, s));
    if (P->opt.subdomain_iters > 0) {
      sys_subdomain_gmres(S, l, s);
      for (int a = 0; a < nv; ++a)
        HIP_OK(launch_scatter(N, L0.f32, u + a * SL.nd, at(SL.du, a), 1, SL.st, L0.d_weights,
                              L0.d_pull, nov_of(P), L0.E, s, first));
    } else {
      // the Laplacian approximation alone: du_a = M_a r_a, one launch for all
      // variables; the scatter of each variable sums its partials
      sys_gemm(S, l, SL.cls_inv, SL.ptr_rs, s);
      for (int a = 0; a < nv; ++a)
        HIP_OK(launch_scatter(N, L0.f32, u + a * SL.nd, at(SL.parts, a), SL.kparts,
                              (long long)nv * SL.st, L0.d_weights, L0.d_pull, nov_of(P), L0.E, s,
                              first));
    }
  }
}

// One V-cycle visit of level l (Sec. III.C.3) on the system
void sys_visit(dgs_system* S, int l, const double* b, double* u, bool u_zero, hipStream_t s) {
  const dgs_problem* P = S->base();
  const int nl = (int)S->lv.size(), nv = S->nv;
  const int pre = l < nl - 1 ? P->opt.pre_smooth : P->opt.pre_smooth + P->opt.post_smooth;
  SysLevel& SL = S->lv[l];
  if (u_zero && pre == 0) HIP_OK(launch_fill(u, 0.0, nv * SL.nd, s));
  sys_schwarz_steps(S, l, b, u, pre, u_zero, s);
  if (l == nl - 1) return;
  sys_residual(S, l, u, b, SL.r, s);
  SysLevel& C = S->lv[l + 1];
  const Level& L = P->levels[l];
  const Level& Lc = P->levels[l + 1];
  for (int a = 0; a < nv; ++a)
    HIP_OK(launch_restrict(P->N, SL.r + a * SL.nd, C.b + a * C.nd, L.n, Lc.n, L.split, P->mt, s));
  sys_visit(S, l + 1, C.b, C.u, true, s);
  for (int a = 0; a < nv; ++a)
    HIP_OK(launch_prolongate_add(P->N, C.u + a * C.nd, u + a * SL.nd, L.n, Lc.n, L.split, P->mt, s));
  sys_schwarz_steps(S, l, b, u, P->opt.post_smooth, false, s);
}

// Couplings D (nv * nv fields of the finest level) copied into the system and
// restricted to the coarse levels, D_{l+1} = R D_l field by field
void sys_set_coupling(dgs_system* sys, const double* D, hipStream_t s) {
  const dgs_problem* P = sys->base();
  const int nv = sys->nv;
  SysLevel& F = sys->lv[0];
  if (D != F.D)
    HIP_OK(hipMemcpyAsync(F.D, D, sizeof(double) * nv * nv * F.nd, hipMemcpyDeviceToDevice, s));
  for (size_t l = 0; l + 1 < sys->lv.size(); ++l) {
    const Level& L = P->levels[l];
    const Level& Lc = P->levels[l + 1];
    for (int ab = 0; ab < nv * nv; ++ab)
      HIP_OK(launch_restrict(P->N, sys->lv[l].D + ab * sys->lv[l].nd,
                             sys->lv[l + 1].D + ab * sys->lv[l + 1].nd, L.n, Lc.n, L.split, P->mt, s));
  }
  sys->coupled = true;
}

void sys_ensure_krylov(dgs_system* S, int m) {
  if (S->kry_m >= m) return;
  if (S->kry_m > 0) HIP_OK(hipDeviceSynchronize());
  dgs_problem* P = S->base();
  for (double* p : {S->V, S->Z, S->partial, S->h, S->y, S->tmp})
    if (p) P->release(p);
  const long long n = S->nv * S->lv[0].nd;
  S->V = S->alloc<double>((size_t)(m + 1) * n);
  S->Z = S->alloc<double>((size_t)m * n);
  S->partial = S->alloc<double>((size_t)multidot_blocks(n) * (m + 2));
  S->h = S->alloc<double>(3 * (m + 2));
  S->y = S->alloc<double>(m + 1);
  S->tmp = S->alloc<double>(n);
  std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
  if (S->h_pinned) (void)hipHostFree(S->h_pinned);
  S->h_pinned = nullptr;
  HIP_OK(hipHostMalloc((void**)&S->h_pinned, sizeof(double) * 4 * (m + 2), hipHostMallocDefault));
  S->kry_m = m;
}

// FGMRES on the system with one V-cycle per iteration (restarts of the
// options' length).
FgmresResult sys_fgmres(dgs_system* S, const double* b, double* x, hipStream_t s,
                        double rtol = -1.0) {
  const dgs_problem* P = S->base();
  const int max_total = P->opt.max_iter;
  const int m = P->opt.restart > 0 ? std::min(P->opt.restart, max_total) : max_total;
  sys_ensure_krylov(S, m);
  KrylovSpace K;
  K.m = m;
  K.n = S->nv * S->lv[0].nd;
  K.V = S->V;
  K.Z = S->Z;
  K.partial = S->partial;
  K.h = S->h;
  K.y = S->y;
  K.tmp = S->tmp;
  K.pinned = S->h_pinned;
  return fgmres_run(
      K, rtol > 0.0 ? rtol : P->opt.rtol, max_total,
      [&](const double* xx, const double* bb, double* out) { sys_residual_fine(S, xx, bb, out, s); },
      [&](const double* z, double* w) { sys_apply(S, z, w, s); },
      [&](const double* v, double* z) { sys_visit(S, 0, v, z, true, s); }, b, x, s);
}

// Newton-Raphson (Sec. III.A) for a system on curved elements with a
// monomial source: F_a = A_a(u_a; u_b,a) + M S_a(u) - b_a; each step sets the
// couplings D = M dS/du, solves blockdiag(A_a) + D by FGMRES with the system
// V-cycle to linear_rtol, and backtracks the step length.
struct SysNewtonRun {
  dgs_system* S = nullptr;
  MonomialSource ms;
  const double *bvals = nullptr, *b = nullptr, *mdiag = nullptr;
  double* u = nullptr;
  double newton_rtol = 0;
  hipStream_t s = nullptr;
  long long nd = 0, n = 0;
  double *F = nullptr, *Ft = nullptr, *du = nullptr, *ut = nullptr, *work = nullptr;
  KrylovSpace K;
  double nrm2 = 0, norm0 = 0;
  std::vector<double> hist;
  int its = 0, steps = 0, backtracks = 0;
  bool converged = false;

  void residual(const double* x, double* out) {
    for (int a = 0; a < S->nv; ++a) {
      dgs_problem* Pa = S->var[a];
      const Level& L0 = Pa->levels[0];
      HIP_OK(launch_curved_apply_bc(Pa->N, x + a * nd, out + a * nd, bvals ? bvals + a * nd : nullptr,
                                    Pa->curved, Pa->metric_on ? &Pa->metric : nullptr, L0.d_nbr,
                                    Pa->penalty, L0.op.neumann, L0.E, s));
    }
    HIP_OK(launch_monomial_source(ms, x, mdiag, b, out, nullptr, nd, s));
  }
  double norm2(const double* x) { return device_norm2(K, x, s); }
  void init(dgs_system* sys, const MonomialSource& src, const double* bv, const double* bb, double* uu,
            double nrt, hipStream_t st) {
    S = sys;
    newton_rtol = nrt;
    ms = src;
    bvals = bv;
    b = bb;
    u = uu;
    s = st;
    dgs_problem* P = S->base();
    nd = S->lv[0].nd;
    n = (long long)S->nv * nd;
    mdiag = ensure_mdiag(P, s);
    const int m = P->opt.restart > 0 ? std::min(P->opt.restart, P->opt.max_iter) : P->opt.max_iter;
    sys_ensure_krylov(S, m);
    K.m = m;
    K.n = n;
    K.V = S->V;
    K.Z = S->Z;
    K.partial = S->partial;
    K.h = S->h;
    K.y = S->y;
    K.tmp = S->tmp;
    K.pinned = S->h_pinned;
    if (!S->d_newton) S->d_newton = S->alloc<double>((size_t)5 * n);
    F = S->d_newton;
    Ft = F + n;
    du = F + 2 * n;
    ut = F + 3 * n;
    work = F + 4 * n;
    residual(u, F);
    nrm2 = norm2(F);
    if (!std::isfinite(nrm2)) throw DgsError(DGS_ERR_NONFINITE, "non-finite nonlinear residual");
    norm0 = std::sqrt(nrm2);
    hist.assign(1, 1.0);
    converged = norm0 == 0.0;
  }
  void step(double linear_rtol) {
    // the couplings of the linearisation, D = M dS/du, written straight into
    // the finest level's coupling fields
    HIP_OK(launch_monomial_source(ms, u, mdiag, nullptr, nullptr, S->lv[0].D, nd, s));
    sys_set_coupling(S, S->lv[0].D, s);
    HIP_OK(launch_fill(work, 0.0, n, s));
    HIP_OK(launch_axpy(work, -1.0, F, n, s));
    HIP_OK(launch_fill(du, 0.0, n, s));
    FgmresResult R = sys_fgmres(S, work, du, s, linear_rtol);
    its += R.iterations;
    const double ft = backtracking_line_search(
        nrm2,
        [&](double lam) {
          HIP_OK(launch_waxpy(ut, u, lam, du, n, s));
          residual(ut, Ft);
          return 0.5 * norm2(Ft);
        },
        backtracks);
    HIP_OK(launch_copy(u, ut, n, s));
    std::swap(F, Ft);
    nrm2 = 2.0 * ft;
    ++steps;
    hist.push_back(std::sqrt(nrm2) / norm0);
    converged = std::sqrt(nrm2) <= newton_rtol * norm0;
    HIP_OK(hipStreamSynchronize(s));
  }
};

}  // namespace

extern "C" {

int dgs_create_system(const dgs_domain* domain, const int elements[3], int p, double penalty,
                      int nvars, const int* neumann_faces, int laplacian_bc,
                      const dgs_options* opt, void* stream, dgs_system** out) {
  return guarded([&]() -> int {
    if (!domain || !elements || !neumann_faces || !out) return fail(DGS_ERR_INVALID, "NULL argument");
    *out = nullptr;
    if (nvars < 1 || nvars > kSysMaxVars) return fail(DGS_ERR_INVALID, "nvars must be in [1, 5]");
    if (laplacian_bc != 0 && laplacian_bc != 1)
      return fail(DGS_ERR_INVALID, "laplacian_bc must be 0 (matched) or 1 (Dirichlet)");
    std::vector<int> masks(neumann_faces, neumann_faces + nvars);
    for (int m : masks)
      if (m < 0 || m >= 63) return fail(DGS_ERR_INVALID, "Neumann faces must leave one face Dirichlet");
    dgs_options o;
    dgs_default_options(&o);
    if (opt) o = *opt;
    const double t0 = now_s();
    hipStream_t s = as_stream(stream);
    std::unique_ptr<dgs_system> S(new dgs_system());
    S->nv = nvars;
    S->matched = laplacian_bc == 0;
    for (int a = 0; a <= nvars; ++a) {
      if (a == nvars && S->matched) break;
      o.neumann_faces = a < nvars ? masks[a] : 0;
      dgs_problem* Pa = nullptr;
      const int rc = create_problem(domain, elements, p, penalty, &o, nullptr, nullptr, nullptr,
                                    stream, &Pa, /*light=*/true, &masks);
      if (rc != DGS_OK) return rc;
      if (a < nvars)
        S->var.push_back(Pa);
      else
        S->dir = Pa;
    }
    dgs_problem* P = S->base();
    for (const Level& L : P->levels)
      if (L.max_n > kSysMaxRows)
        return fail(DGS_ERR_INVALID, "system subdomains are limited to 2048 points (p <= 8 with overlap 2)");
    // tune the first variable; the others share its level shapes
    autotune_apply(P, s);
    autotune_gemm(P, s);
    std::vector<dgs_problem*> others(S->var.begin() + 1, S->var.end());
    if (S->dir) others.push_back(S->dir);
    for (dgs_problem* Q : others)
      for (size_t l = 0; l < P->levels.size(); ++l) {
        Q->levels[l].acfg = P->levels[l].acfg;
        Q->levels[l].acfg_out = P->levels[l].acfg_out;
        Q->levels[l].gemm_variant = P->levels[l].gemm_variant;
        Q->levels[l].kparts = P->levels[l].kparts;
      }
    const int nv = nvars, k = o.subdomain_iters;
    for (size_t l = 0; l < P->levels.size(); ++l) {
      const Level& L = P->levels[l];
      SysLevel SL;
      SL.nd = P->nd((int)l);
      SL.st = L.rs_total;
      const size_t es = L.f32 ? sizeof(float) : sizeof(double);
      // the joined class list of all variables and its tile plan (32 x 64 or
      // 16 x 64 tiles, the instances of the grouped GEMM with class pointers)
      SL.ncls = (int)L.cls.size();
      std::vector<ClassInfo> ci_inv, ci_op;
      for (int a = 0; a < nv; ++a) {
        const Level& La = S->var[a]->levels[l];
        const Level& Lm = (S->matched ? S->var[a] : S->dir)->levels[l];
        for (int c = 0; c < SL.ncls; ++c) {
          ClassInfo I = Lm.cls[c];
          ci_inv.push_back(I);
          ClassInfo O = La.cls[c];
          O.inv = O.op;
          O.scale = O.scale_op;
          ci_op.push_back(O);
        }
      }
      const GemmPlan plan = plan_subdomain_gemm(ci_inv, 2);
      SL.kparts = plan.kparts;
      SL.small = plan.small;
      SL.ntiles = (int)plan.tiles.size();
      SL.tiles = S->alloc<GemmTile>(plan.tiles.size());
      upload(SL.tiles, plan.tiles, s);
      SL.cls_inv = S->alloc<ClassInfo>(ci_inv.size());
      upload(SL.cls_inv, ci_inv, s);
      SL.cls_op = S->alloc<ClassInfo>(ci_op.size());
      upload(SL.cls_op, ci_op, s);
      const int mp = SL.kparts;
      SL.D = S->alloc<double>((size_t)nv * nv * SL.nd);
      HIP_OK(launch_fill(SL.D, 0.0, (long long)nv * nv * SL.nd, s));
      SL.r = S->alloc<double>((size_t)nv * SL.nd);
      if (l > 0) {
        SL.b = S->alloc<double>((size_t)nv * SL.nd);
        SL.u = S->alloc<double>((size_t)nv * SL.nd);
      }
      // rows and products: the class blocks' padding must read as zero
      SL.rs = S->alloc<char>(es * nv * SL.st);
      SL.du = S->alloc<char>(es * nv * SL.st);
      SL.parts = S->alloc<char>(es * (size_t)mp * nv * SL.st);
      HIP_OK(hipMemsetAsync(SL.rs, 0, es * nv * SL.st, s));
      HIP_OK(hipMemsetAsync(SL.du, 0, es * nv * SL.st, s));
      HIP_OK(hipMemsetAsync(SL.parts, 0, es * (size_t)mp * nv * SL.st, s));
      // class (a, c) reads variable a's rows and writes variable a's block of
      // every part ([part][variable][row])
      auto ptr_table = [&](const void* rows_base) {
        std::vector<GemmPtr> t;
        for (int a = 0; a < nv; ++a)
          for (int c = 0; c < SL.ncls; ++c)
            t.push_back(GemmPtr{(const char*)rows_base + es * (size_t)(a * SL.st),
                                (char*)SL.parts + es * (size_t)(a * SL.st), (long long)nv * SL.st});
        GemmPtr* d = S->alloc<GemmPtr>(t.size());
        upload(d, t, s);
        HIP_OK(hipStreamSynchronize(s));  // t goes out of scope
        return d;
      };
      SL.ptr_rs = ptr_table(SL.rs);
      if (k > 0) {
        SL.gV = S->alloc<char>(es * (size_t)(k + 1) * nv * SL.st);
        SL.gZ = S->alloc<char>(es * (size_t)k * nv * SL.st);
        SL.gW = S->alloc<char>(es * nv * SL.st);
        HIP_OK(hipMemsetAsync(SL.gV, 0, es * (size_t)(k + 1) * nv * SL.st, s));
        HIP_OK(hipMemsetAsync(SL.gZ, 0, es * (size_t)k * nv * SL.st, s));
        HIP_OK(hipMemsetAsync(SL.gW, 0, es * nv * SL.st, s));
        SL.H = S->alloc<double>((size_t)L.E * (k + 1) * k);
        SL.beta = S->alloc<double>(L.E);
        for (int j = 0; j < k; ++j) {
          SL.ptr_inv.push_back(ptr_table((const char*)SL.gV + es * (size_t)j * nv * SL.st));
          SL.ptr_op.push_back(ptr_table((const char*)SL.gZ + es * (size_t)j * nv * SL.st));
        }
      }
      HIP_OK(hipStreamSynchronize(s));  // the class lists and the plan go out of scope
      S->lv.push_back(SL);
    }
    HIP_OK(hipStreamSynchronize(s));
    S->t_setup = now_s() - t0;
    *out = S.release();
    return DGS_OK;
  });
}

int dgs_destroy_system(dgs_system* sys) {
  return guarded([&]() -> int {
    delete sys;
    return DGS_OK;
  });
}

int dgs_system_num_dofs(const dgs_system* sys, long long* n) {
  if (!sys || !n) return fail(DGS_ERR_INVALID, "NULL argument");
  *n = sys->lv[0].nd;
  return DGS_OK;
}

int dgs_system_set_coupling(dgs_system* sys, const double* D, void* stream) {
  return guarded([&]() -> int {
    if (!sys) return fail(DGS_ERR_INVALID, "NULL argument");
    hipStream_t s = as_stream(stream);
    const dgs_problem* P = sys->base();
    const int nv = sys->nv;
    if (!D) {
      for (SysLevel& SL : sys->lv) HIP_OK(launch_fill(SL.D, 0.0, (long long)nv * nv * SL.nd, s));
      sys->coupled = false;
      return DGS_OK;
    }
    (void)P;
    (void)nv;
    sys_set_coupling(sys, D, s);
    return DGS_OK;
  });
}

int dgs_system_set_geometry(dgs_system* sys, const double* xyz, void* stream) {
  return guarded([&]() -> int {
    if (!sys) return fail(DGS_ERR_INVALID, "NULL argument");
    for (dgs_problem* p : sys->var) {
      const int rc = dgs_set_geometry(p, xyz, stream);
      if (rc != DGS_OK) return rc;
    }
    return DGS_OK;
  });
}

int dgs_system_set_metric(dgs_system* sys, const double* ginv, const double* sqrtg, void* stream) {
  return guarded([&]() -> int {
    if (!sys) return fail(DGS_ERR_INVALID, "NULL argument");
    for (dgs_problem* p : sys->var) {
      const int rc = dgs_set_metric(p, ginv, sqrtg, stream);
      if (rc != DGS_OK) return rc;
    }
    return DGS_OK;
  });
}

int dgs_system_newton_solve_powers(dgs_system* sys, int nterms, const int* vars, const int* powers,
                                   const double* coef, const double* dirichlet, const double* b,
                                   double* u, double newton_rtol, double linear_rtol, int max_newton,
                                   dgs_stats* stats, void* stream) {
  return guarded([&]() -> int {
    if (!sys || !vars || !powers || !coef || !u) return fail(DGS_ERR_INVALID, "NULL argument");
    const int nv = sys->nv;
    if (nterms < 1 || nterms > kMaxMonomials)
      return fail(DGS_ERR_INVALID, "the sources take 1 to 16 terms");
    MonomialSource ms;
    ms.nv = nv;
    ms.nterm = nterms;
    ms.coef = coef;
    for (int t = 0; t < nterms; ++t) {
      if (vars[t] < 0 || vars[t] >= nv) return fail(DGS_ERR_INVALID, "a term's variable is out of range");
      ms.var[t] = vars[t];
      for (int q = 0; q < nv; ++q) {
        const int k = powers[t * nv + q];
        if (k < -kMaxPower || k > kMaxPower) return fail(DGS_ERR_INVALID, "powers must lie in [-12, 12]");
        ms.power[t][q] = k;
      }
    }
    if (!(newton_rtol > 0.0) || !(linear_rtol > 0.0) || max_newton < 1)
      return fail(DGS_ERR_INVALID, "invalid Newton tolerances");
    for (const dgs_problem* p : sys->var)
      if (!p->curved_on)
        return fail(DGS_ERR_INVALID, "set node coordinates (dgs_system_set_geometry) or a metric first");
    hipStream_t s = as_stream(stream);
    const double t0 = now_s();
    SysNewtonRun nr;
    nr.init(sys, ms, dirichlet, b, u, newton_rtol, s);
    while (!nr.converged && nr.steps < max_newton) nr.step(linear_rtol);
    // the linearisation's couplings are dropped again
    for (SysLevel& SL : sys->lv) HIP_OK(launch_fill(SL.D, 0.0, (long long)nv * nv * SL.nd, s));
    sys->coupled = false;
    HIP_OK(hipStreamSynchronize(s));
    if (stats) {
      stats->iterations = nr.its;
      stats->newton_steps = nr.steps;
      stats->backtracks = nr.backtracks;
      stats->rel_residual = std::sqrt(nr.nrm2) / (nr.norm0 > 0 ? nr.norm0 : 1.0);
      stats->t_solve_s = now_s() - t0;
      stats->t_setup_s = sys->t_setup;
      stats->history_len = 0;
      if (stats->history && stats->history_capacity > 0) {
        const int m = std::min<int>(stats->history_capacity, (int)nr.hist.size());
        for (int i = 0; i < m; ++i) stats->history[i] = nr.hist[i];
        stats->history_len = m;
      }
    }
    return nr.converged ? DGS_OK : DGS_NOT_CONVERGED;
  });
}

int dgs_system_apply(dgs_system* sys, const double* u, double* y, void* stream) {
  return guarded([&]() -> int {
    if (!sys || !u || !y) return fail(DGS_ERR_INVALID, "NULL argument");
    if (u == y) return fail(DGS_ERR_INVALID, "u and y must not overlap");
    sys_apply(sys, u, y, as_stream(stream));
    return DGS_OK;
  });
}

int dgs_system_smooth(dgs_system* sys, const double* b, double* u, int steps, void* stream) {
  return guarded([&]() -> int {
    if (!sys || !b || !u) return fail(DGS_ERR_INVALID, "NULL argument");
    if (steps < 0) return fail(DGS_ERR_INVALID, "steps must be >= 0");
    sys_schwarz_steps(sys, 0, b, u, steps, false, as_stream(stream));
    return DGS_OK;
  });
}

int dgs_system_precondition(dgs_system* sys, const double* r, double* z, void* stream) {
  return guarded([&]() -> int {
    if (!sys || !r || !z) return fail(DGS_ERR_INVALID, "NULL argument");
    if (r == z) return fail(DGS_ERR_INVALID, "r and z must not overlap");
    sys_visit(sys, 0, r, z, true, as_stream(stream));
    return DGS_OK;
  });
}

int dgs_system_solve(dgs_system* sys, const double* b, double* u, dgs_stats* stats, void* stream) {
  return guarded([&]() -> int {
    if (!sys || !b || !u) return fail(DGS_ERR_INVALID, "NULL argument");
    if (b == u) return fail(DGS_ERR_INVALID, "b and u must not overlap");
    const double t0 = now_s();
    FgmresResult R = sys_fgmres(sys, b, u, as_stream(stream));
    fill_stats(stats, R, t0, sys->t_setup);
    if (stats) {
      stats->newton_steps = 0;
      stats->backtracks = 0;
    }
    return R.converged ? DGS_OK : DGS_NOT_CONVERGED;
  });
}

}  // extern "C"
