// Host-side helpers shared by the library's C++ sources: error handling
// (errors travel as DgsError exceptions inside the library and become return
// codes at the C ABI), device allocation under one process-wide lock, and a
// host-driven flexible GMRES over caller-supplied operator callbacks.
#pragma once

#include <chrono>
#include <cmath>
#include <exception>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/dgsolve.h"
#include "dgs_internal.h"

namespace dgs {

inline thread_local std::string g_last_error;

class DgsError {
 public:
  DgsError(int c, std::string m) : code(c), msg(std::move(m)) {}
  int code;
  std::string msg;
};

#define HIP_OK(expr)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::dgs::DgsError(e_ == hipErrorOutOfMemory ? DGS_ERR_OOM : DGS_ERR_HIP,         \
                            std::string(#expr) + ": " + hipGetErrorString(e_));             \
  } while (0)

inline double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// One process-wide lock around the library's device-management calls:
// allocation and release of device and pinned memory, stream creation and
// destruction, and graph capture and instantiation.  Kernel and graph
// launches, copies and stream queries do not take it.  The serving loop's
// worker threads set up requests (allocating, capturing) while others launch,
// and a capture must not overlap another thread's allocation or release (a
// release waits for the device), so these calls are serialised here.
inline std::recursive_mutex g_dev_mutex;

inline void dfree(void* p) {
  std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
  (void)hipFree(p);
}

template <typename T>
T* dalloc(size_t count) {
  if (count == 0) count = 1;
  void* p = nullptr;
  std::lock_guard<std::recursive_mutex> lk(g_dev_mutex);
  hipError_t e = hipMalloc(&p, count * sizeof(T));
  if (e != hipSuccess)
    throw DgsError(e == hipErrorOutOfMemory ? DGS_ERR_OOM : DGS_ERR_HIP,
                   std::string("hipMalloc: ") + hipGetErrorString(e));
  return static_cast<T*>(p);
}

template <typename T>
void upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return;
  HIP_OK(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

template <typename F>
int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const DgsError& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(DGS_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(DGS_ERR_HIP, e.what());
  }
}

struct FgmresResult {
  int iterations = 0;
  double rel_residual = 0;
  bool converged = false;
  std::vector<double> history;
};

// Buffers of a host-driven FGMRES(m) on vectors of n entries: the basis V
// (m + 1 vectors), the preconditioned vectors Z (m), reduction partials,
// 3 (m + 2) device scalars, the m coefficients y, one work vector, and
// 4 (m + 2) doubles of pinned host staging.
struct KrylovSpace {
  int m = 0;
  long long n = 0;
  double *V = nullptr, *Z = nullptr, *partial = nullptr, *h = nullptr, *y = nullptr;
  double* tmp = nullptr;
  double* pinned = nullptr;
};

inline double device_norm2(const KrylovSpace& K, const double* x, hipStream_t s) {
  HIP_OK(launch_multidot(x, K.n, 1, x, K.n, K.partial, K.h, s));
  HIP_OK(hipMemcpyAsync(K.pinned, K.h, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_OK(hipStreamSynchronize(s));
  return K.pinned[0];
}

// Flexible GMRES (Saad Alg. 9.6) with one preconditioner application per
// iteration: classical Gram-Schmidt twice, Givens rotations on the host,
// cycles of at most K.m iterations (restarts from the true residual), and
// convergence decided by the true residual of the solution (a cycle whose
// estimate meets rtol while the true residual does not is followed by
// another cycle).  residual(x, b, out): out = b - A x; apply(z, w): w = A z;
// precondition(v, z): z ~ A^-1 v.  All enqueue on s.
template <class Residual, class Apply, class Precondition>
FgmresResult fgmres_run(const KrylovSpace& K, double rtol, int max_total, Residual&& residual,
                        Apply&& apply, Precondition&& precondition, const double* b, double* x,
                        hipStream_t s) {
  const int m = K.m;
  const long long n = K.n;
  double* hp = K.pinned;
  FgmresResult R;
  double beta0 = 0.0;
  for (int cycle = 0;; ++cycle) {
    residual(x, b, K.V);
    const double beta2 = device_norm2(K, K.V, s);
    if (!std::isfinite(beta2)) throw DgsError(DGS_ERR_NONFINITE, "non-finite initial residual");
    const double beta = std::sqrt(beta2);
    if (cycle == 0) {
      beta0 = beta;
      R.history.push_back(1.0);
    }
    if (beta == 0.0) {
      R.converged = true;
      R.rel_residual = 0.0;
      return R;
    }
    HIP_OK(launch_scale_by_inv_norm(K.V, K.V, K.h, n, s));
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m, 0.0), sn(m, 0.0), g(m + 1, 0.0);
    g[0] = beta;
    int j = 0;
    while (true) {
      double* vj = K.V + (size_t)j * n;
      double* zj = K.Z + (size_t)j * n;
      double* w = K.V + (size_t)(j + 1) * n;
      precondition(vj, zj);
      apply(zj, w);
      double* h1 = K.h;
      double* h2 = K.h + (m + 2);
      double* hn = K.h + 2 * (m + 2);
      HIP_OK(launch_multidot(K.V, n, j + 1, w, n, K.partial, h1, s));
      HIP_OK(launch_axpy_multidot(K.V, n, j + 1, h1, w, n, false, K.partial, h2, s));
      HIP_OK(launch_axpy_multidot(K.V, n, j + 1, h2, w, n, true, K.partial, hn, s));
      HIP_OK(hipMemcpyAsync(hp, K.h, sizeof(double) * (2 * (m + 2) + 1), hipMemcpyDeviceToHost, s));
      HIP_OK(launch_scale_by_inv_norm(w, w, hn, n, s));
      HIP_OK(hipStreamSynchronize(s));
      double* col = &H[(size_t)j * (m + 1)];
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
      if (std::fabs(g[j]) <= rtol * beta0 || hn2 == 0.0 || j >= m || R.iterations >= max_total) break;
    }
    std::vector<double> y(j, 0.0);
    for (int i = j - 1; i >= 0; --i) {
      double t = g[i];
      for (int q = i + 1; q < j; ++q) t -= H[(size_t)q * (m + 1) + i] * y[q];
      y[i] = t / H[(size_t)i * (m + 1) + i];
    }
    double* ypin = hp + 3 * (m + 2);
    for (int i = 0; i < j; ++i) ypin[i] = y[i];
    HIP_OK(hipMemcpyAsync(K.y, ypin, sizeof(double) * j, hipMemcpyHostToDevice, s));
    HIP_OK(launch_combine(x, K.Z, n, j, K.y, n, s));
    residual(x, b, K.tmp);
    R.rel_residual = std::sqrt(device_norm2(K, K.tmp, s)) / beta0;
    if (!std::isfinite(R.rel_residual)) throw DgsError(DGS_ERR_NONFINITE, "non-finite residual");
    R.converged = R.rel_residual <= rtol;
    if (R.converged || R.iterations >= max_total) return R;
  }
}

}  // namespace dgs
