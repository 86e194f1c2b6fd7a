// Shared declarations of the rsfgp HIP library (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/rsfgp.h"

namespace rsf {

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define RSF_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::rsf::Error(e_ == hipErrorOutOfMemory ? RSF_E_OOM : RSF_E_HIP,             \
                         std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

#define RSF_CHECK(cond, code, msg)                     \
  do {                                                 \
    if (!(cond)) throw ::rsf::Error((code), (msg));    \
  } while (0)

// ---------------------------------------------------------------- device memory
// Device allocations owned by a factor (returned to the pool in the
// destructor).  Every allocation is accounted against the handle's memory cap.
void* pool_alloc(size_t nbytes, hipStream_t s);
void pool_free(void* p, size_t nbytes, hipStream_t s);
void pool_trim();
// true: the caller has synchronised the device, so reusing memory released
// on another stream needs no stream synchronisation (used while recording a
// graph, where such a synchronisation is not allowed)
void pool_sync_free(bool on);

struct Arena {
  std::vector<void*> blocks;
  std::vector<size_t> sizes;
  size_t bytes = 0;  // bytes handed out (the cap applies to these)
  size_t cap = 0;    // 0 = unlimited
  // small requests are carved from 4 MiB slabs taken from the pool
  char* slab = nullptr;
  size_t slab_left = 0;
  void* alloc(size_t nbytes);
  template <class T>
  T* make(size_t count) {
    return static_cast<T*>(alloc(count * sizeof(T)));
  }
  void release();
  ~Arena() { release(); }
};

// While alive on a thread, that thread may not take device memory from the
// pool (pool_alloc throws RSF_E_INVALID) and the level-step autotuner runs no
// timing trials: the calls behind the no-allocation entry points.
struct NoAllocScope {
  bool was;
  NoAllocScope();
  ~NoAllocScope();
};
bool no_alloc_active();

// Scratch allocations for one call, returned to the stream-ordered pool when
// the object goes out of scope.  A Scratch made over a fixed device buffer
// instead carves every request from that buffer (256-byte aligned, in order)
// and never touches the pool; a request beyond its end throws RSF_E_INVALID.
struct Scratch {
  std::vector<void*> blocks;
  std::vector<size_t> sizes;
  hipStream_t stream = nullptr;
  size_t cap_left = 0;  // 0 = unlimited
  // small requests (launch descriptors, index lists) are carved from
  // SMALL_SLAB-byte slabs taken from the pool
  static constexpr size_t SMALL_MAX = size_t(256) << 10, SMALL_SLAB = size_t(4) << 20;
  std::vector<void*> slabs;
  char* slab = nullptr;
  size_t slab_left = 0;
  char* fixed = nullptr;  // fixed-buffer mode: base, size and bytes handed out
  size_t fixed_cap = 0, fixed_used = 0;
  explicit Scratch(hipStream_t s) : stream(s) {}
  Scratch(hipStream_t s, void* buf, size_t nbytes) : stream(s), fixed(static_cast<char*>(buf)), fixed_cap(nbytes) {}
  void* alloc(size_t nbytes);
  template <class T>
  T* make(size_t count) {
    return static_cast<T*>(alloc(count * sizeof(T)));
  }
  // Returns one block to the pool early (stream-ordered: later work on the
  // stream may reuse it).  Null pointers, unknown pointers and small requests
  // (carved from a slab) are ignored.
  void release(const void* p);
  ~Scratch();
};

// Host-to-device copy of launch descriptors and index lists, staged through a
// pinned ring buffer so that the copy is asynchronous on stream s.
void upload_bytes(void* dst, const void* src, size_t nbytes, hipStream_t s);
// While a stream capture records a graph, uploads go through pinned blocks
// that the graph keeps (appended to *pins) instead of the reusable ring.
void upload_capture_begin(std::vector<void*>* pins);
void upload_capture_end();

template <class T>
inline void upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (!src.empty()) upload_bytes(dst, src.data(), src.size() * sizeof(T), s);
}

// accumulator of one 16 x 16 x 4 FP64 matrix-core product (4 doubles per lane)
typedef double v4d __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- batched GEMM
// C(i, j) = alpha * sum_p A(i, p) B(p, j) + beta * C(i, j) for one problem.
// Element (i, j) of an operand X lives at X.ptr[row(i) * rs + j * cs] where
// row(i) = idx ? idx[i] : i.  Transposition is a swap of rs and cs (with the
// index map moving along); gathers and scatters of vector-panel rows use idx.
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  const int* aidx;
  const int* bidx;
  const int* cidx;
  const int* kidx;  // A(i, k) reads column kidx[k] of A (the 128 x 128 kernels: k-contiguous A only)
  long long ars, acs, brs, bcs, crs, ccs;
  int M, N, K;
  double alpha, beta;
  int lower;  // 1: only tiles touching the lower triangle of C (i >= j) are computed
  int tri;    // A triangular with zeros stored in its other half: 1 lower (A(i, p) = 0
              // for p > i), 2 upper (A(i, p) = 0 for p < i); each tile then multiplies
              // only the K chunks its rows can reach (plain A only: no row or K map)
  int f32;    // 1: operands rounded to FP32, FP32 matrix-core products with FP32
              //    accumulation; alpha * acc + beta * C is formed in FP64
};

struct Mat {
  const double* p = nullptr;
  long long rs = 0, cs = 0;
  const int* idx = nullptr;
};
// column-major m x n with leading dimension ld
inline Mat colmaj(const double* p, long long ld) { return Mat{p, 1, ld, nullptr}; }
// transpose of a column-major matrix
inline Mat colmajT(const double* p, long long ld) { return Mat{p, ld, 1, nullptr}; }
// rows of a row-major panel (row = DOF, ld = panel width), optional row map
inline Mat panel(const double* p, long long ld, const int* idx = nullptr) {
  return Mat{p, ld, 1, idx};
}

inline GemmDesc gemm_desc(int M, int N, int K, double alpha, Mat A, Mat B, double beta, Mat C) {
  GemmDesc d;
  d.A = A.p;
  d.B = B.p;
  d.C = const_cast<double*>(C.p);
  d.aidx = A.idx;
  d.bidx = B.idx;
  d.cidx = C.idx;
  d.kidx = nullptr;
  d.ars = A.rs;
  d.acs = A.cs;
  d.brs = B.rs;
  d.bcs = B.cs;
  d.crs = C.rs;
  d.ccs = C.cs;
  d.M = M;
  d.N = N;
  d.K = K;
  d.alpha = alpha;
  d.beta = beta;
  d.lower = 0;
  d.tri = 0;
  d.f32 = 0;
  return d;
}

// Launches one batched GEMM over all problems in `descs` (problems with an
// empty output are skipped).  The descriptors are copied to the device.
void gemm_batched(const std::vector<GemmDesc>& descs, Scratch& scr, hipStream_t s);

// Batched blocked Cholesky (lower, in place) with the inverse factor:
// A_p = L_p L_p^T, Linv_p = L_p^-1 (strict upper part zero), and per 64-column
// block of each problem the partial 2 sum log L_jj into logd_p[block].
// Right-looking with 64-column panels: one launch per panel for the diagonal
// blocks of all problems, then the panel and trailing updates as batched
// matrix-core GEMMs; the inverse is built block row by block row the same way.
struct CholProblem {
  double* A;
  long long lda;
  int n;
  double* Linv;
  long long ldi;
  double* logd;  // ceil(n / 64) values, may be null
};
void batched_chol_inv(const std::vector<CholProblem>& P, int* fail, Scratch& scr, hipStream_t s);

// dst(i, j) = src(i, j) for i < m, j < n (column-major); lower: zero for i < j;
// src == nullptr: zero fill
struct CopyBlock {
  const double* src;
  long long lds;
  double* dst;
  long long ldd;
  int m, n, lower;
};
void copy_blocks(const std::vector<CopyBlock>& jobs, Scratch& scr, hipStream_t s);

// Tracing of the batched GEMM launches: HIP events around every launch on
// its stream, with the algorithmic flops (2 M N K) and operand bytes counted.
void trace_enable(bool on);
void trace_read(double* ms, double* flops, double* bytes, long long* launches, bool reset);
// union of the traced launches' intervals (ms) as of the last trace_read
double trace_busy();
// "tag:ms:flops;..." per call-site tag (read after trace_read)
std::string trace_tags();
// algorithmic work booked per kernel name while tracing is on (host counts,
// no events): flops, bytes and dispatches; "name:flops:bytes:dispatches;..."
void trace_kernel_work(const std::string& kernel, double flops, double bytes, double dispatches = 1.0);
std::string trace_kernels();
// The current phase name.
std::string trace_current();
// Times the launches issued on stream s while it is alive (HIP events) and
// counts their algorithmic flops and bytes under the current phase name.
struct TraceLaunch {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipStream_t s;
  double flops, bytes;
  TraceLaunch(hipStream_t st, double fl, double by);
  ~TraceLaunch();
};
// Suspends launch tracing while it is alive (work that is not part of the
// computation, such as autotuning trials).
struct TracePause {
  bool was;
  TracePause();
  ~TracePause();
};
// Names the GEMM launches issued while it is alive (for the per-phase split).
struct TraceTag {
  std::string prev;
  explicit TraceTag(const char* t);
  ~TraceTag();
};

// Reproducible sum of n doubles (fixed reduction tree) into *out (device).
void device_sum(const double* x, long long n, double* out, Scratch& scr, hipStream_t s);
// out[0] = sum_i x[i] * y[i] (fixed reduction tree).
void device_dot(const double* x, const double* y, long long n, double* out, Scratch& scr,
                hipStream_t s);

// ---------------------------------------------------------------- kernel functions
enum { K_MATERN12 = 0, K_MATERN32 = 1, K_MATERN52 = 2, K_RQ = 3, K_MATERN32_ANISO = 4, K_RQ_ANISO = 5 };

struct KernelParams {
  int kernel;
  double rho, sigma2, nugget, alpha;
  double rho2;  // anisotropic kernels: rho = theta_1 (x), rho2 = theta_2 (y), sigma2 = 1
  int deriv;  // 0: Sigma entries, 1: d/drho (d/dtheta_1) entries, 2: d/dtheta_2 entries
  int f32;    // 1: entries evaluated in FP32 arithmetic (mixed precision)
};

__device__ __forceinline__ double corr_dev(double s, int kernel, double alpha) {
  if (kernel == K_MATERN12) return exp(-s);
  if (kernel == K_MATERN32) {
    double t = 1.7320508075688772 * s;
    return (1.0 + t) * exp(-t);
  }
  if (kernel == K_MATERN52) {
    double t = 2.23606797749979 * s;
    return (1.0 + t + (5.0 / 3.0) * s * s) * exp(-t);
  }
  if (alpha == 1.0) return 1.0 / (1.0 + 0.5 * s * s);
  return pow(1.0 + s * s / (2.0 * alpha), -alpha);
}

__device__ __forceinline__ double dcorr_drho_dev(double r, double rho, int kernel, double alpha) {
  double s = r / rho;
  if (kernel == K_MATERN12) return (r / (rho * rho)) * exp(-s);
  if (kernel == K_MATERN32) return 3.0 * r * r / (rho * rho * rho) * exp(-1.7320508075688772 * s);
  if (kernel == K_MATERN52)
    return (5.0 * r * r / (3.0 * rho * rho * rho)) * (1.0 + 2.23606797749979 * s) *
           exp(-2.23606797749979 * s);
  if (alpha == 1.0) {
    double b = 1.0 / (1.0 + 0.5 * s * s);
    return (r * r / (rho * rho * rho)) * b * b;
  }
  return (r * r / (rho * rho * rho)) * pow(1.0 + s * s / (2.0 * alpha), -alpha - 1.0);
}

// FP32 forms of the two functions above (mixed precision).
__device__ __forceinline__ float corr_dev32(float s, int kernel, float alpha) {
  if (kernel == K_MATERN12) return expf(-s);
  if (kernel == K_MATERN32) {
    const float t = 1.7320508f * s;
    return (1.0f + t) * expf(-t);
  }
  if (kernel == K_MATERN52) {
    const float t = 2.2360680f * s;
    return (1.0f + t + (5.0f / 3.0f) * s * s) * expf(-t);
  }
  if (alpha == 1.0f) return 1.0f / (1.0f + 0.5f * s * s);
  return powf(1.0f + s * s / (2.0f * alpha), -alpha);
}

__device__ __forceinline__ float dcorr_drho_dev32(float r, float rho, int kernel, float alpha) {
  const float s = r / rho, c = r * r / (rho * rho * rho);
  if (kernel == K_MATERN12) return (r / (rho * rho)) * expf(-s);
  if (kernel == K_MATERN32) return 3.0f * c * expf(-1.7320508f * s);
  if (kernel == K_MATERN52) return (5.0f / 3.0f) * c * (1.0f + 2.2360680f * s) * expf(-2.2360680f * s);
  if (alpha == 1.0f) {
    const float b = 1.0f / (1.0f + 0.5f * s * s);
    return c * b * b;
  }
  return c * powf(1.0f + s * s / (2.0f * alpha), -alpha - 1.0f);
}

// Anisotropic kernels of the runtime experiments (eq. specmatern, eq. specrq):
// k(s) with the scaled distance s^2 = dx^2 / theta_1^2 + dy^2 / theta_2^2,
// no variance factor.  With h = -dk/d(s^2) (Matern 3/2: 3/2 exp(-sqrt3 s);
// RQ(alpha): 1/2 (1 + s^2 / (2 alpha))^(-alpha-1)),
// dk/dtheta_i = h * 2 d_i^2 / theta_i^3.
__device__ __forceinline__ double kentry_aniso(double dx, double dy, const KernelParams& kp) {
  const double ux = dx / kp.rho, uy = dy / kp.rho2, s2 = ux * ux + uy * uy;
  const bool m32 = kp.kernel == K_MATERN32_ANISO;
  if (!kp.deriv) return corr_dev(sqrt(s2), m32 ? K_MATERN32 : K_RQ, kp.alpha);
  const double h = m32 ? 1.5 * exp(-1.7320508075688772 * sqrt(s2)) : 0.5 * pow(1.0 + s2 / (2.0 * kp.alpha), -kp.alpha - 1.0);
  const double d = kp.deriv == 1 ? dx : dy, th = kp.deriv == 1 ? kp.rho : kp.rho2;
  return h * 2.0 * d * d / (th * th * th);
}

// Kernel entry between two distinct sites at distance components (dx, dy).
// The components are differences of FP64 coordinates (exact for nearby
// sites); in mixed precision the distance and the kernel are then evaluated
// in FP32.
__device__ __forceinline__ double kentry(double dx, double dy, const KernelParams& kp) {
  if (kp.kernel >= K_MATERN32_ANISO) return kentry_aniso(dx, dy, kp);
  if (kp.f32) {
    const float fx = (float)dx, fy = (float)dy;
    const float r = sqrtf(fx * fx + fy * fy);
    const float v = kp.deriv ? dcorr_drho_dev32(r, (float)kp.rho, kp.kernel, (float)kp.alpha)
                             : corr_dev32(r / (float)kp.rho, kp.kernel, (float)kp.alpha);
    return (double)((float)kp.sigma2 * v);
  }
  double r = sqrt(dx * dx + dy * dy);
  if (kp.deriv) return kp.sigma2 * dcorr_drho_dev(r, kp.rho, kp.kernel, kp.alpha);
  return kp.sigma2 * corr_dev(r / kp.rho, kp.kernel, kp.alpha);
}

// Diagonal entry (same observation).
__device__ __forceinline__ double kdiag(const KernelParams& kp) {
  return kp.deriv ? 0.0 : kp.sigma2 + kp.nugget;
}

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

constexpr int WG = 256;

}  // namespace rsf
