// Recursive skeletonization factorization on the GPU (Sections 2.1 - 2.3):
// per quadtree level, one launch set covers every box of that depth:
//   near field (modified proxy trick, Section 2.3.1)  -> near_kernel
//   compression matrix [Sigma(N, I); M(Gamma, I)]     -> kaux_kernel
//   interpolative decomposition by pivoted QR         -> cpqr_* kernels
//   block elimination (X_sr, X_rr = L L^T, W, X_ss)   -> assemble_kernel, schur_kernel
// and the remaining DOFs of the root get a blocked dense Cholesky.
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "rsf.h"

namespace rsf {

// ------------------------------------------------------------------ small helpers
// A second stream per device for work that runs beside the caller's stream
// (created on first use, default priority, kept until the process ends: the
// device pool may hold extents released on it).
hipStream_t side_stream() {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  RSF_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = streams.find(dev);
  if (it != streams.end()) return it->second;
  hipStream_t s = nullptr;
  RSF_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  streams[dev] = s;
  return s;
}

__global__ void fill_kernel(double* p, long long n, double v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

void fill_zero(double* p, long long n, hipStream_t s) {
  if (n <= 0) return;
  long long blocks = std::min<long long>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, 0.0);
  RSF_HIP(hipGetLastError());
}

void copy_dev(double* dst, const double* src, long long n, hipStream_t s) {
  if (n > 0) RSF_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s));
}

// dst[t] = src ? src[t] : base + t
struct CopySeg {
  int* dst;
  const int* src;
  int base;
  int count;
};

__global__ void copy_segs_kernel(const CopySeg* __restrict__ segs) {
  const CopySeg g = segs[blockIdx.x];
  for (int t = threadIdx.x; t < g.count; t += blockDim.x) g.dst[t] = g.src ? g.src[t] : g.base + t;
}

static void run_copy_segs(const std::vector<CopySeg>& segs, Scratch& scr, hipStream_t s) {
  if (segs.empty()) return;
  CopySeg* d = scr.make<CopySeg>(segs.size());
  upload(d, segs, s);
  hipLaunchKernelGGL(copy_segs_kernel, dim3((unsigned)segs.size()), dim3(256), 0, s, d);
  RSF_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ near field
// For box B: every active DOF outside B whose distance to B's centre is below
// r_near * h.  Candidate groups (boxes of the same depth and shallower leaves
// whose square meets the disc) come from the host; the kernel filters their
// DOFs and compacts the survivors in order (wave ballots).
struct NearJob {
  double cx, cy, r2;
  int owner;        // this box's group id (its own DOFs are excluded)
  int cand0, cand1; // range into the candidate list
  int* out;
  int* cnt;
};

__global__ __launch_bounds__(256) void near_kernel(const NearJob* __restrict__ jobs,
                                                    const int* __restrict__ cand,
                                                    const long long* __restrict__ seg_off,
                                                    const int* __restrict__ seg_len,
                                                    const int* __restrict__ seg_owner,
                                                    const int* __restrict__ dofs,
                                                    const double* __restrict__ px,
                                                    const double* __restrict__ py) {
  __shared__ int wave_tot[4];
  const NearJob J = jobs[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int base = 0;
  for (int c = J.cand0; c < J.cand1; ++c) {
    const int sg = cand[c];
    if (seg_owner[sg] == J.owner) continue;
    const long long off = seg_off[sg];
    const int len = seg_len[sg];
    for (int t0 = 0; t0 < len; t0 += 256) {
      const int t = t0 + tid;
      int dof = -1;
      bool keep = false;
      if (t < len) {
        dof = dofs[off + t];
        const double dx = px[dof] - J.cx, dy = py[dof] - J.cy;
        keep = dx * dx + dy * dy < J.r2;
      }
      const unsigned long long m = __ballot(keep);
      const int before = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) wave_tot[wave] = __popcll(m);
      __syncthreads();
      int wofs = 0;
      for (int w = 0; w < wave; ++w) wofs += wave_tot[w];
      const int tot = wave_tot[0] + wave_tot[1] + wave_tot[2] + wave_tot[3];
      if (keep) J.out[base + wofs + before] = dof;
      base += tot;
      __syncthreads();
    }
  }
  if (tid == 0) *J.cnt = base;
}

// ------------------------------------------------------------------ compression matrix
struct KauxJob {
  double* A;
  long long ld;
  int a, inst;
  const int* act;
  const int* near;
  const int* ncnt;
  double cx, cy, h;
};

__global__ __launch_bounds__(256) void kaux_kernel(const KauxJob* __restrict__ jobs,
                                                    const KernelParams* __restrict__ kps,
                                                    const double* __restrict__ px,
                                                    const double* __restrict__ py,
                                                    const double* __restrict__ pu, int nprox) {
  const KauxJob J = jobs[blockIdx.x];
  const KernelParams kp = kps[J.inst];
  const int nc = *J.ncnt;
  const long long m = nc + nprox;
  const long long tot = m * J.a;
  for (long long e = blockIdx.y * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.y) {
    const int j = (int)(e / m), i = (int)(e - (long long)j * m);
    const int q = J.act[j];
    double xr, yr;
    if (i < nc) {
      const int p = J.near[i];
      xr = px[p];
      yr = py[p];
    } else {
      xr = J.cx + J.h * pu[i - nc];
      yr = J.cy + J.h * pu[nprox + i - nc];
    }
    J.A[(long long)j * J.ld + i] = kentry(xr - px[q], yr - py[q], kp);
  }
}

// ------------------------------------------------------------------ pivoted QR (ID)
// Householder QR with column pivoting; the pivot is the column with the
// largest residual norm (recomputed from the residual rows at every step,
// ties to the lowest index); stop when that norm is <= eps * |R_11|.  After
// the loop T = R_11^-1 R_12 overwrites R_12 in place.
struct CpqrJob {
  double* A;
  long long ld;
  int a;
  const int* ncnt;
  int* piv;
  int* kout;
  // multi-workgroup path only
  double* norms;
  double* v;
  double* scal;  // [0] = v^T v, [1] = |R_11|
  int* done;
};

struct ArgMax {
  double v;
  int i;
};

__device__ __forceinline__ bool better(double v1, int i1, double v2, int i2) {
  return v1 > v2 || (v1 == v2 && i1 < i2);
}

// workgroup-wide argmax of norms[s .. a), lowest index among ties
__device__ ArgMax wg_argmax(const double* norms, int s, int a, ArgMax* red) {
  const int tid = threadIdx.x;
  double bv = -1.0;
  int bi = 0x7fffffff;
  for (int j = s + tid; j < a; j += blockDim.x) {
    const double v = norms[j];
    if (better(v, j, bv, bi)) {
      bv = v;
      bi = j;
    }
  }
  red[tid].v = bv;
  red[tid].i = bi;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (tid < w && better(red[tid + w].v, red[tid + w].i, red[tid].v, red[tid].i)) red[tid] = red[tid + w];
    __syncthreads();
  }
  ArgMax r = red[0];
  __syncthreads();
  return r;
}

__device__ double wg_sum(double v, double* red) {
  const int tid = threadIdx.x;
  v = wave_sum(v);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

// Swap columns s and p, build the Householder vector of column s into vbuf,
// write alpha on the diagonal and zeros below.  Returns v^T v.
__device__ double householder_step(double* A, long long ld, long long m, int s, int p, int* piv,
                                   double* vbuf, double* red) {
  const int tid = threadIdx.x;
  const long long bd = blockDim.x;
  // every loop loads four entries per thread before it stores any (a store
  // would otherwise hold back the next load's round trip); sums keep the order
  if (p != s) {
    double* cs = A + (long long)s * ld;
    double* cq = A + (long long)p * ld;
    for (long long i = tid; i < m; i += 4 * bd) {
      double ts[4], tq[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const long long ii = i + u * bd;
        ts[u] = ii < m ? cs[ii] : 0.0;
        tq[u] = ii < m ? cq[ii] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const long long ii = i + u * bd;
        if (ii < m) {
          cs[ii] = tq[u];
          cq[ii] = ts[u];
        }
      }
    }
    if (tid == 0) {
      const int t = piv[s];
      piv[s] = piv[p];
      piv[p] = t;
    }
  }
  __syncthreads();
  double* col = A + (long long)s * ld;
  double ss = 0.0;
  for (long long i = s + tid; i < m; i += 4 * bd) {
    double x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = i + u * bd < m ? col[i + u * bd] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * bd < m) {
        vbuf[i + u * bd - s] = x[u];
        ss += x[u] * x[u];
      }
  }
  const double sigma2 = wg_sum(ss, red);
  const double sigma = sqrt(sigma2);
  const double x0 = col[s];
  const double alpha = x0 >= 0.0 ? -sigma : sigma;
  const double v0 = x0 - alpha;
  // v^T v = sigma^2 - x0^2 + v0^2 summed as in a direct dot product
  double vv = 0.0;
  for (long long i = s + 1 + tid; i < m; i += 4 * bd) {
    double x[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) x[u] = i + u * bd < m ? vbuf[i + u * bd - s] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * bd < m) vv += x[u] * x[u];
  }
  const double vtv = wg_sum(vv, red) + v0 * v0;
  __syncthreads();
  if (tid == 0) vbuf[0] = v0;
  for (long long i = s + 1 + tid; i < m; i += blockDim.x) col[i] = 0.0;
  if (tid == 0) col[s] = alpha;
  __syncthreads();
  return vtv;
}

// Apply the reflector to columns [j0, j1) (j > s), one wave per column, and
// recompute each column's residual norm over rows s+1 .. m-1.
__device__ void reflect_columns(double* A, long long ld, long long m, int s, int j0, int j1,
                                const double* v, double vtv, double* norms) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  // four rows per lane are loaded together (the stores of one group would
  // otherwise hold back the loads of the next); the sums keep the row order
  for (int j = j0 + wave; j < j1; j += nw) {
    double* col = A + (long long)j * ld;
    double w = 0.0;
    long long i = s + lane;
    for (; i + 192 < m; i += 256) {
      const double c0 = col[i], c1 = col[i + 64], c2 = col[i + 128], c3 = col[i + 192];
      w += v[i - s] * c0;
      w += v[i - s + 64] * c1;
      w += v[i - s + 128] * c2;
      w += v[i - s + 192] * c3;
    }
    for (; i < m; i += 64) w += v[i - s] * col[i];
    w = wave_sum(w);
    const double f = vtv > 0.0 ? 2.0 * w / vtv : 0.0;
    double sq = 0.0;
    i = s + lane;
    for (; i + 192 < m; i += 256) {
      const double c0 = col[i], c1 = col[i + 64], c2 = col[i + 128], c3 = col[i + 192];
      const double x0 = c0 - f * v[i - s], x1 = c1 - f * v[i - s + 64];
      const double x2 = c2 - f * v[i - s + 128], x3 = c3 - f * v[i - s + 192];
      col[i] = x0;
      col[i + 64] = x1;
      col[i + 128] = x2;
      col[i + 192] = x3;
      if (i > s) sq += x0 * x0;
      sq += x1 * x1;
      sq += x2 * x2;
      sq += x3 * x3;
    }
    for (; i < m; i += 64) {
      const double x = col[i] - f * v[i - s];
      col[i] = x;
      if (i > s) sq += x * x;
    }
    sq = wave_sum(sq);
    if (lane == 0) norms[j] = sqrt(sq);
  }
}

// T = R_11^-1 R_12 in place (columns k .. a-1), one thread per column.
__device__ void backsub_columns(double* A, long long ld, int k, int j0, int j1, int stride) {
  for (int j = j0; j < j1; j += stride) {
    double* col = A + (long long)j * ld;
    for (int i = k - 1; i >= 0; --i) {
      double x = col[i];
      for (int l = i + 1; l < k; ++l) x -= A[(long long)l * ld + i] * col[l];
      col[i] = x / A[(long long)i * ld + i];
    }
  }
}

constexpr int CPQR_MAXA = 512;
constexpr int SCHUR_FUSED_MAXA = 128;
constexpr int CPQR_MAXM = 4096;
constexpr int CPQR_BOX_MAXA = 64;

__global__ __launch_bounds__(256) void cpqr_box_kernel(const CpqrJob* __restrict__ jobs,
                                                        double eps, int nprox) {
  __shared__ double norms[CPQR_MAXA];
  __shared__ double v[CPQR_MAXM];
  __shared__ ArgMax red[256];
  __shared__ double redd[8];
  const CpqrJob J = jobs[blockIdx.x];
  const int a = J.a;
  const long long m = (long long)*J.ncnt + nprox;
  const int mn = (int)std::min<long long>(m, a);
  double* A = J.A;
  for (int j = threadIdx.x; j < a; j += blockDim.x) J.piv[j] = j;
  {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j < a; j += 4) {
      double sq = 0.0;
      for (long long i = lane; i < m; i += 64) {
        const double x = A[(long long)j * J.ld + i];
        sq += x * x;
      }
      sq = wave_sum(sq);
      if (lane == 0) norms[j] = sqrt(sq);
    }
  }
  __syncthreads();
  double r11 = 0.0;
  int k = 0;
  for (int s = 0; s < mn; ++s) {
    const ArgMax am = wg_argmax(norms, s, a, red);
    if (s == 0) r11 = am.v;
    if (!(am.v > eps * r11) || am.v == 0.0) break;
    if (threadIdx.x == 0 && am.i != s) norms[am.i] = norms[s];
    const double vtv = householder_step(A, J.ld, m, s, am.i, J.piv, v, redd);
    reflect_columns(A, J.ld, m, s, s + 1, a, v, vtv, norms);
    __syncthreads();
    k = s + 1;
  }
  __syncthreads();
  backsub_columns(A, J.ld, k, k + (int)threadIdx.x, a, blockDim.x);
  if (threadIdx.x == 0) *J.kout = k;
}

// Multi-workgroup path for large boxes: one launch per pivoting step.
__global__ __launch_bounds__(256) void cpqr_big_init_kernel(const CpqrJob* __restrict__ jobs,
                                                             int nprox) {
  const CpqrJob J = jobs[blockIdx.x];
  const long long m = (long long)*J.ncnt + nprox;
  const int j0 = blockIdx.y * 16, j1 = std::min(J.a, j0 + 16);
  if (blockIdx.y == 0 && threadIdx.x == 0) {
    *J.done = 0;
    *J.kout = 0;
  }
  for (int j = j0 + (int)threadIdx.x; j < j1; j += blockDim.x) J.piv[j] = j;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int j = j0 + wave; j < j1; j += 4) {
    double sq = 0.0;
    for (long long i = lane; i < m; i += 64) {
      const double x = J.A[(long long)j * J.ld + i];
      sq += x * x;
    }
    sq = wave_sum(sq);
    if (lane == 0) J.norms[j] = sqrt(sq);
  }
}

__global__ __launch_bounds__(256) void cpqr_big_pivot_kernel(const CpqrJob* __restrict__ jobs,
                                                              int s, double eps, int nprox,
                                                              int* ndone) {
  __shared__ ArgMax red[256];
  __shared__ double redd[8];
  const CpqrJob J = jobs[blockIdx.x];
  if (*J.done) return;
  const long long m = (long long)*J.ncnt + nprox;
  const int mn = (int)std::min<long long>(m, J.a);
  bool finish = s >= mn;
  ArgMax am{0.0, 0};
  if (!finish) {
    am = wg_argmax(J.norms, s, J.a, red);
    if (s == 0 && threadIdx.x == 0) J.scal[1] = am.v;
    __syncthreads();
    const double r11 = (s == 0) ? am.v : J.scal[1];
    finish = !(am.v > eps * r11) || am.v == 0.0;
  }
  if (finish) {
    if (threadIdx.x == 0) {
      *J.kout = s;
      *J.done = 1;
      atomicAdd(ndone, 1);
    }
    return;
  }
  if (threadIdx.x == 0 && am.i != s) J.norms[am.i] = J.norms[s];
  const double vtv = householder_step(J.A, J.ld, m, s, am.i, J.piv, J.v, redd);
  if (threadIdx.x == 0) J.scal[0] = vtv;
}

constexpr int BIG_MAXM = 12288;

// reflect_columns with each column held in registers between the dot product
// and the update (rows s + lane + 64 u, u < R; every row below m - s <= 64 R):
// one read and one write per entry, every load of a column in flight at once,
// and the same operations in the same order.
template <int R>
__device__ void reflect_columns_reg(double* A, long long ld, long long m, int s, int j0, int j1,
                                    const double* v, double vtv, double* norms) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = j0 + wave; j < j1; j += nw) {
    double* col = A + (long long)j * ld;
    double x[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const long long i = s + lane + 64LL * u;
      x[u] = i < m ? col[i] : 0.0;
    }
    double w = 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const long long i = s + lane + 64LL * u;
      if (i < m) w += v[i - s] * x[u];
    }
    w = wave_sum(w);
    const double f = vtv > 0.0 ? 2.0 * w / vtv : 0.0;
    double sq = 0.0;
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const long long i = s + lane + 64LL * u;
      if (i < m) {
        const double y = x[u] - f * v[i - s];
        col[i] = y;
        if (i > s) sq += y * y;
      }
    }
    sq = wave_sum(sq);
    if (lane == 0) norms[j] = sqrt(sq);
  }
}

// One workgroup per cw columns of a box (cw = 4, 8 or 16: levels with few
// boxes take narrow chunks so that one step still spreads over the CUs).
// The reflector is staged in dynamic LDS sized by the level's longest
// compression matrix (so short ones leave room for many workgroups per CU).
// R > 0: the columns' rows below the step stay in registers in boxes where
// they are at most 64 R (taller boxes take the two-pass form).
template <int R>
__global__ __launch_bounds__(256) void cpqr_big_update_kernel(const CpqrJob* __restrict__ jobs,
                                                               int s, int nprox, int cw) {
  extern __shared__ double v[];
  const CpqrJob J = jobs[blockIdx.x];
  if (*J.done) return;
  const int j0 = std::max(s + 1, (int)blockIdx.y * cw), j1 = std::min(J.a, (int)blockIdx.y * cw + cw);
  if (j0 >= j1) return;
  const long long m = (long long)*J.ncnt + nprox;
  for (long long i = s + threadIdx.x; i < m; i += blockDim.x) v[i - s] = J.v[i - s];
  __syncthreads();
  if (R > 0 && m - s <= 64LL * R)
    reflect_columns_reg<(R > 0 ? R : 1)>(J.A, J.ld, m, s, j0, j1, v, J.scal[0], J.norms);
  else
    reflect_columns(J.A, J.ld, m, s, j0, j1, v, J.scal[0], J.norms);
}

// The same for compression matrices taller than BIG_MAXM rows: the reflector
// is read from global memory (it stays in L2 across the columns).
__global__ __launch_bounds__(256) void cpqr_big_update_tall_kernel(const CpqrJob* __restrict__ jobs,
                                                                    int s, int nprox, int cw) {
  const CpqrJob J = jobs[blockIdx.x];
  if (*J.done) return;
  const int j0 = std::max(s + 1, (int)blockIdx.y * cw), j1 = std::min(J.a, (int)blockIdx.y * cw + cw);
  if (j0 >= j1) return;
  const long long m = (long long)*J.ncnt + nprox;
  reflect_columns(J.A, J.ld, m, s, j0, j1, J.v, J.scal[0], J.norms);
}

// T = R_11^-1 R_12 for the multi-workgroup path, by row blocks of at most
// TRSM_ROWS rows solved from the last block up: each diagonal block by
// trsm_upper_kernel, then the rows above it updated by one batched GEMM.
// trsm_upper_kernel solves R X = B in place for an upper triangular kb x kb
// block R (kb <= 256 KQ): one workgroup per eight columns of B, held in
// registers (thread t owns rows t, t + 256, ...), solved right-looking from
// the last row up.  Column i of R is contiguous, so each step reads it
// coalesced; it is fetched one step ahead.
constexpr int TRSM_C = 8;
constexpr int TRSM_ROWS = 2048;
static inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

struct TrsmJob {
  const double* R;  // kb x kb upper triangular, column-major, leading dimension ldr
  long long ldr;
  int kb;
  double* B;  // kb x nc, column-major, leading dimension ldb; overwritten by R^-1 B
  long long ldb;
  int nc;
};

template <int KQ>
__global__ __launch_bounds__(256) void trsm_upper_kernel(const TrsmJob* __restrict__ jobs) {
  __shared__ double xs[2][TRSM_C];
  const TrsmJob J = jobs[blockIdx.x];
  const int k = J.kb, tid = threadIdx.x;
  const int c0 = (int)blockIdx.y * TRSM_C;
  if (k == 0 || c0 >= J.nc) return;
  const int nc = std::min(TRSM_C, J.nc - c0);
  const long long ld = J.ldr;
  const double* A = J.R;
  double* Bc = J.B + (long long)c0 * J.ldb;
  double b[KQ][TRSM_C], rc[KQ];
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    const int r = q * 256 + tid;
#pragma unroll
    for (int c = 0; c < TRSM_C; ++c) b[q][c] = (r < k && c < nc) ? Bc[(long long)c * J.ldb + r] : 0.0;
    rc[q] = (r < k) ? A[(long long)(k - 1) * ld + r] : 0.0;
  }
  int buf = 0;
#pragma unroll
  for (int q = KQ - 1; q >= 0; --q) {
    const int ihi = std::min(k, (q + 1) * 256) - 1;
    for (int i = ihi; i >= q * 256; --i) {
      double rn[KQ];
#pragma unroll
      for (int qq = 0; qq < KQ; ++qq) {
        const int r = qq * 256 + tid;
        rn[qq] = (qq <= q && i > 0 && r < i) ? A[(long long)(i - 1) * ld + r] : 0.0;
      }
      if (tid == (i & 255)) {
        const double d = rc[q];
#pragma unroll
        for (int c = 0; c < TRSM_C; ++c) {
          b[q][c] = b[q][c] / d;
          xs[buf][c] = b[q][c];
        }
      }
      __syncthreads();
      double x[TRSM_C];
#pragma unroll
      for (int c = 0; c < TRSM_C; ++c) x[c] = xs[buf][c];
#pragma unroll
      for (int qq = 0; qq <= q; ++qq) {
        if (qq * 256 + tid < i) {
#pragma unroll
          for (int c = 0; c < TRSM_C; ++c) b[qq][c] -= x[c] * rc[qq];
        }
      }
#pragma unroll
      for (int qq = 0; qq < KQ; ++qq) rc[qq] = rn[qq];
      buf ^= 1;
    }
  }
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    const int r = q * 256 + tid;
#pragma unroll
    for (int c = 0; c < TRSM_C; ++c)
      if (r < k && c < nc) Bc[(long long)c * J.ldb + r] = b[q][c];
  }
}

// T = R_11^-1 R_12 in place for the boxes of a level whose ranks k[i] are
// known on the host: A_i is the box's compression matrix after the pivoted QR
// (leading dimension ld[i], a[i] columns).  Row blocks of rows_per_block rows
// (TRSM_ROWS, or less when a test asks for it) from the last one up.
static void blocked_back_substitution(const std::vector<double*>& A, const std::vector<long long>& ld,
                                      const std::vector<int>& a, const std::vector<int>& k, int rows_per_block,
                                      Scratch& scr, hipStream_t s) {
  const int nb = (int)A.size();
  int rounds = 0;
  for (int i = 0; i < nb; ++i)
    if (k[i] > 0 && a[i] > k[i]) rounds = std::max(rounds, (k[i] + rows_per_block - 1) / rows_per_block);
  for (int step = 0; step < rounds; ++step) {
    std::vector<TrsmJob> jobs;
    std::vector<GemmDesc> upd;
    int kbmax = 0, ncmax = 0;
    for (int i = 0; i < nb; ++i) {
      const int nr = a[i] - k[i];
      if (k[i] == 0 || nr == 0) continue;
      const int nblk = (k[i] + rows_per_block - 1) / rows_per_block;
      if (step >= nblk) continue;
      const int bi = nblk - 1 - step;
      const int r0 = bi * rows_per_block, r1 = std::min(k[i], r0 + rows_per_block);
      double* R12 = A[i] + (long long)k[i] * ld[i];
      jobs.push_back(TrsmJob{A[i] + r0 + (long long)r0 * ld[i], ld[i], r1 - r0, R12 + r0, ld[i], nr});
      kbmax = std::max(kbmax, r1 - r0);
      ncmax = std::max(ncmax, nr);
      // the rows above: R12[0, r0) -= R11[0, r0; r0, r1) X[r0, r1)
      if (r0 > 0)
        upd.push_back(gemm_desc(r0, nr, r1 - r0, -1.0, colmaj(A[i] + (long long)r0 * ld[i], ld[i]),
                                colmaj(R12 + r0, ld[i]), 1.0, colmaj(R12, ld[i])));
    }
    if (jobs.empty()) continue;
    TrsmJob* dj = scr.make<TrsmJob>(jobs.size());
    upload(dj, jobs, s);
    const dim3 g((unsigned)jobs.size(), (unsigned)std::max(1, ceil_div(ncmax, TRSM_C)));
    if (kbmax <= 256)
      hipLaunchKernelGGL(trsm_upper_kernel<1>, g, dim3(256), 0, s, dj);
    else if (kbmax <= 512)
      hipLaunchKernelGGL(trsm_upper_kernel<2>, g, dim3(256), 0, s, dj);
    else if (kbmax <= 1024)
      hipLaunchKernelGGL(trsm_upper_kernel<4>, g, dim3(256), 0, s, dj);
    else
      hipLaunchKernelGGL(trsm_upper_kernel<8>, g, dim3(256), 0, s, dj);
    RSF_HIP(hipGetLastError());
    gemm_batched(upd, scr, s);
  }
}

// ------------------------------------------------------------------ elimination
// Diagonal block of a box in pivot order.  Chol form at a parent: the
// children's X_ss blocks on the diagonal, kernel entries between different
// children; elsewhere kernel entries (the nugget on the diagonal).
struct AsmJob {
  double* A;  // a x a, ld a
  int a, inst;
  const int* act;
  const int* piv;       // nullptr = identity
  int nchild;
  int coff[5];          // child segments of the active list
  const double* xss[4]; // child X_ss (k_c x k_c); nullptr = use kernel entries
  int xld[4];           // leading dimension of each child's X_ss
};

__global__ __launch_bounds__(256) void assemble_kernel(const AsmJob* __restrict__ jobs,
                                                        const KernelParams* __restrict__ kps,
                                                        const double* __restrict__ px,
                                                        const double* __restrict__ py) {
  const AsmJob J = jobs[blockIdx.x];
  const KernelParams kp = kps[J.inst];
  const long long tot = (long long)J.a * J.a;
  for (long long e = blockIdx.y * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.y) {
    const int j = (int)(e / J.a), i = (int)(e - (long long)j * J.a);
    const int u = J.piv ? J.piv[i] : i, w = J.piv ? J.piv[j] : j;
    double val;
    int cu = -1, cw = -1;
    if (J.nchild > 0) {
      for (int c = 0; c < J.nchild; ++c) {
        if (u >= J.coff[c] && u < J.coff[c + 1]) cu = c;
        if (w >= J.coff[c] && w < J.coff[c + 1]) cw = c;
      }
    }
    if (cu >= 0 && cu == cw && J.xss[cu]) {
      val = J.xss[cu][(long long)(w - J.coff[cu]) * J.xld[cu] + (u - J.coff[cu])];
    } else {
      const int p = J.act[u], q = J.act[w];
      val = (p == q) ? kdiag(kp) : kentry(px[p] - px[q], py[p] - py[q], kp);
    }
    J.A[(long long)j * J.a + i] = val;
  }
}

// Block elimination of one box (one workgroup), partition [S, R] of I:
//   X_sr = A_sr - A_ss T,  X_rr = A_rr - T^T X_sr - A_rs T,
//   chol form:  X_rr = L L^T, Linv = L^-1, W = X_sr L^-T, X_ss = A_ss - W W^T,
//               logdet_b = 2 sum log L_jj;
//   mult form:  keep X_sr and X_rr.
struct SchurJob {
  const double* A;    // a x a, ld a
  const double* Tsrc; // T inside the compression matrix (rows 0..k-1, columns k..a-1)
  long long ldts;
  double* T;          // k x r
  double* Xsr;        // k x r
  double* L;          // r x r work (chol) / X_rr output (mult)
  double* Linv;       // r x r (chol)
  double* W;          // k x r (chol)
  double* Xss;        // k x k (chol)
  double* logdet;     // one value
  int* fail;
  int a, k;
};

__global__ __launch_bounds__(256) void schur_kernel(const SchurJob* __restrict__ jobs, int mult) {
  __shared__ double redd[8];
  const SchurJob J = jobs[blockIdx.x];
  const int a = J.a, k = J.k, r = a - k, tid = threadIdx.x, nt = blockDim.x;
  const double* A = J.A;
#define AA(i, j) A[(long long)(j) * a + (i)]
  for (long long e = tid; e < (long long)k * r; e += nt) {
    const int p = (int)(e % k), j = (int)(e / k);
    J.T[e] = J.Tsrc[(long long)(k + j) * J.ldts + p];
  }
  __syncthreads();
  const double* T = J.T;
  for (long long e = tid; e < (long long)k * r; e += nt) {
    const int i = (int)(e % k), j = (int)(e / k);
    double x = AA(i, k + j);
    for (int p = 0; p < k; ++p) x -= AA(i, p) * T[(long long)j * k + p];
    J.Xsr[e] = x;
  }
  __syncthreads();
  for (long long e = tid; e < (long long)r * r; e += nt) {
    const int i = (int)(e % r), j = (int)(e / r);
    if (!mult && i < j) {
      J.L[e] = 0.0;
      continue;
    }
    double x = AA(k + i, k + j);
    for (int p = 0; p < k; ++p)
      x -= T[(long long)i * k + p] * J.Xsr[(long long)j * k + p] + AA(k + i, p) * T[(long long)j * k + p];
    J.L[e] = x;
  }
  __syncthreads();
  if (mult) return;
  double* L = J.L;
  // right-looking Cholesky of the lower triangle
  for (int j = 0; j < r; ++j) {
    const double d = L[(long long)j * r + j];
    if (!(d > 0.0)) {
      if (tid == 0) *J.fail = 1;
      return;
    }
    const double ljj = sqrt(d);
    __syncthreads();
    if (tid == 0) L[(long long)j * r + j] = ljj;
    for (int i = j + 1 + tid; i < r; i += nt) L[(long long)j * r + i] /= ljj;
    __syncthreads();
    const long long rem = r - j - 1;
    for (long long e = tid; e < rem * rem; e += nt) {
      const int ii = j + 1 + (int)(e % rem), ll = j + 1 + (int)(e / rem);
      if (ii >= ll) L[(long long)ll * r + ii] -= L[(long long)j * r + ii] * L[(long long)j * r + ll];
    }
    __syncthreads();
  }
  {
    double ld = 0.0;
    if (tid == 0)
      for (int j = 0; j < r; ++j) ld += log(L[(long long)j * r + j]);
    if (tid == 0) *J.logdet = 2.0 * ld;
  }
  // Linv = L^-1, one column per thread (forward substitution)
  for (int c = tid; c < r; c += nt) {
    double* col = J.Linv + (long long)c * r;
    for (int i = 0; i < c; ++i) col[i] = 0.0;
    col[c] = 1.0 / L[(long long)c * r + c];
    for (int i = c + 1; i < r; ++i) {
      double x = 0.0;
      for (int l = c; l < i; ++l) x -= L[(long long)l * r + i] * col[l];
      col[i] = x / L[(long long)i * r + i];
    }
  }
  __syncthreads();
  // W = X_sr L^-T:  W(i, j) = sum_{l <= j} X_sr(i, l) Linv(j, l)
  for (long long e = tid; e < (long long)k * r; e += nt) {
    const int i = (int)(e % k), j = (int)(e / k);
    double x = 0.0;
    for (int l = 0; l <= j; ++l) x += J.Xsr[(long long)l * k + i] * J.Linv[(long long)l * r + j];
    J.W[e] = x;
  }
  __syncthreads();
  for (long long e = tid; e < (long long)k * k; e += nt) {
    const int i = (int)(e % k), j = (int)(e / k);
    double x = AA(i, j);
    for (int l = 0; l < r; ++l) x -= J.W[(long long)l * k + i] * J.W[(long long)l * k + j];
    J.Xss[e] = x;
  }
#undef AA
}

// S and R lists of each box from its active list and pivots.
struct SplitJob {
  const int* act;
  const int* piv;
  int* S;
  int* R;
  int a, k;
};

__global__ void split_kernel(const SplitJob* __restrict__ jobs) {
  const SplitJob J = jobs[blockIdx.x];
  for (int t = threadIdx.x; t < J.a; t += blockDim.x) {
    const int d = J.act[J.piv[t]];
    if (t < J.k)
      J.S[t] = d;
    else
      J.R[t - J.k] = d;
  }
}

__global__ void triu_zero_kernel(double* A, int N) {
  for (int j = blockIdx.x; j < N; j += gridDim.x)
    for (int i = threadIdx.x; i < j; i += blockDim.x) A[(long long)j * N + i] = 0.0;
}

// ------------------------------------------------------------------ host driver
void build_factor(rsf_factor_s* h, FactorData& F, int mult, hipStream_t s) {
  TraceTag tag(mult ? "factor_rho" : "factor");
  const Tree& t = h->tree;
  const Options& o = h->opt;
  F.mult = mult;
  F.arena.release();
  F.arena.cap = o.mem_cap == 0 ? 0 : std::max<long long>(1, (long long)o.mem_cap - (long long)h->arena.bytes);
  F.levels.assign(t.maxdepth + 1, LevelFactor());
  const int ni = t.ninst;
  F.kp.assign(ni, KernelParams{});
  for (int i = 0; i < ni; ++i) {
    KernelParams& kp = F.kp[i];
    kp.kernel = h->kernel;
    if (h->kernel >= K_MATERN32_ANISO) {
      kp.rho = h->thetas[3 * i];
      kp.rho2 = h->thetas[3 * i + 1];
      kp.sigma2 = 1.0;
    } else {
      kp.rho = h->thetas[3 * i];
      kp.rho2 = 0.0;
      kp.sigma2 = h->thetas[3 * i + 1];
    }
    kp.nugget = h->thetas[3 * i + 2];
    kp.alpha = o.rq_alpha;
    kp.deriv = mult;
    kp.f32 = o.mixed ? 1 : 0;
  }
  F.dkp = F.arena.make<KernelParams>(ni);
  upload(F.dkp, F.kp, s);
  F.logdet.assign(ni, 0.0);
  const int D = t.maxdepth, nprox = o.n_prox;
  Scratch keep(s);  // lives through the whole build: X_ss of the previous level
  std::vector<double*> xss(t.nbox(), nullptr);
  std::vector<int> xld(t.nbox(), 0);
  std::vector<int> kbox(t.nbox(), 0);
  std::vector<const int*> sbox(t.nbox(), nullptr);
  // partial log-determinants in a fixed order, with their instance
  std::vector<double> ld_parts;
  std::vector<int> ld_inst;
  int* fail = keep.make<int>(1);
  RSF_HIP(hipMemsetAsync(fail, 0, sizeof(int), s));
  const bool stats = std::getenv("RSFGP_FACTOR_STATS") != nullptr;
  // Test-only overrides that send small problems down the paths large ones
  // take: the row-block size of the back-substitution T = R_11^-1 R_12 and
  // the height above which a pivoting step reads its reflector from global
  // memory instead of LDS.
  int trsm_rows = TRSM_ROWS, big_maxm = BIG_MAXM;
  if (const char* e = std::getenv("RSFGP_TEST_TRSM_ROWS")) trsm_rows = std::max(1, std::min(TRSM_ROWS, atoi(e)));
  if (const char* e = std::getenv("RSFGP_TEST_BIG_MAXM")) big_maxm = std::max(1, std::min(BIG_MAXM, atoi(e)));

  for (int d = D; d >= 1; --d) {
    Scratch scr(s);
    LevelFactor& L = F.levels[d];
    const int b0 = t.lev[d], b1 = t.lev[d + 1], nb = b1 - b0;
    L.depth = d;
    L.box0 = b0;
    L.nb = nb;
    L.a.assign(nb, 0);
    L.k.assign(nb, 0);
    std::vector<long long> aoff(nb + 1, 0);
    for (int i = 0; i < nb; ++i) {
      const int b = b0 + i;
      int a = 0;
      if (t.leaf[b])
        a = t.count[b];
      else
        for (int c : t.child[b])
          if (c >= 0) a += kbox[c];
      L.a[i] = a;
      aoff[i + 1] = aoff[i] + a;
    }
    // DOF lists of the groups active at this level: the depth-d boxes, then
    // the points of shallower leaves
    std::vector<long long> seg_off;
    std::vector<int> seg_len, seg_owner, seg_box;
    long long tot = aoff[nb];
    for (int i = 0; i < nb; ++i) {
      seg_off.push_back(aoff[i]);
      seg_len.push_back(L.a[i]);
      seg_owner.push_back(b0 + i);
      seg_box.push_back(b0 + i);
    }
    for (int b = 0; b < b0; ++b)
      if (t.leaf[b]) {
        seg_off.push_back(tot);
        seg_len.push_back(t.count[b]);
        seg_owner.push_back(b);
        seg_box.push_back(b);
        tot += t.count[b];
      }
    int* dofs = scr.make<int>(std::max<long long>(tot, 1));
    std::vector<CopySeg> cs;
    for (int i = 0; i < nb; ++i) {
      const int b = b0 + i;
      if (t.leaf[b]) {
        cs.push_back({dofs + aoff[i], nullptr, t.begin[b], t.count[b]});
      } else {
        long long o2 = aoff[i];
        for (int c : t.child[b])
          if (c >= 0 && kbox[c] > 0) {
            cs.push_back({dofs + o2, sbox[c], 0, kbox[c]});
            o2 += kbox[c];
          }
      }
    }
    for (size_t g = nb; g < seg_off.size(); ++g)
      cs.push_back({dofs + seg_off[g], nullptr, t.begin[seg_box[g]], seg_len[g]});
    run_copy_segs(cs, scr, s);
    const int* act = dofs;  // the first aoff[nb] entries

    // candidate groups per box (geometry only, within the box's instance)
    std::vector<std::vector<int>> inst_segs(ni);
    for (size_t g = 0; g < seg_off.size(); ++g) inst_segs[t.inst[seg_box[g]]].push_back((int)g);
    std::vector<int> cand;
    std::vector<NearJob> nj(nb);
    std::vector<long long> mub(nb), kaoff(nb + 1, 0), noff(nb + 1, 0);
    for (int i = 0; i < nb; ++i) {
      const int b = b0 + i;
      const double R = o.r_near * t.half[b];
      nj[i].cx = t.cx[b];
      nj[i].cy = t.cy[b];
      nj[i].r2 = R * R;
      nj[i].owner = b;
      nj[i].cand0 = (int)cand.size();
      long long ub = 0;
      for (int g : inst_segs[t.inst[b]]) {
        const int gb = seg_box[g];
        if (gb == b || seg_len[g] == 0) continue;
        const double dx = std::max(std::fabs(t.cx[gb] - t.cx[b]) - t.half[gb], 0.0);
        const double dy = std::max(std::fabs(t.cy[gb] - t.cy[b]) - t.half[gb], 0.0);
        if (dx * dx + dy * dy < R * R * (1.0 + 1e-12) + 1e-300) {
          cand.push_back((int)g);
          ub += seg_len[g];
        }
      }
      nj[i].cand1 = (int)cand.size();
      noff[i + 1] = noff[i] + ub;
      mub[i] = ub + nprox;
      kaoff[i + 1] = kaoff[i] + mub[i] * L.a[i];
    }
    int* near = scr.make<int>(std::max<long long>(noff[nb], 1));
    int* ncnt = scr.make<int>(nb);
    for (int i = 0; i < nb; ++i) {
      nj[i].out = near + noff[i];
      nj[i].cnt = ncnt + i;
    }
    {
      NearJob* dj = scr.make<NearJob>(nb);
      int* dc = scr.make<int>(std::max<size_t>(cand.size(), 1));
      long long* dso = scr.make<long long>(seg_off.size());
      int* dsl = scr.make<int>(seg_len.size());
      int* dsw = scr.make<int>(seg_owner.size());
      upload(dj, nj, s);
      upload(dc, cand, s);
      upload(dso, seg_off, s);
      upload(dsl, seg_len, s);
      upload(dsw, seg_owner, s);
      hipLaunchKernelGGL(near_kernel, dim3(nb), dim3(256), 0, s, dj, dc, dso, dsl, dsw, dofs, h->px, h->py);
      RSF_HIP(hipGetLastError());
    }
    // compression matrices
    double* Kaux = scr.make<double>(std::max<long long>(kaoff[nb], 1));
    {
      std::vector<KauxJob> kj(nb);
      for (int i = 0; i < nb; ++i) {
        const int b = b0 + i;
        kj[i] = KauxJob{Kaux + kaoff[i], mub[i], L.a[i], t.inst[b], act + aoff[i], near + noff[i], ncnt + i,
                        t.cx[b], t.cy[b], t.half[b]};
      }
      KauxJob* dk = scr.make<KauxJob>(nb);
      upload(dk, kj, s);
      long long maxe = 0;
      for (int i = 0; i < nb; ++i) maxe = std::max(maxe, mub[i] * L.a[i]);
      const int gy = std::max(1, std::min(64, ceil_div(maxe, 256 * 8)));
      hipLaunchKernelGGL(kaux_kernel, dim3(nb, gy), dim3(256), 0, s, dk, F.dkp, h->px, h->py, h->prox_u, nprox);
      RSF_HIP(hipGetLastError());
    }
    // interpolative decompositions
    hipEvent_t ev_id[2] = {nullptr, nullptr};
    if (stats) {
      RSF_HIP(hipEventCreate(&ev_id[0]));
      RSF_HIP(hipEventCreate(&ev_id[1]));
      RSF_HIP(hipEventRecord(ev_id[0], s));
    }
    int* piv = scr.make<int>(std::max<long long>(aoff[nb], 1));
    int* kout = scr.make<int>(nb);
    bool id_big = false, id_tall = false;
    long long n_pivot = 0, n_update = 0;  // pivoting-step launches
    std::vector<int> nh(nb);              // exact row counts (big form)
    {
      int maxa = 0;
      long long maxm = 0;
      for (int i = 0; i < nb; ++i) {
        maxa = std::max(maxa, L.a[i]);
        maxm = std::max(maxm, mub[i]);
      }
      std::vector<CpqrJob> cj(nb);
      // one workgroup per box only for the smallest boxes; larger ones (or
      // few boxes) spread every pivoting step over many workgroups
      const bool big = (maxa > CPQR_BOX_MAXA || maxm > CPQR_MAXM || nb < 128);
      id_big = big;
      double* norms = big ? scr.make<double>(std::max<long long>(aoff[nb], 1)) : nullptr;
      double* vb = big ? scr.make<double>(std::max<long long>(noff[nb] + (long long)nb * nprox, 1)) : nullptr;
      double* scal = big ? scr.make<double>(2 * nb) : nullptr;
      int* done = big ? scr.make<int>(nb + 1) : nullptr;
      for (int i = 0; i < nb; ++i) {
        cj[i] = CpqrJob{Kaux + kaoff[i], mub[i], L.a[i], ncnt + i, piv + aoff[i], kout + i,
                        big ? norms + aoff[i] : nullptr, big ? vb + noff[i] + (long long)i * nprox : nullptr,
                        big ? scal + 2 * i : nullptr, big ? done + i : nullptr};
      }
      CpqrJob* dj = scr.make<CpqrJob>(nb);
      upload(dj, cj, s);
      if (!big) {
        hipLaunchKernelGGL(cpqr_box_kernel, dim3(nb), dim3(256), 0, s, dj, h->eps, nprox);
        RSF_HIP(hipGetLastError());
      } else {
        int* ndone = done + nb;
        RSF_HIP(hipMemsetAsync(ndone, 0, sizeof(int), s));
        // exact row counts (the near field is compacted on the device)
        RSF_HIP(hipMemcpyAsync(nh.data(), ncnt, nb * sizeof(int), hipMemcpyDeviceToHost, s));
        RSF_HIP(hipStreamSynchronize(s));
        maxm = 0;
        for (int i = 0; i < nb; ++i) maxm = std::max<long long>(maxm, (long long)nh[i] + nprox);
        static bool upd_lds = false;
        if (!upd_lds) {
          for (const void* kf : {(const void*)cpqr_big_update_kernel<16>,
                                 (const void*)cpqr_big_update_kernel<32>, (const void*)cpqr_big_update_kernel<48>,
                                 (const void*)cpqr_big_update_kernel<64>, (const void*)cpqr_big_update_kernel<80>,
                                 (const void*)cpqr_big_update_kernel<96>})
            RSF_HIP(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, BIG_MAXM * (int)sizeof(double)));
          upd_lds = true;
        }
        if (stats) {
          long long sm = 0;
          for (int i = 0; i < nb; ++i) sm += nh[i] + nprox;
          fprintf(stderr, "[factor%s] depth %d rows mean %.0f max %lld\n", mult ? "_rho" : "", d, (double)sm / nb, maxm);
        }
        const int chunks = std::max(1, ceil_div(maxa, 16));
        hipLaunchKernelGGL(cpqr_big_init_kernel, dim3(nb, chunks), dim3(256), 0, s, dj, nprox);
        RSF_HIP(hipGetLastError());
        int cw = 16;
        while (cw > 4 && (long long)nb * ceil_div(maxa, cw) < 2048) cw /= 2;
        const int ucols = ceil_div(maxa, cw);
        long long steps = 0;
        for (int i = 0; i < nb; ++i) steps = std::max<long long>(steps, std::min<long long>((long long)nh[i] + nprox, L.a[i]));
        for (int st = 0; st <= steps; ++st) {
          hipLaunchKernelGGL(cpqr_big_pivot_kernel, dim3(nb), dim3(256), 0, s, dj, st, h->eps, nprox, ndone);
          RSF_HIP(hipGetLastError());
          ++n_pivot;
          if (st == steps) break;
          ++n_update;
          id_tall = maxm > big_maxm;
          if (maxm <= big_maxm) {
            // the register form for the shortest bucket that holds the rows below
            // the step (the largest bucket when none does: taller boxes fall back)
            const long long below = maxm - st;
            const dim3 ug(nb, ucols);
            const size_t lds = (size_t)maxm * sizeof(double);
#define RSF_UPD(RV) hipLaunchKernelGGL(cpqr_big_update_kernel<RV>, ug, dim3(256), lds, s, dj, st, nprox, cw)
            if (below <= 64 * 16)
              RSF_UPD(16);
            else if (below <= 64 * 32)
              RSF_UPD(32);
            else if (below <= 64 * 48)
              RSF_UPD(48);
            else if (below <= 64 * 64)
              RSF_UPD(64);
            else if (below <= 64 * 80)
              RSF_UPD(80);
            else
              RSF_UPD(96);
#undef RSF_UPD
          } else
            hipLaunchKernelGGL(cpqr_big_update_tall_kernel, dim3(nb, ucols), dim3(256), 0, s, dj, st, nprox, cw);
          RSF_HIP(hipGetLastError());
          if ((st & 15) == 15) {
            int nd = 0;
            RSF_HIP(hipMemcpyAsync(&nd, ndone, sizeof(int), hipMemcpyDeviceToHost, s));
            RSF_HIP(hipStreamSynchronize(s));
            if (nd >= nb) break;
          }
        }
      }
    }
    std::vector<int> kh(nb);
    RSF_HIP(hipMemcpyAsync(kh.data(), kout, nb * sizeof(int), hipMemcpyDeviceToHost, s));
    int fh = 0;
    RSF_HIP(hipMemcpyAsync(&fh, fail, sizeof(int), hipMemcpyDeviceToHost, s));
    RSF_HIP(hipStreamSynchronize(s));
    RSF_CHECK(fh == 0, RSF_E_NOT_SPD, "redundant block not positive definite at depth " + std::to_string(d + 1));
    {
      // algorithmic work of the pivoting steps: step s of a box with m rows
      // and a columns reads and writes the trailing (m - s) x (a - s - 1)
      // block once (a dot product, an update and the recomputed norm: 6 flops
      // and 16 bytes per entry)
      double fl = 0.0, by = 0.0;
      for (int i = 0; i < nb; ++i) {
        // sum over s < k of (m - s)(a - 1 - s), k <= min(m, a)
        const double m = id_big ? (double)nh[i] + nprox : (double)mub[i], v = L.a[i] - 1.0, k = kh[i];
        const double e = k * m * v - (m + v) * k * (k - 1.0) / 2.0 + (k - 1.0) * k * (2.0 * k - 1.0) / 6.0;
        fl += 6.0 * e;
        by += 16.0 * e;
      }
      if (!id_big) {
        trace_kernel_work("cpqr_box_kernel", fl, by);
      } else {
        trace_kernel_work(id_tall ? "cpqr_big_update_tall_kernel" : "cpqr_big_update_kernel", fl, by, (double)n_update);
        trace_kernel_work("cpqr_big_pivot_kernel", 0.0, 0.0, (double)n_pivot);
      }
    }
    if (id_big) {
      // T = R_11^-1 R_12 with the ranks now on the host
      std::vector<double*> Ab(nb);
      for (int i = 0; i < nb; ++i) Ab[i] = Kaux + kaoff[i];
      blocked_back_substitution(Ab, mub, L.a, kh, trsm_rows, scr, s);
    }
    if (stats) {
      RSF_HIP(hipEventRecord(ev_id[1], s));
      RSF_HIP(hipEventSynchronize(ev_id[1]));
      float ms = 0.f;
      RSF_HIP(hipEventElapsedTime(&ms, ev_id[0], ev_id[1]));
      RSF_HIP(hipEventDestroy(ev_id[0]));
      RSF_HIP(hipEventDestroy(ev_id[1]));
      long long sa = 0, sm = 0, sk = 0, ma = 0, mm = 0, mk = 0;
      for (int i = 0; i < nb; ++i) {
        sa += L.a[i];
        sm += mub[i];
        sk += kh[i];
        ma = std::max<long long>(ma, L.a[i]);
        mm = std::max<long long>(mm, mub[i]);
        mk = std::max<long long>(mk, kh[i]);
      }
      fprintf(stderr, "[factor%s] depth %d boxes %d a mean %.0f max %lld  m<= mean %.0f max %lld  k mean %.0f max %lld  ID %.2f ms\n",
              mult ? "_rho" : "", d, nb, (double)sa / nb, ma, (double)sm / nb, mm, (double)sk / nb, mk, ms);
    }
    // factor storage
    L.k = kh;
    L.s_off.assign(nb + 1, 0);
    L.r_off.assign(nb + 1, 0);
    L.t_off.assign(nb + 1, 0);
    L.l_off.assign(nb + 1, 0);
    for (int i = 0; i < nb; ++i) {
      const long long k = kh[i], r = L.a[i] - kh[i];
      RSF_CHECK(k >= 0 && r >= 0, RSF_E_HIP, "bad rank from the ID kernel");
      L.s_off[i + 1] = L.s_off[i] + k;
      L.r_off[i + 1] = L.r_off[i] + r;
      L.t_off[i + 1] = L.t_off[i] + k * r;
      L.l_off[i + 1] = L.l_off[i] + r * r;
      L.max_k = std::max<int>(L.max_k, (int)k);
      L.max_r = std::max<int>(L.max_r, (int)r);
    }
    L.total_s = L.s_off[nb];
    L.total_r = L.r_off[nb];
    L.total_t = L.t_off[nb];
    L.total_l = L.l_off[nb];
    {
      std::vector<BoxRec> br(nb);
      for (int i = 0; i < nb; ++i)
        br[i] = BoxRec{kh[i], L.a[i] - kh[i], L.s_off[i], L.r_off[i], L.t_off[i], L.l_off[i]};
      L.box = F.arena.make<BoxRec>(std::max(nb, 1));
      upload(L.box, br, s);
    }
    L.S = F.arena.make<int>(std::max<long long>(L.total_s, 1));
    L.R = F.arena.make<int>(std::max<long long>(L.total_r, 1));
    L.T = F.arena.make<double>(std::max<long long>(L.total_t, 1));
    L.W = F.arena.make<double>(std::max<long long>(L.total_t, 1));
    L.Lm = F.arena.make<double>(std::max<long long>(L.total_l, 1));
    {
      std::vector<SplitJob> sj(nb);
      for (int i = 0; i < nb; ++i)
        sj[i] = SplitJob{act + aoff[i], piv + aoff[i], L.S + L.s_off[i], L.R + L.r_off[i], L.a[i], kh[i]};
      SplitJob* dj = scr.make<SplitJob>(nb);
      upload(dj, sj, s);
      hipLaunchKernelGGL(split_kernel, dim3(nb), dim3(256), 0, s, dj);
      RSF_HIP(hipGetLastError());
    }
    // diagonal blocks and elimination
    std::vector<long long> a2off(nb + 1, 0), k2off(nb + 1, 0);
    for (int i = 0; i < nb; ++i) {
      a2off[i + 1] = a2off[i] + (long long)L.a[i] * L.a[i];
      k2off[i + 1] = k2off[i] + (long long)kh[i] * kh[i];
    }
    double* Ablk = scr.make<double>(std::max<long long>(a2off[nb], 1));
    {
      std::vector<AsmJob> aj(nb);
      long long maxe = 1;
      for (int i = 0; i < nb; ++i) {
        const int b = b0 + i;
        AsmJob& J = aj[i];
        J.A = Ablk + a2off[i];
        J.a = L.a[i];
        J.inst = t.inst[b];
        J.act = act + aoff[i];
        J.piv = piv + aoff[i];
        J.nchild = 0;
        J.coff[0] = 0;
        if (!t.leaf[b]) {
          for (int c : t.child[b])
            if (c >= 0) {
              J.xss[J.nchild] = mult ? nullptr : xss[c];
              J.xld[J.nchild] = xld[c];
              J.coff[J.nchild + 1] = J.coff[J.nchild] + kbox[c];
              J.nchild++;
            }
        }
        maxe = std::max(maxe, (long long)J.a * J.a);
      }
      AsmJob* dj = scr.make<AsmJob>(nb);
      upload(dj, aj, s);
      const int gy = std::max(1, std::min(64, ceil_div(maxe, 256 * 8)));
      hipLaunchKernelGGL(assemble_kernel, dim3(nb, gy), dim3(256), 0, s, dj, F.dkp, h->px, h->py);
      RSF_HIP(hipGetLastError());
    }
    int maxa = 0;
    for (int i = 0; i < nb; ++i) maxa = std::max(maxa, L.a[i]);
    if (!mult) L.Lf = F.arena.make<double>(std::max<long long>(L.total_l, 1));
    // Ablk lives on (in `keep`) when the parent reads X_ss from it
    // mixed precision takes every level through the GEMM path, whose products run in FP32
    const bool gemm_path = maxa > SCHUR_FUSED_MAXA || o.mixed;
    if (!gemm_path) {
      double* Xsr = mult ? L.W : scr.make<double>(std::max<long long>(L.total_t, 1));
      double* Lw = mult ? L.Lm : L.Lf;
      double* Xss = mult ? nullptr : keep.make<double>(std::max<long long>(k2off[nb], 1));
      double* ldp = scr.make<double>(nb);
      fill_zero(ldp, nb, s);
      std::vector<SchurJob> sj(nb);
      for (int i = 0; i < nb; ++i) {
        sj[i] = SchurJob{Ablk + a2off[i], Kaux + kaoff[i], mub[i], L.T + L.t_off[i], Xsr + L.t_off[i],
                         Lw + L.l_off[i], mult ? nullptr : L.Lm + L.l_off[i], mult ? nullptr : L.W + L.t_off[i],
                         mult ? nullptr : Xss + k2off[i], ldp + i, fail, L.a[i], kh[i]};
      }
      SchurJob* dj = scr.make<SchurJob>(nb);
      upload(dj, sj, s);
      hipLaunchKernelGGL(schur_kernel, dim3(nb), dim3(256), 0, s, dj, mult);
      RSF_HIP(hipGetLastError());
      if (!mult) {
        std::vector<double> lh(nb);
        RSF_HIP(hipMemcpyAsync(lh.data(), ldp, nb * sizeof(double), hipMemcpyDeviceToHost, s));
        RSF_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < nb; ++i) {
          ld_parts.push_back(lh[i]);
          ld_inst.push_back(t.inst[b0 + i]);
        }
      }
      for (int i = 0; i < nb; ++i) {
        xss[b0 + i] = mult ? nullptr : Xss + k2off[i];
        xld[b0 + i] = kh[i];
      }
    } else {
      // the same elimination as matrix-core GEMMs batched over the boxes, in
      // place in the assembled blocks A = [A_ss A_sr; A_rs A_rr]
      double* Akeep = keep.make<double>(std::max<long long>(a2off[nb], 1));
      copy_dev(Akeep, Ablk, a2off[nb], s);
      std::vector<CopyBlock> tc;
      std::vector<GemmDesc> g1, g2, g3;
      for (int i = 0; i < nb; ++i) {
        const int a = L.a[i], k = kh[i], r = a - k;
        double* A = Akeep + a2off[i];
        double* T = L.T + L.t_off[i];
        tc.push_back(CopyBlock{Kaux + kaoff[i] + (long long)k * mub[i], mub[i], T, k, k, r, 0});
        g1.push_back(gemm_desc(k, r, k, -1.0, colmaj(A, a), colmaj(T, k), 1.0, colmaj(A + (long long)k * a, a)));
        GemmDesc d2 = gemm_desc(r, r, k, -1.0, colmajT(T, k), colmaj(A + (long long)k * a, a), 1.0,
                                colmaj(A + (long long)k * a + k, a));
        GemmDesc d3 = gemm_desc(r, r, k, -1.0, colmaj(A + k, a), colmaj(T, k), 1.0, colmaj(A + (long long)k * a + k, a));
        d2.lower = d3.lower = !mult;
        g1.back().f32 = d2.f32 = d3.f32 = o.mixed;
        g2.push_back(d2);
        g3.push_back(d3);
      }
      copy_blocks(tc, scr, s);
      gemm_batched(g1, scr, s);
      gemm_batched(g2, scr, s);
      gemm_batched(g3, scr, s);
      if (mult) {
        std::vector<CopyBlock> cp;
        for (int i = 0; i < nb; ++i) {
          const int a = L.a[i], k = kh[i], r = a - k;
          double* A = Akeep + a2off[i];
          cp.push_back(CopyBlock{A + (long long)k * a, a, L.W + L.t_off[i], k, k, r, 0});
          cp.push_back(CopyBlock{A + (long long)k * a + k, a, L.Lm + L.l_off[i], r, r, r, 0});
        }
        copy_blocks(cp, scr, s);
      } else {
        std::vector<CholProblem> cps;
        std::vector<long long> lo(nb + 1, 0);
        for (int i = 0; i < nb; ++i) lo[i + 1] = lo[i] + (L.a[i] - kh[i] + 63) / 64;
        double* logd = scr.make<double>(std::max<long long>(lo[nb], 1));
        fill_zero(logd, lo[nb], s);
        for (int i = 0; i < nb; ++i) {
          const int a = L.a[i], k = kh[i], r = a - k;
          cps.push_back(CholProblem{Akeep + a2off[i] + (long long)k * a + k, a, r, L.Lm + L.l_off[i], r, logd + lo[i]});
        }
        batched_chol_inv(cps, fail, scr, s);
        std::vector<CopyBlock> cp;
        std::vector<GemmDesc> gw, gx;
        for (int i = 0; i < nb; ++i) {
          const int a = L.a[i], k = kh[i], r = a - k;
          double* A = Akeep + a2off[i];
          cp.push_back(CopyBlock{A + (long long)k * a + k, a, L.Lf + L.l_off[i], r, r, r, 1});
          gw.push_back(gemm_desc(k, r, r, 1.0, colmaj(A + (long long)k * a, a), colmajT(L.Lm + L.l_off[i], r), 0.0,
                                 colmaj(L.W + L.t_off[i], k)));
          gx.push_back(gemm_desc(k, k, r, -1.0, colmaj(L.W + L.t_off[i], k), colmajT(L.W + L.t_off[i], k), 1.0,
                                 colmaj(A, a)));
        }
        copy_blocks(cp, scr, s);
        for (GemmDesc& g : gw) g.f32 = o.mixed;
        for (GemmDesc& g : gx) g.f32 = o.mixed;
        gemm_batched(gw, scr, s);
        gemm_batched(gx, scr, s);
        std::vector<double> lh(lo[nb]);
        if (!lh.empty()) RSF_HIP(hipMemcpyAsync(lh.data(), logd, lh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        RSF_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < nb; ++i)
          for (long long q = lo[i]; q < lo[i + 1]; ++q) {
            ld_parts.push_back(lh[q]);
            ld_inst.push_back(t.inst[b0 + i]);
          }
      }
      for (int i = 0; i < nb; ++i) {
        xss[b0 + i] = mult ? nullptr : Akeep + a2off[i];
        xld[b0 + i] = L.a[i];
      }
    }
    for (int i = 0; i < nb; ++i) {
      const int b = b0 + i;
      kbox[b] = kh[i];
      sbox[b] = L.S + L.s_off[i];
    }
  }
  // roots: the remaining DOFs of each instance's top box, factored together
  {
    Scratch scr(s);
    std::vector<CopySeg> cs;
    std::vector<AsmJob> aj;
    F.roots.assign(ni, RootBlock{});
    int N = 0;
    for (int i = 0; i < ni; ++i) {
      const int b = i;  // the depth-0 boxes are the instances' roots
      RootBlock& rb = F.roots[i];
      rb.off = N;
      AsmJob J{};
      J.nchild = 0;
      J.coff[0] = 0;
      J.inst = i;
      if (t.leaf[b]) {
        rb.N = t.count[b];
      } else {
        for (int c : t.child[b])
          if (c >= 0) {
            J.xss[J.nchild] = mult ? nullptr : xss[c];
            J.xld[J.nchild] = xld[c];
            J.coff[J.nchild + 1] = J.coff[J.nchild] + kbox[c];
            J.nchild++;
            rb.N += kbox[c];
          }
      }
      N += rb.N;
      if (rb.N > 0) {
        J.a = rb.N;
        J.piv = nullptr;
        aj.push_back(J);
      }
    }
    F.nroot = N;
    F.root_idx = F.arena.make<int>(std::max(N, 1));
    for (int i = 0; i < ni; ++i) {
      const int b = i;
      RootBlock& rb = F.roots[i];
      if (t.leaf[b]) {
        if (rb.N > 0) cs.push_back({F.root_idx + rb.off, nullptr, t.begin[b], rb.N});
      } else {
        int o2 = rb.off;
        for (int c : t.child[b])
          if (c >= 0 && kbox[c] > 0) {
            cs.push_back({F.root_idx + o2, sbox[c], 0, kbox[c]});
            o2 += kbox[c];
          }
      }
    }
    run_copy_segs(cs, scr, s);
    if (!aj.empty()) {
      long long maxe = 1;
      std::vector<CholProblem> cp;
      std::vector<long long> lo(1, 0);
      std::vector<int> lo_inst;
      for (AsmJob& J : aj) {
        RootBlock& rb = F.roots[J.inst];
        rb.L = F.arena.make<double>((size_t)rb.N * rb.N);
        J.A = rb.L;
        J.act = F.root_idx + rb.off;
        maxe = std::max(maxe, (long long)rb.N * rb.N);
        if (!mult) {
          rb.Linv = F.arena.make<double>((size_t)rb.N * rb.N);
          lo.push_back(lo.back() + (rb.N + 63) / 64);
          lo_inst.push_back(J.inst);
        }
      }
      AsmJob* dj = scr.make<AsmJob>(aj.size());
      upload(dj, aj, s);
      const int gy = std::max(1, std::min(1024, ceil_div(maxe, 256 * 8)));
      hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)aj.size(), gy), dim3(256), 0, s, dj, F.dkp, h->px, h->py);
      RSF_HIP(hipGetLastError());
      if (!mult) {
        double* logd = scr.make<double>(std::max<long long>(lo.back(), 1));
        fill_zero(logd, lo.back(), s);
        for (size_t q = 0; q < aj.size(); ++q) {
          RootBlock& rb = F.roots[aj[q].inst];
          cp.push_back(CholProblem{rb.L, rb.N, rb.N, rb.Linv, rb.N, logd + lo[q]});
        }
        batched_chol_inv(cp, fail, scr, s);
        std::vector<double> lh(lo.back());
        int fh = 0;
        RSF_HIP(hipMemcpyAsync(lh.data(), logd, lh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        RSF_HIP(hipMemcpyAsync(&fh, fail, sizeof(int), hipMemcpyDeviceToHost, s));
        RSF_HIP(hipStreamSynchronize(s));
        RSF_CHECK(fh == 0, RSF_E_NOT_SPD, "covariance factor lost positive definiteness (root or a redundant block)");
        for (size_t q = 0; q < aj.size(); ++q) {
          const RootBlock& rb = F.roots[aj[q].inst];
          hipLaunchKernelGGL(triu_zero_kernel, dim3(std::min(rb.N, 4096)), dim3(256), 0, s, rb.L, rb.N);
          RSF_HIP(hipGetLastError());
          for (long long u = lo[q]; u < lo[q + 1]; ++u) {
            ld_parts.push_back(lh[u]);
            ld_inst.push_back(lo_inst[q]);
          }
        }
      }
    }
  }
  if (!mult) {
    for (size_t q = 0; q < ld_parts.size(); ++q) F.logdet[ld_inst[q]] += ld_parts[q];
  }
}

}  // namespace rsf
