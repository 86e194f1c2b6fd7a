// Sweeps over the skeletonization factors (Section 2.4 of the paper): F^-1,
// F^(1/2), (F^(1/2))^T and the multiply-only product with the derivative
// operator.  Vectors are row-major panels in tree order (row = DOF), so each
// box's S and R rows are gathered / scattered through index maps inside one
// batched matrix-core GEMM per step and level.
#include "rsf.h"

namespace rsf {

__global__ void to_panel_kernel(const int* __restrict__ perm, long long n, const double* __restrict__ src,
                                long long ld, double* __restrict__ P, int nc, long long ldp) {
  const long long tot = n * nc;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
    const long long t = e / nc;
    const int c = (int)(e - t * nc);
    P[t * ldp + c] = src[(long long)perm[t] + c * ld];
  }
}

__global__ void from_panel_kernel(const int* __restrict__ perm, long long n, const double* __restrict__ P,
                                  int nc, long long ldp, double* __restrict__ dst, long long ld) {
  const long long tot = n * nc;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
    const long long t = e / nc;
    const int c = (int)(e - t * nc);
    dst[(long long)perm[t] + c * ld] = P[t * ldp + c];
  }
}

static unsigned grid_for(long long tot) {
  long long b = (tot + 255) / 256;
  return (unsigned)std::max<long long>(1, std::min<long long>(b, 8192));
}

void to_panel(const rsf_factor_s* h, const double* src, long long ld, double* P, int nc, long long ldp,
              hipStream_t s) {
  hipLaunchKernelGGL(to_panel_kernel, dim3(grid_for(h->tree.n * nc)), dim3(256), 0, s, h->perm, h->tree.n,
                     src, ld, P, nc, ldp);
  RSF_HIP(hipGetLastError());
}

void from_panel(const rsf_factor_s* h, const double* P, int nc, long long ldp, double* dst, long long ld,
                hipStream_t s) {
  hipLaunchKernelGGL(from_panel_kernel, dim3(grid_for(h->tree.n * nc)), dim3(256), 0, s, h->perm, h->tree.n,
                     P, nc, ldp, dst, ld);
  RSF_HIP(hipGetLastError());
}

// X[rows[q], :] = Tmp[q, :] for q < nrows
__global__ void scatter_rows_kernel(const int* __restrict__ rows, long long nrows, const double* __restrict__ Tmp,
                                    int nc, double* __restrict__ X, long long ld) {
  const long long tot = nrows * nc;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
    const long long q = e / nc;
    const int c = (int)(e - q * nc);
    X[(long long)rows[q] * ld + c] = Tmp[q * nc + c];
  }
}

static void scatter_rows(const int* rows, long long nrows, const double* Tmp, int nc, double* X, long long ld,
                         hipStream_t s) {
  if (nrows <= 0 || nc <= 0) return;
  hipLaunchKernelGGL(scatter_rows_kernel, dim3(grid_for(nrows * nc)), dim3(256), 0, s, rows, nrows, Tmp, nc,
                     X, ld);
  RSF_HIP(hipGetLastError());
}

// One batched GEMM over the boxes of a level:
//   C_b = alpha op(A_b) B_b + beta C_b
// with A_b a per-box dense block and B_b / C_b row sets of panels.
enum Rows { RS, RR, RTMP };

template <class AFn>
static void level_gemm(const LevelFactor& L, int nc, double alpha, AFn afn, Rows brows, const double* Bp,
                       long long ldb, double beta, Rows crows, double* Cp, long long ldc, Scratch& scr,
                       hipStream_t s) {
  std::vector<GemmDesc> g;
  g.reserve(L.nb);
  for (int i = 0; i < L.nb; ++i) {
    const int k = L.k[i], r = L.a[i] - L.k[i];
    int M, K;
    Mat A = afn(i, k, r, M, K);
    if (M == 0 || K == 0) {
      if (beta == 1.0 || M == 0) continue;
    }
    auto rowsel = [&](Rows w, const double* P, long long ld) -> Mat {
      if (w == RS) return panel(P, ld, L.S + L.s_off[i]);
      if (w == RR) return panel(P, ld, L.R + L.r_off[i]);
      return panel(P + L.r_off[i] * nc, nc);
    };
    g.push_back(gemm_desc(M, nc, K, alpha, A, rowsel(brows, Bp, ldb), beta, rowsel(crows, Cp, ldc)));
  }
  gemm_batched(g, scr, s);
}

void sweep_solve(const rsf_factor_s* h, const FactorData& F, double* X, int nc, long long ld, Scratch& scr,
                 hipStream_t s) {
  TraceTag tag("sweep_solve");
  const int D = h->tree.maxdepth;
  long long maxr = 1;
  for (int d = 1; d <= D; ++d) maxr = std::max(maxr, F.levels[d].total_r);
  maxr = std::max<long long>(maxr, F.nroot);
  double* tmp = scr.make<double>((size_t)maxr * nc);
  for (int d = D; d >= 1; --d) {
    const LevelFactor& L = F.levels[d];
    // X_R -= T^T X_S
    level_gemm(L, nc, -1.0, [&](int i, int k, int r, int& M, int& K) { M = r; K = k; return colmajT(L.T + L.t_off[i], k); },
               RS, X, ld, 1.0, RR, X, ld, scr, s);
    // tmp = L^-1 X_R
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = r; K = r; return colmaj(L.Lm + L.l_off[i], r); },
               RR, X, ld, 0.0, RTMP, tmp, nc, scr, s);
    // X_S -= W tmp
    level_gemm(L, nc, -1.0, [&](int i, int k, int r, int& M, int& K) { M = k; K = r; return colmaj(L.W + L.t_off[i], k); },
               RTMP, tmp, nc, 1.0, RS, X, ld, scr, s);
    scatter_rows(L.R, L.total_r, tmp, nc, X, ld, s);
  }
  if (F.nroot > 0) {
    const int N = F.nroot;
    std::vector<GemmDesc> g1{gemm_desc(N, nc, N, 1.0, colmaj(F.Lroot_inv, N), panel(X, ld, F.root_idx), 0.0,
                                       panel(tmp, nc))};
    gemm_batched(g1, scr, s);
    std::vector<GemmDesc> g2{gemm_desc(N, nc, N, 1.0, colmajT(F.Lroot_inv, N), panel(tmp, nc), 0.0,
                                       panel(X, ld, F.root_idx))};
    gemm_batched(g2, scr, s);
  }
  for (int d = 1; d <= D; ++d) {
    const LevelFactor& L = F.levels[d];
    // X_R -= W^T X_S
    level_gemm(L, nc, -1.0, [&](int i, int k, int r, int& M, int& K) { M = r; K = k; return colmajT(L.W + L.t_off[i], k); },
               RS, X, ld, 1.0, RR, X, ld, scr, s);
    // tmp = L^-T X_R
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = r; K = r; return colmajT(L.Lm + L.l_off[i], r); },
               RR, X, ld, 0.0, RTMP, tmp, nc, scr, s);
    scatter_rows(L.R, L.total_r, tmp, nc, X, ld, s);
    // X_S -= T tmp
    level_gemm(L, nc, -1.0, [&](int i, int k, int r, int& M, int& K) { M = k; K = r; return colmaj(L.T + L.t_off[i], k); },
               RTMP, tmp, nc, 1.0, RS, X, ld, scr, s);
  }
}

void sweep_sqrt_t(const rsf_factor_s* h, const FactorData& F, double* X, double* Out, int nc, long long ld,
                  Scratch& scr, hipStream_t s) {
  TraceTag tag("sweep_sqrt");
  const int D = h->tree.maxdepth;
  for (int d = D; d >= 1; --d) {
    const LevelFactor& L = F.levels[d];
    // X_S += T X_R
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = k; K = r; return colmaj(L.T + L.t_off[i], k); },
               RR, X, ld, 1.0, RS, X, ld, scr, s);
    // Out_R = L^T X_R + W^T X_S
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = r; K = r; return colmajT(L.Lf + L.l_off[i], r); },
               RR, X, ld, 0.0, RR, Out, ld, scr, s);
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = r; K = k; return colmajT(L.W + L.t_off[i], k); },
               RS, X, ld, 1.0, RR, Out, ld, scr, s);
  }
  if (F.nroot > 0) {
    const int N = F.nroot;
    std::vector<GemmDesc> g{gemm_desc(N, nc, N, 1.0, colmajT(F.Lroot, N), panel(X, ld, F.root_idx), 0.0,
                                      panel(Out, ld, F.root_idx))};
    gemm_batched(g, scr, s);
  }
}

void sweep_sqrt(const rsf_factor_s* h, const FactorData& F, const double* Y, double* V, int nc, long long ld,
                Scratch& scr, hipStream_t s) {
  TraceTag tag("sweep_sqrt");
  const int D = h->tree.maxdepth;
  for (int d = D; d >= 1; --d) {
    const LevelFactor& L = F.levels[d];
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = r; K = r; return colmaj(L.Lf + L.l_off[i], r); },
               RR, Y, ld, 0.0, RR, V, ld, scr, s);
  }
  if (F.nroot > 0) {
    const int N = F.nroot;
    std::vector<GemmDesc> g{gemm_desc(N, nc, N, 1.0, colmaj(F.Lroot, N), panel(Y, ld, F.root_idx), 0.0,
                                      panel(V, ld, F.root_idx))};
    gemm_batched(g, scr, s);
  }
  for (int d = 1; d <= D; ++d) {
    const LevelFactor& L = F.levels[d];
    // V_S += W Y_R
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = k; K = r; return colmaj(L.W + L.t_off[i], k); },
               RR, Y, ld, 1.0, RS, V, ld, scr, s);
    // V_R += T^T V_S
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = r; K = k; return colmajT(L.T + L.t_off[i], k); },
               RS, V, ld, 1.0, RR, V, ld, scr, s);
  }
}

void sweep_apply_mult(const rsf_factor_s* h, const FactorData& F, double* X, double* Y, int nc, long long ld,
                      Scratch& scr, hipStream_t s) {
  TraceTag tag("sweep_mult");
  const int D = h->tree.maxdepth;
  fill_zero(Y, h->tree.n * ld, s);
  for (int d = D; d >= 1; --d) {
    const LevelFactor& L = F.levels[d];
    // X_S += T X_R
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = k; K = r; return colmaj(L.T + L.t_off[i], k); },
               RR, X, ld, 1.0, RS, X, ld, scr, s);
    // Y_R += X_rr X_R + X_sr^T X_S
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = r; K = r; return colmaj(L.Lm + L.l_off[i], r); },
               RR, X, ld, 1.0, RR, Y, ld, scr, s);
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = r; K = k; return colmajT(L.W + L.t_off[i], k); },
               RS, X, ld, 1.0, RR, Y, ld, scr, s);
  }
  if (F.nroot > 0) {
    const int N = F.nroot;
    std::vector<GemmDesc> g{gemm_desc(N, nc, N, 1.0, colmaj(F.Aroot, N), panel(X, ld, F.root_idx), 1.0,
                                      panel(Y, ld, F.root_idx))};
    gemm_batched(g, scr, s);
  }
  for (int d = 1; d <= D; ++d) {
    const LevelFactor& L = F.levels[d];
    // Y_S += X_sr X_R  (after the coarser levels' L operators)
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = k; K = r; return colmaj(L.W + L.t_off[i], k); },
               RR, X, ld, 1.0, RS, Y, ld, scr, s);
    // Y_R += T^T Y_S
    level_gemm(L, nc, 1.0, [&](int i, int k, int r, int& M, int& K) { M = r; K = k; return colmajT(L.T + L.t_off[i], k); },
               RS, Y, ld, 1.0, RR, Y, ld, scr, s);
  }
}

}  // namespace rsf
