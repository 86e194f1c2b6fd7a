// Score equations (eq. gradient; Algorithm 1) on top of the factorizations,
// with the traces taken by matrix peeling for weakly admissible operators
// (Section 3.2):
//   per quadtree level, Gaussian probes restricted to the boxes of one
//   quadrant, one multi-column product with the operator (the sweeps), the
//   coarser levels' low-rank blocks subtracted, and a randomized low-rank
//   approximation (eq. lowrankapprox) of every sibling block; at the leaves the
//   diagonal blocks are extracted and their traces summed (Section 3.2.4).
// Section 3 allows any symmetric operator with the trace of F^-1 F_rho: with
// F^-1 = B^T B (the two halves of the solve sweep), B B^T (trace Tr F^-1) and
// B F_rho B^T (trace Tr F^-1 F_rho) are peeled together from the same probes
// and share the product B^T W, so one probe block costs one and a half solve
// sweeps and one multiply sweep.
#include <algorithm>
#include <chrono>
#include <exception>
#include <thread>
#include <cstdio>
#include <cstdlib>
#include <cmath>

#include "rsf.h"

namespace rsf {

// ------------------------------------------------------------------ Philox4x32-10
// Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): ten rounds of two 32-bit multiply-hi/lo mixes with a Weyl key
// schedule.  Counter (dof, column, level, stream), key = the 64-bit seed.
__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

// Standard normal by Box-Muller from two 53-bit uniforms in (0, 1).
__device__ __forceinline__ double probe_normal(uint32_t d, uint32_t j, uint32_t level, uint32_t stream,
                                               uint64_t seed) {
  uint32_t c[4] = {d, j, level, stream};
  philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t a = (((uint64_t)c[0] << 32) | c[1]) >> 11;
  const uint64_t b = (((uint64_t)c[2] << 32) | c[3]) >> 11;
  const double u1 = ((double)a + 0.5) * 0x1.0p-53;
  const double u2 = ((double)b + 0.5) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Probe columns of one chunk for the DOFs of the nodes peeled at `level`
// (qd[d] = the column block of d's node: its quadrant in the weak form, its
// colour in the strong form; -1 for rows without one): for t < act[i] (i =
// instance of d),
//   W[d, ncol t + q(d)] = Om[d, j0[i] + t] = N(d, j0[i] + t, level, stream),
// W is zero elsewhere.  W interleaves the ncol column blocks (column
// ncol t + q), so every instance's active columns form a prefix of the panel;
// with qmajor (one instance) the blocks are contiguous instead (column
// q ncw + t).
__device__ __forceinline__ long long probe_col(int t, int q, int ncol, int ncw, int qmajor) {
  return qmajor ? (long long)q * ncw + t : (long long)ncol * t + q;
}
__global__ void probe_kernel(const int* __restrict__ qd, const int* __restrict__ rinst, const int* __restrict__ act,
                             const int* __restrict__ j0, long long n, int ncw, int ncol, int qmajor, int level,
                             uint32_t stream, uint64_t seed, double* __restrict__ W, double* __restrict__ Om,
                             long long ldo) {
  const long long tot = n * ncw;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
    const long long d = e / ncw;
    const int t = (int)(e - d * ncw);
    const int q = qd[d];
    if (q < 0) continue;
    const int i = rinst[d];
    if (t >= act[i]) continue;
    const double v = probe_normal((uint32_t)d, (uint32_t)(j0[i] + t), (uint32_t)level, stream, seed);
    W[d * (long long)ncol * ncw + probe_col(t, q, ncol, ncw, qmajor)] = v;
    Om[d * ldo + j0[i] + t] = v;
  }
}

// Y[d, q * C + j0[i] + t] = B[d, column of (t, q)] for the rows of the nodes
// peeled at this level and t < act[i] (i = instance of d).
__global__ void store_samples_kernel(const int* __restrict__ qd, const int* __restrict__ rinst,
                                     const int* __restrict__ act, const int* __restrict__ j0, long long n, int ncw,
                                     int ncol, int qmajor, int C, const double* __restrict__ B, double* __restrict__ Y) {
  const long long w = (long long)ncol * ncw;
  const long long tot = n * w;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
    const long long d = e / w;
    const int c = (int)(e - d * w);
    if (qd[d] < 0) continue;
    const int i = rinst[d];
    const int t = qmajor ? c % ncw : c / ncol, q = qmajor ? c / ncw : c - (c / ncol) * ncol;
    if (t >= act[i]) continue;
    Y[d * (long long)ncol * C + (long long)q * C + j0[i] + t] = B[e];
  }
}

// dst[d, q * Cd + t] = src[d, q * Cs + t] for t < cols, q < nq
__global__ void regrid_kernel(long long n, int nq, int cols, const double* __restrict__ src, int Cs,
                              double* __restrict__ dst, int Cd) {
  const long long tot = n * nq * (long long)cols;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
    const long long d = e / ((long long)nq * cols);
    const int c = (int)(e - d * nq * (long long)cols);
    const int q = c / cols, t = c - q * cols;
    dst[d * (long long)nq * Cd + (long long)q * Cd + t] = src[d * (long long)nq * Cs + (long long)q * Cs + t];
  }
}

// E[begin_b + t, col0_b + t] = 1 for every leaf b and t < count_b (E: ld
// columns; col0 null: every leaf's block starts at column 0)
__global__ void eye_blocks_kernel(const int* __restrict__ lbeg, const int* __restrict__ lcnt,
                                  const int* __restrict__ lcol0, int nleaf, double* __restrict__ E, int ld) {
  const int b = blockIdx.x;
  if (b >= nleaf) return;
  const int c0 = lcol0 ? lcol0[b] : 0;
  for (int t = threadIdx.x; t < lcnt[b]; t += blockDim.x) E[(long long)(lbeg[b] + t) * ld + c0 + t] = 1.0;
}

// sum over leaves b and t < count_b of H[begin_b + t, col0_b + t], in a fixed order
__global__ __launch_bounds__(256) void leaf_trace_kernel(const int* __restrict__ lbeg, const int* __restrict__ lcnt,
                                                          const int* __restrict__ lcol0, int nleaf,
                                                          const double* __restrict__ H, int ld, double* out) {
  __shared__ double part[256];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nleaf; b += 256) {
    double s = 0.0;
    const int c0 = lcol0 ? lcol0[b] : 0;
    for (int t = 0; t < lcnt[b]; ++t) s += H[(long long)(lbeg[b] + t) * ld + c0 + t];
    acc += s;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

// ------------------------------------------------------------------ pivoted Cholesky of the sample Gram matrices
// The range finder of the low-rank step needs, for each sample block Y, the
// column pivots and the numerical rank of column-pivoted QR of Y.  Pivoted
// Cholesky of the Gram matrix G = Y^T Y picks the same pivots in exact
// arithmetic (the residual diagonal is the squared residual column norm) and
// stops when the largest residual diagonal is <= tol^2 times the first pivot's.
// Blocked right-looking form: one launch factors up to NB further columns of
// every unfinished Gram matrix in one workgroup (the panel lives in registers,
// one row per thread and panel column), then the trailing matrix takes
// Gw -= Lp Lp^T as a batched matrix-core GEMM.  Rows are never swapped: the
// panel and the residual diagonal stay indexed by the original column, and a
// row that has been chosen as pivot is marked in the residual diagonal.
struct PpanelJob {
  const double* Gw;  // c x c (ld c), the Gram matrix minus the previous panels' products (lower triangle)
  double* d;         // c residual diagonal; PIV_DONE marks chosen rows
  double* Lp;        // c x NB panel (ld c): this launch's columns of the factor
  int* piv;          // c pivots in order
  int* state;        // [0] columns factored so far, [1] finished
  double* d1;        // residual of the first pivot
  int c;
};

constexpr int PCHOL_MAXN = 4096;
constexpr int PCHOL_WG = 1024;
constexpr double PIV_DONE = -1.0e300;

template <int RPT, int NB, int WGS>
__global__ __launch_bounds__(WGS) void ppanel_kernel(const PpanelJob* __restrict__ jobs, double tol2) {
  __shared__ double wv[WGS / 64];
  __shared__ int wi[WGS / 64];
  __shared__ double lp[NB];
  __shared__ double sel_v;
  __shared__ int sel_i;
  const PpanelJob J = jobs[blockIdx.x];
  if (J.state[1]) return;
  const int c = J.c, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int s0 = J.state[0];
  double d1 = *J.d1;
  // dl: residual diagonal of the thread's rows; lr: their panel entries, zero
  // in the columns not yet formed, so the full-width dot below sums only the
  // previous columns and no register array is indexed at run time
  double dl[RPT];
  double lr[RPT][NB];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + r * WGS;
    dl[r] = i < c ? J.d[i] : PIV_DONE;
#pragma unroll
    for (int t = 0; t < NB; ++t) lr[r][t] = 0.0;
  }
  if (tid < NB) lp[tid] = 0.0;
  int steps = 0;
  bool fin = false;
#pragma unroll 1
  for (int j = 0; j < NB && !fin; ++j) {
    // largest residual diagonal among unchosen rows, ties to the lowest index
    double bv = 0.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + r * WGS;
      if (dl[r] != PIV_DONE && (bi == 0x7fffffff || dl[r] > bv)) {
        bv = dl[r];
        bi = i;
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double v2 = __shfl_xor(bv, o, 64);
      const int i2 = __shfl_xor(bi, o, 64);
      if (i2 != 0x7fffffff && (bi == 0x7fffffff || v2 > bv || (v2 == bv && i2 < bi))) {
        bv = v2;
        bi = i2;
      }
    }
    if (lane == 0) {
      wv[wid] = bv;
      wi[wid] = bi;
    }
    __syncthreads();
    if (wid == 0) {
      bv = lane < WGS / 64 ? wv[lane] : 0.0;
      bi = lane < WGS / 64 ? wi[lane] : 0x7fffffff;
#pragma unroll
      for (int o = 8; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(bv, o, 64);
        const int i2 = __shfl_xor(bi, o, 64);
        if (i2 != 0x7fffffff && (bi == 0x7fffffff || v2 > bv || (v2 == bv && i2 < bi))) {
          bv = v2;
          bi = i2;
        }
      }
      if (lane == 0) {
        sel_v = bv;
        sel_i = bi;
      }
    }
    __syncthreads();
    const double dp = sel_v;
    const int p = sel_i;
    if (s0 + j == 0 && p != 0x7fffffff) d1 = dp;
    if (p == 0x7fffffff || !(dp > 0.0) || !(dp > tol2 * d1)) {
      fin = true;
      break;
    }
    // the pivot row's entries of this panel's earlier columns
    if (tid == (p & (WGS - 1))) {
#pragma unroll
      for (int r = 0; r < RPT; ++r)
        if (r == p / WGS) {
#pragma unroll
          for (int t = 0; t < NB; ++t) lp[t] = lr[r][t];
        }
    }
    __syncthreads();
    const double lss = sqrt(dp);
    // column p of the symmetric matrix from its lower triangle: rows below p
    // down the column, rows above p along row p
    const double* Gp = J.Gw + (long long)p * c;
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + r * WGS;
      double x = 0.0;
      if (i == p) {
        x = lss;
        dl[r] = PIV_DONE;
      } else if (dl[r] != PIV_DONE) {
        double a0 = i > p ? Gp[i] : J.Gw[(long long)i * c + p], a1 = 0.0;
#pragma unroll
        for (int t = 0; t < NB; t += 2) {
          a0 -= lr[r][t] * lp[t];
          a1 -= lr[r][t + 1] * lp[t + 1];
        }
        x = (a0 + a1) / lss;
        dl[r] -= x * x;
      }
#pragma unroll
      for (int t = 0; t < NB; ++t)
        if (t == j) lr[r][t] = x;
    }
    if (tid == 0) J.piv[s0 + j] = p;
    steps = j + 1;
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + r * WGS;
    if (i < c) {
      J.d[i] = dl[r];
#pragma unroll
      for (int t = 0; t < NB; ++t) J.Lp[(long long)t * c + i] = lr[r][t];
    }
  }
  if (tid == 0) {
    J.state[0] = s0 + steps;
    if (fin) J.state[1] = 1;
    if (s0 == 0) *J.d1 = d1;
  }
}

// d_e(i) = Gw_e(i, i); state and d1 cleared (one workgroup per job)
__global__ void ppanel_init_kernel(const PpanelJob* __restrict__ jobs) {
  const PpanelJob J = jobs[blockIdx.x];
  for (int i = threadIdx.x; i < J.c; i += blockDim.x) J.d[i] = J.Gw[(long long)i * J.c + i];
  if (threadIdx.x == 0) {
    J.state[0] = 0;
    J.state[1] = 0;
    *J.d1 = 0.0;
  }
}

// out(u, j) = Y(u, piv[j]) for u < cnt, j < k: the pivot columns of a sample
// block (row-major rows of ld doubles) as a column-major cnt x k matrix.
struct GatherColsJob {
  const double* Y;
  long long ld;
  const int* piv;
  int k, cnt;
  double* out;
};
__global__ void gather_cols_kernel(const GatherColsJob* __restrict__ jobs) {
  const GatherColsJob J = jobs[blockIdx.y];
  const long long tot = (long long)J.k * J.cnt;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
    const long long u = e / J.k;
    const int j = (int)(e - u * J.k);
    J.out[(long long)j * J.cnt + u] = J.Y[u * J.ld + J.piv[j]];
  }
}

// ------------------------------------------------------------------ host side
static unsigned grid_of(long long tot) {
  return (unsigned)std::max<long long>(1, std::min<long long>((tot + 255) / 256, 8192));
}

namespace {

constexpr int OVERSAMPLE = 10;
// device memory for the work panels of one chunk of probe columns, for the
// Gram matrices of one chunk of sample blocks and for the bases and core
// matrices of one chunk of sibling pairs
constexpr long long PEEL_CHUNK_BYTES = 24LL << 30;
constexpr long long GRAM_CHUNK_BYTES = 8LL << 30;
constexpr long long LOWRANK_CHUNK_BYTES = 8LL << 30;
constexpr long long SUB_CHUNK_BYTES = 4LL << 30;
// nodes of at least this many rows on average take the per-node subtraction
// that skips their own quadrant's columns
constexpr int SPLIT_MIN_ROWS = 128;
constexpr int FIRST_COLS = 64;
constexpr int MIN_COLS = 24;

int round8(int c) { return (c + 7) / 8 * 8; }

long long isqrt(long long n) {
  long long r = (long long)std::sqrt((double)n);
  while (r * r > n) --r;
  while ((r + 1) * (r + 1) <= n) ++r;
  return r;
}

// Probe columns at the first peeled level: sibling blocks of the top level
// have ranks that grow like sqrt(n) (Section 3.3), so start at 9/4 sqrt(n), at
// least FIRST_COLS.
int first_cols(long long n) { return round8((int)std::max<long long>(FIRST_COLS, 9 * isqrt(n) / 4)); }

// Probe columns at the next level from the largest rank found at the level
// above, plus the oversampling, at least MIN_COLS, rounded up to a multiple
// of 8: the second peeled level's sibling blocks of B F_rho B^T and B B^T
// have larger ranks than the first level's (1.5x); the third level's shrink
// by up to 0.65x (0.7x), later levels' by at most 0.5x (0.6x).
int next_cols(int prev_rank, int peeled) {
  int c;
  if (peeled == 1)
    c = (3 * prev_rank + 1) / 2;
  else if (peeled == 2)
    c = (7 * prev_rank + 9) / 10;
  else
    c = (3 * prev_rank + 4) / 5;
  return round8(std::max(MIN_COLS, c + OVERSAMPLE));
}

// Growth when some block's rank is not resolved: 1.5x, at least the rank
// found plus twice the oversampling.
int grow_cols(int total, int maxrank) { return round8(std::max((3 * total + 1) / 2, maxrank + 2 * OVERSAMPLE)); }

}  // namespace
namespace {

struct PairLR {
  int i, j;     // box ids (i before j in sibling order)
  int k1 = 0, k2 = 0;
  double* M = nullptr;  // k1 x k2, column-major
};

// Low-rank blocks of one level for one operator.
struct LevelLR {
  bool any = false;
  std::vector<int> boxes;                // boxes of this level that are in some pair
  std::vector<int> K;                    // per box: total basis columns
  std::vector<double*> U;                // per box: count_b x K_b, column-major
  std::vector<std::vector<int>> koff;    // per box: offset of the basis for each pair entry
  std::vector<PairLR> pairs;
  // per pair: position of the pair's bases inside U_i and U_j
  std::vector<int> off_i, off_j, pos_i, pos_j;
};

// ---- geometry of the strongly admissible format
// Integer cell coordinates of every box at its own depth (each instance's
// root at (0, 0); a child at quadrant q of (X, Y) is (2X + [q east],
// 2Y + [q north])), so that touching squares are decided exactly.
struct Cells {
  std::vector<long long> X, Y;
};

Cells cell_coords(const Tree& t) {
  Cells c;
  c.X.assign(t.nbox(), 0);
  c.Y.assign(t.nbox(), 0);
  for (int b = 0; b < t.nbox(); ++b) {  // parents precede children in box order
    const int p = t.parent[b], q = t.quad[b];
    if (p < 0) continue;
    c.X[b] = 2 * c.X[p] + ((q == 1 || q == 3) ? 1 : 0);
    c.Y[b] = 2 * c.Y[p] + ((q == 0 || q == 1) ? 1 : 0);
  }
  return c;
}

// the closed squares of boxes a and b intersect (boxes of one instance)
bool touch(const Tree& t, const Cells& c, int a, int b) {
  if (t.inst[a] != t.inst[b]) return false;
  const int D = std::max(t.depth[a], t.depth[b]);
  const long long sa = 1LL << (D - t.depth[a]), sb = 1LL << (D - t.depth[b]);
  return c.X[a] * sa <= (c.X[b] + 1) * sb && c.X[b] * sb <= (c.X[a] + 1) * sa && c.Y[a] * sa <= (c.Y[b] + 1) * sb &&
         c.Y[b] * sb <= (c.Y[a] + 1) * sa;
}

// Smallest colour not taken by an already coloured conflicting node, in node order.
std::vector<int> greedy_colors(const std::vector<int>& nodes, const std::vector<std::vector<int>>& conflicts,
                               const std::vector<int>& pos) {
  std::vector<int> col(nodes.size(), -1);
  std::vector<char> used;
  for (size_t a = 0; a < nodes.size(); ++a) {
    used.assign(conflicts[a].size() + 1, 0);
    for (int b : conflicts[a]) {
      const int k = col[pos[b]];
      if (k >= 0 && k < (int)used.size()) used[k] = 1;
    }
    int k = 0;
    while (used[k]) ++k;
    col[a] = k;
  }
  return col;
}

// The strongly admissible structure of one level: nodes (boxes of depth lev
// and leaves of smaller depth, in box order), their colours for the probes
// (nodes whose parent nodes both touch the parent node of some node get
// different colours) and the admissible pairs (nodes that do not touch while
// their parent nodes touch).  A depth-lev box's parent node is its parent; a
// leaf carried down is its own parent node.
struct StrongLevel {
  std::vector<int> nodes, color;  // color: per box id (-1: not a node)
  int ncol = 0;
  std::vector<std::pair<int, int>> pairs;
};

StrongLevel strong_level(const Tree& t, const Cells& cells, int lev) {
  StrongLevel L;
  const int nbx = t.nbox();
  std::vector<int> pos(nbx, -1), par;
  for (int b = 0; b < nbx; ++b)
    if (t.depth[b] == lev || (t.leaf[b] && t.depth[b] < lev)) {
      pos[b] = (int)L.nodes.size();
      L.nodes.push_back(b);
      par.push_back(t.depth[b] == lev ? t.parent[b] : b);
    }
  L.color.assign(nbx, -1);
  const int nn = (int)L.nodes.size();
  if (nn == 0) return L;
  // distinct parent nodes, the nodes under each, and which parents touch
  std::vector<int> plist(par);
  std::sort(plist.begin(), plist.end());
  plist.erase(std::unique(plist.begin(), plist.end()), plist.end());
  std::vector<int> ppos(nbx, -1);
  for (size_t a = 0; a < plist.size(); ++a) ppos[plist[a]] = (int)a;
  std::vector<std::vector<int>> under(plist.size());
  for (int a = 0; a < nn; ++a) under[ppos[par[a]]].push_back(L.nodes[a]);
  std::vector<std::vector<int>> near(plist.size());
  for (size_t a = 0; a < plist.size(); ++a)
    for (size_t c = 0; c < plist.size(); ++c)
      if (touch(t, cells, plist[a], plist[c])) near[a].push_back((int)c);
  // conflicts: the nodes of one window (every node under a parent touching p)
  std::vector<std::vector<int>> conf(nn);
  for (size_t a = 0; a < plist.size(); ++a) {
    std::vector<int> win;
    for (int c : near[a]) win.insert(win.end(), under[c].begin(), under[c].end());
    for (int b : win)
      for (int b2 : win)
        if (b2 != b) conf[pos[b]].push_back(b2);
  }
  const std::vector<int> col = greedy_colors(L.nodes, conf, pos);
  for (int a = 0; a < nn; ++a) {
    L.color[L.nodes[a]] = col[a];
    L.ncol = std::max(L.ncol, col[a] + 1);
  }
  // admissible pairs (i before j in node order)
  for (int a = 0; a < nn; ++a) {
    const int i = L.nodes[a];
    for (int c : near[ppos[par[a]]])
      for (int j : under[c])
        if (pos[j] > a && !touch(t, cells, i, j)) L.pairs.emplace_back(i, j);
  }
  std::sort(L.pairs.begin(), L.pairs.end(), [&](const std::pair<int, int>& x, const std::pair<int, int>& y) {
    return std::make_pair(pos[x.first], pos[x.second]) < std::make_pair(pos[y.first], pos[y.second]);
  });
  return L;
}

// Colours of the leaves with no two touching leaves alike (the extraction of
// the diagonal blocks in the strong form); returns the number of colours.
int leaf_colors(const Tree& t, const Cells& cells, const std::vector<int>& leaves, std::vector<int>& col) {
  std::vector<int> pos(t.nbox(), -1);
  for (size_t a = 0; a < leaves.size(); ++a) pos[leaves[a]] = (int)a;
  std::vector<std::vector<int>> conf(leaves.size());
  for (size_t a = 0; a < leaves.size(); ++a)
    for (size_t c = a + 1; c < leaves.size(); ++c)
      if (touch(t, cells, leaves[a], leaves[c])) {
        conf[a].push_back(leaves[c]);
        conf[c].push_back(leaves[a]);
      }
  col = greedy_colors(leaves, conf, pos);
  int nc = 0;
  for (int k : col) nc = std::max(nc, k + 1);
  return nc;
}

// Probe counts of the strong form: 64 at the first level with admissible
// blocks; then the largest rank found at the level above plus the
// oversampling (the ranks of separated blocks change little between levels).
constexpr int FIRST_COLS_STRONG = 64;
int next_cols_strong(int prev_rank) { return round8(std::max(MIN_COLS, prev_rank + OVERSAMPLE)); }

struct Peeler {
  // per-phase wall times (host clock around the enqueue and its waits), for
  // RSFGP_PEEL_TIMES diagnostics
  double tm[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const rsf_factor_s* h;
  const Tree& t;
  hipStream_t s;
  Arena store;  // low-rank blocks of every level
  // operator 0 is B B^T; operator k >= 1 is B F_k B^T with F_k = Fd[k - 1]
  static constexpr int MAXOP = 3;
  std::vector<LevelLR> lr[MAXOP];
  const FactorData* Fd[MAXOP - 1];  // the derivative factorizations
  int nop;
  bool strong = false;  // strongly admissible format (else weakly admissible)
  Peeler(const rsf_factor_s* hh, const FactorData* const* fd, int nd, hipStream_t ss, bool strong_form = false)
      : h(hh), t(hh->tree), s(ss), nop(1 + nd), strong(strong_form) {
    RSF_CHECK(nd >= 1 && nd <= MAXOP - 1, RSF_E_INVALID, "peeling takes one or two derivative factorizations");
    for (int k = 0; k < nd; ++k) Fd[k] = fd[k];
  }

  // out[op] = G_op X for every operator (X row-major n x nc); X is preserved.
  // cols (host, per instance, or null): the leading columns each instance's
  // rows take part in.
  void apply_ops(const double* X, int nc, double* const* out, Scratch& scr, const int* cols) {
    const long long n = t.n, sz = n * nc;
    double* H = scr.make<double>(sz);
    copy_dev(H, X, sz, s);
    sweep_half_down(h, h->F, H, nc, nc, scr, s, cols);  // B^T X
    copy_dev(out[0], H, sz, s);
    double* H2 = nullptr;
    if (nop == 3) {
      H2 = scr.make<double>(sz);
      copy_dev(H2, H, sz, s);
    }
    // B B^T X (and B F_2 B^T X) beside F_1 B^T X and B F_1 B^T X: the sweeps
    // are independent and each leaves part of the GPU idle
    beside(
        [&](hipStream_t s2) {
          Scratch sc2(s2);
          sweep_half_up(h, h->F, out[0], nc, nc, sc2, s2, cols);  // B B^T X
          if (nop == 3) {
            sweep_apply_mult(h, *Fd[1], H2, out[2], nc, nc, sc2, s2, cols);  // F_2 B^T X (H2 is consumed)
            sweep_half_up(h, h->F, out[2], nc, nc, sc2, s2, cols);           // B F_2 B^T X
          }
        },
        [&] {
          sweep_apply_mult(h, *Fd[0], H, out[1], nc, nc, scr, s, cols);  // F_1 B^T X (H is consumed)
          sweep_half_up(h, h->F, out[1], nc, nc, scr, s, cols);          // B F_1 B^T X
        });
  }

  // Runs side(s2) on the library's side stream from a second host thread
  // while here() runs on s; the side work starts after everything already
  // enqueued on s, and s waits for it before this returns.
  template <class SideFn, class HereFn>
  void beside(SideFn side, HereFn here) {
    hipStream_t s2 = side_stream();
    hipEvent_t fork = nullptr, done = nullptr;
    RSF_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    RSF_HIP(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    RSF_HIP(hipEventRecord(fork, s));
    RSF_HIP(hipStreamWaitEvent(s2, fork, 0));
    std::exception_ptr err;
    std::thread th([&] {
      try {
        side(s2);
        RSF_HIP(hipEventRecord(done, s2));
      } catch (...) {
        err = std::current_exception();
      }
    });
    try {
      here();
    } catch (...) {
      th.join();
      (void)hipStreamSynchronize(s2);
      (void)hipEventDestroy(fork);
      (void)hipEventDestroy(done);
      throw;
    }
    th.join();
    if (err) {
      (void)hipStreamSynchronize(s2);
      (void)hipEventDestroy(fork);
      (void)hipEventDestroy(done);
      std::rethrow_exception(err);
    }
    RSF_HIP(hipStreamWaitEvent(s, done, 0));
    (void)hipEventDestroy(fork);
    (void)hipEventDestroy(done);
  }

  int cols_of(const int* cols, int box, int nc) const { return cols ? std::min(nc, cols[t.inst[box]]) : nc; }

  // Probes of one chunk in compact form: row d holds its own column block's
  // columns, Om[d * ldo + j0[instance] + t] = X[d, ncol t + qd[d]] (qd: the
  // column block of d's node at the level being peeled, -1 for rows without
  // one; ncol blocks).
  struct CompactProbes {
    const double* Om;
    long long ldo;
    const std::vector<int>* j0;
    const std::vector<int>* qd;
    int ncol;
    int qmajor;                      // column blocks contiguous (q ncw + t) rather than interleaved
    int lev;                         // the level being peeled
    const std::vector<int>* qbox;    // column block of every node peeled at lev (-1 elsewhere)
  };

  // out -= sum_{m < upto} G^(m) X  for operator op (same column rule as apply_ops).
  // With cp, X is a probe chunk and U_b^T X[I_b] is formed per column block
  // from the rows of that block only (the other rows are zero in its columns).
  // The coarser levels' products U_b^T X and M (U^T X) are kept for a slice of
  // the columns at a time, sized so that both stay within SUB_CHUNK_BYTES (the
  // strong form's boxes carry bases for up to 27 partners).
  void subtract_lowrank(int op, int upto, const double* X, int nc, double* out, Scratch& scr, const int* cols,
                        const CompactProbes* cp = nullptr, hipStream_t st = nullptr) {
    if (!st) st = s;
    // phase "peel_subtract/<level being peeled>" (L = the leaf extraction)
    const std::string tname = std::string("peel_subtract/") + (cp ? std::to_string(cp->lev) : std::string("L"));
    TraceTag tag(tname.c_str());
    const int unit = cp ? cp->ncol : 1;
    // the level's nodes in tree order (their rows are contiguous): with
    // contiguous quadrant blocks and nodes of at least SPLIT_MIN_ROWS rows on
    // average, the last product is split per node (see below)
    std::vector<int> lbeg, lnode;
    bool split = false;
    if (cp && cp->qmajor) {
      long long rows = 0;
      for (int b = 0; b < t.nbox(); ++b)
        if ((*cp->qbox)[b] >= 0) {
          lbeg.push_back(t.begin[b]);
          lnode.push_back(b);
          rows += t.count[b];
        }
      std::vector<int> ord(lbeg.size());
      for (size_t u = 0; u < ord.size(); ++u) ord[u] = (int)u;
      std::sort(ord.begin(), ord.end(), [&](int x, int y) { return lbeg[x] < lbeg[y]; });
      std::vector<int> b2(ord.size()), n2(ord.size());
      for (size_t u = 0; u < ord.size(); ++u) {
        b2[u] = lbeg[ord[u]];
        n2[u] = lnode[ord[u]];
      }
      lbeg.swap(b2);
      lnode.swap(n2);
      split = !lnode.empty() && rows >= (long long)SPLIT_MIN_ROWS * (long long)lnode.size();
    }
    for (int m = 1; m < upto && m < (int)lr[op].size(); ++m) {
      const LevelLR& L = lr[op][m];
      if (!L.any) continue;
      const int nbx = (int)L.boxes.size();
      long long ksum = 0;
      for (int b = 0; b < nbx; ++b) ksum += L.K[b];
      if (ksum == 0) continue;
      int w = (int)std::min<long long>(nc, std::max<long long>(unit, SUB_CHUNK_BYTES / (16 * ksum) / unit * unit));
      // contiguous quadrant blocks are kept whole (one slice)
      if (cp && cp->qmajor) w = nc;
      // rows of each box by column block (box-relative), for the compact probes
      std::vector<int> rows;
      std::vector<long long> lo;
      int* drows = nullptr;
      if (cp) {
        const std::vector<int>& qd = *cp->qd;
        const int ncol = cp->ncol;
        lo.assign((long long)ncol * nbx + 1, 0);
        std::vector<std::vector<int>> byq(ncol);
        for (int b = 0; b < nbx; ++b) {
          const int box = L.boxes[b], b0 = t.begin[box], cnt = t.count[box];
          for (auto& v : byq) v.clear();
          for (int u = 0; u < cnt; ++u)
            if (qd[b0 + u] >= 0) byq[qd[b0 + u]].push_back(u);
          for (int q = 0; q < ncol; ++q) {
            rows.insert(rows.end(), byq[q].begin(), byq[q].end());
            lo[(long long)ncol * b + q + 1] = (long long)rows.size();
          }
        }
        drows = scr.make<int>(std::max<size_t>(rows.size(), 1));
        upload(drows, rows, st);
      }
      std::vector<long long> poff(nbx + 1, 0);
      for (int b = 0; b < nbx; ++b) poff[b + 1] = poff[b] + (long long)L.K[b] * w;
      double* P = scr.make<double>(std::max<long long>(poff[nbx], 1));
      double* Q = scr.make<double>(std::max<long long>(poff[nbx], 1));
      for (int c0 = 0; c0 < nc; c0 += w) {
        const int wc = std::min(w, nc - c0);
        // columns of this slice each box takes part in
        auto cols_in = [&](int box) { return std::max(0, std::min(wc, cols_of(cols, box, nc) - c0)); };
        // a pair with one empty basis contributes nothing: its Q segment stays zero
        fill_zero(Q, poff[nbx], st);
        std::vector<GemmDesc> g1;
        if (!cp) {
          for (int b = 0; b < nbx; ++b) {
            const int box = L.boxes[b];
            g1.push_back(gemm_desc(L.K[b], cols_in(box), t.count[box], 1.0, colmajT(L.U[b], t.count[box]),
                                   panel(X + (long long)t.begin[box] * nc + c0, nc), 0.0, panel(P + poff[b], w)));
          }
        } else {
          // a block whose rows form one run is passed as a contiguous block;
          // column blocks without rows in a box leave their columns of P zero
          const int ncol = cp->ncol;
          fill_zero(P, poff[nbx], st);
          for (int b = 0; b < nbx; ++b) {
            const int box = L.boxes[b], cnt = t.count[box];
            const int N = cols_in(box) / ncol;
            if (N == 0) continue;
            const double* Ob = cp->Om + (long long)t.begin[box] * cp->ldo + (*cp->j0)[t.inst[box]] + c0 / ncol;
            for (int q = 0; q < ncol; ++q) {
              const long long a = lo[(long long)ncol * b + q], e = lo[(long long)ncol * b + q + 1];
              const int K = (int)(e - a);
              if (K == 0) continue;
              const Mat C = cp->qmajor ? Mat{P + poff[b] + (long long)q * (wc / ncol), w, 1, nullptr}
                                     : Mat{P + poff[b] + q, w, ncol, nullptr};
              if (rows[e - 1] - rows[a] == K - 1) {
                const int r0 = rows[a];
                g1.push_back(gemm_desc(L.K[b], N, K, 1.0, colmajT(L.U[b] + r0, cnt),
                                       panel(Ob + (long long)r0 * cp->ldo, cp->ldo), 0.0, C));
              } else {
                GemmDesc d = gemm_desc(L.K[b], N, K, 1.0, colmajT(L.U[b], cnt), Mat{Ob, cp->ldo, 1, drows + a}, 0.0, C);
                d.kidx = drows + a;
                g1.push_back(d);
              }
            }
          }
        }
        gemm_batched(g1, scr, st);
        std::vector<GemmDesc> g2;
        for (size_t p = 0; p < L.pairs.size(); ++p) {
          const PairLR& pr = L.pairs[p];
          if (pr.k1 == 0 || pr.k2 == 0) continue;
          const int N = cols_in(pr.i);
          // Q_i[seg(i, j)] = M P_j[seg(j, i)],  Q_j[seg(j, i)] = M^T P_i[seg(i, j)]
          g2.push_back(gemm_desc(pr.k1, N, pr.k2, 1.0, colmaj(pr.M, pr.k1),
                                 panel(P + poff[L.pos_j[p]] + (long long)L.off_j[p] * w, w), 0.0,
                                 panel(Q + poff[L.pos_i[p]] + (long long)L.off_i[p] * w, w)));
          g2.push_back(gemm_desc(pr.k2, N, pr.k1, 1.0, colmajT(pr.M, pr.k1),
                                 panel(P + poff[L.pos_i[p]] + (long long)L.off_i[p] * w, w), 0.0,
                                 panel(Q + poff[L.pos_j[p]] + (long long)L.off_j[p] * w, w)));
        }
        gemm_batched(g2, scr, st);
        std::vector<GemmDesc> g3;
        if (split) {
          // rows of the level's nodes only (the samples are taken there), and
          // of each node only the column blocks of the other quadrants (the
          // node's own block is never used as a sample)
          const int qw = wc / cp->ncol;
          for (int b = 0; b < nbx; ++b) {
            const int box = L.boxes[b], bb = t.begin[box], be = bb + t.count[box];
            auto it = std::lower_bound(lbeg.begin(), lbeg.end(), bb);
            for (size_t u = it - lbeg.begin(); u < lbeg.size() && lbeg[u] < be; ++u) {
              const int node = lnode[u], q = (*cp->qbox)[node];
              const int r0 = t.begin[node], rc = t.count[node];
              const Mat A = colmaj(L.U[b] + (r0 - bb), t.count[box]);
              // columns [0, q qw) and [(q + 1) qw, ncol qw)
              if (q > 0)
                g3.push_back(gemm_desc(rc, q * qw, L.K[b], -1.0, A, panel(Q + poff[b], w), 1.0,
                                       panel(out + (long long)r0 * nc, nc)));
              if (q + 1 < cp->ncol)
                g3.push_back(gemm_desc(rc, (cp->ncol - q - 1) * qw, L.K[b], -1.0, A,
                                       panel(Q + poff[b] + (long long)(q + 1) * qw, w), 1.0,
                                       panel(out + (long long)r0 * nc + (long long)(q + 1) * qw, nc)));
            }
          }
        } else {
          for (int b = 0; b < nbx; ++b) {
            const int box = L.boxes[b];
            g3.push_back(gemm_desc(t.count[box], cols_in(box), L.K[b], -1.0, colmaj(L.U[b], t.count[box]),
                                   panel(Q + poff[b], w), 1.0, panel(out + (long long)t.begin[box] * nc + c0, nc)));
          }
        }
        gemm_batched(g3, scr, st);
      }
      scr.release(P);
      scr.release(Q);
    }
  }

  // Pivots and ranks of nj Gram matrices (G + goff[e], c[e] x c[e], ld c[e])
  // by blocked pivoted Cholesky; pivots of matrix e go to dpiv + poff[e].
  // G is preserved.
  void pivot_ranks(const double* G, const std::vector<long long>& goff, const std::vector<int>& c,
                   const std::vector<long long>& poff, double tol2, int* dpiv, std::vector<int>& rk,
                   hipStream_t st) {
    TraceTag tag("peel_pivot");
    Scratch ws(st);  // work buffers live only through this call
    const int nj = (int)c.size();
    const int cmax = *std::max_element(c.begin(), c.end());
    RSF_CHECK(cmax <= PCHOL_MAXN, RSF_E_INVALID,
              "peeling needs more than " + std::to_string(PCHOL_MAXN) + " probe columns per block");
    const int NB = cmax <= 1024 ? 32 : cmax <= 2048 ? 16 : 8;
    std::vector<long long> doff(nj + 1, 0);
    for (int e = 0; e < nj; ++e) doff[e + 1] = doff[e] + c[e];
    double* Gw = ws.make<double>(std::max<long long>(goff[nj], 1));
    copy_dev(Gw, G, goff[nj], st);
    double* d = ws.make<double>(std::max<long long>(doff[nj], 1));
    double* Lp = ws.make<double>(std::max<long long>(doff[nj] * NB, 1));
    double* d1 = ws.make<double>(nj);
    int* state = ws.make<int>(2 * nj);
    std::vector<PpanelJob> all(nj);
    for (int e = 0; e < nj; ++e)
      all[e] = PpanelJob{Gw + goff[e], d + doff[e], Lp + doff[e] * NB, dpiv + poff[e], state + 2 * e, d1 + e, c[e]};
    // the job table goes up once: every panel launch covers all matrices,
    // and a finished one's workgroup returns at once (its state says so)
    PpanelJob* dj = ws.make<PpanelJob>(nj);
    upload(dj, all, st);
    hipLaunchKernelGGL(ppanel_init_kernel, dim3(nj), dim3(256), 0, st, dj);
    RSF_HIP(hipGetLastError());
    std::vector<int> active(nj);
    for (int e = 0; e < nj; ++e) active[e] = e;
    std::vector<int> hs(2 * nj, 0);
    const int npanel = (cmax + NB - 1) / NB;
    for (int pnl = 0; pnl <= npanel && !active.empty(); ++pnl) {
      const dim3 grid((unsigned)nj), blk(PCHOL_WG);
      // one row per thread and panel column: small Gram matrices take small workgroups
      if (cmax <= 256)
        hipLaunchKernelGGL((ppanel_kernel<1, 32, 256>), grid, dim3(256), 0, st, dj, tol2);
      else if (cmax <= 1024)
        hipLaunchKernelGGL((ppanel_kernel<1, 32, 1024>), grid, blk, 0, st, dj, tol2);
      else if (cmax <= 2048)
        hipLaunchKernelGGL((ppanel_kernel<2, 16, 1024>), grid, blk, 0, st, dj, tol2);
      else
        hipLaunchKernelGGL((ppanel_kernel<4, 8, 1024>), grid, blk, 0, st, dj, tol2);
      RSF_HIP(hipGetLastError());
      // every few panels, drop the matrices that have reached their rank
      if (pnl % 4 == 3 || pnl + 1 >= npanel) {
        RSF_HIP(hipMemcpyAsync(hs.data(), state, hs.size() * sizeof(int), hipMemcpyDeviceToHost, st));
        RSF_HIP(hipStreamSynchronize(st));
        std::vector<int> still;
        for (int e : active)
          if (!hs[2 * e + 1]) still.push_back(e);
        active.swap(still);
        if (active.empty()) break;
      }
      std::vector<GemmDesc> tg;
      for (int e : active) {
        GemmDesc gd = gemm_desc(c[e], c[e], NB, -1.0, colmaj(all[e].Lp, c[e]), colmajT(all[e].Lp, c[e]), 1.0,
                                colmaj(Gw + goff[e], c[e]));
        gd.lower = true;
        tg.push_back(gd);
      }
      gemm_batched(tg, ws, st);
    }
    RSF_CHECK(active.empty(), RSF_E_INVALID, "pivoted Cholesky did not terminate");
    rk.assign(nj, 0);
    for (int e = 0; e < nj; ++e) rk[e] = hs[2 * e];
  }

  // Bases and core matrices of the sibling pairs [p0, p1) of one level and
  // operator (eq. lowrankapprox), the pairs' instances peeling tot[] columns:
  //   U = orth(Y_ij): Yg = Y_ij(:, piv[:k]), U = Yg L1^-T with L1 L1^T = Yg^T Yg
  //     (the leading factor of the pivoted Cholesky, recomputed on the pivot
  //     columns by the batched blocked Cholesky);
  //   M = (Om_i^T U1)^+ (Om_i^T Y_ij) (U2^T Om_j)^+ through the normal
  //     equations, with (Om_i^T U1)^T (Om_i^T Y_ij) formed as (Om_i A1)^T Y_ij.
  // Y: samples, row d holds quadrant block q at columns [q C, q C + tot); Om:
  // probes (ld C); pivots of block e at dpiv + poff[e].
  // Every sibling pair of one level and operator, in chunks that bound the
  // work memory.
  void lowrank_level(LevelLR& L, const std::vector<int>& tot, int C, int ncol, const std::vector<int>& qbox,
                     const double* Yop, const double* Om, const int* dpiv, const std::vector<long long>& poff,
                     int blk0, hipStream_t st) {
    TraceTag tg("peel_lowrank");
    const int np = (int)L.pairs.size();
    int p0 = 0;
    while (p0 < np) {
      long long bytes = 0;
      int p1 = p0;
      while (p1 < np) {
        const PairLR& pr = L.pairs[p1];
        const long long ci = t.count[pr.i], cj = t.count[pr.j], k1 = pr.k1, k2 = pr.k2;
        const long long total = tot[t.inst[pr.i]];
        const long long est = 8 * (2 * (ci * k1 + cj * k2) + 4 * (k1 * k1 + k2 * k2) + 2 * total * (k1 + k2) +
                                   total * k1 + 3 * k1 * k2 + 64);
        if (p1 > p0 && bytes + est > LOWRANK_CHUNK_BYTES) break;
        bytes += est;
        ++p1;
      }
      lowrank_chunk(L, p0, p1, tot, C, ncol, qbox, Yop, Om, dpiv, poff, blk0, st);
      p0 = p1;
    }
  }

  void lowrank_chunk(LevelLR& L, int p0, int p1, const std::vector<int>& tot, int C, int ncol,
                     const std::vector<int>& qbox, const double* Yop, const double* Om, const int* dpiv,
                     const std::vector<long long>& poff, int blk0, hipStream_t st) {
    Scratch ms(st);
    const long long ld = (long long)ncol * C;
    // every per-pair buffer is carved from one block (one allocation per chunk)
    long long need = 0;
    for (int p = p0; p < p1; ++p) {
      const PairLR& pr = L.pairs[p];
      const long long ci = t.count[pr.i], cj = t.count[pr.j], k1 = pr.k1, k2 = pr.k2, tt = tot[t.inst[pr.i]];
      need += ci * k1 + cj * k2 + 2 * (k1 * k1 + k2 * k2);  // Yg, G, Li of both blocks
      if (k1 > 0 && k2 > 0) need += 2 * tt * k1 + k2 * tt + ci * k1 + 2 * (k1 * k1 + k2 * k2) + 2 * k1 * k2;
    }
    // a fixed-size block (when it suffices) is reused by every chunk
    double* pool = ms.make<double>(std::max<long long>(need, LOWRANK_CHUNK_BYTES / 8));
    long long used = 0;
    auto carve = [&](long long count) {
      double* q = pool + used;
      used += count;
      return q;
    };
    int* fail = ms.make<int>(1);
    RSF_HIP(hipMemsetAsync(fail, 0, sizeof(int), st));
    struct Blk {
      int e, k, cnt;
      const double* Yb;
      double *Yg, *G, *Li, *U;
    };
    std::vector<Blk> bl;
    for (int p = p0; p < p1; ++p) {
      const PairLR& pr = L.pairs[p];
      for (int side = 0; side < 2; ++side) {
        const int rb = side ? pr.j : pr.i, cb = side ? pr.i : pr.j, k = side ? pr.k2 : pr.k1;
        if (k == 0) continue;
        Blk b;
        b.e = blk0 + 2 * p + side;
        b.k = k;
        b.cnt = t.count[rb];
        b.Yb = Yop + (long long)t.begin[rb] * ld + (long long)qbox[cb] * C;
        b.Yg = carve((long long)b.cnt * k);
        b.G = carve((long long)k * k);
        b.Li = carve((long long)k * k);
        b.U = side ? L.U[L.pos_j[p]] + (long long)L.off_j[p] * b.cnt : L.U[L.pos_i[p]] + (long long)L.off_i[p] * b.cnt;
        bl.push_back(b);
      }
    }
    RSF_CHECK(used <= need, RSF_E_HIP, "peeling work buffer overrun");
    if (!bl.empty()) {
      std::vector<GatherColsJob> gj;
      long long maxe = 1;
      std::vector<GemmDesc> g1, g2;
      std::vector<CholProblem> cp;
      for (const Blk& b : bl) {
        gj.push_back(GatherColsJob{b.Yb, ld, dpiv + poff[b.e], b.k, b.cnt, b.Yg});
        maxe = std::max(maxe, (long long)b.cnt * b.k);
        // G = Yg^T Yg: the lower triangle (all the Cholesky reads)
        g1.push_back(gemm_desc(b.k, b.k, b.cnt, 1.0, colmajT(b.Yg, b.cnt), colmaj(b.Yg, b.cnt), 0.0, colmaj(b.G, b.k)));
        g1.back().lower = true;
        cp.push_back(CholProblem{b.G, b.k, b.k, b.Li, b.k, nullptr});
        // U = Yg Li^T, formed as U^T = Li Yg^T so that the triangular factor is
        // the A operand (its zero upper triangle skipped)
        g2.push_back(gemm_desc(b.k, b.cnt, b.k, 1.0, colmaj(b.Li, b.k), colmajT(b.Yg, b.cnt), 0.0, colmajT(b.U, b.cnt)));
        g2.back().tri = 1;
      }
      GatherColsJob* dg = ms.make<GatherColsJob>(gj.size());
      upload(dg, gj, st);
      hipLaunchKernelGGL(gather_cols_kernel, dim3(grid_of(maxe), (unsigned)gj.size()), dim3(256), 0, st, dg);
      RSF_HIP(hipGetLastError());
      gemm_batched(g1, ms, st);
      batched_chol_inv(cp, fail, ms, st);
      gemm_batched(g2, ms, st);
    }
    std::vector<GemmDesc> ga, gb, gc, gd, ge, gf, gg, gh;
    std::vector<CholProblem> cn;
    for (int p = p0; p < p1; ++p) {
      PairLR& pr = L.pairs[p];
      const int k1 = pr.k1, k2 = pr.k2;
      if (k1 == 0 || k2 == 0) continue;
      const int bi = pr.i, bj = pr.j, ci = t.count[bi], cj = t.count[bj];
      const int total = tot[t.inst[bi]];
      const double* U1 = L.U[L.pos_i[p]] + (long long)L.off_i[p] * ci;
      const double* U2 = L.U[L.pos_j[p]] + (long long)L.off_j[p] * cj;
      const Mat OmiT{Om + (long long)t.begin[bi] * C, 1, (long long)C, nullptr};
      const Mat Omi = panel(Om + (long long)t.begin[bi] * C, C);
      const Mat Omj = panel(Om + (long long)t.begin[bj] * C, C);
      const double* Yij = Yop + (long long)t.begin[bi] * ld + (long long)qbox[bj] * C;
      double* A1 = carve((long long)total * k1);
      double* A2 = carve((long long)k2 * total);
      double* W1 = carve((long long)ci * k1);
      double* N1 = carve((long long)k1 * k1);
      double* N2 = carve((long long)k2 * k2);
      double* N1i = carve((long long)k1 * k1);
      double* N2i = carve((long long)k2 * k2);
      double* T1 = carve((long long)k1 * total);
      double* T2 = carve((long long)k1 * k2);
      double* X = carve((long long)k1 * k2);
      // A1 = Om_i^T U1, A2 = U2^T Om_j
      ga.push_back(gemm_desc(total, k1, ci, 1.0, OmiT, colmaj(U1, ci), 0.0, colmaj(A1, total)));
      ga.push_back(gemm_desc(k2, total, cj, 1.0, colmajT(U2, cj), Omj, 0.0, colmaj(A2, k2)));
      // W1 = Om_i A1, N1 = A1^T A1, N2 = A2 A2^T
      gb.push_back(gemm_desc(ci, k1, total, 1.0, Omi, colmaj(A1, total), 0.0, colmaj(W1, ci)));
      gb.push_back(gemm_desc(k1, k1, total, 1.0, colmajT(A1, total), colmaj(A1, total), 0.0, colmaj(N1, k1)));
      gb.back().lower = true;
      gb.push_back(gemm_desc(k2, k2, total, 1.0, colmaj(A2, k2), colmajT(A2, k2), 0.0, colmaj(N2, k2)));
      gb.back().lower = true;
      cn.push_back(CholProblem{N1, k1, k1, N1i, k1, nullptr});
      cn.push_back(CholProblem{N2, k2, k2, N2i, k2, nullptr});
      // T1 = W1^T Y_ij, T2 = T1 A2^T
      gc.push_back(gemm_desc(k1, total, ci, 1.0, colmajT(W1, ci), panel(Yij, ld), 0.0, colmaj(T1, k1)));
      gd.push_back(gemm_desc(k1, k2, total, 1.0, colmaj(T1, k1), colmajT(A2, k2), 0.0, colmaj(T2, k1)));
      // M = N1^-1 T2 N2^-1 with N^-1 = Linv^T Linv
      ge.push_back(gemm_desc(k1, k2, k1, 1.0, colmaj(N1i, k1), colmaj(T2, k1), 0.0, colmaj(X, k1)));
      ge.back().tri = 1;  // the inverse Cholesky factors are lower triangular
      gf.push_back(gemm_desc(k1, k2, k1, 1.0, colmajT(N1i, k1), colmaj(X, k1), 0.0, colmaj(T2, k1)));
      gf.back().tri = 2;
      gg.push_back(gemm_desc(k1, k2, k2, 1.0, colmaj(T2, k1), colmajT(N2i, k2), 0.0, colmaj(X, k1)));
      gh.push_back(gemm_desc(k1, k2, k2, 1.0, colmaj(X, k1), colmaj(N2i, k2), 0.0, colmaj(pr.M, k1)));
    }
    RSF_CHECK(used <= need, RSF_E_HIP, "peeling work buffer overrun");
    gemm_batched(ga, ms, st);
    gemm_batched(gb, ms, st);
    batched_chol_inv(cn, fail, ms, st);
    gemm_batched(gc, ms, st);
    gemm_batched(gd, ms, st);
    gemm_batched(ge, ms, st);
    gemm_batched(gf, ms, st);
    gemm_batched(gg, ms, st);
    gemm_batched(gh, ms, st);
    int fh = 0;
    RSF_HIP(hipMemcpyAsync(&fh, fail, sizeof(int), hipMemcpyDeviceToHost, st));
    RSF_HIP(hipStreamSynchronize(st));
    RSF_CHECK(fh == 0, RSF_E_NOT_SPD, "peeling: singular normal equations of a basis or core matrix");
  }

  // traces[op][i]: the trace of operator op for instance i
  void run(double eps_peel, uint64_t seed, double* const* traces, PeelStats* st) {
    const long long n = t.n;
    const int D = t.maxdepth, ni = t.ninst;
    for (int op = 0; op < nop; ++op) lr[op].assign(D + 1, LevelLR());
    // relative pivots below ~1e-13 of the Gram diagonal are rounding noise
    // (the Gram squares the singular values), so the threshold is floored there
    const double tol2 = std::max(eps_peel * eps_peel, 1e-13);
    // per instance: the largest sibling-block rank of the previous level (-1: none yet)
    std::vector<int> prev(ni, -1), peeled(ni, 0);
    std::vector<int> qd(n), rinst(n);
    for (int i = 0; i < ni; ++i)
      for (long long d = t.ioff[i]; d < t.ioff[i + 1]; ++d) rinst[d] = i;
    // Test-only: RSFGP_TEST_PEEL_COLS = "c1,c2,..." starts level l at c_l
    // probe columns per quadrant block (every instance), so that a parity test
    // can run the probe schedule of a reference run; growth still applies.
    std::vector<int> forced;
    if (const char* e = std::getenv("RSFGP_TEST_PEEL_COLS")) {
      for (const char* q = e; *q;) {
        char* end = nullptr;
        const long v = strtol(q, &end, 10);
        if (end == q) break;
        forced.push_back((int)std::max(1L, std::min(v, 1L << 20)));
        q = *end == ',' ? end + 1 : end;
      }
    }
    Scratch keep(s);
    int* drinst = keep.make<int>(n);
    upload(drinst, rinst, s);
    // probe and sample stores, kept across levels (capacity: Ccap probe columns
    // per row, Ycap sample columns per row)
    double* Om = nullptr;
    double* Y[MAXOP] = {nullptr, nullptr, nullptr};
    int Ccap = 0;
    long long Ycap = 0;
    const Cells cells = strong ? cell_coords(t) : Cells();
    const uint32_t stream_id = strong ? 2u : 0u;
    for (int lev = 1; lev <= D; ++lev) {
      const auto cl0 = std::chrono::steady_clock::now();
      struct LevelClock {
        double& acc;
        std::chrono::steady_clock::time_point t0;
        ~LevelClock() { acc += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
      } level_clock{tm[7], cl0};
      Scratch scr(s);
      // the blocks peeled at this level and the column block of every node's
      // probes: sibling pairs by quadrant (weak form), or the admissible pairs
      // by colour (strong form)
      std::vector<std::pair<int, int>> pairs;
      std::vector<int> qbox(t.nbox(), -1);
      int ncol = 4;
      if (strong) {
        StrongLevel sl = strong_level(t, cells, lev);
        pairs.swap(sl.pairs);
        qbox.swap(sl.color);
        ncol = std::max(1, sl.ncol);
      } else {
        for (int p = t.lev[lev - 1]; p < t.lev[lev]; ++p) {
          std::vector<int> ks;
          for (int c : t.child[p])
            if (c >= 0) ks.push_back(c);
          for (size_t a = 0; a < ks.size(); ++a)
            for (size_t b = a + 1; b < ks.size(); ++b) pairs.emplace_back(ks[a], ks[b]);
        }
        for (int b = t.lev[lev]; b < t.lev[lev + 1]; ++b) qbox[b] = t.quad[b];
      }
      if (pairs.empty()) continue;
      std::fill(qd.begin(), qd.end(), -1);
      for (int b = 0; b < t.nbox(); ++b)
        if (qbox[b] >= 0)
          for (int u = 0; u < t.count[b]; ++u) qd[t.begin[b] + u] = qbox[b];
      int* dqd = scr.make<int>(n);
      upload(dqd, qd, s);
      // per ordered sample block: (row box, column-block box)
      std::vector<std::pair<int, int>> blocks;
      for (auto& pr : pairs) {
        blocks.emplace_back(pr.first, pr.second);
        blocks.emplace_back(pr.second, pr.first);
      }
      const int nblk = (int)blocks.size();
      // probe columns per quadrant block, per instance: target c, done tot
      std::vector<int> has(ni, 0), cc(ni, 0), tot(ni, 0);
      for (auto& pr : pairs) has[t.inst[pr.first]] = 1;
      for (int i = 0; i < ni; ++i)
        if (has[i]) {
          if (strong)
            cc[i] = prev[i] < 0 ? FIRST_COLS_STRONG : next_cols_strong(prev[i]);
          else
            cc[i] = prev[i] < 0 ? first_cols(t.ioff[i + 1] - t.ioff[i]) : next_cols(prev[i], peeled[i]);
          if (lev <= (int)forced.size()) cc[i] = forced[lev - 1];
        }
      int C = 0;  // layout of the probe and sample stores (columns per quadrant block)
      const int nsb = nop * nblk;  // sample blocks of every operator
      std::vector<int> rk(nsb), maxr(ni, 0);
      std::vector<long long> poff(nsb + 1, 0);
      int* dpiv = nullptr;
      while (true) {
        const int cnew = *std::max_element(cc.begin(), cc.end());
        auto cg0 = std::chrono::steady_clock::now();
        if (C == 0 && cnew <= Ccap && (long long)ncol * cnew <= Ycap) {
          C = cnew;  // a new level reuses the stores of the previous ones
        } else if (cnew > C) {
          // grow the probe and sample stores: a new layout, the samples taken so far copied over
          const int cap = std::max(cnew, Ccap);
          const long long ycap = std::max<long long>((long long)ncol * cnew, Ycap);
          double* Om2 = keep.make<double>((size_t)n * cap);
          double* Y2[MAXOP] = {nullptr, nullptr, nullptr};
          for (int op = 0; op < nop; ++op) Y2[op] = keep.make<double>((size_t)n * ycap);
          if (C > 0) {
            hipLaunchKernelGGL(regrid_kernel, dim3(grid_of(n * C)), dim3(256), 0, s, n, 1, C, Om, C, Om2, cnew);
            for (int op = 0; op < nop; ++op)
              hipLaunchKernelGGL(regrid_kernel, dim3(grid_of(n * ncol * C)), dim3(256), 0, s, n, ncol, C, Y[op], C,
                                 Y2[op], cnew);
            RSF_HIP(hipGetLastError());
          }
          keep.release(Om);
          for (int op = 0; op < nop; ++op) {
            keep.release(Y[op]);
            Y[op] = Y2[op];
          }
          Om = Om2;
          Ccap = cap;
          Ycap = ycap;
          C = cnew;
        }
        tm[6] += std::chrono::duration<double>(std::chrono::steady_clock::now() - cg0).count();
        // the new probe columns of every instance go through the operators
        // together, in chunks that keep the 2 nop n x 4 cw work panels within
        // PEEL_CHUNK_BYTES
        int newmax = 0;
        for (int i = 0; i < ni; ++i) newmax = std::max(newmax, cc[i] - tot[i]);
        const long long per_col = 2LL * nop * n * ncol * (long long)sizeof(double);
        const int cw = std::min(newmax, (int)std::max<long long>(8, PEEL_CHUNK_BYTES / per_col / 8 * 8));
        int* dact = scr.make<int>(ni);
        int* dj0 = scr.make<int>(ni);
        // one instance in the weak form: contiguous quadrant blocks, so that the
        // coarser levels' subtraction can skip each row's own quadrant
        const bool qmajor = !strong && ni == 1;
        for (int t0 = 0; t0 < newmax; t0 += cw) {
          const int ncw = std::min(cw, newmax - t0);
          std::vector<int> act(ni), j0(ni), pcols(ni);
          for (int i = 0; i < ni; ++i) {
            act[i] = std::max(0, std::min(ncw, cc[i] - tot[i] - t0));
            j0[i] = tot[i] + t0;
            pcols[i] = ncol * act[i];
          }
          upload(dact, act, s);
          upload(dj0, j0, s);
          Scratch rs(s);
          const long long sz = n * (long long)ncol * ncw;
          double* Wm = rs.make<double>(n * (long long)ncol * cw);  // full-chunk sizes: reused by every chunk
          fill_zero(Wm, sz, s);
          hipLaunchKernelGGL(probe_kernel, dim3(grid_of(n * ncw)), dim3(256), 0, s, dqd, drinst, dact, dj0, n, ncw,
                             ncol, qmajor ? 1 : 0, lev, stream_id, seed, Wm, Om, (long long)C);
          RSF_HIP(hipGetLastError());
          double* Bo[MAXOP] = {nullptr, nullptr, nullptr};
          for (int op = 0; op < nop; ++op) Bo[op] = rs.make<double>(n * (long long)ncol * cw);
          const int* pc = ni > 1 ? pcols.data() : nullptr;
          auto c0 = std::chrono::steady_clock::now();
          apply_ops(Wm, ncol * ncw, Bo, rs, pc);
          auto c1 = std::chrono::steady_clock::now();
          const CompactProbes cpr{Om, (long long)C, &j0, &qd, ncol, qmajor ? 1 : 0, lev, &qbox};
          auto sub_store = [&](int op, Scratch& r, hipStream_t st) {
            subtract_lowrank(op, lev, Wm, ncol * ncw, Bo[op], r, pc, &cpr, st);
            hipLaunchKernelGGL(store_samples_kernel, dim3(grid_of(sz)), dim3(256), 0, st, dqd, drinst, dact, dj0, n,
                               ncw, ncol, qmajor ? 1 : 0, C, Bo[op], Y[op]);
            RSF_HIP(hipGetLastError());
          };
          // the operators' subtractions and sample stores side by side
          // (operator 1 on the side stream)
          beside(
              [&](hipStream_t s2) {
                Scratch r2(s2);
                sub_store(1, r2, s2);
              },
              [&] {
                for (int op = 0; op < nop; ++op)
                  if (op != 1) sub_store(op, rs, s);
              });
          auto c2 = std::chrono::steady_clock::now();
          tm[0] += std::chrono::duration<double>(c1 - c0).count();
          tm[1] += std::chrono::duration<double>(c2 - c1).count();
        }
        for (int i = 0; i < ni; ++i) tot[i] = cc[i];
        // ranks of every sample block (both operators) by pivoted Cholesky of
        // its Gram matrix, in chunks that bound the Gram storage
        std::vector<int> bc(nsb);
        for (int idx = 0; idx < nsb; ++idx) {
          bc[idx] = tot[t.inst[blocks[idx % nblk].first]];
          poff[idx + 1] = poff[idx] + bc[idx];
        }
        scr.release(dpiv);
        dpiv = scr.make<int>(std::max<long long>(poff[nsb], 1));
        // the sample blocks of the operators side by side (operator 1 on the
        // side stream), each in chunks that bound the Gram storage
        auto gram_ranks = [&](int ebeg, int eend, hipStream_t st) {
          for (int e0 = ebeg; e0 < eend;) {
            std::vector<long long> goff(1, 0);
            std::vector<int> cs;
            int e1 = e0;
            while (e1 < eend) {
              const long long add = (long long)bc[e1] * bc[e1];
              if (e1 > e0 && 8 * 2 * (goff.back() + add) > GRAM_CHUNK_BYTES) break;
              goff.push_back(goff.back() + add);
              cs.push_back(bc[e1]);
              ++e1;
            }
            Scratch gs(st);
            double* Gram = gs.make<double>(std::max<long long>(goff.back(), GRAM_CHUNK_BYTES / 16));
            std::vector<GemmDesc> g;
            for (int idx = e0; idx < e1; ++idx) {
              const int op = idx / nblk, e = idx % nblk;
              const int rb = blocks[e].first, cbx = blocks[e].second, c = bc[idx];
              const long long ldy = (long long)ncol * C;
              const double* Yb = Y[op] + (long long)t.begin[rb] * ldy + (long long)qbox[cbx] * C;
              // the lower triangle only (the pivoted Cholesky reads no other entry)
              GemmDesc gd = gemm_desc(c, c, t.count[rb], 1.0, Mat{Yb, 1, ldy, nullptr}, panel(Yb, ldy), 0.0,
                                      colmaj(Gram + goff[idx - e0], c));
              gd.lower = true;
              g.push_back(gd);
            }
            {
              TraceTag tg("peel_gram");
              gemm_batched(g, gs, st);
            }
            std::vector<long long> pv(poff.begin() + e0, poff.begin() + e1);
            std::vector<int> rq;
            pivot_ranks(Gram, goff, cs, pv, tol2, dpiv, rq, st);
            for (int q = 0; q < e1 - e0; ++q) rk[e0 + q] = rq[q];
            e0 = e1;
          }
        };
        {
          auto c0 = std::chrono::steady_clock::now();
          beside([&](hipStream_t s2) { gram_ranks(nblk, 2 * nblk, s2); },
                 [&] {
                   gram_ranks(0, nblk, s);
                   if (nop > 2) gram_ranks(2 * nblk, nsb, s);
                 });
          tm[2] += std::chrono::duration<double>(std::chrono::steady_clock::now() - c0).count();
        }
        // an instance needs more columns while a block's rank is not
        // resolved (rank + oversampling above its columns, which are fewer
        // than the block's own)
        std::vector<int> need(ni, 0);
        std::fill(maxr.begin(), maxr.end(), 0);
        for (int idx = 0; idx < nsb; ++idx) {
          const int e = idx % nblk, i = t.inst[blocks[e].first], k = rk[idx];
          maxr[i] = std::max(maxr[i], k);
          if (k + OVERSAMPLE > tot[i] && tot[i] < t.count[blocks[e].second]) need[i] = 1;
        }
        bool any = false;
        for (int i = 0; i < ni; ++i)
          if (need[i]) {
            cc[i] = grow_cols(tot[i], maxr[i]);
            any = true;
          }
        if (!any) break;
      }
      int colmax = 0, rankmax = 0;
      for (int i = 0; i < ni; ++i)
        if (has[i]) {
          prev[i] = maxr[i];
          ++peeled[i];
          colmax = std::max(colmax, tot[i]);
          rankmax = std::max(rankmax, maxr[i]);
        }
      if (st && lev < 32) {
        st->cols[lev] = colmax;
        st->rank[lev] = rankmax;
      }
      TraceTag tg("peel_lowrank");
      const int np = (int)pairs.size();
      for (int op = 0; op < nop; ++op) {
        LevelLR& L = lr[op][lev];
        L.any = true;
        std::vector<int> pos(t.nbox(), -1);
        for (auto& pr : pairs)
          for (int bx : {pr.first, pr.second})
            if (pos[bx] < 0) {
              pos[bx] = (int)L.boxes.size();
              L.boxes.push_back(bx);
            }
        const int nbx = (int)L.boxes.size();
        L.K.assign(nbx, 0);
        std::vector<int> blk_off(nblk);
        for (int e = 0; e < nblk; ++e) {
          const int b = pos[blocks[e].first];
          blk_off[e] = L.K[b];
          L.K[b] += rk[op * nblk + e];
        }
        // one block holds every basis and core matrix of this level and operator
        long long lvl = 0;
        for (int b = 0; b < nbx; ++b) lvl += (long long)t.count[L.boxes[b]] * L.K[b];
        for (int p = 0; p < np; ++p) {
          const long long k1 = rk[op * nblk + 2 * p], k2 = rk[op * nblk + 2 * p + 1];
          if (k1 > 0 && k2 > 0) lvl += k1 * k2;
        }
        double* lblock = store.make<double>(std::max<long long>(lvl, 1));
        long long lused = 0;
        L.U.assign(nbx, nullptr);
        for (int b = 0; b < nbx; ++b) {
          L.U[b] = lblock + lused;
          lused += (long long)t.count[L.boxes[b]] * L.K[b];
        }
        L.pairs.resize(np);
        L.off_i.resize(np);
        L.off_j.resize(np);
        L.pos_i.resize(np);
        L.pos_j.resize(np);
        for (int p = 0; p < np; ++p) {
          PairLR& pr = L.pairs[p];
          pr.i = pairs[p].first;
          pr.j = pairs[p].second;
          pr.k1 = rk[op * nblk + 2 * p];
          pr.k2 = rk[op * nblk + 2 * p + 1];
          L.off_i[p] = blk_off[2 * p];
          L.off_j[p] = blk_off[2 * p + 1];
          L.pos_i[p] = pos[pr.i];
          L.pos_j[p] = pos[pr.j];
          if (pr.k1 > 0 && pr.k2 > 0) {
            pr.M = lblock + lused;
            lused += (long long)pr.k1 * pr.k2;
          }
        }
        RSF_CHECK(lused <= std::max<long long>(lvl, 1), RSF_E_HIP, "low-rank store overrun");
      }
      // bases and core matrices: operator 1 on the side stream beside operator 0
      auto c0 = std::chrono::steady_clock::now();
      beside([&](hipStream_t s2) { lowrank_level(lr[1][lev], tot, C, ncol, qbox, Y[1], Om, dpiv, poff, nblk, s2); },
             [&] {
               for (int op = 0; op < nop; ++op)
                 if (op != 1) lowrank_level(lr[op][lev], tot, C, ncol, qbox, Y[op], Om, dpiv, poff, op * nblk, s);
             });
      tm[3] += std::chrono::duration<double>(std::chrono::steady_clock::now() - c0).count();
    }
    // extraction at the leaves: traces of every instance over its own leaves.
    // Weak form: every leaf's identity block in the same n_L columns (only the
    // leaves' own diagonal blocks remain after the subtraction).  Strong form:
    // the near field remains, so touching leaves get different column blocks.
    const auto cx0 = std::chrono::steady_clock::now();
    Scratch scr(s);
    std::vector<int> lbeg, lcnt, lbox, lfirst(ni + 1, 0);
    int nL = 1;
    for (int i = 0; i < ni; ++i) {
      for (int b = 0; b < t.nbox(); ++b)
        if (t.leaf[b] && t.inst[b] == i) {
          lbeg.push_back(t.begin[b]);
          lcnt.push_back(t.count[b]);
          lbox.push_back(b);
          nL = std::max(nL, t.count[b]);
        }
      lfirst[i + 1] = (int)lbeg.size();
    }
    const int nleaf = (int)lbeg.size();
    int ncl = 1;
    std::vector<int> lcol0;
    if (strong) {
      std::vector<int> lc;
      ncl = std::max(1, leaf_colors(t, cells, lbox, lc));
      lcol0.resize(nleaf);
      for (int a = 0; a < nleaf; ++a) lcol0[a] = lc[a] * nL;
    }
    const int ncE = ncl * nL;
    int* dlb = scr.make<int>(nleaf);
    int* dlc = scr.make<int>(nleaf);
    int* dl0 = strong ? scr.make<int>(nleaf) : nullptr;
    upload(dlb, lbeg, s);
    upload(dlc, lcnt, s);
    if (strong) upload(dl0, lcol0, s);
    const long long sz = n * ncE;
    double* E = scr.make<double>(sz);
    fill_zero(E, sz, s);
    hipLaunchKernelGGL(eye_blocks_kernel, dim3(nleaf), dim3(256), 0, s, dlb, dlc, dl0, nleaf, E, ncE);
    RSF_HIP(hipGetLastError());
    double* Ho[MAXOP] = {nullptr, nullptr, nullptr};
    for (int op = 0; op < nop; ++op) Ho[op] = scr.make<double>(sz);
    apply_ops(E, ncE, Ho, scr, nullptr);
    for (int op = 0; op < nop; ++op) subtract_lowrank(op, D + 1, E, ncE, Ho[op], scr, nullptr);
    double* tr = scr.make<double>(nop * ni);
    for (int i = 0; i < ni; ++i) {
      const int l0 = lfirst[i], nl = lfirst[i + 1] - lfirst[i];
      for (int op = 0; op < nop; ++op)
        hipLaunchKernelGGL(leaf_trace_kernel, dim3(1), dim3(256), 0, s, dlb + l0, dlc + l0, dl0 ? dl0 + l0 : nullptr,
                           nl, Ho[op], ncE, tr + op * ni + i);
    }
    RSF_HIP(hipGetLastError());
    std::vector<double> th(nop * ni);
    RSF_HIP(hipMemcpyAsync(th.data(), tr, th.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    RSF_HIP(hipStreamSynchronize(s));
    for (int op = 0; op < nop; ++op)
      for (int i = 0; i < ni; ++i) traces[op][i] = th[op * ni + i];
    if (st) {
      st->levels = D;
      st->leaf_cols = ncE;
    }
    tm[5] = std::chrono::duration<double>(std::chrono::steady_clock::now() - cx0).count();
    if (std::getenv("RSFGP_PEEL_TIMES"))
      fprintf(stderr, "[peel] apply %.3f subtract %.3f pivot %.3f lowrank %.3f gram %.3f extract %.3f grow %.3f levels %.3f s\n",
              tm[0], tm[1], tm[2], tm[3], tm[4], tm[5], tm[6], tm[7]);
  }
};


}  // namespace

void peel_traces(const rsf_factor_s* h, double eps_peel, uint64_t seed, double* tr_inv, double* tr_rho,
                 PeelStats* st, hipStream_t s, const FactorData* Fd2, double* tr_rho2) {
  const FactorData* fd[2] = {h->Frho.get(), Fd2};
  double* traces[3] = {tr_inv, tr_rho, tr_rho2};
  Peeler p(h, fd, Fd2 ? 2 : 1, s, h->opt.strong_peeling);
  p.run(eps_peel, seed, traces, st);
}

}  // namespace rsf

namespace rsf {

// Rademacher probes of Hutchinson's estimator (eq. hutch): U[d, j] = +1 or
// -1 from the lowest bit of the first Philox4x32-10 word for counter
// (d_local, j, 0, 1), d_local = d's tree-order index inside its instance
// (ioff: the instances' first rows), so a batch draws the probes each
// instance would draw alone; stream 1 keeps them apart from the peeling's
// Gaussian probes.
__global__ void rademacher_kernel(long long n, int q, const long long* __restrict__ ioff, int ni, uint64_t seed,
                                  double* __restrict__ U) {
  const long long tot = n * q;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
    const long long d = e / q;
    const int j = (int)(e - d * q);
    int lo = 0, hi = ni;  // last instance with ioff <= d
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (ioff[mid] <= d)
        lo = mid;
      else
        hi = mid;
    }
    uint32_t c[4] = {(uint32_t)(d - ioff[lo]), (uint32_t)j, 0u, 1u};
    philox(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    U[e] = (c[0] & 1u) ? -1.0 : 1.0;
  }
}

// Hutchinson estimates of Tr F^-1 and Tr F^-1 F_rho per instance: with
// w_j = B^T u_j (F^-1 = B^T B), |w_j|^2 and w_j^T F_rho w_j have expectations
// Tr B B^T = Tr F^-1 and Tr B F_rho B^T = Tr F^-1 F_rho; one half solve sweep
// and one multiply sweep over the q probe columns.
// With Fd2 (the anisotropic kernels' second derivative factorization), also
// trho2 = mean w^T F_2 w from the same w.
static void hutch_traces(rsf_factor_s* f, int q, uint64_t seed, double* tinv, double* trho, hipStream_t s,
                         const FactorData* Fd2 = nullptr, double* trho2 = nullptr) {
  const FactorData* Fd = f->Frho.get();
  const int nd = Fd2 ? 3 : 2;  // dot products per instance
  TraceTag tag("hutch");
  const Tree& t = f->tree;
  const long long n = t.n;
  const int ni = t.ninst;
  Scratch scr(s);
  double* W = scr.make<double>(n * q);
  double* X = scr.make<double>(n * q);
  double* V = scr.make<double>(n * q);
  double* V2 = Fd2 ? scr.make<double>(n * q) : nullptr;
  double* dots = scr.make<double>(nd * ni);
  std::vector<long long> io(t.ioff.begin(), t.ioff.end());
  long long* dio = scr.make<long long>(io.size());
  upload(dio, io, s);
  hipLaunchKernelGGL(rademacher_kernel, dim3(grid_of(n * q)), dim3(256), 0, s, n, q, dio, ni, seed, W);
  RSF_HIP(hipGetLastError());
  sweep_half_down(f, f->F, W, q, q, scr, s);  // W = B^T U
  copy_dev(X, W, n * q, s);
  sweep_apply_mult(f, *Fd, X, V, q, q, scr, s);  // V = F_rho W (X is consumed)
  if (Fd2) {
    copy_dev(X, W, n * q, s);
    sweep_apply_mult(f, *Fd2, X, V2, q, q, scr, s);  // V2 = F_2 W
  }
  for (int i = 0; i < ni; ++i) {
    const long long o = t.ioff[i] * (long long)q, m = (t.ioff[i + 1] - t.ioff[i]) * (long long)q;
    device_dot(W + o, W + o, m, dots + nd * i, scr, s);
    device_dot(W + o, V + o, m, dots + nd * i + 1, scr, s);
    if (Fd2) device_dot(W + o, V2 + o, m, dots + nd * i + 2, scr, s);
  }
  std::vector<double> hd(nd * ni);
  RSF_HIP(hipMemcpyAsync(hd.data(), dots, hd.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  RSF_HIP(hipStreamSynchronize(s));
  for (int i = 0; i < ni; ++i) {
    tinv[i] = hd[nd * i] / q;
    trho[i] = hd[nd * i + 1] / q;
    if (Fd2) trho2[i] = hd[nd * i + 2] / q;
  }
}

void grad_eval(rsf_factor f, const double* d_z, double eps_peel, uint64_t seed, double* g, rsf_grad_info* info,
               void* stream, int hutch_probes) {
  using clk = std::chrono::steady_clock;
  RSF_CHECK(f != nullptr, RSF_E_INVALID, "null factor handle");
  RSF_CHECK(d_z != nullptr && g != nullptr, RSF_E_INVALID, "null argument");
  if (!(eps_peel > 0.0)) eps_peel = f->eps;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const Tree& tr = f->tree;
  const int ni = tr.ninst;
  const auto t0 = clk::now();
  // anisotropic kernels: derivatives with respect to theta_1 and theta_2
  // (two multiply-only factorizations) and the nugget
  const bool aniso = f->kernel >= K_MATERN32_ANISO;
  if (!f->Frho) {
    f->Frho.reset(new FactorData());
    build_factor(f, *f->Frho, 1, s);
  }
  if (aniso && !f->Frho2) {
    f->Frho2.reset(new FactorData());
    build_factor(f, *f->Frho2, 2, s);
  }
  RSF_HIP(hipStreamSynchronize(s));
  const auto t1 = clk::now();
  Scratch scr(s);
  const long long n = tr.n;
  double* Z = scr.make<double>(n);
  double* A = scr.make<double>(n);
  double* X = scr.make<double>(n);
  double* Y = scr.make<double>(n);
  double* Y2 = aniso ? scr.make<double>(n) : nullptr;
  double* dots = scr.make<double>(4 * ni);
  to_panel(f, d_z, n, Z, 1, 1, s);
  copy_dev(A, Z, n, s);
  sweep_solve(f, f->F, A, 1, 1, scr, s);
  copy_dev(X, A, n, s);
  sweep_apply_mult(f, *f->Frho, X, Y, 1, 1, scr, s);
  if (aniso) {
    copy_dev(X, A, n, s);
    sweep_apply_mult(f, *f->Frho2, X, Y2, 1, 1, scr, s);
  }
  // per instance (tree-order range [ioff[i], ioff[i + 1])): a^T F_rho a, z^T a,
  // a^T a (and a^T F_theta2 a)
  for (int i = 0; i < ni; ++i) {
    const long long o = tr.ioff[i], m = tr.ioff[i + 1] - tr.ioff[i];
    device_dot(A + o, Y + o, m, dots + 4 * i, scr, s);
    device_dot(Z + o, A + o, m, dots + 4 * i + 1, scr, s);
    device_dot(A + o, A + o, m, dots + 4 * i + 2, scr, s);
    if (aniso) device_dot(A + o, Y2 + o, m, dots + 4 * i + 3, scr, s);
  }
  std::vector<double> hd(4 * ni, 0.0);
  RSF_HIP(hipMemcpyAsync(hd.data(), dots, hd.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  RSF_HIP(hipStreamSynchronize(s));
  const auto t2 = clk::now();
  std::vector<double> trinv(ni), trrho(ni), trrho2(ni);
  PeelStats ps;
  if (hutch_probes > 0) {
    hutch_traces(f, hutch_probes, seed, trinv.data(), trrho.data(), s, aniso ? f->Frho2.get() : nullptr,
                 aniso ? trrho2.data() : nullptr);
  } else {
    // anisotropic kernels: B B^T, B F_theta1 B^T and B F_theta2 B^T from one set of probes
    peel_traces(f, eps_peel, seed, trinv.data(), trrho.data(), &ps, s, aniso ? f->Frho2.get() : nullptr,
                aniso ? trrho2.data() : nullptr);
  }
  const auto t3 = clk::now();
  double q0[3] = {0, 0, 0}, tt0[3] = {0, 0, 0};
  for (int i = 0; i < ni; ++i) {
    const double s2 = f->thetas[3 * i + 1], nug = f->thetas[3 * i + 2];
    const double m = (double)(tr.ioff[i + 1] - tr.ioff[i]);
    double q[3] = {0.5 * hd[4 * i], 0.5 * (hd[4 * i + 1] - nug * hd[4 * i + 2]) / s2, 0.5 * hd[4 * i + 2]};
    double tt[3] = {trrho[i], (m - nug * trinv[i]) / s2, trinv[i]};
    if (aniso) {
      q[1] = 0.5 * hd[4 * i + 3];
      tt[1] = trrho2[i];
    }
    for (int j = 0; j < 3; ++j) g[3 * i + j] = q[j] - 0.5 * tt[j];
    if (i == 0)
      for (int j = 0; j < 3; ++j) {
        q0[j] = q[j];
        tt0[j] = tt[j];
      }
  }
  if (info) {
    for (int i = 0; i < 3; ++i) {
      info->q[i] = q0[i];
      info->t[i] = tt0[i];
    }
    info->trace_inv = trinv[0];
    info->peel_levels = ps.levels;
    for (int i = 0; i < 32; ++i) {
      info->peel_cols[i] = ps.cols[i];
      info->peel_rank[i] = ps.rank[i];
    }
    info->leaf_cols = ps.leaf_cols;
    info->seconds[0] = std::chrono::duration<double>(t1 - t0).count();
    info->seconds[1] = std::chrono::duration<double>(t2 - t1).count();
    info->seconds[2] = std::chrono::duration<double>(t3 - t2).count();
    info->seconds[3] = std::chrono::duration<double>(t3 - t0).count();
  }
}

__global__ void set_kernel(long long n, double v, double* __restrict__ out) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) out[i] = v;
}

// beta = a - c b (device)
__global__ void axmy_kernel(long long n, const double* __restrict__ a, double c, const double* __restrict__ b,
                            double* __restrict__ out) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) out[i] = a[i] - c * b[i];
}

void profile_eval(rsf_factor f, const double* d_z, double eps_peel, uint64_t seed, double* ell, double* g,
                  rsf_grad_info* info, void* stream) {
  RSF_CHECK(f != nullptr, RSF_E_INVALID, "null factor handle");
  RSF_CHECK(d_z != nullptr && ell != nullptr, RSF_E_INVALID, "null argument");
  RSF_CHECK(f->tree.ninst == 1, RSF_E_INVALID, "the profile likelihood takes a single handle");
  RSF_CHECK(f->kernel < K_MATERN32_ANISO, RSF_E_INVALID, "the profile likelihood takes the isotropic kernels");
  if (!(eps_peel > 0.0)) eps_peel = f->eps;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const long long n = f->tree.n;
  Scratch scr(s);
  double* Z = scr.make<double>(n);
  double* A = scr.make<double>(n);
  double* Bv = scr.make<double>(n);
  double* dots = scr.make<double>(8);
  to_panel(f, d_z, n, Z, 1, 1, s);
  copy_dev(A, Z, n, s);
  hipLaunchKernelGGL(set_kernel, dim3(grid_of(n)), dim3(256), 0, s, n, 1.0, Bv);
  RSF_HIP(hipGetLastError());
  double* ones = scr.make<double>(n);
  copy_dev(ones, Bv, n, s);
  sweep_solve(f, f->F, A, 1, 1, scr, s);   // a = F^-1 z
  sweep_solve(f, f->F, Bv, 1, 1, scr, s);  // b = F^-1 1
  device_dot(ones, A, n, dots + 0, scr, s);  // 1^T a
  device_dot(ones, Bv, n, dots + 1, scr, s); // 1^T b
  device_dot(Z, A, n, dots + 2, scr, s);     // z^T a
  double hd[8];
  RSF_HIP(hipMemcpyAsync(hd, dots, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  RSF_HIP(hipStreamSynchronize(s));
  double logdet = 0.0;
  for (double v : f->F.logdet) logdet += v;
  const double sa = hd[0], sb = hd[1], za = hd[2];
  // z^T beta with beta = (Sigma + 1 1^T)^-1 z = a - b (1^T a) / (1 + 1^T b)
  const double c = sa / (1.0 + sb), zb = za - c * sa;
  RSF_CHECK(zb > 0.0, RSF_E_NOT_SPD, "z^T (Sigma + 1 1^T)^-1 z is not positive");
  const double dn = (double)n;
  *ell = -0.5 * logdet - 0.5 * dn * std::log(zb) + 0.5 * dn * (std::log(dn) - 1.0 - std::log(2.0 * M_PI));
  if (!g) return;
  if (!f->Frho) {
    f->Frho.reset(new FactorData());
    build_factor(f, *f->Frho, 1, s);
  }
  double* beta = scr.make<double>(n);
  double* X = scr.make<double>(n);
  double* Y = scr.make<double>(n);
  hipLaunchKernelGGL(axmy_kernel, dim3(grid_of(n)), dim3(256), 0, s, n, A, c, Bv, beta);
  RSF_HIP(hipGetLastError());
  copy_dev(X, beta, n, s);
  sweep_apply_mult(f, *f->Frho, X, Y, 1, 1, scr, s);  // F_rho beta
  device_dot(beta, Y, n, dots + 3, scr, s);   // beta^T F_rho beta
  device_dot(beta, Z, n, dots + 4, scr, s);   // beta^T z
  device_dot(ones, beta, n, dots + 5, scr, s);  // 1^T beta
  device_dot(beta, beta, n, dots + 6, scr, s);  // beta^T beta
  RSF_HIP(hipMemcpyAsync(hd, dots, 7 * sizeof(double), hipMemcpyDeviceToHost, s));
  RSF_HIP(hipStreamSynchronize(s));
  double trinv = 0.0, trrho = 0.0;
  PeelStats ps;
  peel_traces(f, eps_peel, seed, &trinv, &trrho, &ps, s);
  const double s2 = f->thetas[1], nug = f->thetas[2];
  // beta^T Sigma beta = beta^T z - (1^T beta)^2 since (Sigma + 1 1^T) beta = z
  const double sbeta = hd[4] - hd[5] * hd[5];
  const double quad[3] = {hd[3], (sbeta - nug * hd[6]) / s2, hd[6]};
  const double t[3] = {trrho, (dn - nug * trinv) / s2, trinv};
  for (int i = 0; i < 3; ++i) g[i] = -0.5 * t[i] + 0.5 * dn * quad[i] / zb;
  if (info) {
    for (int i = 0; i < 3; ++i) {
      info->q[i] = quad[i];
      info->t[i] = t[i];
    }
    info->trace_inv = trinv;
    info->peel_levels = ps.levels;
    for (int i = 0; i < 32; ++i) {
      info->peel_cols[i] = ps.cols[i];
      info->peel_rank[i] = ps.rank[i];
    }
    info->leaf_cols = ps.leaf_cols;
  }
}

}  // namespace rsf
