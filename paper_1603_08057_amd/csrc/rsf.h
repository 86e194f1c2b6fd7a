// Internal state of a factor handle: the quadtree (host), the per-level
// skeletonization factors (device) and the operations on them.
#pragma once
#include <array>
#include <memory>

#include "common.h"

namespace rsf {

// Quadtree over the observation sites (Section 2.1).  Box ids are breadth
// first, so the boxes of one depth form the id range [lev[d], lev[d + 1]).
// Every box covers the contiguous tree-order range [begin, begin + count).
struct Tree {
  int64_t n = 0;
  std::vector<double> cx, cy, half;
  std::vector<int> depth, parent, quad, begin, count;
  std::vector<std::array<int, 4>> child;
  std::vector<char> leaf;
  std::vector<int> lev;   // size maxdepth + 2
  std::vector<int> perm;  // perm[t] = caller index of tree position t
  int maxdepth = 0;
  // independent instances (a forest): instance of each box, and the
  // tree-order (= caller-order) range [ioff[i], ioff[i + 1]) of instance i
  std::vector<int> inst;
  std::vector<int64_t> ioff{0, 0};
  int ninst = 1;
  int nbox() const { return (int)cx.size(); }
};

// Builds the tree (root = square on the bounding-box midpoint, split while a
// box holds more than `leaf` points, x >= cx east, y >= cy north, children
// NW, NE, SW, SE, stable partition).  Throws on duplicate sites.
Tree build_tree(const double* xy_host, int64_t n, int leaf);
// The same for independent instances (host n_i x 2 arrays), roots at depth 0.
Tree build_forest(const std::vector<const double*>& xy_host, const std::vector<int64_t>& n, int leaf);

// Factors of the boxes of one depth.  Per box b (local index within the level):
// k skeleton DOFs S, r = a - k redundant DOFs R (tree-order DOF ids, pivot
// order), and dense blocks, all column-major:
//   T (k x r)       interpolation matrix of the ID,
//   chol mode:  Linv (r x r) = L^-1 with X_rr = L L^T,  W (k x r) = X_sr L^-T,
//   mult mode:  Xsr (k x r), Xrr (r x r).
// One box of a level as the fused sweep kernels see it (device copy).
struct BoxRec {
  int k, r;
  long long s_off, r_off, t_off, l_off;
};

struct LevelFactor {
  int depth = 0, box0 = 0, nb = 0;
  BoxRec* box = nullptr;                   // device, nb records
  std::vector<int> a, k;
  std::vector<long long> s_off, r_off;     // offsets into S / R (ints)
  std::vector<long long> t_off, l_off;     // offsets into T/W/Xsr and Linv/Xrr (doubles)
  int* S = nullptr;
  int* R = nullptr;
  double* T = nullptr;
  double* W = nullptr;     // chol: W; mult: Xsr
  double* Lm = nullptr;    // chol: Linv; mult: Xrr
  double* Lf = nullptr;    // chol: L (Cholesky factor of X_rr, lower)
  long long total_s = 0, total_r = 0, total_t = 0, total_l = 0;
  int max_k = 0, max_r = 0;
};

// The DOFs left at the root of one instance and their dense block.
struct RootBlock {
  int off = 0, N = 0;           // rows root_idx[off, off + N)
  double* L = nullptr;          // chol: Cholesky factor (lower); mult: the block itself
  double* Linv = nullptr;       // chol: its inverse (lower)
};

struct FactorData {
  int mult = 0;             // 0: Schur/Cholesky form of Sigma; 1: multiply-only form
  std::vector<KernelParams> kp;     // per instance
  KernelParams* dkp = nullptr;      // device copy
  std::vector<LevelFactor> levels;  // index = depth (0 unused)
  int nroot = 0;                    // sum of the roots' N
  int* root_idx = nullptr;
  std::vector<RootBlock> roots;     // per instance (N may be 0)
  std::vector<double> logdet;       // per instance: log|F_i| (chol form)
  Arena arena;
};

struct Options {
  int n_prox = 256, prox_rings = 4;
  double r_near = 1.8, r_in = 1.75, r_out = 2.45, rq_alpha = 1.0;
  size_t mem_cap = 0;
  bool mixed = false;  // FP32 kernel entries and Schur-complement products
  bool strong_peeling = false;  // traces peeled in the strongly admissible format
};

}  // namespace rsf

namespace rsf {
// The single-vector log-likelihood of a factor recorded once as a HIP graph
// (gather into tree order, the solve sweep, the per-instance dot products,
// the scatter of alpha) and replayed for later calls.  The graph owns the
// device buffers and the pinned host copies of the launch descriptors it
// reads.
struct LoglikGraph {
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;  // the caller's stream the graph is replayed on
  hipStream_t cap = nullptr;     // the stream it was recorded on
  std::unique_ptr<Scratch> mem;
  std::vector<void*> pinned;
  double* zin = nullptr;    // caller order
  double* alpha = nullptr;  // caller order
  double* dots = nullptr;   // one per instance
  ~LoglikGraph();
};
}  // namespace rsf

struct rsf_factor_s {
  rsf::Tree tree;
  rsf::Options opt;
  int kernel = 0;
  double eps = 0.0;
  int leaf = 0;
  double theta[3] = {0, 0, 0};  // instance 0
  std::vector<double> thetas;   // 3 per instance
  double* px = nullptr;  // device, tree order
  double* py = nullptr;
  int* perm = nullptr;   // device copy of tree.perm
  rsf::Arena arena;      // points, permutation, proxy table
  double* prox_u = nullptr;  // device unit offsets of the proxy points (x then y)
  rsf::FactorData F;
  std::unique_ptr<rsf::FactorData> Frho;   // d/drho (d/dtheta_1 for anisotropic kernels)
  std::unique_ptr<rsf::FactorData> Frho2;  // d/dtheta_2 (anisotropic kernels only)
  std::unique_ptr<rsf::LoglikGraph> lgraph;
  int lgraph_state = 0;  // 0: not yet, 1: captured, -1: capture failed (eager from then on)
  int loglik_calls = 0;  // single-vector log-likelihood calls so far (the graph is recorded on the second)
};

namespace rsf {

// Builds one factorization over h's tree (Sections 2.1-2.3).
void build_factor(rsf_factor_s* h, FactorData& F, int mult, hipStream_t s);

// Sweeps over vector panels in tree order, row-major n x nc with leading
// dimension ld (row = DOF).  X is overwritten.
// inst_cols (host, one value per instance, or null): the leading panel
// columns each instance takes part in; the other columns of its rows are left
// undefined.
void sweep_solve(const rsf_factor_s* h, const FactorData& F, double* X, int nc, long long ld,
                 Scratch& scr, hipStream_t s, const int* inst_cols = nullptr);
// The library's second stream on the current device (for work that runs
// beside the caller's stream; never destroyed).
hipStream_t side_stream();

// X = B X and X = B^T X for F^-1 = B^T B (B: the up sweep, then L_root^-1)
void sweep_half_up(const rsf_factor_s* h, const FactorData& F, double* X, int nc, long long ld, Scratch& scr,
                   hipStream_t s, const int* inst_cols = nullptr);
void sweep_half_down(const rsf_factor_s* h, const FactorData& F, double* X, int nc, long long ld, Scratch& scr,
                     hipStream_t s, const int* inst_cols = nullptr);
void sweep_sqrt(const rsf_factor_s* h, const FactorData& F, const double* Y, double* V, int nc,
                long long ld, Scratch& scr, hipStream_t s);
void sweep_sqrt_t(const rsf_factor_s* h, const FactorData& F, double* X, double* Out, int nc,
                  long long ld, Scratch& scr, hipStream_t s);
void sweep_apply_mult(const rsf_factor_s* h, const FactorData& F, double* X, double* Y, int nc,
                      long long ld, Scratch& scr, hipStream_t s, const int* inst_cols = nullptr);

// user order column-major (ld) <-> tree order row-major panel (ldp)
void to_panel(const rsf_factor_s* h, const double* src, long long ld, double* P, int nc,
              long long ldp, hipStream_t s);
void from_panel(const rsf_factor_s* h, const double* P, int nc, long long ldp, double* dst,
                long long ld, hipStream_t s);

// Peeled traces of B B^T = Tr F^-1 and B F_rho B^T = Tr F^-1 F_rho, with
// F^-1 = B^T B (Section 3.2), one value per instance in tr_inv and tr_rho.
struct PeelStats {
  int levels = 0;
  int cols[32] = {0};
  int rank[32] = {0};
  int leaf_cols = 0;
};
// Traces per instance of B B^T (tr_inv) and B Frho B^T (tr_rho), and with Fd2
// also of B Fd2 B^T (tr_rho2), peeled jointly from one set of probes.
void peel_traces(const rsf_factor_s* h, double eps_peel, uint64_t seed, double* tr_inv,
                 double* tr_rho, PeelStats* st, hipStream_t s, const FactorData* Fd2 = nullptr,
                 double* tr_rho2 = nullptr);

// Score equations of every instance: g (3 values per instance, host); d_z in
// caller order (instances concatenated).  info (may be null) gets instance 0's
// split terms and the peeling statistics.
// Log profile likelihood of eq. prof (*ell) and, when g is not null, its
// gradient (3 values); info gets beta^T Sigma_i beta in q and the traces in t.
void profile_eval(rsf_factor_s* f, const double* d_z, double eps_peel, uint64_t seed, double* ell, double* g,
                  rsf_grad_info* info, void* stream);

// hutch_probes > 0: the traces by Hutchinson's estimator with that many
// Rademacher probes instead of peeling (eps_peel unused).
void grad_eval(rsf_factor_s* f, const double* d_z, double eps_peel, uint64_t seed, double* g,
               rsf_grad_info* info, void* stream, int hutch_probes = 0);

void fill_zero(double* p, long long n, hipStream_t s);
void copy_dev(double* dst, const double* src, long long n, hipStream_t s);

}  // namespace rsf
