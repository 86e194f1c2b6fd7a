/*
 * rsfgp — recursive skeletonization factorization (RSF) of a spatial
 * Gaussian-process covariance matrix on one AMD Instinct MI355X (gfx950), and
 * the log-likelihood and score equations built on it.
 *
 * The method is that of Minden, Damle, Ho and Ying, "Fast spatial Gaussian
 * process maximum likelihood estimation via skeletonization factorizations":
 *   - Section 2 (eq. rskelf): Sigma(theta) ~= F, a product of block
 *     unit-triangular skeletonization operators and a block-diagonal Cholesky
 *     factor, built level by level over a quadtree of the observation sites;
 *   - Section 2.4: F^-1 b, F^(1/2) w and log|F| from sweeps over the factors;
 *   - eq. loglikelihood and Algorithm 1: l(theta) = -1/2 z^T F^-1 z
 *     - 1/2 log|F| - (n/2) log 2 pi;
 *   - eq. gradient and Section 3: g_i = 1/2 z^T F^-1 Sigma_i F^-1 z
 *     - 1/2 Tr(F^-1 Sigma_i), the trace taken by matrix peeling (Section 3.2).
 *
 * Conventions for every entry point:
 *   - Return value: RSF_OK (0) or a negative rsf_status.  No C++ exception
 *     crosses this interface.  On error, outputs are left untouched and a
 *     message is available from rsf_last_error() (thread-local).
 *   - Pointers named d_* are device (HIP) pointers; all others are host.
 *     The caller owns every input and output buffer.  A factor handle owns
 *     all device memory it allocates until rsf_factor_destroy().
 *   - Vectors are in the caller's point order; the library keeps its tree
 *     permutation internal.  Blocks of vectors are column-major n x nrhs with
 *     leading dimension ld >= n.
 *   - `stream` is a hipStream_t (NULL = the default stream).  A handle is used
 *     by one stream at a time.  Calls that return a host scalar synchronise
 *     that stream.
 *   - theta = (rho, sigma2, nugget): length scale, variance, nugget.  The
 *     covariance is Sigma_ij = sigma2 k(|x_i - x_j| / rho) + nugget [i == j]
 *     with k from the Matern closed forms (eq. diffkernels) or the rational
 *     quadratic kernel (eq. rationalquadratic with the length scale).
 */
#ifndef RSFGP_H
#define RSFGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int rsf_status;
typedef struct rsf_factor_s* rsf_factor;

enum {
  RSF_OK = 0,
  RSF_E_INVALID = -1,   /* bad argument: n < 1, leaf < 1, eps <= 0, rho <= 0, ... */
  RSF_E_NOT_SPD = -2,   /* a diagonal block (or the root) lost positive definiteness
                           (the remark after eq. rskelf: a crude eps can do this) */
  RSF_E_OOM = -3,       /* device allocation failed or opts.mem_cap_bytes exceeded */
  RSF_E_HIP = -4,       /* a HIP runtime call failed */
  RSF_E_DUPLICATE = -5, /* two observation sites coincide (the nugget is a delta on
                           observation indices, so sites must be unique) */
  RSF_E_NONFINITE = -6  /* a coordinate or parameter is NaN or infinite */
};

/* Covariance families.  Matern nu = 1/2, 3/2, 5/2 closed forms (eq. diffkernels)
 * and the rational quadratic kernel with fixed shape alpha (opts.rq_alpha),
 * with theta = (rho, sigma2, nugget); and the anisotropic kernels of the
 * runtime experiments (eq. specmatern, eq. specrq: Matern 3/2 and RQ(alpha)
 * of the scaled distance dx^2 / theta_1^2 + dy^2 / theta_2^2, no variance
 * factor) with theta = (theta_1, theta_2, nugget); their score is with respect
 * to theta_1, theta_2 and the nugget. */
enum { RSF_MATERN12 = 0, RSF_MATERN32 = 1, RSF_MATERN52 = 2, RSF_RQ = 3, RSF_MATERN32_ANISO = 4, RSF_RQ_ANISO = 5 };

typedef struct {
  int n_prox;           /* proxy points per box (Section 2.3.1; Section 5 uses 256) */
  int prox_rings;       /* rings the proxy points are spread over (Fig. 3 draws an annulus) */
  double r_near;        /* near-field radius in box half-widths (Fig. 3: 1.8) */
  double prox_r_in;     /* inner / outer radius of the proxy annulus in half-widths */
  double prox_r_out;    /*   (Fig. 3: 1.75 and 2.45) */
  double rq_alpha;      /* shape alpha of the rational quadratic kernel */
  size_t mem_cap_bytes; /* 0 = unlimited; otherwise RSF_E_OOM beyond this many bytes */
  int precision;        /* RSF_FP64 (default) or RSF_MIXED: kernel entries evaluated in
                           FP32 and the Schur-complement products of the elimination
                           (X_sr, X_rr, W, X_ss) on FP32 matrix cores with FP32
                           accumulation; the IDs, the Cholesky factors of the redundant
                           blocks and of the root, log|F| and every sweep stay FP64 */
  int with_score;       /* 1: rsf_factor_create also factors the derivative matrix
                           Sigma_rho that rsf_grad needs (Algorithm 1; both
                           Sigma_theta1 and Sigma_theta2 for the anisotropic
                           kernels), on a second stream while Sigma is factored;
                           rsf_grad then reuses them.  0 (default): rsf_grad
                           factors them itself */
  int peeling;          /* how the score's traces are peeled (Section 3):
                           RSF_PEEL_WEAK (default): the weakly admissible format of
                           Section 3.2, every sibling block compressed (four probe
                           blocks per level, one per quadrant);
                           RSF_PEEL_STRONG: the strongly admissible format the remark
                           after Theorem 2 points to: only blocks of boxes that do not
                           touch (while their parents do) are compressed, their probes
                           coloured so that each sampled box sees one source box per
                           colour (36 colours on a complete quadtree, counter stream 2 of
                           the same Gaussian probes), the near field of touching leaves
                           never compressed and the leaves' diagonal blocks extracted with
                           colours that separate touching leaves */
} rsf_opts;

enum { RSF_FP64 = 0, RSF_MIXED = 1 };
enum { RSF_PEEL_WEAK = 0, RSF_PEEL_STRONG = 1 };

/* Fills *opts with the defaults above (n_prox 256, 4 rings, 1.8, 1.75, 2.45,
 * alpha 1, no cap, FP64, with_score 0, weak peeling).  Errors: RSF_E_INVALID if
 * opts is NULL. */
rsf_status rsf_opts_default(rsf_opts* opts);

/* Builds F ~= Sigma(theta) (Section 2, eq. rskelf; Algorithm 1, step "factor").
 *   d_points  device, n x 2 row-major FP64 (x_i, y_i), caller's order; copied.
 *   n         number of observations (>= 1).
 *   theta     host, p = 3 values (rho, sigma2, nugget).
 *   kernel    RSF_MATERN12 .. RSF_RQ.
 *   eps       relative tolerance of every interpolative decomposition
 *             (Definition "interpolative decomposition"), > 0.
 *   leaf      maximum points per quadtree leaf (n_occ of Section 5), >= 1.
 *   opts      NULL for defaults.
 *   out       receives the new handle (unchanged on error).
 * Errors: RSF_E_INVALID, RSF_E_NONFINITE, RSF_E_DUPLICATE, RSF_E_NOT_SPD,
 *         RSF_E_OOM, RSF_E_HIP. */
rsf_status rsf_factor_create(const double* d_points, int64_t n, const double* theta, int p,
                             int kernel, double eps, int leaf, const rsf_opts* opts,
                             void* stream, rsf_factor* out);

/* Releases every device buffer of f.  NULL is a no-op. */
void rsf_factor_destroy(rsf_factor f);

/* log|F| = 2 log|C| (Section 2.4), summed in a fixed order.  out: host scalar. */
rsf_status rsf_logdet(rsf_factor f, double* out);

/* d_x = F^-1 d_b for nrhs columns (Section 2.4, the F^-1 product formula).
 * d_b, d_x: device, n x nrhs column-major, leading dimension ld >= n; d_x may
 * alias d_b.  Errors: RSF_E_INVALID, RSF_E_OOM, RSF_E_HIP. */
rsf_status rsf_solve(rsf_factor f, const double* d_b, double* d_x, int64_t nrhs, int64_t ld,
                     void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): d_x =
 * F^-1 d_b exactly as rsf_solve (same arguments, layout and errors), but every
 * device work buffer (the tree-order panel, the sweep's level temporaries, the
 * launch descriptors) is carved from one fixed 64 MiB device array per GPU
 * that the library holds until the process ends.  The call makes no hipMalloc,
 * hipFree or other allocating call: launch descriptors travel through the
 * pinned staging ring that creating the handle already set up, and a level
 * shape that no earlier call has autotuned takes the fused per-box kernel
 * without timing trials.
 * Limit: 8 (n nrhs + r nrhs) bytes + 8 MiB of descriptors must fit in 64 MiB
 * (r: the largest number of redundant DOFs of one level, or the root size);
 * larger calls return RSF_E_INVALID before any device work, and a call whose
 * descriptors overrun the array returns RSF_E_INVALID with d_x untouched.
 * Every call on one GPU uses the same array, which keeps the previous call's
 * contents (nothing in it has to start at zero): calls on one stream are
 * ordered by the stream, but calls that overlap on one GPU (other streams, or
 * other host threads) race on it. */
rsf_status rsf_solve_noalloc(rsf_factor f, const double* d_b, double* d_x, int64_t nrhs, int64_t ld,
                             void* stream);

/* d_y = F d_x (Section 2.4).  Same layout rules as rsf_solve. */
rsf_status rsf_apply(rsf_factor f, const double* d_x, double* d_y, int64_t nrhs, int64_t ld,
                     void* stream);

/* d_z = F^(1/2) d_w with F = F^(1/2) (F^(1/2))^T (Section 2.4, the generalized
 * square root): a draw from N(0, F) when d_w ~ N(0, I).  Same layout rules. */
rsf_status rsf_apply_sqrt(rsf_factor f, const double* d_w, double* d_z, int64_t nrhs,
                          int64_t ld, void* stream);

/* Log-likelihood of observations d_z (device, n values, caller's order):
 * l = -1/2 z^T F^-1 z - 1/2 log|F| - (n/2) log 2 pi (eq. loglikelihood; the
 * reading of Algorithm 1 keeps the (n/2) factor of the equation).
 *   out            host scalar.
 *   d_alpha_or_null  if not NULL, receives F^-1 z (device, n values). */
rsf_status rsf_loglik(rsf_factor f, const double* d_z, double* out, double* d_alpha_or_null,
                      void* stream);

/* The first rsf_loglik call on a handle runs eagerly (and tunes the sweep's
 * level steps); the second records the same work (the solve sweep and the
 * dot products) as a HIP graph and replays it on the caller's stream, and
 * later calls on that stream replay it too (one graph launch instead of the
 * sweep's launches).  A handle used for one call records nothing.
 * *state: 0 = not recorded yet, 1 = recorded, -1 = recording failed or
 * disabled (RSFGP_NO_GRAPH set): calls stay eager. */
rsf_status rsf_graph_state(rsf_factor f, int* state);

typedef struct {
  double q[3];          /* 1/2 alpha^T Sigma_i alpha, alpha = F^-1 z */
  double t[3];          /* Tr(F^-1 Sigma_i) */
  double trace_inv;     /* Tr F^-1 (peeled) */
  int peel_levels;      /* quadtree levels peeled */
  int peel_cols[32];    /* probe columns per quadrant block at each level */
  int peel_rank[32];    /* largest sibling-block rank found at each level */
  int leaf_cols;        /* n_L of the extraction step */
  double seconds[4];    /* factor Sigma_rho, quadratic terms, peeling, total */
} rsf_grad_info;

/* Score equations g (eq. gradient; Algorithm 1): for theta = (rho, sigma2,
 * nugget) (eps_peel <= 0 selects the factorization tolerance eps),
 *   g_i = q_i - t_i / 2,  q_i = 1/2 alpha^T Sigma_i alpha,  t_i = Tr(F^-1 Sigma_i),
 * with Sigma_rho represented by its own skeletonization (multiply-only form),
 * Sigma_sigma2 = (Sigma - nugget I) / sigma2 and Sigma_nugget = I, and the
 * traces taken by matrix peeling (Section 3.2) of symmetric operators with the
 * traces of F^-1 and F^-1 F_rho (Section 3 allows any such symmetrized form):
 * B B^T and B F_rho B^T for F^-1 = B^T B (B: the up half of the solve sweep),
 * to relative tolerance eps_peel, with Gaussian probes from Philox4x32-10 keyed by
 * seed.  For the anisotropic kernels theta = (theta_1, theta_2, nugget): q and
 * t of theta_1 and theta_2 come from two derivative skeletonizations, and the
 * three operators B B^T, B F_theta1 B^T and B F_theta2 B^T are peeled from one
 * set of probes.
 *   d_z       device, n observations (caller's order).
 *   g         host, 3 values.
 *   info_or_null  host; receives the split terms and peeling statistics. */
rsf_status rsf_grad(rsf_factor f, const double* d_z, double eps_peel, uint64_t seed, double* g,
                    rsf_grad_info* info_or_null, void* stream);

/* ---- batches of independent instances ------------------------------------
 * One handle holds nb independent GP instances (their own sites, sizes and
 * theta; one kernel, eps, leaf and options).  Their quadtrees form one forest
 * whose depth-0 boxes are the instances' roots, so every level of the
 * factorization, of every sweep and of the peeling is one set of launches
 * over the boxes of all instances (the boxes of one level are independent,
 * Section 2.2).  Instance i occupies the caller-order range
 * [sum_{j<i} n_j, sum_{j<=i} n_j) of the single-vector calls above, which
 * act on the block-diagonal operator (rsf_logdet and rsf_loglik then return
 * the sums over the instances, rsf_grad is refused).  Ownership and errors as
 * for the single-instance calls.
 *   d_points  host array of nb device pointers, instance i: n[i] x 2 row-major.
 *   n         host, nb sizes (>= 1 each).
 *   theta     host, nb x p values (p = 3: rho, sigma2, nugget per instance). */
rsf_status rsf_factor_create_batched(const double* const* d_points, const int64_t* n, int nb,
                                     const double* theta, int p, int kernel, double eps, int leaf,
                                     const rsf_opts* opts, void* stream, rsf_factor* out);

/* *nb = number of instances of f (1 for a single-instance handle). */
rsf_status rsf_batch_size(rsf_factor f, int* nb);

/* out_nb (host, nb values) = log|F_i| per instance. */
rsf_status rsf_logdet_batched(rsf_factor f, double* out_nb);

/* out_nb (host, nb values) = l_i(theta_i) per instance; d_z: host array of nb
 * device pointers, instance i holds n[i] observations. */
rsf_status rsf_loglik_batched(rsf_factor f, const double* const* d_z, double* out_nb, void* stream);

/* g_nb_p (host, nb x 3 values) = the score of every instance, as rsf_grad.
 * Every level of every instance's peeling runs in one set of launches, each
 * instance with its own probe counts (its own ranks decide them, so a small
 * instance does not pay for the largest one's ranks); info_or_null receives
 * instance 0's split terms and, per level, the largest probe count and rank
 * over the instances. */
rsf_status rsf_grad_batched(rsf_factor f, const double* const* d_z, double eps_peel, uint64_t seed,
                            double* g_nb_p, rsf_grad_info* info_or_null, void* stream);

/* Log profile likelihood (eq. prof: the mean and the variance profiled out)
 *   l~ = -1/2 log|F| - n/2 log(z^T (F + 1 1^T)^-1 z) + n/2 (log n - 1 - log 2 pi)
 * and, when g_or_null is not NULL, its gradient (3 values, host)
 *   g~_i = -1/2 Tr(F^-1 Sigma_i) + n/2 beta^T Sigma_i beta / z^T beta,
 * beta = (F + 1 1^T)^-1 z by Sherman-Morrison from F^-1 z and F^-1 1, the
 * traces peeled as in rsf_grad (the paper's model fixes sigma2 = 1; the
 * derivative for sigma2 is returned all the same).  info_or_null gets
 * beta^T Sigma_i beta in q and the traces in t.  Single handles only.
 * Errors: RSF_E_INVALID, RSF_E_NOT_SPD if z^T (F + 1 1^T)^-1 z <= 0. */
rsf_status rsf_profile_loglik(rsf_factor f, const double* d_z, double eps_peel, uint64_t seed, double* ell,
                              double* g_or_null, rsf_grad_info* info_or_null, void* stream);

/* Conditional distribution of z' given z (the remark after Algorithm 1).
 * f: the handle factored on the joint sites [x'; x] (the n1 prediction sites
 * first, then the n2 observed sites, in that order in its points array);
 * f22: the handle on the observed sites x alone; both single-instance with
 * the same kernel and theta (else RSF_E_INVALID).  With
 * Sigma_12 v = the first block of F [0; v] and Sigma_22^-1 b = F22^-1 b:
 *   rsf_cond_mean:   d_mean (n1 x nrhs, column-major, ld n1) =
 *                    Sigma_12 Sigma_22^-1 d_z (d_z: n2 x nrhs, ld n2);
 *   rsf_cond_sample: d_dev (n1 x nrhs, ld n1) = S d_xi with
 *                    S S^T = Sigma_11 - Sigma_12 Sigma_22^-1 Sigma_12^T,
 *                    S = [I, -Sigma_12 Sigma_22^-1] F^(1/2); d_xi (n x nrhs,
 *                    ld n = n1 + n2) holds the caller's standard normal draws;
 *                    a conditional sample is the mean plus this deviation.
 * All arrays are device memory in the caller's site order. */
rsf_status rsf_cond_mean(rsf_factor f, rsf_factor f22, const double* d_z, double* d_mean, int64_t nrhs,
                         void* stream);
rsf_status rsf_cond_sample(rsf_factor f, rsf_factor f22, const double* d_xi, double* d_dev, int64_t nrhs,
                           void* stream);

/* The score with the traces by Hutchinson's estimator (eq. hutch) instead of
 * peeling: nprobe Rademacher vectors u_j (Philox4x32-10 keyed by seed, counter
 * (the DOF's tree-order index within its instance, j, 0, 1), sign from the
 * lowest bit of the first word; a batch draws what each instance draws alone),
 * w_j = B^T u_j for F^-1 = B^T B, Tr F^-1 ~= mean |w_j|^2 and
 * Tr F^-1 F_rho ~= mean w_j^T F_rho w_j (unbiased; the symmetric forms of
 * Section 3 in place of the unsymmetric Sigma^-1 Sigma_rho of Section 5.2).
 * Cheap and of statistical accuracy (the cross-check of peeling and the
 * early-iteration gradient of Section 5.2).  Arguments as rsf_grad /
 * rsf_grad_batched; info's peeling statistics are zero.  Errors:
 * RSF_E_INVALID for nprobe < 1, a null argument or the wrong handle kind. */
rsf_status rsf_grad_hutch(rsf_factor f, const double* d_z, int nprobe, uint64_t seed, double* g,
                          rsf_grad_info* info_or_null, void* stream);
rsf_status rsf_grad_hutch_batched(rsf_factor f, const double* const* d_z, int nprobe, uint64_t seed,
                                  double* g_nb_p, rsf_grad_info* info_or_null, void* stream);

typedef struct {
  int64_t n;
  int depth;            /* deepest level L */
  int nbox;             /* quadtree boxes */
  int root_size;        /* DOFs left for the dense root factor */
  int64_t factor_bytes; /* device bytes held by the factors */
} rsf_tree_info;

/* Tree introspection.  perm (host, n values or NULL) receives the tree order:
 * perm[t] = caller index of the t-th point. */
rsf_status rsf_tree_export(rsf_factor f, int32_t* perm, rsf_tree_info* info);

/* Skeletons of the boxes at depth `level` (1 .. depth) in breadth-first box
 * order: counts (host, boxes-at-level + 1 values or NULL) receives prefix
 * offsets, idx (host or NULL) the skeleton DOFs as caller indices in pivot
 * order.  *nbox_out (host) receives the number of boxes at that level. */
rsf_status rsf_skeleton_export(rsf_factor f, int level, int32_t* offsets, int32_t* idx,
                               int32_t* nbox_out);

/* Launch tracing (the library's profiling hook).  While enabled, every launch
 * of the batched matrix-core GEMM kernel (the kernel behind the sweeps and
 * the peeling products) is bracketed by HIP events recorded on the stream it
 * is launched on, and its algorithmic work is counted: 2 M N K flops and
 * 8 (M K + K N + M N [+ M N when C is read]) bytes per problem.
 * rsf_trace_read synchronises on the recorded events and returns the summed
 * kernel time (ms), flops, bytes and launch count (any output may be NULL);
 * reset != 0 clears the counters.  Launches from the library's own helper
 * threads are recorded too; one tracing client (caller) at a time. */
rsf_status rsf_trace_enable(int on);
rsf_status rsf_trace_read(double* gemm_ms, double* gemm_flops, double* gemm_bytes, int64_t* gemm_launches,
                          int reset);
/* The traced launches' busy time: the length (ms) of the union of their
 * intervals, which is below the summed time when launches on the library's
 * two streams overlap; as of the last rsf_trace_read (before its reset). */
rsf_status rsf_trace_busy(double* busy_ms);
/* The same GEMM time split by phase, as "phase:ms:flops;..." (NUL-terminated,
 * truncated to len - 1 characters); call after rsf_trace_read without reset.
 * Phases: factor, factor_rho, chol, sweep_solve, sweep_mult, sweep_sqrt,
 * peel_subtract, peel_gram, peel_lowrank. */
rsf_status rsf_trace_phases(char* buf, size_t len);
/* Algorithmic work booked per kernel while tracing was on, from host counts
 * (no events): "kernel:flops:bytes:dispatches;..." (NUL-terminated, truncated
 * to len - 1 characters).  The matrix-core kernels count as in rsf_trace_read
 * (a lower-triangle or triangular-operand product M N K flops); the fused
 * level steps 2 c r (2 k + r) flops per box of k skeleton and r redundant
 * DOFs and c columns (2 c k r to multiply down); the pivoting steps of the
 * interpolative decompositions 6 flops and 16 bytes per entry of the trailing
 * block they read and write.  Cleared by rsf_trace_read with reset. */
rsf_status rsf_trace_kernels(char* buf, size_t len);

/* Message describing the last error on this thread ("" if none). */
const char* rsf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RSFGP_H */
