// The C ABI of rsfgp (declared in include/rsfgp.h).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <map>
#include <mutex>
#include <thread>

#include "rsf.h"

using namespace rsf;

namespace {
thread_local std::string g_last_error;

int fail_with(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

template <class F>
int guarded(F&& f) {
  try {
    g_last_error.clear();
    f();
    return RSF_OK;
  } catch (const Error& e) {
    return fail_with(e.code, e.what());
  } catch (const std::bad_alloc&) {
    return fail_with(RSF_E_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail_with(RSF_E_HIP, e.what());
  }
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

void check_handle(rsf_factor f) { RSF_CHECK(f != nullptr, RSF_E_INVALID, "null factor handle"); }

void make_proxy_table(rsf_factor_s* h) {
  const Options& o = h->opt;
  const int per = o.n_prox / o.prox_rings;
  std::vector<double> u(2 * (size_t)o.n_prox);
  const double two_pi = 6.283185307179586476925286766559;
  for (int q = 0; q < o.prox_rings; ++q) {
    const double rad = o.r_in + (o.r_out - o.r_in) * (q + 0.5) / o.prox_rings;
    for (int j = 0; j < per; ++j) {
      const double ang = two_pi * (j + (double)q / o.prox_rings) / per;
      u[q * per + j] = rad * std::cos(ang);
      u[o.n_prox + q * per + j] = rad * std::sin(ang);
    }
  }
  h->prox_u = h->arena.make<double>(u.size());
  RSF_HIP(hipMemcpy(h->prox_u, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice));
}
}  // namespace

extern "C" {

const char* rsf_last_error(void) { return g_last_error.c_str(); }

rsf_status rsf_opts_default(rsf_opts* o) {
  if (!o) return fail_with(RSF_E_INVALID, "opts is NULL");
  o->n_prox = 256;
  o->prox_rings = 4;
  o->r_near = 1.8;
  o->prox_r_in = 1.75;
  o->prox_r_out = 2.45;
  o->rq_alpha = 1.0;
  o->mem_cap_bytes = 0;
  o->precision = RSF_FP64;
  o->with_score = 0;
  o->peeling = RSF_PEEL_WEAK;
  return RSF_OK;
}

static void check_theta(const double* theta) {
  for (int i = 0; i < 3; ++i) RSF_CHECK(std::isfinite(theta[i]), RSF_E_NONFINITE, "non-finite theta");
  RSF_CHECK(theta[0] > 0.0, RSF_E_INVALID, "rho (theta_1) must be > 0");
  RSF_CHECK(theta[1] > 0.0, RSF_E_INVALID, "sigma2 (theta_2) must be > 0");
}

// Shared by the single and the batched constructor: host copies of every
// instance's sites, 3 parameters per instance.
// Argument checks that need no device access (run before any copy).
static void check_args(const double* thetas, int ni, int kernel, double eps, int leaf) {
  RSF_CHECK(leaf >= 1, RSF_E_INVALID, "leaf must be >= 1");
  RSF_CHECK(kernel >= RSF_MATERN12 && kernel <= RSF_RQ_ANISO, RSF_E_INVALID, "unknown kernel");
  RSF_CHECK(std::isfinite(eps), RSF_E_NONFINITE, "non-finite eps");
  RSF_CHECK(eps > 0.0, RSF_E_INVALID, "eps must be > 0");
  for (int i = 0; i < ni; ++i) check_theta(thetas + 3 * i);
}

static rsf_factor_s* create_handle(const std::vector<std::vector<double>>& xy, const std::vector<int64_t>& ns,
                                   const double* thetas, int kernel, double eps, int leaf, const rsf_opts* opts,
                                   hipStream_t s) {
  const int ni = (int)ns.size();
  check_args(thetas, ni, kernel, eps, leaf);
  rsf_opts o;
  if (opts)
    o = *opts;
  else
    rsf_opts_default(&o);
  RSF_CHECK(o.n_prox >= 1 && o.prox_rings >= 1 && o.n_prox % o.prox_rings == 0, RSF_E_INVALID,
            "n_prox must be a positive multiple of prox_rings");
  RSF_CHECK(o.r_near > 0 && o.prox_r_in > 0 && o.prox_r_out >= o.prox_r_in && o.rq_alpha > 0, RSF_E_INVALID,
            "bad proxy geometry or rq_alpha");
  RSF_CHECK(o.precision == RSF_FP64 || o.precision == RSF_MIXED, RSF_E_INVALID, "unknown precision");
  RSF_CHECK(o.with_score == 0 || o.with_score == 1, RSF_E_INVALID, "with_score must be 0 or 1");
  RSF_CHECK(o.peeling == RSF_PEEL_WEAK || o.peeling == RSF_PEEL_STRONG, RSF_E_INVALID, "unknown peeling form");
  RSF_CHECK(!(o.precision == RSF_MIXED && kernel >= RSF_MATERN32_ANISO), RSF_E_INVALID,
            "mixed precision takes the isotropic kernels only");
  std::unique_ptr<rsf_factor_s> h(new rsf_factor_s());
  h->opt.n_prox = o.n_prox;
  h->opt.prox_rings = o.prox_rings;
  h->opt.r_near = o.r_near;
  h->opt.r_in = o.prox_r_in;
  h->opt.r_out = o.prox_r_out;
  h->opt.rq_alpha = o.rq_alpha;
  h->opt.mem_cap = o.mem_cap_bytes;
  h->opt.mixed = o.precision == RSF_MIXED;
  h->opt.strong_peeling = o.peeling == RSF_PEEL_STRONG;
  h->arena.cap = o.mem_cap_bytes;
  h->kernel = kernel;
  h->eps = eps;
  h->leaf = leaf;
  h->thetas.assign(thetas, thetas + 3 * ni);
  for (int i = 0; i < 3; ++i) h->theta[i] = thetas[i];
  std::vector<const double*> ptrs(ni);
  for (int i = 0; i < ni; ++i) ptrs[i] = xy[i].data();
  h->tree = build_forest(ptrs, ns, leaf);
  const int64_t n = h->tree.n;
  std::vector<double> px(n), py(n);
  for (int64_t t = 0; t < n; ++t) {
    // caller index c = ioff[i] + local index of instance i
    const int64_t c = h->tree.perm[t];
    const int i = (int)(std::upper_bound(h->tree.ioff.begin(), h->tree.ioff.end(), c) - h->tree.ioff.begin()) - 1;
    const int64_t u = c - h->tree.ioff[i];
    px[t] = xy[i][2 * (size_t)u];
    py[t] = xy[i][2 * (size_t)u + 1];
  }
  h->px = h->arena.make<double>(n);
  h->py = h->arena.make<double>(n);
  h->perm = h->arena.make<int>(n);
  RSF_HIP(hipMemcpy(h->px, px.data(), n * sizeof(double), hipMemcpyHostToDevice));
  RSF_HIP(hipMemcpy(h->py, py.data(), n * sizeof(double), hipMemcpyHostToDevice));
  RSF_HIP(hipMemcpy(h->perm, h->tree.perm.data(), n * sizeof(int), hipMemcpyHostToDevice));
  make_proxy_table(h.get());
  if (o.with_score) {
    // Sigma and Sigma_rho are independent factorizations whose level loops
    // are mostly latency-bound: Sigma_rho is built by a second host thread on
    // the library's side stream while this thread builds Sigma on s
    RSF_HIP(hipStreamSynchronize(s));
    hipStream_t s2 = side_stream();
    h->Frho.reset(new FactorData());
    std::exception_ptr err;
    std::thread th([&] {
      try {
        build_factor(h.get(), *h->Frho, 1, s2);
        if (kernel >= RSF_MATERN32_ANISO) {
          h->Frho2.reset(new FactorData());
          build_factor(h.get(), *h->Frho2, 2, s2);
        }
        RSF_HIP(hipStreamSynchronize(s2));
      } catch (...) {
        err = std::current_exception();
      }
    });
    try {
      build_factor(h.get(), h->F, 0, s);
    } catch (...) {
      th.join();
      throw;
    }
    th.join();
    if (err) std::rethrow_exception(err);
  } else {
    build_factor(h.get(), h->F, 0, s);
  }
  RSF_HIP(hipStreamSynchronize(s));
  return h.release();
}

rsf_status rsf_factor_create(const double* d_points, int64_t n, const double* theta, int p, int kernel,
                             double eps, int leaf, const rsf_opts* opts, void* stream, rsf_factor* out) {
  return guarded([&] {
    RSF_CHECK(out != nullptr && d_points != nullptr && theta != nullptr, RSF_E_INVALID, "null argument");
    RSF_CHECK(p == 3, RSF_E_INVALID, "theta must hold 3 values (rho, sigma2, nugget)");
    RSF_CHECK(n >= 1, RSF_E_INVALID, "n must be >= 1");
    check_args(theta, 1, kernel, eps, leaf);
    hipStream_t s = as_stream(stream);
    std::vector<std::vector<double>> xy(1, std::vector<double>(2 * (size_t)n));
    RSF_HIP(hipMemcpyAsync(xy[0].data(), d_points, xy[0].size() * sizeof(double), hipMemcpyDeviceToHost, s));
    RSF_HIP(hipStreamSynchronize(s));
    *out = create_handle(xy, std::vector<int64_t>{n}, theta, kernel, eps, leaf, opts, s);
  });
}

rsf_status rsf_factor_create_batched(const double* const* d_points, const int64_t* n, int nb, const double* theta,
                                     int p, int kernel, double eps, int leaf, const rsf_opts* opts, void* stream,
                                     rsf_factor* out) {
  return guarded([&] {
    RSF_CHECK(out != nullptr && d_points != nullptr && n != nullptr && theta != nullptr, RSF_E_INVALID,
              "null argument");
    RSF_CHECK(nb >= 1, RSF_E_INVALID, "nb must be >= 1");
    RSF_CHECK(p == 3, RSF_E_INVALID, "theta must hold 3 values per instance (rho, sigma2, nugget)");
    check_args(theta, nb, kernel, eps, leaf);
    hipStream_t s = as_stream(stream);
    std::vector<std::vector<double>> xy(nb);
    std::vector<int64_t> ns(n, n + nb);
    for (int i = 0; i < nb; ++i) {
      RSF_CHECK(d_points[i] != nullptr, RSF_E_INVALID, "null point array of instance " + std::to_string(i));
      RSF_CHECK(ns[i] >= 1, RSF_E_INVALID, "n must be >= 1 (instance " + std::to_string(i) + ")");
      xy[i].resize(2 * (size_t)ns[i]);
      RSF_HIP(hipMemcpyAsync(xy[i].data(), d_points[i], xy[i].size() * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    RSF_HIP(hipStreamSynchronize(s));
    *out = create_handle(xy, ns, theta, kernel, eps, leaf, opts, s);
  });
}

rsf_status rsf_batch_size(rsf_factor f, int* nb) {
  return guarded([&] {
    check_handle(f);
    RSF_CHECK(nb != nullptr, RSF_E_INVALID, "null output");
    *nb = f->tree.ninst;
  });
}

void rsf_factor_destroy(rsf_factor f) {
  if (!f) return;
  (void)hipDeviceSynchronize();
  delete f;
}

rsf_status rsf_logdet(rsf_factor f, double* out) {
  return guarded([&] {
    check_handle(f);
    RSF_CHECK(out != nullptr, RSF_E_INVALID, "null output");
    double sum = 0.0;
    for (double v : f->F.logdet) sum += v;
    *out = sum;
  });
}

rsf_status rsf_logdet_batched(rsf_factor f, double* out_nb) {
  return guarded([&] {
    check_handle(f);
    RSF_CHECK(out_nb != nullptr, RSF_E_INVALID, "null output");
    for (int i = 0; i < f->tree.ninst; ++i) out_nb[i] = f->F.logdet[i];
  });
}

static void check_block(rsf_factor f, const void* a, const void* b, int64_t nrhs, int64_t ld) {
  check_handle(f);
  RSF_CHECK(a != nullptr && b != nullptr, RSF_E_INVALID, "null vector");
  RSF_CHECK(nrhs >= 0, RSF_E_INVALID, "nrhs must be >= 0");
  RSF_CHECK(ld >= f->tree.n, RSF_E_INVALID, "ld must be >= n");
  RSF_CHECK(nrhs < (int64_t(1) << 24), RSF_E_INVALID, "nrhs too large");
}

rsf_status rsf_solve(rsf_factor f, const double* d_b, double* d_x, int64_t nrhs, int64_t ld, void* stream) {
  return guarded([&] {
    check_block(f, d_b, d_x, nrhs, ld);
    if (nrhs == 0) return;
    hipStream_t s = as_stream(stream);
    Scratch scr(s);
    const int nc = (int)nrhs;
    double* P = scr.make<double>((size_t)f->tree.n * nc);
    to_panel(f, d_b, ld, P, nc, nc, s);
    sweep_solve(f, f->F, P, nc, nc, scr, s);
    from_panel(f, P, nc, nc, d_x, ld, s);
  });
}

}  // extern "C"

// ---- the solve without device allocation
// Work space of rsf_solve_noalloc: one fixed array per GPU, held until the
// process ends.  Host code never uses the array's name as an address: the
// device address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept in g_noalloc_ptr.
namespace {
constexpr size_t NOALLOC_BYTES = size_t(64) << 20;
// bytes kept free for launch descriptors and tile tables beside the panel and
// the level temporaries
constexpr size_t NOALLOC_DESC_RESERVE = size_t(8) << 20;
static __device__ __align__(256) char scratch[NOALLOC_BYTES];
std::mutex g_noalloc_mu;
std::map<int, char*> g_noalloc_ptr;  // device ordinal -> its copy of scratch

char* noalloc_scratch() {
  int dev = 0;
  RSF_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc_ptr.find(dev);
  if (it != g_noalloc_ptr.end()) return it->second;
  void* ptr = nullptr;
  RSF_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  RSF_CHECK(ptr != nullptr, RSF_E_HIP, "no device address for the no-allocation work space");
  g_noalloc_ptr[dev] = static_cast<char*>(ptr);
  return static_cast<char*>(ptr);
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
}  // namespace

extern "C" {

rsf_status rsf_solve_noalloc(rsf_factor f, const double* d_b, double* d_x, int64_t nrhs, int64_t ld, void* stream) {
  return guarded([&] {
    check_block(f, d_b, d_x, nrhs, ld);
    if (nrhs == 0) return;
    const int nc = (int)nrhs;
    const long long n = f->tree.n;
    long long maxr = 1;
    for (size_t d = 1; d < f->F.levels.size(); ++d) maxr = std::max(maxr, f->F.levels[d].total_r);
    maxr = std::max<long long>(maxr, f->F.nroot);
    // the tree-order panel and the sweep's level temporaries, plus room for
    // the launch descriptors
    const size_t need = align256((size_t)n * nc * sizeof(double)) + align256((size_t)maxr * nc * sizeof(double)) +
                        NOALLOC_DESC_RESERVE;
    RSF_CHECK(need <= NOALLOC_BYTES, RSF_E_INVALID,
              "rsf_solve_noalloc: n = " + std::to_string(n) + " with nrhs = " + std::to_string(nc) + " needs " +
                  std::to_string(need) + " bytes of work space, more than its fixed " +
                  std::to_string(NOALLOC_BYTES) + " (use rsf_solve, or fewer columns per call)");
    char* ptr = noalloc_scratch();
    hipStream_t s = as_stream(stream);
    NoAllocScope na;
    Scratch scr(s, ptr, NOALLOC_BYTES);
    double* P = scr.make<double>((size_t)n * nc);
    to_panel(f, d_b, ld, P, nc, nc, s);
    sweep_solve(f, f->F, P, nc, nc, scr, s);
    from_panel(f, P, nc, nc, d_x, ld, s);
  });
}

rsf_status rsf_apply(rsf_factor f, const double* d_x, double* d_y, int64_t nrhs, int64_t ld, void* stream) {
  return guarded([&] {
    check_block(f, d_x, d_y, nrhs, ld);
    if (nrhs == 0) return;
    hipStream_t s = as_stream(stream);
    Scratch scr(s);
    const int nc = (int)nrhs;
    const size_t sz = (size_t)f->tree.n * nc;
    double* P = scr.make<double>(sz);
    double* Q = scr.make<double>(sz);
    to_panel(f, d_x, ld, P, nc, nc, s);
    sweep_sqrt_t(f, f->F, P, Q, nc, nc, scr, s);
    sweep_sqrt(f, f->F, Q, P, nc, nc, scr, s);
    from_panel(f, P, nc, nc, d_y, ld, s);
  });
}

rsf_status rsf_apply_sqrt(rsf_factor f, const double* d_w, double* d_z, int64_t nrhs, int64_t ld,
                          void* stream) {
  return guarded([&] {
    check_block(f, d_w, d_z, nrhs, ld);
    if (nrhs == 0) return;
    hipStream_t s = as_stream(stream);
    Scratch scr(s);
    const int nc = (int)nrhs;
    const size_t sz = (size_t)f->tree.n * nc;
    double* P = scr.make<double>(sz);
    double* Q = scr.make<double>(sz);
    to_panel(f, d_w, ld, P, nc, nc, s);
    sweep_sqrt(f, f->F, P, Q, nc, nc, scr, s);
    from_panel(f, Q, nc, nc, d_z, ld, s);
  });
}

// ---- conditional distribution (the remark after Algorithm 1)
// F factors the joint covariance of [x'; x] (the n1 prediction sites first),
// F22 that of the observed sites x.  Sigma_12 v is the first block of
// F [0; v]; Sigma_22^-1 b is F22^-1 b.
static void check_pair(rsf_factor f, rsf_factor f22) {
  check_handle(f);
  check_handle(f22);
  RSF_CHECK(f->tree.ninst == 1 && f22->tree.ninst == 1, RSF_E_INVALID, "conditional sampling takes single handles");
  RSF_CHECK(f->tree.n > f22->tree.n, RSF_E_INVALID, "the joint handle must hold more sites than the observed one");
  RSF_CHECK(f->kernel == f22->kernel && f->theta[0] == f22->theta[0] && f->theta[1] == f22->theta[1] &&
                f->theta[2] == f22->theta[2],
            RSF_E_INVALID, "the joint and observed handles must share kernel and theta");
}

// out(i, c) = Y(i, c) - U(i, c) for the first n1 rows (Y: leading dimension ldy)
__global__ void cond_dev_kernel(const double* __restrict__ Y, long long ldy, const double* __restrict__ U, long long n1,
                                int nc, double* __restrict__ out) {
  const long long tot = n1 * nc;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
    const long long c = e / n1, i = e - c * n1;
    out[e] = Y[c * ldy + i] - U[e];
  }
}

// Y (n1 x nc, leading dimension ld1) = first n1 rows of F [0; F22^-1 B],
// B: n2 x nc with leading dimension ldb (device, caller order)
static void sigma12_sigma22inv(rsf_factor f, rsf_factor f22, const double* B, long long ldb, double* Y, long long ld1,
                               int nc, Scratch& scr, hipStream_t s) {
  const long long n = f->tree.n, n2 = f22->tree.n, n1 = n - n2;
  double* V = scr.make<double>((size_t)n * nc);
  double* P2 = scr.make<double>((size_t)n2 * nc);
  double* P = scr.make<double>((size_t)n * nc);
  double* Q = scr.make<double>((size_t)n * nc);
  fill_zero(V, n * nc, s);
  to_panel(f22, B, ldb, P2, nc, nc, s);
  sweep_solve(f22, f22->F, P2, nc, nc, scr, s);
  from_panel(f22, P2, nc, nc, V + n1, n, s);  // rows n1 .. n - 1 of V
  to_panel(f, V, n, P, nc, nc, s);
  sweep_sqrt_t(f, f->F, P, Q, nc, nc, scr, s);
  sweep_sqrt(f, f->F, Q, P, nc, nc, scr, s);
  from_panel(f, P, nc, nc, V, n, s);
  RSF_HIP(hipMemcpy2DAsync(Y, ld1 * sizeof(double), V, n * sizeof(double), n1 * sizeof(double), nc,
                           hipMemcpyDeviceToDevice, s));
}

namespace rsf {
LoglikGraph::~LoglikGraph() {
  if (exec) (void)hipGraphExecDestroy(exec);
  mem.reset();
  for (void* p : pinned) (void)hipHostFree(p);
  if (cap) (void)hipStreamDestroy(cap);
}
}  // namespace rsf

// The tree-order solve and dot products of loglik_all, recorded on stream s
// into f->lgraph (after an eager call has tuned every level step of this
// shape).  On any failure the capture is abandoned and the factor stays eager.
static void capture_loglik(rsf_factor f, hipStream_t s) {
  if (std::getenv("RSFGP_NO_GRAPH")) {
    f->lgraph_state = -1;
    return;
  }
  const Tree& t = f->tree;
  const long long n = t.n;
  std::unique_ptr<LoglikGraph> g(new LoglikGraph());
  g->stream = s;
  // recorded on a stream of its own (the legacy default stream cannot be
  // captured); replays go to the caller's stream
  RSF_HIP(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking));
  const hipStream_t cs = g->cap;
  // the graph's buffers are released in the caller's stream order (the
  // recording stream is destroyed with the graph)
  g->mem.reset(new Scratch(s));
  Scratch& m = *g->mem;
  g->zin = m.make<double>(n);
  g->alpha = m.make<double>(n);
  g->dots = m.make<double>(t.ninst);
  double* Z = m.make<double>(n);
  double* A = m.make<double>(n);
  TracePause tp;
  // every earlier use of the pool's memory has finished: allocations made
  // while recording need no stream synchronisation
  RSF_HIP(hipDeviceSynchronize());
  std::string why;
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) == hipSuccess;
  if (!ok) why = "begin capture";
  if (ok) {
    upload_capture_begin(&g->pinned);
    pool_sync_free(true);
    try {
      to_panel(f, g->zin, n, Z, 1, 1, cs);
      copy_dev(A, Z, n, cs);
      sweep_solve(f, f->F, A, 1, 1, m, cs);
      for (int i = 0; i < t.ninst; ++i)
        device_dot(Z + t.ioff[i], A + t.ioff[i], t.ioff[i + 1] - t.ioff[i], g->dots + i, m, cs);
      from_panel(f, A, 1, 1, g->alpha, n, cs);
    } catch (const std::exception& e) {
      ok = false;
      why = e.what();
    } catch (...) {
      ok = false;
      why = "exception";
    }
    pool_sync_free(false);
    upload_capture_end();
    hipGraph_t graph = nullptr;
    const hipError_t ee = hipStreamEndCapture(cs, &graph);
    if (ok && (ee != hipSuccess || !graph)) {
      ok = false;
      why = std::string("end capture: ") + hipGetErrorString(ee);
    }
    if (ok && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      ok = false;
      why = "instantiate";
    }
    if (graph) (void)hipGraphDestroy(graph);
  }
  (void)hipGetLastError();
  if (!ok && std::getenv("RSFGP_GRAPH_DEBUG")) fprintf(stderr, "[graph] not recorded: %s\n", why.c_str());
  if (ok) {
    f->lgraph = std::move(g);
    f->lgraph_state = 1;
  } else {
    f->lgraph_state = -1;
  }
}

// l_i = -1/2 z_i^T alpha_i - 1/2 log|F_i| - (n_i / 2) log 2 pi for every
// instance, alpha = F^-1 z (eq. loglikelihood); d_z in caller order (all
// instances concatenated).
static void loglik_all(rsf_factor f, const double* d_z, double* out, double* d_alpha, hipStream_t s) {
  const Tree& t = f->tree;
  const long long n = t.n;
  const int ni = t.ninst;
  const double log2pi = 1.8378770664093454835606594728112;
  // the graph is recorded on a handle's second call (the first one runs
  // eagerly and tunes every level step of this shape), so a handle used once
  // never pays for a recording it would not replay
  if (f->lgraph_state == 0 && f->loglik_calls >= 1) capture_loglik(f, s);
  ++f->loglik_calls;
  if (f->lgraph && f->lgraph->stream == s) {
    LoglikGraph& g = *f->lgraph;
    RSF_HIP(hipMemcpyAsync(g.zin, d_z, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    RSF_HIP(hipGraphLaunch(g.exec, s));
    std::vector<double> zt(ni);
    RSF_HIP(hipMemcpyAsync(zt.data(), g.dots, ni * sizeof(double), hipMemcpyDeviceToHost, s));
    if (d_alpha) RSF_HIP(hipMemcpyAsync(d_alpha, g.alpha, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    RSF_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < ni; ++i)
      out[i] = -0.5 * zt[i] - 0.5 * f->F.logdet[i] - 0.5 * (double)(t.ioff[i + 1] - t.ioff[i]) * log2pi;
    return;
  }
  Scratch scr(s);
  double* Z = scr.make<double>(n);
  double* A = scr.make<double>(n);
  double* dot = scr.make<double>(ni);
  to_panel(f, d_z, n, Z, 1, 1, s);
  copy_dev(A, Z, n, s);
  sweep_solve(f, f->F, A, 1, 1, scr, s);
  // instance i is the tree-order range [ioff[i], ioff[i + 1])
  for (int i = 0; i < ni; ++i)
    device_dot(Z + t.ioff[i], A + t.ioff[i], t.ioff[i + 1] - t.ioff[i], dot + i, scr, s);
  std::vector<double> zt(ni);
  RSF_HIP(hipMemcpyAsync(zt.data(), dot, ni * sizeof(double), hipMemcpyDeviceToHost, s));
  RSF_HIP(hipStreamSynchronize(s));
  if (d_alpha) from_panel(f, A, 1, 1, d_alpha, n, s);
  for (int i = 0; i < ni; ++i)
    out[i] = -0.5 * zt[i] - 0.5 * f->F.logdet[i] - 0.5 * (double)(t.ioff[i + 1] - t.ioff[i]) * log2pi;
}

rsf_status rsf_graph_state(rsf_factor f, int* state) {
  return guarded([&] {
    check_handle(f);
    RSF_CHECK(state != nullptr, RSF_E_INVALID, "null output");
    *state = f->lgraph_state;
  });
}

// The caller's per-instance vectors, concatenated in caller order.
static double* gather_instances(rsf_factor f, const double* const* d_z, Scratch& scr, hipStream_t s) {
  const Tree& t = f->tree;
  double* Z = scr.make<double>(t.n);
  for (int i = 0; i < t.ninst; ++i) {
    RSF_CHECK(d_z[i] != nullptr, RSF_E_INVALID, "null vector of instance " + std::to_string(i));
    RSF_HIP(hipMemcpyAsync(Z + t.ioff[i], d_z[i], (t.ioff[i + 1] - t.ioff[i]) * sizeof(double),
                           hipMemcpyDeviceToDevice, s));
  }
  return Z;
}

rsf_status rsf_loglik(rsf_factor f, const double* d_z, double* out, double* d_alpha_or_null, void* stream) {
  return guarded([&] {
    check_handle(f);
    RSF_CHECK(d_z != nullptr && out != nullptr, RSF_E_INVALID, "null argument");
    std::vector<double> l(f->tree.ninst);
    loglik_all(f, d_z, l.data(), d_alpha_or_null, as_stream(stream));
    double sum = 0.0;  // independent instances: the joint log-likelihood
    for (double v : l) sum += v;
    *out = sum;
  });
}

rsf_status rsf_loglik_batched(rsf_factor f, const double* const* d_z, double* out_nb, void* stream) {
  return guarded([&] {
    check_handle(f);
    RSF_CHECK(d_z != nullptr && out_nb != nullptr, RSF_E_INVALID, "null argument");
    hipStream_t s = as_stream(stream);
    Scratch scr(s);
    const double* Z = gather_instances(f, d_z, scr, s);
    loglik_all(f, Z, out_nb, nullptr, s);
  });
}

rsf_status rsf_tree_export(rsf_factor f, int32_t* perm, rsf_tree_info* info) {
  return guarded([&] {
    check_handle(f);
    if (perm) std::memcpy(perm, f->tree.perm.data(), f->tree.n * sizeof(int32_t));
    if (info) {
      info->n = f->tree.n;
      info->depth = f->tree.maxdepth;
      info->nbox = f->tree.nbox();
      info->root_size = f->F.nroot;
      info->factor_bytes = (int64_t)f->F.arena.bytes;
    }
  });
}

rsf_status rsf_skeleton_export(rsf_factor f, int level, int32_t* offsets, int32_t* idx, int32_t* nbox_out) {
  return guarded([&] {
    check_handle(f);
    RSF_CHECK(level >= 1 && level <= f->tree.maxdepth, RSF_E_INVALID, "level out of range");
    const LevelFactor& L = f->F.levels[level];
    if (nbox_out) *nbox_out = L.nb;
    if (offsets)
      for (int i = 0; i <= L.nb; ++i) offsets[i] = (int32_t)L.s_off[i];
    if (idx && L.total_s > 0) {
      std::vector<int> tmp(L.total_s);
      RSF_HIP(hipMemcpy(tmp.data(), L.S, L.total_s * sizeof(int), hipMemcpyDeviceToHost));
      for (long long q = 0; q < L.total_s; ++q) idx[q] = f->tree.perm[tmp[q]];
    }
  });
}

rsf_status rsf_trace_enable(int on) {
  return guarded([&] { trace_enable(on != 0); });
}

rsf_status rsf_trace_read(double* gemm_ms, double* gemm_flops, double* gemm_bytes, int64_t* gemm_launches,
                          int reset) {
  return guarded([&] {
    long long l = 0;
    trace_read(gemm_ms, gemm_flops, gemm_bytes, &l, reset != 0);
    if (gemm_launches) *gemm_launches = l;
  });
}

rsf_status rsf_trace_busy(double* busy_ms) {
  return guarded([&] {
    RSF_CHECK(busy_ms != nullptr, RSF_E_INVALID, "null output");
    *busy_ms = trace_busy();
  });
}

rsf_status rsf_trace_phases(char* buf, size_t len) {
  return guarded([&] {
    RSF_CHECK(buf != nullptr && len > 0, RSF_E_INVALID, "null buffer");
    const std::string t = trace_tags();
    std::strncpy(buf, t.c_str(), len - 1);
    buf[len - 1] = 0;
  });
}

rsf_status rsf_trace_kernels(char* buf, size_t len) {
  return guarded([&] {
    RSF_CHECK(buf != nullptr && len > 0, RSF_E_INVALID, "null buffer");
    const std::string t = trace_kernels();
    std::strncpy(buf, t.c_str(), len - 1);
    buf[len - 1] = 0;
  });
}

rsf_status rsf_grad(rsf_factor f, const double* d_z, double eps_peel, uint64_t seed, double* g,
                    rsf_grad_info* info, void* stream) {
  return guarded([&] {
    check_handle(f);
    RSF_CHECK(f->tree.ninst == 1, RSF_E_INVALID, "a batched handle takes rsf_grad_batched");
    grad_eval(f, d_z, eps_peel, seed, g, info, stream);
  });
}

rsf_status rsf_profile_loglik(rsf_factor f, const double* d_z, double eps_peel, uint64_t seed, double* ell,
                              double* g_or_null, rsf_grad_info* info_or_null, void* stream) {
  return guarded([&] {
    check_handle(f);
    profile_eval(f, d_z, eps_peel, seed, ell, g_or_null, info_or_null, stream);
  });
}

rsf_status rsf_cond_mean(rsf_factor f, rsf_factor f22, const double* d_z, double* d_mean, int64_t nrhs,
                         void* stream) {
  return guarded([&] {
    check_pair(f, f22);
    RSF_CHECK(d_z != nullptr && d_mean != nullptr, RSF_E_INVALID, "null vector");
    RSF_CHECK(nrhs >= 0 && nrhs < (int64_t(1) << 24), RSF_E_INVALID, "bad nrhs");
    if (nrhs == 0) return;
    hipStream_t s = as_stream(stream);
    Scratch scr(s);
    const long long n1 = f->tree.n - f22->tree.n;
    sigma12_sigma22inv(f, f22, d_z, f22->tree.n, d_mean, n1, (int)nrhs, scr, s);
  });
}

rsf_status rsf_cond_sample(rsf_factor f, rsf_factor f22, const double* d_xi, double* d_dev, int64_t nrhs,
                           void* stream) {
  return guarded([&] {
    check_pair(f, f22);
    RSF_CHECK(d_xi != nullptr && d_dev != nullptr, RSF_E_INVALID, "null vector");
    RSF_CHECK(nrhs >= 0 && nrhs < (int64_t(1) << 24), RSF_E_INVALID, "bad nrhs");
    if (nrhs == 0) return;
    hipStream_t s = as_stream(stream);
    Scratch scr(s);
    const long long n = f->tree.n, n1 = n - f22->tree.n;
    const int nc = (int)nrhs;
    // y = F^(1/2) xi; deviation = y_1 - Sigma_12 Sigma_22^-1 y_2
    double* P = scr.make<double>((size_t)n * nc);
    double* Q = scr.make<double>((size_t)n * nc);
    double* Yc = scr.make<double>((size_t)n * nc);
    double* U = scr.make<double>((size_t)n1 * nc);
    to_panel(f, d_xi, n, P, nc, nc, s);
    sweep_sqrt(f, f->F, P, Q, nc, nc, scr, s);
    from_panel(f, Q, nc, nc, Yc, n, s);
    sigma12_sigma22inv(f, f22, Yc + n1, n, U, n1, nc, scr, s);
    const long long tot = n1 * nc;
    hipLaunchKernelGGL(cond_dev_kernel, dim3((unsigned)std::min<long long>(4096, (tot + 255) / 256)), dim3(256), 0, s,
                       Yc, n, U, n1, nc, d_dev);
    RSF_HIP(hipGetLastError());
  });
}

rsf_status rsf_grad_hutch(rsf_factor f, const double* d_z, int nprobe, uint64_t seed, double* g,
                          rsf_grad_info* info, void* stream) {
  return guarded([&] {
    check_handle(f);
    RSF_CHECK(f->tree.ninst == 1, RSF_E_INVALID, "a batched handle takes rsf_grad_hutch_batched");
    RSF_CHECK(d_z != nullptr && g != nullptr, RSF_E_INVALID, "null argument");
    RSF_CHECK(nprobe >= 1, RSF_E_INVALID, "nprobe must be >= 1");
    grad_eval(f, d_z, 0.0, seed, g, info, stream, nprobe);
  });
}

rsf_status rsf_grad_hutch_batched(rsf_factor f, const double* const* d_z, int nprobe, uint64_t seed, double* g_nb_p,
                                  rsf_grad_info* info_or_null, void* stream) {
  return guarded([&] {
    check_handle(f);
    RSF_CHECK(d_z != nullptr && g_nb_p != nullptr, RSF_E_INVALID, "null argument");
    RSF_CHECK(nprobe >= 1, RSF_E_INVALID, "nprobe must be >= 1");
    hipStream_t s = as_stream(stream);
    Scratch scr(s);
    const double* Z = gather_instances(f, d_z, scr, s);
    grad_eval(f, Z, 0.0, seed, g_nb_p, info_or_null, stream, nprobe);
  });
}

rsf_status rsf_grad_batched(rsf_factor f, const double* const* d_z, double eps_peel, uint64_t seed,
                            double* g_nb_p, rsf_grad_info* info_or_null, void* stream) {
  return guarded([&] {
    check_handle(f);
    RSF_CHECK(d_z != nullptr && g_nb_p != nullptr, RSF_E_INVALID, "null argument");
    hipStream_t s = as_stream(stream);
    Scratch scr(s);
    const double* Z = gather_instances(f, d_z, scr, s);
    grad_eval(f, Z, eps_peel, seed, g_nb_p, info_or_null, stream);
  });
}

}  // extern "C"
