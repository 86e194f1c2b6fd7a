// Batched FP64 GEMM on the gfx950 matrix cores, device memory helpers and
// fixed-order reductions.
#include <map>
#include <mutex>

#include "common.h"

namespace rsf {


// ---- device memory pool
// Freed blocks are kept per size class and handed out again in stream order:
// a block released on stream s is reused on s without a synchronisation (later
// work on s runs after the work that used it); reuse on another stream waits
// for the releasing stream first.  Size classes: four per power of two.
namespace {
struct FreeBlock {
  void* p;
  hipStream_t s;
};
struct Pool {
  std::mutex mu;
  std::map<size_t, std::vector<FreeBlock>> free;
} g_pool;

size_t size_class(size_t n) {
  if (n <= 4096) return 4096;
  size_t top = size_t(1) << (63 - __builtin_clzll(n));
  size_t step = top / 4;
  return (n + step - 1) / step * step;
}
}  // namespace

void* pool_alloc(size_t nbytes, hipStream_t s) {
  const size_t c = size_class(nbytes);
  {
    std::lock_guard<std::mutex> lk(g_pool.mu);
    auto it = g_pool.free.find(c);
    if (it != g_pool.free.end() && !it->second.empty()) {
      auto& v = it->second;
      for (size_t i = v.size(); i-- > 0;)
        if (v[i].s == s) {
          void* p = v[i].p;
          v.erase(v.begin() + i);
          return p;
        }
      FreeBlock b = v.back();
      v.pop_back();
      RSF_HIP(hipStreamSynchronize(b.s));
      return b.p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, c);
  if (e != hipSuccess) {
    // give cached blocks back to the device and try once more
    (void)hipGetLastError();
    pool_trim();
    RSF_HIP(hipMalloc(&p, c));
  }
  return p;
}

void pool_free(void* p, size_t nbytes, hipStream_t s) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pool.mu);
  g_pool.free[size_class(nbytes)].push_back(FreeBlock{p, s});
}

void pool_trim() {
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_pool.mu);
  for (auto& kv : g_pool.free)
    for (auto& b : kv.second) (void)hipFree(b.p);
  g_pool.free.clear();
}

void* Arena::alloc(size_t nbytes) {
  if (nbytes == 0) nbytes = 8;
  nbytes = (nbytes + 255) & ~size_t(255);
  RSF_CHECK(cap == 0 || bytes + nbytes <= cap, RSF_E_OOM,
            "factor memory cap exceeded (" + std::to_string(bytes + nbytes) + " > " +
                std::to_string(cap) + " bytes)");
  void* p = pool_alloc(nbytes, nullptr);
  blocks.push_back(p);
  sizes.push_back(nbytes);
  bytes += nbytes;
  return p;
}

void Arena::release() {
  if (!blocks.empty()) (void)hipDeviceSynchronize();
  for (size_t i = 0; i < blocks.size(); ++i) pool_free(blocks[i], sizes[i], nullptr);
  blocks.clear();
  sizes.clear();
  bytes = 0;
}

void* Scratch::alloc(size_t nbytes) {
  if (nbytes == 0) nbytes = 8;
  void* p = pool_alloc(nbytes, stream);
  blocks.push_back(p);
  sizes.push_back(nbytes);
  return p;
}

void Scratch::release(const void* p) {
  for (size_t i = 0; i < blocks.size(); ++i)
    if (blocks[i] == p) {
      pool_free(blocks[i], sizes[i], stream);
      blocks.erase(blocks.begin() + i);
      sizes.erase(sizes.begin() + i);
      return;
    }
}

Scratch::~Scratch() {
  for (size_t i = 0; i < blocks.size(); ++i) pool_free(blocks[i], sizes[i], stream);
}

// One 256-thread workgroup computes a 64 x 64 tile of C; each of the four
// waves owns a 32 x 32 quarter as 2 x 2 blocks of v_mfma_f64_16x16x4.  The A
// and B tiles pass through LDS in chunks of 16 along K; the load pattern
// follows whichever index of the operand is contiguous in memory.
//
// Operand layout of v_mfma_f64_16x16x4f64 (lane l, register r):
//   A(row l % 16, k l / 16),  B(k l / 16, col l % 16),  D(row 4 r + l / 16, col l % 16).
__device__ __forceinline__ void store_block(const GemmDesc& d, const v4d& acc, int ib, int jb,
                                            int lane) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int gi = ib + 4 * r + (lane >> 4);
    const int gj = jb + (lane & 15);
    if (gi < d.M && gj < d.N) {
      const long long row = d.cidx ? (long long)d.cidx[gi] : (long long)gi;
      double* c = d.C + row * d.crs + (long long)gj * d.ccs;
      *c = (d.beta == 0.0) ? d.alpha * acc[r] : d.alpha * acc[r] + d.beta * *c;
    }
  }
}

__global__ __launch_bounds__(256) void gemm_tiles_kernel(const GemmDesc* __restrict__ descs,
                                                          const int4* __restrict__ tiles) {
  __shared__ double As[16][66];  // As[k][i]
  __shared__ double Bs[16][66];  // Bs[k][j]
  const int4 t = tiles[blockIdx.x];
  const GemmDesc d = descs[t.x];
  const int i0 = t.y * 64, j0 = t.z * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rb = (wave >> 1) * 32, cb = (wave & 1) * 32;
  v4d acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
  const bool a_icontig = (d.ars == 1 && d.aidx == nullptr);
  const bool b_jcontig = (d.bcs == 1);
  for (int k0 = 0; k0 < d.K; k0 += 16) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int i, kk;
      if (a_icontig) {
        i = tid & 63;
        kk = (tid >> 6) + 4 * r;
      } else {
        kk = tid & 15;
        i = (tid >> 4) + 16 * r;
      }
      const int gi = i0 + i, gk = k0 + kk;
      double v = 0.0;
      if (gi < d.M && gk < d.K) {
        const long long row = d.aidx ? (long long)d.aidx[gi] : (long long)gi;
        v = d.A[row * d.ars + (long long)gk * d.acs];
      }
      As[kk][i] = v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int j, kk;
      if (b_jcontig) {
        j = tid & 63;
        kk = (tid >> 6) + 4 * r;
      } else {
        kk = tid & 15;
        j = (tid >> 4) + 16 * r;
      }
      const int gj = j0 + j, gk = k0 + kk;
      double v = 0.0;
      if (gj < d.N && gk < d.K) {
        const long long row = d.bidx ? (long long)d.bidx[gk] : (long long)gk;
        v = d.B[row * d.brs + (long long)gj * d.bcs];
      }
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      const double a0 = As[kk][rb + (lane & 15)];
      const double a1 = As[kk][rb + 16 + (lane & 15)];
      const double b0 = Bs[kk][cb + (lane & 15)];
      const double b1 = Bs[kk][cb + 16 + (lane & 15)];
      acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc01, 0, 0, 0);
      acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc10, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc11, 0, 0, 0);
    }
  }
  store_block(d, acc00, i0 + rb, j0 + cb, lane);
  store_block(d, acc01, i0 + rb, j0 + cb + 16, lane);
  store_block(d, acc10, i0 + rb + 16, j0 + cb, lane);
  store_block(d, acc11, i0 + rb + 16, j0 + cb + 16, lane);
}

// The 64 x 64 tile kernel in mixed precision: operands are rounded to FP32 as
// they are staged in LDS, the products run on v_mfma_f32_16x16x4f32 with FP32
// accumulation, and C = alpha * acc + beta * C is formed in FP64.  The FP32
// accumulator of lane l holds rows 4 (l / 16) + v, column l mod 16.
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void store_block32(const GemmDesc& d, const v4f& acc, int ib, int jb, int lane) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int gi = ib + 4 * (lane >> 4) + v;
    const int gj = jb + (lane & 15);
    if (gi < d.M && gj < d.N) {
      const long long row = d.cidx ? (long long)d.cidx[gi] : (long long)gi;
      double* c = d.C + row * d.crs + (long long)gj * d.ccs;
      const double a = (double)acc[v];
      *c = (d.beta == 0.0) ? d.alpha * a : d.alpha * a + d.beta * *c;
    }
  }
}

__global__ __launch_bounds__(256) void gemm_tiles_f32_kernel(const GemmDesc* __restrict__ descs,
                                                              const int4* __restrict__ tiles) {
  __shared__ float As[16][68];  // As[k][i]
  __shared__ float Bs[16][68];  // Bs[k][j]
  const int4 t = tiles[blockIdx.x];
  const GemmDesc d = descs[t.x];
  const int i0 = t.y * 64, j0 = t.z * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rb = (wave >> 1) * 32, cb = (wave & 1) * 32;
  v4f acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
  const bool a_icontig = (d.ars == 1 && d.aidx == nullptr);
  const bool b_jcontig = (d.bcs == 1);
  for (int k0 = 0; k0 < d.K; k0 += 16) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int i, kk;
      if (a_icontig) {
        i = tid & 63;
        kk = (tid >> 6) + 4 * r;
      } else {
        kk = tid & 15;
        i = (tid >> 4) + 16 * r;
      }
      const int gi = i0 + i, gk = k0 + kk;
      float v = 0.0f;
      if (gi < d.M && gk < d.K) {
        const long long row = d.aidx ? (long long)d.aidx[gi] : (long long)gi;
        v = (float)d.A[row * d.ars + (long long)gk * d.acs];
      }
      As[kk][i] = v;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int j, kk;
      if (b_jcontig) {
        j = tid & 63;
        kk = (tid >> 6) + 4 * r;
      } else {
        kk = tid & 15;
        j = (tid >> 4) + 16 * r;
      }
      const int gj = j0 + j, gk = k0 + kk;
      float v = 0.0f;
      if (gj < d.N && gk < d.K) {
        const long long row = d.bidx ? (long long)d.bidx[gk] : (long long)gk;
        v = (float)d.B[row * d.brs + (long long)gj * d.bcs];
      }
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      const float a0 = As[kk][rb + (lane & 15)];
      const float a1 = As[kk][rb + 16 + (lane & 15)];
      const float b0 = Bs[kk][cb + (lane & 15)];
      const float b1 = Bs[kk][cb + 16 + (lane & 15)];
      acc00 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc01, 0, 0, 0);
      acc10 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc10, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc11, 0, 0, 0);
    }
  }
  store_block32(d, acc00, i0 + rb, j0 + cb, lane);
  store_block32(d, acc01, i0 + rb, j0 + cb + 16, lane);
  store_block32(d, acc10, i0 + rb + 16, j0 + cb, lane);
  store_block32(d, acc11, i0 + rb + 16, j0 + cb + 16, lane);
}

// ---- launch tracing of the batched GEMM (events on the launch stream)
namespace {
struct TraceEv {
  hipEvent_t a, b;
  std::string tag;
};
struct GemmTrace {
  bool on = false;
  std::vector<TraceEv> ev;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
  long long launches = 0;
  std::string tag = "other";
  std::map<std::string, double> tag_ms, tag_flops;
} g_trace;
}  // namespace

void trace_enable(bool on) { g_trace.on = on; }

std::string trace_current() { return g_trace.tag; }

TraceLaunch::TraceLaunch(hipStream_t st, double fl, double by) : s(st), flops(fl), bytes(by) {
  if (!g_trace.on) return;
  RSF_HIP(hipEventCreate(&e0));
  RSF_HIP(hipEventCreate(&e1));
  RSF_HIP(hipEventRecord(e0, s));
}
TraceLaunch::~TraceLaunch() {
  if (!e0) return;
  (void)hipEventRecord(e1, s);
  g_trace.ev.push_back(TraceEv{e0, e1, g_trace.tag});
  g_trace.flops += flops;
  g_trace.bytes += bytes;
  g_trace.launches += 1;
  g_trace.tag_flops[g_trace.tag] += flops;
}
TraceTag::TraceTag(const char* t) : prev(g_trace.tag) { g_trace.tag = t; }
TraceTag::~TraceTag() { g_trace.tag = prev; }

void trace_read(double* ms, double* flops, double* bytes, long long* launches, bool reset) {
  for (auto& e : g_trace.ev) {
    float t = 0.f;
    RSF_HIP(hipEventSynchronize(e.b));
    RSF_HIP(hipEventElapsedTime(&t, e.a, e.b));
    g_trace.ms += t;
    g_trace.tag_ms[e.tag] += t;
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  g_trace.ev.clear();
  if (ms) *ms = g_trace.ms;
  if (flops) *flops = g_trace.flops;
  if (bytes) *bytes = g_trace.bytes;
  if (launches) *launches = g_trace.launches;
  if (reset) {
    g_trace.ms = g_trace.flops = g_trace.bytes = 0.0;
    g_trace.launches = 0;
    g_trace.tag_ms.clear();
    g_trace.tag_flops.clear();
  }
}

std::string trace_tags() {
  std::string out;
  for (auto& kv : g_trace.tag_ms) {
    char buf[160];
    snprintf(buf, sizeof(buf), "%s%s:%.3f:%.6g", out.empty() ? "" : ";", kv.first.c_str(), kv.second,
             g_trace.tag_flops[kv.first]);
    out += buf;
  }
  return out;
}

// 128 x 128 tiles for the large products: each wave owns a 64 x 64 quarter as
// 4 x 4 blocks of v_mfma_f64_16x16x4 (16 accumulators), eight LDS reads feed
// sixteen MFMAs per k-step, and the next 16-wide K chunk is fetched into
// registers while the current one is multiplied.  One kernel per operand
// layout (A: rows contiguous or k contiguous; B: columns contiguous, with or
// without a row map, or k contiguous), chosen on the host.  Interior tiles
// and full K chunks take unchecked loads through per-thread pointers that
// advance by a fixed stride per chunk; only edge tiles pay for bounds checks.
constexpr int BT = 128;

template <bool AI, bool BJ, bool BIDX>
__global__ __launch_bounds__(256, 2) void gemm_big_kernel(const GemmDesc* __restrict__ descs,
                                                           const int4* __restrict__ tiles) {
  __shared__ double As[16][BT + 4];
  __shared__ double Bs[16][BT + 4];
  const int4 t = tiles[blockIdx.x];
  const GemmDesc& dg = descs[t.x];
  const int M = dg.M, N = dg.N, K = dg.K;
  const int i0 = t.y * BT, j0 = t.z * BT;
  const int tid = threadIdx.x;
  const bool full = (i0 + BT <= M) && (j0 + BT <= N);
  // fetch geometry (see the layout note above):
  //   AI: A(i0 + (tid & 127), k0 + (tid >> 7) + 2 r)   else A(i0 + (tid >> 4) + 16 r, k0 + (tid & 15))
  //   BJ: B(k0 + (tid >> 7) + 2 r, j0 + (tid & 127))   else B(k0 + (tid & 15), j0 + (tid >> 4) + 16 r)
  const int a_i = AI ? (tid & 127) : (tid >> 4);
  const int a_k = AI ? (tid >> 7) : (tid & 15);
  const int b_j = BJ ? (tid & 127) : (tid >> 4);
  const int b_k = BJ ? (tid >> 7) : (tid & 15);
  const long long astr = AI ? dg.acs : dg.ars;  // AI: step along k; else: step between the 8 rows (x16)
  const long long bstr = BJ ? dg.brs : dg.bcs;
  const double* __restrict__ pa = dg.A + (long long)(i0 + a_i) * (AI ? 1 : dg.ars);
  const double* __restrict__ pb = dg.B + (long long)(j0 + b_j) * (BJ ? 1 : dg.bcs);
  const int* __restrict__ bidx = dg.bidx;
  unsigned amask = 0, bmask = 0;  // bit r: row / column r of this thread is inside the problem
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    if (i0 + (AI ? a_i : a_i + 16 * r) < M) amask |= 1u << r;
    if (j0 + (BJ ? b_j : b_j + 16 * r) < N) bmask |= 1u << r;
  }
  v4d acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[m][q] = v4d{0, 0, 0, 0};
  double ra[8], rbv[8];
  auto fetch = [&](int k0) {
    if (full && k0 + 16 <= K) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        ra[r] = AI ? pa[(long long)(k0 + a_k + 2 * r) * astr] : pa[(long long)(16 * r) * astr + k0 + a_k];
        if (BJ) {
          const int kb = k0 + b_k + 2 * r;
          rbv[r] = pb[(long long)(BIDX ? bidx[kb] : kb) * bstr];
        } else {
          rbv[r] = pb[(long long)(16 * r) * bstr + k0 + b_k];
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int ka = k0 + a_k + (AI ? 2 * r : 0);
        ra[r] = ((amask >> r) & 1u) && ka < K
                    ? (AI ? pa[(long long)ka * astr] : pa[(long long)(16 * r) * astr + ka])
                    : 0.0;
        const int kb = k0 + b_k + (BJ ? 2 * r : 0);
        double v = 0.0;
        if (((bmask >> r) & 1u) && kb < K)
          v = BJ ? pb[(long long)(BIDX ? bidx[kb] : kb) * bstr] : pb[(long long)(16 * r) * bstr + kb];
        rbv[r] = v;
      }
    }
  };
  fetch(0);
  const int lane = tid & 63, wave = tid >> 6;
  const int rb0 = (wave >> 1) * 64, cb0 = (wave & 1) * 64;
  for (int k0 = 0; k0 < K; k0 += 16) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (AI)
        As[a_k + 2 * r][a_i] = ra[r];
      else
        As[a_k][a_i + 16 * r] = ra[r];
      if (BJ)
        Bs[b_k + 2 * r][b_j] = rbv[r];
      else
        Bs[b_k][b_j + 16 * r] = rbv[r];
    }
    __syncthreads();
    if (k0 + 16 < K) fetch(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      double a[4], b[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) a[m] = As[kk][rb0 + m * 16 + (lane & 15)];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = Bs[kk][cb0 + q * 16 + (lane & 15)];
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[q], acc[m][q], 0, 0, 0);
    }
  }
  const double alpha = dg.alpha, beta = dg.beta;
  const int* __restrict__ cidx = dg.cidx;
  double* __restrict__ Cb = dg.C;
  const long long crs = dg.crs, ccs = dg.ccs;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gi = i0 + rb0 + m * 16 + 4 * r + (lane >> 4);
      if (!full && gi >= M) continue;
      const long long row = cidx ? (long long)cidx[gi] : (long long)gi;
      double* crow = Cb + row * crs;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int gj = j0 + cb0 + q * 16 + (lane & 15);
        if (!full && gj >= N) continue;
        double* c = crow + (long long)gj * ccs;
        const double v = acc[m][q][r];
        *c = (beta == 0.0) ? alpha * v : alpha * v + beta * *c;
      }
    }
}

// layout class of a problem for the 128 x 128 kernels: bit 2 = A rows
// contiguous (else k contiguous), bit 1 = B columns contiguous (else k
// contiguous), bit 0 = B has a row map (only with contiguous columns);
// -1 = no fitting layout, use the 64 x 64 kernel
static int big_class(const GemmDesc& d) {
  const bool ai = (d.ars == 1 && d.aidx == nullptr), ak = (d.acs == 1 && d.aidx == nullptr);
  const bool bj = (d.bcs == 1), bk = (d.brs == 1 && d.bidx == nullptr);
  if (!(ai || ak) || !(bj || bk)) return -1;
  return (ai ? 4 : 0) | (bj ? 2 : 0) | ((bj && d.bidx) ? 1 : 0);
}

void gemm_batched(const std::vector<GemmDesc>& descs, Scratch& scr, hipStream_t s) {
  std::vector<int4> tiles, btiles[8], tiles32;
  std::vector<GemmDesc> live;
  double flops = 0.0, bytes = 0.0;
  for (const GemmDesc& d : descs) {
    if (d.M <= 0 || d.N <= 0) continue;
    flops += (d.lower ? 1.0 : 2.0) * d.M * d.N * d.K;
    bytes += 8.0 * ((double)d.M * d.K + (double)d.K * d.N + (d.beta != 0.0 ? 2.0 : 1.0) * d.M * d.N);
    const int p = (int)live.size();
    live.push_back(d);
    const int cls = big_class(d);
    if (d.f32) {
      const int tm = (d.M + 63) / 64, tn = (d.N + 63) / 64;
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b)
          if (!d.lower || b <= a) tiles32.push_back(make_int4(p, a, b, 0));
    } else if (cls >= 0 && d.M >= 96 && d.N >= 96 && d.K >= 32) {
      const int tm = (d.M + BT - 1) / BT, tn = (d.N + BT - 1) / BT;
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b)
          if (!d.lower || b <= a) btiles[cls].push_back(make_int4(p, a, b, 0));
    } else {
      const int tm = (d.M + 63) / 64, tn = (d.N + 63) / 64;
      for (int a = 0; a < tm; ++a)
        for (int b = 0; b < tn; ++b)
          if (!d.lower || b <= a) tiles.push_back(make_int4(p, a, b, 0));
    }
  }
  size_t nt = tiles.size() + tiles32.size();
  for (auto& v : btiles) nt += v.size();
  if (nt == 0) return;
  GemmDesc* dd = scr.make<GemmDesc>(live.size());
  upload(dd, live, s);
  std::vector<int4> all(tiles);
  size_t boff[9];
  boff[0] = all.size();
  for (int c = 0; c < 8; ++c) {
    all.insert(all.end(), btiles[c].begin(), btiles[c].end());
    boff[c + 1] = all.size();
  }
  const size_t off32 = all.size();
  all.insert(all.end(), tiles32.begin(), tiles32.end());
  int4* dt = scr.make<int4>(all.size());
  upload(dt, all, s);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (g_trace.on) {
    RSF_HIP(hipEventCreate(&e0));
    RSF_HIP(hipEventCreate(&e1));
    RSF_HIP(hipEventRecord(e0, s));
  }
  // the grid is limited to 2^31 - 1 blocks in x; tile lists here stay far below
#define RSF_BIG(c, AI, BJ, BX)                                                                        \
  if (!btiles[c].empty())                                                                             \
    hipLaunchKernelGGL((gemm_big_kernel<AI, BJ, BX>), dim3((unsigned)btiles[c].size()), dim3(256), 0, s, dd, \
                       dt + boff[c]);
  RSF_BIG(7, true, true, true)
  RSF_BIG(6, true, true, false)
  RSF_BIG(4, true, false, false)
  RSF_BIG(3, false, true, true)
  RSF_BIG(2, false, true, false)
  RSF_BIG(0, false, false, false)
#undef RSF_BIG
  if (!tiles.empty())
    hipLaunchKernelGGL(gemm_tiles_kernel, dim3((unsigned)tiles.size()), dim3(256), 0, s, dd, dt);
  if (!tiles32.empty())
    hipLaunchKernelGGL(gemm_tiles_f32_kernel, dim3((unsigned)tiles32.size()), dim3(256), 0, s, dd, dt + off32);
  RSF_HIP(hipGetLastError());
  if (g_trace.on) {
    RSF_HIP(hipEventRecord(e1, s));
    // launches with FP32 products are booked under "<phase>/f32"
    const std::string tag = tiles32.empty() ? g_trace.tag : g_trace.tag + "/f32";
    g_trace.ev.push_back(TraceEv{e0, e1, tag});
    g_trace.flops += flops;
    g_trace.bytes += bytes;
    g_trace.launches += 1;
    g_trace.tag_flops[tag] += flops;
  }
}

// ---- batched blocked Cholesky with inverse
__global__ __launch_bounds__(256) void copy_blocks_kernel(const CopyBlock* __restrict__ jobs) {
  const CopyBlock J = jobs[blockIdx.x];
  const long long tot = (long long)J.m * J.n;
  for (long long e = blockIdx.y * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.y) {
    const int i = (int)(e % J.m), j = (int)(e / J.m);
    J.dst[(long long)j * J.ldd + i] = (J.src == nullptr || (J.lower && i < j)) ? 0.0 : J.src[(long long)j * J.lds + i];
  }
}

void copy_blocks(const std::vector<CopyBlock>& jobs, Scratch& scr, hipStream_t s) {
  std::vector<CopyBlock> live;
  long long mx = 1;
  for (const CopyBlock& j : jobs)
    if (j.m > 0 && j.n > 0) {
      live.push_back(j);
      mx = std::max(mx, (long long)j.m * j.n);
    }
  if (live.empty()) return;
  CopyBlock* d = scr.make<CopyBlock>(live.size());
  upload(d, live, s);
  const unsigned gy = (unsigned)std::max<long long>(1, std::min<long long>(64, (mx + 2047) / 2048));
  hipLaunchKernelGGL(copy_blocks_kernel, dim3((unsigned)live.size(), gy), dim3(256), 0, s, d);
  RSF_HIP(hipGetLastError());
}

struct DiagJob {
  double* A;  // the diagonal block, ld lda
  long long lda;
  int nb;
  double* Dinv;  // 64 x 64
  double* logd;  // one value or null
};

// Cholesky of one diagonal block (nb <= 64) in LDS, written back in place
// (zero above the diagonal), its log-diagonal sum and its inverse.
__global__ __launch_bounds__(256) void diag_chol_batched_kernel(const DiagJob* __restrict__ jobs, int* fail) {
  __shared__ double B[64][65];
  __shared__ double I[64][65];
  const DiagJob J = jobs[blockIdx.x];
  const int nb = J.nb, tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e % nb, j = e / nb;
    B[i][j] = J.A[(long long)j * J.lda + i];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double d = B[j][j];
    if (!(d > 0.0)) {
      if (tid == 0) *fail = 1;
      return;
    }
    const double sq = sqrt(d);
    __syncthreads();
    if (tid == 0) B[j][j] = sq;
    for (int i = j + 1 + tid; i < nb; i += 256) B[i][j] /= sq;
    __syncthreads();
    for (int e = tid; e < nb * nb; e += 256) {
      const int i = e % nb, l = e / nb;
      if (l > j && i >= l) B[i][l] -= B[i][j] * B[l][j];
    }
    __syncthreads();
  }
  if (tid == 0 && J.logd) {
    double sm = 0.0;
    for (int j = 0; j < nb; ++j) sm += log(B[j][j]);
    *J.logd = 2.0 * sm;
  }
  for (int c = tid; c < nb; c += 256) {
    for (int i = 0; i < nb; ++i) I[i][c] = 0.0;
    I[c][c] = 1.0 / B[c][c];
    for (int i = c + 1; i < nb; ++i) {
      double x = 0.0;
      for (int l = c; l < i; ++l) x -= B[i][l] * I[l][c];
      I[i][c] = x / B[i][i];
    }
  }
  __syncthreads();
  for (int e = tid; e < nb * nb; e += 256) {
    const int i = e % nb, j = e / nb;
    J.A[(long long)j * J.lda + i] = (i >= j) ? B[i][j] : 0.0;
    J.Dinv[(long long)j * 64 + i] = I[i][j];
  }
}

void batched_chol_inv(const std::vector<CholProblem>& P, int* fail, Scratch& scr, hipStream_t s) {
  TraceTag tag("chol");
  int maxn = 0;
  std::vector<long long> doff(P.size() + 1, 0), qoff(P.size() + 1, 0);
  for (size_t p = 0; p < P.size(); ++p) {
    maxn = std::max(maxn, P[p].n);
    doff[p + 1] = doff[p] + (long long)((P[p].n + 63) / 64) * 4096;
    qoff[p + 1] = qoff[p] + (long long)64 * std::max(P[p].n, 1);
  }
  if (maxn == 0) return;
  double* Dinv = scr.make<double>(std::max<long long>(doff.back(), 1));
  double* Q = scr.make<double>(std::max<long long>(qoff.back(), 1));
  const int nbk = (maxn + 63) / 64;
  for (int b = 0; b < nbk; ++b) {
    const int kb = b * 64;
    std::vector<DiagJob> dj;
    std::vector<GemmDesc> pan, trl;
    for (size_t p = 0; p < P.size(); ++p) {
      const CholProblem& c = P[p];
      if (c.n <= kb) continue;
      const int nb = std::min(64, c.n - kb), rest = c.n - kb - nb;
      double* Akk = c.A + (long long)kb * c.lda + kb;
      double* Dk = Dinv + doff[p] + (long long)b * 4096;
      dj.push_back(DiagJob{Akk, c.lda, nb, Dk, c.logd ? c.logd + b : nullptr});
      if (rest > 0) {
        // panel L(kb+nb:, kb:kb+nb) = A(kb+nb:, kb:kb+nb) Dinv^T, in place (one
        // tile column: every tile reads its rows completely before writing them)
        double* Pn = c.A + (long long)kb * c.lda + kb + nb;
        pan.push_back(gemm_desc(rest, nb, nb, 1.0, colmaj(Pn, c.lda), colmajT(Dk, 64), 0.0, colmaj(Pn, c.lda)));
        GemmDesc t = gemm_desc(rest, rest, nb, -1.0, colmaj(Pn, c.lda), colmajT(Pn, c.lda), 1.0,
                               colmaj(c.A + (long long)(kb + nb) * c.lda + kb + nb, c.lda));
        t.lower = 1;
        trl.push_back(t);
      }
    }
    if (!dj.empty()) {
      DiagJob* d = scr.make<DiagJob>(dj.size());
      upload(d, dj, s);
      hipLaunchKernelGGL(diag_chol_batched_kernel, dim3((unsigned)dj.size()), dim3(256), 0, s, d, fail);
      RSF_HIP(hipGetLastError());
    }
    gemm_batched(pan, scr, s);
    gemm_batched(trl, scr, s);
  }
  // inverse: Linv(i, i) = Dinv_i;  Linv(i, 0:i) = -Dinv_i L(i, 0:i) Linv(0:i, 0:i)
  {
    std::vector<CopyBlock> z;
    for (const CholProblem& c : P) z.push_back(CopyBlock{nullptr, 0, c.Linv, c.ldi, c.n, c.n, 0});
    copy_blocks(z, scr, s);
  }
  for (int b = 0; b < nbk; ++b) {
    const int kb = b * 64;
    std::vector<CopyBlock> cp;
    std::vector<GemmDesc> g1, g2;
    for (size_t p = 0; p < P.size(); ++p) {
      const CholProblem& c = P[p];
      if (c.n <= kb) continue;
      const int nb = std::min(64, c.n - kb);
      const double* Dk = Dinv + doff[p] + (long long)b * 4096;
      cp.push_back(CopyBlock{Dk, 64, c.Linv + (long long)kb * c.ldi + kb, c.ldi, nb, nb, 1});
      if (kb > 0) {
        double* Qp = Q + qoff[p];
        g1.push_back(gemm_desc(nb, kb, kb, 1.0, colmaj(c.A + kb, c.lda), colmaj(c.Linv, c.ldi), 0.0,
                               colmaj(Qp, nb)));
        g2.push_back(gemm_desc(nb, kb, nb, -1.0, colmaj(Dk, 64), colmaj(Qp, nb), 0.0, colmaj(c.Linv + kb, c.ldi)));
      }
    }
    copy_blocks(cp, scr, s);
    gemm_batched(g1, scr, s);
    gemm_batched(g2, scr, s);
  }
}

// Single-workgroup reduction in a fixed order: thread t sums elements
// t, t + 256, ... sequentially, then a binary tree over the 256 partials.
__global__ __launch_bounds__(256) void sum_kernel(const double* __restrict__ x,
                                                   const double* __restrict__ y, long long n,
                                                   double* out) {
  __shared__ double part[256];
  double acc = 0.0;
  for (long long i = threadIdx.x; i < n; i += 256) acc += y ? x[i] * y[i] : x[i];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = part[0];
}

void device_sum(const double* x, long long n, double* out, Scratch&, hipStream_t s) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, x, (const double*)nullptr, n, out);
  RSF_HIP(hipGetLastError());
}

void device_dot(const double* x, const double* y, long long n, double* out, Scratch&,
                hipStream_t s) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, x, y, n, out);
  RSF_HIP(hipGetLastError());
}

}  // namespace rsf
