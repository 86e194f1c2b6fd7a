// Batched FP64 GEMM on the gfx950 matrix cores, device memory helpers and
// fixed-order reductions.
#include "common.h"

namespace rsf {

typedef double v4d __attribute__((ext_vector_type(4)));

void* Arena::alloc(size_t nbytes) {
  if (nbytes == 0) nbytes = 8;
  nbytes = (nbytes + 255) & ~size_t(255);
  RSF_CHECK(cap == 0 || bytes + nbytes <= cap, RSF_E_OOM,
            "factor memory cap exceeded (" + std::to_string(bytes + nbytes) + " > " +
                std::to_string(cap) + " bytes)");
  void* p = nullptr;
  RSF_HIP(hipMalloc(&p, nbytes));
  blocks.push_back(p);
  bytes += nbytes;
  return p;
}

void Arena::release() {
  for (void* p : blocks) (void)hipFree(p);
  blocks.clear();
  bytes = 0;
}

void* Scratch::alloc(size_t nbytes) {
  if (nbytes == 0) nbytes = 8;
  nbytes = (nbytes + 255) & ~size_t(255);
  void* p = nullptr;
  RSF_HIP(hipMalloc(&p, nbytes));
  blocks.push_back(p);
  return p;
}

Scratch::~Scratch() {
  if (!blocks.empty()) (void)hipStreamSynchronize(stream);
  for (void* p : blocks) (void)hipFree(p);
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

// ---- launch tracing of the batched GEMM (events on the launch stream)
namespace {
struct GemmTrace {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
  long long launches = 0;
} g_trace;
}

void trace_enable(bool on) { g_trace.on = on; }

void trace_read(double* ms, double* flops, double* bytes, long long* launches, bool reset) {
  for (auto& e : g_trace.ev) {
    float t = 0.f;
    RSF_HIP(hipEventSynchronize(e.second));
    RSF_HIP(hipEventElapsedTime(&t, e.first, e.second));
    g_trace.ms += t;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  g_trace.ev.clear();
  if (ms) *ms = g_trace.ms;
  if (flops) *flops = g_trace.flops;
  if (bytes) *bytes = g_trace.bytes;
  if (launches) *launches = g_trace.launches;
  if (reset) {
    g_trace.ms = g_trace.flops = g_trace.bytes = 0.0;
    g_trace.launches = 0;
  }
}

void gemm_batched(const std::vector<GemmDesc>& descs, Scratch& scr, hipStream_t s) {
  std::vector<int4> tiles;
  std::vector<GemmDesc> live;
  double flops = 0.0, bytes = 0.0;
  for (const GemmDesc& d : descs) {
    if (d.M <= 0 || d.N <= 0) continue;
    flops += 2.0 * d.M * d.N * d.K;
    bytes += 8.0 * ((double)d.M * d.K + (double)d.K * d.N + (d.beta != 0.0 ? 2.0 : 1.0) * d.M * d.N);
    const int p = (int)live.size();
    live.push_back(d);
    const int tm = (d.M + 63) / 64, tn = (d.N + 63) / 64;
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) tiles.push_back(make_int4(p, a, b, 0));
  }
  if (tiles.empty()) return;
  GemmDesc* dd = scr.make<GemmDesc>(live.size());
  int4* dt = scr.make<int4>(tiles.size());
  upload(dd, live, s);
  upload(dt, tiles, s);
  // the grid is limited to 2^31 - 1 blocks in x; tile lists here stay far below
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (g_trace.on) {
    RSF_HIP(hipEventCreate(&e0));
    RSF_HIP(hipEventCreate(&e1));
    RSF_HIP(hipEventRecord(e0, s));
  }
  hipLaunchKernelGGL(gemm_tiles_kernel, dim3((unsigned)tiles.size()), dim3(256), 0, s, dd, dt);
  RSF_HIP(hipGetLastError());
  if (g_trace.on) {
    RSF_HIP(hipEventRecord(e1, s));
    g_trace.ev.emplace_back(e0, e1);
    g_trace.flops += flops;
    g_trace.bytes += bytes;
    g_trace.launches += 1;
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
