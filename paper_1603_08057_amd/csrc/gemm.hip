// Batched FP64 GEMM on the gfx950 matrix cores, device memory helpers and
// fixed-order reductions.
#include <array>
#include <cmath>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <map>
#include <atomic>
#include <mutex>
#include <tuple>

#include "common.h"

namespace rsf {


// ---- device memory pool
// Large regions are taken from the device once (hipMalloc of many gigabytes
// costs milliseconds per gigabyte) and carved into blocks: best fit among the
// free extents, neighbours coalesced on release.  Reuse is stream ordered: an
// extent released on stream s is handed out again on s without a
// synchronisation (later work on s runs after the work that used it); on
// another stream the releasing stream is synchronised first, and extents
// released on different streams are not merged.
namespace {
constexpr size_t POOL_ALIGN = 256;
constexpr size_t REGION_MIN = size_t(2) << 30;
struct Extent {
  size_t size;
  hipStream_t s;
};
struct Region {
  char* base;
  size_t size;
  size_t used = 0;
  std::map<size_t, Extent> free;  // offset -> free extent
};
struct Pool {
  std::mutex mu;
  std::vector<Region> regions;
  std::map<const void*, std::pair<int, size_t>> live;  // block -> (region, size)
} g_pool;

// best-fitting free extent over all regions, preferring extents released on
// stream s (reusing another stream's extent costs a synchronisation of that
// stream); false if none
bool pool_find(size_t n, hipStream_t s, int& ri, size_t& off, Extent& ex) {
  bool found = false, same = false;
  for (int r = 0; r < (int)g_pool.regions.size(); ++r)
    for (const auto& kv : g_pool.regions[r].free) {
      if (kv.second.size < n) continue;
      const bool sm = kv.second.s == s;
      if (!found || (sm && !same) || (sm == same && kv.second.size < ex.size)) {
        found = true;
        same = sm;
        ri = r;
        off = kv.first;
        ex = kv.second;
      }
    }
  return found;
}

// gives regions with no live block back to the device
size_t pool_release_empty() {
  size_t freed = 0;
  std::vector<Region> keep;
  for (Region& g : g_pool.regions) {
    if (g.used == 0) {
      for (const auto& kv : g.free) (void)hipStreamSynchronize(kv.second.s);
      (void)hipFree(g.base);
      freed += g.size;
    } else {
      keep.push_back(std::move(g));
    }
  }
  g_pool.regions.swap(keep);
  for (auto& kv : g_pool.live) {  // region indices moved: rebuild them
    const char* p = static_cast<const char*>(kv.first);
    for (int r = 0; r < (int)g_pool.regions.size(); ++r)
      if (p >= g_pool.regions[r].base && p < g_pool.regions[r].base + g_pool.regions[r].size) kv.second.first = r;
  }
  return freed;
}
}  // namespace

static thread_local bool g_pool_no_sync = false;
void pool_sync_free(bool on) { g_pool_no_sync = on; }

static thread_local bool g_no_alloc = false;
NoAllocScope::NoAllocScope() : was(g_no_alloc) { g_no_alloc = true; }
NoAllocScope::~NoAllocScope() { g_no_alloc = was; }
bool no_alloc_active() { return g_no_alloc; }

void* pool_alloc(size_t nbytes, hipStream_t s) {
  RSF_CHECK(!g_no_alloc, RSF_E_INVALID, "device allocation requested inside a no-allocation call");
  const size_t n = (std::max<size_t>(nbytes, 1) + POOL_ALIGN - 1) / POOL_ALIGN * POOL_ALIGN;
  std::lock_guard<std::mutex> lk(g_pool.mu);
  int ri = -1;
  size_t off = 0;
  Extent ex{0, nullptr};
  if (!pool_find(n, s, ri, off, ex)) {
    // a new region: at least REGION_MIN, or the request rounded to 2 MiB
    const size_t rs = std::max(REGION_MIN, (n + (size_t(2) << 20) - 1) / (size_t(2) << 20) * (size_t(2) << 20));
    void* base = nullptr;
    hipError_t e = hipMalloc(&base, rs);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      pool_release_empty();
      e = hipMalloc(&base, rs);
      if (e != hipSuccess && rs > n) {
        (void)hipGetLastError();
        e = hipMalloc(&base, n);  // no room for a full region: exactly the request
        if (e == hipSuccess) {
          Region g{static_cast<char*>(base), n};
          g.free[0] = Extent{n, s};
          g_pool.regions.push_back(std::move(g));
        }
      } else if (e == hipSuccess) {
        Region g{static_cast<char*>(base), rs};
        g.free[0] = Extent{rs, s};
        g_pool.regions.push_back(std::move(g));
      }
    } else {
      Region g{static_cast<char*>(base), rs};
      g.free[0] = Extent{rs, s};
      g_pool.regions.push_back(std::move(g));
    }
    RSF_HIP(e);
    RSF_CHECK(pool_find(n, s, ri, off, ex), RSF_E_OOM, "device pool: no extent after growth");
  }
  Region& g = g_pool.regions[ri];
  g.free.erase(off);
  if (ex.size > n) g.free[off + n] = Extent{ex.size - n, ex.s};
  if (ex.s != s && !g_pool_no_sync) RSF_HIP(hipStreamSynchronize(ex.s));
  g.used += n;
  void* p = g.base + off;
  g_pool.live[p] = std::make_pair(ri, n);
  return p;
}

void pool_free(void* p, size_t /*nbytes*/, hipStream_t s) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pool.mu);
  auto it = g_pool.live.find(p);
  if (it == g_pool.live.end()) return;
  const int ri = it->second.first;
  size_t n = it->second.second;
  g_pool.live.erase(it);
  Region& g = g_pool.regions[ri];
  g.used -= n;
  size_t off = static_cast<char*>(p) - g.base;
  // merge with the free neighbours released on the same stream
  auto nx = g.free.lower_bound(off);
  if (nx != g.free.end() && nx->first == off + n && nx->second.s == s) {
    n += nx->second.size;
    nx = g.free.erase(nx);
  }
  if (nx != g.free.begin()) {
    auto pv = std::prev(nx);
    if (pv->first + pv->second.size == off && pv->second.s == s) {
      off = pv->first;
      n += pv->second.size;
      g.free.erase(pv);
    }
  }
  g.free[off] = Extent{n, s};
}

void pool_trim() {
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> lk(g_pool.mu);
  pool_release_empty();
}

// ---- staging of host-to-device uploads
// A pinned ring: each upload is copied into the next stretch and sent with
// hipMemcpyAsync; an event recorded after the copy marks when the stretch is
// free again, and wrapping around waits for the whole lap.  Uploads larger
// than half the ring go directly (and synchronously).
namespace {
struct Ring {
  std::mutex mu;
  char* buf = nullptr;
  size_t cap = 0, head = 0;
  struct Use {
    size_t beg, end;
    hipEvent_t ev;
  };
  std::deque<Use> inflight;
  std::vector<hipEvent_t> spare;  // events of retired stretches, reused
} g_ring;
constexpr size_t RING_BYTES = size_t(512) << 20;
}  // namespace

static thread_local std::vector<void*>* g_capture_pins = nullptr;
void upload_capture_begin(std::vector<void*>* pins) { g_capture_pins = pins; }
void upload_capture_end() { g_capture_pins = nullptr; }

void upload_bytes(void* dst, const void* src, size_t nbytes, hipStream_t s) {
  if (nbytes == 0) return;
  if (g_capture_pins) {
    void* p = nullptr;
    RSF_HIP(hipHostMalloc(&p, nbytes, hipHostMallocDefault));
    g_capture_pins->push_back(p);
    std::memcpy(p, src, nbytes);
    RSF_HIP(hipMemcpyAsync(dst, p, nbytes, hipMemcpyHostToDevice, s));
    return;
  }
  std::lock_guard<std::mutex> lk(g_ring.mu);
  if (!g_ring.buf && !g_no_alloc) {
    void* p = nullptr;
    if (hipHostMalloc(&p, RING_BYTES, hipHostMallocDefault) == hipSuccess) {
      g_ring.buf = static_cast<char*>(p);
      g_ring.cap = RING_BYTES;
    } else {
      (void)hipGetLastError();
    }
  }
  if (!g_ring.buf || nbytes > g_ring.cap / 2) {
    RSF_HIP(hipMemcpyAsync(dst, src, nbytes, hipMemcpyHostToDevice, s));
    RSF_HIP(hipStreamSynchronize(s));  // the source may be freed by the caller
    return;
  }
  const size_t n = (nbytes + 255) & ~size_t(255);
  size_t a = g_ring.head;
  if (a + n > g_ring.cap) {
    // wrap around: every stretch of the lap that ends here must have been sent
    for (const auto& u : g_ring.inflight) {
      RSF_HIP(hipEventSynchronize(u.ev));
      g_ring.spare.push_back(u.ev);
    }
    g_ring.inflight.clear();
    a = 0;
  }
  std::memcpy(g_ring.buf + a, src, nbytes);
  RSF_HIP(hipMemcpyAsync(dst, g_ring.buf + a, nbytes, hipMemcpyHostToDevice, s));
  hipEvent_t ev;
  if (!g_ring.spare.empty()) {
    ev = g_ring.spare.back();
    g_ring.spare.pop_back();
  } else {
    RSF_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  }
  RSF_HIP(hipEventRecord(ev, s));
  g_ring.inflight.push_back(Ring::Use{a, a + n, ev});
  g_ring.head = a + n;
  // retire finished stretches from the front
  while (!g_ring.inflight.empty() && hipEventQuery(g_ring.inflight.front().ev) == hipSuccess) {
    g_ring.spare.push_back(g_ring.inflight.front().ev);
    g_ring.inflight.pop_front();
  }
}

void* Arena::alloc(size_t nbytes) {
  if (nbytes == 0) nbytes = 8;
  nbytes = (nbytes + 255) & ~size_t(255);
  RSF_CHECK(cap == 0 || bytes + nbytes <= cap, RSF_E_OOM,
            "factor memory cap exceeded (" + std::to_string(bytes + nbytes) + " > " +
                std::to_string(cap) + " bytes)");
  bytes += nbytes;
  if (nbytes <= Scratch::SMALL_MAX) {
    constexpr size_t ARENA_SLAB = size_t(64) << 20;
    if (nbytes > slab_left) {
      slab = static_cast<char*>(pool_alloc(ARENA_SLAB, nullptr));
      blocks.push_back(slab);
      sizes.push_back(ARENA_SLAB);
      slab_left = ARENA_SLAB;
    }
    void* p = slab;
    slab += nbytes;
    slab_left -= nbytes;
    return p;
  }
  void* p = pool_alloc(nbytes, nullptr);
  blocks.push_back(p);
  sizes.push_back(nbytes);
  return p;
}

void Arena::release() {
  if (!blocks.empty()) (void)hipDeviceSynchronize();
  for (size_t i = 0; i < blocks.size(); ++i) pool_free(blocks[i], sizes[i], nullptr);
  blocks.clear();
  sizes.clear();
  bytes = 0;
  slab = nullptr;
  slab_left = 0;
}

void* Scratch::alloc(size_t nbytes) {
  if (nbytes == 0) nbytes = 8;
  if (fixed) {
    const size_t n = (nbytes + 255) & ~size_t(255);
    RSF_CHECK(n <= fixed_cap - fixed_used, RSF_E_INVALID,
              "work space of a no-allocation call exhausted (" + std::to_string(fixed_used + n) + " > " +
                  std::to_string(fixed_cap) + " bytes)");
    void* p = fixed + fixed_used;
    fixed_used += n;
    return p;
  }
  if (nbytes <= SMALL_MAX) {
    const size_t n = (nbytes + 255) & ~size_t(255);
    if (n > slab_left) {
      slab = static_cast<char*>(pool_alloc(SMALL_SLAB, stream));
      blocks.push_back(slab);
      sizes.push_back(SMALL_SLAB);
      slab_left = SMALL_SLAB;
    }
    void* p = slab;
    slab += n;
    slab_left -= n;
    return p;
  }
  void* p = pool_alloc(nbytes, stream);
  blocks.push_back(p);
  sizes.push_back(nbytes);
  return p;
}

void Scratch::release(const void* p) {
  if (fixed) return;
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
  for (void* p : slabs) pool_free(p, SMALL_SLAB, stream);
}

// One 256-thread workgroup computes a 64 x 64 tile of C; each of the four
// waves owns a 32 x 32 quarter as 2 x 2 blocks of v_mfma_f64_16x16x4.  The A
// and B tiles pass through LDS in chunks of 16 along K; the load pattern
// follows whichever index of the operand is contiguous in memory.
//
// Operand layout of v_mfma_f64_16x16x4f64 (lane l, register r):
//   A(row l % 16, k l / 16),  B(k l / 16, col l % 16),  D(row 4 r + l / 16, col l % 16).
// A wave's 32 x 32 quarter (2 x 2 MFMA blocks) to C: the row map and every C
// entry the update reads are loaded before any store, so the loads overlap.
__device__ __forceinline__ void store_tile32(const GemmDesc& d, const v4d& a00, const v4d& a01, const v4d& a10,
                                             const v4d& a11, int ib, int jb, int lane) {
  // per 16-row half, so that the batch's pointers and values stay few
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double* cp[4][2];
    bool ok[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gi = ib + 16 * h + 4 * r + (lane >> 4);
      const bool rin = gi < d.M;
      const long long row = d.cidx ? (rin ? (long long)d.cidx[gi] : 0LL) : (long long)gi;
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const int gj = jb + 16 * w + (lane & 15);
        ok[r][w] = rin && gj < d.N;
        cp[r][w] = d.C + row * d.crs + (long long)gj * d.ccs;
      }
    }
    double cv[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int w = 0; w < 2; ++w) cv[r][w] = (d.beta != 0.0 && ok[r][w]) ? *cp[r][w] : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const double a = h == 0 ? (w == 0 ? a00[r] : a01[r]) : (w == 0 ? a10[r] : a11[r]);
        if (ok[r][w]) *cp[r][w] = (d.beta == 0.0) ? d.alpha * a : d.alpha * a + d.beta * cv[r][w];
      }
  }
}

// The tile of workgroup `bid` in a launch over problems probs[0 .. np) whose
// tiles are numbered consecutively (toff: prefix counts): row-major over the
// tile grid, or over its lower triangle (b <= a) for lower problems.
// Returns (problem, tile row, tile column).
// (tile row, tile column) of tile l of a problem: row-major over its tile grid,
// or over the grid's lower triangle (b <= a) for lower problems.
__device__ __forceinline__ int2 tile_of(const GemmDesc& d, int l, int ts) {
  int a, b;
  if (d.lower) {
    a = (int)((sqrt(8.0 * l + 1.0) - 1.0) * 0.5);
    while ((a + 1) * (a + 2) / 2 <= l) ++a;
    while (a * (a + 1) / 2 > l) --a;
    b = l - a * (a + 1) / 2;
  } else {
    const int tn = (d.N + ts - 1) / ts;
    a = l / tn;
    b = l - a * tn;
  }
  return make_int2(a, b);
}

__device__ __forceinline__ int3 find_tile(const GemmDesc* __restrict__ descs, const int* __restrict__ probs,
                                          const int* __restrict__ toff, int np, int ts, int bid) {
  int lo = 0, hi = np;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (toff[mid] <= bid)
      lo = mid;
    else
      hi = mid;
  }
  const int p = probs[lo];
  const int2 ab = tile_of(descs[p], bid - toff[lo], ts);
  return make_int3(p, ab.x, ab.y);
}

// Launch groups of at most PACK_NP problems pass their descriptors and tile
// prefix counts in the kernel arguments (read in place from the argument
// segment), so that the launch needs no upload.
constexpr int PACK_NP = 20;
struct GemmPack {
  GemmDesc d[PACK_NP];
  int toff[PACK_NP + 1];
  int np;
};

__device__ __forceinline__ int3 find_tile_pack(const GemmPack& pk, int ts, int bid) {
  int lo = 0, hi = pk.np;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pk.toff[mid] <= bid)
      lo = mid;
    else
      hi = mid;
  }
  const int2 ab = tile_of(pk.d[lo], bid - pk.toff[lo], ts);
  return make_int3(lo, ab.x, ab.y);
}

__device__ __forceinline__ void tile64(const GemmDesc& dref, int ti, int tj) {
  const GemmDesc d = dref;
  __shared__ double As[16][66];  // As[k][i]
  __shared__ double Bs[16][66];  // Bs[k][j]
  const int i0 = ti * 64, j0 = tj * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rb = (wave >> 1) * 32, cb = (wave & 1) * 32;
  v4d acc00 = {0, 0, 0, 0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
  const bool a_icontig = (d.ars == 1 && d.aidx == nullptr);
  const bool b_jcontig = (d.bcs == 1);
  // this thread's four A and four B elements of every K chunk: fixed tile
  // positions, the K index advancing by 16 per chunk; A's row map is read once
  int ia[4], ka[4], jb[4], kb[4];
  long long arow[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    if (a_icontig) {
      ia[r] = tid & 63;
      ka[r] = (tid >> 6) + 4 * r;
    } else {
      ka[r] = tid & 15;
      ia[r] = (tid >> 4) + 16 * r;
    }
    const int gi = i0 + ia[r];
    arow[r] = gi < d.M ? (d.aidx ? (long long)d.aidx[gi] : (long long)gi) * d.ars : -1;
    if (b_jcontig) {
      jb[r] = tid & 63;
      kb[r] = (tid >> 6) + 4 * r;
    } else {
      kb[r] = tid & 15;
      jb[r] = (tid >> 4) + 16 * r;
    }
  }
  double ra[4], rbv[4];
  // mapped K indices are loaded one chunk ahead of the operands they address
  int aix[4], bix[4];
  auto load_idx = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ga = k0 + ka[r], gb = k0 + kb[r];
      aix[r] = d.kidx ? (ga < d.K ? d.kidx[ga] : 0) : ga;
      bix[r] = d.bidx ? (gb < d.K ? d.bidx[gb] : 0) : gb;
    }
  };
  // the next chunk is fetched into registers while the current one is multiplied
  auto fetch = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gk = k0 + ka[r];
      ra[r] = (arow[r] >= 0 && gk < d.K) ? d.A[arow[r] + (long long)aix[r] * d.acs] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gj = j0 + jb[r], gk = k0 + kb[r];
      double v = 0.0;
      if (gj < d.N && gk < d.K) v = d.B[(long long)bix[r] * d.brs + (long long)gj * d.bcs];
      rbv[r] = v;
    }
    load_idx(k0 + 16);
  };
  // a triangular A reaches only the K chunks of the tile's rows
  const int kbeg = d.tri == 2 ? i0 : 0, kend = d.tri == 1 ? min(d.K, i0 + 64) : d.K;
  load_idx(kbeg);
  fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += 16) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      As[ka[r]][ia[r]] = ra[r];
      Bs[kb[r]][jb[r]] = rbv[r];
    }
    __syncthreads();
    if (k0 + 16 < kend) fetch(k0 + 16);
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
  store_tile32(d, acc00, acc01, acc10, acc11, i0 + rb, j0 + cb, lane);
}

__global__ __launch_bounds__(256, 4) void gemm_tiles_kernel(const GemmDesc* __restrict__ descs,
                                                          const int* __restrict__ probs,
                                                          const int* __restrict__ toff, int np) {
  const int3 t = find_tile(descs, probs, toff, np, 64, blockIdx.x);
  tile64(descs[t.x], t.y, t.z);
}

__global__ __launch_bounds__(256, 4) void gemm_tiles_kernel_p(const GemmPack pk) {
  const int3 t = find_tile_pack(pk, 64, blockIdx.x);
  tile64(pk.d[t.x], t.y, t.z);
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
                                                              const int* __restrict__ probs,
                                                              const int* __restrict__ toff, int np) {
  __shared__ float As[16][68];  // As[k][i]
  __shared__ float Bs[16][68];  // Bs[k][j]
  const int3 t = find_tile(descs, probs, toff, np, 64, blockIdx.x);
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
  double flops;
  const void* stream;
};
// One record for the process; launches may come from several host threads
// (the two factorizations built side by side), so the record is locked and
// the call-site tag and the pause flag are per thread.
struct GemmTrace {
  std::atomic<bool> on{false};
  std::mutex mu;
  std::vector<TraceEv> ev;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
  double busy = 0.0, last_busy = 0.0;  // union of the launch intervals (ms)
  long long launches = 0;
  std::map<std::string, double> tag_ms, tag_flops;
  std::map<std::string, std::array<double, 3>> kern;  // flops, bytes, dispatches per kernel
} g_trace;
thread_local std::string t_tag = "other";
thread_local bool t_paused = false;
bool tracing() { return g_trace.on.load() && !t_paused; }
void trace_push(hipEvent_t e0, hipEvent_t e1, const std::string& tag, double flops, double bytes,
                const void* stream) {
  std::lock_guard<std::mutex> lk(g_trace.mu);
  g_trace.ev.push_back(TraceEv{e0, e1, tag, flops, stream});
  g_trace.flops += flops;
  g_trace.bytes += bytes;
  g_trace.launches += 1;
  g_trace.tag_flops[tag] += flops;
}
}  // namespace

void trace_enable(bool on) { g_trace.on = on; }

void trace_kernel_work(const std::string& kernel, double flops, double bytes, double dispatches) {
  if (!tracing()) return;
  std::lock_guard<std::mutex> lk(g_trace.mu);
  auto& a = g_trace.kern[kernel];
  a[0] += flops;
  a[1] += bytes;
  a[2] += dispatches;
}

std::string trace_kernels() {
  std::lock_guard<std::mutex> lk(g_trace.mu);
  std::string out;
  for (auto& kv : g_trace.kern) {
    char buf[256];
    snprintf(buf, sizeof(buf), "%s%s:%.6g:%.6g:%.0f", out.empty() ? "" : ";", kv.first.c_str(), kv.second[0],
             kv.second[1], kv.second[2]);
    out += buf;
  }
  return out;
}

std::string trace_current() { return t_tag; }
TracePause::TracePause() : was(t_paused) { t_paused = true; }
TracePause::~TracePause() { t_paused = was; }

TraceLaunch::TraceLaunch(hipStream_t st, double fl, double by) : s(st), flops(fl), bytes(by) {
  if (!tracing()) return;
  RSF_HIP(hipEventCreate(&e0));
  RSF_HIP(hipEventCreate(&e1));
  RSF_HIP(hipEventRecord(e0, s));
}
TraceLaunch::~TraceLaunch() {
  if (!e0) return;
  (void)hipEventRecord(e1, s);
  trace_push(e0, e1, t_tag, flops, bytes, s);
}
TraceTag::TraceTag(const char* t) : prev(t_tag) { t_tag = t; }
TraceTag::~TraceTag() { t_tag = prev; }

void trace_read(double* ms, double* flops, double* bytes, long long* launches, bool reset) {
  std::lock_guard<std::mutex> lk(g_trace.mu);
  // launches on different streams may overlap: besides the summed durations,
  // the length of the union of the intervals (timestamps relative to the
  // first launch's start event)
  std::vector<std::pair<double, double>> iv;
  // RSFGP_TRACE_DUMP=<file>: one line per traced launch (start and duration
  // in ms from the first traced launch, flops, stream, tag), appended
  static const char* dump_path = std::getenv("RSFGP_TRACE_DUMP");
  FILE* dump = dump_path ? fopen(dump_path, "a") : nullptr;
  for (auto& e : g_trace.ev) {
    float t = 0.f, a = 0.f;
    RSF_HIP(hipEventSynchronize(e.b));
    RSF_HIP(hipEventElapsedTime(&t, e.a, e.b));
    RSF_HIP(hipEventElapsedTime(&a, g_trace.ev.front().a, e.a));
    iv.emplace_back((double)a, (double)a + t);
    g_trace.ms += t;
    g_trace.tag_ms[e.tag] += t;
    if (dump) fprintf(dump, "%.4f %.4f %.6e %p %s\n", a, t, e.flops, e.stream, e.tag.c_str());
  }
  if (dump) fclose(dump);
  std::sort(iv.begin(), iv.end());
  double cur0 = 0.0, cur1 = 0.0;
  bool open = false;
  for (const auto& x : iv) {
    if (open && x.first <= cur1) {
      cur1 = std::max(cur1, x.second);
    } else {
      if (open) g_trace.busy += cur1 - cur0;
      cur0 = x.first;
      cur1 = x.second;
      open = true;
    }
  }
  if (open) g_trace.busy += cur1 - cur0;
  for (auto& e : g_trace.ev) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  g_trace.ev.clear();
  g_trace.last_busy = g_trace.busy;
  if (ms) *ms = g_trace.ms;
  if (flops) *flops = g_trace.flops;
  if (bytes) *bytes = g_trace.bytes;
  if (launches) *launches = g_trace.launches;
  if (reset) {
    g_trace.ms = g_trace.flops = g_trace.bytes = g_trace.busy = 0.0;
    g_trace.launches = 0;
    g_trace.tag_ms.clear();
    g_trace.tag_flops.clear();
    g_trace.kern.clear();
  }
}

double trace_busy() {
  std::lock_guard<std::mutex> lk(g_trace.mu);
  return g_trace.last_busy;
}

std::string trace_tags() {
  std::lock_guard<std::mutex> lk(g_trace.mu);
  std::string out;
  for (auto& kv : g_trace.tag_ms) {
    char buf[160];
    snprintf(buf, sizeof(buf), "%s%s:%.3f:%.6g", out.empty() ? "" : ";", kv.first.c_str(), kv.second,
             g_trace.tag_flops[kv.first]);
    out += buf;
  }
  return out;
}

// 128 x 128 tiles for the large products, eight waves per workgroup: each
// wave owns a 64 x 32 block as 4 x 2 blocks of v_mfma_f64_16x16x4 (8
// accumulators), six LDS reads feed eight MFMAs per k-step, and the next
// 16-wide K chunk is fetched into registers while the current one is
// multiplied.  Small accumulators leave room for four waves per SIMD (two
// workgroups per CU), which hide the chunk loads better than two waves with
// 64 x 64 blocks.  One kernel per operand
// layout (A: rows contiguous or k contiguous; B: columns contiguous, with or
// without a row map, or k contiguous), chosen on the host.  Interior tiles
// and full K chunks take unchecked loads through per-thread pointers that
// advance by a fixed stride per chunk; only edge tiles pay for bounds checks.
constexpr int BT = 128;

template <bool AI, bool BJ, bool BIDX>
__device__ __forceinline__ void big_tile(const GemmDesc& dg, int ti, int tj) {
  __shared__ double As[16][BT + 5];  // odd row stride: conflict-free column writes
  __shared__ double Bs[16][BT + 5];
  const int M = dg.M, N = dg.N, K = dg.K;
  const int i0 = ti * BT, j0 = tj * BT;
  const int tid = threadIdx.x;
  constexpr int NT = 512, LPT = 2048 / NT, KST = NT / 128, RST = NT / 16;
  const bool full = (i0 + BT <= M) && (j0 + BT <= N);
  // fetch geometry (see the layout note above):
  //   AI: A(i0 + (tid & 127), k0 + (tid >> 7) + 2 r)   else A(i0 + (tid >> 4) + 16 r, k0 + (tid & 15))
  //   BJ: B(k0 + (tid >> 7) + 2 r, j0 + (tid & 127))   else B(k0 + (tid & 15), j0 + (tid >> 4) + 16 r)
  const int a_i = AI ? (tid & 127) : (tid >> 4);  // NT / 16 rows per pass
  const int a_k = AI ? (tid >> 7) : (tid & 15);
  const int b_j = BJ ? (tid & 127) : (tid >> 4);
  const int b_k = BJ ? (tid >> 7) : (tid & 15);
  const long long astr = AI ? dg.acs : dg.ars;  // AI: step along k; else: step between the 8 rows (x16)
  const long long bstr = BJ ? dg.brs : dg.bcs;
  // AI: this thread's row of A, through the row map when there is one
  const long long arow0 = AI ? (dg.aidx ? (i0 + a_i < M ? (long long)dg.aidx[i0 + a_i] : 0LL) : (long long)(i0 + a_i))
                             : (long long)(i0 + a_i) * dg.ars;
  const double* __restrict__ pa = dg.A + arow0;
  const double* __restrict__ pb = dg.B + (long long)(j0 + b_j) * (BJ ? 1 : dg.bcs);
  const int* __restrict__ bidx = dg.bidx;
  unsigned amask = 0, bmask = 0;  // bit r: row / column r of this thread is inside the problem
#pragma unroll
  for (int r = 0; r < LPT; ++r) {
    if (i0 + (AI ? a_i : a_i + RST * r) < M) amask |= 1u << r;
    if (j0 + (BJ ? b_j : b_j + RST * r) < N) bmask |= 1u << r;
  }
  v4d acc[4][2];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[m][q] = v4d{0, 0, 0, 0};
  double ra[LPT], rbv[LPT];
  // k-contiguous A may read its columns through a map (A(i, kidx[k])); one
  // index per thread and chunk.  Mapped indices are loaded one chunk ahead of
  // the operands they address, so that the operand loads do not wait for them.
  const int* __restrict__ kidx = AI ? nullptr : dg.kidx;
  int kix = 0, bix[LPT];
  auto load_idx = [&](int k0) {
    if (!AI && kidx) kix = k0 + a_k < K ? kidx[k0 + a_k] : 0;
    if (BJ && BIDX) {
#pragma unroll
      for (int r = 0; r < LPT; ++r) bix[r] = k0 + b_k + KST * r < K ? bidx[k0 + b_k + KST * r] : 0;
    }
  };
  auto fetch = [&](int k0) {
    if (full && k0 + 16 <= K) {
      const int kA = AI ? 0 : (kidx ? kix : k0 + a_k);
#pragma unroll
      for (int r = 0; r < LPT; ++r) {
        ra[r] = AI ? pa[(long long)(k0 + a_k + KST * r) * astr] : pa[(long long)(RST * r) * astr + kA];
        if (BJ) {
          const int kb = k0 + b_k + KST * r;
          rbv[r] = pb[(long long)(BIDX ? bix[r] : kb) * bstr];
        } else {
          rbv[r] = pb[(long long)(RST * r) * bstr + k0 + b_k];
        }
      }
    } else {
      const int kc = k0 + a_k;
      const int kA = AI ? 0 : (kc < K ? (kidx ? kix : kc) : 0);
#pragma unroll
      for (int r = 0; r < LPT; ++r) {
        const int ka = k0 + a_k + (AI ? KST * r : 0);
        ra[r] = ((amask >> r) & 1u) && ka < K
                    ? (AI ? pa[(long long)ka * astr] : pa[(long long)(RST * r) * astr + kA])
                    : 0.0;
        const int kb = k0 + b_k + (BJ ? KST * r : 0);
        double v = 0.0;
        if (((bmask >> r) & 1u) && kb < K)
          v = BJ ? pb[(long long)(BIDX ? bix[r] : kb) * bstr] : pb[(long long)(RST * r) * bstr + kb];
        rbv[r] = v;
      }
    }
    load_idx(k0 + 16);
  };
  // a triangular A reaches only the K chunks of the tile's rows
  const int kbeg = dg.tri == 2 ? i0 : 0, kend = dg.tri == 1 ? min(K, i0 + BT) : K;
  load_idx(kbeg);
  fetch(kbeg);
  const int lane = tid & 63, wave = tid >> 6;
  const int rb0 = (wave >> 2) * 64, cb0 = (wave & 3) * 32;
  for (int k0 = kbeg; k0 < kend; k0 += 16) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < LPT; ++r) {
      if (AI)
        As[a_k + KST * r][a_i] = ra[r];
      else
        As[a_k][a_i + RST * r] = ra[r];
      if (BJ)
        Bs[b_k + KST * r][b_j] = rbv[r];
      else
        Bs[b_k][b_j + RST * r] = rbv[r];
    }
    __syncthreads();
    if (k0 + 16 < kend) fetch(k0 + 16);
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      double a[4], b[2];
#pragma unroll
      for (int m = 0; m < 4; ++m) a[m] = As[kk][rb0 + m * 16 + (lane & 15)];
#pragma unroll
      for (int q = 0; q < 2; ++q) b[q] = Bs[kk][cb0 + q * 16 + (lane & 15)];
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[m][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b[q], acc[m][q], 0, 0, 0);
    }
  }
  const double alpha = dg.alpha, beta = dg.beta;
  const int* __restrict__ cidx = dg.cidx;
  double* __restrict__ Cb = dg.C;
  const long long crs = dg.crs, ccs = dg.ccs;
  // per 16-row block: the row map, then every C entry the update reads, are
  // loaded together before any store (a load after a store to C would wait
  // for the memory round trip of each entry in turn)
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    double* cp[4][2];
    bool ok[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gi = i0 + rb0 + m * 16 + 4 * r + (lane >> 4);
      const bool rin = full || gi < M;
      const long long row = cidx ? (rin ? (long long)cidx[gi] : 0LL) : (long long)gi;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int gj = j0 + cb0 + q * 16 + (lane & 15);
        ok[r][q] = rin && (full || gj < N);
        cp[r][q] = Cb + row * crs + (long long)gj * ccs;
      }
    }
    double cv[4][2];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q) cv[r][q] = (beta != 0.0 && ok[r][q]) ? *cp[r][q] : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (ok[r][q]) *cp[r][q] = (beta == 0.0) ? alpha * acc[m][q][r] : alpha * acc[m][q][r] + beta * cv[r][q];
  }
}

template <bool AI, bool BJ, bool BIDX>
__global__ __launch_bounds__(512, 2) void gemm_big_kernel(const GemmDesc* __restrict__ descs,
                                                           const int* __restrict__ probs,
                                                           const int* __restrict__ toff, int np) {
  const int3 t = find_tile(descs, probs, toff, np, BT, blockIdx.x);
  big_tile<AI, BJ, BIDX>(descs[t.x], t.y, t.z);
}

template <bool AI, bool BJ, bool BIDX>
__global__ __launch_bounds__(512, 2) void gemm_big_kernel_p(const GemmPack pk) {
  const int3 t = find_tile_pack(pk, BT, blockIdx.x);
  big_tile<AI, BJ, BIDX>(pk.d[t.x], t.y, t.z);
}

// layout class of a problem for the 128 x 128 kernels: bit 2 = A rows
// contiguous (else k contiguous), bit 1 = B columns contiguous (else k
// contiguous), bit 0 = B has a row map (only with contiguous columns);
// -1 = no fitting layout, use the 64 x 64 kernel
// Split-K: partial products of K slices land in a workspace (column-major,
// one M x N block per slice) and are summed in slice order into C.
struct SplitRed {
  const double* W;
  long long M, N;
  int s;
  double alpha, beta;
  double* C;
  const int* cidx;
  long long crs, ccs;
  int lower;  // only the lower triangle (i >= j) is formed
};

__global__ __launch_bounds__(256) void splitk_reduce_kernel(const SplitRed* __restrict__ jobs) {
  const SplitRed J = jobs[blockIdx.y];
  const long long tot = J.M * J.N, blk = tot;
  for (long long e = blockIdx.x * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.x) {
    const long long i = e % J.M, j = e / J.M;
    if (J.lower && i < j) continue;
    double v = 0.0;
    for (int p = 0; p < J.s; ++p) v += J.W[p * blk + e];
    const long long row = J.cidx ? (long long)J.cidx[i] : i;
    double* c = J.C + row * J.crs + j * J.ccs;
    *c = (J.beta == 0.0) ? J.alpha * v : J.alpha * v + J.beta * *c;
  }
}

static int big_class(const GemmDesc& d) {
  // rows-contiguous A may take a row map (one row pointer per thread),
  // k-contiguous A a column map
  if (d.kidx) {
    if (d.acs != 1 || d.aidx) return -1;
    const bool bj = (d.bcs == 1), bk = (d.brs == 1 && d.bidx == nullptr);
    if (!(bj || bk)) return -1;
    return (bj ? 2 : 0) | ((bj && d.bidx) ? 1 : 0);
  }
  const bool ai = d.ars == 1, ak = (d.acs == 1 && d.aidx == nullptr);
  const bool bj = (d.bcs == 1), bk = (d.brs == 1 && d.bidx == nullptr);
  if (!(ai || ak) || !(bj || bk)) return -1;
  return (ai ? 4 : 0) | (bj ? 2 : 0) | ((bj && d.bidx) ? 1 : 0);
}

// ---- tile-shape autotuning of the batched products
// Problems that fit the 128 x 128 kernels can run on the 64 x 64 one as well.
// Both accumulate every output entry over K in the same order with the same
// instruction, so the choice changes no result, only the time.  The first
// call of a launch shape (the layout classes present, the number of such
// problems and their mean M, N and K in quarter-octave buckets, lower and
// triangular problems) times both forms on scratch outputs and keeps the
// faster; later calls of that shape reuse the choice.  No-allocation calls
// and calls under stream capture run no trials (the 128 x 128 form, not
// recorded).
namespace {
struct TileKey {
  unsigned classes;
  int count, m, n, k, lower, tri;
  bool operator<(const TileKey& o) const {
    return std::tie(classes, count, m, n, k, lower, tri) < std::tie(o.classes, o.count, o.m, o.n, o.k, o.lower, o.tri);
  }
};
std::mutex g_tile_mu;
std::map<TileKey, int> g_tile;  // 1: 128 x 128 tiles, 0: 64 x 64 tiles
thread_local int g_tile_force = -1;

int quarter_octave_of(double x) { return (int)std::floor(4.0 * std::log2(std::max(1.0, x))); }

bool fits_big(const GemmDesc& d) {
  return !d.f32 && big_class(d) >= 0 && d.M >= 96 && d.N >= 96 && d.K >= 32;
}

float time_launch(hipStream_t s, const std::function<void()>& fn) {
  hipEvent_t e0, e1;
  RSF_HIP(hipEventCreate(&e0));
  RSF_HIP(hipEventCreate(&e1));
  RSF_HIP(hipEventRecord(e0, s));
  fn();
  RSF_HIP(hipEventRecord(e1, s));
  RSF_HIP(hipEventSynchronize(e1));
  float ms = 0.f;
  RSF_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return ms;
}
}  // namespace

// 1 when the problems that fit the 128 x 128 kernels take them, 0 when they
// take the 64 x 64 kernel (timed at the first call of the launch shape).
static int tile_choice(const std::vector<GemmDesc>& descs, hipStream_t s) {
  if (g_tile_force >= 0) return g_tile_force;
  // tests may fix the form for every call (read at each call)
  if (const char* e = std::getenv("RSFGP_TEST_TILES")) {
    if (!std::strcmp(e, "64")) return 0;
    if (!std::strcmp(e, "128")) return 1;
  }
  unsigned classes = 0;
  long long cnt = 0;
  double sm = 0.0, sn = 0.0, sk = 0.0;
  int lower = 0, tri = 0;
  for (const GemmDesc& d : descs) {
    if (d.M <= 0 || d.N <= 0 || !fits_big(d)) continue;
    classes |= 1u << big_class(d);
    ++cnt;
    sm += d.M;
    sn += d.N;
    sk += d.K;
    lower |= d.lower ? 1 : 0;
    tri |= d.tri ? 1 : 0;
  }
  if (cnt == 0) return 1;
  const TileKey key{classes, quarter_octave_of((double)cnt), quarter_octave_of(sm / cnt),
                    quarter_octave_of(sn / cnt), quarter_octave_of(sk / cnt), lower, tri};
  {
    std::lock_guard<std::mutex> lk(g_tile_mu);
    auto it = g_tile.find(key);
    if (it != g_tile.end()) return it->second;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  RSF_HIP(hipStreamIsCapturing(s, &cap));
  if (no_alloc_active() || cap != hipStreamCaptureStatusNone) return 1;
  // trial problems: the same operands, each C a fresh column-major block
  // written with beta = 0 (the caller's C is not touched)
  TracePause tp;
  Scratch ts(s);
  long long tot = 0;
  for (const GemmDesc& d : descs)
    if (d.M > 0 && d.N > 0 && fits_big(d)) tot += (long long)d.M * d.N;
  double* W = ts.make<double>(tot);
  std::vector<GemmDesc> trial;
  long long off = 0;
  for (const GemmDesc& d : descs) {
    if (d.M <= 0 || d.N <= 0 || !fits_big(d)) continue;
    GemmDesc e = d;
    e.C = W + off;
    e.cidx = nullptr;
    e.crs = 1;
    e.ccs = d.M;
    e.beta = 0.0;
    off += (long long)d.M * d.N;
    trial.push_back(e);
  }
  auto run = [&](int force) {
    const int was = g_tile_force;
    g_tile_force = force;
    gemm_batched(trial, ts, s);
    g_tile_force = was;
  };
  // each form runs once untimed, then three timed runs of each alternate and
  // the fastest of each counts (work that the other stream runs at the same
  // time stretches single timings); the 64 x 64 form must win by 15 %, since
  // the trials time each launch alone and the 128 x 128 tiles read less
  // beside a second stream's work
  run(1);
  run(0);
  float tb = 1e30f, tt = 1e30f;
  for (int rep = 0; rep < 3; ++rep) {
    tb = std::min(tb, time_launch(s, [&] { run(1); }));
    tt = std::min(tt, time_launch(s, [&] { run(0); }));
  }
  const int choice = tt < 0.85f * tb ? 0 : 1;
  static const bool dbg = std::getenv("RSFGP_TUNE_DEBUG") != nullptr;
  if (dbg)
    fprintf(stderr, "[tune] gemm %s classes %x probs %lld M %.0f N %.0f K %.0f: 128x128 %.3f ms 64x64 %.3f ms -> %s\n",
            t_tag.c_str(), classes, cnt, sm / cnt, sn / cnt, sk / cnt, tb, tt, choice ? "128x128" : "64x64");
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tile[key] = choice;
  return choice;
}

void gemm_batched(const std::vector<GemmDesc>& descs, Scratch& scr, hipStream_t s) {
  const int use_big = tile_choice(descs, s);
  // launch groups: 0 = 64 x 64 FP64 tiles, 1 + c = 128 x 128 tiles of layout
  // class c, 9 = 64 x 64 FP32 tiles; per group the problems and their tile
  // prefix counts (the kernels find their tile from these)
  constexpr int NG = 10;
  std::vector<int> probs[NG], toff[NG];
  for (auto& v : toff) v.push_back(0);
  std::vector<GemmDesc> live;
  double flops = 0.0, bytes = 0.0, gfl[NG] = {}, gby[NG] = {};
  // the launch group each problem takes without the tile choice, and those
  // groups' tile counts: split-K decides from these, so that the tile choice
  // changes no result
  std::vector<int> gnat;
  long long tnat[NG] = {};
  for (const GemmDesc& d : descs) {
    if (d.M <= 0 || d.N <= 0) continue;
    RSF_CHECK(!d.lower || d.M == d.N, RSF_E_INVALID, "lower-triangle GEMM needs a square C");
    RSF_CHECK(!(d.kidx && d.f32), RSF_E_INVALID, "column-mapped A needs the FP64 tile kernel");
    RSF_CHECK(!d.tri || (!d.aidx && !d.kidx && !d.f32), RSF_E_INVALID, "triangular A must be a plain matrix");
    // a triangular A (K = M) holds about half the products
    const double pf = (d.lower || d.tri ? 1.0 : 2.0) * d.M * d.N * d.K;
    const double pb = 8.0 * ((double)d.M * d.K + (double)d.K * d.N + (d.beta != 0.0 ? 2.0 : 1.0) * d.M * d.N);
    flops += pf;
    bytes += pb;
    const int p = (int)live.size();
    live.push_back(d);
    const int cls = big_class(d);
    const int gn = d.f32 ? 9 : fits_big(d) ? 1 + cls : 0;
    {
      const int tsn = gn >= 1 && gn <= 8 ? BT : 64;
      const long long tmn = (d.M + tsn - 1) / tsn, tnn = (d.N + tsn - 1) / tsn;
      tnat[gn] += d.lower ? tmn * (tmn + 1) / 2 : tmn * tnn;
      gnat.push_back(gn);
    }
    int g, ts;
    if (d.f32) {
      g = 9;
      ts = 64;
    } else if (use_big && fits_big(d)) {
      g = 1 + cls;
      ts = BT;
    } else {
      g = 0;
      ts = 64;
    }
    const long long tm = (d.M + ts - 1) / ts, tn = (d.N + ts - 1) / ts;
    const long long nt = d.lower ? tm * (tm + 1) / 2 : tm * tn;
    RSF_CHECK(toff[g].back() + nt < (1LL << 31), RSF_E_INVALID, "too many GEMM tiles in one launch");
    probs[g].push_back(p);
    toff[g].push_back(toff[g].back() + (int)nt);
    gfl[g] += pf;
    gby[g] += pb;
  }
  if (live.empty()) return;
  // Split-K for launch groups with fewer tiles than two per CU: problems with
  // a long K are cut into slices of at least 512 that run as separate
  // problems of the same launch, then summed (fixed order: deterministic).
  constexpr int SPLIT_TILES = 512, SPLIT_MIN_K = 512, SPLIT_MAX = 8;
  std::vector<SplitRed> reds;
  for (int g = 0; g < 9; ++g) {
    if (toff[g].back() == 0) continue;
    const int ts = g == 0 ? 64 : BT;
    const size_t np0 = probs[g].size();
    for (size_t u = 0; u < np0; ++u) {
      const int p = probs[g][u];
      const long long T = tnat[gnat[p]];
      if (T == 0 || T >= SPLIT_TILES) continue;
      const int want = std::min<long long>(SPLIT_MAX, SPLIT_TILES / T);
      if (want < 2) continue;
      const GemmDesc d = live[p];
      const int sp = std::min(want, d.K / SPLIT_MIN_K);
      if (d.tri || sp < 2) continue;
      const int kpart = (d.K + sp - 1) / sp / 16 * 16 + 16;
      const int nparts = (d.K + kpart - 1) / kpart;
      if (nparts < 2) continue;
      double* W = scr.make<double>((size_t)nparts * d.M * d.N);
      reds.push_back(SplitRed{W, d.M, d.N, nparts, d.alpha, d.beta, d.C, d.cidx, d.crs, d.ccs, d.lower ? 1 : 0});
      for (int q = 0; q < nparts; ++q) {
        const int k0 = q * kpart;
        GemmDesc e = d;
        e.K = std::min(kpart, d.K - k0);
        if (d.kidx)
          e.kidx = d.kidx + k0;
        else
          e.A = d.A + (long long)k0 * d.acs;
        if (d.bidx)
          e.bidx = d.bidx + k0;
        else
          e.B = d.B + (long long)k0 * d.brs;
        e.C = W + (size_t)q * d.M * d.N;
        e.cidx = nullptr;
        e.crs = 1;
        e.ccs = d.M;
        e.alpha = 1.0;
        e.beta = 0.0;
        if (q == 0) {
          live[p] = e;
        } else {
          probs[g].push_back((int)live.size());
          live.push_back(e);
        }
      }
    }
    toff[g].assign(1, 0);
    for (int p : probs[g]) {
      const GemmDesc& d = live[p];
      const long long tm = (d.M + ts - 1) / ts, tn = (d.N + ts - 1) / ts;
      const long long nt = d.lower ? tm * (tm + 1) / 2 : tm * tn;
      RSF_CHECK(toff[g].back() + nt < (1LL << 31), RSF_E_INVALID, "too many GEMM tiles in one launch");
      toff[g].push_back(toff[g].back() + (int)nt);
    }
  }
  static const bool gstats = std::getenv("RSFGP_GEMM_STATS") != nullptr;
  if (gstats) {
    // per launch group: problems, tiles, GFLOP and mean shape
    for (int g = 0; g < NG; ++g) {
      if (probs[g].empty()) continue;
      double fl = 0.0, sm = 0.0, sn = 0.0, sk = 0.0;
      for (int p : probs[g]) {
        const GemmDesc& d = live[p];
        fl += 2.0 * d.M * d.N * d.K;
        sm += d.M;
        sn += d.N;
        sk += d.K;
      }
      const double np = (double)probs[g].size();
      fprintf(stderr, "[gemm] %s g%d probs %zu tiles %d gflop %.3f M %.0f N %.0f K %.0f\n", t_tag.c_str(), g,
              probs[g].size(), toff[g].back(), fl * 1e-9, sm / np, sn / np, sk / np);
    }
  }
  // launch groups of at most PACK_NP problems pass them in the kernel
  // arguments when no group needs more (and no split-K sums are queued);
  // otherwise every table goes up in one copy
  bool packed = reds.empty();
  for (int g = 0; g < NG; ++g)
    if (!probs[g].empty() && (g == 9 || probs[g].size() > (size_t)PACK_NP)) packed = false;
  size_t po[NG] = {}, to[NG] = {};
  size_t b_desc = 0, b_cat = 0;
  char* dblk = nullptr;
  GemmDesc* dd = nullptr;
  int* dc = nullptr;
  if (!packed) {
    std::vector<int> cat;
    for (int g = 0; g < NG; ++g) {
      po[g] = cat.size();
      cat.insert(cat.end(), probs[g].begin(), probs[g].end());
      to[g] = cat.size();
      cat.insert(cat.end(), toff[g].begin(), toff[g].end());
    }
    // descriptors, problem / tile tables and split-K jobs go up in one copy
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    b_desc = al(live.size() * sizeof(GemmDesc));
    b_cat = al(cat.size() * sizeof(int));
    const size_t b_red = reds.size() * sizeof(SplitRed);
    std::vector<char> stage(b_desc + b_cat + b_red);
    std::memcpy(stage.data(), live.data(), live.size() * sizeof(GemmDesc));
    std::memcpy(stage.data() + b_desc, cat.data(), cat.size() * sizeof(int));
    if (b_red) std::memcpy(stage.data() + b_desc + b_cat, reds.data(), b_red);
    dblk = scr.make<char>(stage.size());
    upload_bytes(dblk, stage.data(), stage.size(), s);
    dd = reinterpret_cast<GemmDesc*>(dblk);
    dc = reinterpret_cast<int*>(dblk + b_desc);
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool traced = tracing();
  if (traced) {
    RSF_HIP(hipEventCreate(&e0));
    RSF_HIP(hipEventCreate(&e1));
    RSF_HIP(hipEventRecord(e0, s));
  }
  auto grid = [&](int g) { return dim3((unsigned)toff[g].back()); };
  if (packed) {
    auto pack = [&](int g) {
      GemmPack pk;
      pk.np = (int)probs[g].size();
      for (int u = 0; u < pk.np; ++u) {
        pk.d[u] = live[probs[g][u]];
        pk.toff[u] = toff[g][u];
      }
      pk.toff[pk.np] = toff[g][pk.np];
      return pk;
    };
#define RSF_PLAUNCH(KERNEL, g)                                        \
  if (!probs[g].empty()) {                                            \
    const GemmPack pk_ = pack(g);                                     \
    hipLaunchKernelGGL(KERNEL, grid(g), dim3(g == 0 ? 256 : 512), 0, s, pk_); \
  }
    RSF_PLAUNCH((gemm_big_kernel_p<true, true, true>), 1 + 7)
    RSF_PLAUNCH((gemm_big_kernel_p<true, true, false>), 1 + 6)
    RSF_PLAUNCH((gemm_big_kernel_p<true, false, false>), 1 + 4)
    RSF_PLAUNCH((gemm_big_kernel_p<false, true, true>), 1 + 3)
    RSF_PLAUNCH((gemm_big_kernel_p<false, true, false>), 1 + 2)
    RSF_PLAUNCH((gemm_big_kernel_p<false, false, false>), 1 + 0)
    RSF_PLAUNCH(gemm_tiles_kernel_p, 0)
#undef RSF_PLAUNCH
  } else {
    auto args = [&](int g) { return std::make_tuple(dc + po[g], dc + to[g], (int)probs[g].size()); };
#define RSF_LAUNCH(KERNEL, g)                                                                        \
  if (!probs[g].empty()) {                                                                           \
    auto a_ = args(g);                                                                               \
    hipLaunchKernelGGL(KERNEL, grid(g), dim3(g == 0 || g == 9 ? 256 : 512), 0, s, dd, std::get<0>(a_), std::get<1>(a_), std::get<2>(a_)); \
  }
    RSF_LAUNCH((gemm_big_kernel<true, true, true>), 1 + 7)
    RSF_LAUNCH((gemm_big_kernel<true, true, false>), 1 + 6)
    RSF_LAUNCH((gemm_big_kernel<true, false, false>), 1 + 4)
    RSF_LAUNCH((gemm_big_kernel<false, true, true>), 1 + 3)
    RSF_LAUNCH((gemm_big_kernel<false, true, false>), 1 + 2)
    RSF_LAUNCH((gemm_big_kernel<false, false, false>), 1 + 0)
    RSF_LAUNCH(gemm_tiles_kernel, 0)
    RSF_LAUNCH(gemm_tiles_f32_kernel, 9)
#undef RSF_LAUNCH
  }
  RSF_HIP(hipGetLastError());
  if (!reds.empty()) {
    SplitRed* dr = reinterpret_cast<SplitRed*>(dblk + b_desc + b_cat);
    long long mx = 1;
    for (const SplitRed& r : reds) mx = std::max(mx, r.M * r.N);
    const unsigned gx = (unsigned)std::min<long long>(1024, (mx + 255) / 256);
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(gx, (unsigned)reds.size()), dim3(256), 0, s, dr);
    RSF_HIP(hipGetLastError());
  }
  if (traced) {
    RSF_HIP(hipEventRecord(e1, s));
    // launches with FP32 products are booked under "<phase>/f32"
    trace_push(e0, e1, probs[9].empty() ? t_tag : t_tag + "/f32", flops, bytes, s);
    for (int g = 0; g < NG; ++g) {
      if (probs[g].empty()) continue;
      const char* tf[2] = {"false", "true"};
      const int c = g - 1;
      const std::string sfx = packed ? "_p" : "";
      const std::string name = g == 0 ? "gemm_tiles_kernel" + sfx
                               : g == 9 ? std::string("gemm_tiles_f32_kernel")
                                        : "gemm_big_kernel" + sfx + "<" + tf[(c >> 2) & 1] + ", " +
                                              tf[(c >> 1) & 1] + ", " + tf[c & 1] + ">";
      trace_kernel_work(name, gfl[g], gby[g]);
    }
    for (const SplitRed& r : reds) trace_kernel_work("splitk_reduce_kernel", 0.0, 8.0 * (r.s + 2.0) * r.M * r.N);
  }
}

// ---- batched blocked Cholesky with inverse
__device__ __forceinline__ void copy_block(const CopyBlock& J) {
  const long long tot = (long long)J.m * J.n;
  for (long long e = blockIdx.y * 256LL + threadIdx.x; e < tot; e += 256LL * gridDim.y) {
    const int i = (int)(e % J.m), j = (int)(e / J.m);
    J.dst[(long long)j * J.ldd + i] = (J.src == nullptr || (J.lower && i < j)) ? 0.0 : J.src[(long long)j * J.lds + i];
  }
}

__global__ __launch_bounds__(256) void copy_blocks_kernel(const CopyBlock* __restrict__ jobs) {
  const CopyBlock J = jobs[blockIdx.x];
  copy_block(J);
}

// up to JOB_PACK jobs travel in the kernel arguments (no upload before the launch)
constexpr int JOB_PACK = 32;
struct CopyPack {
  CopyBlock j[JOB_PACK];
};
__global__ __launch_bounds__(256) void copy_blocks_kernel_p(const CopyPack pk) { copy_block(pk.j[blockIdx.x]); }

void copy_blocks(const std::vector<CopyBlock>& jobs, Scratch& scr, hipStream_t s) {
  std::vector<CopyBlock> live;
  long long mx = 1;
  for (const CopyBlock& j : jobs)
    if (j.m > 0 && j.n > 0) {
      live.push_back(j);
      mx = std::max(mx, (long long)j.m * j.n);
    }
  if (live.empty()) return;
  const unsigned gy = (unsigned)std::max<long long>(1, std::min<long long>(64, (mx + 2047) / 2048));
  if (live.size() <= (size_t)JOB_PACK) {
    CopyPack pk;
    for (size_t u = 0; u < live.size(); ++u) pk.j[u] = live[u];
    hipLaunchKernelGGL(copy_blocks_kernel_p, dim3((unsigned)live.size(), gy), dim3(256), 0, s, pk);
  } else {
    CopyBlock* d = scr.make<CopyBlock>(live.size());
    upload(d, live, s);
    hipLaunchKernelGGL(copy_blocks_kernel, dim3((unsigned)live.size(), gy), dim3(256), 0, s, d);
  }
  RSF_HIP(hipGetLastError());
}

struct DiagJob {
  double* A;  // the diagonal block, ld lda
  long long lda;
  int nb;
  double* Dinv;  // 64 x 64
  double* logd;  // one value or null
};

// Cholesky of one diagonal block (nb <= 64), written back in place (zero
// above the diagonal), its log-diagonal sum and its inverse.  Thread (row
// i = tid mod 64, group g = tid / 64) keeps row i's entries in columns g,
// g + 4, ..., g + 60 in registers, as a shift register: after the four
// steps of column block jj (columns 4 jj .. 4 jj + 3) each thread's slot 0,
// now final, goes to LDS and the slots move down by one, so that every
// register index is a constant while the loop over jj stays a loop (the
// code fits the instruction cache).  Column j lives in the wave of group
// j mod 4: that wave reads the pivot from lane j, scales the column and puts
// it in LDS; after one barrier every thread updates its own entries, and the
// wave owning column j + 1 forms it at once (two LDS column buffers).  The
// inverse X = L^-1 is formed by forward substitution over the rows, column c
// of X on threads (c, g), row l in the registers of group l mod 4; the dot
// products are split over the four groups and summed in group order.
__device__ __forceinline__ void diag_chol_block(const DiagJob& J, int* fail) {
  __shared__ double colb[2][64];  // the scaled column of the current step
  __shared__ double Ls[64][65];   // L, for the inverse
  __shared__ double part[2][4][64];
  __shared__ double dg[64];
  __shared__ int bad;
  const int nb = J.nb, tid = threadIdx.x, i = tid & 63, g = tid >> 6;
  double r[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int l = g + 4 * u;
    r[u] = (i < nb && l <= i) ? J.A[(long long)l * J.lda + i] : 0.0;
  }
  if (tid == 0) bad = 0;
  // L's LDS copy starts at zero (the forward substitution below reads whole rows)
  for (int e = tid; e < 64 * 65; e += 256) (&Ls[0][0])[e] = 0.0;
  __syncthreads();
  // the owner wave of column j forms it (rv: this lane's entry of column j)
  auto form = [&](int j, double& rv) {
    // the pivot from lane j through scalar registers (j is the same in every lane)
    const unsigned long long bits = __double_as_longlong(rv);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)bits, j);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(bits >> 32), j);
    const double d = __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
    // a failed pivot is only recorded: the steps run on (their values are
    // discarded) and the flag is read once, after the loop
    if (!(d > 0.0) && i == 0) bad = 1;
    const double sq = sqrt(d);
    if (i == j) {
      rv = sq;
      dg[j] = sq;
    } else if (i > j && i < nb) {
      rv /= sq;
    }
    colb[j & 1][i] = (i >= j && i < nb) ? rv : 0.0;
  };
  if (g == 0) form(0, r[0]);
  __syncthreads();
  const int nblk = (nb + 3) >> 2;
  for (int jj = 0; jj < nblk; ++jj) {
    // slot u holds column g + 4 (u + jj)
#pragma unroll
    for (int gg = 0; gg < 4; ++gg) {
      const int j = 4 * jj + gg;
      if (j < nb) {
        // branch-free (a multiplier of zero leaves an entry unchanged), so the
        // sixteen column reads go out together
        const double lij = (i > j && i < nb) ? colb[j & 1][i] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int l = g + 4 * (u + jj);
          const double cl = colb[j & 1][l & 63];
          const double f = (l > j && l <= i) ? lij : 0.0;
          r[u] = r[u] - f * cl;
        }
        if (j + 1 < nb && g == ((gg + 1) & 3)) form(j + 1, r[gg == 3 ? 1 : 0]);
        __syncthreads();
      }
    }
    // slot 0 (column g + 4 jj) is final: to LDS and memory; shift down
    const int l0 = g + 4 * jj;
    if (i < nb && l0 < nb) {
      const double v = l0 <= i ? r[0] : 0.0;
      J.A[(long long)l0 * J.lda + i] = v;
      Ls[i][l0] = v;
    }
#pragma unroll
    for (int u = 0; u < 15; ++u) r[u] = r[u + 1];
    r[15] = 0.0;
  }
  if (bad) {
    if (tid == 0) *fail = 1;
    return;
  }
  if (tid == 0 && J.logd) {
    double sm = 0.0;
    for (int q = 0; q < nb; ++q) sm += log(dg[q]);
    *J.logd = 2.0 * sm;
  }
  __syncthreads();
  // X = L^-1: thread (c, g), rows g + 4 u of column c
  const int c = i;
  double x[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) x[u] = 0.0;
  for (int uu = 0; uu < nblk; ++uu)
#pragma unroll
    for (int gg = 0; gg < 4; ++gg) {
      const int row = 4 * uu + gg;
      if (row < nb) {
        // whole row: L is zero above the diagonal and x is still zero at
        // row and below, so the added terms are exact zeros
        double p = 0.0;
#pragma unroll
        for (int u = 0; u < 16; ++u) p += Ls[row][g + 4 * u] * x[u];
        part[row & 1][g][c] = p;
        __syncthreads();
        if (g == gg) {
          const double sm = ((part[row & 1][0][c] + part[row & 1][1][c]) + part[row & 1][2][c]) + part[row & 1][3][c];
          const double v = ((row == c ? 1.0 : 0.0) - sm) / Ls[row][row];
#pragma unroll
          for (int u = 0; u < 16; ++u)
            if (u == uu) x[u] = v;
        }
      }
    }
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int l = g + 4 * u;
    if (c < nb && l < nb) J.Dinv[(long long)c * 64 + l] = x[u];
  }
}

__global__ __launch_bounds__(256) void diag_chol_batched_kernel(const DiagJob* __restrict__ jobs, int* fail) {
  const DiagJob J = jobs[blockIdx.x];
  diag_chol_block(J, fail);
}

struct DiagPack {
  DiagJob j[JOB_PACK];
};
__global__ __launch_bounds__(256) void diag_chol_batched_kernel_p(const DiagPack pk, int* fail) {
  const DiagJob J = pk.j[blockIdx.x];
  diag_chol_block(J, fail);
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
      if (dj.size() <= (size_t)JOB_PACK) {
        DiagPack pk;
        for (size_t u = 0; u < dj.size(); ++u) pk.j[u] = dj[u];
        hipLaunchKernelGGL(diag_chol_batched_kernel_p, dim3((unsigned)dj.size()), dim3(256), 0, s, pk, fail);
      } else {
        DiagJob* d = scr.make<DiagJob>(dj.size());
        upload(d, dj, s);
        hipLaunchKernelGGL(diag_chol_batched_kernel, dim3((unsigned)dj.size()), dim3(256), 0, s, d, fail);
      }
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
