// Utility kernels: fills, prefix sums, deterministic reductions, hashing.
#include <map>
#include <mutex>

#include "fpc_internal.hpp"

namespace fpc {

namespace {

template <typename T>
__global__ void k_fill(T* p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

constexpr int SCAN_T = 256, SCAN_E = 8, SCAN_CH = SCAN_T * SCAN_E;

__global__ __launch_bounds__(SCAN_T) void k_scan_bsum(const int64_t* in,
                                                      int64_t n,
                                                      int64_t* bsum) {
  __shared__ int64_t sh[SCAN_T];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * SCAN_CH + (int64_t)tid * SCAN_E;
  int64_t acc = 0;
  for (int e = 0; e < SCAN_E; ++e) {
    int64_t i = base + e;
    if (i < n) acc += in[i];
  }
  sh[tid] = acc;
  __syncthreads();
  for (int s = SCAN_T / 2; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  if (tid == 0) bsum[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(SCAN_T) void k_scan_apply(const int64_t* in,
                                                       int64_t n,
                                                       const int64_t* boff,
                                                       int64_t* out) {
  __shared__ int64_t sh[SCAN_T];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * SCAN_CH + (int64_t)tid * SCAN_E;
  int64_t v[SCAN_E];
  int64_t acc = 0;
  for (int e = 0; e < SCAN_E; ++e) {
    int64_t i = base + e;
    v[e] = (i < n) ? in[i] : 0;
    acc += v[e];
  }
  sh[tid] = acc;
  __syncthreads();
  for (int off = 1; off < SCAN_T; off <<= 1) {
    int64_t t = (tid >= off) ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += t;
    __syncthreads();
  }
  int64_t run = (boff ? boff[blockIdx.x] : 0) + sh[tid] - acc;
  for (int e = 0; e < SCAN_E; ++e) {
    int64_t i = base + e;
    run += v[e];
    if (i < n) out[i + 1] = run;
  }
  if (blockIdx.x == 0 && tid == 0) out[0] = 0;
}

__global__ void k_i32_to_i64(const int32_t* in, int64_t* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

constexpr int RED_T = 256;

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(RED_T) void k_dot_partial(const double* x,
                                                       const double* y,
                                                       int64_t n,
                                                       double* partials) {
  __shared__ double sh[RED_T / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * RED_T + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * RED_T)
    acc += x[i] * y[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < RED_T / 64; ++w) t += sh[w];
    partials[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(RED_T) void k_sum_partials(const double* partials,
                                                        int np, double* out) {
  __shared__ double sh[RED_T / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += RED_T) acc += partials[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < RED_T / 64; ++w) t += sh[w];
    out[0] = t;
  }
}

__global__ void k_hash(uint32_t first, int64_t n, uint32_t* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = lowbias32(first + (uint32_t)i);
}

__global__ void k_check_finite(const double* v, int64_t n, int* flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (; i < n; i += stride) bad |= !isfinite(v[i]);
  if (bad) atomicOr(&flags[FLAG_NAN], 1);
}

__global__ void k_cast(const double* in, float* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

}  // namespace

void fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = grid_for(n, 256);
  if (g > 65536) g = 65536;
  k_fill<double><<<g, 256, 0, s>>>(p, v, n);
  FPC_LAUNCH_CHECK();
}
void fill_f32(float* p, float v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = grid_for(n, 256);
  if (g > 65536) g = 65536;
  k_fill<float><<<g, 256, 0, s>>>(p, v, n);
  FPC_LAUNCH_CHECK();
}
void fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = grid_for(n, 256);
  if (g > 65536) g = 65536;
  k_fill<int32_t><<<g, 256, 0, s>>>(p, v, n);
  FPC_LAUNCH_CHECK();
}
void fill_i64(int64_t* p, int64_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = grid_for(n, 256);
  if (g > 65536) g = 65536;
  k_fill<int64_t><<<g, 256, 0, s>>>(p, v, n);
  FPC_LAUNCH_CHECK();
}

void scan_counts(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) {
    fill_i64(out, 0, 1, s);
    return;
  }
  int64_t nb = (n + SCAN_CH - 1) / SCAN_CH;
  if (nb == 1) {
    k_scan_apply<<<1, SCAN_T, 0, s>>>(in, n, nullptr, out);
    FPC_LAUNCH_CHECK();
    return;
  }
  DevBuf<int64_t> bsum(nb), boff(nb + 1);
  k_scan_bsum<<<(unsigned)nb, SCAN_T, 0, s>>>(in, n, bsum.p);
  FPC_LAUNCH_CHECK();
  scan_counts(bsum.p, boff.p, nb, s);
  k_scan_apply<<<(unsigned)nb, SCAN_T, 0, s>>>(in, n, boff.p, out);
  FPC_LAUNCH_CHECK();
  // the temporaries are released in stream order: no wait needed
}

int64_t scan_counts_total(const int64_t* in, int64_t* out, int64_t n,
                          hipStream_t s) {
  scan_counts(in, out, n, s);
  return read_i64(out + n, s);
}

void i32_to_i64(const int32_t* in, int64_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_i32_to_i64<<<grid_for(n, 256), 256, 0, s>>>(in, out, n);
  FPC_LAUNCH_CHECK();
}

void dot_f64(const double* x, const double* y, int64_t n, double* out,
             double* partials, hipStream_t s) {
  k_dot_partial<<<kRedBlocks, RED_T, 0, s>>>(x, y, n, partials);
  FPC_LAUNCH_CHECK();
  k_sum_partials<<<1, RED_T, 0, s>>>(partials, kRedBlocks, out);
  FPC_LAUNCH_CHECK();
}

void hash32_range(uint32_t first, int64_t n, uint32_t* out, hipStream_t s) {
  if (n <= 0) return;
  k_hash<<<grid_for(n, 256), 256, 0, s>>>(first, n, out);
  FPC_LAUNCH_CHECK();
}

void check_finite(const double* v, int64_t n, int* flags, hipStream_t s) {
  if (n <= 0) return;
  unsigned g = grid_for(n, 256);
  if (g > 4096) g = 4096;
  k_check_finite<<<g, 256, 0, s>>>(v, n, flags);
  FPC_LAUNCH_CHECK();
}

void cast_f64_f32(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast<<<grid_for(n, 256), 256, 0, s>>>(in, out, n);
  FPC_LAUNCH_CHECK();
}

// a = b + scalar * c.  Main part: each thread moves four 16-byte pairs, all
// loads issued before the stores, nontemporal (the arrays are streamed
// once); 1024 pairs per block.  The rest (fewer than 2049 doubles) by a
// plain one-element-per-thread kernel.
typedef double dpair __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void k_triad(const dpair* __restrict__ b,
                                               const dpair* __restrict__ c,
                                               double scalar,
                                               dpair* __restrict__ a) {
  const int64_t base = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  dpair x[4], y[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    x[u] = __builtin_nontemporal_load(b + base + 256 * u);
    y[u] = __builtin_nontemporal_load(c + base + 256 * u);
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const dpair r = {x[u].x + scalar * y[u].x, x[u].y + scalar * y[u].y};
    __builtin_nontemporal_store(r, a + base + 256 * u);
  }
}

__global__ void k_triad_tail(const double* b, const double* c, double scalar,
                             double* a, int64_t i0, int64_t n) {
  const int64_t i = i0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = b[i] + scalar * c[i];
}

void stream_triad(const double* b, const double* c, double scalar, double* a,
                  int64_t n, hipStream_t s) {
  if (n <= 0) return;
  if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) & 15)
    throw Error(FPC_ERR_ARG, "stream_triad: arrays must be 16-byte aligned");
  const int64_t nblk = n / 2048;  // 1024 pairs each
  if (nblk)
    k_triad<<<(unsigned)nblk, 256, 0, s>>>((const dpair*)b, (const dpair*)c,
                                           scalar, (dpair*)a);
  const int64_t i0 = nblk * 2048;
  if (i0 < n)
    k_triad_tail<<<grid_for(n - i0, 256), 256, 0, s>>>(b, c, scalar, a, i0, n);
  FPC_LAUNCH_CHECK();
}

template <typename I>
__global__ void k_neq(const I* a, const I* b, int64_t n, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && a[i] != b[i]) atomicOr(flag, 1);
}

bool same_pattern(const int64_t* rp_a, const int32_t* col_a,
                  const int64_t* rp_b, const int32_t* col_b, int64_t nrows,
                  int64_t nnz, hipStream_t s) {
  DevBuf<int> f(1);
  FPC_HIP(hipMemsetAsync(f.p, 0, sizeof(int), s));
  k_neq<int64_t><<<grid_for(nrows + 1, 256), 256, 0, s>>>(rp_a, rp_b,
                                                          nrows + 1, f.p);
  if (nnz > 0)
    k_neq<int32_t><<<grid_for(nnz, 256), 256, 0, s>>>(col_a, col_b, nnz, f.p);
  FPC_LAUNCH_CHECK();
  return read_i32(f.p, s) == 0;
}

bool same_values(const double* a, const double* b, int64_t n, hipStream_t s) {
  if (n <= 0) return true;
  DevBuf<int> f(1);
  fill_i32(f.p, 0, 1, s);
  k_neq<uint64_t><<<grid_for(n, 256), 256, 0, s>>>(
      reinterpret_cast<const uint64_t*>(a), reinterpret_cast<const uint64_t*>(b),
      n, f.p);
  FPC_LAUNCH_CHECK();
  return read_i32(f.p, s) == 0;
}

// ------------------------------------------------------- block cache
namespace {

constexpr size_t kDevCacheLimit = size_t(8) << 30;
struct CacheKey {
  int dev;
  hipStream_t s;
  size_t cap;
  bool operator<(const CacheKey& o) const {
    if (dev != o.dev) return dev < o.dev;
    if (s != o.s) return s < o.s;
    return cap < o.cap;
  }
};
std::mutex g_cache_mu;
std::map<CacheKey, std::vector<void*>> g_cache;
size_t g_cached = 0;

// size classes: 256 B, then eight steps per power of two (at most 1/8
// rounded up)
size_t size_class(size_t b) {
  if (b <= 256) return 256;
  int e = 63 - __builtin_clzll((unsigned long long)(b - 1));
  const size_t base = size_t(1) << e, step = base / 8;
  return base + ((b - base + step - 1) / step) * step;
}

int current_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}

}  // namespace

void* dev_alloc(size_t bytes, hipStream_t s, size_t* cap) {
  const size_t c = size_class(bytes);
  const CacheKey key{current_device(), s, c};
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end() && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      g_cached -= c;
      *cap = c;
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMallocAsync(&p, c, s);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    dev_cache_trim();
    e = hipMallocAsync(&p, c, s);
  }
  if (e != hipSuccess)
    throw Error(e == hipErrorOutOfMemory ? FPC_ERR_OOM : FPC_ERR_HIP,
                std::string("hipMallocAsync: ") + hipGetErrorString(e));
  *cap = c;
  return p;
}

void dev_free(void* p, size_t cap, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (g_cached + cap <= kDevCacheLimit) {
      g_cache[CacheKey{current_device(), s, cap}].push_back(p);
      g_cached += cap;
      return;
    }
  }
  (void)hipFreeAsync(p, s);
}

// Every cached block back to the pool, on the stream it was last used on
// (the device current for each is the one it belongs to).
void dev_cache_trim() {
  std::map<CacheKey, std::vector<void*>> all;
  {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    all.swap(g_cache);
    g_cached = 0;
  }
  const int home = current_device();
  int cur = home;
  for (auto& kv : all) {
    if (kv.first.dev != cur) {
      (void)hipSetDevice(kv.first.dev);
      cur = kv.first.dev;
    }
    for (void* p : kv.second) (void)hipFreeAsync(p, kv.first.s);
  }
  if (cur != home) (void)hipSetDevice(home);
}

hipStream_t& alloc_stream() {
  static thread_local hipStream_t s = nullptr;
  return s;
}

double read_f64(const double* p, hipStream_t s) {
  double v = 0;
  FPC_HIP(hipMemcpyAsync(&v, p, sizeof(double), hipMemcpyDeviceToHost, s));
  FPC_HIP(hipStreamSynchronize(s));
  return v;
}
int64_t read_i64(const int64_t* p, hipStream_t s) {
  int64_t v = 0;
  FPC_HIP(hipMemcpyAsync(&v, p, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  FPC_HIP(hipStreamSynchronize(s));
  return v;
}
int read_i32(const int32_t* p, hipStream_t s) {
  int32_t v = 0;
  FPC_HIP(hipMemcpyAsync(&v, p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  FPC_HIP(hipStreamSynchronize(s));
  return v;
}

}  // namespace fpc
