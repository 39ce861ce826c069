// Stable least-significant-digit radix sort of (key, int32 value) pairs and
// an exclusive prefix sum of int32, the two primitives of the cell-list
// build (cell keys, the Morton centre order, the cells of the reduced
// catalogues).  Both are deterministic: no result depends on scheduling.
//
// Radix pass (4-bit digits, tiles of 4096 elements, one workgroup per tile):
//  rs_hist_kernel    : digit counts of every tile, stored digit-major
//                      cnt[d * ntiles + tile], so that one exclusive scan of
//                      cnt gives every (digit, tile) its first output slot
//  (exclusive scan of cnt)
//  rs_scatter_kernel : each thread takes 16 consecutive elements; per-thread
//                      digit counts in LDS are scanned digit-major over the
//                      threads, so equal digits keep their input order
//                      (stability) and land at the scanned global slot.
//
// Exclusive scan (tiles of 4096, 256 threads of 16 consecutive elements):
//  scan_sum_kernel   : tile sums
//  scan_carry_kernel : one workgroup scans the tile sums in place
//  scan_apply_kernel : tile-local exclusive scan plus the tile's carry
#include <utility>

#include "fpcf4_internal.hpp"

namespace fpcf4 {

namespace {
constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;   // 4096
constexpr int kDigitBits = 4;
constexpr int kDigits = 1 << kDigitBits;

// Exclusive scan of one int32 per thread over the workgroup (256 threads,
// four waves); *total receives the sum of all 256.
__device__ __forceinline__ int32_t block_exclusive_scan(int32_t v, int32_t* total) {
  __shared__ int32_t wsum[kThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  int32_t before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kThreads / 64; ++k) {
    const int32_t s = wsum[k];
    if (k < wv) before += s;
    all += s;
  }
  __syncthreads();   // wsum may be reused by the next call
  *total = all;
  return before + inc - v;
}
}  // namespace

__global__ __launch_bounds__(kThreads) void scan_sum_kernel(const int32_t* __restrict__ in, int64_t n,
                                                            int32_t* __restrict__ part) {
  const int64_t base = (int64_t)blockIdx.x * kTile;
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const int64_t j = base + i * kThreads + threadIdx.x;
    if (j < n) s += in[j];
  }
  int32_t total;
  (void)block_exclusive_scan(s, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// one workgroup: exclusive scan of part[0, m) in place, 256 entries a round
__global__ __launch_bounds__(kThreads) void scan_carry_kernel(int32_t* part, int64_t m) {
  int32_t carry = 0;
  for (int64_t b = 0; b < m; b += kThreads) {
    const int64_t j = b + threadIdx.x;
    const int32_t v = j < m ? part[j] : 0;
    int32_t total;
    const int32_t ex = block_exclusive_scan(v, &total);
    if (j < m) part[j] = carry + ex;
    carry += total;
  }
}

__global__ __launch_bounds__(kThreads) void scan_apply_kernel(const int32_t* __restrict__ in, int64_t n,
                                                              const int32_t* __restrict__ part,
                                                              int32_t* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  int32_t v[kItems];
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    s += v[i];
  }
  int32_t total;
  int32_t run = part[blockIdx.x] + block_exclusive_scan(s, &total);
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

template <typename K>
__global__ __launch_bounds__(kThreads) void rs_hist_kernel(const K* __restrict__ key, int64_t n, int shift,
                                                           int64_t ntiles, int32_t* __restrict__ cnt) {
  __shared__ int32_t h[kDigits];
  if (threadIdx.x < kDigits) h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const int64_t j = base + i * kThreads + threadIdx.x;
    if (j < n) atomicAdd(&h[(int)((key[j] >> shift) & (kDigits - 1))], 1);
  }
  __syncthreads();
  if (threadIdx.x < kDigits) cnt[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// off: the exclusive scan of rs_hist_kernel's cnt
template <typename K>
__global__ __launch_bounds__(kThreads) void rs_scatter_kernel(const K* __restrict__ kin,
                                                              const int32_t* __restrict__ vin, int64_t n,
                                                              int shift, int64_t ntiles,
                                                              const int32_t* __restrict__ off,
                                                              K* __restrict__ kout, int32_t* __restrict__ vout) {
  // c[d * 256 + t]: first the count of digit d among thread t's elements, then its
  // exclusive prefix in digit-major, thread-minor order over the tile
  __shared__ int32_t c[kDigits * kThreads];
  __shared__ int32_t goff[kDigits], dbase[kDigits];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)t * kItems;
  K k[kItems];
  int32_t v[kItems];
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    const bool in = base + i < n;
    k[i] = in ? kin[base + i] : K(0);
    v[i] = in ? vin[base + i] : 0;
  }
#pragma unroll
  for (int d = 0; d < kDigits; ++d) c[d * kThreads + t] = 0;
#pragma unroll
  for (int i = 0; i < kItems; ++i)
    if (base + i < n) c[(int)((k[i] >> shift) & (kDigits - 1)) * kThreads + t] += 1;
  if (t < kDigits) goff[t] = off[t * ntiles + blockIdx.x];
  __syncthreads();
  // thread t scans the 16 entries [16 t, 16 t + 16) of c (digit t / 16)
  int32_t s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) s += c[kItems * t + j];
  int32_t total;
  int32_t run = block_exclusive_scan(s, &total);
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const int32_t x = c[kItems * t + j];
    c[kItems * t + j] = run;
    run += x;
  }
  __syncthreads();
  if (t < kDigits) dbase[t] = c[t * kThreads];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kItems; ++i) {
    if (base + i < n) {
      const int d = (int)((k[i] >> shift) & (kDigits - 1));
      const int64_t p = (int64_t)goff[d] + (c[d * kThreads + t] - dbase[d]);
      c[d * kThreads + t] += 1;
      kout[p] = k[i];
      vout[p] = v[i];
    }
  }
}

template <typename K>
__global__ void rs_copy_kernel(const K* __restrict__ ks, const int32_t* __restrict__ vs, int64_t n,
                               K* __restrict__ kd, int32_t* __restrict__ vd) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    kd[i] = ks[i];
    vd[i] = vs[i];
  }
}

namespace {
inline size_t up256(size_t v) { return (v + 255) & ~size_t(255); }
inline int64_t tiles_of(int64_t n) { return n > 0 ? (n + kTile - 1) / kTile : 1; }
}  // namespace

size_t scan_temp_bytes(int64_t n) { return up256((size_t)(tiles_of(n) + 1) * 4); }

hipError_t exclusive_scan_i32(void* tmp, size_t tmp_bytes, const int32_t* in, int32_t* out, int64_t n,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n >= (int64_t(1) << 31) || tmp_bytes < scan_temp_bytes(n)) return hipErrorInvalidValue;
  const int64_t nt = tiles_of(n);
  int32_t* part = static_cast<int32_t*>(tmp);
  hipLaunchKernelGGL(scan_sum_kernel, dim3((unsigned)nt), dim3(kThreads), 0, s, in, n, part);
  hipLaunchKernelGGL(scan_carry_kernel, dim3(1), dim3(kThreads), 0, s, part, nt);
  hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nt), dim3(kThreads), 0, s, in, n, part, out);
  return hipGetLastError();
}

size_t radix_sort_temp_bytes(int64_t n) {
  const size_t cnt = (size_t)kDigits * tiles_of(n);
  return 2 * up256(cnt * 4) + scan_temp_bytes((int64_t)cnt);
}

template <typename K>
hipError_t radix_sort_pairs(void* tmp, size_t tmp_bytes, K* key_a, K* key_b, int32_t* val_a, int32_t* val_b,
                            int64_t n, int bits, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n >= (int64_t(1) << 31) || bits < 1 || bits > (int)(8 * sizeof(K)) ||
      tmp_bytes < radix_sort_temp_bytes(n))
    return hipErrorInvalidValue;
  const int64_t nt = tiles_of(n);
  const size_t cbytes = up256((size_t)kDigits * nt * 4);
  char* t = static_cast<char*>(tmp);
  int32_t* cnt = reinterpret_cast<int32_t*>(t);
  int32_t* off = reinterpret_cast<int32_t*>(t + cbytes);
  void* stmp = t + 2 * cbytes;
  const size_t sbytes = tmp_bytes - 2 * cbytes;
  K* ks = key_a;
  K* kd = key_b;
  int32_t* vs = val_a;
  int32_t* vd = val_b;
  const int passes = (bits + kDigitBits - 1) / kDigitBits;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * kDigitBits;
    hipLaunchKernelGGL(rs_hist_kernel<K>, dim3((unsigned)nt), dim3(kThreads), 0, s, ks, n, shift, nt, cnt);
    hipError_t e = exclusive_scan_i32(stmp, sbytes, cnt, off, (int64_t)kDigits * nt, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(rs_scatter_kernel<K>, dim3((unsigned)nt), dim3(kThreads), 0, s, ks, vs, n, shift, nt,
                       off, kd, vd);
    std::swap(ks, kd);
    std::swap(vs, vd);
  }
  // after an even number of passes the result sits in the a buffers
  if (ks != key_b) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(rs_copy_kernel<K>, dim3((unsigned)blocks), dim3(256), 0, s, ks, vs, n, key_b, val_b);
  }
  return hipGetLastError();
}

template hipError_t radix_sort_pairs<uint32_t>(void*, size_t, uint32_t*, uint32_t*, int32_t*, int32_t*, int64_t,
                                               int, hipStream_t);
template hipError_t radix_sort_pairs<uint64_t>(void*, size_t, uint64_t*, uint64_t*, int32_t*, int32_t*, int64_t,
                                               int, hipStream_t);

}  // namespace fpcf4
