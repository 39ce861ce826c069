// Spatial sort of the catalogue into a row-major cell grid (the neighbour
// search structure of stage (a)), and the centre order.
//
//  bbox_kernel    : min/max of x and y and a count of non-finite inputs
//  key_kernel     : cell key cy * ncx + cx of every galaxy
//  (hipcub radix sort of (key, index) pairs: stable, deterministic)
//  starts_kernel  : cell_start[c] = first sorted position of cell c
//  gather_kernel  : sorted galaxy records (x, y, w g1, w g2, w) and the
//                   inverse permutation
//  morton_kernel  : Morton key of each sorted galaxy's cell, so that the
//                   centre list (sorted by it) visits space in compact blocks
#include <hipcub/hipcub.hpp>

#include "fpcf4_internal.hpp"

namespace fpcf4 {

__global__ void bbox_partial_kernel(const double* x, const double* y, const double* g1,
                                    const double* g2, const double* w, int64_t n,
                                    double* part /* [nblk][4] */, unsigned* bad) {
  __shared__ double s[4][256];
  double mnx = INFINITY, mxx = -INFINITY, mny = INFINITY, mxy = -INFINITY;
  unsigned nbad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double xv = x[i], yv = y[i];
    if (!isfinite(xv) || !isfinite(yv) || !isfinite(g1[i]) || !isfinite(g2[i]) || !isfinite(w[i])) {
      ++nbad;
      continue;
    }
    mnx = fmin(mnx, xv);
    mxx = fmax(mxx, xv);
    mny = fmin(mny, yv);
    mxy = fmax(mxy, yv);
  }
  s[0][threadIdx.x] = mnx;
  s[1][threadIdx.x] = mxx;
  s[2][threadIdx.x] = mny;
  s[3][threadIdx.x] = mxy;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + st]);
      s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + st]);
      s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + st]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k) part[blockIdx.x * 4 + k] = s[k][0];
  }
  if (nbad) atomicAdd(bad, nbad);
}

__global__ void bbox_final_kernel(const double* part, int nblk, double* out) {
  if (threadIdx.x != 0) return;
  double mnx = INFINITY, mxx = -INFINITY, mny = INFINITY, mxy = -INFINITY;
  for (int b = 0; b < nblk; ++b) {
    mnx = fmin(mnx, part[4 * b + 0]);
    mxx = fmax(mxx, part[4 * b + 1]);
    mny = fmin(mny, part[4 * b + 2]);
    mxy = fmax(mxy, part[4 * b + 3]);
  }
  out[0] = mnx;
  out[1] = mxx;
  out[2] = mny;
  out[3] = mxy;
}

__device__ __forceinline__ int cell_of(double v, double v0, double inv_h, int nc) {
  int c = (int)floor((v - v0) * inv_h);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void key_kernel(const double* x, const double* y, int64_t n, Grid g,
                           uint32_t* key, int32_t* idx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int cx = cell_of(x[i], g.x0, g.inv_h, g.ncx);
    const int cy = cell_of(y[i], g.y0, g.inv_h, g.ncy);
    key[i] = (uint32_t)cy * (uint32_t)g.ncx + (uint32_t)cx;
    idx[i] = (int32_t)i;
  }
}

// cell_start[c] for c in (skey[i-1], skey[i]] is i; the tail up to ncells gets n.
__global__ void starts_kernel(const uint32_t* skey, int64_t n, int64_t ncells, int32_t* start) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t prev = (i == 0) ? -1 : (int64_t)skey[i - 1];
    const int64_t cur = (i == n) ? ncells : (int64_t)skey[i];
    for (int64_t c = prev + 1; c <= cur; ++c) start[c] = (int32_t)i;
  }
}

template <typename T>
__global__ void gather_kernel(const double* x, const double* y, const double* g1,
                              const double* g2, const double* w, const int32_t* perm,
                              int64_t n, Gal<T>* gal, int32_t* inv) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t p = perm[i];
    const double wv = w[p];
    Gal<T> r{};
    r.x = x[p];
    r.y = y[p];
    r.a = (T)(wv * g1[p]);
    r.b = (T)(wv * g2[p]);
    r.w = (T)wv;
    gal[i] = r;
    if (inv) inv[p] = (int32_t)i;
  }
}

__device__ __forceinline__ uint32_t spread16(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__global__ void morton_kernel(const uint32_t* skey, int64_t n, int ncx, uint32_t* mkey,
                              int32_t* idx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = skey[i];
    const uint32_t cy = k / (uint32_t)ncx, cx = k - cy * (uint32_t)ncx;
    mkey[i] = spread16(cx) | (spread16(cy) << 1);
    idx[i] = (int32_t)i;
  }
}

__global__ void map_centres_kernel(const int64_t* centres, int64_t nc, const int32_t* inv,
                                   int32_t* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nc;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = inv[centres[i]];
}

static inline int grid1d(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t cells_bbox(const double* x, const double* y, const double* g1, const double* g2,
                      const double* w, int64_t n, double* part, unsigned* bad, double* out,
                      hipStream_t s) {
  const int nblk = 256;
  hipLaunchKernelGGL(bbox_partial_kernel, dim3(nblk), dim3(256), 0, s, x, y, g1, g2, w, n, part, bad);
  hipLaunchKernelGGL(bbox_final_kernel, dim3(1), dim3(64), 0, s, part, nblk, out);
  return hipGetLastError();
}

size_t cells_sort_temp_bytes(int64_t n) {
  size_t b1 = 0, b2 = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b1, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const int32_t*)nullptr, (int32_t*)nullptr, (int)n, 0, 32);
  b2 = b1 + 4096;
  return b1 > b2 ? b1 : b2;
}

static int bits_for(uint64_t v) {
  int b = 1;
  while (b < 32 && (1ull << b) <= v) ++b;
  return b;
}

// Builds the sorted galaxy records and cell starts.  All scratch arrays are
// caller-provided; gal holds Gal<double> when fp64 != 0, else Gal<float>.
hipError_t cells_build(const double* x, const double* y, const double* g1, const double* g2,
                       const double* w, int64_t n, const Grid& g, uint32_t* key_a,
                       uint32_t* key_b, int32_t* idx_a, int32_t* idx_b, void* sort_tmp,
                       size_t sort_tmp_bytes, void* gal, int fp64, int32_t* cell_start,
                       int32_t* inv, hipStream_t s) {
  const int64_t ncells = (int64_t)g.ncx * g.ncy;
  hipLaunchKernelGGL(key_kernel, dim3(grid1d(n)), dim3(256), 0, s, x, y, n, g, key_a, idx_a);
  size_t tb = sort_tmp_bytes;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(sort_tmp, tb, key_a, key_b, idx_a, idx_b, (int)n,
                                                    0, bits_for((uint64_t)ncells), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(starts_kernel, dim3(grid1d(n + 1)), dim3(256), 0, s, key_b, n, ncells, cell_start);
  if (fp64)
    hipLaunchKernelGGL(gather_kernel<double>, dim3(grid1d(n)), dim3(256), 0, s, x, y, g1, g2, w, idx_b,
                       n, reinterpret_cast<Gal<double>*>(gal), inv);
  else
    hipLaunchKernelGGL(gather_kernel<float>, dim3(grid1d(n)), dim3(256), 0, s, x, y, g1, g2, w, idx_b,
                       n, reinterpret_cast<Gal<float>*>(gal), inv);
  return hipGetLastError();
}

// Morton-ordered list of all sorted positions (uses key_b from cells_build).
hipError_t cells_centre_order(const uint32_t* skey, int64_t n, const Grid& g, uint32_t* mkey_a,
                              uint32_t* mkey_b, int32_t* idx_a, int32_t* out, void* sort_tmp,
                              size_t sort_tmp_bytes, hipStream_t s) {
  hipLaunchKernelGGL(morton_kernel, dim3(grid1d(n)), dim3(256), 0, s, skey, n, g.ncx, mkey_a, idx_a);
  size_t tb = sort_tmp_bytes;
  return hipcub::DeviceRadixSort::SortPairs(sort_tmp, tb, mkey_a, mkey_b, idx_a, out, (int)n, 0, 32, s);
}

hipError_t cells_map_centres(const int64_t* centres, int64_t nc, const int32_t* inv, int32_t* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(map_centres_kernel, dim3(grid1d(nc)), dim3(256), 0, s, centres, nc, inv, out);
  return hipGetLastError();
}

}  // namespace fpcf4
