// Spatial sort of the catalogue into a row-major cell grid (the neighbour
// search structure of stage (a)), and the centre order.
//
//  bbox_kernel    : min/max of x and y and a count of non-finite inputs
//  key_kernel     : cell key cy * ncx + cx of every galaxy
//  (radix_sort_pairs of (key, index) pairs: stable, deterministic)
//  starts_kernel  : cell_start[c] = first sorted position of cell c
//  gather_kernel  : sorted galaxy records (x, y, w g1, w g2, w) and the
//                   inverse permutation
//  morton_kernel  : Morton key of each sorted galaxy's cell, so that the
//                   centre list (sorted by it) visits space in compact blocks
#include <algorithm>

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

size_t cells_sort_temp_bytes(int64_t n) { return radix_sort_temp_bytes(n); }

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
  hipError_t e = radix_sort_pairs(sort_tmp, sort_tmp_bytes, key_a, key_b, idx_a, idx_b, n, bits_for((uint64_t)ncells), s);
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

// Morton-ordered list of all sorted positions (uses key_b from cells_build;
// mkey_a and idx_a are overwritten).
hipError_t cells_centre_order(const uint32_t* skey, int64_t n, const Grid& g, uint32_t* mkey_a,
                              uint32_t* mkey_b, int32_t* idx_a, int32_t* out, void* sort_tmp,
                              size_t sort_tmp_bytes, hipStream_t s) {
  hipLaunchKernelGGL(morton_kernel, dim3(grid1d(n)), dim3(256), 0, s, skey, n, g.ncx, mkey_a, idx_a);
  // cell coordinates below 2^b interleave into keys below 2^(2b); spread16
  // keeps 16 bits of each coordinate
  const int b = bits_for((uint64_t)std::max(g.ncx, g.ncy));
  return radix_sort_pairs(sort_tmp, sort_tmp_bytes, mkey_a, mkey_b, idx_a, out, n, b > 16 ? 32 : 2 * b, s);
}

// ---------------------------------------------------------------------------
// Reduced catalogues (tree approximation): one pseudo-galaxy per non-empty
// cell of side delta anchored at (x0, y0), at the cell's w-weighted centre
// of mass, carrying the cell sums of every family weight.
// ---------------------------------------------------------------------------
constexpr int RED_FIELDS = 14;   // x, y, a, b, c, d, e, v, w, p3, q3, ea, eb, u

__global__ void rkey_kernel(const double* x, const double* y, int64_t n, double x0, double y0,
                            double delta, int64_t nx, int64_t ny, uint64_t* key, int32_t* idx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t ix = (int64_t)floor((x[i] - x0) / delta);
    int64_t iy = (int64_t)floor((y[i] - y0) / delta);
    ix = ix < 0 ? 0 : (ix >= nx ? nx - 1 : ix);
    iy = iy < 0 ? 0 : (iy >= ny ? ny - 1 : iy);
    key[i] = (uint64_t)iy * (uint64_t)nx + (uint64_t)ix;
    idx[i] = (int32_t)i;
  }
}

__global__ void rhead_kernel(const uint64_t* key, int64_t n, int32_t* head) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    head[i] = (i == 0 || key[i] != key[i - 1]) ? 1 : 0;
}

// segstart[s] = first sorted position of cell segment s; segstart[m] = n
__global__ void rsegstart_kernel(const int32_t* head, const int32_t* segid, int64_t n,
                                 int32_t* segstart) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (head[i]) segstart[segid[i]] = (int32_t)i;
    if (i == n - 1) segstart[segid[i] + head[i]] = (int32_t)n;
  }
}

// Cell sums in binary64, galaxies of a cell in catalogue order (the sort is
// stable), products and sums rounded separately; pd[field][m].
__global__ void rsum_kernel(const double* x, const double* y, const double* g1, const double* g2,
                            const double* w, const int32_t* perm, const int32_t* head,
                            const int32_t* segid, const int32_t* segstart, int64_t n,
                            double* pd) {
#pragma clang fp contract(off)
  const int64_t m = (int64_t)segid[n - 1] + head[n - 1];
  for (int64_t sg = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; sg < m;
       sg += (int64_t)gridDim.x * blockDim.x) {
    double W = 0, WX = 0, WY = 0, SX = 0, SY = 0, A = 0, B = 0, C = 0, D = 0, E = 0, V = 0;
    double P3 = 0, Q3 = 0, EA = 0, EB = 0, U = 0;
    const int32_t t0 = segstart[sg], t1 = segstart[sg + 1];
    for (int32_t t = t0; t < t1; ++t) {
      const int32_t p = perm[t];
      const double wv = w[p], xv = x[p], yv = y[p];
      const double gr = wv * g1[p], gi = wv * g2[p];
      const double cr = gr * gr - gi * gi, ci = 2.0 * gr * gi;
      const double ab = gr * gr + gi * gi;
      W += wv;
      WX += wv * xv;
      WY += wv * yv;
      SX += xv;
      SY += yv;
      A += gr;
      B += gi;
      C += cr;
      D += ci;
      E += ab;
      V += wv * wv;
      P3 += cr * gr - ci * gi;
      Q3 += cr * gi + ci * gr;
      EA += ab * gr;
      EB += ab * gi;
      U += wv * wv * wv;
    }
    const double cnt = (double)(t1 - t0);
    const double f[RED_FIELDS] = {W != 0.0 ? WX / W : SX / cnt, W != 0.0 ? WY / W : SY / cnt,
                                  A, B, C, D, E, V, W, P3, Q3, EA, EB, U};
#pragma unroll
    for (int k = 0; k < RED_FIELDS; ++k) pd[k * n + sg] = f[k];
  }
}

__global__ void rgather_kernel(const double* pd, int64_t ldp, const int32_t* perm, int64_t m,
                               GalR<float>* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = perm[i];
    GalR<float> r;
    r.x = pd[0 * ldp + p];
    r.y = pd[1 * ldp + p];
    r.a = (float)pd[2 * ldp + p];
    r.b = (float)pd[3 * ldp + p];
    r.c = (float)pd[4 * ldp + p];
    r.d = (float)pd[5 * ldp + p];
    r.e = (float)pd[6 * ldp + p];
    r.v = (float)pd[7 * ldp + p];
    r.w = (float)pd[8 * ldp + p];
    r.p3 = (float)pd[9 * ldp + p];
    r.q3 = (float)pd[10 * ldp + p];
    r.ea = (float)pd[11 * ldp + p];
    r.eb = (float)pd[12 * ldp + p];
    r.u = (float)pd[13 * ldp + p];
    out[i] = r;
  }
}

// pseudo-galaxy of every galaxy: seg_final[segment] = final index, then
// out[original index] = seg_final[segment of its sorted position]
__global__ void rinvert_kernel(const int32_t* pb, int64_t m, int32_t* seg_final) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    seg_final[pb[i]] = (int32_t)i;
}
__global__ void rmember_kernel(const int32_t* ib, const int32_t* head, const int32_t* segid,
                               const int32_t* seg_final, int64_t n, int32_t* out) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    out[ib[t]] = seg_final[segid[t] + head[t] - 1];
}

namespace {
struct RedLayout {
  size_t k64a, k64b, ia, ib, head, segid, segstart, pd, ka, kb, pa, pb, tmp, tmp_bytes, total;
};
RedLayout red_layout(int64_t n) {
  const int64_t nn = n > 0 ? n : 1;
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  const size_t tsort = radix_sort_temp_bytes(nn), tsc = scan_temp_bytes(nn);
  RedLayout L{};
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o += up(b); return r; };
  L.k64a = take(nn * 8);
  L.k64b = take(nn * 8);
  L.ia = take(nn * 4);
  L.ib = take(nn * 4);
  L.head = take(nn * 4);
  L.segid = take(nn * 4);
  L.segstart = take((nn + 1) * 4);
  L.pd = take((size_t)RED_FIELDS * nn * 8);
  L.ka = take(nn * 4);
  L.kb = take(nn * 4);
  L.pa = take(nn * 4);
  L.pb = take(nn * 4);
  L.tmp_bytes = std::max(tsort, tsc);
  L.tmp = take(L.tmp_bytes);
  L.total = o;
  return L;
}
}  // namespace

size_t reduced_scratch_bytes(int64_t n) { return red_layout(n).total; }

hipError_t reduced_build(const double* x, const double* y, const double* g1, const double* g2,
                         const double* w, int64_t n, double x0, double y0, double xmax, double ymax,
                         double delta, const Grid& g, void* scratch, void* gal_out,
                         int32_t* cell_start, int64_t* m_out, hipStream_t s, int32_t* member) {
  *m_out = 0;
  if (n <= 0) return hipSuccess;
  const RedLayout L = red_layout(n);
  char* sc = static_cast<char*>(scratch);
  auto at = [&](size_t o) { return sc + o; };
  uint64_t* k64a = reinterpret_cast<uint64_t*>(at(L.k64a));
  uint64_t* k64b = reinterpret_cast<uint64_t*>(at(L.k64b));
  int32_t* ia = reinterpret_cast<int32_t*>(at(L.ia));
  int32_t* ib = reinterpret_cast<int32_t*>(at(L.ib));
  int32_t* head = reinterpret_cast<int32_t*>(at(L.head));
  int32_t* segid = reinterpret_cast<int32_t*>(at(L.segid));
  int32_t* segstart = reinterpret_cast<int32_t*>(at(L.segstart));
  double* pd = reinterpret_cast<double*>(at(L.pd));
  uint32_t* ka = reinterpret_cast<uint32_t*>(at(L.ka));
  uint32_t* kb = reinterpret_cast<uint32_t*>(at(L.kb));
  int32_t* pa = reinterpret_cast<int32_t*>(at(L.pa));
  int32_t* pb = reinterpret_cast<int32_t*>(at(L.pb));
  void* tmp = at(L.tmp);
  const int64_t nx = (int64_t)floor((xmax - x0) / delta) + 1;
  const int64_t ny = (int64_t)floor((ymax - y0) / delta) + 1;
  if (nx <= 0 || ny <= 0 || (double)nx * (double)ny >= 1.8e19) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rkey_kernel, dim3(grid1d(n)), dim3(256), 0, s, x, y, n, x0, y0, delta, nx, ny, k64a, ia);
  int kbits = 1;
  while (kbits < 64 && (1ull << kbits) <= (uint64_t)nx * (uint64_t)ny) ++kbits;
  hipError_t e = radix_sort_pairs(tmp, L.tmp_bytes, k64a, k64b, ia, ib, n, kbits, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rhead_kernel, dim3(grid1d(n)), dim3(256), 0, s, k64b, n, head);
  e = exclusive_scan_i32(tmp, L.tmp_bytes, head, segid, n, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(rsegstart_kernel, dim3(grid1d(n)), dim3(256), 0, s, head, segid, n, segstart);
  hipLaunchKernelGGL(rsum_kernel, dim3(grid1d(n)), dim3(256), 0, s, x, y, g1, g2, w, ib, head, segid,
                     segstart, n, pd);
  int32_t hm[2] = {0, 0};
  e = hipMemcpyAsync(&hm[0], segid + (n - 1), 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&hm[1], head + (n - 1), 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  const int64_t m = (int64_t)hm[0] + hm[1];
  // search-grid order of the pseudo-galaxies, cell starts, records
  const int64_t ncells = (int64_t)g.ncx * g.ncy;
  hipLaunchKernelGGL(key_kernel, dim3(grid1d(m)), dim3(256), 0, s, pd, pd + n, m, g, ka, pa);
  e = radix_sort_pairs(tmp, L.tmp_bytes, ka, kb, pa, pb, m, bits_for((uint64_t)ncells), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(starts_kernel, dim3(grid1d(m + 1)), dim3(256), 0, s, kb, m, ncells, cell_start);
  hipLaunchKernelGGL(rgather_kernel, dim3(grid1d(m)), dim3(256), 0, s, pd, n, pb, m,
                     reinterpret_cast<GalR<float>*>(gal_out));
  if (member != nullptr) {
    // pa is free once the sort has consumed it
    hipLaunchKernelGGL(rinvert_kernel, dim3(grid1d(m)), dim3(256), 0, s, pb, m, pa);
    hipLaunchKernelGGL(rmember_kernel, dim3(grid1d(n)), dim3(256), 0, s, ib, head, segid, pa, n, member);
  }
  *m_out = m;
  return hipGetLastError();
}

hipError_t cells_map_centres(const int64_t* centres, int64_t nc, const int32_t* inv, int32_t* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(map_centres_kernel, dim3(grid1d(nc)), dim3(256), 0, s, centres, nc, inv, out);
  return hipGetLastError();
}

}  // namespace fpcf4
