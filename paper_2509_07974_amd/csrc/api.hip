// Host side of the C ABI: validation, planning, workspace layout and the
// request life cycle (create -> step per centre tile -> finalize).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fpcf4_internal.hpp"

namespace fpcf4 {
hipError_t cells_bbox(const double*, const double*, const double*, const double*, const double*,
                      int64_t, double*, unsigned*, double*, hipStream_t);
size_t cells_sort_temp_bytes(int64_t n);
hipError_t cells_build(const double*, const double*, const double*, const double*, const double*,
                       int64_t, const Grid&, uint32_t*, uint32_t*, int32_t*, int32_t*, void*, size_t,
                       void*, int, int32_t*, int32_t*, hipStream_t);
hipError_t cells_centre_order(const uint32_t*, int64_t, const Grid&, uint32_t*, uint32_t*, int32_t*,
                              int32_t*, void*, size_t, hipStream_t);
hipError_t cells_map_centres(const int64_t*, int64_t, const int32_t*, int32_t*, hipStream_t);
hipError_t natural_triplets(const double* ups, int nb, int nmax, int nphi, const int32_t* trip,
                            int64_t ntrip, double* sel, double* tmp, double* binned, double* gamma,
                            double* norm, hipStream_t s);
hipError_t natural_components(const double* ups_dev, int nb, int nmax, int nphi, double* tmp,
                              double* gamma_dev, double* norm_dev, hipStream_t s);
}  // namespace fpcf4

using namespace fpcf4;

namespace {

thread_local std::string g_err;

fpcf4_status fail(fpcf4_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(call)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(e_ == hipErrorOutOfMemory ? FPCF4_E_OUT_OF_MEMORY : FPCF4_E_DEVICE,  \
                  "%s failed: %s", #call, hipGetErrorString(e_));                      \
  } while (0)

constexpr size_t ALIGN = 256;
inline size_t up(size_t v) { return (v + ALIGN - 1) & ~(ALIGN - 1); }

// Default centre tile: records of one tile stay below this many bytes.
constexpr size_t kTileRecordBudget = size_t(32) << 30;
// Centre slices of the pair contraction each own a binary64 partial of all
// work items; their number is cut so the partials stay below this many bytes
// (one slice at least: at 65 bins and nmax 15 one slice is about 10 GB).
constexpr size_t kPairPartialBudget = size_t(48) << 30;
// Scheduling counters of stage (a) (8 per launch, two launches), then the
// per-bin scaling maxima.
constexpr int kSchedCounters = 128;
constexpr int kCounterWords = kSchedCounters + MAXIMA_WORDS;

struct PlanInfo {
  int64_t n = 0, ncent = 0, tile = 0, ntiles = 0, ldc = 0;
  int nb = 0, nmax = 0, precision = 0, subtract = 1;
  int order = 4;               // 4: shear 4PCF; 3: shear 3PCF from records of order nmax
  int m3 = 0;                  // 3PCF: largest multipole (<= 2 nmax)
  size_t ups_bytes = 0, corr_bytes = 0, acc3_bytes = 0;
  Layout L{};
  size_t tsize = 8;            // bytes per real in records
  int64_t ncell_cap = 0;
  size_t sort_tmp = 0;
  // persistent buffers
  size_t o_gal, o_cells, o_centres, o_e2, o_edges, o_counters, o_bbox, o_bad,
      o_pairs, o_part, o_ups, o_corr, o_cpart, o_acc3, o_part3, o_xg, o_xw, o_counts,
      o_aos, o_region, o_pitems, o_pout, o_ppart, o_csums, o_cmap;
  // contraction work items (each distinct product of three blocks once)
  int pslices = 0;
  int64_t pitems = 0, prows = 0;
  // distinct degenerate-term sums
  int csums = 0, cpair = 0, cmap = 0;
  // tree approximation
  int tree_levels = 0;                      // grids in use (highest level of any bin)
  double tree_delta1 = 0.0;
  int8_t level[FPCF4_NBINS_SUPPORTED] = {};  // per bin: 0 = galaxies, d = grid d
  size_t o_rgal[TREE_LEVELS_MAX] = {}, o_rcell[TREE_LEVELS_MAX] = {}, t_red = 0;
  size_t region = 0;           // records of one tile, or create-time temporaries
  // create-time temporaries inside the region
  size_t t_raw, t_key_a, t_key_b, t_idx_a, t_idx_b, t_inv, t_sort, t_cent64;
  size_t total = 0;
};

fpcf4_status validate_common(const fpcf4_catalogue* cat, const fpcf4_bins* bins,
                             const fpcf4_options* opts) {
  if (!cat || !bins || !opts) return fail(FPCF4_E_INVALID_ARG, "null argument");
  if (cat->n < 0) return fail(FPCF4_E_INVALID_ARG, "catalogue size %lld < 0", (long long)cat->n);
  if (cat->n >= (int64_t(1) << 31) - 1) return fail(FPCF4_E_UNSUPPORTED, "catalogue larger than 2^31-2");
  if (cat->mem != FPCF4_MEM_HOST && cat->mem != FPCF4_MEM_DEVICE)
    return fail(FPCF4_E_INVALID_ARG, "catalogue mem flag %d", cat->mem);
  if (bins->nbins < 1) return fail(FPCF4_E_INVALID_ARG, "nbins must be >= 1");
  if (bins->nbins > FPCF4_NBINS_SUPPORTED)
    return fail(FPCF4_E_UNSUPPORTED, "nbins %d > %d", bins->nbins, FPCF4_NBINS_SUPPORTED);
  if (!bins->edges) return fail(FPCF4_E_INVALID_ARG, "null edges");
  for (int b = 0; b <= bins->nbins; ++b)
    if (!std::isfinite(bins->edges[b])) return fail(FPCF4_E_INVALID_ARG, "non-finite edge %d", b);
  if (!(bins->edges[0] > 0.0)) return fail(FPCF4_E_INVALID_ARG, "edges[0] must be > 0");
  for (int b = 0; b < bins->nbins; ++b)
    if (!(bins->edges[b + 1] > bins->edges[b]))
      return fail(FPCF4_E_INVALID_ARG, "edges not strictly increasing at %d", b);
  if (opts->nmax < 0) return fail(FPCF4_E_INVALID_ARG, "nmax < 0");
  if (opts->nmax > FPCF4_NMAX_SUPPORTED)
    return fail(FPCF4_E_UNSUPPORTED, "nmax %d > %d", opts->nmax, FPCF4_NMAX_SUPPORTED);
  if (opts->precision < FPCF4_FP64 || opts->precision > FPCF4_MIXED_BF16)
    return fail(FPCF4_E_INVALID_ARG, "precision %d", opts->precision);
  if (opts->centers && opts->ncenters < 0) return fail(FPCF4_E_INVALID_ARG, "ncenters < 0");
  if (opts->tile_centers < 0) return fail(FPCF4_E_INVALID_ARG, "tile_centers < 0");
  if (cat->n > 0 && (!cat->x || !cat->y || !cat->g1 || !cat->g2 || !cat->w))
    return fail(FPCF4_E_INVALID_ARG, "null catalogue array");
  return FPCF4_OK;
}

fpcf4_status make_plan(const fpcf4_catalogue* cat, const fpcf4_bins* bins,
                       const fpcf4_options* opts, PlanInfo& P, int order = 4, int m3 = 0,
                       const fpcf4_tree* tree = nullptr) {
  fpcf4_status st = validate_common(cat, bins, opts);
  if (st != FPCF4_OK) return st;
  if (tree) {
    if (tree->nlevels < 1 || tree->nlevels > TREE_LEVELS_MAX)
      return fail(FPCF4_E_INVALID_ARG, "tree levels %d not in 1..%d", tree->nlevels, TREE_LEVELS_MAX);
    if (!(tree->delta1 > 0.0) || !std::isfinite(tree->delta1))
      return fail(FPCF4_E_INVALID_ARG, "tree delta1 must be > 0");
    if (!(tree->rmin >= 2.0) || !std::isfinite(tree->rmin))
      return fail(FPCF4_E_INVALID_ARG, "tree rmin must be >= 2");
    if (opts->precision == FPCF4_FP64)
      return fail(FPCF4_E_UNSUPPORTED, "the tree approximation runs in the mixed paths only");
    // per bin the coarsest grid with edges[b] / Delta_d >= rmin
    P.tree_delta1 = tree->delta1;
    for (int b = 0; b < bins->nbins; ++b) {
      int best = 0;
      for (int d = 1; d <= tree->nlevels; ++d)
        if (bins->edges[b] / (tree->delta1 * std::ldexp(1.0, d - 1)) >= tree->rmin) best = d;
      P.level[b] = (int8_t)best;
      P.tree_levels = std::max(P.tree_levels, best);
    }
  }
  P.order = order;
  P.m3 = m3;
  P.n = cat->n;
  P.nb = bins->nbins;
  P.nmax = opts->nmax;
  P.precision = opts->precision;
  P.subtract = opts->subtract_degenerate ? 1 : 0;
  P.ncent = opts->centers ? opts->ncenters : cat->n;
  P.L = make_layout(P.nmax);
  P.tsize = (P.precision == FPCF4_FP64) ? 8 : 4;
  const size_t rec_per_centre = (size_t)P.nb * P.L.mpc * 2 * P.tsize;
  int64_t tile = opts->tile_centers;
  if (tile <= 0) tile = (int64_t)(kTileRecordBudget / rec_per_centre);
  if (tile > P.ncent) tile = P.ncent;
  if (tile < 1) tile = 1;
  if (tile > (int64_t(1) << 28)) tile = int64_t(1) << 28;   // <= 8 work-items per centre along x of the relayout grid
  P.tile = tile;
  P.ldc = (tile + 15) / 16 * 16;
  P.ntiles = P.ncent > 0 ? (P.ncent + tile - 1) / tile : 0;
  const int64_t n = P.n > 0 ? P.n : 1;
  P.ncell_cap = std::max<int64_t>(int64_t(1) << 16, 4 * n);
  P.sort_tmp = cells_sort_temp_bytes(n);
  const int nn = 2 * P.nmax + 1;

  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += up(bytes); return o; };
  P.o_gal = take(n * (P.precision == FPCF4_FP64 ? sizeof(Gal<double>) : sizeof(Gal<float>)));
  P.o_cells = take((P.ncell_cap + 1) * 4);
  P.o_centres = take((size_t)std::max<int64_t>(P.ncent, 1) * 4);
  P.o_e2 = take((P.nb + 1) * 8);
  P.o_edges = take((P.nb + 1) * 8);
  P.o_counters = take(kCounterWords * 4);   // scheduling counters, then the scaling maxima
  P.o_bbox = take(4 * 8);
  P.o_bad = take(16);
  P.o_pairs = take(16);
  P.o_part = take(256 * 4 * 8);
  P.ups_bytes = order == 4 ? (size_t)9 * P.nb * P.nb * P.nb * nn * nn * 16 : 0;
  P.corr_bytes = order == 4 ? corr_elems(P.nb, P.nmax) * 16 : 0;
  P.acc3_bytes = order == 3 ? three_elems(P.nb, m3) * 16 : 0;
  P.o_ups = take(P.ups_bytes);
  const bool pairs = order == 4;
  if (pairs) {
    const PairPlanHost pp = make_pair_plan(P.nmax, P.nb);
    for (const PairOut& o : pp.out)
      if (o.item < 0 || o.item >= (int32_t)pp.items.size())
        return fail(FPCF4_E_DEVICE, "internal: contraction plan leaves an output unassigned");
    P.pitems = (int64_t)pp.items.size();
    P.prows = pp.total_rows;
    const size_t slice_bytes = (size_t)P.prows * P.nb * P.nb * 8;
    const int64_t fit = std::max<int64_t>(1, (int64_t)(kPairPartialBudget / std::max<size_t>(slice_bytes, 1)));
    P.pslices = (int)std::min<int64_t>(pair_slices(P.tile), fit);
  }
  P.o_pitems = take((size_t)P.pitems * sizeof(PairItem));
  P.o_pout = take(pairs ? (size_t)FPCF4_NCORR * nn * nn * sizeof(PairOut) : 0);
  P.o_ppart = take((size_t)P.pslices * P.prows * P.nb * P.nb * 8);
  P.o_corr = take(P.corr_bytes);
  P.o_cpart = take(P.corr_bytes * CORR_SLICES);
  if (pairs) {
    const CorrPlanHost cp = make_corr_plan(P.nmax);
    P.csums = (int)cp.sums.size();
    P.cpair = cp.npair;
    P.cmap = (int)cp.map.size();
  }
  P.o_csums = take((size_t)P.csums * sizeof(CorrSum));
  P.o_cmap = take((size_t)P.cmap * 4);
  P.o_acc3 = take(P.acc3_bytes);
  P.o_part3 = take(P.acc3_bytes * THREE_SLICES);
  for (int d = 1; d <= P.tree_levels; ++d) {
    P.o_rgal[d - 1] = take(n * sizeof(GalR<float>));
    P.o_rcell[d - 1] = take((P.ncell_cap + 1) * 4);
  }
  P.o_xg = take((size_t)P.ldc * 2 * P.tsize);
  P.o_xw = take((size_t)P.ldc * P.tsize);
  P.o_aos = take((size_t)P.tile * rec_per_centre);
  P.o_counts = take((size_t)P.tile * P.nb * 4);
  // region: one tile of records, or the create-time temporaries
  size_t t = 0;
  auto ttake = [&](size_t bytes) { size_t o = t; t += up(bytes); return o; };
  P.t_raw = ttake(n * 8 * 5);
  P.t_key_a = ttake(n * 4);
  P.t_key_b = ttake(n * 4);
  P.t_idx_a = ttake(n * 4);
  P.t_idx_b = ttake(n * 4);
  P.t_inv = ttake(n * 4);
  P.t_cent64 = ttake((size_t)std::max<int64_t>(P.ncent, 1) * 8);
  P.t_sort = ttake(P.sort_tmp);
  if (P.tree_levels > 0) P.t_red = ttake(reduced_scratch_bytes(n));
  P.region = std::max(t, up((size_t)P.ldc * rec_per_centre));
  P.o_region = take(P.region);
  P.total = off;
  return FPCF4_OK;
}

std::once_flag g_pool_once;
void setup_pool() {
  std::call_once(g_pool_once, [] {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) return;
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  });
}

std::mutex g_prof_mu;
bool g_prof_on = false;
fpcf4_profile g_prof{};

__global__ void zero_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Device address of the static scratch array of the allocation-free entry
// point, looked up once per device (the array's host-side name is only a
// stand-in for the symbol, never a device address).
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

}  // namespace

// Workspace of estimate_4pcf_multipoles_noalloc: one copy per device, held
// until the process ends.  Every call on a device shares it.
static __device__ __align__(256) unsigned char scratch[FPCF4_NOALLOC_SCRATCH_BYTES];

struct fpcf4_request {
  PlanInfo P;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Grid grid{};
  std::vector<char> stepped;
  PairPlanHost pplan;           // the contraction plan uploaded into the workspace (4PCF)
  CorrPlanHost cplan;           // the distinct degenerate-term sums, likewise
  bool want_counts = false;
  bool no_events = false;       // allocation-free path: never create profiling events
  std::vector<hipEvent_t> ev;   // 4 per profiled step
  int64_t prof_a_launches = 0, prof_b_launches = 0, prof_steps = 0, prof_centres = 0;
  double prof_b_flops = 0.0, prof_b_useful = 0.0;
  ~fpcf4_request() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  template <typename U> U* at(size_t off) const { return reinterpret_cast<U*>(ws + off); }
};

namespace {

fpcf4_status request_init(const fpcf4_catalogue* cat, const fpcf4_bins* bins,
                          const fpcf4_options* opts, void* wsp, size_t bytes, fpcf4_request* R,
                          int order = 4, int m3 = 0, const fpcf4_tree* tree = nullptr) {
  PlanInfo& P = R->P;
  fpcf4_status st = make_plan(cat, bins, opts, P, order, m3, tree);
  if (st != FPCF4_OK) return st;
  if (!wsp) return fail(FPCF4_E_INVALID_ARG, "null workspace");
  if (reinterpret_cast<uintptr_t>(wsp) % ALIGN) return fail(FPCF4_E_INVALID_ARG, "workspace not 256-byte aligned");
  if (bytes < P.total) return fail(FPCF4_E_BUDGET, "workspace %zu bytes < planned %zu", bytes, P.total);
  R->ws = static_cast<char*>(wsp);
  R->stream = static_cast<hipStream_t>(opts->stream);
  R->stepped.assign((size_t)P.ntiles, 0);
  hipStream_t s = R->stream;
  const int64_t n = P.n;

  // centre subset: validate on the host
  std::vector<int64_t> hc;
  if (opts->centers && P.ncent > 0) {
    hc.resize((size_t)P.ncent);
    if (cat->mem == FPCF4_MEM_HOST) {
      std::memcpy(hc.data(), opts->centers, hc.size() * 8);
    } else {
      HIPCHK(hipMemcpyAsync(hc.data(), opts->centers, hc.size() * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    for (int64_t k = 0; k < P.ncent; ++k)
      if (hc[k] < 0 || hc[k] >= n) return fail(FPCF4_E_INVALID_ARG, "centre index %lld out of range", (long long)hc[k]);
  }

  if (P.pitems > 0) {
    R->pplan = make_pair_plan(P.nmax, P.nb);
    HIPCHK(hipMemcpyAsync(R->ws + P.o_pitems, R->pplan.items.data(), R->pplan.items.size() * sizeof(PairItem),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(R->ws + P.o_pout, R->pplan.out.data(), R->pplan.out.size() * sizeof(PairOut),
                          hipMemcpyHostToDevice, s));
  }
  if (P.csums > 0) {
    R->cplan = make_corr_plan(P.nmax);
    for (int32_t v : R->cplan.map)
      if (v < 0 || v >= P.csums) return fail(FPCF4_E_DEVICE, "internal: correction plan leaves a sum unassigned");
    HIPCHK(hipMemcpyAsync(R->ws + P.o_csums, R->cplan.sums.data(), R->cplan.sums.size() * sizeof(CorrSum),
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(R->ws + P.o_cmap, R->cplan.map.data(), R->cplan.map.size() * 4, hipMemcpyHostToDevice,
                          s));
  }
  HIPCHK(hipMemsetAsync(R->ws + P.o_pairs, 0, 16, s));
  if (P.ups_bytes) HIPCHK(hipMemsetAsync(R->ws + P.o_ups, 0, P.ups_bytes, s));
  if (P.corr_bytes) HIPCHK(hipMemsetAsync(R->ws + P.o_corr, 0, P.corr_bytes, s));
  if (P.acc3_bytes) HIPCHK(hipMemsetAsync(R->ws + P.o_acc3, 0, P.acc3_bytes, s));
  double e2[FPCF4_NBINS_SUPPORTED + 1];
  for (int b = 0; b <= P.nb; ++b) e2[b] = bins->edges[b] * bins->edges[b];
  HIPCHK(hipMemcpyAsync(R->ws + P.o_e2, e2, (P.nb + 1) * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(R->ws + P.o_edges, bins->edges, (P.nb + 1) * 8, hipMemcpyHostToDevice, s));
  // the copy from the stack array must complete before it goes out of scope
  HIPCHK(hipStreamSynchronize(s));
  if (n == 0) {
    HIPCHK(hipStreamSynchronize(s));
    return FPCF4_OK;
  }

  char* reg = R->ws + P.o_region;
  const double *x, *y, *g1, *g2, *w;
  if (cat->mem == FPCF4_MEM_HOST) {
    double* raw = reinterpret_cast<double*>(reg + P.t_raw);
    const double* src[5] = {cat->x, cat->y, cat->g1, cat->g2, cat->w};
    for (int k = 0; k < 5; ++k)
      HIPCHK(hipMemcpyAsync(raw + k * n, src[k], n * 8, hipMemcpyHostToDevice, s));
    x = raw; y = raw + n; g1 = raw + 2 * n; g2 = raw + 3 * n; w = raw + 4 * n;
  } else {
    x = cat->x; y = cat->y; g1 = cat->g1; g2 = cat->g2; w = cat->w;
  }
  unsigned* bad = R->at<unsigned>(P.o_bad);
  HIPCHK(hipMemsetAsync(bad, 0, 16, s));
  HIPCHK(cells_bbox(x, y, g1, g2, w, n, R->at<double>(P.o_part), bad, R->at<double>(P.o_bbox), s));
  double bb[4];
  unsigned hbad = 0;
  HIPCHK(hipMemcpyAsync(bb, R->ws + P.o_bbox, 32, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&hbad, bad, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hbad) return fail(FPCF4_E_INVALID_ARG, "catalogue has %u non-finite entries", hbad);

  // cell grid: side ~ outer edge / 48 (<= ~99 cell rows per annulus, two row
  // tables of 64), capped cell count.  Finer cells walk fewer candidates
  // outside the bin, for more and shorter row segments (10^6 galaxies on
  // 600x600 arcmin, 12 bins 1-100: 1.14 candidates per in-bin pair, 1.28 at
  // outer edge / 24).
  const double rmax = bins->edges[P.nb];
  double h = rmax / 48.0;
  const double wx = bb[1] - bb[0], wy = bb[3] - bb[2];
  for (;;) {
    const double ncx = std::floor(wx / h) + 1.0, ncy = std::floor(wy / h) + 1.0;
    if (ncx * ncy <= (double)P.ncell_cap) break;
    h *= 1.25;
  }
  Grid& g = R->grid;
  g.x0 = bb[0];
  g.y0 = bb[2];
  g.h = h;
  g.inv_h = 1.0 / h;
  g.ncx = (int)(std::floor(wx / h) + 1.0);
  g.ncy = (int)(std::floor(wy / h) + 1.0);

  uint32_t* key_a = reinterpret_cast<uint32_t*>(reg + P.t_key_a);
  uint32_t* key_b = reinterpret_cast<uint32_t*>(reg + P.t_key_b);
  int32_t* idx_a = reinterpret_cast<int32_t*>(reg + P.t_idx_a);
  int32_t* idx_b = reinterpret_cast<int32_t*>(reg + P.t_idx_b);
  int32_t* inv = reinterpret_cast<int32_t*>(reg + P.t_inv);
  void* sort_tmp = reg + P.t_sort;
  HIPCHK(cells_build(x, y, g1, g2, w, n, g, key_a, key_b, idx_a, idx_b, sort_tmp, P.sort_tmp,
                     R->ws + P.o_gal, P.precision == FPCF4_FP64 ? 1 : 0, R->at<int32_t>(P.o_cells),
                     inv, s));
  int32_t* centres = R->at<int32_t>(P.o_centres);
  if (opts->centers) {
    if (P.ncent > 0) {
      int64_t* c64 = reinterpret_cast<int64_t*>(reg + P.t_cent64);
      HIPCHK(hipMemcpyAsync(c64, hc.data(), hc.size() * 8, hipMemcpyHostToDevice, s));
      HIPCHK(cells_map_centres(c64, P.ncent, inv, centres, s));
    }
  } else {
    // key_a / idx_a are free again after the sort; reuse them for the Morton sort
    HIPCHK(cells_centre_order(key_b, n, g, key_a, reinterpret_cast<uint32_t*>(inv), idx_a, centres,
                              sort_tmp, P.sort_tmp, s));
  }
  // reduced catalogues of the tree approximation, on the same search grid
  for (int d = 1; d <= P.tree_levels; ++d) {
    int64_t m = 0;
    HIPCHK(reduced_build(x, y, g1, g2, w, n, bb[0], bb[2], bb[1], bb[3],
                         P.tree_delta1 * std::ldexp(1.0, d - 1), g, reg + P.t_red,
                         R->ws + P.o_rgal[d - 1], R->at<int32_t>(P.o_rcell[d - 1]), &m, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  return FPCF4_OK;
}

fpcf4_status request_step(fpcf4_request* R, int64_t tile, bool stage_b) {
  PlanInfo& P = R->P;
  if (tile < 0 || tile >= P.ntiles) return fail(FPCF4_E_INVALID_ARG, "tile %lld out of range", (long long)tile);
  if (R->stepped[(size_t)tile]) return fail(FPCF4_E_INVALID_ARG, "tile %lld already stepped", (long long)tile);
  hipStream_t s = R->stream;
  const int64_t c0 = tile * P.tile;
  const int ncent = (int)std::min<int64_t>(P.tile, P.ncent - c0);
  int32_t* counters = R->at<int32_t>(P.o_counters);
  bool prof;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof = g_prof_on && stage_b && !R->no_events;
  }
  hipEvent_t evs[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  if (prof) {
    for (auto& e : evs) HIPCHK(hipEventCreate(&e));
    for (auto e : evs) R->ev.push_back(e);
    HIPCHK(hipEventRecord(evs[0], s));
  }
  hipLaunchKernelGGL(zero_kernel, dim3((kCounterWords + 255) / 256), dim3(256), 0, s, counters,
                     kCounterWords);
  HIPCHK(hipGetLastError());
  StageAArgs a{};
  a.cat.n = P.n;
  a.cat.gal = R->ws + P.o_gal;
  a.cat.cell_start = R->at<int32_t>(P.o_cells);
  a.cat.g = R->grid;
  a.centres = R->at<int32_t>(P.o_centres) + c0;
  a.cgal = a.cat.gal;
  a.ncent = ncent;
  a.nb = P.nb;
  a.ldc = (int32_t)P.ldc;
  a.xg = R->ws + P.o_xg;
  a.xw = R->ws + P.o_xw;
  a.maxima = P.precision == FPCF4_FP64 ? nullptr : reinterpret_cast<unsigned*>(counters + kSchedCounters);
  a.e2 = R->at<double>(P.o_e2);
  a.edges = R->at<double>(P.o_edges);
  a.rec = R->ws + P.o_region;
  a.rec_aos = R->ws + P.o_aos;
  a.counts = R->want_counts ? R->at<int32_t>(P.o_counts) : nullptr;
  a.work_counter = counters;
  a.pairs = R->at<unsigned long long>(P.o_pairs);
  a.b_lo = 0;
  a.b_hi = P.nb;
  for (int b = 0; b < P.nb; ++b) a.level[b] = P.level[b];
  for (int d = 1; d <= P.tree_levels; ++d) {
    a.rgal[d - 1] = R->ws + P.o_rgal[d - 1];
    a.rcell[d - 1] = R->at<int32_t>(P.o_rcell[d - 1]);
  }
  int nlaunch = 0;
  if (P.precision == FPCF4_FP64) HIPCHK(launch_stage_a<double>(P.nmax, P.order, a, s, &nlaunch, evs[1]));
  else HIPCHK(launch_stage_a<float>(P.nmax, P.order, a, s, &nlaunch, evs[1]));
  if (prof) HIPCHK(hipEventRecord(evs[2], s));
  if (stage_b && P.order == 3) {
    ThreeArgs t3{a.rec, a.xg, a.xw, ncent, P.nb, P.nmax, P.m3, 2 * P.m3 + 1, (int32_t)P.ldc,
                 R->at<double>(P.o_part3), R->at<double>(P.o_acc3),
                 a.rec, (int32_t)P.ldc, nullptr, nullptr, 0, P.nb, 0, P.nb};
    if (P.precision == FPCF4_FP64) HIPCHK(launch_three<double>(t3, s));
    else HIPCHK(launch_three<float>(t3, s));
    if (prof) {
      HIPCHK(hipEventRecord(evs[3], s));
      HIPCHK(hipEventRecord(evs[4], s));
      R->prof_a_launches += nlaunch;
      R->prof_b_launches += 3;
      R->prof_steps += 1;
      R->prof_centres += ncent;
    }
  } else if (stage_b) {
    PairLaunch pl{};
    pl.rec = a.rec;
    pl.ldc = P.ldc;
    pl.xg = a.xg;
    pl.xw = a.xw;
    pl.maxima = a.maxima;
    pl.items = R->at<PairItem>(P.o_pitems);
    pl.out = R->at<PairOut>(P.o_pout);
    for (int c = 0; c <= PAIR_MAX_BLK; ++c) {
      pl.cls_start[c] = R->pplan.cls_start[c];
      pl.cls_count[c] = R->pplan.cls_count[c];
    }
    pl.ncent = ncent;
    pl.nb = P.nb;
    pl.nmax = P.nmax;
    pl.precision = P.precision;
    pl.max_slices = P.pslices;
    pl.part = R->at<double>(P.o_ppart);
    pl.total_rows = P.prows;
    pl.ups = R->at<double>(P.o_ups);
    HIPCHK(launch_contract_pairs(pl, s));
    if (prof) HIPCHK(hipEventRecord(evs[3], s));
    CorrArgs ca{a.rec, a.xg, a.xw, ncent, P.nb, P.nmax, (int32_t)P.ldc, R->at<double>(P.o_corr),
                R->at<double>(P.o_cpart), R->at<CorrSum>(P.o_csums), R->at<int32_t>(P.o_cmap), P.csums,
                P.cpair};
    if (P.precision == FPCF4_FP64) HIPCHK(launch_corrections<double>(ca, s));
    else HIPCHK(launch_corrections<float>(ca, s));
    if (prof) {
      HIPCHK(hipEventRecord(evs[4], s));
      R->prof_b_flops += pair_issued_flops(R->pplan, P.nb, ncent, P.precision);
      R->prof_b_useful += pair_useful_flops(R->pplan, P.nb, ncent);
      R->prof_a_launches += nlaunch;
      // one kernel per row-block class, the slice sum (several slices), the scatter
      R->prof_b_launches += (R->pplan.cls_count[1] > 0) + (R->pplan.cls_count[2] > 0) +
                            (std::min(pair_slices(ncent), P.pslices) > 1) + 1;
      R->prof_steps += 1;
      R->prof_centres += ncent;
    }
  }
  R->stepped[(size_t)tile] = 1;
  return FPCF4_OK;
}

// ---------------------------------------------------------------------------
// BaseTree / DoubleTree shear 3PCF (the appendix on Nth-order statistics,
// algorithmic implementation): base points on reduced catalogues, one grid
// per radial bin; x times the finer-bin block is carried to the coarser
// grid through the parent map of nested cells.
// ---------------------------------------------------------------------------
__global__ void base_centres_kernel(const GalR<float>* r, int64_t m, Gal<float>* g, int32_t* idx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const GalR<float> q = r[i];
    g[i] = Gal<float>{q.x, q.y, q.a, q.b, q.w, 0.0f};
    idx[i] = (int32_t)i;
  }
}
// parent of every discrete base point (record column c, sorted position
// centres[c]) on a coarser grid
__global__ void parent_galaxy_kernel(const int32_t* centres, const int32_t* sorted_to_orig,
                                     const int32_t* member, int64_t n, int32_t* par) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * blockDim.x)
    par[c] = member[sorted_to_orig[centres[c]]];
}
// parent of every pseudo-galaxy of a finer grid: each of its galaxies names
// the same coarse cell (nested grids), so the writes agree
__global__ void parent_cell_kernel(const int32_t* member_f, const int32_t* member_c, int64_t n,
                                   int32_t* par) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n;
       g += (int64_t)gridDim.x * blockDim.x)
    par[member_f[g]] = member_c[g];
}
__global__ void zero_f64_kernel(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1 << 16)); }

fpcf4_status check_tree(const fpcf4_tree* t, const char* what) {
  if (t->nlevels < 1 || t->nlevels > TREE_LEVELS_MAX)
    return fail(FPCF4_E_INVALID_ARG, "%s levels %d not in 1..%d", what, t->nlevels, TREE_LEVELS_MAX);
  if (!(t->delta1 > 0.0) || !std::isfinite(t->delta1)) return fail(FPCF4_E_INVALID_ARG, "%s delta1 must be > 0", what);
  if (!(t->rmin >= 2.0) || !std::isfinite(t->rmin)) return fail(FPCF4_E_INVALID_ARG, "%s rmin must be >= 2", what);
  return FPCF4_OK;
}

// Device buffers of the driver, freed in reverse order on the stream.
struct StreamBuffers {
  hipStream_t s;
  std::vector<void*> p;
  explicit StreamBuffers(hipStream_t st) : s(st) {}
  hipError_t get(void** out, size_t bytes) {
    *out = nullptr;
    hipError_t e = hipMallocAsync(out, std::max<size_t>(bytes, 256), s);
    if (e == hipSuccess) p.push_back(*out);
    return e;
  }
  ~StreamBuffers() {
    for (auto it = p.rbegin(); it != p.rend(); ++it) (void)hipFreeAsync(*it, s);
  }
};

fpcf4_status run_3pcf_basetree(fpcf4_request* R, const fpcf4_catalogue* cat, const fpcf4_bins* bins,
                               const fpcf4_tree* base) {
  PlanInfo& P = R->P;
  hipStream_t s = R->stream;
  const int64_t n = P.n;
  const int nb = P.nb;
  // base grid of every bin (coarsest d with edges[b] / Delta_d >= rmin), a
  // non-decreasing function of b: the bins of one grid are a range
  int lvl[FPCF4_NBINS_SUPPORTED];
  for (int b = 0; b < nb; ++b) {
    int best = 0;
    for (int d = 1; d <= base->nlevels; ++d)
      if (bins->edges[b] / (base->delta1 * std::ldexp(1.0, d - 1)) >= base->rmin) best = d;
    lvl[b] = best;
  }
  int lo[TREE_LEVELS_MAX + 1], hi[TREE_LEVELS_MAX + 1];
  for (int d = 0; d <= TREE_LEVELS_MAX; ++d) lo[d] = hi[d] = -1;
  for (int b = 0; b < nb; ++b) {
    if (lo[lvl[b]] < 0) lo[lvl[b]] = b;
    hi[lvl[b]] = b + 1;
  }
  std::vector<int> D;
  for (int d = 0; d <= TREE_LEVELS_MAX; ++d)
    if (lo[d] >= 0) D.push_back(d);

  StreamBuffers buf(s);
  const Layout L = make_layout(P.nmax);
  const size_t rec_per_centre = (size_t)nb * L.mpc * 2 * sizeof(float);
  // per grid: base points, records, centre factors; member maps of the galaxies
  struct Grid_ {
    int64_t m = 0, ldc = 0;
    const void* cgal = nullptr;
    const int32_t* centres = nullptr;
    void* rec = nullptr;
    void* xg = nullptr;
    void* xw = nullptr;
    int32_t* member = nullptr;
  } G[TREE_LEVELS_MAX + 1];
  // the discrete grid: the request's own sorted catalogue and buffers
  G[0].m = P.ncent;
  G[0].ldc = P.ldc;
  G[0].cgal = R->ws + P.o_gal;
  G[0].centres = R->at<int32_t>(P.o_centres);
  G[0].rec = R->ws + P.o_region;
  G[0].xg = R->ws + P.o_xg;
  G[0].xw = R->ws + P.o_xw;
  // raw catalogue (a host catalogue's device copy sits in the region, which
  // the discrete grid's records overwrite only after the reduced builds)
  const double *x, *y, *g1, *g2, *w;
  if (cat->mem == FPCF4_MEM_HOST) {
    const double* raw = reinterpret_cast<const double*>(R->ws + P.o_region + P.t_raw);
    x = raw; y = raw + n; g1 = raw + 2 * n; g2 = raw + 3 * n; w = raw + 4 * n;
  } else {
    x = cat->x; y = cat->y; g1 = cat->g1; g2 = cat->g2; w = cat->w;
  }
  double bb[4];
  HIPCHK(hipMemcpyAsync(bb, R->ws + P.o_bbox, 32, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  void* scratch = nullptr;
  const bool any_red = D.back() > 0;
  if (any_red) HIPCHK(buf.get(&scratch, reduced_scratch_bytes(n)));
  for (int d : D) {
    if (d == 0) continue;
    void *galr, *cs, *mem, *cg, *ci;
    HIPCHK(buf.get(&galr, (size_t)n * sizeof(GalR<float>)));
    HIPCHK(buf.get(&cs, ((size_t)R->grid.ncx * R->grid.ncy + 1) * 4));
    HIPCHK(buf.get(&mem, (size_t)n * 4));
    int64_t m = 0;
    HIPCHK(reduced_build(x, y, g1, g2, w, n, bb[0], bb[2], bb[1], bb[3], base->delta1 * std::ldexp(1.0, d - 1),
                         R->grid, scratch, galr, reinterpret_cast<int32_t*>(cs), &m, s,
                         reinterpret_cast<int32_t*>(mem)));
    HIPCHK(buf.get(&cg, (size_t)std::max<int64_t>(m, 1) * sizeof(Gal<float>)));
    HIPCHK(buf.get(&ci, (size_t)std::max<int64_t>(m, 1) * 4));
    hipLaunchKernelGGL(base_centres_kernel, dim3(blocks_for(m)), dim3(256), 0, s,
                       reinterpret_cast<const GalR<float>*>(galr), m, reinterpret_cast<Gal<float>*>(cg),
                       reinterpret_cast<int32_t*>(ci));
    HIPCHK(hipGetLastError());
    G[d].m = m;
    G[d].ldc = (m + 15) / 16 * 16;
    G[d].cgal = cg;
    G[d].centres = reinterpret_cast<const int32_t*>(ci);
    G[d].member = reinterpret_cast<int32_t*>(mem);
    HIPCHK(buf.get(&G[d].rec, (size_t)G[d].ldc * rec_per_centre));
    HIPCHK(buf.get(&G[d].xg, (size_t)G[d].ldc * 2 * sizeof(float)));
    HIPCHK(buf.get(&G[d].xw, (size_t)G[d].ldc * sizeof(float)));
  }
  // parent maps from every grid to every coarser one (before the discrete
  // records overwrite the sort's index arrays in the region)
  int32_t* par[TREE_LEVELS_MAX + 1][TREE_LEVELS_MAX + 1] = {};
  const int32_t* sorted_to_orig = reinterpret_cast<const int32_t*>(R->ws + P.o_region + P.t_idx_b);
  for (int f : D)
    for (int c : D) {
      if (c <= f) continue;
      void* pp;
      HIPCHK(buf.get(&pp, (size_t)std::max<int64_t>(G[f].m, 1) * 4));
      par[f][c] = reinterpret_cast<int32_t*>(pp);
      if (f == 0)
        hipLaunchKernelGGL(parent_galaxy_kernel, dim3(blocks_for(G[0].m)), dim3(256), 0, s, G[0].centres,
                           sorted_to_orig, G[c].member, G[0].m, par[f][c]);
      else
        hipLaunchKernelGGL(parent_cell_kernel, dim3(blocks_for(n)), dim3(256), 0, s, G[f].member,
                           G[c].member, n, par[f][c]);
      HIPCHK(hipGetLastError());
    }
  // stage (a): the blocks of every bin at the base points of its grid
  int32_t* counters = R->at<int32_t>(P.o_counters);
  for (int d : D) {
    hipLaunchKernelGGL(zero_kernel, dim3((kCounterWords + 255) / 256), dim3(256), 0, s, counters, kCounterWords);
    HIPCHK(hipGetLastError());
    StageAArgs a{};
    a.cat.n = P.n;
    a.cat.gal = R->ws + P.o_gal;
    a.cat.cell_start = R->at<int32_t>(P.o_cells);
    a.cat.g = R->grid;
    a.centres = G[d].centres;
    a.cgal = G[d].cgal;
    a.ncent = (int32_t)G[d].m;
    a.nb = nb;
    a.ldc = (int32_t)G[d].ldc;
    a.xg = G[d].xg;
    a.xw = G[d].xw;
    a.maxima = nullptr;
    a.e2 = R->at<double>(P.o_e2);
    a.edges = R->at<double>(P.o_edges);
    a.rec = G[d].rec;
    a.rec_aos = R->ws + P.o_aos;
    a.counts = nullptr;
    a.work_counter = counters;
    a.pairs = R->at<unsigned long long>(P.o_pairs);
    a.b_lo = lo[d];
    a.b_hi = hi[d];
    for (int b = 0; b < nb; ++b) a.level[b] = P.level[b];
    for (int t = 1; t <= P.tree_levels; ++t) {
      a.rgal[t - 1] = R->ws + P.o_rgal[t - 1];
      a.rcell[t - 1] = R->at<int32_t>(P.o_rcell[t - 1]);
    }
    int nl = 0;
    if (G[d].m > 0) HIPCHK(launch_stage_a<float>(P.nmax, 3, a, s, &nl, nullptr));
  }
  // contraction for every pair of grids: over the base points of the finer
  // one, the coarser slot read at the parent; each pair writes only its own
  // bins of the zeroed slice partials, which are then added to the sums
  double* part = R->at<double>(P.o_part3);
  const int64_t part_elems = (int64_t)THREE_SLICES * 2 * (int64_t)three_elems(nb, P.m3);
  for (int d1 : D)
    for (int d2 : D) {
      const int f = std::min(d1, d2);
      if (G[f].m == 0) continue;
      hipLaunchKernelGGL(zero_f64_kernel, dim3(blocks_for(part_elems)), dim3(256), 0, s, part, part_elems);
      HIPCHK(hipGetLastError());
      ThreeArgs t{G[d1].rec, G[f].xg, G[f].xw, (int32_t)G[f].m, nb, P.nmax, P.m3, 2 * P.m3 + 1,
                  (int32_t)G[d1].ldc, part, R->at<double>(P.o_acc3),
                  G[d2].rec, (int32_t)G[d2].ldc, d1 > f ? par[f][d1] : nullptr, d2 > f ? par[f][d2] : nullptr,
                  lo[d1], hi[d1] - lo[d1], lo[d2], hi[d2] - lo[d2]};
      HIPCHK(launch_three<float>(t, s));
    }
  HIPCHK(hipStreamSynchronize(s));
  R->stepped.assign(R->stepped.size(), 1);
  return FPCF4_OK;
}

}  // namespace

extern "C" {

int64_t fpcf4_output_elems(int32_t nbins, int32_t nmax) {
  if (nbins < 0 || nmax < 0) return 0;
  const int64_t nn = 2 * (int64_t)nmax + 1;
  return 9 * (int64_t)nbins * nbins * nbins * nn * nn;
}

int64_t fpcf4_output3_elems(int32_t nbins, int32_t nmax) {
  if (nbins < 0 || nmax < 0) return 0;
  return 5 * (int64_t)nbins * nbins * (2 * (int64_t)nmax + 1);
}

const char* fpcf4_last_error(void) { return g_err.c_str(); }
const char* fpcf4_version(void) { return "fpcf4 0.1 (gfx950)"; }

fpcf4_status fpcf4_plan(const fpcf4_catalogue* cat, const fpcf4_bins* bins, const fpcf4_options* opts,
                        size_t* device_bytes, int64_t* ntiles) {
  PlanInfo P;
  fpcf4_status st = make_plan(cat, bins, opts, P);
  if (st != FPCF4_OK) return st;
  if (device_bytes) *device_bytes = P.total;
  if (ntiles) *ntiles = P.ntiles;
  return FPCF4_OK;
}

fpcf4_status fpcf4_request_create(const fpcf4_catalogue* cat, const fpcf4_bins* bins,
                                  const fpcf4_options* opts, void* ws, size_t bytes,
                                  fpcf4_request** req) {
  if (!req) return fail(FPCF4_E_INVALID_ARG, "null request pointer");
  *req = nullptr;
  fpcf4_request* R = new (std::nothrow) fpcf4_request();
  if (!R) return fail(FPCF4_E_OUT_OF_MEMORY, "host allocation failed");
  fpcf4_status st = request_init(cat, bins, opts, ws, bytes, R);
  if (st != FPCF4_OK) {
    delete R;
    return st;
  }
  *req = R;
  return FPCF4_OK;
}

fpcf4_status fpcf4_request_step(fpcf4_request* req, int64_t tile) {
  if (!req) return fail(FPCF4_E_INVALID_ARG, "null request");
  return request_step(req, tile, true);
}

fpcf4_status fpcf4_request_finalize(fpcf4_request* req, double* upsilon, int32_t out_mem) {
  if (!req || !upsilon) return fail(FPCF4_E_INVALID_ARG, "null argument");
  if (out_mem != FPCF4_MEM_HOST && out_mem != FPCF4_MEM_DEVICE) return fail(FPCF4_E_INVALID_ARG, "out_mem %d", out_mem);
  PlanInfo& P = req->P;
  for (size_t t = 0; t < req->stepped.size(); ++t)
    if (!req->stepped[t]) return fail(FPCF4_E_INVALID_ARG, "tile %zu not stepped", t);
  hipStream_t s = req->stream;
  if (P.order == 3) {
    // the slice partials are free once every tile is reduced: stage the host copy there
    const size_t bytes = (size_t)fpcf4_output3_elems(P.nb, P.m3) * 16;
    double* dst = out_mem == FPCF4_MEM_DEVICE ? upsilon : req->at<double>(P.o_part3);
    HIPCHK(launch_finalize3(req->at<double>(P.o_acc3), P.nb, P.m3, P.subtract, dst, s));
    if (out_mem == FPCF4_MEM_HOST) HIPCHK(hipMemcpyAsync(upsilon, dst, bytes, hipMemcpyDeviceToHost, s));
  } else {
    double* ups = req->at<double>(P.o_ups);
    HIPCHK(launch_finalize(ups, req->at<double>(P.o_corr), P.nb, P.nmax, P.subtract, ups, s));
    const size_t bytes = (size_t)fpcf4_output_elems(P.nb, P.nmax) * 16;
    HIPCHK(hipMemcpyAsync(upsilon, ups, bytes,
                          out_mem == FPCF4_MEM_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  if (!req->ev.empty()) {
    unsigned long long pairs = 0;
    HIPCHK(hipMemcpy(&pairs, req->ws + P.o_pairs, 8, hipMemcpyDeviceToHost));
    double ta = 0, tr = 0, tb = 0, tc = 0;
    for (size_t k = 0; k + 4 < req->ev.size(); k += 5) {
      float x = 0;
      HIPCHK(hipEventElapsedTime(&x, req->ev[k], req->ev[k + 1]));
      ta += x;
      HIPCHK(hipEventElapsedTime(&x, req->ev[k + 1], req->ev[k + 2]));
      tr += x;
      HIPCHK(hipEventElapsedTime(&x, req->ev[k + 2], req->ev[k + 3]));
      tb += x;
      HIPCHK(hipEventElapsedTime(&x, req->ev[k + 3], req->ev[k + 4]));
      tc += x;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof.stage_a_ms += ta;
    g_prof.relayout_ms += tr;
    g_prof.stage_b_ms += tb;
    g_prof.corr_ms += tc;
    g_prof.stage_a_launches += req->prof_a_launches;
    g_prof.stage_b_launches += req->prof_b_launches;
    g_prof.steps += req->prof_steps;
    g_prof.pairs += (int64_t)pairs;
    g_prof.centres += req->prof_centres;
    g_prof.stage_b_mfma_flops += req->prof_b_flops;
    g_prof.stage_b_useful_flops += req->prof_b_useful;
  }
  return FPCF4_OK;
}

void fpcf4_request_destroy(fpcf4_request* req) { delete req; }

fpcf4_status fpcf4_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = on != 0;
  g_prof = fpcf4_profile{};
  return FPCF4_OK;
}

fpcf4_status fpcf4_profile_read(fpcf4_profile* out) {
  if (!out) return fail(FPCF4_E_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  *out = g_prof;
  return FPCF4_OK;
}

fpcf4_status estimate_4pcf_multipoles(const fpcf4_catalogue* cat, const fpcf4_bins* bins,
                                      const fpcf4_options* opts, double* upsilon, int32_t out_mem) {
  if (!upsilon) return fail(FPCF4_E_INVALID_ARG, "null output");
  PlanInfo P;
  fpcf4_status st = make_plan(cat, bins, opts, P);
  if (st != FPCF4_OK) return st;
  setup_pool();
  hipStream_t s = static_cast<hipStream_t>(opts->stream);
  void* ws = nullptr;
  HIPCHK(hipMallocAsync(&ws, P.total, s));
  fpcf4_request* R = nullptr;
  st = fpcf4_request_create(cat, bins, opts, ws, P.total, &R);
  for (int64_t t = 0; st == FPCF4_OK && t < P.ntiles; ++t) st = fpcf4_request_step(R, t);
  if (st == FPCF4_OK) st = fpcf4_request_finalize(R, upsilon, out_mem);
  fpcf4_request_destroy(R);
  hipError_t e = hipFreeAsync(ws, s);
  if (st == FPCF4_OK && e != hipSuccess) return fail(FPCF4_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
  return st;
}

fpcf4_status estimate_4pcf_multipoles_noalloc(const fpcf4_catalogue* cat, const fpcf4_bins* bins,
                                              const fpcf4_options* opts, double* upsilon, int32_t out_mem) {
  if (!upsilon) return fail(FPCF4_E_INVALID_ARG, "null output");
  if (out_mem != FPCF4_MEM_HOST && out_mem != FPCF4_MEM_DEVICE) return fail(FPCF4_E_INVALID_ARG, "out_mem %d", out_mem);
  PlanInfo P;
  fpcf4_status st = make_plan(cat, bins, opts, P);
  if (st != FPCF4_OK) return st;
  fpcf4_options o = *opts;
  if (P.total > FPCF4_NOALLOC_SCRATCH_BYTES && opts->tile_centers == 0) {
    // smaller centre tiles shrink the per-tile record buffers
    for (int64_t tile = P.tile / 2; tile >= 64 && P.total > FPCF4_NOALLOC_SCRATCH_BYTES; tile /= 2) {
      o.tile_centers = tile;
      if ((st = make_plan(cat, bins, &o, P)) != FPCF4_OK) return st;
    }
  }
  if (P.total > FPCF4_NOALLOC_SCRATCH_BYTES)
    return fail(FPCF4_E_BUDGET, "workspace of %zu bytes exceeds the static scratch of %zu bytes", P.total,
                (size_t)FPCF4_NOALLOC_SCRATCH_BYTES);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(FPCF4_E_UNSUPPORTED, "device index %d", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);   // one call at a time in this process
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(FPCF4_E_DEVICE, "no device address for the static scratch");
    g_scratch_ptr[dev] = p;
  }
  fpcf4_request R;
  R.no_events = true;
  st = request_init(cat, bins, &o, g_scratch_ptr[dev], FPCF4_NOALLOC_SCRATCH_BYTES, &R);
  for (int64_t t = 0; st == FPCF4_OK && t < R.P.ntiles; ++t) st = request_step(&R, t, true);
  if (st == FPCF4_OK) st = fpcf4_request_finalize(&R, upsilon, out_mem);
  // leave the scratch idle for the next call even after an error
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(o.stream));
  if (st == FPCF4_OK && e != hipSuccess) return fail(FPCF4_E_DEVICE, "sync: %s", hipGetErrorString(e));
  return st;
}

fpcf4_status estimate_4pcf_multipoles_tree(const fpcf4_catalogue* cat, const fpcf4_bins* bins,
                                           const fpcf4_options* opts, const fpcf4_tree* tree,
                                           double* upsilon, int32_t out_mem) {
  if (!upsilon || !tree) return fail(FPCF4_E_INVALID_ARG, "null argument");
  if (out_mem != FPCF4_MEM_HOST && out_mem != FPCF4_MEM_DEVICE) return fail(FPCF4_E_INVALID_ARG, "out_mem %d", out_mem);
  PlanInfo P;
  fpcf4_status st = make_plan(cat, bins, opts, P, 4, 0, tree);
  if (st != FPCF4_OK) return st;
  setup_pool();
  hipStream_t s = static_cast<hipStream_t>(opts->stream);
  void* ws = nullptr;
  HIPCHK(hipMallocAsync(&ws, P.total, s));
  fpcf4_request* R = new (std::nothrow) fpcf4_request();
  if (!R) st = fail(FPCF4_E_OUT_OF_MEMORY, "host allocation failed");
  if (st == FPCF4_OK) st = request_init(cat, bins, opts, ws, P.total, R, 4, 0, tree);
  for (int64_t t = 0; st == FPCF4_OK && t < P.ntiles; ++t) st = request_step(R, t, true);
  if (st == FPCF4_OK) st = fpcf4_request_finalize(R, upsilon, out_mem);
  delete R;
  hipError_t e = hipFreeAsync(ws, s);
  if (st == FPCF4_OK && e != hipSuccess) return fail(FPCF4_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
  return st;
}

fpcf4_status estimate_3pcf_multipoles(const fpcf4_catalogue* cat, const fpcf4_bins* bins,
                                      const fpcf4_options* opts, double* upsilon3, int32_t out_mem) {
  if (!upsilon3 || !opts) return fail(FPCF4_E_INVALID_ARG, "null argument");
  if (out_mem != FPCF4_MEM_HOST && out_mem != FPCF4_MEM_DEVICE) return fail(FPCF4_E_INVALID_ARG, "out_mem %d", out_mem);
  if (opts->nmax < 0) return fail(FPCF4_E_INVALID_ARG, "nmax < 0");
  if (opts->nmax > FPCF4_NMAX3_SUPPORTED)
    return fail(FPCF4_E_UNSUPPORTED, "3PCF nmax %d > %d", opts->nmax, FPCF4_NMAX3_SUPPORTED);
  // stage (a) records of order ceil(m/2) hold every block the 3PCF reads
  const int m = opts->nmax;
  fpcf4_options o = *opts;
  o.nmax = (m + 1) / 2;
  PlanInfo P;
  fpcf4_status st = make_plan(cat, bins, &o, P, 3, m);
  if (st != FPCF4_OK) return st;
  setup_pool();
  hipStream_t s = static_cast<hipStream_t>(o.stream);
  void* ws = nullptr;
  HIPCHK(hipMallocAsync(&ws, P.total, s));
  fpcf4_request* R = new (std::nothrow) fpcf4_request();
  if (!R) st = fail(FPCF4_E_OUT_OF_MEMORY, "host allocation failed");
  if (st == FPCF4_OK) st = request_init(cat, bins, &o, ws, P.total, R, 3, m);
  for (int64_t t = 0; st == FPCF4_OK && t < P.ntiles; ++t) st = request_step(R, t, true);
  if (st == FPCF4_OK) st = fpcf4_request_finalize(R, upsilon3, out_mem);
  delete R;
  hipError_t e = hipFreeAsync(ws, s);
  if (st == FPCF4_OK && e != hipSuccess) return fail(FPCF4_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
  return st;
}

fpcf4_status estimate_3pcf_multipoles_doubletree(const fpcf4_catalogue* cat, const fpcf4_bins* bins,
                                                 const fpcf4_options* opts, const fpcf4_tree* base,
                                                 const fpcf4_tree* tree, double* upsilon3, int32_t out_mem) {
  if (!upsilon3 || !opts) return fail(FPCF4_E_INVALID_ARG, "null argument");
  if (out_mem != FPCF4_MEM_HOST && out_mem != FPCF4_MEM_DEVICE) return fail(FPCF4_E_INVALID_ARG, "out_mem %d", out_mem);
  if (opts->nmax < 0) return fail(FPCF4_E_INVALID_ARG, "nmax < 0");
  if (opts->nmax > FPCF4_NMAX3_SUPPORTED)
    return fail(FPCF4_E_UNSUPPORTED, "3PCF nmax %d > %d", opts->nmax, FPCF4_NMAX3_SUPPORTED);
  fpcf4_status st = FPCF4_OK;
  if (base && (st = check_tree(base, "base")) != FPCF4_OK) return st;
  if (tree && (st = check_tree(tree, "tree")) != FPCF4_OK) return st;
  if ((base || tree) && opts->precision == FPCF4_FP64)
    return fail(FPCF4_E_UNSUPPORTED, "the tree approximations run in the mixed paths only");
  if (base && opts->centers)
    return fail(FPCF4_E_INVALID_ARG, "BaseTree: every galaxy is a base point (no centre subset)");
  const int m = opts->nmax;
  fpcf4_options o = *opts;
  o.nmax = (m + 1) / 2;
  if (base) o.tile_centers = 0;
  PlanInfo P;
  st = make_plan(cat, bins, &o, P, 3, m, tree);
  if (st != FPCF4_OK) return st;
  if (base && P.ntiles > 1)
    return fail(FPCF4_E_UNSUPPORTED, "BaseTree: the records of all %lld galaxies must fit one tile",
                (long long)P.n);
  setup_pool();
  hipStream_t s = static_cast<hipStream_t>(o.stream);
  void* ws = nullptr;
  HIPCHK(hipMallocAsync(&ws, P.total, s));
  fpcf4_request* R = new (std::nothrow) fpcf4_request();
  if (!R) st = fail(FPCF4_E_OUT_OF_MEMORY, "host allocation failed");
  if (st == FPCF4_OK) st = request_init(cat, bins, &o, ws, P.total, R, 3, m, tree);
  if (base) {
    if (st == FPCF4_OK && P.n > 0) st = run_3pcf_basetree(R, cat, bins, base);
  } else {
    // neighbours on the tree's grids, base points the galaxies: the tiled path
    for (int64_t t = 0; st == FPCF4_OK && t < P.ntiles; ++t) st = request_step(R, t, true);
  }
  if (st == FPCF4_OK) st = fpcf4_request_finalize(R, upsilon3, out_mem);
  delete R;
  hipError_t e = hipFreeAsync(ws, s);
  if (st == FPCF4_OK && e != hipSuccess) return fail(FPCF4_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
  return st;
}

fpcf4_status fpcf4_debug_pair_plan(int32_t nmax, int32_t* out, int64_t* nitems) {
  if (nmax < 0 || nmax > FPCF4_NMAX_SUPPORTED) return fail(FPCF4_E_INVALID_ARG, "nmax %d outside [0, %d]", nmax,
                                                          FPCF4_NMAX_SUPPORTED);
  if (!out) return fail(FPCF4_E_INVALID_ARG, "null out");
  const PairPlanHost pp = make_pair_plan(nmax, 1);
  for (size_t o = 0; o < pp.out.size(); ++o) {
    const PairOut& po = pp.out[o];
    int32_t* v = out + 16 * o;
    if (po.item < 0 || po.item >= (int32_t)pp.items.size())
      return fail(FPCF4_E_DEVICE, "internal: contraction plan leaves an output unassigned");
    const PairItem& it = pp.items[po.item];
    const PairRow& r = it.blk[po.blk];
    const int32_t vals[16] = {r.x, r.fam, r.conj, r.order, it.famB, it.conjB, it.ordB, it.famC, it.conjC, it.ordC,
                              po.perm & 3, (po.perm >> 2) & 3, (po.perm >> 4) & 3, po.item, po.blk, it.nblk};
    for (int k = 0; k < 16; ++k) v[k] = vals[k];
  }
  if (nitems) *nitems = (int64_t)pp.items.size();
  return FPCF4_OK;
}

fpcf4_status fpcf4_debug_corr_plan(int32_t nmax, int32_t* out, int64_t* nsums) {
  if (nmax < 0 || nmax > FPCF4_NMAX_SUPPORTED) return fail(FPCF4_E_INVALID_ARG, "nmax %d outside [0, %d]", nmax,
                                                          FPCF4_NMAX_SUPPORTED);
  if (!out) return fail(FPCF4_E_INVALID_ARG, "null out");
  const CorrPlanHost cp = make_corr_plan(nmax);
  const Layout L = make_layout(nmax);
  // record entry -> (family code, signed order) of the block it holds
  auto block_of = [&](int e, int flip, int& fam, int& ord) {
    if (e >= L.offS) {   // triple blocks T_-8, T_-4, M_-4, M_0, U
      static const int tf[5] = {5, 5, 6, 6, 7}, to[5] = {-8, -4, -4, 0, 0};
      fam = tf[e - L.offS];
      ord = to[e - L.offS];
    } else if (e >= L.offV) {
      fam = 4;
      ord = flip ? -(e - L.offV) : e - L.offV;
    } else if (e >= L.offA) {
      fam = 3;
      ord = flip ? -(e - L.offA) : e - L.offA;
    } else if (e >= L.offQ) {
      fam = 2;
      ord = e - L.offQ + L.qlo;
    } else if (e >= L.offW) {
      fam = 1;   // W
      ord = e - L.offW - 2 * nmax;
    } else {
      fam = 0;   // G
      ord = e - L.offG - (2 * nmax + 3);
    }
  };
  for (size_t m = 0; m < cp.map.size(); ++m) {
    const int sidx = cp.map[m];
    if (sidx < 0 || sidx >= (int)cp.sums.size())
      return fail(FPCF4_E_DEVICE, "internal: correction plan leaves a sum unassigned");
    const CorrSum& c = cp.sums[sidx];
    int ef, eo, ff = -1, fo = 0;
    block_of(c.eidx, c.eflip, ef, eo);
    if (!c.triple) block_of(c.fidx, 0, ff, fo);
    const int32_t vals[8] = {c.x, ef, eo, ff, c.triple ? 0 : c.fconj, fo, sidx, 0};
    for (int k = 0; k < 8; ++k) out[8 * m + k] = vals[k];
  }
  if (nsums) *nsums = (int64_t)cp.sums.size();
  return FPCF4_OK;
}

fpcf4_status fpcf4_debug_sort_pairs(const uint64_t* keys, const int32_t* vals, int64_t n, int32_t key_bits,
                                    int32_t key_bytes, uint64_t* keys_out, int32_t* vals_out) {
  if (n < 0 || n >= (int64_t(1) << 31)) return fail(FPCF4_E_INVALID_ARG, "n %lld outside [0, 2^31)", (long long)n);
  if (key_bytes != 4 && key_bytes != 8) return fail(FPCF4_E_INVALID_ARG, "key_bytes %d is not 4 or 8", key_bytes);
  if (key_bits < 1 || key_bits > 8 * key_bytes)
    return fail(FPCF4_E_INVALID_ARG, "key_bits %d outside [1, %d]", key_bits, 8 * key_bytes);
  if (n == 0) return FPCF4_OK;
  if (!keys || !vals || !keys_out || !vals_out) return fail(FPCF4_E_INVALID_ARG, "null argument");
  for (int64_t i = 0; i < n; ++i)
    if (key_bits < 64 && (keys[i] >> key_bits) != 0)
      return fail(FPCF4_E_INVALID_ARG, "key %lld is not below 2^%d", (long long)i, key_bits);
  const size_t kb = (size_t)n * key_bytes, vb = (size_t)n * 4, tb = radix_sort_temp_bytes(n);
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  char* d = nullptr;
  HIPCHK(hipMalloc(&d, 2 * up(kb) + 2 * up(vb) + tb));
  std::vector<uint32_t> k32(key_bytes == 4 ? n : 0);
  for (size_t i = 0; i < k32.size(); ++i) k32[i] = (uint32_t)keys[i];
  char *ka = d, *kbuf = d + up(kb), *va = d + 2 * up(kb), *vbuf = va + up(vb), *tmp = vbuf + up(vb);
  hipError_t e = hipMemcpy(ka, key_bytes == 4 ? (const void*)k32.data() : (const void*)keys, kb, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(va, vals, vb, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = key_bytes == 4
            ? radix_sort_pairs(tmp, tb, reinterpret_cast<uint32_t*>(ka), reinterpret_cast<uint32_t*>(kbuf),
                               reinterpret_cast<int32_t*>(va), reinterpret_cast<int32_t*>(vbuf), n, key_bits, nullptr)
            : radix_sort_pairs(tmp, tb, reinterpret_cast<uint64_t*>(ka), reinterpret_cast<uint64_t*>(kbuf),
                               reinterpret_cast<int32_t*>(va), reinterpret_cast<int32_t*>(vbuf), n, key_bits, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(key_bytes == 4 ? (void*)k32.data() : (void*)keys_out, kbuf, kb, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(vals_out, vbuf, vb, hipMemcpyDeviceToHost);
  const hipError_t ef = hipFree(d);
  if (e == hipSuccess) e = ef;
  if (e != hipSuccess) return fail(FPCF4_E_DEVICE, "sort: %s", hipGetErrorString(e));
  for (size_t i = 0; i < k32.size(); ++i) keys_out[i] = k32[i];
  return FPCF4_OK;
}

fpcf4_status fpcf4_debug_multipoles(const fpcf4_catalogue* cat, const fpcf4_bins* bins,
                                    const fpcf4_options* opts_in, int64_t* counts, double* G, double* W) {
  if (!cat || !bins || !opts_in) return fail(FPCF4_E_INVALID_ARG, "null argument");
  // without a subset, report every galaxy in catalogue order
  fpcf4_options o = *opts_in;
  std::vector<int64_t> all;
  fpcf4_catalogue c = *cat;
  if (!o.centers && cat->n > 0) {
    if (cat->mem == FPCF4_MEM_DEVICE) {
      // the subset array lives in the catalogue's memory space; use a host copy
      return fail(FPCF4_E_INVALID_ARG, "debug on a device catalogue needs an explicit centre list");
    }
    all.resize((size_t)cat->n);
    for (int64_t i = 0; i < cat->n; ++i) all[(size_t)i] = i;
    o.centers = all.data();
    o.ncenters = cat->n;
  }
  const fpcf4_options* opts = &o;
  cat = &c;
  PlanInfo P;
  fpcf4_status st = make_plan(cat, bins, opts, P);
  if (st != FPCF4_OK) return st;
  setup_pool();
  hipStream_t s = static_cast<hipStream_t>(opts->stream);
  void* ws = nullptr;
  HIPCHK(hipMallocAsync(&ws, P.total, s));
  fpcf4_request* R = new fpcf4_request();
  R->want_counts = true;
  st = request_init(cat, bins, opts, ws, P.total, R);
  const Layout& L = R->P.L;
  const int nb = P.nb, n = P.nmax;
  std::vector<int32_t> hcnt;
  std::vector<char> hrec;
  for (int64_t t = 0; st == FPCF4_OK && t < P.ntiles; ++t) {
    st = request_step(R, t, false);
    if (st != FPCF4_OK) break;
    const int64_t c0 = t * P.tile;
    const int64_t nc = std::min<int64_t>(P.tile, P.ncent - c0);
    hcnt.resize((size_t)(nc * nb));
    hrec.resize((size_t)(L.mpc * nb * P.ldc * 2 * P.tsize));
    hipError_t e = hipMemcpyAsync(hcnt.data(), R->ws + P.o_counts, hcnt.size() * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hrec.data(), R->ws + P.o_region, hrec.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { st = fail(FPCF4_E_DEVICE, "debug copy: %s", hipGetErrorString(e)); break; }
    for (int64_t c = 0; c < nc; ++c) {
      for (int b = 0; b < nb; ++b) {
        const int64_t cb = c * nb + b, gcb = (c0 + c) * nb + b;
        if (counts) counts[gcb] = hcnt[(size_t)cb];
        auto val = [&](int e, int part) -> double {
          const size_t o = (((size_t)e * nb + b) * P.ldc + c) * 2 + part;
          if (P.tsize == 8) return reinterpret_cast<const double*>(hrec.data())[o];
          return (double)reinterpret_cast<const float*>(hrec.data())[o];
        };
        if (G)
          for (int k = 0; k < 4 * n + 3; ++k) {
            G[(gcb * (4 * n + 3) + k) * 2] = val(L.offG + k, 0);
            G[(gcb * (4 * n + 3) + k) * 2 + 1] = val(L.offG + k, 1);
          }
        if (W)
          for (int k = 0; k < 4 * n + 1; ++k) {
            W[(gcb * (4 * n + 1) + k) * 2] = val(L.offW + k, 0);
            W[(gcb * (4 * n + 1) + k) * 2 + 1] = val(L.offW + k, 1);
          }
      }
    }
  }
  delete R;
  hipError_t e = hipFreeAsync(ws, s);
  if (st == FPCF4_OK && e != hipSuccess) return fail(FPCF4_E_DEVICE, "hipFreeAsync: %s", hipGetErrorString(e));
  if (st == FPCF4_OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(FPCF4_E_DEVICE, "sync: %s", hipGetErrorString(e));
  }
  return st;
}

fpcf4_status fpcf4_to_natural(const double* upsilon, int32_t nbins, int32_t nmax, int32_t nphi,
                              double* gamma_out, double* norm_out, void* stream) {
  if (!upsilon || !gamma_out) return fail(FPCF4_E_INVALID_ARG, "null argument");
  if (nbins < 1 || nbins > FPCF4_NBINS_SUPPORTED) return fail(FPCF4_E_INVALID_ARG, "nbins %d", nbins);
  if (nmax < 0 || nmax > FPCF4_NMAX_SUPPORTED) return fail(FPCF4_E_INVALID_ARG, "nmax %d", nmax);
  if (nphi < 1 || nphi > 4096) return fail(FPCF4_E_INVALID_ARG, "nphi %d", nphi);
  hipStream_t s = static_cast<hipStream_t>(stream);
  setup_pool();
  const int64_t nb3 = (int64_t)nbins * nbins * nbins, nn = 2 * nmax + 1;
  const size_t in_b = (size_t)(9 * nb3 * nn * nn) * 16;
  const size_t tmp_b = (size_t)(9 * nb3 * nphi * nn) * 16;
  const size_t g_b = (size_t)(8 * nb3 * nphi * nphi) * 16;
  const size_t n_b = (size_t)(nb3 * nphi * nphi) * 8;
  char* buf = nullptr;
  HIPCHK(hipMallocAsync(reinterpret_cast<void**>(&buf), up(in_b) + up(tmp_b) + up(g_b) + up(n_b), s));
  double* din = reinterpret_cast<double*>(buf);
  double* dtmp = reinterpret_cast<double*>(buf + up(in_b));
  double* dg = reinterpret_cast<double*>(buf + up(in_b) + up(tmp_b));
  double* dn = reinterpret_cast<double*>(buf + up(in_b) + up(tmp_b) + up(g_b));
  fpcf4_status st = FPCF4_OK;
  hipError_t e = hipMemcpyAsync(din, upsilon, in_b, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = natural_components(din, nbins, nmax, nphi, dtmp, dg, dn, s);
  if (e == hipSuccess) e = hipMemcpyAsync(gamma_out, dg, g_b, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess && norm_out) e = hipMemcpyAsync(norm_out, dn, n_b, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) st = fail(FPCF4_E_DEVICE, "to_natural: %s", hipGetErrorString(e));
  (void)hipFreeAsync(buf, s);
  (void)hipStreamSynchronize(s);
  return st;
}

fpcf4_status fpcf4_to_natural_triplets(const double* upsilon, int32_t ups_mem, int32_t nbins,
                                       int32_t nmax, int32_t nphi, const int32_t* triplets,
                                       int64_t ntrip, double* gamma_out, double* norm_out,
                                       int32_t out_mem, void* stream) {
  if (!upsilon || !gamma_out || (ntrip > 0 && !triplets)) return fail(FPCF4_E_INVALID_ARG, "null argument");
  if (ups_mem != FPCF4_MEM_HOST && ups_mem != FPCF4_MEM_DEVICE) return fail(FPCF4_E_INVALID_ARG, "ups_mem %d", ups_mem);
  if (out_mem != FPCF4_MEM_HOST && out_mem != FPCF4_MEM_DEVICE) return fail(FPCF4_E_INVALID_ARG, "out_mem %d", out_mem);
  if (nbins < 1 || nbins > FPCF4_NBINS_SUPPORTED) return fail(FPCF4_E_INVALID_ARG, "nbins %d", nbins);
  if (nmax < 0 || nmax > FPCF4_NMAX_SUPPORTED) return fail(FPCF4_E_INVALID_ARG, "nmax %d", nmax);
  if (nphi < 1 || nphi > 4096) return fail(FPCF4_E_INVALID_ARG, "nphi %d", nphi);
  if (ntrip < 0 || ntrip > (int64_t(1) << 24)) return fail(FPCF4_E_INVALID_ARG, "ntrip %lld", (long long)ntrip);
  for (int64_t t = 0; t < 3 * ntrip; ++t)
    if (triplets[t] < 0 || triplets[t] >= nbins)
      return fail(FPCF4_E_INVALID_ARG, "triplet bin %d out of range", triplets[t]);
  if (ntrip == 0) return FPCF4_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  setup_pool();
  const int64_t nn = 2 * nmax + 1;
  const size_t in_b = ups_mem == FPCF4_MEM_HOST ? (size_t)fpcf4_output_elems(nbins, nmax) * 16 : 0;
  const size_t trip_b = (size_t)ntrip * 3 * 4;
  const size_t sel_b = (size_t)(9 * ntrip * nn * nn) * 16;
  const size_t tmp_b = (size_t)(9 * ntrip * nphi * nn) * 16;
  const size_t bin_b = (size_t)(9 * ntrip * nphi * nphi) * 16;
  const size_t g_b = out_mem == FPCF4_MEM_HOST ? (size_t)(8 * ntrip * nphi * nphi) * 16 : 0;
  const size_t n_b = (size_t)(ntrip * nphi * nphi) * 8;   // always staged unless written in place
  const size_t o_in = 0, o_trip = up(in_b), o_sel = o_trip + up(trip_b), o_tmp = o_sel + up(sel_b),
               o_bin = o_tmp + up(tmp_b), o_g = o_bin + up(bin_b), o_n = o_g + up(g_b),
               total = o_n + up(n_b);
  char* buf = nullptr;
  HIPCHK(hipMallocAsync(reinterpret_cast<void**>(&buf), total, s));
  const double* ups = ups_mem == FPCF4_MEM_HOST ? reinterpret_cast<const double*>(buf + o_in) : upsilon;
  const bool dev_out = out_mem == FPCF4_MEM_DEVICE;
  double* gdst = dev_out ? gamma_out : reinterpret_cast<double*>(buf + o_g);
  double* ndst = dev_out && norm_out ? norm_out : reinterpret_cast<double*>(buf + o_n);
  fpcf4_status st = FPCF4_OK;
  hipError_t e = hipSuccess;
  if (in_b) e = hipMemcpyAsync(buf + o_in, upsilon, in_b, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(buf + o_trip, triplets, trip_b, hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = natural_triplets(ups, nbins, nmax, nphi, reinterpret_cast<const int32_t*>(buf + o_trip), ntrip,
                         reinterpret_cast<double*>(buf + o_sel), reinterpret_cast<double*>(buf + o_tmp),
                         reinterpret_cast<double*>(buf + o_bin), gdst, ndst, s);
  if (e == hipSuccess && !dev_out) {
    e = hipMemcpyAsync(gamma_out, gdst, g_b, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && norm_out) e = hipMemcpyAsync(norm_out, ndst, n_b, hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) st = fail(FPCF4_E_DEVICE, "to_natural_triplets: %s", hipGetErrorString(e));
  (void)hipFreeAsync(buf, s);
  (void)hipStreamSynchronize(s);
  return st;
}

}  // extern "C"
