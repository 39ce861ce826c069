// Internal declarations of libfpcf4 (host and device).
//
// Per-centre multipole record.  For every centre and radial bin, stage (a)
// writes one record of complex entries (binary64 in the FP64 path, binary32
// in the mixed paths).  The entries are the blocks the contraction and the
// degenerate-term subtraction read (Sect. 3.1, App. A.1 Table 1):
//
//   G_k = sum_j w_j gamma_j e^{ik phi_ij}       k = -2n-3 .. 2n-1
//   W_k = sum_j w_j e^{ik phi_ij}               k = -2n   .. 2n
//   Q_k = sum_j (w_j gamma_j)^2 e^{ik phi_ij}   k = qlo   .. qhi
//   A_k = sum_j |w_j gamma_j|^2 e^{ik phi_ij}   k = 0 .. ka  (A_-k = conj A_k)
//   V_k = sum_j w_j^2 e^{ik phi_ij}             k = 0 .. 2n  (V_-k = conj V_k)
//   T_-8, T_-4 with T_k = sum_j (w_j gamma_j)^3 e^{ik phi_ij}
//   M_-4, M_0  with M_k = sum_j |w_j gamma_j|^2 w_j gamma_j e^{ik phi_ij}
//   U = sum_j w_j^3
//
// with qlo = min(-2n-5, -n-6), qhi = max(2n-3, n-2), ka = max(2n+1, n+2):
// exactly the orders the factor table of Sect. 3.1 and Table 1 touch for
// |n2|, |n3| <= n.  Records are laid out [entry][bin][centre] (centre
// contiguous, row stride ldc), so the contraction and the correction sums
// stream centres with coalesced loads.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/fpcf4.h"

namespace fpcf4 {

struct Layout {
  int n;                // nmax
  int qlo, qhi, ka;     // Q order range, A top order
  int offG, offW, offQ, offA, offV, offS;
  int mpc;              // complex entries used
  int rec;              // complex entries per record (even)
};

__host__ __device__ constexpr int imax(int a, int b) { return a > b ? a : b; }
__host__ __device__ constexpr int imin(int a, int b) { return a < b ? a : b; }

__host__ __device__ inline Layout make_layout(int n) {
  Layout L{};
  L.n = n;
  L.qlo = imin(-2 * n - 5, -n - 6);
  L.qhi = imax(2 * n - 3, n - 2);
  L.ka = imax(2 * n + 1, n + 2);
  L.offG = 0;
  L.offW = L.offG + 4 * n + 3;
  L.offQ = L.offW + 4 * n + 1;
  L.offA = L.offQ + (L.qhi - L.qlo + 1);
  L.offV = L.offA + L.ka + 1;
  L.offS = L.offV + 2 * n + 1;
  L.mpc = L.offS + 5;
  L.rec = (L.mpc + 1) & ~1;
  return L;
}

// entry indices inside a record
__host__ __device__ inline int eG(const Layout& L, int k) { return L.offG + k + 2 * L.n + 3; }
__host__ __device__ inline int eW(const Layout& L, int k) { return L.offW + k + 2 * L.n; }
__host__ __device__ inline int eQ(const Layout& L, int k) { return L.offQ + k - L.qlo; }
__host__ __device__ inline int eA(const Layout& L, int k) { return L.offA + k; }
__host__ __device__ inline int eV(const Layout& L, int k) { return L.offV + k; }
enum { S_T8 = 0, S_T4 = 1, S_M4 = 2, S_M0 = 3, S_U = 4 };

// Cell grid of the spatially sorted catalogue (row-major cells).
struct Grid {
  double x0, y0, h, inv_h;
  int ncx, ncy;
};

// One galaxy of the spatially sorted catalogue (array of structures, one
// 16-byte aligned record per galaxy so a neighbour costs two or three vector
// loads).  The weights are pre-multiplied: a = w g1, b = w g2, and they are
// held in the accumulation type of stage (a) (binary32 in the mixed paths,
// rounded once from the binary64 products).  Positions stay binary64: the
// bin decision is taken on binary64 separations.
template <typename T> struct alignas(16) Gal;
template <> struct alignas(16) Gal<float> { double x, y; float a, b, w, pad; };
template <> struct alignas(16) Gal<double> { double x, y, a, b, w, pad; };
static_assert(sizeof(Gal<float>) == 32 && sizeof(Gal<double>) == 48, "galaxy record size");

// One pseudo-galaxy of a reduced catalogue (tree approximation): the cell's
// w-weighted centre of mass and the cell sums of every per-galaxy family
// weight (Re/Im w g, Re/Im (w g)^2, |w g|^2, w^2, w, Re/Im (w g)^3,
// Re/Im |w g|^2 w g, w^3), each rounded once from its binary64 sum.
template <typename T> struct alignas(16) GalR;
template <> struct alignas(16) GalR<float> {
  double x, y;
  float a, b, c, d, e, v, w, p3, q3, ea, eb, u;
};
static_assert(sizeof(GalR<float>) == 64, "pseudo-galaxy record size");
constexpr int TREE_LEVELS_MAX = 4;

// Per-bin maxima of the records of a tile, written by stage (a) and read by
// the mixed-precision contraction to pick its power-of-two operand scales:
// float bits (all values are >= 0, so unsigned max is float max).
constexpr int MAXIMA_G = 0;                              // [nb] max |G_k| component per bin
constexpr int MAXIMA_W = FPCF4_NBINS_SUPPORTED;          // [nb] max |W_k| component per bin
constexpr int MAXIMA_X = 2 * FPCF4_NBINS_SUPPORTED;      // +0: max |w g| component, +1: max |w|
constexpr int MAXIMA_WORDS = 2 * FPCF4_NBINS_SUPPORTED + 2;

// Bin tiles of the contraction kernels: each workgroup holds at most
// BIN_TILE_MAX radial bins per bin dimension, so nb bins are cut into nt
// near-equal tiles of at most tb bins (one tile when nb <= BIN_TILE_MAX).
constexpr int BIN_TILE_MAX = 16;
struct BinTiles {
  int tb, nt;
};
__host__ __device__ inline BinTiles bin_tiles(int nb) {
  const int nt = (nb + BIN_TILE_MAX - 1) / BIN_TILE_MAX;
  return BinTiles{nt > 0 ? (nb + nt - 1) / nt : 0, nt};
}

// Sorted catalogue on the device.
struct SortedCat {
  int64_t n;
  const void* gal;            // Gal<T>[n], T = accumulation type of stage (a)
  const int32_t* cell_start;  // [ncx*ncy + 1]
  Grid g;
};

struct StageAArgs {
  SortedCat cat;
  const int32_t* centres;   // positions in cgal of this tile's centres
  const void* cgal;         // Gal<T> records of the centres: cat.gal, or base pseudo-galaxies
  int32_t ncent;
  int32_t nb;
  int32_t ldc;              // centre stride of record rows (>= ncent, multiple of 16)
  const double* e2;         // device squared edges [nb+1]
  const double* edges;      // device edges [nb+1]
  void* rec;                // records [entry][bin][ldc] complex (T)
  void* rec_aos;            // staging [centre][bin][entry] complex (T)
  void* xg;                 // [ldc] complex (T): w g of each tile centre
  void* xw;                 // [ldc] (T): w of each tile centre
  unsigned* maxima;         // scaling maxima (float bits, MAXIMA_* layout) or null
  int32_t* counts;          // [ncent][nb] or null
  int32_t* work_counter;    // dynamic centre scheduling counters, one per XCD
  unsigned long long* pairs;  // in-bin pair counter (may be null)
  int32_t b_lo, b_hi;       // bins to accumulate: [b_lo, b_hi); the rest are left alone
  // tree approximation: bins with level[b] = d >= 1 take their neighbours
  // from reduced catalogue d (same search grid as cat); 0 = discrete
  int8_t level[FPCF4_NBINS_SUPPORTED];
  const void* rgal[TREE_LEVELS_MAX];         // GalR<float>, sorted by search cell
  const int32_t* rcell[TREE_LEVELS_MAX];     // their cell starts
};

// Stable radix sort of (key, value) pairs on the low `bits` bits of the keys
// (every key must be below 2^bits), 1 <= bits <= 8 sizeof(K), n < 2^31.
// Sorted pairs in key_b / val_b; key_a / val_a are overwritten.  tmp holds at
// least radix_sort_temp_bytes(n) bytes.  Instantiated for uint32_t and
// uint64_t keys.
size_t radix_sort_temp_bytes(int64_t n);
template <typename K>
hipError_t radix_sort_pairs(void* tmp, size_t tmp_bytes, K* key_a, K* key_b, int32_t* val_a, int32_t* val_b,
                            int64_t n, int bits, hipStream_t s);
// out[i] = in[0] + ... + in[i-1] (int32, n < 2^31; in and out may not
// overlap); tmp holds at least scan_temp_bytes(n) bytes.
size_t scan_temp_bytes(int64_t n);
hipError_t exclusive_scan_i32(void* tmp, size_t tmp_bytes, const int32_t* in, int32_t* out, int64_t n,
                              hipStream_t s);

// Reduced catalogue of cell side delta anchored at (x0, y0) (tree
// approximation): pseudo-galaxies sorted on the search grid g, with cell
// starts.  Scratch is caller-provided (reduced_scratch_bytes); returns the
// number of pseudo-galaxies in *m (host, after a stream synchronisation).
// member (optional, [n]): the pseudo-galaxy of every galaxy (catalogue order).
size_t reduced_scratch_bytes(int64_t n);
hipError_t reduced_build(const double* x, const double* y, const double* g1, const double* g2,
                         const double* w, int64_t n, double x0, double y0, double xmax, double ymax,
                         double delta, const Grid& g, void* scratch, void* gal_out,
                         int32_t* cell_start, int64_t* m, hipStream_t s, int32_t* member = nullptr);

// stage (a) launcher, T = double or float: the pair-multipole kernel, then
// the relayout of its records to centre-contiguous rows.  Returns the number
// of pair-kernel launches in *nlaunch; records `mid` (if not null) between
// the two.
template <typename T>
hipError_t launch_stage_a(int nmax, int order, const StageAArgs& a, hipStream_t s, int* nlaunch, hipEvent_t mid);

// One distinct degenerate-term sum, a GEMM over centres
//   S[b, b'] = sum_i x_i E_i(b) F_i(b')
// with E a Table 1 block at the equal bins and F the remaining factor; the
// triple term has F = 1 (one column).
struct CorrSum {
  int8_t x, triple, eflip, fconj;  // centre factor (X_*); triple term; conjugate E / F
  int32_t eidx, fidx;              // record entries of E and F
};
// Every (mu, kind, order) of the correction buffer (kind 0: Theta_1 = Theta_2,
// 1: Theta_1 = Theta_3, 2: Theta_2 = Theta_3, 3: all equal) is one of a few
// hundred distinct sums: the three pair kinds are all x E(b) F(b'), and
// correlators share blocks.  sums holds the pair sums first, then the
// triple sums; map[mu][slot] (slot = kind 0 orders, kind 1 orders, kind 2
// orders, kind 3) names the sum.
struct CorrPlanHost {
  std::vector<CorrSum> sums;
  int npair = 0;
  std::vector<int32_t> map;        // [9][2 (2nmax+1) + (4nmax+1) + 1]
};
CorrPlanHost make_corr_plan(int nmax);
struct CorrArgs {
  const void* rec;
  const void* xg;
  const void* xw;
  int32_t ncent, nb, nmax, ldc;
  double* corr;             // correction sums, accumulated over tiles
  double* part;             // [CORR_SLICES][corr_elems] per-slice partial sums: the
                            // distinct sums, [npair][nb][nb] then [ntriple][nb]
  const CorrSum* sums;      // the distinct sums (device)
  const int32_t* map;       // (mu, kind, order) -> sum (device)
  int32_t nsums, npair;
};
constexpr int CORR_SLICES = 13;  // centre slices of the correction sums

template <typename T> hipError_t launch_corrections(const CorrArgs& a, hipStream_t s);

// Contraction on the matrix cores (stage_b_pairs.hip; every precision).
// Each distinct product x D E F of three blocks (with the centre factor x)
// is formed once over all bin triples: a work item is an unordered pair of
// column blocks (E, F), each (family, conjugation, order), whose Khatri-Rao
// product is formed once; its row blocks are the third blocks x D of the
// products assigned to that pair.  Every (mu, n2, n3) reads its product at
// its bins permuted into the item's roles.
constexpr int PAIR_MAX_BLK = 2;    // row blocks per work item (pairs with more are split)
constexpr int PAIR_SUB = 8192;     // centres per binary32 running sum before binary64
struct PairRow {
  int8_t x, fam, conj, pad;        // centre factor kind (X_*), row block family (F_*), conjugated
  int32_t order;                   // row block order
};
struct PairItem {
  int8_t famB, conjB, famC, conjC; // first and second column block: family, conjugated
  int32_t ordB, ordC;              // their orders
  int32_t nblk;                    // row blocks
  int32_t row0;                    // first row of the item in the partial layout
  int32_t pad;
  PairRow blk[PAIR_MAX_BLK];
};
struct PairOut {                   // where (mu, n2, n3) is computed
  // perm: bits 2j..2j+1 name which of (b1, b2, b3) supplies the bin of role j
  // of the item (0: its row block, 1 and 2: its first and second column block)
  int32_t item, blk, perm, pad;
};
struct PairPlanHost {
  std::vector<PairItem> items;     // grouped by row-block count
  int cls_start[PAIR_MAX_BLK + 1], cls_count[PAIR_MAX_BLK + 1];
  std::vector<PairOut> out;        // [9][2nmax+1][2nmax+1]
  int64_t total_rows;              // sum of 2 nb nblk over items
};
PairPlanHost make_pair_plan(int nmax, int nb);
int pair_slices(int64_t ncent);    // centre slices (partial regions) for a tile
struct PairArgs {
  const void* rec;                 // records (binary32 or binary64 complex)
  int64_t ldc;
  const void* xg;                  // [ldc] complex w g
  const void* xw;                  // [ldc] w
  const unsigned* maxima;
  const PairItem* items;
  int32_t item0, nitems, ncent, nb, nmax;
  int32_t tb, nt;                  // bin tiles (bin_tiles(nb)); blockIdx.z = (t1 nt + t2) nt + t3
  double* part;                    // [slices][total_rows][nb^2]
  int64_t total_rows;
};
struct PairLaunch {
  const void* rec;
  int64_t ldc;
  const void* xg;
  const void* xw;
  const unsigned* maxima;
  const PairItem* items;           // device copy of the plan
  const PairOut* out;
  int cls_start[PAIR_MAX_BLK + 1], cls_count[PAIR_MAX_BLK + 1];
  int ncent, nb, nmax, precision;
  int max_slices;                  // centre slices the partial buffer holds
  double* part;
  int64_t total_rows;
  double* ups;                     // accumulated into
};
hipError_t launch_contract_pairs(const PairLaunch& pl, hipStream_t s);
// matrix-core flops the pair contraction issues for ncent centres
double pair_issued_flops(const PairPlanHost& pp, int nb, int64_t ncent, int precision);
// 8 flop per complex multiply-add of the distinct products: row blocks x nb^3
double pair_useful_flops(const PairPlanHost& pp, int nb, int64_t ncent);
size_t corr_elems(int nb, int nmax);  // complex elements of the correction buffer
hipError_t launch_finalize(const double* ups_raw, const double* corr, int nb, int nmax,
                           int subtract, double* out, hipStream_t s);

// Shear 3PCF multipoles from the same records (threepcf.hip).
constexpr int THREE_SLICES = 16;   // centre slices of the 3PCF sums
// complex elements of the 3PCF accumulator: [5][2m+1][nb][nb] multipole sums,
// then [5][nb] same-neighbour sums
__host__ __device__ inline size_t three_elems(int nb, int m) {
  return (size_t)5 * (2 * m + 1) * nb * nb + (size_t)5 * nb;
}
struct ThreeArgs {
  const void* rec;          // records of the tile (stage (a) of order n4): the Theta_1 slot
  const void* xg;           // [ldc] complex (T): w g of each tile centre
  const void* xw;           // [ldc] (T): w of each tile centre
  int32_t ncent, nb, n4, m, nn, ldc;   // m: largest 3PCF multipole (<= 2 n4), nn = 2m+1
  double* part;             // [THREE_SLICES][three_elems] complex partial sums
  double* acc;              // [three_elems] complex, accumulated over tiles
  // BaseTree: the Theta_2 slot may read other records (another base grid),
  // and either slot may read its record at the centre's parent on a coarser
  // grid.  Plain estimate: rec2 = rec, ldc2 = ldc, no parents, all bins.
  const void* rec2;
  int32_t ldc2;
  const int32_t* par1;      // [ncent] record column of slot 1, or null (= centre)
  const int32_t* par2;      // [ncent] record column of slot 2, or null
  int32_t lo1, nb1, lo2, nb2;   // bins of slot 1: [lo1, lo1 + nb1); of slot 2 likewise
};
template <typename T> hipError_t launch_three(const ThreeArgs& a, hipStream_t s);
// out[mu][b1][b2][n] (complex128) from the accumulator, minus the
// same-neighbour sums on b1 == b2 when subtract != 0
hipError_t launch_finalize3(const double* acc, int nb, int m, int subtract, double* out, hipStream_t s);

}  // namespace fpcf4
