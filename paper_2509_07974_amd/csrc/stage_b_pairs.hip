// Stage (b) on the matrix cores (every precision), organised by pairs of
// blocks whose Khatri-Rao product is formed once (Sect. 3.1):
//
//   Upsilon_mu[b1,b2,b3; n2,n3] = sum_i (x A)_i(b1) * B_i(b2) C_i(b3),
//
// with x the centre factor, A the block at Theta_1 (order depending on
// n2 + n3), B and C the blocks at Theta_2 and Theta_3 (orders depending on n2
// and n3).  The contraction is a GEMM over the centre index whose right
// operand, the Khatri-Rao product R(b2,b3) = B(b2) C(b3), has to be formed on
// the vector ALUs; the left operand y(b1) = x A(b1) is a per-centre vector.
//
// Many (mu, n2, n3) need the same product of three blocks.  Upsilon is a
// sum over centres of x times a block at each of the three bins, and which
// block is called the one at Theta_1, 2 or 3 is only a labelling of those
// bins: if the blocks (A, B, C) of one (mu, n2, n3) are a permutation of the
// blocks (D, E, F) of another (same x), then its Upsilon[b1, b2, b3] is the
// other's sum read at the correspondingly permuted bins.  This is the
// radial symmetry of Sect. 3.1 and Table 2 (a correlator at permuted radii
// is another correlator at other multipoles) taken at the level of the
// blocks, and it holds for every (n2, n3) in range, so no extended multipole
// range is needed.  The factor table uses only G_k (plain or conjugated) and
// W_k, so the 9 (2nmax+1)^2 products reduce to 1121 distinct multisets of
// three blocks (with x) at nmax = 10.  The host plan (make_pair_plan) covers
// them with few column pairs: a work item is an unordered pair (E, F) whose
// Khatri-Rao product R(c2, c3) = E(c2) F(c3) is formed once, over all bins;
// its rows are the third blocks x D(c1) of the multisets assigned to it.  An
// output map sends each (mu, n2, n3) to (item, row block, permutation of
// (b1, b2, b3) into (c1, c2, c3)).  At nmax = 10: 665 work items and 1121
// row blocks, against 3969 (mu, n2, n3) GEMMs of one row block each.
//
// Per work item and centre slice, one workgroup of W waves: a chunk of 32
// centres is staged in LDS as B and C rows (binary32 complex, power-of-two
// scaled per bin) and as the left operand y = x A in MFMA lane order, split
// y = hi + lo in the 16-bit format; every wave forms R for its column tiles
// (16 columns (b2, b3) each), splits it, and issues
// v_mfma_f32_16x16x32_{f16,bf16} for hi*hi + hi*lo + lo*hi over all row
// tiles.  Complex products are real-split: rows (block, re/im, b1) hold
// [y_r, -y_i] or [y_i, y_r] per centre against columns [R_r; R_i].
//
// Accumulation: fp32 in the MFMA accumulators over 512 centres, added into
// an fp32 running sum over at most 8192 centres, which is converted to
// binary64 (unscaled exactly) and written into the workgroup's own region of
// the slice partial buffer (the first sub-slice stores, later ones add: the
// same lanes read back what they wrote).  pair_slice_sum_kernel adds the
// slices in order (coalesced, into the first slice) and pair_reduce_kernel
// scatters every (mu, n2, n3) from its item and permutation into the output
// tensor.  No atomics: the result is deterministic.
#include <algorithm>
#include <array>
#include <map>
#include <tuple>
#include <type_traits>
#include <vector>

#include "factors.hpp"
#include "fpcf4_internal.hpp"

namespace fpcf4 {

// ---------------------------------------------------------------------------
// host: the plan
// ---------------------------------------------------------------------------
PairPlanHost make_pair_plan(int nmax, int nb) {
  typedef std::tuple<int, int, int> Spec;            // family, conj, order
  typedef std::array<Spec, 3> Triple;                // sorted blocks of a product
  typedef std::pair<int, Triple> Multi;              // (x kind, sorted blocks)
  typedef std::pair<Spec, Spec> Pair;                // sorted column blocks
  const int nn = 2 * nmax + 1;
  // 1. every (mu, n2, n3): its centre factor, the blocks at Theta_1,2,3 and
  // the multiset they form
  struct Tuple { int x; Spec s[3]; int ms; };
  std::vector<Tuple> tup((size_t)FPCF4_NCORR * nn * nn);
  std::map<Multi, int> ms_id;
  for (int mu = 0; mu < FPCF4_NCORR; ++mu) {
    const MuFactors F = mu_factors(mu);
    for (int n2 = -nmax; n2 <= nmax; ++n2)
      for (int n3 = -nmax; n3 <= nmax; ++n3) {
        Tuple& t = tup[((size_t)mu * nn + (n2 + nmax)) * nn + (n3 + nmax)];
        t.x = F.x;
        t.s[0] = Spec{F.A.fam, F.A.conj, F.A.a * n2 + F.A.b * n3 + F.A.c};
        t.s[1] = Spec{F.B.fam, F.B.conj, F.B.a * n2 + F.B.b * n3 + F.B.c};
        t.s[2] = Spec{F.C.fam, F.C.conj, F.C.a * n2 + F.C.b * n3 + F.C.c};
        Triple m{t.s[0], t.s[1], t.s[2]};
        std::sort(m.begin(), m.end());
        ms_id.emplace(Multi{t.x, m}, 0);
      }
  }
  std::vector<Multi> ms;
  for (auto& kv : ms_id) {
    kv.second = (int)ms.size();
    ms.push_back(kv.first);
  }
  for (Tuple& t : tup) {
    Triple m{t.s[0], t.s[1], t.s[2]};
    std::sort(m.begin(), m.end());
    t.ms = ms_id.at(Multi{t.x, m});
  }
  // the (up to three) pairs each multiset can be formed from, ids in pair order
  std::map<Pair, int> pair_id;
  for (const Multi& m : ms)
    for (int i = 0; i < 3; ++i) pair_id.emplace(Pair{m.second[i == 0 ? 1 : 0], m.second[i == 2 ? 1 : 2]}, 0);
  std::vector<Pair> pairs;
  for (auto& kv : pair_id) {
    kv.second = (int)pairs.size();
    pairs.push_back(kv.first);
  }
  std::vector<std::vector<int>> cands(ms.size()), ms_of(pairs.size());
  for (size_t k = 0; k < ms.size(); ++k)
    for (int i = 0; i < 3; ++i) {
      const int q = pair_id.at(Pair{ms[k].second[i == 0 ? 1 : 0], ms[k].second[i == 2 ? 1 : 2]});
      if (std::find(cands[k].begin(), cands[k].end(), q) != cands[k].end()) continue;
      cands[k].push_back(q);
      ms_of[q].push_back((int)k);
    }
  // 2. cover the multisets with few pairs (greedy: the pair that forms the
  // most uncovered multisets first), then move multisets between chosen
  // pairs so that fewer pairs carry an odd number of rows (an odd one leaves
  // a one-block item)
  std::vector<int> open(pairs.size()), assign(ms.size(), -1), nrows(pairs.size(), 0);
  for (size_t q = 0; q < pairs.size(); ++q) open[q] = (int)ms_of[q].size();
  for (size_t left = ms.size(); left > 0;) {
    const int best = (int)(std::max_element(open.begin(), open.end()) - open.begin());
    for (int k : ms_of[best]) {
      if (assign[k] >= 0) continue;
      assign[k] = best;
      nrows[best] += 1;
      --left;
      for (int q : cands[k]) open[q] -= 1;
    }
  }
  for (bool moved = true; moved;) {                  // each move evens two pairs: terminates
    moved = false;
    for (size_t k = 0; k < ms.size(); ++k) {
      if (nrows[assign[k]] % 2 == 0) continue;
      for (int q : cands[k])
        if (q != assign[k] && nrows[q] % 2 == 1) {
          nrows[assign[k]] -= 1;
          nrows[q] += 1;
          assign[k] = q;
          moved = true;
          break;
        }
    }
  }
  // 3. rows of every pair: the block of each multiset that is not in the pair
  typedef std::tuple<int, int, int, int> RowKey;     // x kind, family, conj, order
  auto row_spec = [&](int k) {
    const Pair& q = pairs[assign[k]];
    std::vector<Spec> rest(ms[k].second.begin(), ms[k].second.end());
    rest.erase(std::find(rest.begin(), rest.end(), q.first));
    rest.erase(std::find(rest.begin(), rest.end(), q.second));
    return rest[0];
  };
  std::vector<std::vector<std::pair<RowKey, int>>> rows_of(pairs.size());
  for (size_t k = 0; k < ms.size(); ++k) {
    const Spec r = row_spec((int)k);
    rows_of[assign[k]].push_back({RowKey{ms[k].first, std::get<0>(r), std::get<1>(r), std::get<2>(r)}, (int)k});
  }
  // 4. work items of at most PAIR_MAX_BLK row blocks (a pair with more rows
  // is split over several items that form the same R), grouped by their
  // number of row blocks (one kernel per class)
  PairPlanHost P;
  P.out.assign((size_t)FPCF4_NCORR * nn * nn, PairOut{-1, 0, 0, 0});
  for (int c = 0; c <= PAIR_MAX_BLK; ++c) P.cls_start[c] = P.cls_count[c] = 0;
  struct Unit { int pair; std::vector<std::pair<RowKey, int>> rows; };
  std::vector<Unit> units;
  for (size_t q = 0; q < pairs.size(); ++q) {
    auto& rr = rows_of[q];
    std::sort(rr.begin(), rr.end());
    for (size_t k = 0; k < rr.size(); k += PAIR_MAX_BLK) {
      Unit u{(int)q, {}};
      for (size_t j = k; j < rr.size() && j < k + PAIR_MAX_BLK; ++j) u.rows.push_back(rr[j]);
      units.push_back(u);
    }
  }
  std::vector<std::pair<int, int>> where(ms.size());  // multiset -> (item, row block)
  int64_t rows = 0;
  for (int nbk = 1; nbk <= PAIR_MAX_BLK; ++nbk) {
    P.cls_start[nbk] = (int)P.items.size();
    for (const Unit& un : units) {
      if ((int)un.rows.size() != nbk) continue;
      const Pair& key = pairs[un.pair];
      PairItem it{};
      it.famB = (int8_t)std::get<0>(key.first);
      it.conjB = (int8_t)std::get<1>(key.first);
      it.ordB = std::get<2>(key.first);
      it.famC = (int8_t)std::get<0>(key.second);
      it.conjC = (int8_t)std::get<1>(key.second);
      it.ordC = std::get<2>(key.second);
      it.nblk = nbk;
      it.row0 = (int32_t)rows;
      for (int k = 0; k < nbk; ++k) {
        const RowKey& rk = un.rows[k].first;
        it.blk[k].x = (int8_t)std::get<0>(rk);
        it.blk[k].fam = (int8_t)std::get<1>(rk);
        it.blk[k].conj = (int8_t)std::get<2>(rk);
        it.blk[k].order = std::get<3>(rk);
        where[un.rows[k].second] = {(int)P.items.size(), k};
      }
      rows += (int64_t)nbk * 2 * nb;
      P.items.push_back(it);
    }
    P.cls_count[nbk] = (int)P.items.size() - P.cls_start[nbk];
  }
  P.total_rows = rows;
  // 5. the output map: (mu, n2, n3) reads its item's region at the bins of
  // its blocks permuted into the item's (row, column-pair) roles
  for (size_t o = 0; o < tup.size(); ++o) {
    const Tuple& t = tup[o];
    const Pair& q = pairs[assign[t.ms]];
    const Spec role[3] = {row_spec(t.ms), q.first, q.second};
    // src[j]: which of (b1, b2, b3) supplies the bin of role j
    bool used[3] = {false, false, false};
    int code = 0;
    for (int j = 0; j < 3; ++j) {
      int i = 0;
      while (used[i] || t.s[i] != role[j]) ++i;
      used[i] = true;
      code |= i << (2 * j);
    }
    P.out[o] = PairOut{where[t.ms].first, where[t.ms].second, code, 0};
  }
  return P;
}

// centre slices of the pair contraction: enough workgroups to fill the chip,
// at most 32 (each slice owns a binary64 partial region of every item)
int pair_slices(int64_t ncent) {
  int64_t s = (ncent + PAIR_SUB - 1) / PAIR_SUB;
  return (int)std::max<int64_t>(1, std::min<int64_t>(s, 32));
}

// ---------------------------------------------------------------------------
// device
// ---------------------------------------------------------------------------
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 bh8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __fp16 h2 __attribute__((ext_vector_type(2)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

template <int PREC> struct H8of;
template <> struct H8of<FPCF4_MIXED_FP16> { typedef h8 type; };
template <> struct H8of<FPCF4_MIXED_BF16> { typedef bh8 type; };

struct cf {
  float r, i;
};

constexpr int PKC = 32;             // centres per staged chunk (two K-steps of 16)
constexpr int PKS = PKC / 16;

// row tiles, column tiles, waves and column tiles per wave for NBLK row
// blocks at bin-count class NBC (8, 12 or 16 bins)
__host__ __device__ constexpr int pair_mt(int nblk, int nbc) { return (nblk * 2 * nbc + 15) / 16; }
__host__ __device__ constexpr int pair_ct(int nbc) { return (nbc * nbc + 15) / 16; }
__host__ __device__ constexpr int pair_waves(int nblk, int nbc) {
  return nbc == 8 ? 2 : nbc == 12 ? 3 : (nblk > 1 ? 8 : 4);
}
__host__ __device__ constexpr int pair_nt(int nblk, int nbc) {
  return (pair_ct(nbc) + pair_waves(nblk, nbc) - 1) / pair_waves(nblk, nbc);
}

__device__ __forceinline__ float pow2_under(float m, int target_exp) {
  if (!(m > 0.0f)) return 1.0f;
  int e;
  frexpf(m, &e);                  // m < 2^e
  return ldexpf(1.0f, target_exp - e);
}

// lo = fp16(v - hi) for a packed pair, hi read from its half of `hh`
// (v_fma_mix{lo,hi}_f16: v * 1 - hi in binary32, one rounding to fp16)
__device__ __forceinline__ h2 lo_pair(float x0, float x1, h2 hh) {
  h2 lo;
  asm("v_fma_mixlo_f16 %0, %1, 1.0, -%3 op_sel_hi:[0,0,1]\n\t"
      "v_fma_mixhi_f16 %0, %2, 1.0, -%3 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
      : "=&v"(lo)
      : "v"(x0), "v"(x1), "v"(hh));
  return lo;
}

// v = hi + lo in the 16-bit format of PREC, eight values
template <int PREC>
__device__ __forceinline__ void split8(const float (&v)[8], typename H8of<PREC>::type& hi,
                                       typename H8of<PREC>::type& lo) {
  if constexpr (PREC == FPCF4_MIXED_FP16) {
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
      const h2 hh = __builtin_amdgcn_cvt_pkrtz(v[q], v[q + 1]);
      const h2 ll = lo_pair(v[q], v[q + 1], hh);
      hi[q] = (_Float16)hh[0];
      hi[q + 1] = (_Float16)hh[1];
      lo[q] = (_Float16)ll[0];
      lo[q + 1] = (_Float16)ll[1];
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const __bf16 h = (__bf16)v[q];
      hi[q] = h;
      lo[q] = (__bf16)(v[q] - (float)h);
    }
  }
}

template <int PREC>
__device__ __forceinline__ f4 mma(const typename H8of<PREC>::type& a, const typename H8of<PREC>::type& b, f4 c) {
  if constexpr (PREC == FPCF4_MIXED_FP16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int rec_entry(const Layout& L, int fam, int k) {
  return fam == F_G ? eG(L, k) : eW(L, k);
}

// The bin tile of this workgroup (blockIdx.z = (t1 nt + t2) nt + t3): the
// bins b1, b2, b3 it covers are [o, o + n) with n <= tb.
struct BinRange {
  int o1, o2, o3, n1, n2, n3;
};
__device__ __forceinline__ BinRange bin_range(const PairArgs& a) {
  const int z = (int)blockIdx.z, nt = a.nt, tb = a.tb;
  const int t3 = z % nt, t2 = (z / nt) % nt, t1 = z / (nt * nt);
  BinRange r;
  r.o1 = t1 * tb;
  r.o2 = t2 * tb;
  r.o3 = t3 * tb;
  r.n1 = imin(tb, a.nb - r.o1);
  r.n2 = imin(tb, a.nb - r.o2);
  r.n3 = imin(tb, a.nb - r.o3);
  return r;
}

// The hardware deals workgroups to the 8 XCDs round-robin in dispatch order.
// Renumber them so that each XCD runs a contiguous range of (slice, item):
// the items of one centre slice, which read the same record columns, then
// share that XCD's L2.  A bijection of the grid onto itself.
__device__ __forceinline__ void xcd_contiguous(int& bx, int& by) {
  const int gx = (int)gridDim.x, total = gx * (int)gridDim.y;
  const int lin = (int)blockIdx.y * gx + (int)blockIdx.x;
  const int per = total >> 3, rem = total & 7;
  const int x = lin & 7, i = lin >> 3;
  const int l = x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
  bx = l % gx;
  by = l / gx;
}

// Three waves per SIMD (the compiler keeps the kernel within 168 registers):
// four 3-wave workgroups per CU at 12 bins, whose LDS (38 KB each) fits.
template <int PREC, int NBLK, int NBC>
__global__ __launch_bounds__(64 * pair_waves(NBLK, NBC)) __attribute__((amdgpu_waves_per_eu(3)))
void contract_pair_kernel(PairArgs a) {
  typedef typename H8of<PREC>::type H8;
  constexpr int MT = pair_mt(NBLK, NBC);
  constexpr int W = pair_waves(NBLK, NBC);
  constexpr int NT = pair_nt(NBLK, NBC);
  constexpr int NTH = 64 * W;
  constexpr int BS = PKC + 2;            // LDS row stride (complex): 16-byte rows, conflict-free
  static_assert(NBC * PKC / 2 <= NTH, "one B/C centre pair per thread");
  static_assert(NBLK * NBC * 4 * PKS <= NTH, "one left-operand unit per thread");
  const int nb = a.nb, n = a.nmax;
  const Layout L = make_layout(n);
  int bx, by;
  xcd_contiguous(bx, by);
  const PairItem it = a.items[a.item0 + bx];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  // bin tile: b1 in [o1, o1 + n1), b2 in [o2, o2 + n2), b3 in [o3, o3 + n3)
  const BinRange br = bin_range(a);
  const int o1 = br.o1, o2 = br.o2, o3 = br.o3, n1 = br.n1, n2 = br.n2, n3 = br.n3;
  const int ncols = n2 * n3;              // columns (b2, b3) of the tile
  const int ntiles = (ncols + 15) >> 4;
  const int mrows = NBLK * 2 * n1;
  // centres [cbase, cbase + ncent) of this slice
  const int per = (int)((((int64_t)a.ncent + gridDim.y - 1) / gridDim.y + PKC - 1) / PKC * PKC);
  const int cbase = by * per;
  const int ncent = imax(0, imin(a.ncent - cbase, per));
  const int64_t ldc = a.ldc;
  const int lastc = (int)ldc - 4;         // last 4-aligned group start inside a record row

  __shared__ cf Bs[2][NBC][BS];
  __shared__ cf Cs[2][NBC][BS];
  __shared__ H8 Ys[2][PKS][MT][2][64];    // left operand in MFMA lane order, hi / lo
  __shared__ float scl[3][16];            // scales of y (per b1), B (per b2), C (per b3)
  __shared__ float inv[3][16];            // their inverses (exact: powers of two)

  if (tid < 16) {
    const unsigned* M = a.maxima;
    float sy = 1.0f, sb = 1.0f, sc = 1.0f;
    // y = x A below 2^14 per component, B and C below 2^6: R = B C below 2^13
    if (tid < n1) {
      const int famA = it.blk[0].fam == F_G ? MAXIMA_G : MAXIMA_W;
      const float mx = __uint_as_float(M[MAXIMA_X + (it.blk[0].x == X_W ? 1 : 0)]);
      sy = pow2_under(2.0f * mx * __uint_as_float(M[famA + o1 + tid]), 14);
    }
    if (tid < n2) sb = pow2_under(1.5f * __uint_as_float(M[(it.famB == F_G ? MAXIMA_G : MAXIMA_W) + o2 + tid]), 6);
    if (tid < n3) sc = pow2_under(1.5f * __uint_as_float(M[(it.famC == F_G ? MAXIMA_G : MAXIMA_W) + o3 + tid]), 6);
    scl[0][tid] = sy; inv[0][tid] = 1.0f / sy;
    scl[1][tid] = sb; inv[1][tid] = 1.0f / sb;
    scl[2][tid] = sc; inv[2][tid] = 1.0f / sc;
  }
  // left-operand rows past the used ones stay zero in both buffers
  {
    u4* yz = reinterpret_cast<u4*>(&Ys[0][0][0][0][0]);
    for (int z = tid; z < 2 * PKS * MT * 2 * 64; z += NTH) {
      const int m = (z / 128) % MT;
      const int l = z & 63;
      if (16 * m + (l & 15) >= mrows) yz[z] = u4{0u, 0u, 0u, 0u};
    }
  }

  // ---- staging slots of this thread (one each)
  // B / C: a pair of centres 2p, 2p+1 of bin sb, loaded as 16 bytes
  const int sbin = tid >> 4, spair = tid & 15;
  const bool sb_on = sbin < n2, sc_on = sbin < n3;
  const float* recf = reinterpret_cast<const float*>(a.rec);
  const float* rowBp = recf + 2 * (((int64_t)rec_entry(L, it.famB, it.ordB) * nb + o2 + (sb_on ? sbin : 0)) * ldc);
  const float* rowCp = recf + 2 * (((int64_t)rec_entry(L, it.famC, it.ordC) * nb + o3 + (sc_on ? sbin : 0)) * ldc);
  // left operand: unit (block, b1, K-step, lane group q) = four consecutive
  // centres 16 ks + 4 q + (0..3) of row (block, b1); it writes the
  // real-output and the imaginary-output rows of that b1
  // b1 runs fastest over the threads, so that the 64 lanes of a wave write
  // consecutive 16-byte slots of the operand (no LDS bank conflicts)
  const int ub1 = tid % NBC, urest = tid / NBC;
  const int uq = urest & 3, uks = (urest >> 2) & 1, ublk = urest >> 3;
  const bool u_on = ublk < NBLK && ub1 < n1;
  PairRow rb = it.blk[0];
  if (NBLK > 1 && ublk == 1) rb = it.blk[1];
  const float* rowAp = recf + 2 * (((int64_t)rec_entry(L, rb.fam, rb.order) * nb + o1 + (u_on ? ub1 : 0)) * ldc);
  const bool xconj = rb.x == X_GC, aconj = rb.conj != 0;
  const bool x_is_w = it.blk[0].x == X_W;   // the W items use w; all others w g
  const float4* xg4 = reinterpret_cast<const float4*>(a.xg);
  const float4* xw4 = reinterpret_cast<const float4*>(a.xw);

  float4 pb, pc, pa0, pa1, px0, px1;
  auto issue = [&](int c0) {
    const int gp = imin(cbase + c0 + 2 * spair, (int)ldc - 2);
    pb = *reinterpret_cast<const float4*>(rowBp + 2 * (int64_t)gp);
    pc = *reinterpret_cast<const float4*>(rowCp + 2 * (int64_t)gp);
    const int gu = imin(cbase + c0 + 16 * uks + 4 * uq, lastc);
    const float4* pa = reinterpret_cast<const float4*>(rowAp + 2 * (int64_t)gu);
    pa0 = pa[0];
    pa1 = pa[1];
    if (x_is_w) {
      px0 = xw4[gu >> 2];
    } else {
      px0 = xg4[gu >> 1];
      px1 = xg4[(gu >> 1) + 1];
    }
  };
  auto commit = [&](int c0, int buf) {
    if (sb_on || sc_on) {
      // centres past the tile read stale record memory (possibly NaN
      // patterns) inside the row stride: select zeros, never multiply.
      // (A row past n2 or n3 holds a clamped bin and is never read.)
      const int cc = 2 * spair;
      const bool l0 = c0 + cc < ncent, l1 = c0 + cc + 1 < ncent;
      const float sb = scl[1][sbin], sc = scl[2][sbin];
      const float bs = it.conjB ? -sb : sb, cs = it.conjC ? -sc : sc;
      *reinterpret_cast<float4*>(&Bs[buf][sbin][cc]) =
          float4{l0 ? pb.x * sb : 0.0f, l0 ? pb.y * bs : 0.0f, l1 ? pb.z * sb : 0.0f, l1 ? pb.w * bs : 0.0f};
      *reinterpret_cast<float4*>(&Cs[buf][sbin][cc]) =
          float4{l0 ? pc.x * sc : 0.0f, l0 ? pc.y * cs : 0.0f, l1 ? pc.z * sc : 0.0f, l1 ? pc.w * cs : 0.0f};
    }
    if (u_on) {
      const float sy = scl[0][ub1];
      const float A[8] = {pa0.x, pa0.y, pa0.z, pa0.w, pa1.x, pa1.y, pa1.z, pa1.w};
      float X[8];
      if (x_is_w) {
        X[0] = px0.x; X[2] = px0.y; X[4] = px0.z; X[6] = px0.w;
        X[1] = X[3] = X[5] = X[7] = 0.0f;
      } else {
        X[0] = px0.x; X[1] = px0.y; X[2] = px0.z; X[3] = px0.w;
        X[4] = px1.x; X[5] = px1.y; X[6] = px1.z; X[7] = px1.w;
      }
      float vr[8], vi[8];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool live = c0 + 16 * uks + 4 * uq + v < ncent;
        const float xr = X[2 * v], xi = xconj ? -X[2 * v + 1] : X[2 * v + 1];
        const float ar = A[2 * v], ai = aconj ? -A[2 * v + 1] : A[2 * v + 1];
        // explicit fused forms: the rounding does not depend on how the
        // compiler would contract the expression
        float yr = __builtin_fmaf(xr, ar, -(xi * ai));
        float yi = __builtin_fmaf(xr, ai, xi * ar);
        yr = live ? yr * sy : 0.0f;
        yi = live ? yi * sy : 0.0f;
        vr[2 * v] = yr;      // real-output row: [y_r, -y_i]
        vr[2 * v + 1] = -yi;
        vi[2 * v] = yi;      // imaginary-output row: [y_i, y_r]
        vi[2 * v + 1] = yr;
      }
      H8 hr, lr, hi, li;
      split8<PREC>(vr, hr, lr);
      split8<PREC>(vi, hi, li);
      const int r_re = ublk * 2 * n1 + ub1, r_im = r_re + n1;
      Ys[buf][uks][r_re >> 4][0][16 * uq + (r_re & 15)] = hr;
      Ys[buf][uks][r_re >> 4][1][16 * uq + (r_re & 15)] = lr;
      Ys[buf][uks][r_im >> 4][0][16 * uq + (r_im & 15)] = hi;
      Ys[buf][uks][r_im >> 4][1][16 * uq + (r_im & 15)] = li;
    }
  };

  // this wave's column tiles T = wr + W t (valid for t < ntw); the wave
  // holding one more tile rotates with the item so co-resident workgroups
  // differ
  const int wr = (wv + bx) % W;
  const int ntw = imin(NT, imax(0, (ntiles - wr + W - 1) / W));
  int b2c[NT], b3c[NT];
  bool colok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = 16 * (wr + W * t) + (lane & 15);
    colok[t] = t < ntw && j < ncols;
    b2c[t] = colok[t] ? j / n3 : 0;
    b3c[t] = colok[t] ? j % n3 : 0;
  }

  f4 acc[MT][NT], mid[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc[m][t] = f4{0.f, 0.f, 0.f, 0.f};
      mid[m][t] = f4{0.f, 0.f, 0.f, 0.f};
    }

  // One chunk of compute over all NT column tiles of the wave.  A wave with
  // fewer valid tiles (bin counts whose nb^2 tiles do not divide evenly)
  // computes the surplus ones on columns it never writes: no branch inside
  // the MFMA sequence, and a single code path keeps the register count low.
  auto compute = [&](auto Vc, int buf) {
    constexpr int V = decltype(Vc)::value;
#pragma unroll
    for (int ks = 0; ks < PKS; ++ks) {
      const int cb = 16 * ks + 4 * (lane >> 4);
      H8 rh[V], rl[V];
#pragma unroll
      for (int t = 0; t < V; ++t) {
        const float4 b01 = *reinterpret_cast<const float4*>(&Bs[buf][b2c[t]][cb]);
        const float4 b23 = *reinterpret_cast<const float4*>(&Bs[buf][b2c[t]][cb + 2]);
        const float4 c01 = *reinterpret_cast<const float4*>(&Cs[buf][b3c[t]][cb]);
        const float4 c23 = *reinterpret_cast<const float4*>(&Cs[buf][b3c[t]][cb + 2]);
        const float B[8] = {b01.x, b01.y, b01.z, b01.w, b23.x, b23.y, b23.z, b23.w};
        const float Cv[8] = {c01.x, c01.y, c01.z, c01.w, c23.x, c23.y, c23.z, c23.w};
        float v[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          v[2 * u] = __builtin_fmaf(B[2 * u], Cv[2 * u], -(B[2 * u + 1] * Cv[2 * u + 1]));
          v[2 * u + 1] = __builtin_fmaf(B[2 * u], Cv[2 * u + 1], B[2 * u + 1] * Cv[2 * u]);
        }
        split8<PREC>(v, rh[t], rl[t]);
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const H8 yh = Ys[buf][ks][m][0][lane];
        const H8 yl = Ys[buf][ks][m][1][lane];
#pragma unroll
        for (int t = 0; t < V; ++t) acc[m][t] = mma<PREC>(yh, rh[t], acc[m][t]);
#pragma unroll
        for (int t = 0; t < V; ++t) acc[m][t] = mma<PREC>(yh, rl[t], acc[m][t]);
#pragma unroll
        for (int t = 0; t < V; ++t) acc[m][t] = mma<PREC>(yl, rh[t], acc[m][t]);
      }
    }
  };

  // write (first) or add the running sum, unscaled (exact powers of two), into
  // this workgroup's region of the slice partial buffer, then clear it
  // the item's region holds rows (block, re/im, b1) x columns (b2, b3) over
  // all nb bins; this workgroup owns the tile's rows and columns in it
  const int64_t gcols = (int64_t)nb * nb;
  double* part = a.part + ((int64_t)by * a.total_rows + it.row0) * gcols;
  auto flush = [&](bool first) {
    // opaque to the optimiser: the flush runs once per 8192 centres, so its
    // addresses are recomputed there instead of being hoisted out of the
    // chunk loop and held in registers across it
    double* pbase = part;
    int ln = lane;
    asm volatile("" : "+s"(pbase), "+v"(ln));
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (colok[t]) {
        const int j = 16 * (wr + W * t) + (ln & 15);
        const int b2 = j / n3, b3 = j - b2 * n3;
        const float ubc = inv[1][b2] * inv[2][b3];
        const int64_t gj = (int64_t)(o2 + b2) * nb + o3 + b3;
#pragma unroll
        for (int m = 0; m < MT; ++m) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * m + 4 * (ln >> 4) + r;
            if (row < mrows) {
              // row = k n1 + b1 with k = 2 block + (re/im) < 4; in the item's
              // region that row sits at k nb + o1 + b1
              const int k = (row >= n1) + (row >= 2 * n1) + (row >= 3 * n1);
              const int b1 = row - k * n1;
              const double v = (double)mid[m][t][r] * (double)ubc * (double)inv[0][b1];
              double* p = pbase + (int64_t)(k * nb + o1 + b1) * gcols + gj;
              *p = first ? v : *p + v;
            }
          }
          // one row tile at a time: keeps the read-modify-writes from being
          // gathered into one long-lived batch of registers
          __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) mid[m][t] = f4{0.f, 0.f, 0.f, 0.f};
    }
  };

  const int nchunks = (ncent + PKC - 1) / PKC;
  __syncthreads();                 // scales and zero rows visible
  if (ncent > 0) {                 // uniform: an empty slice only writes zeros
    issue(0);
    commit(0, 0);
  }
  __syncthreads();
  bool first = true;
  for (int ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunks;
    if (more) issue((ch + 1) * PKC);
    compute(std::integral_constant<int, NT>{}, buf);
    if ((ch & 15) == 15 || !more) {      // every 512 centres: fp32 block into the running sum
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          mid[m][t] += acc[m][t];
          acc[m][t] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    if ((ch + 1) % (PAIR_SUB / PKC) == 0 || !more) {   // every 8192 centres: into binary64
      flush(first);
      first = false;
    }
    if (more) commit((ch + 1) * PKC, buf ^ 1);
    __syncthreads();
  }
  if (first) flush(true);          // empty slice: zeros
}

// ---------------------------------------------------------------------------
// binary64: the same work items on v_mfma_f64_16x16x4_f64, no operand split,
// no scaling, binary64 accumulation over the whole slice.  K-step = 2 centres
// x (re, im): lane L holds k = L / 16, i.e. centre 2 ks + k / 2, part k % 2.
// The left operand y = x A is staged as complex values and each lane builds
// its [y_r, -y_i] / [y_i, y_r] entry; the right operand entry is the real or
// imaginary part of B(b2) C(b3) for the lane's column.
// ---------------------------------------------------------------------------
struct cd {
  double r, i;
};
typedef double d4 __attribute__((ext_vector_type(4)));

template <int NBLK, int NBC>
__global__ __launch_bounds__(64 * pair_waves(NBLK, NBC)) void contract_pair_f64_kernel(PairArgs a) {
  constexpr int MT = pair_mt(NBLK, NBC);
  constexpr int W = pair_waves(NBLK, NBC);
  constexpr int NT = pair_nt(NBLK, NBC);
  constexpr int NTH = 64 * W;
  constexpr int BS = PKC + 1;
  static_assert(NBC * PKC / 2 <= NTH, "one B/C centre pair per thread");
  static_assert(NBLK * NBC * 8 <= NTH, "one left-operand unit per thread");
  const int nb = a.nb, n = a.nmax;
  const Layout L = make_layout(n);
  int bx, by;
  xcd_contiguous(bx, by);
  const PairItem it = a.items[a.item0 + bx];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const BinRange br = bin_range(a);
  const int o1 = br.o1, o2 = br.o2, o3 = br.o3, n1 = br.n1, n2 = br.n2, n3 = br.n3;
  const int ncols = n2 * n3;
  const int ntiles = (ncols + 15) >> 4;
  const int mrows = NBLK * 2 * n1;
  const int per = (int)((((int64_t)a.ncent + gridDim.y - 1) / gridDim.y + PKC - 1) / PKC * PKC);
  const int cbase = by * per;
  const int ncent = imax(0, imin(a.ncent - cbase, per));
  const int64_t ldc = a.ldc;
  const double* rec = reinterpret_cast<const double*>(a.rec);

  __shared__ cd Bs[2][NBC][BS];
  __shared__ cd Cs[2][NBC][BS];
  __shared__ cd Ys[2][NBLK][NBC][BS];

  // staging slots: B / C pair of centres 2p, 2p+1 of bin sbin; left-operand
  // unit (block, b1, group of 4 centres)
  const int sbin = tid >> 4, spair = tid & 15;
  const bool sb_on = sbin < n2, sc_on = sbin < n3;
  const double* rowBp = rec + 2 * (((int64_t)rec_entry(L, it.famB, it.ordB) * nb + o2 + (sb_on ? sbin : 0)) * ldc);
  const double* rowCp = rec + 2 * (((int64_t)rec_entry(L, it.famC, it.ordC) * nb + o3 + (sc_on ? sbin : 0)) * ldc);
  const int ug = tid & 7, ub1 = (tid >> 3) % NBC, ublk = (tid >> 3) / NBC;
  const bool u_on = ublk < NBLK && ub1 < n1;
  PairRow rb = it.blk[0];
  if (NBLK > 1 && ublk == 1) rb = it.blk[1];
  const double* rowAp = rec + 2 * (((int64_t)rec_entry(L, rb.fam, rb.order) * nb + o1 + (u_on ? ub1 : 0)) * ldc);
  const bool xconj = rb.x == X_GC, aconj = rb.conj != 0;
  const bool x_is_w = it.blk[0].x == X_W;
  const double* xg = reinterpret_cast<const double*>(a.xg);
  const double* xw = reinterpret_cast<const double*>(a.xw);
  const int lastc = (int)ldc - 4;

  cd pb[2], pc[2], pa[4], px[4];
  auto issue = [&](int c0) {
    const int gp = imin(cbase + c0 + 2 * spair, (int)ldc - 2);
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      pb[v] = {rowBp[2 * ((int64_t)gp + v)], rowBp[2 * ((int64_t)gp + v) + 1]};
      pc[v] = {rowCp[2 * ((int64_t)gp + v)], rowCp[2 * ((int64_t)gp + v) + 1]};
    }
    const int gu = imin(cbase + c0 + 4 * ug, lastc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      pa[v] = {rowAp[2 * ((int64_t)gu + v)], rowAp[2 * ((int64_t)gu + v) + 1]};
      px[v] = x_is_w ? cd{xw[gu + v], 0.0} : cd{xg[2 * ((int64_t)gu + v)], xg[2 * ((int64_t)gu + v) + 1]};
    }
  };
  auto commit = [&](int c0, int buf) {
    if (sb_on || sc_on) {   // a row past n2 or n3 holds a clamped bin and is never read
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const bool live = c0 + 2 * spair + v < ncent;   // past the tile: stale memory, select zeros
        const double bi = it.conjB ? -pb[v].i : pb[v].i, ci = it.conjC ? -pc[v].i : pc[v].i;
        Bs[buf][sbin][2 * spair + v] = live ? cd{pb[v].r, bi} : cd{0.0, 0.0};
        Cs[buf][sbin][2 * spair + v] = live ? cd{pc[v].r, ci} : cd{0.0, 0.0};
      }
    }
    if (u_on) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool live = c0 + 4 * ug + v < ncent;
        const double xr = px[v].r, xi = xconj ? -px[v].i : px[v].i;
        const double ar = pa[v].r, ai = aconj ? -pa[v].i : pa[v].i;
        const cd y{xr * ar - xi * ai, xr * ai + xi * ar};
        Ys[buf][ublk][ub1][4 * ug + v] = live ? y : cd{0.0, 0.0};
      }
    }
  };

  const int wr = (wv + bx) % W;
  const int ntw = imin(NT, imax(0, (ntiles - wr + W - 1) / W));
  int b2c[NT], b3c[NT];
  bool colok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = 16 * (wr + W * t) + (lane & 15);
    colok[t] = t < ntw && j < ncols;
    b2c[t] = colok[t] ? j / n3 : 0;
    b3c[t] = colok[t] ? j % n3 : 0;
  }
  // this lane's left-operand row in each row tile: (block, re/im, b1)
  int rblk[MT], rb1[MT];
  bool rpart[MT], rok[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int r = 16 * m + (lane & 15);
    rok[m] = r < mrows;
    const int rr = rok[m] ? r : 0;
    rblk[m] = rr / (2 * n1);
    rpart[m] = (rr % (2 * n1)) >= n1;
    rb1[m] = rr % n1;
  }
  d4 acc[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[m][t] = d4{0.0, 0.0, 0.0, 0.0};

  const int kq = lane >> 4;
  const bool pk = kq & 1;
  const int nchunks = (ncent + PKC - 1) / PKC;
  if (ncent > 0) {
    issue(0);
    commit(0, 0);
  }
  __syncthreads();
  for (int ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunks;
    if (more) issue((ch + 1) * PKC);
#pragma unroll 4
    for (int ks = 0; ks < PKC / 2; ++ks) {
      const int cc = 2 * ks + (kq >> 1);
      double bv[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        const cd b = Bs[buf][b2c[t]][cc], c = Cs[buf][b3c[t]][cc];
        bv[t] = pk ? b.r * c.i + b.i * c.r : b.r * c.r - b.i * c.i;
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const cd y = Ys[buf][rblk[m]][rb1[m]][cc];
        // [y_r, -y_i] on real-output rows, [y_i, y_r] on imaginary-output rows
        double av = rpart[m] ? (pk ? y.r : y.i) : (pk ? -y.i : y.r);
        av = rok[m] ? av : 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[m][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv[t], acc[m][t], 0, 0, 0);
      }
    }
    if (more) commit((ch + 1) * PKC, buf ^ 1);
    __syncthreads();
  }
  // f64 D layout: element r of lane L is row 4 r + L / 16, column L % 16
  // the item's region spans all nb bins: tile row k n1 + b1 (k = 2 block +
  // re/im) sits at k nb + o1 + b1, tile column (b2, b3) at (o2 + b2) nb + o3 + b3
  const int64_t gcols = (int64_t)nb * nb;
  double* part = a.part + ((int64_t)by * a.total_rows + it.row0) * gcols;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (!colok[t]) continue;
    const int j = 16 * (wr + W * t) + (lane & 15);
    const int b2 = j / n3, b3 = j - b2 * n3;
    const int64_t gj = (int64_t)(o2 + b2) * nb + o3 + b3;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * m + 4 * r + (lane >> 4);
        if (row < mrows) {
          const int k = (row >= n1) + (row >= 2 * n1) + (row >= 3 * n1);
          part[(int64_t)(k * nb + o1 + row - k * n1) * gcols + gj] = acc[m][t][r];
        }
      }
  }
}

// part[0][e] = sum over the slices of part[k][e], in slice order (the
// contraction rewrites every slice it reads next time)
__global__ void pair_slice_sum_kernel(double* part, int nsl, int64_t slice_elems) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < slice_elems;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int k = 0; k < nsl; ++k) v += part[(int64_t)k * slice_elems + e];
    part[e] = v;
  }
}

// ups[mu][b1][b2][b3][n2][n3] += sum over slices of the item region that holds
// (mu, n2, n3), read at (b1, b2, b3) permuted into the item's roles
__global__ void pair_reduce_kernel(const double* part, int nsl, int64_t slice_elems, const PairItem* items,
                                   const PairOut* out, int nb, int nmax, double* ups) {
  const int nn = 2 * nmax + 1;
  const int64_t total = 2LL * FPCF4_NCORR * nb * nb * nb * nn * nn;
  // grid-stride: at 65 bins and nmax 15 there are 4.8e9 values, more
  // work-items than one dispatch dimension holds (2^32)
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(i & 1);
    int64_t r = i >> 1;
    const int n3i = (int)(r % nn); r /= nn;
    const int n2i = (int)(r % nn); r /= nn;
    const int b3 = (int)(r % nb); r /= nb;
    const int b2 = (int)(r % nb); r /= nb;
    const int b1 = (int)(r % nb); r /= nb;
    const int mu = (int)r;
    const PairOut po = out[((int64_t)mu * nn + n2i) * nn + n3i];
    // the bins of the item's row block and of its two column blocks
    const int s0 = po.perm & 3, s1 = (po.perm >> 2) & 3, s2 = (po.perm >> 4) & 3;
    const int c1 = s0 == 0 ? b1 : s0 == 1 ? b2 : b3;
    const int c2 = s1 == 0 ? b1 : s1 == 1 ? b2 : b3;
    const int c3 = s2 == 0 ? b1 : s2 == 1 ? b2 : b3;
    const int row = items[po.item].row0 + po.blk * 2 * nb + p * nb + c1;
    const int col = c2 * nb + c3;
    const int64_t src = (int64_t)row * nb * nb + col;
    double v = 0.0;
    for (int k = 0; k < nsl; ++k) v += part[(int64_t)k * slice_elems + src];
    ups[i] += v;
  }
}

template <int PREC, int NBLK, int NBC>
static void launch_cls(const PairArgs& a, int nsl, hipStream_t s) {
  const dim3 grid(a.nitems, nsl, a.nt * a.nt * a.nt), block(64 * pair_waves(NBLK, NBC));
  hipLaunchKernelGGL((contract_pair_kernel<PREC, NBLK, NBC>), grid, block, 0, s, a);
}

template <int PREC, int NBC>
static void launch_prec_nbc(const PairArgs& a, int nblk, int nsl, hipStream_t s) {
  if (nblk == 1) launch_cls<PREC, 1, NBC>(a, nsl, s);
  else launch_cls<PREC, 2, NBC>(a, nsl, s);
}

template <int NBC>
static void launch_f64_nbc(const PairArgs& a, int nblk, int nsl, hipStream_t s) {
  const dim3 grid(a.nitems, nsl, a.nt * a.nt * a.nt);
  if (nblk == 1)
    hipLaunchKernelGGL((contract_pair_f64_kernel<1, NBC>), grid, dim3(64 * pair_waves(1, NBC)), 0, s, a);
  else
    hipLaunchKernelGGL((contract_pair_f64_kernel<2, NBC>), grid, dim3(64 * pair_waves(2, NBC)), 0, s, a);
}

double pair_issued_flops(const PairPlanHost& pp, int nb, int64_t ncent, int precision) {
  const BinTiles bt = bin_tiles(nb);
  const int nbc = bt.tb <= 8 ? 8 : bt.tb <= 12 ? 12 : 16;
  double f = 0.0;
  for (int k = 1; k <= PAIR_MAX_BLK; ++k) {
    const int cols = 16 * pair_waves(k, nbc) * pair_nt(k, nbc);   // surplus tiles included
    // rows x columns x K (real, imaginary) x 2 flop (x 3 hi/lo products in the 16-bit paths)
    f += (double)pp.cls_count[k] * 16.0 * pair_mt(k, nbc) * cols * 2.0 * 2.0 *
         (precision == FPCF4_FP64 ? 1.0 : 3.0);
  }
  return f * (double)ncent * bt.nt * bt.nt * bt.nt;
}

double pair_useful_flops(const PairPlanHost& pp, int nb, int64_t ncent) {
  double blocks = 0.0;
  for (const PairItem& it : pp.items) blocks += it.nblk;
  return 8.0 * blocks * (double)nb * nb * nb * (double)ncent;
}

hipError_t launch_contract_pairs(const PairLaunch& pl, hipStream_t s) {
  if (pl.ncent <= 0) return hipSuccess;
  const int nsl = std::min(pair_slices(pl.ncent), std::max(1, pl.max_slices));
  const BinTiles bt = bin_tiles(pl.nb);
  for (int nblk = 1; nblk <= PAIR_MAX_BLK; ++nblk) {
    if (pl.cls_count[nblk] == 0) continue;
    PairArgs a{};
    a.rec = pl.rec;
    a.ldc = pl.ldc;
    a.xg = pl.xg;
    a.xw = pl.xw;
    a.maxima = pl.maxima;
    a.items = pl.items;
    a.item0 = pl.cls_start[nblk];
    a.nitems = pl.cls_count[nblk];
    a.ncent = pl.ncent;
    a.nb = pl.nb;
    a.nmax = pl.nmax;
    a.tb = bt.tb;
    a.nt = bt.nt;
    a.part = pl.part;
    a.total_rows = pl.total_rows;
    // kernel class by the bins per tile
    if (pl.precision == FPCF4_FP64) {
      if (bt.tb <= 8) launch_f64_nbc<8>(a, nblk, nsl, s);
      else if (bt.tb <= 12) launch_f64_nbc<12>(a, nblk, nsl, s);
      else launch_f64_nbc<16>(a, nblk, nsl, s);
    } else if (bt.tb <= 8) {
      if (pl.precision == FPCF4_MIXED_FP16) launch_prec_nbc<FPCF4_MIXED_FP16, 8>(a, nblk, nsl, s);
      else launch_prec_nbc<FPCF4_MIXED_BF16, 8>(a, nblk, nsl, s);
    } else if (bt.tb <= 12) {
      if (pl.precision == FPCF4_MIXED_FP16) launch_prec_nbc<FPCF4_MIXED_FP16, 12>(a, nblk, nsl, s);
      else launch_prec_nbc<FPCF4_MIXED_BF16, 12>(a, nblk, nsl, s);
    } else {
      if (pl.precision == FPCF4_MIXED_FP16) launch_prec_nbc<FPCF4_MIXED_FP16, 16>(a, nblk, nsl, s);
      else launch_prec_nbc<FPCF4_MIXED_BF16, 16>(a, nblk, nsl, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int nn = 2 * pl.nmax + 1;
  const int64_t slice_elems = pl.total_rows * pl.nb * pl.nb;
  if (nsl > 1) {
    const int64_t sblocks = std::min<int64_t>((slice_elems + 255) / 256, 1 << 16);
    hipLaunchKernelGGL(pair_slice_sum_kernel, dim3((unsigned)sblocks), dim3(256), 0, s, pl.part, nsl,
                       slice_elems);
  }
  const int64_t total = 2LL * FPCF4_NCORR * pl.nb * pl.nb * pl.nb * nn * nn;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(pair_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, pl.part, 1, slice_elems,
                     pl.items, pl.out, pl.nb, pl.nmax, pl.ups);
  return hipGetLastError();
}

}  // namespace fpcf4
