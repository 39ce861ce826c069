// Stage (b) of the mixed-precision paths on the matrix cores, organised by
// the pair of blocks at Theta_2 and Theta_3 (Sect. 3.1):
//
//   Upsilon_mu[b1,b2,b3; n2,n3] = sum_i (x A)_i(b1) * B_i(b2) C_i(b3),
//
// with x the centre factor, A the block at Theta_1 (order depending on
// n2 + n3), B and C the blocks at Theta_2 and Theta_3 (orders depending on n2
// and n3).  The contraction is a GEMM over the centre index whose right
// operand, the Khatri-Rao product R(b2,b3) = B(b2) C(b3), has to be formed on
// the vector ALUs; the left operand y(b1) = x A(b1) is a per-centre vector.
//
// Many (mu, n2, n3) share the same R: the factor table of Sect. 3.1 uses only
// G_k (plain or conjugated) and W_k, so every B C product is one of a few
// kinds of block pairs with two orders, e.g. G_p(b2) G_q(b3) is the R of
// mu = 0, 2 at (n2, n3) = (-p-2, -q-3) and of mu = 1, 5 at (-p-2, -q-1).
// The Theta_2 <-> Theta_3 relation of Table 2 (the (Theta_1, Theta_3,
// Theta_2) column) is the same statement for the transposed pair:
// G_p(b2) G_q(b3) = G_q(b3) G_p(b2) read with b2 and b3 exchanged.  The host
// plan (make_pair_plan) therefore lists every distinct unordered pair of
// (family, conjugation, order) once as a work item; its rows are the distinct
// left factors (x kind, A family, A conjugation, A order) of every (mu, n2,
// n3) that uses the pair, in either orientation; and an output map sends each
// (mu, n2, n3) to (item, row block, transposed).  At nmax = 10 this forms
// 1029 pairs instead of 7 * 441 and issues half the MFMA work of one GEMM
// per (mu group, n2, n3).
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
// same lanes read back what they wrote).  pair_reduce_kernel adds the slices
// in order and scatters every (mu, n2, n3) from its item and orientation into
// the output tensor.  No atomics: the result is deterministic.
#include <map>
#include <tuple>
#include <vector>

#include "factors.hpp"
#include "fpcf4_internal.hpp"

namespace fpcf4 {

// ---------------------------------------------------------------------------
// host: the plan
// ---------------------------------------------------------------------------
PairPlanHost make_pair_plan(int nmax, int nb) {
  typedef std::tuple<int, int, int> Spec;            // family, conj, order
  typedef std::tuple<int, int, int, int> RowKey;     // x kind, A family, A conj, A order
  struct Tgt { int mu, n2, n3, tr; };
  std::map<std::pair<Spec, Spec>, std::map<RowKey, std::vector<Tgt>>> items;
  for (int mu = 0; mu < FPCF4_NCORR; ++mu) {
    const MuFactors F = mu_factors(mu);
    for (int n2 = -nmax; n2 <= nmax; ++n2)
      for (int n3 = -nmax; n3 <= nmax; ++n3) {
        const Spec sb{F.B.fam, F.B.conj, F.B.a * n2 + F.B.b * n3 + F.B.c};
        const Spec sc{F.C.fam, F.C.conj, F.C.a * n2 + F.C.b * n3 + F.C.c};
        const bool tr = sc < sb;
        const std::pair<Spec, Spec> key = tr ? std::make_pair(sc, sb) : std::make_pair(sb, sc);
        const RowKey rk{F.x, F.A.fam, F.A.conj, F.A.a * n2 + F.A.b * n3 + F.A.c};
        items[key][rk].push_back({mu, n2, n3, tr ? 1 : 0});
      }
  }
  PairPlanHost P;
  const int nn = 2 * nmax + 1;
  P.out.assign((size_t)FPCF4_NCORR * nn * nn, PairOut{-1, 0, 0, 0});
  for (int c = 0; c <= PAIR_MAX_BLK; ++c) P.cls_start[c] = P.cls_count[c] = 0;
  // items grouped by their number of row blocks (one kernel per class)
  int64_t rows = 0;
  for (int nbk = 1; nbk <= PAIR_MAX_BLK; ++nbk) {
    P.cls_start[nbk] = (int)P.items.size();
    for (const auto& kv : items) {
      if ((int)kv.second.size() != nbk) continue;
      PairItem it{};
      it.famB = (int8_t)std::get<0>(kv.first.first);
      it.conjB = (int8_t)std::get<1>(kv.first.first);
      it.ordB = std::get<2>(kv.first.first);
      it.famC = (int8_t)std::get<0>(kv.first.second);
      it.conjC = (int8_t)std::get<1>(kv.first.second);
      it.ordC = std::get<2>(kv.first.second);
      it.nblk = nbk;
      it.row0 = (int32_t)rows;
      int k = 0;
      for (const auto& rv : kv.second) {
        it.blk[k].x = (int8_t)std::get<0>(rv.first);
        it.blk[k].fam = (int8_t)std::get<1>(rv.first);
        it.blk[k].conj = (int8_t)std::get<2>(rv.first);
        it.blk[k].order = std::get<3>(rv.first);
        for (const Tgt& t : rv.second)
          P.out[((size_t)t.mu * nn + (t.n2 + nmax)) * nn + (t.n3 + nmax)] =
              PairOut{(int32_t)P.items.size(), k, t.tr, 0};
        ++k;
      }
      rows += (int64_t)nbk * 2 * nb;
      P.items.push_back(it);
    }
    P.cls_count[nbk] = (int)P.items.size() - P.cls_start[nbk];
  }
  P.total_rows = rows;
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
  return nbc == 8 ? 2 : nbc == 12 ? 3 : (pair_mt(nblk, nbc) > 4 ? 8 : 4);
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

template <int PREC, int NBLK, int NBC>
__global__ __launch_bounds__(64 * pair_waves(NBLK, NBC)) void contract_pair_kernel(PairArgs a) {
  typedef typename H8of<PREC>::type H8;
  constexpr int MT = pair_mt(NBLK, NBC);
  constexpr int W = pair_waves(NBLK, NBC);
  constexpr int NT = pair_nt(NBLK, NBC);
  constexpr int NTH = 64 * W;
  constexpr int NXS = (NBC * PKC + NTH - 1) / NTH;              // B/C (bin, centre) slots per thread
  constexpr int NRU = (NBLK * NBC * PKS * 4 + NTH - 1) / NTH;   // left-operand units per thread
  const int nb = a.nb, n = a.nmax;
  const Layout L = make_layout(n);
  int bx, by;
  xcd_contiguous(bx, by);
  const PairItem it = a.items[a.item0 + bx];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ncols = nb * nb;
  const int ntiles = (ncols + 15) >> 4;
  const int mrows = NBLK * 2 * nb;
  // centres [cbase, cbase + ncent) of this slice
  const int per = (int)(((int64_t)a.ncent + gridDim.y - 1) / gridDim.y + PKC - 1) / PKC * PKC;
  const int cbase = by * per;
  const int ncent = imax(0, imin(a.ncent - cbase, per));
  const float* rec = a.rec + 2 * (int64_t)cbase;
  const int64_t ldc = a.ldc;
  const int rowB = rec_entry(L, it.famB, it.ordB);
  const int rowC = rec_entry(L, it.famC, it.ordC);

  __shared__ cf Bs[2][NBC][PKC + 1];
  __shared__ cf Cs[2][NBC][PKC + 1];
  __shared__ H8 Ys[2][PKS][MT][2][64];    // left operand in MFMA lane order, hi / lo
  __shared__ float scl[3][16];            // scales of y (per b1), B (per b2), C (per b3)

  if (tid < 16) {
    const unsigned* M = a.maxima;
    float sy = 1.0f, sb = 1.0f, sc = 1.0f;
    if (tid < nb) {
      const int famA = it.blk[0].fam == F_G ? 0 : 16;
      const float mx = __uint_as_float(M[it.blk[0].x == X_W ? 33 : 32]);
      // y = x A below 2^14 per component, B and C below 2^6: R = B C below 2^13
      sy = pow2_under(2.0f * mx * __uint_as_float(M[famA + tid]), 14);
      sb = pow2_under(1.5f * __uint_as_float(M[(it.famB == F_G ? 0 : 16) + tid]), 6);
      sc = pow2_under(1.5f * __uint_as_float(M[(it.famC == F_G ? 0 : 16) + tid]), 6);
    }
    scl[0][tid] = sy;
    scl[1][tid] = sb;
    scl[2][tid] = sc;
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

  // ---- this thread's staging slots
  // B / C: slot s -> (bin s / 32, centre s % 32)
  // left operand: unit u -> (block, b1, K-step, lane group q): four centres
  //   16 ks + 4 q + (0..3) of row (block, b1); writes the real-output and the
  //   imaginary-output rows of that b1.
  // All units of a thread share (K-step, lane group) (NTH is a multiple of 8),
  // so they share the four centres and their centre factor.
  const int ru_q = tid & 3, ru_ks = (tid >> 2) % PKS;
  int ru_blk[NRU], ru_b1[NRU], ru_rowA[NRU], ru_xc[NRU], ru_ac[NRU];
  bool ru_on[NRU];
#pragma unroll
  for (int h = 0; h < NRU; ++h) {
    const int u = tid + NTH * h;
    const int b1 = (u / (4 * PKS)) % NBC, blk = u / (4 * PKS * NBC);
    ru_on[h] = blk < NBLK && b1 < nb;
    ru_blk[h] = ru_on[h] ? blk : 0;
    ru_b1[h] = ru_on[h] ? b1 : 0;
    // the block's fields selected without a dynamic index into the item
    PairRow rb = it.blk[0];
#pragma unroll
    for (int k = 1; k < NBLK; ++k)
      if (ru_blk[h] == k) rb = it.blk[k];
    ru_rowA[h] = ru_on[h] ? rec_entry(L, rb.fam, rb.order) : 0;
    ru_xc[h] = rb.x == X_GC;
    ru_ac[h] = rb.conj;
  }
  const bool x_is_w = it.blk[0].x == X_W;   // the W items use w; all others w g
  struct Pf {
    cf bv[NXS], cv[NXS];
    cf av[NRU][4], xv[4];
  } pf;
  auto issue = [&](int c0) {
#pragma unroll
    for (int h = 0; h < NXS; ++h) {
      const int s = tid + NTH * h;
      const int b = s / PKC, c = c0 + s % PKC;
      const int bl = b < nb ? b : nb - 1, cl = c < ncent ? c : ncent - 1;
      const float* pb = rec + 2 * (((int64_t)rowB * nb + bl) * ldc + cl);
      const float* pc = rec + 2 * (((int64_t)rowC * nb + bl) * ldc + cl);
      pf.bv[h] = {pb[0], pb[1]};
      pf.cv[h] = {pc[0], pc[1]};
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int c = c0 + 16 * ru_ks + 4 * ru_q + v;
      const int cl = c < ncent ? c : ncent - 1;
      if (x_is_w) pf.xv[v] = {a.xw[cbase + cl], 0.0f};
      else pf.xv[v] = {a.xg[2 * (int64_t)(cbase + cl)], a.xg[2 * (int64_t)(cbase + cl) + 1]};
#pragma unroll
      for (int h = 0; h < NRU; ++h) {
        const float* pa = rec + 2 * (((int64_t)ru_rowA[h] * nb + ru_b1[h]) * ldc + cl);
        pf.av[h][v] = {pa[0], pa[1]};
      }
    }
  };
  auto commit = [&](int c0, int buf) {
#pragma unroll
    for (int h = 0; h < NXS; ++h) {
      const int s = tid + NTH * h;
      const int b = s / PKC, cc = s % PKC;
      if (b < nb) {
        const bool live = c0 + cc < ncent;
        const float sb = live ? scl[1][b] : 0.0f, sc = live ? scl[2][b] : 0.0f;
        const float bi = it.conjB ? -pf.bv[h].i : pf.bv[h].i;
        const float ci = it.conjC ? -pf.cv[h].i : pf.cv[h].i;
        Bs[buf][b][cc] = {pf.bv[h].r * sb, bi * sb};
        Cs[buf][b][cc] = {pf.cv[h].r * sc, ci * sc};
      }
    }
#pragma unroll
    for (int h = 0; h < NRU; ++h) {
      if (!ru_on[h]) continue;
      const int blk = ru_blk[h], b1 = ru_b1[h], ks = ru_ks, q = ru_q;
      const float sy = scl[0][b1];
      float vr[8], vi[8];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool live = c0 + 16 * ks + 4 * q + v < ncent;
        cf x = pf.xv[v], A = pf.av[h][v];
        if (ru_xc[h]) x.i = -x.i;
        if (ru_ac[h]) A.i = -A.i;
        // explicit fused forms: the rounding does not depend on how the
        // compiler would contract the expression
        float yr = __builtin_fmaf(x.r, A.r, -(x.i * A.i));
        float yi = __builtin_fmaf(x.r, A.i, x.i * A.r);
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
      const int r_re = blk * 2 * nb + b1, r_im = r_re + nb;
      Ys[buf][ks][r_re >> 4][0][16 * q + (r_re & 15)] = hr;
      Ys[buf][ks][r_re >> 4][1][16 * q + (r_re & 15)] = lr;
      Ys[buf][ks][r_im >> 4][0][16 * q + (r_im & 15)] = hi;
      Ys[buf][ks][r_im >> 4][1][16 * q + (r_im & 15)] = li;
    }
  };

  // this wave's column tiles T = wr + W t; the wave holding one more tile
  // rotates with the item so co-resident workgroups differ
  const int wr = (wv + bx) % W;
  int b2c[NT], b3c[NT];
  bool colok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int j = 16 * (wr + W * t) + (lane & 15);
    colok[t] = j < ncols;
    b2c[t] = colok[t] ? j / nb : 0;
    b3c[t] = colok[t] ? j % nb : 0;
  }

  f4 acc[MT][NT], mid[MT][NT];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      acc[m][t] = f4{0.f, 0.f, 0.f, 0.f};
      mid[m][t] = f4{0.f, 0.f, 0.f, 0.f};
    }

  // write (first == true) or add the running sum, unscaled, into this
  // workgroup's region of the slice partial buffer, then clear it
  double* part = a.part + ((int64_t)by * a.total_rows + it.row0) * ncols;
  auto flush = [&](bool first) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (!colok[t]) continue;
      const int j = 16 * (wr + W * t) + (lane & 15);
      const double ubc = 1.0 / ((double)scl[1][b2c[t]] * (double)scl[2][b3c[t]]);
#pragma unroll
      for (int m = 0; m < MT; ++m) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * m + 4 * (lane >> 4) + r;
          if (row < mrows) {
            const double v = (double)mid[m][t][r] * (ubc / (double)scl[0][row % nb]);
            double* p = part + (int64_t)row * ncols + j;
            *p = first ? v : *p + v;
          }
        }
        mid[m][t] = f4{0.f, 0.f, 0.f, 0.f};
      }
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
#pragma unroll
    for (int ks = 0; ks < PKS; ++ks) {
      const int cb = 16 * ks + 4 * (lane >> 4);
      H8 rh[NT], rl[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const cf bv = Bs[buf][b2c[t]][cb + u];
          const cf cv = Cs[buf][b3c[t]][cb + u];
          v[2 * u] = __builtin_fmaf(bv.r, cv.r, -(bv.i * cv.i));
          v[2 * u + 1] = __builtin_fmaf(bv.r, cv.i, bv.i * cv.r);
        }
        split8<PREC>(v, rh[t], rl[t]);
      }
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const H8 yh = Ys[buf][ks][m][0][lane];
        const H8 yl = Ys[buf][ks][m][1][lane];
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (wr + W * t < ntiles) acc[m][t] = mma<PREC>(yh, rh[t], acc[m][t]);
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (wr + W * t < ntiles) acc[m][t] = mma<PREC>(yh, rl[t], acc[m][t]);
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (wr + W * t < ntiles) acc[m][t] = mma<PREC>(yl, rh[t], acc[m][t]);
      }
    }
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

// ups[mu][b1][b2][b3][n2][n3] += sum over slices of the item region that holds
// (mu, n2, n3), read transposed in (b2, b3) where the plan says so
__global__ void pair_reduce_kernel(const double* part, int nsl, int64_t slice_elems, const PairItem* items,
                                   const PairOut* out, int nb, int nmax, double* ups) {
  const int nn = 2 * nmax + 1;
  const int64_t total = 2LL * FPCF4_NCORR * nb * nb * nb * nn * nn;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int p = (int)(i & 1);
  int64_t r = i >> 1;
  const int n3i = (int)(r % nn); r /= nn;
  const int n2i = (int)(r % nn); r /= nn;
  const int b3 = (int)(r % nb); r /= nb;
  const int b2 = (int)(r % nb); r /= nb;
  const int b1 = (int)(r % nb); r /= nb;
  const int mu = (int)r;
  const PairOut po = out[((int64_t)mu * nn + n2i) * nn + n3i];
  const int row = items[po.item].row0 + po.blk * 2 * nb + p * nb + b1;
  const int col = po.transposed ? b3 * nb + b2 : b2 * nb + b3;
  const int64_t src = (int64_t)row * nb * nb + col;
  double v = 0.0;
  for (int k = 0; k < nsl; ++k) v += part[(int64_t)k * slice_elems + src];
  ups[i] += v;
}

template <int PREC, int NBLK, int NBC>
static void launch_cls(const PairArgs& a, int nsl, hipStream_t s) {
  const dim3 grid(a.nitems, nsl), block(64 * pair_waves(NBLK, NBC));
  hipLaunchKernelGGL((contract_pair_kernel<PREC, NBLK, NBC>), grid, block, 0, s, a);
}

template <int PREC, int NBC>
static void launch_prec_nbc(const PairArgs& a, int nblk, int nsl, hipStream_t s) {
  switch (nblk) {
    case 1: launch_cls<PREC, 1, NBC>(a, nsl, s); break;
    case 2: launch_cls<PREC, 2, NBC>(a, nsl, s); break;
    case 3: launch_cls<PREC, 3, NBC>(a, nsl, s); break;
    default: launch_cls<PREC, 4, NBC>(a, nsl, s); break;
  }
}

hipError_t launch_contract_pairs(const PairLaunch& pl, hipStream_t s) {
  if (pl.ncent <= 0) return hipSuccess;
  const int nsl = pair_slices(pl.ncent);
  for (int nblk = 1; nblk <= PAIR_MAX_BLK; ++nblk) {
    if (pl.cls_count[nblk] == 0) continue;
    PairArgs a{};
    a.rec = reinterpret_cast<const float*>(pl.rec);
    a.ldc = pl.ldc;
    a.xg = reinterpret_cast<const float*>(pl.xg);
    a.xw = reinterpret_cast<const float*>(pl.xw);
    a.maxima = pl.maxima;
    a.items = pl.items;
    a.item0 = pl.cls_start[nblk];
    a.nitems = pl.cls_count[nblk];
    a.ncent = pl.ncent;
    a.nb = pl.nb;
    a.nmax = pl.nmax;
    a.part = pl.part;
    a.total_rows = pl.total_rows;
    if (pl.nb <= 8) {
      if (pl.precision == FPCF4_MIXED_FP16) launch_prec_nbc<FPCF4_MIXED_FP16, 8>(a, nblk, nsl, s);
      else launch_prec_nbc<FPCF4_MIXED_BF16, 8>(a, nblk, nsl, s);
    } else if (pl.nb <= 12) {
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
  const int64_t total = 2LL * FPCF4_NCORR * pl.nb * pl.nb * pl.nb * nn * nn;
  hipLaunchKernelGGL(pair_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, pl.part, nsl,
                     pl.total_rows * pl.nb * pl.nb, pl.items, pl.out, pl.nb, pl.nmax, pl.ups);
  return hipGetLastError();
}

}  // namespace fpcf4
