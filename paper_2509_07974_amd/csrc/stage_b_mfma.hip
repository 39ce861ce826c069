// Stage (b) on the matrix cores: contraction of three per-centre blocks into
// the 4PCF multipoles (Sect. 3.1)
//
//   Upsilon_mu[b1,b2,b3; n2,n3] = sum_i X[i,b1] Y[i,b2] Z[i,b3],
//   X = x_i A^mu(b1, n2+n3),  Y = B^mu(b2, n2),  Z = C^mu(b3, n3).
//
// For fixed (mu, n2, n3) this is a GEMM over the centre index i:
//   Out[(mu, b2), (b1, b3)] = sum_i Y[i, b2] * R[i, (b1, b3)],  R = X (x) Z,
// i.e. Y is the left operand and the Khatri-Rao product R (formed on the
// fly) the right one.  Correlators that share (x, A, C) share R and are
// stacked as extra rows (mu 0 and 3; mu 1 and 6), so 7 formations serve 9
// correlators.  Complex arithmetic is split into real MFMAs:
//   [Out_r; Out_i] = [[Y_r, -Y_i], [Y_i, Y_r]] [R_r; R_i]
// (rows: (mu, re/im, b2); columns: (b1, b3) packed densely; K: (centre,
// re/im)).
//
// Mixed precision (FP16 / BF16): every operand v is split v = hi + lo with
// hi, lo in the 16-bit format and v_mfma_f32_16x16x32_{f16,bf16} forms
// hi*hi + hi*lo + lo*hi with fp32 accumulation.  Operands are pre-scaled by
// per-bin powers of two (from the tile's maxima) so the fp16 range is never
// exceeded; the scale is undone exactly.  The fp32 accumulators are folded
// into binary64 registers every 512 centres and the binary64 sums are added
// to the output in a fixed order (deterministic, no atomics).
//
// Binary64: the same GEMM with v_mfma_f64_16x16x4_f64, no split, no scale.
//
// Work decomposition: one workgroup of 4 waves per (correlator group, n2,
// n3); the waves share the LDS-staged chunk of 32 centres (X, Z, and the
// split Y operand) and take disjoint (b1, b3) column tiles.  The global loads
// of chunk k+1 are issued into registers before the MFMAs of chunk k and
// committed to the other LDS buffer after them.
//
// The split Y operand depends on (n2, centre) only, so in the mixed paths it
// is formed once per group by yprep_kernel (conjugated, scaled, split into
// hi/lo and laid out in MFMA lane order for every 32-centre chunk) instead
// of once per (n2, n3) workgroup; the contraction copies it into LDS.  The
// mixed paths also carry the centre factor x on that operand (Y = x B, X = A),
// which moves the complex product x A out of the (n2, n3) workgroups.
#include "factors.hpp"
#include "fpcf4_internal.hpp"

namespace fpcf4 {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 bh8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

struct Group {
  int nmu;
  int mu[2];
};
__host__ __device__ constexpr Group group_of(int g) {
  return g == 0 ? Group{2, {0, 3}}
       : g == 1 ? Group{2, {1, 6}}
       : g == 2 ? Group{1, {2, 2}}
       : g == 3 ? Group{1, {4, 4}}
       : g == 4 ? Group{1, {5, 5}}
       : g == 5 ? Group{1, {7, 7}}
                : Group{1, {8, 8}};
}
constexpr int NGROUPS = 7;
__host__ __device__ constexpr bool same_fac(const Fac& a, const Fac& b) {
  return a.fam == b.fam && a.conj == b.conj && a.a == b.a && a.b == b.b && a.c == b.c;
}
// correlators stacked in a group must share the centre factor, A and C
static_assert(mu_factors(0).x == mu_factors(3).x && same_fac(mu_factors(0).A, mu_factors(3).A) &&
                  same_fac(mu_factors(0).C, mu_factors(3).C),
              "mu 0/3 must share x, A, C");
static_assert(mu_factors(1).x == mu_factors(6).x && same_fac(mu_factors(1).A, mu_factors(6).A) &&
                  same_fac(mu_factors(1).C, mu_factors(6).C),
              "mu 1/6 must share x, A, C");

constexpr int KC = 32;       // centres per LDS chunk (two fp16 MFMA K-steps)

// row tiles (16 rows of (mu, re/im, b2)), waves per workgroup and column
// tiles per wave (16 columns of (b1, b3), tile T = wave + WB t) for a
// bin-count class NBC in {8, 12, 16}.  A wave skips a whole column tile
// past the used ones (a wave-uniform branch); inside a tile the MFMA
// sequence is straight-line.
__host__ __device__ constexpr int mt_of(int nmu, int nbc) { return (nmu * 2 * nbc + 15) / 16; }
__host__ __device__ constexpr int wb_of(int nbc) { return nbc == 16 ? 8 : 4; }
__host__ __device__ constexpr int ntw_of(int nbc) {
  return ((nbc * nbc + 15) / 16 + wb_of(nbc) - 1) / wb_of(nbc);
}

__device__ __forceinline__ int fac_entry_k(const Layout& L, const Fac& f, int k) {
  return f.fam == F_G ? eG(L, k) : eW(L, k);
}

template <typename T>
struct C2 {
  T r, i;
};

template <typename T>
__device__ __forceinline__ C2<T> ldrec(const T* rec, int64_t row, int64_t ldc, int c) {
  const T* p = rec + 2 * (row * ldc + c);
  return {p[0], p[1]};
}

// maxima used for the fp16 scaling (set by stage (a)): [0..15] G per bin,
// [16..31] W per bin, [32] |x| for w g, [33] w; stored as float bits.
__device__ __forceinline__ float pow2_below(float m, int target_exp) {
  if (!(m > 0.0f)) return 1.0f;
  int e;
  frexpf(m, &e);                  // m < 2^e
  return ldexpf(1.0f, target_exp - e);
}

template <int PREC>
struct Half8;
template <>
struct Half8<FPCF4_MIXED_FP16> {
  typedef h8 type;
};
template <>
struct Half8<FPCF4_MIXED_BF16> {
  typedef bh8 type;
};

typedef __fp16 h2 __attribute__((ext_vector_type(2)));

// lo = fp16(v - hi) for a packed pair: v_fma_mix{lo,hi}_f16 form v*1 - hi
// with hi read as fp16 from its half of the packed register (exact in
// binary32, since hi is v truncated) and round the result to fp16 into the
// low / high half of the destination.  The compiler does not select these
// from plain code when binary32 denormals are enabled; only the fp16 result
// of a tiny lo could differ, and lo only refines hi.
__device__ __forceinline__ h2 split_lo2(float x0, float x1, h2 hh) {
  h2 lo;
  asm("v_fma_mixlo_f16 %0, %1, 1.0, -%3 op_sel_hi:[0,0,1]\n\t"
      "v_fma_mixhi_f16 %0, %2, 1.0, -%3 op_sel:[0,0,1] op_sel_hi:[0,0,1]"
      : "=&v"(lo)
      : "v"(x0), "v"(x1), "v"(hh));
  return lo;
}

template <int PREC>
__device__ __forceinline__ void split8v(const float (&v)[8], typename Half8<PREC>::type& hi,
                                        typename Half8<PREC>::type& lo) {
  if constexpr (PREC == FPCF4_MIXED_FP16) {
    // hi = v rounded toward zero to fp16 (two per instruction); lo = fp16(v - hi)
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
      const h2 hh = __builtin_amdgcn_cvt_pkrtz(v[q], v[q + 1]);
      const h2 ll = split_lo2(v[q], v[q + 1], hh);
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
__device__ __forceinline__ f4 mfma16(const typename Half8<PREC>::type& a,
                                     const typename Half8<PREC>::type& b, f4 c) {
  if constexpr (PREC == FPCF4_MIXED_FP16)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

struct BArgs {
  StageBArgs s;
  int ldc;                 // centre stride of the record rows
  const void* xg;          // per tile centre: complex (w g) in record precision
  const void* xw;          // per tile centre: w
  const unsigned* maxima;  // scaling maxima (mixed only)
  void* yprep;             // mixed only: split Y operand of the group (yprep_kernel)
};

typedef unsigned u4 __attribute__((ext_vector_type(4)));   // 16 bytes: one H8

// Mixed paths: the split Y operand of one correlator group, for every n2 and
// every 32-centre chunk of the tile, in the order the contraction stages it:
// [n2 + nmax][chunk][K-step][row tile][hi, lo][lane] of 8 16-bit values.
// Entry (ks, m, lane) holds row r = 16 m + lane % 16 of (mu, re/im, b2) and
// centres 16 ks + 4 (lane / 16) + (0..3) of the chunk, as
// [ y_r, -y_i ] (real-output rows) or [ y_i, y_r ] (imaginary-output rows)
// per centre, y = x B^mu(b2, n2) (x the centre factor, both conjugated where
// the factor table says so) times the power-of-two scale of b2; rows past the
// used ones and centres past the tile are zero.
__host__ __device__ constexpr int yprep_slots(int nmu, int nbc) { return (KC / 16) * mt_of(nmu, nbc) * 64; }
inline size_t yprep_bytes_for(int nbc, int nmax, int64_t ncent) {
  const int64_t nchunk = (ncent + KC - 1) / KC;
  return (size_t)(2 * nmax + 1) * (size_t)nchunk * yprep_slots(2, nbc) * 2 * 16;
}

// Values a thread stages for one chunk: X and Z for NXS (bin, centre) slots
// and the split Y operand of NYS (K-step, row tile, lane) slots, held in
// registers across the compute of the previous chunk (software pipelining).
template <typename T, int NXS, int NYS>
struct PrefetchP {
  C2<T> av[NXS], cv[NXS];
  u4 yh[NYS], yl[NYS];
};

// Power-of-two operand scales of the mixed paths from the stage (a) maxima
// (component maxima per bin; [32] |w g|, [33] w): Y = x B is below
// 2 max|x| max|B| per component and is scaled below 2^14; X = A and Z = C
// are below 1.5 max per component and are scaled below 2^6, so that the
// Khatri-Rao products X Z stay below 2^13 (fp16 max 65504).
__device__ __forceinline__ float y_scale(const unsigned* M, int xkind, int famB, int b2) {
  const float mx = __uint_as_float(M[xkind == X_W ? 33 : 32]);
  return pow2_below(2.0f * mx * __uint_as_float(M[famB + b2]), 14);
}
__device__ __forceinline__ float xz_scale(const unsigned* M, int fam, int b) {
  return pow2_below(1.5f * __uint_as_float(M[fam + b]), 6);
}

template <int PREC, int G, int NBC>
__global__ __launch_bounds__(256) void yprep_kernel(BArgs a) {
  typedef typename Half8<PREC>::type H8;
  constexpr Group GR = group_of(G);
  constexpr MuFactors F0 = mu_factors(GR.mu[0]);
  constexpr MuFactors F1 = mu_factors(GR.mu[1]);
  constexpr int MT = mt_of(GR.nmu, NBC);
  constexpr int NQ = yprep_slots(GR.nmu, NBC);
  constexpr int NQX = yprep_slots(2, NBC);        // slot stride of the buffer (largest group)
  const int nb = a.s.nb, n = a.s.nmax, nn = 2 * n + 1;
  const int ncent = a.s.ncent;
  const int64_t nchunk = (ncent + KC - 1) / KC;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nn * nchunk * NQ) return;
  const int q = (int)(t % NQ);
  const int64_t r1 = t / NQ;
  const int64_t ch = r1 % nchunk;
  const int n2i = (int)(r1 / nchunk);
  const int n2 = n2i - n;
  const Layout L = make_layout(n);
  const int rowB0 = fac_entry_k(L, F0.B, F0.B.a * n2 + F0.B.c);
  const int rowB1 = fac_entry_k(L, F1.B, F1.B.a * n2 + F1.B.c);
  constexpr int famB = F0.B.fam == F_G ? 0 : 16;
  const int ks = q / (MT * 64), m = (q / 64) % MT, l = q & 63;
  const int r = 16 * m + (l & 15);
  const int mrows = GR.nmu * 2 * nb;
  float v[8];
  if (r < mrows) {
    const int mi = r / (2 * nb), part = (r % (2 * nb)) / nb, b2 = r % nb;
    const int row = (mi ? rowB1 : rowB0) * nb + b2;
    const bool cj = mi ? F1.B.conj : F0.B.conj;
    const float sy = y_scale(a.maxima, F0.x, famB, b2);
    const float* rec = reinterpret_cast<const float*>(a.s.rec);
    const C2<float>* xg = reinterpret_cast<const C2<float>*>(a.xg);
    const float* xw = reinterpret_cast<const float*>(a.xw);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t c = ch * KC + 16 * ks + 4 * (l >> 4) + u;
      C2<float> y{0.f, 0.f};
      if (c < ncent) {
        C2<float> b = ldrec(rec, (int64_t)row, a.ldc, (int)c);
        C2<float> xc = F0.x == X_W ? C2<float>{xw[c], 0.f} : xg[c];
        if (cj) b.i = -b.i;
        if (F0.x == X_GC) xc.i = -xc.i;
        // explicit fused forms: the rounding does not depend on how the
        // compiler would contract the expression
        y = {__builtin_fmaf(xc.r, b.r, -(xc.i * b.i)), __builtin_fmaf(xc.r, b.i, xc.i * b.r)};
      }
      v[2 * u] = (part ? y.i : y.r) * sy;
      v[2 * u + 1] = (part ? y.r : -y.i) * sy;
    }
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = 0.f;
  }
  H8 hi, lo;
  split8v<PREC>(v, hi, lo);
  u4* out = reinterpret_cast<u4*>(a.yprep) + ((int64_t)n2i * nchunk + ch) * NQX * 2;
  const int e = (ks * MT + m) * 2 * 64 + l;
  out[e] = __builtin_bit_cast(u4, hi);
  out[e + 64] = __builtin_bit_cast(u4, lo);
}

// ---------------------------------------------------------------------------
// mixed precision
// ---------------------------------------------------------------------------
// Workgroups are dealt to the 8 XCDs round-robin in dispatch order (x
// fastest, then y).  The contraction kernels renumber them so that every
// XCD runs a contiguous range of (slice, n2, n3): the 2n+1 workgroups of one
// (slice, n2), which stage the same prepared Y chunks, then run on one XCD
// at the same time and share its L2.  A bijection of the grid onto itself.
__device__ __forceinline__ void xcd_block(int& bx, int& by) {
  const int gx = (int)gridDim.x, total = gx * (int)gridDim.y;
  const int lin = (int)blockIdx.y * gx + (int)blockIdx.x;
  const int per = total >> 3, rem = total & 7;
  const int x = lin & 7, i = lin >> 3;
  const int l = x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
  bx = l % gx;
  by = l / gx;
}

template <int PREC, int G, int NBC>
__global__ __launch_bounds__(512) void contract_mixed_kernel(BArgs a) {
  typedef typename Half8<PREC>::type H8;
  constexpr Group GR = group_of(G);
  constexpr MuFactors F0 = mu_factors(GR.mu[0]);
  constexpr MuFactors F1 = mu_factors(GR.mu[1]);
  constexpr int MT = mt_of(GR.nmu, NBC);
  constexpr int NTW = ntw_of(NBC);
  constexpr int KS = KC / 16;          // fp16 K-steps (16 centres) per chunk
  constexpr int WB = wb_of(NBC);       // waves per workgroup
  constexpr int NT = 64 * WB;
  constexpr int NXS = (NBC * KC + NT - 1) / NT;       // (bin, centre) staging slots per thread
  constexpr int NYS = (KS * MT * 64 + NT - 1) / NT;   // Y operand slots per thread
  const int nb = a.s.nb, n = a.s.nmax, nn = 2 * n + 1;
  const Layout L = make_layout(n);
  int bx, by;
  xcd_block(bx, by);
  const int lb = bx;
  const int n2 = lb / nn - n;
  const int n3 = lb % nn - n;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  // column tiles of this wave: T = wr + WB t.  When the tiles do not split
  // evenly, the wave holding one more is rotated with the block index, so
  // that co-resident workgroups put their longer waves on different SIMDs.
  const int wr = (wv + bx) & (WB - 1);
  const int mrows = GR.nmu * 2 * nb;
  const int ncols = nb * nb;
  const int ntiles = (ncols + 15) >> 4;
  // centre slice of this workgroup (by): centres [cbase, cbase + ncent)
  const int per = contract_slice_len(a.s.ncent, (int)gridDim.y);
  const int cbase = by * per;
  const int ncent = imax(0, imin(a.s.ncent - cbase, per));
  const float* rec = reinterpret_cast<const float*>(a.s.rec) + 2 * (int64_t)cbase;
  const int ldc = a.ldc;

  const int rowA = fac_entry_k(L, F0.A, F0.A.a * n2 + F0.A.b * n3 + F0.A.c);
  const int rowC = fac_entry_k(L, F0.C, F0.C.b * n3 + F0.C.c);
  constexpr int famA = F0.A.fam == F_G ? 0 : 16;
  constexpr int famB = F0.B.fam == F_G ? 0 : 16;
  constexpr int famC = F0.C.fam == F_G ? 0 : 16;

  // rows padded by one element: rows of different bins start in different LDS banks
  __shared__ C2<float> Xs[2][16][KC + 1];
  __shared__ C2<float> Zs[2][16][KC + 1];
  __shared__ H8 Ys[2][KS][MT][2][64];   // split Y operand in MFMA lane order
  __shared__ float sc_lds[3][16];       // scales of X (per b1), Y (b2), Z (b3)

  if (tid < 16) {
    const unsigned* M = a.maxima;
    // the scales yprep_kernel and the staging below apply (undone exactly at the end)
    float sx = 1.0f, sy = 1.0f, sz = 1.0f;
    if (tid < nb) {
      sx = xz_scale(M, famA, tid);
      sy = y_scale(M, F0.x, famB, tid);
      sz = xz_scale(M, famC, tid);
    }
    sc_lds[0][tid] = sx;
    sc_lds[1][tid] = sy;
    sc_lds[2][tid] = sz;
  }

  // ---- staging: global -> registers (issue), registers -> LDS (commit)
  PrefetchP<float, NXS, NYS> pf;
  // this thread's Y slots (K-step, row tile, lane): 16-byte copies from the
  // split operand of this n2 (yprep_kernel)
  constexpr int NQX = yprep_slots(2, NBC);
  const int64_t ychunks = (a.s.ncent + KC - 1) / KC;
  const u4* yp = reinterpret_cast<const u4*>(a.yprep) + (int64_t)(n2 + n) * ychunks * NQX * 2;
  int y_off[NYS];
  bool y_on[NYS];
#pragma unroll
  for (int h = 0; h < NYS; ++h) {
    const int q = tid + NT * h;
    const int ks = q / (MT * 64), m = (q / 64) % MT, l = q & 63;
    y_on[h] = ks < KS;
    y_off[h] = y_on[h] ? (ks * MT + m) * 2 * 64 + l : 0;
  }
  // Loads are unconditional (bin and centre clamped into the tile) so that
  // they stay in flight across the MFMAs; commit masks what lies outside.
  auto issue = [&](int c0) {
#pragma unroll
    for (int h = 0; h < NXS; ++h) {
      const int slot = tid + NT * h;           // (bin, centre) slot of X and Z
      const int b = slot / KC, c = c0 + slot % KC;
      const int bl = b < nb ? b : nb - 1, cl = c < ncent ? c : ncent - 1;
      pf.av[h] = ldrec(rec, (int64_t)rowA * nb + bl, ldc, cl);
      pf.cv[h] = ldrec(rec, (int64_t)rowC * nb + bl, ldc, cl);
    }
    const u4* yc = yp + ((int64_t)(cbase + c0) / KC) * NQX * 2;
#pragma unroll
    for (int h = 0; h < NYS; ++h) {
      pf.yh[h] = yc[y_off[h]];
      pf.yl[h] = yc[y_off[h] + 64];
    }
  };
  auto commit = [&](int c0, int buf) {
#pragma unroll
    for (int h = 0; h < NXS; ++h) {
      const int slot = tid + NT * h;
      const int b = slot / KC, cc = slot % KC;
      if (b < nb) {
        C2<float> av = pf.av[h], cv = pf.cv[h];
        if (F0.A.conj) av.i = -av.i;
        if (F0.C.conj) cv.i = -cv.i;
        const bool live = c0 + cc < ncent;
        const float sx = live ? sc_lds[0][b] : 0.f, sz = live ? sc_lds[2][b] : 0.f;
        Xs[buf][b][cc] = {av.r * sx, av.i * sx};
        Zs[buf][b][cc] = {cv.r * sz, cv.i * sz};
      }
    }
    // the split Y operand, copied as prepared (slots in the order of Ys)
    H8* ys = &Ys[buf][0][0][0][0];
#pragma unroll
    for (int h = 0; h < NYS; ++h) {
      if (!y_on[h]) continue;
      ys[y_off[h]] = __builtin_bit_cast(H8, pf.yh[h]);
      ys[y_off[h] + 64] = __builtin_bit_cast(H8, pf.yl[h]);
    }
  };

  // per-lane column (b1, b3) of each of this wave's tiles; padding columns
  // read the zero row nb of the X buffer (nb < 16 whenever nb^2 % 16 != 0)
  int b1c[NTW], b3c[NTW];
  bool colok[NTW];
#pragma unroll
  for (int t = 0; t < NTW; ++t) {
    const int T = wr + WB * t;
    const int j = 16 * T + (lane & 15);
    colok[t] = j < ncols;
    b1c[t] = colok[t] ? j / nb : (nb < 16 ? nb : 0);
    b3c[t] = colok[t] ? j % nb : 0;
  }
  for (int z = tid; z < 2 * 16 * (KC + 1); z += NT) {
    const int bb = (z / (KC + 1)) % 16;
    if (bb >= nb) Xs[z / (16 * (KC + 1))][bb][z % (KC + 1)] = {0.f, 0.f};
  }

  f4 acc[MT][NTW];
  double acc64[MT][NTW][4];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NTW; ++t) {
      acc[m][t] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[m][t][r] = 0.0;
    }

  const int nchunks = (ncent + KC - 1) / KC;
  __syncthreads();              // scales visible
  if (ncent > 0) {              // uniform: an empty slice only writes zeros
    issue(0);
    commit(0, 0);
  }
  __syncthreads();
  for (int ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunks;
    if (more) issue((ch + 1) * KC);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      H8 yh[MT], yl[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        yh[m] = Ys[buf][ks][m][0][lane];
        yl[m] = Ys[buf][ks][m][1][lane];
      }
      const int cb = 16 * ks + 4 * (lane >> 4);
      // form the Khatri-Rao operand of one column tile, then issue its MFMAs
      // product by product over the row tiles, so that consecutive MFMAs
      // accumulate into different registers.  Row tiles past the used rows
      // multiply zero Y rows.
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        if (wr + WB * t >= ntiles) break;   // wave-uniform
        float v[8];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const C2<float> xv = Xs[buf][b1c[t]][cb + u];
          const C2<float> zv = Zs[buf][b3c[t]][cb + u];
          v[2 * u] = __builtin_fmaf(xv.r, zv.r, -(xv.i * zv.i));
          v[2 * u + 1] = __builtin_fmaf(xv.r, zv.i, xv.i * zv.r);
        }
        H8 rh, rl;
        split8v<PREC>(v, rh, rl);
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m][t] = mfma16<PREC>(yh[m], rh, acc[m][t]);
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m][t] = mfma16<PREC>(yh[m], rl, acc[m][t]);
#pragma unroll
        for (int m = 0; m < MT; ++m) acc[m][t] = mfma16<PREC>(yl[m], rh, acc[m][t]);
      }
    }
    if ((ch & 15) == 15 || !more) {       // fold fp32 into binary64 every 512 centres
#pragma unroll
      for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int t = 0; t < NTW; ++t) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[m][t][r] += (double)acc[m][t][r];
          acc[m][t] = f4{0.f, 0.f, 0.f, 0.f};
        }
    }
    if (more) commit((ch + 1) * KC, buf ^ 1);
    __syncthreads();
  }

  // write: D row = 4*(lane/16) + r in tile m, column = lane%16 in tile t.  With
  // several centre slices each slice writes its own binary64 partial buffer.
  const int64_t ups2 = 2 * (int64_t)9 * nb * nb * nb * nn * nn;
#pragma unroll
  for (int t = 0; t < NTW; ++t) {
    if (!colok[t]) continue;
    const int b1 = b1c[t], b3 = b3c[t];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * m + 4 * (lane >> 4) + r;
        if (row >= mrows) continue;
        const int mi = row / (2 * nb), rem = row % (2 * nb), part = rem / nb, b2 = rem % nb;
        const int mu = mi ? GR.mu[1] : GR.mu[0];
        const double unscale = 1.0 / ((double)sc_lds[0][b1] * sc_lds[1][b2] * sc_lds[2][b3]);
        const int64_t o = (((((int64_t)mu * nb + b1) * nb + b2) * nb + b3) * nn + (n2 + n)) * nn + (n3 + n);
        const double v = acc64[m][t][r] * unscale;
        if (gridDim.y == 1) a.s.ups[2 * o + part] += v;
        else a.s.part[(int64_t)by * ups2 + 2 * o + part] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// binary64
// ---------------------------------------------------------------------------
template <int G, int NBC>
__global__ __launch_bounds__(512) void contract_f64_kernel(BArgs a) {
  constexpr Group GR = group_of(G);
  constexpr MuFactors F0 = mu_factors(GR.mu[0]);
  constexpr MuFactors F1 = mu_factors(GR.mu[1]);
  constexpr int MT = mt_of(GR.nmu, NBC);
  constexpr int NTW = ntw_of(NBC);
  constexpr int WB = wb_of(NBC);
  constexpr int NT = 64 * WB;
  constexpr int NXS = (NBC * KC + NT - 1) / NT;  // (bin, centre) staging slots per thread
  const int nb = a.s.nb, n = a.s.nmax, nn = 2 * n + 1;
  const Layout L = make_layout(n);
  int bx, by;
  xcd_block(bx, by);
  const int lb = bx;
  const int n2 = lb / nn - n;
  const int n3 = lb % nn - n;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  // column tiles of this wave: T = wr + WB t.  When the tiles do not split
  // evenly, the wave holding one more is rotated with the block index, so
  // that co-resident workgroups put their longer waves on different SIMDs.
  const int wr = (wv + bx) & (WB - 1);
  const int mrows = GR.nmu * 2 * nb;
  const int ncols = nb * nb;
  const int ntiles = (ncols + 15) >> 4;
  const int per = contract_slice_len(a.s.ncent, (int)gridDim.y);
  const int cbase = by * per;
  const int ncent = imax(0, imin(a.s.ncent - cbase, per));
  const double* rec = reinterpret_cast<const double*>(a.s.rec) + 2 * (int64_t)cbase;
  const int ldc = a.ldc;
  const int rowA = fac_entry_k(L, F0.A, F0.A.a * n2 + F0.A.b * n3 + F0.A.c);
  const int rowC = fac_entry_k(L, F0.C, F0.C.b * n3 + F0.C.c);
  const int rowB0 = fac_entry_k(L, F0.B, F0.B.a * n2 + F0.B.c);
  const int rowB1 = fac_entry_k(L, F1.B, F1.B.a * n2 + F1.B.c);

  __shared__ C2<double> Xs[2][16][KC + 1];
  __shared__ C2<double> Zs[2][16][KC + 1];
  __shared__ C2<double> Ys[2][GR.nmu][16][KC + 1];   // [mu idx][b2][centre]

  const C2<double>* xg = reinterpret_cast<const C2<double>*>(a.xg) + cbase;
  const double* xw = reinterpret_cast<const double*>(a.xw) + cbase;
  struct PF {
    C2<double> xc, av, cv, y0, y1;
  } pf[NXS];
  // unconditional loads (clamped into the tile), masked in commit
  auto issue = [&](int c0) {
#pragma unroll
    for (int h = 0; h < NXS; ++h) {
      const int slot = tid + NT * h;
      const int b = slot / KC, c = c0 + slot % KC;
      const int bl = b < nb ? b : nb - 1, cl = c < ncent ? c : ncent - 1;
      if (F0.x == X_W) pf[h].xc = {xw[cl], 0.0};
      else pf[h].xc = xg[cl];
      pf[h].av = ldrec(rec, (int64_t)rowA * nb + bl, ldc, cl);
      pf[h].cv = ldrec(rec, (int64_t)rowC * nb + bl, ldc, cl);
      pf[h].y0 = ldrec(rec, (int64_t)rowB0 * nb + bl, ldc, cl);
      if (GR.nmu == 2) pf[h].y1 = ldrec(rec, (int64_t)rowB1 * nb + bl, ldc, cl);
    }
  };
  auto commit = [&](int c0, int buf) {
#pragma unroll
    for (int h = 0; h < NXS; ++h) {
      const int slot = tid + NT * h;
      const int b = slot / KC, cc = slot % KC;
      if (b < nb) {
        C2<double> xc = pf[h].xc, av = pf[h].av, cv = pf[h].cv, y0 = pf[h].y0, y1 = pf[h].y1;
        if (c0 + cc >= ncent) xc = av = cv = y0 = y1 = {0.0, 0.0};
        if (F0.x == X_GC) xc.i = -xc.i;
        if (F0.A.conj) av.i = -av.i;
        if (F0.C.conj) cv.i = -cv.i;
        if (F0.B.conj) y0.i = -y0.i;
        if (F1.B.conj) y1.i = -y1.i;
        Xs[buf][b][cc] = {xc.r * av.r - xc.i * av.i, xc.r * av.i + xc.i * av.r};
        Zs[buf][b][cc] = cv;
        Ys[buf][0][b][cc] = y0;
        if (GR.nmu == 2) Ys[buf][GR.nmu - 1][b][cc] = y1;
      }
    }
  };

  int arow_mi[MT], arow_part[MT], arow_b2[MT];
  bool arow_ok[MT];
#pragma unroll
  for (int m = 0; m < MT; ++m) {
    const int r = 16 * m + (lane & 15);
    arow_ok[m] = r < mrows;
    const int rr = arow_ok[m] ? r : 0;
    arow_mi[m] = rr / (2 * nb);
    arow_part[m] = (rr % (2 * nb)) / nb;
    arow_b2[m] = rr % nb;
  }
  int b1c[NTW], b3c[NTW];
  bool colok[NTW];
#pragma unroll
  for (int t = 0; t < NTW; ++t) {
    const int T = wr + WB * t;
    const int j = 16 * T + (lane & 15);
    colok[t] = j < ncols;
    b1c[t] = colok[t] ? j / nb : 0;
    b3c[t] = colok[t] ? j % nb : 0;
  }
  d4 acc[MT][NTW];
#pragma unroll
  for (int m = 0; m < MT; ++m)
#pragma unroll
    for (int t = 0; t < NTW; ++t) acc[m][t] = d4{0.0, 0.0, 0.0, 0.0};

  const int nchunks = (ncent + KC - 1) / KC;
  const int kq = lane >> 4;  // k within the K=4 step: (centre = kq/2, part = kq%2)
  if (ncent > 0) {           // uniform: an empty slice only writes zeros
    issue(0);
    commit(0, 0);
  }
  __syncthreads();
  for (int ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunks;
    if (more) issue((ch + 1) * KC);
#pragma unroll 4
    for (int ks = 0; ks < KC / 2; ++ks) {
      const int cc = 2 * ks + (kq >> 1);
      const int pk = kq & 1;
      double av[MT];
#pragma unroll
      for (int m = 0; m < MT; ++m) {
        const C2<double> y = Ys[buf][arow_mi[m]][arow_b2[m]][cc];
        // [[y_r, -y_i], [y_i, y_r]]
        const double v = arow_part[m] ? (pk ? y.r : y.i) : (pk ? -y.i : y.r);
        av[m] = arow_ok[m] ? v : 0.0;
      }
#pragma unroll
      for (int t = 0; t < NTW; ++t) {
        if (wr + WB * t >= ntiles) break;   // wave-uniform
        const C2<double> xv = Xs[buf][b1c[t]][cc];
        const C2<double> zv = Zs[buf][b3c[t]][cc];
        double bv = pk ? xv.r * zv.i + xv.i * zv.r : xv.r * zv.r - xv.i * zv.i;
        bv = colok[t] ? bv : 0.0;
#pragma unroll
        for (int m = 0; m < MT; ++m)
          acc[m][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[m], bv, acc[m][t], 0, 0, 0);
      }
    }
    if (more) commit((ch + 1) * KC, buf ^ 1);
    __syncthreads();
  }

  // f64 D layout: element r of lane L is row 4 r + L/16, column L%16.  With
  // several centre slices each slice writes its own partial buffer.
  const int64_t ups2 = 2 * (int64_t)9 * nb * nb * nb * nn * nn;
#pragma unroll
  for (int t = 0; t < NTW; ++t) {
    if (!colok[t]) continue;
    const int b1 = b1c[t], b3 = b3c[t];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * m + 4 * r + (lane >> 4);
        if (row >= mrows) continue;
        const int mi = row / (2 * nb), rem = row % (2 * nb), part = rem / nb, b2 = rem % nb;
        const int mu = mi ? GR.mu[1] : GR.mu[0];
        const int64_t o = (((((int64_t)mu * nb + b1) * nb + b2) * nb + b3) * nn + (n2 + n)) * nn + (n3 + n);
        if (gridDim.y == 1) a.s.ups[2 * o + part] += acc[m][t][r];
        else a.s.part[(int64_t)by * ups2 + 2 * o + part] = acc[m][t][r];
      }
    }
  }
}

template <int G, int NBC>
static void launch_group_nbc(const BArgs& a, int precision, int nsl, hipStream_t s) {
  const int nn = 2 * a.s.nmax + 1;
  const dim3 grid(nn * nn, nsl), block(64 * wb_of(NBC));
  if (precision == FPCF4_FP64) {
    hipLaunchKernelGGL((contract_f64_kernel<G, NBC>), grid, block, 0, s, a);
    return;
  }
  // the group's split Y operand, then the contraction that copies it
  const int64_t nchunk = (a.s.ncent + KC - 1) / KC;
  const int64_t nthreads = (int64_t)nn * nchunk * yprep_slots(group_of(G).nmu, NBC);
  const dim3 pgrid((unsigned)((nthreads + 255) / 256));
  if (precision == FPCF4_MIXED_FP16) {
    hipLaunchKernelGGL((yprep_kernel<FPCF4_MIXED_FP16, G, NBC>), pgrid, dim3(256), 0, s, a);
    hipLaunchKernelGGL((contract_mixed_kernel<FPCF4_MIXED_FP16, G, NBC>), grid, block, 0, s, a);
  } else {
    hipLaunchKernelGGL((yprep_kernel<FPCF4_MIXED_BF16, G, NBC>), pgrid, dim3(256), 0, s, a);
    hipLaunchKernelGGL((contract_mixed_kernel<FPCF4_MIXED_BF16, G, NBC>), grid, block, 0, s, a);
  }
}

template <int G>
static hipError_t launch_group(const BArgs& a, int precision, int nsl, hipStream_t s) {
  if (a.s.nb <= 8) launch_group_nbc<G, 8>(a, precision, nsl, s);
  else if (a.s.nb <= 12) launch_group_nbc<G, 12>(a, precision, nsl, s);
  else launch_group_nbc<G, 16>(a, precision, nsl, s);
  return hipGetLastError();
}

// ups[i] += sum of the slice partials, slices in order
__global__ void contract_reduce_kernel(const double* part, int nsl, int64_t n2, double* ups) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2) return;
  double v = 0.0;
  for (int k = 0; k < nsl; ++k) v += part[(int64_t)k * n2 + i];
  ups[i] += v;
}

double contract_f64_issued_flops(int nb, int nmax, int64_t ncent) {
  const int nbc = nb <= 8 ? 8 : (nb <= 12 ? 12 : 16);
  const int nn = 2 * nmax + 1;
  double rows = 0.0;
  for (int g = 0; g < NGROUPS; ++g) rows += 16.0 * mt_of(group_of(g).nmu, nbc);
  const double cols = 16.0 * ((nb * nb + 15) / 16);
  return rows * cols * 2.0 * 2.0 * (double)nn * nn * (double)ncent;
}

size_t yprep_bytes(int nb, int nmax, int64_t ncent) {
  const int nbc = nb <= 8 ? 8 : (nb <= 12 ? 12 : 16);
  return yprep_bytes_for(nbc, nmax, ncent);
}

hipError_t launch_contract(const StageBArgs& sb, int precision, int ldc, const void* xg,
                           const void* xw, const unsigned* maxima, hipStream_t s) {
  if (sb.ncent <= 0) return hipSuccess;
  if (precision != FPCF4_FP64 && sb.yprep == nullptr) return hipErrorInvalidValue;
  BArgs a{sb, ldc, xg, xw, maxima, sb.yprep};
  const int nsl = sb.part ? contract_slices(sb.ncent, sb.nmax) : 1;
  hipError_t e;
  if ((e = launch_group<0>(a, precision, nsl, s)) != hipSuccess) return e;
  if ((e = launch_group<1>(a, precision, nsl, s)) != hipSuccess) return e;
  if ((e = launch_group<2>(a, precision, nsl, s)) != hipSuccess) return e;
  if ((e = launch_group<3>(a, precision, nsl, s)) != hipSuccess) return e;
  if ((e = launch_group<4>(a, precision, nsl, s)) != hipSuccess) return e;
  if ((e = launch_group<5>(a, precision, nsl, s)) != hipSuccess) return e;
  if ((e = launch_group<6>(a, precision, nsl, s)) != hipSuccess) return e;
  if (nsl > 1) {
    const int nn = 2 * sb.nmax + 1;
    const int64_t n2 = 2 * (int64_t)9 * sb.nb * sb.nb * sb.nb * nn * nn;
    hipLaunchKernelGGL(contract_reduce_kernel, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s,
                       (const double*)sb.part, nsl, n2, sb.ups);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace fpcf4
