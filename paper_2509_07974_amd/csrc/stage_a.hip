// Stage (a): per-centre multipoles in radial bins (the quadratic pair stage).
//
// For every centre i of a tile and every radial bin b the kernel forms the
// real-weight power sums
//
//     S_f,k(i, b) = sum_{j : theta_ij in Theta_b} v_f(j) z_ij^k,   k >= 0,
//     z_ij = e^{i phi_ij} = (dx + i dy) / |theta_ij|,
//
// for the seven per-galaxy weights v_f = Re(w g), Im(w g), Re((w g)^2),
// Im((w g)^2), w, |w g|^2, w^2 (plus the few orders the triple-counting
// blocks need), and turns them into the record blocks of Sect. 3.1 and
// App. A.1 (see fpcf4_internal.hpp), e.g.
//     G_k  = S_a,k + i S_b,k,   G_-k = conj(S_a,k) + i conj(S_b,k).
// Every block of the paper is a sum of a real weight times e^{+-ik phi},
// so accumulating only k >= 0 halves the complex multiply-adds.
//
// Mapping on CDNA4 (wave64):
//  * one workgroup owns one centre at a time (dynamic per-XCD queues, with
//    stealing, over a Morton-ordered centre list); its W waves each own one
//    pass, i.e. one range of orders k whose accumulators fit the register
//    file (the units of all passes together cover every order once);
//  * for each bin the annulus is a list of row segments of the cell grid
//    (row bounds computed lane-parallel, one row per lane); the workgroup
//    walks its flat candidate list in rounds of W chunks of 64: wave w loads
//    chunk W r + w (one 32- or 48-byte galaxy record per lane), forms r^2 in
//    binary64 without contraction and tests the bin against the squared
//    edges -- the same arithmetic as the oracle, so binning is bit-exact --
//    and compacts its in-bin neighbours with a ballot into LDS;
//  * after one barrier per round every wave consumes all compacted
//    neighbours of the round in full batches of 64 (each lane forms z, its
//    power chain z^k and adds to its own partial sums), so the binning is
//    done once and shared by every pass;
//  * partial sums are combined across lanes by a transposing butterfly
//    (log2 64 levels, halving the live values per level), so each lane ends
//    with complete sums of its own units; the binary32 variant folds into
//    binary64 masters every few batches (blocked summation).
#include <type_traits>

#include "fpcf4_internal.hpp"

namespace fpcf4 {
namespace sa {

enum { FA = 0, FB, FC, FD, FW, FE, FV, NF };

// Order plan.  The plan index n is the record order nmax for the 4PCF; an
// index 3PCF_PLAN + m selects the plan of the shear 3PCF on records of order
// m: the same record layout, but only the orders the 3PCF reads are formed
// (G up to 2m + 3, W up to 2m, and of the same-neighbour families Q up to 6,
// A up to 2, V at 0: the blocks Q_-6, Q_-2, A_2, V_0 of its corrections),
// and no triple-counting blocks.
constexpr int PLAN3 = 100;
__host__ __device__ constexpr bool is3(int n) { return n >= PLAN3; }
__host__ __device__ constexpr int nord(int n) { return is3(n) ? n - PLAN3 : n; }
// special units of pass 0: P8, Q8, P4, Q4, EA4, EB4 (complex); EA0, EB0, U (real)
__host__ __device__ constexpr int nspecial(int n) { return is3(n) ? 0 : 15; }

__host__ __device__ constexpr int kmax_f(int n, int f) {
  return is3(n) ? ((f == FA || f == FB) ? 2 * nord(n) + 3
                 : (f == FC || f == FD) ? 6
                 : (f == FE)            ? 2
                 : (f == FW)            ? 2 * nord(n)
                                        : 0)
                : ((f == FA || f == FB) ? 2 * n + 3
                 : (f == FC || f == FD) ? imax(2 * n + 5, n + 6)
                 : (f == FE)            ? imax(2 * n + 1, n + 2)
                                        : 2 * n);
}
__host__ __device__ constexpr int ktop(int n) {
  return is3(n) ? imax(2 * nord(n) + 3, 6) : imax(2 * n + 5, n + 6);
}
__host__ __device__ constexpr int units_at(int n, int k) {
  int u = 0;
  for (int f = 0; f < NF; ++f)
    if (k <= kmax_f(n, f)) u += (k == 0 ? 1 : 2);
  return u;
}
__host__ __device__ constexpr int total_units(int n) {
  int u = nspecial(n);
  for (int k = 0; k <= ktop(n); ++k) u += units_at(n, k);
  return u;
}
// Split of the orders 0..ktop into passes of at most `cap` accumulator
// units each (greedy, in order); pass 0 also holds the 15 special units
// (orders 0, 4, 8 of the triple blocks, accumulated from z^4 and z^8 formed
// by squaring).
struct PassPlan {
  int np;
  int k0[32], k1[32], units[32];
};
__host__ __device__ constexpr PassPlan greedy(int n, int cap) {
  PassPlan P{};
  int k = 0;
  while (k <= ktop(n) && P.np < 32) {
    int used = (P.np == 0) ? nspecial(n) : 0;
    const int start = k;
    while (k <= ktop(n) && (k == start || used + units_at(n, k) <= cap)) {
      used += units_at(n, k);
      ++k;
    }
    P.k0[P.np] = start;
    P.k1[P.np] = k - 1;
    P.units[P.np] = used;
    ++P.np;
  }
  return P;
}
// Exactly W passes with the smallest largest pass: the smallest cap that
// needs at most W passes, then the largest passes split in two (at the
// order that balances their halves) until there are W.
__host__ __device__ constexpr PassPlan plan_exact(int n, int w) {
  int cap = (total_units(n) + w - 1) / w;
  while (greedy(n, cap).np > w) ++cap;
  PassPlan P = greedy(n, cap);
  while (P.np < w) {
    int big = -1;
    for (int p = 0; p < P.np; ++p)
      if (P.k1[p] > P.k0[p] && (big < 0 || P.units[p] > P.units[big])) big = p;
    if (big < 0) break;   // every pass is a single order
    const int k0 = P.k0[big], k1 = P.k1[big];
    int best = k0, bestmax = 1 << 30;
    for (int split = k0; split < k1; ++split) {
      int lo = (big == 0) ? nspecial(n) : 0, hi = 0;
      for (int k = k0; k <= split; ++k) lo += units_at(n, k);
      for (int k = split + 1; k <= k1; ++k) hi += units_at(n, k);
      const int m = imax(lo, hi);
      if (m < bestmax) { bestmax = m; best = split; }
    }
    for (int p = P.np; p > big + 1; --p) {
      P.k0[p] = P.k0[p - 1];
      P.k1[p] = P.k1[p - 1];
      P.units[p] = P.units[p - 1];
    }
    int lo = (big == 0) ? nspecial(n) : 0, hi = 0;
    for (int k = k0; k <= best; ++k) lo += units_at(n, k);
    for (int k = best + 1; k <= k1; ++k) hi += units_at(n, k);
    P.k1[big] = best;
    P.units[big] = lo;
    P.k0[big + 1] = best + 1;
    P.k1[big + 1] = k1;
    P.units[big + 1] = hi;
    ++P.np;
  }
  return P;
}
__host__ __device__ constexpr int max_units(const PassPlan& P) {
  int m = 0;
  for (int p = 0; p < P.np; ++p) m = imax(m, P.units[p]);
  return m;
}
// Waves per workgroup (one per pass): a power of two, so that two or more
// workgroups tile the four SIMDs of a CU evenly.  Binary32: the fewest waves
// whose passes fit 132 accumulators, at least four from nmax 5 on (4PCF
// plan) or at least two (3PCF plan, measured best at record order 5: two
// passes of 54 units ahead of one and four); binary64 (two registers per
// accumulator): passes of at most 72.
__host__ __device__ constexpr int choose_waves(int n, bool fp64) {
  const int lim = fp64 ? 72 : 132;
  int w = 1;
  while (w < 8 && max_units(plan_exact(n, w)) > lim) w *= 2;
  if (!fp64 && !is3(n) && n >= 5 && w < 4) w = 4;
  if (!fp64 && is3(n) && w < 2) w = 2;
  return w;
}

__host__ __device__ constexpr int ubase(int n, int k0, int k) {
  int b = 0;
  for (int kk = k0; kk < k; ++kk) b += units_at(n, kk);
  return b;
}
__host__ __device__ constexpr int uidx(int n, int k0, int f, int k) {
  int u = ubase(n, k0, k);
  for (int g = 0; g < f; ++g)
    if (k <= kmax_f(n, g)) u += (k == 0 ? 1 : 2);
  return u;
}

template <typename T> struct Budget;
template <> struct Budget<float> { static constexpr int fold = 128; };
template <> struct Budget<double> { static constexpr int fold = 1 << 30; };

__device__ __forceinline__ double r2_exact(double dx, double dy) {
#pragma clang fp contract(off)
  const double a = dx * dx;
  const double b = dy * dy;
  return a + b;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned rank_in_mask(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

template <typename T> __device__ __forceinline__ T rsq(T v);
template <> __device__ __forceinline__ float rsq<float>(float v) { return __frsqrt_rn(v); }
template <> __device__ __forceinline__ double rsq<double>(double v) { return rsqrt(v); }

// Cross-lane primitives of the transposing butterfly.  swap32/swap16
// exchange halves between two registers (v_permlane32_swap /
// v_permlane16_swap): afterwards r0 + r1 holds, in lanes 0-31 (rows 0, 2),
// the pair sums of the first register and in lanes 32-63 (rows 1, 3) those
// of the second.  dpp(v, ctrl) reads the partner lane given by a DPP pattern
// (row mirror, half-row mirror, quad permutations).
__device__ __forceinline__ float swap_add32(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap_add16(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ double swap_add32(double a, double b) {
  const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  return __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0])) +
         __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ double swap_add16(double a, double b) {
  const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  return __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0])) +
         __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)u, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
constexpr int DPP_ROW_MIRROR = 0x140;       // lane i <- 15 - i within 16
constexpr int DPP_ROW_HALF_MIRROR = 0x141;  // lane i <- 7 - i within 8
constexpr int DPP_QUAD_XOR2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int DPP_QUAD_XOR1 = 0xB1;         // quad_perm [1,0,3,2]

// One level of the butterfly for partner patterns that swap the lane bit
// `bit`: lanes with the bit clear keep the lower half of the live values.
template <typename T, int D, int CTRL>
__device__ __forceinline__ void level_dpp(T* v, unsigned lane, unsigned bit) {
  const bool up = (lane & bit) != 0;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const T lo = v[k] + dpp<CTRL>(v[k]);
    const T hi = v[k + D] + dpp<CTRL>(v[k + D]);
    v[k] = up ? hi : lo;
  }
}

// Sum unit 64*M + lane over all 64 lanes (transposing butterfly): each level
// pairs lanes that hold the same live units and halves that set, so lane l
// ends with the complete sum of unit 64*M + l.
template <typename T, int NU, int M>
__device__ __forceinline__ T butterfly_block(const T* acc, unsigned lane) {
  T v[64];
#pragma unroll
  for (int k = 0; k < 64; ++k) v[k] = (64 * M + k < NU) ? acc[64 * M + k] : T(0);
#pragma unroll
  for (int k = 0; k < 32; ++k) v[k] = swap_add32(v[k], v[k + 32]);   // lane bit 5
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = swap_add16(v[k], v[k + 16]);   // lane bit 4
  level_dpp<T, 8, DPP_ROW_MIRROR>(v, lane, 8);
  level_dpp<T, 4, DPP_ROW_HALF_MIRROR>(v, lane, 4);
  level_dpp<T, 2, DPP_QUAD_XOR2>(v, lane, 2);
  level_dpp<T, 1, DPP_QUAD_XOR1>(v, lane, 1);
  return v[0];
}

template <typename T, int NU, int NM, int M = 0>
__device__ __forceinline__ void fold_all(T* acc, double* mst, unsigned lane) {
  if constexpr (M < NM) {
    mst[M] += (double)butterfly_block<T, NU, M>(acc, lane);
    fold_all<T, NU, NM, M + 1>(acc, mst, lane);
  }
}

// Accumulate one neighbour (weights val[], power chain p = z^K starting at
// K = K0) into the order units of the pass; all unit indices are
// compile-time constants, so the accumulators stay in registers.
template <typename T, int N, int K0, int K1, int K, int F>
__device__ __forceinline__ void acc_fields(T* acc, const T* val, T pr, T pi) {
  if constexpr (F < NF) {
    if constexpr (K <= kmax_f(N, F)) {
      constexpr int u = uidx(N, K0, F, K);
      if constexpr (K == 0) {
        acc[u] += val[F];
      } else {
        acc[u] += val[F] * pr;
        acc[u + 1] += val[F] * pi;
      }
    }
    acc_fields<T, N, K0, K1, K, F + 1>(acc, val, pr, pi);
  }
}

template <typename T>
__device__ __forceinline__ T fmadd(T a, T b, T c) {
  if constexpr (sizeof(T) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

// Sign of the power a pass holds at offset d = K - K0 of its chain:
// +, +, -, -, +, +, ...  The units of order K accumulate that multiple of
// their sums; the epilogue multiplies it back.
__host__ __device__ constexpr int chain_sign(int d) { return ((d >> 1) & 1) ? -1 : 1; }

// The power chain alternates a complex product z^(K+1) = z^K z with the
// two-term recurrence z^(K+1) = 2 Re(z) z^K - z^(K-1) (two fused
// multiply-adds instead of four).  A recurrence step from exact powers errs
// by (|z|^2 - 1) z^(K-1), independent of the angle, and the interleaved
// products keep later errors from growing: in binary32 the powers up to
// z^26 stay within 1.4x the error of the all-product chain.
// Every step is a multiply-add with no negated operand (-Im z comes with
// the neighbour, -2 Re z is formed once per neighbour), so that it encodes as
// the two-operand accumulate (VOP2), which can issue in the same cycle as
// another VALU instruction; the recurrence then yields -z^(K+1), hence the
// alternating chain_sign.
template <typename T, int N, int K0, int K1, int K>
__device__ __forceinline__ void acc_orders(T* acc, const T* val, T pr, T pi, T qr, T qi, T zr,
                                           T zi, T nzi, T nc2) {
  acc_fields<T, N, K0, K1, K, 0>(acc, val, pr, pi);
  if constexpr (K < K1) {
    T tr, ti;
    if constexpr (K == 0) {
      tr = zr;   // z^0 z
      ti = zi;
    } else if constexpr (((K - K0) & 1) == 0) {
      tr = fmadd(pr, zr, pi * nzi);
      ti = fmadd(pr, zi, pi * zr);
    } else {
      tr = fmadd(nc2, pr, qr);
      ti = fmadd(nc2, pi, qi);
    }
    acc_orders<T, N, K0, K1, K + 1>(acc, val, tr, ti, pr, pi, zr, zi, nzi, nc2);
  }
}

// z^E by squaring; the first factor is taken as it is (no product with 1)
template <typename T, int E>
__device__ __forceinline__ void cpow(T zr, T zi, T& pr, T& pi) {
  pr = T(1);
  pi = T(0);
  T br = zr, bi = zi;
  int e = E;
  bool one = true;
#pragma unroll
  for (int it = 0; it < 6; ++it) {
    if (e & 1) {
      if (one) {
        pr = br;
        pi = bi;
        one = false;
      } else {
        const T tr = pr * br - pi * bi;
        pi = pr * bi + pi * br;
        pr = tr;
      }
    }
    e >>= 1;
    if (e) {
      const T tr = br * br - bi * bi;
      bi = T(2) * br * bi;
      br = tr;
    }
  }
}

// One in-bin neighbour as every pass consumes it: z = e^{i phi} and the
// seven real weights (a = Re wg, b = Im wg, c = Re (wg)^2, d = Im (wg)^2,
// e = |wg|^2, v = w^2, and w), formed once by the lane that binned it.
template <typename T> struct alignas(16) Q4 { T x, y, z, w; };
template <typename T> struct alignas(2 * sizeof(T)) Q2 { T x, y; };
template <typename T> struct Nb {
  T zr, zi, a, b, c, d, e, v, w;
  T sr, si;   // z^K0 of the consuming pass, when the binning lane formed it
  T nzi;      // -Im z
  T p3, q3, ea, eb, u;   // triple-block weights of a pseudo-galaxy (reduced catalogues)
};

// binary32 passes take their first power z^K0 from the ring (formed once per
// neighbour by the lane that binned it); binary64 rings would not fit LDS
template <typename T> constexpr bool kRingStarts = sizeof(T) == 4;
// Exact binary32 ring: the weight w and -Im z travel in the third and fourth
// components of the start slots, so that every ring array a pass reads has
// the 16-byte stride of q0 and one address serves all reads of a neighbour.  The reduced-
// catalogue kernel keeps separate 8-byte starts and w (its ring also holds
// the triple-block weights, and the larger slots would cost occupancy).
template <typename T, bool RED> constexpr bool kPackW = sizeof(T) == 4 && !RED;
template <typename T, bool PACK> struct QKsel { using type = Q2<T>; };
template <typename T> struct QKsel<T, true> { using type = Q4<T>; };

// Add one neighbour to the units of one pass.  Lanes with valid == false
// add nothing.
template <typename T, int N, int K0, int K1, bool P0, int NUO, bool RED>
__device__ __forceinline__ void add_pair(T* acc, bool valid, Nb<T> q) {
  if (!valid) q = Nb<T>{};
  T val[NF];
  val[FA] = q.a;
  val[FB] = q.b;
  val[FC] = q.c;
  val[FD] = q.d;
  val[FW] = q.w;
  val[FE] = q.e;
  val[FV] = q.v;
  const T zr = q.zr, zi = q.zi;
  T pr, pi;
  if constexpr (K0 > 0 && kRingStarts<T>) {
    pr = q.sr;
    pi = q.si;
  } else {
    cpow<T, K0>(zr, zi, pr, pi);
  }
  acc_orders<T, N, K0, K1, K0>(acc, val, pr, pi, T(0), T(0), zr, zi, q.nzi, T(-2) * zr);
  if constexpr (P0 && !is3(N)) {
    // triple-counting blocks: T_-8, T_-4 (weight (w g)^3), M_-4, M_0
    // (weight |w g|^2 w g) and U (weight w^3)
    const T z2r = zr * zr - zi * zi, z2i = T(2) * zr * zi;
    const T z4r = z2r * z2r - z2i * z2i, z4i = T(2) * z2r * z2i;
    const T z8r = z4r * z4r - z4i * z4i, z8i = T(2) * z4r * z4i;
    // per galaxy: Re/Im (w g)^3 and |w g|^2 w g from w g; a pseudo-galaxy
    // carries the cell sums of these weights
    const T p3 = RED ? q.p3 : q.c * q.a - q.d * q.b;
    const T q3 = RED ? q.q3 : q.c * q.b + q.d * q.a;
    const T ea = RED ? q.ea : q.e * q.a, eb = RED ? q.eb : q.e * q.b;
    acc[NUO + 0] += p3 * z8r;
    acc[NUO + 1] += p3 * z8i;
    acc[NUO + 2] += q3 * z8r;
    acc[NUO + 3] += q3 * z8i;
    acc[NUO + 4] += p3 * z4r;
    acc[NUO + 5] += p3 * z4i;
    acc[NUO + 6] += q3 * z4r;
    acc[NUO + 7] += q3 * z4i;
    acc[NUO + 8] += ea * z4r;
    acc[NUO + 9] += ea * z4i;
    acc[NUO + 10] += eb * z4r;
    acc[NUO + 11] += eb * z4i;
    acc[NUO + 12] += ea;
    acc[NUO + 13] += eb;
    acc[NUO + 14] += RED ? q.u : q.w * q.v;
  }
}

__host__ __device__ constexpr int max_blocks64(const PassPlan& P) {
  int m = 1;
  for (int p = 0; p < P.np; ++p) m = imax(m, (P.units[p] + 63) / 64);
  return m;
}

template <typename T, int N> struct Conf {
  static constexpr int W = choose_waves(N, sizeof(T) == 8);   // waves per workgroup = passes
  static constexpr PassPlan PP = plan_exact(N, W);
  static constexpr int NMX = max_blocks64(PP);
  // waves per SIMD the register allocation aims at: binary32 passes of up
  // to 96 accumulators fit 168 VGPRs (three waves per SIMD), larger ones and
  // binary64 passes take two
  static constexpr int EU = (sizeof(T) == 4 && max_units(PP) <= 96) ? 3 : 2;
  static_assert(PP.np == W, "one pass per wave");
  static_assert(W == 1 || W == 2 || W == 4 || W == 8, "power-of-two workgroups");
  static_assert((4 * EU) % W == 0 || W % 4 == 0, "workgroups must tile the SIMDs");
};

__host__ __device__ constexpr int ring_cap(int w) {
  int c = 64;
  while (c < 64 * (w + 1)) c *= 2;
  return c;
}

template <typename T, int W, int NMX, bool RED> struct Shared {
  static constexpr int CAP = ring_cap(W);
  // ring of in-bin neighbours (z, a, b | c, d, e, v | w); the entries of a
  // round are appended in wave order, so a batch is 64 consecutive slots
  static constexpr bool PACK = kPackW<T, RED>;
  using QK = typename QKsel<T, PACK>::type;
  static constexpr int NQK = kRingStarts<T> && W > 1 ? W - 1 : 1;
  static constexpr bool HASQK = (kRingStarts<T> && W > 1) || PACK;
  Q4<T> q0[CAP];
  Q4<T> q1[CAP];
  QK qk[NQK][HASQK ? CAP : 1];  // z^K0 of passes 1..W-1 (and w, when PACK)
  T qw[PACK ? 1 : CAP];
  Q4<T> q2[RED ? CAP : 1];  // pseudo-galaxies: (w g)^3, |w g|^2 w g cell sums
  T qu[RED ? CAP : 1];      // pseudo-galaxies: w^3 cell sum
  double stage[W][NMX * 64];  // per-wave epilogue staging of the binary64 sums
  int rows[2][5][64];       // row table: s1, l1, s2, row length, inclusive prefix
  int cnt[W];               // in-bin count of each wave's chunk in this round
  int cent[2];              // centre broadcast
  // per-bin record maxima of the workgroup (G, W), float bits; binary32
  // records only (the binary64 path does not scale its operands)
  unsigned bmax[2][sizeof(T) == 4 ? FPCF4_NBINS_SUPPORTED : 1];
};

// First powers z^K0 of passes P..W-1, each the previous one times
// z^(K0[P] - K0[P-1]), written to the ring slot of the neighbour.
template <typename T, int N, int P, typename SH>
__device__ __forceinline__ void put_starts(SH& sh, unsigned slot, T zr, T zi, T pr, T pi, T w) {
  if constexpr (P < Conf<T, N>::W) {
    constexpr int D = Conf<T, N>::PP.k0[P] - Conf<T, N>::PP.k0[P - 1];
    T dr, di;
    cpow<T, D>(zr, zi, dr, di);
    T nr = dr, ni = di;   // pass 1 starts at z^D itself
    if constexpr (P > 1) {
      nr = pr * dr - pi * di;
      ni = pr * di + pi * dr;
    }
    if constexpr (SH::PACK) sh.qk[P - 1][slot] = Q4<T>{nr, ni, w, -zi};
    else sh.qk[P - 1][slot] = Q2<T>{nr, ni};
    put_starts<T, N, P + 1>(sh, slot, zr, zi, nr, ni, w);
  }
}

// One wave = one pass (an order range of the accumulators).  The waves of a
// workgroup share the walk: in every round wave w bins chunk (W r + w) of the
// annulus' flat candidate list and forms z and the weights of its in-bin
// neighbours; after a barrier the in-bin counts of all waves are known and
// each wave appends its neighbours to the LDS ring at its prefix offset
// (wave order); after a second barrier every wave adds all complete batches
// of 64 ring slots to its own units.  A remainder below 64 stays in the ring
// for the next round; the last one of a bin is added as a partial batch.
// The order is the same in every wave and every run (no atomics), so
// results are reproducible bit for bit.
template <typename T, int N, int PASS, bool RED>
__device__ __forceinline__ void pass_body(const StageAArgs& a,
                                          Shared<T, Conf<T, N>::W, Conf<T, N>::NMX, RED>& sh,
                                          unsigned lane) {
  // neighbour records: galaxies, or the pseudo-galaxies of reduced catalogues
  using Rec = typename std::conditional<RED, GalR<T>, Gal<T>>::type;
  constexpr int W = Conf<T, N>::W;
  constexpr int K0 = Conf<T, N>::PP.k0[PASS];
  constexpr int K1 = Conf<T, N>::PP.k1[PASS];
  constexpr bool P0 = (PASS == 0);
  constexpr int NUO = ubase(N, K0, K1 + 1);          // order units
  constexpr int NU = NUO + (P0 ? nspecial(N) : 0);
  constexpr int NM = (NU + 63) / 64;
  constexpr int FOLD = Budget<T>::fold;
  static_assert(NM <= Conf<T, N>::NMX, "staging block");

  // centres: the galaxies, or the pseudo-galaxies of a base grid (BaseTree)
  const Gal<T>* __restrict__ gal = reinterpret_cast<const Gal<T>*>(a.cgal);
  const Grid g = a.cat.g;
  constexpr int NO = nord(N);   // record order
  const Layout L = make_layout(NO);
  const int nb = a.nb;

  const int xcd0 = blockIdx.x & 7;
  int xs = 0;          // pass 0: XCD cursor of the centre grab
  constexpr unsigned CAP = Shared<T, W, Conf<T, N>::NMX, RED>::CAP;
  unsigned head = 0, tail = 0;   // ring: appended / consumed neighbours
  auto fetch = [&](unsigned slot) -> Nb<T> {
    const Q4<T> u = sh.q0[slot];
    const Q4<T> v = sh.q1[slot];
    T sr = T(0), si = T(0), ww, nzi = -u.y;
    constexpr bool PK = kPackW<T, RED>;
    if constexpr (PASS > 0 && kRingStarts<T>) {
      const auto k = sh.qk[PASS - 1][slot];
      sr = k.x;
      si = k.y;
      if constexpr (PK) { ww = k.z; nzi = k.w; }
      else ww = sh.qw[slot];
    } else {
      if constexpr (PK) {
        const Q4<T> k = sh.qk[0][slot];
        ww = k.z;
        nzi = k.w;
      } else {
        ww = sh.qw[slot];
      }
    }
    Nb<T> q{u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w, ww, sr, si, nzi};
    if constexpr (RED && PASS == 0) {
      const Q4<T> t = sh.q2[slot];
      q.p3 = t.x;
      q.q3 = t.y;
      q.ea = t.z;
      q.eb = t.w;
      q.u = sh.qu[slot];
    }
    return q;
  };
  unsigned tc = 0;     // centres so far (broadcast-slot parity)
  unsigned tt = 0;     // row tables so far (table parity)
  unsigned long long wave_pairs = 0;
  float lane_xmax = 0.f, lane_wxmax = 0.f;  // lane 0: |w g| and |w| maxima
  if constexpr (sizeof(T) == 4) {
    // cleared before the first barrier of the centre loop orders it
    for (int q = (int)threadIdx.x; q < 2 * FPCF4_NBINS_SUPPORTED; q += (int)blockDim.x)
      sh.bmax[q / FPCF4_NBINS_SUPPORTED][q % FPCF4_NBINS_SUPPORTED] = 0u;
  }

  for (;;) {
    if constexpr (P0) {
      // dynamic centre scheduling: the XCD's own range of the centre list
      // first, then the other XCDs' ranges
      if (lane == 0) {
        int idx = -1;
        while (xs < 8) {
          const int xcd = (xcd0 + xs) & 7;
          const int lo = (int)(((int64_t)a.ncent * xcd) >> 3);
          const int hi = (int)(((int64_t)a.ncent * (xcd + 1)) >> 3);
          const int c = atomicAdd(a.work_counter + xcd, 1);
          if (lo + c < hi) {
            idx = lo + c;
            break;
          }
          ++xs;
        }
        sh.cent[tc & 1] = idx;
      }
    }
    __syncthreads();
    const int idx = __builtin_amdgcn_readfirstlane(sh.cent[tc & 1]);
    ++tc;
    if (idx < 0) break;
    const int i = a.centres[idx];
    const Gal<T> gi = gal[i];
    const double xi = gi.x, yi = gi.y;
    if constexpr (P0 && !RED) {
      if (lane == 0) {
        // centre factors of this tile position
        T* xg = reinterpret_cast<T*>(a.xg);
        xg[2 * idx] = gi.a;
        xg[2 * idx + 1] = gi.b;
        reinterpret_cast<T*>(a.xw)[idx] = gi.w;
        lane_xmax = fmaxf(lane_xmax, (float)fmax(fabs((double)gi.a), fabs((double)gi.b)));
        lane_wxmax = fmaxf(lane_wxmax, (float)fabs((double)gi.w));
      }
    }

    // the launch's bins (discrete or reduced catalogues); the others are left alone
    for (int b = a.b_lo; b < a.b_hi; ++b) {
      const Rec* __restrict__ ngal = reinterpret_cast<const Rec*>(RED ? a.rgal[a.level[b] - 1] : a.cat.gal);
      const int32_t* __restrict__ cstart = RED ? a.rcell[a.level[b] - 1] : a.cat.cell_start;
      const double e2lo = a.e2[b], e2hi = a.e2[b + 1];
      // conservative culling radii and cell margin (binning itself is exact)
      const double rin = a.edges[b] * (1.0 - 1e-9);
      const double rout = a.edges[b + 1] * (1.0 + 1e-9);
      const double dlt = 1e-9 * g.h;
      int cy0 = (int)floor((yi - rout - g.y0) * g.inv_h) - 1;
      int cy1 = (int)floor((yi + rout - g.y0) * g.inv_h) + 1;
      cy0 = imax(cy0, 0);
      cy1 = imin(cy1, g.ncy - 1);
      const int nrows = cy1 - cy0 + 1;

      T acc[NU];
#pragma unroll
      for (int u = 0; u < NU; ++u) acc[u] = T(0);
      double mst[NM];
#pragma unroll
      for (int m = 0; m < NM; ++m) mst[m] = 0.0;
      int nblk = 0;
      int cnt = 0;

      for (int rg = 0; rg < nrows; rg += 64) {
        // ---- row table, one row per lane: segments [s1, s1 + l1) and
        // [s2, s2 + l2) of the sorted catalogue (cells entirely inside the
        // inner circle are skipped).  Wave 0 builds it and publishes it
        // through LDS, so every wave walks the same list and takes the same
        // number of barriers.
        const unsigned tb = tt & 1u;
        ++tt;
        if constexpr (P0) {
          int s1 = 0, l1 = 0, s2 = 0, l2 = 0;
          const int cy = cy0 + rg + (int)lane;
          if (rg + (int)lane < nrows) {
            const double ylo = g.y0 + cy * g.h - dlt;
            const double yhi = g.y0 + (cy + 1) * g.h + dlt;
            const double dymin = fmax(0.0, fmax(ylo - yi, yi - yhi));
            if (dymin < rout) {
              const double hw = sqrt(rout * rout - dymin * dymin) + dlt;
              int cx0 = (int)floor((xi - hw - g.x0) * g.inv_h);
              int cx1 = (int)floor((xi + hw - g.x0) * g.inv_h);
              cx0 = imax(cx0, 0);
              cx1 = imin(cx1, g.ncx - 1);
              if (cx0 <= cx1) {
                const double dymax = fmax(fabs(ylo - yi), fabs(yhi - yi));
                int hx0 = cx1 + 1, hx1 = cx1;
                if (dymax < rin) {
                  const double hwi = sqrt(rin * rin - dymax * dymax) - 2.0 * dlt;
                  hx0 = (int)ceil((xi - hwi - g.x0) * g.inv_h + 1e-7);
                  hx1 = (int)floor((xi + hwi - g.x0) * g.inv_h - 1e-7) - 1;
                  hx0 = imax(hx0, cx0);
                  hx1 = imin(hx1, cx1);
                  if (hx0 > hx1) { hx0 = cx1 + 1; hx1 = cx1; }
                }
                const int32_t* cs = cstart + (int64_t)cy * g.ncx;
                s1 = cs[cx0];
                l1 = cs[hx0] - s1;
                s2 = cs[hx1 + 1];
                l2 = cs[cx1 + 1] - s2;
              }
            }
          }
          const int rl0 = l1 + l2;
          int pe0 = rl0;   // inclusive prefix over rows
#pragma unroll
          for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(pe0, d, 64);
            if ((int)lane >= d) pe0 += t;
          }
          sh.rows[tb][0][lane] = s1;
          sh.rows[tb][1][lane] = l1;
          sh.rows[tb][2][lane] = s2;
          sh.rows[tb][3][lane] = rl0;
          sh.rows[tb][4][lane] = pe0;
        }
        __syncthreads();
        const int s1 = sh.rows[tb][0][lane];
        const int l1 = sh.rows[tb][1][lane];
        const int s2 = sh.rows[tb][2][lane];
        const int rl = sh.rows[tb][3][lane];
        const int pe = sh.rows[tb][4][lane];
        const int ro = pe - rl;   // first flat index of this row
        const int tot = __builtin_amdgcn_readlane(pe, 63);
        const int nch = (tot + 63) >> 6;
        const int rounds = (nch + W - 1) / W;

        // sorted position of flat candidate 64 c + lane (-1 beyond the end)
        auto locate = [&](int c) -> int {
          const int f0 = c << 6;
          const int f = f0 + (int)lane;
          int j = -1;
          unsigned long long m = __ballot(rl > 0 && ro < f0 + 64 && pe > f0);
          while (m) {
            const int r = __builtin_ctzll(m);
            m &= m - 1;
            const int orr = __builtin_amdgcn_readlane(ro, r);
            const int rlr = __builtin_amdgcn_readlane(rl, r);
            const int l1r = __builtin_amdgcn_readlane(l1, r);
            const int s1r = __builtin_amdgcn_readlane(s1, r);
            const int s2r = __builtin_amdgcn_readlane(s2, r);
            const int off = f - orr;
            if (off >= 0 && off < rlr) j = off < l1r ? s1r + off : s2r + (off - l1r);
          }
          return j;
        };

        Rec gn{};
        bool vn = false;
        if (PASS < nch) {
          const int j = locate(PASS);
          if (j >= 0) { gn = ngal[j]; vn = true; }
        }
        for (int r = 0; r < rounds; ++r) {
          // ---- bin this wave's chunk (binary64 r^2, no contraction)
          const Rec gc = gn;
          const bool vc = vn;
          bool inb = false;
          double dx = 0.0, dy = 0.0;
          if (vc) {
            dx = gc.x - xi;
            dy = gc.y - yi;
            const double rr = r2_exact(dx, dy);
            inb = (rr >= e2lo) && (rr < e2hi);
          }
          const unsigned long long mm = __ballot(inb);
          if (lane == 0) sh.cnt[PASS] = (int)__popcll(mm);
          // ---- load the next round's chunk while this round is consumed
          {
            const int cn = (r + 1) * W + PASS;
            vn = false;
            if (cn < nch) {
              const int j = locate(cn);
              if (j >= 0) { gn = ngal[j]; vn = true; }
            }
          }
          __syncthreads();
          // ---- append this wave's in-bin neighbours at its prefix offset
          int before = 0, added = 0;
#pragma unroll
          for (int w = 0; w < W; ++w) {
            const int cw = __builtin_amdgcn_readfirstlane(sh.cnt[w]);
            if (w < PASS) before += cw;
            added += cw;
          }
          if (inb) {
            const unsigned slot = (head + (unsigned)before + rank_in_mask(mm)) & (CAP - 1);
            const T ex = (T)dx, ey = (T)dy;
            const T inv = rsq<T>(ex * ex + ey * ey);
            const T va = gc.a, vb = gc.b, vw = gc.w;
            const T zr = ex * inv, zi = ey * inv;
            sh.q0[slot] = Q4<T>{zr, zi, va, vb};
            if constexpr (RED) {
              sh.q1[slot] = Q4<T>{gc.c, gc.d, gc.e, gc.v};
              sh.q2[slot] = Q4<T>{gc.p3, gc.q3, gc.ea, gc.eb};
              sh.qu[slot] = gc.u;
            }
            if constexpr (kRingStarts<T> && W > 1) put_starts<T, N, 1>(sh, slot, zr, zi, T(1), T(0), vw);
            else if constexpr (kPackW<T, RED>) sh.qk[0][slot] = Q4<T>{T(0), T(0), vw, -zi};
            if constexpr (!RED) sh.q1[slot] = Q4<T>{va * va - vb * vb, T(2) * va * vb, va * va + vb * vb, vw * vw};
            if constexpr (!kPackW<T, RED>) sh.qw[slot] = vw;
          }
          head += (unsigned)added;
          cnt += added;
          __syncthreads();
          // ---- every pass adds the complete batches
          while (head - tail >= 64u) {
            // batches start on multiples of 64 (the ring is realigned at the
            // end of every bin), so a batch never wraps around the ring
            __builtin_assume((tail & 63u) == 0u);
            add_pair<T, N, K0, K1, P0, NUO, RED>(acc, true, fetch((tail & (CAP - 1)) + lane));
            tail += 64u;
            if (++nblk == FOLD) {
              fold_all<T, NU, NM>(acc, mst, lane);
#pragma unroll
              for (int u = 0; u < NU; ++u) acc[u] = T(0);
              nblk = 0;
            }
          }
        }
      }
      if (head != tail) {
        const bool valid = lane < head - tail;
        Nb<T> q{};
        __builtin_assume((tail & 63u) == 0u);
        if (valid) q = fetch((tail & (CAP - 1)) + lane);
        add_pair<T, N, K0, K1, P0, NUO, RED>(acc, valid, q);
      }
      // realign the ring: the next bin's first batch starts on a multiple of 64
      head = (head + 63u) & ~63u;
      tail = head;
      fold_all<T, NU, NM>(acc, mst, lane);

      // ---- epilogue: masters -> LDS -> record blocks of this pass
      double* S = sh.stage[PASS];
#pragma unroll
      for (int m = 0; m < NM; ++m) S[64 * m + lane] = mst[m];
      wave_sync();
      T* rec = reinterpret_cast<T*>(a.rec_aos);
      float gmax = 0.f, wmax = 0.f;   // block maxima for the fp16 operand scaling
      auto su = [&](int f, int k, int part) -> double {
        if (k == 0 && part == 1) return 0.0;
        return (double)chain_sign(k - K0) * S[uidx(N, K0, f, k) + part];
      };
      for (int e = (int)lane; e < L.mpc; e += 64) {
        double re = 0.0, im = 0.0;
        bool mine = false;
        // orders the plan does not form (3PCF plan) are written as zeros by pass 0
        if (e < L.offW) {                       // G_k
          const int k = e - (2 * NO + 3);
          const int ko = k < 0 ? -k : k;
          if (ko > kmax_f(N, FA)) {
            mine = P0;
          } else if (ko >= K0 && ko <= K1) {
            mine = true;
            const double ar = su(FA, ko, 0), ai = su(FA, ko, 1);
            const double br = su(FB, ko, 0), bi = su(FB, ko, 1);
            if (k >= 0) { re = ar - bi; im = ai + br; }
            else        { re = ar + bi; im = br - ai; }
          }
        } else if (e < L.offQ) {                // W_k
          const int k = e - L.offW - 2 * NO;
          const int ko = k < 0 ? -k : k;
          if (ko > kmax_f(N, FW)) {
            mine = P0;
          } else if (ko >= K0 && ko <= K1) {
            mine = true;
            re = su(FW, ko, 0);
            im = (k >= 0 ? 1.0 : -1.0) * su(FW, ko, 1);
          }
        } else if (e < L.offA) {                // Q_k
          const int k = e - L.offQ + L.qlo;
          const int ko = k < 0 ? -k : k;
          if (ko > kmax_f(N, FC)) {
            mine = P0;
          } else if (ko >= K0 && ko <= K1) {
            mine = true;
            const double cr = su(FC, ko, 0), ci = su(FC, ko, 1);
            const double dr = su(FD, ko, 0), di = su(FD, ko, 1);
            if (k >= 0) { re = cr - di; im = ci + dr; }
            else        { re = cr + di; im = dr - ci; }
          }
        } else if (e < L.offV) {                // A_k, k >= 0
          const int k = e - L.offA;
          if (k > kmax_f(N, FE)) mine = P0;
          else if (k >= K0 && k <= K1) { mine = true; re = su(FE, k, 0); im = su(FE, k, 1); }
        } else if (e < L.offS) {                // V_k, k >= 0
          const int k = e - L.offV;
          if (k > kmax_f(N, FV)) mine = P0;
          else if (k >= K0 && k <= K1) { mine = true; re = su(FV, k, 0); im = su(FV, k, 1); }
        } else if (P0 && is3(N)) {              // no triple-counting blocks in the 3PCF plan
          mine = true;
        } else if (P0) {                        // T_-8, T_-4, M_-4, M_0, U
          const int sp = e - L.offS;
          mine = true;
          const double* X = S + NUO;
          if (sp == S_T8)      { re = X[0] + X[3];  im = X[2] - X[1]; }
          else if (sp == S_T4) { re = X[4] + X[7];  im = X[6] - X[5]; }
          else if (sp == S_M4) { re = X[8] + X[11]; im = X[10] - X[9]; }
          else if (sp == S_M0) { re = X[12];        im = X[13]; }
          else                 { re = X[14];        im = 0.0; }
        }
        if (mine) {
          const int64_t o = 2 * (((int64_t)idx * nb + b) * L.mpc + e);
          rec[o] = (T)re;
          rec[o + 1] = (T)im;
          const float mx = (float)fmax(fabs(re), fabs(im));
          if (e < L.offW) gmax = fmaxf(gmax, mx);
          else if (e < L.offQ) wmax = fmaxf(wmax, mx);
        }
      }
      if constexpr (sizeof(T) == 4) {
        if (a.maxima != nullptr) {
#pragma unroll
          for (int d = 32; d >= 1; d >>= 1) {
            gmax = fmaxf(gmax, __shfl_xor(gmax, d, 64));
            wmax = fmaxf(wmax, __shfl_xor(wmax, d, 64));
          }
          if (lane == 0) {
            atomicMax(&sh.bmax[0][b], __float_as_uint(gmax));
            atomicMax(&sh.bmax[1][b], __float_as_uint(wmax));
          }
        }
      }
      if (P0) {
        if (a.counts != nullptr && lane == 0) a.counts[(int64_t)idx * nb + b] = cnt;
        wave_pairs += (unsigned long long)cnt;
      }
      wave_sync();
    }
  }
  if (P0 && a.pairs != nullptr && lane == 0 && wave_pairs) atomicAdd(a.pairs, wave_pairs);
  if constexpr (sizeof(T) == 4) {
    if (a.maxima != nullptr) {
      // every wave left the centre loop after the same barrier, so the
      // workgroup's LDS maxima are complete
      for (int q = (int)threadIdx.x; q < nb; q += (int)blockDim.x) {
        atomicMax(a.maxima + MAXIMA_G + q, sh.bmax[0][q]);
        atomicMax(a.maxima + MAXIMA_W + q, sh.bmax[1][q]);
      }
      if (P0 && lane == 0) {
        atomicMax(a.maxima + MAXIMA_X, __float_as_uint(lane_xmax));
        atomicMax(a.maxima + MAXIMA_X + 1, __float_as_uint(lane_wxmax));
      }
    }
  }
}

template <typename T, int N, int P, bool RED>
__device__ __forceinline__ void dispatch(int wv, const StageAArgs& a,
                                         Shared<T, Conf<T, N>::W, Conf<T, N>::NMX, RED>& sh, unsigned lane) {
  if constexpr (P < Conf<T, N>::W) {
    if (wv == P) pass_body<T, N, P, RED>(a, sh, lane);
    else dispatch<T, N, P + 1, RED>(wv, a, sh, lane);
  }
}

// RED: neighbours from the reduced catalogues of the tree approximation
// (binary32 only); the launch accumulates the bins [a.b_lo, a.b_hi).
template <typename T, int N, bool RED>
__global__ __launch_bounds__((64 * Conf<T, N>::W)) __attribute__((amdgpu_waves_per_eu(Conf<T, N>::EU))) void stage_a_kernel(StageAArgs a) {
  __shared__ Shared<T, Conf<T, N>::W, Conf<T, N>::NMX, RED> sh;
  // wave index as a scalar, so each wave branches to its own pass only
  const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  dispatch<T, N, 0, RED>(wv, a, sh, lane_id());
}

// [centre][bin][entry] (as written per centre) -> [entry][bin][centre], for
// binary32 records.  A workgroup takes relayout_centres<T>() consecutive
// centres (256 bytes of every output row) and walks the bins: each
// (centre, bin) row of mpc entries is read whole, and the next bin's row
// continues where it ended, so every fetched line is used; rows are staged
// in LDS with a stride of relayout_row<T>(mpc) entries, which spreads the
// column reads of the write phase over the banks.
template <typename T>
__host__ __device__ constexpr int relayout_centres() { return 256 / (2 * (int)sizeof(T)); }
template <typename T>
__host__ __device__ constexpr int relayout_row(int mpc) {
  constexpr int P = sizeof(T) == 4 ? 16 : 8;
  return mpc + (((1 - mpc) % P) + P) % P;
}

template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ src, T* __restrict__ dst,
                                                        int ncent, int nb, int mpc, int ldc) {
  using V = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
  constexpr int CT = relayout_centres<T>();
  constexpr int EPI = 256 / CT;   // output rows written per pass of the workgroup
  extern __shared__ __align__(16) unsigned char relayout_lds[];
  V* tile = reinterpret_cast<V*>(relayout_lds);
  const int row = relayout_row<T>(mpc);
  const int t = threadIdx.x;
  const int c0 = blockIdx.x * CT;
  const int nc = min(CT, ncent - c0);
  const V* vsrc = reinterpret_cast<const V*>(src);
  V* vdst = reinterpret_cast<V*>(dst);
  const int cl = t % CT, ej = t / CT;
  // flat index f = c mpc + e over the workgroup's rows of one bin; thread t
  // takes f = t, t + 256, ..., eight loads in flight at a time
  const int total = nc * mpc, q = 256 / mpc, rm = 256 % mpc;
  for (int b = 0; b < nb; ++b) {
    int c = t / mpc, e = t % mpc;
    for (int f0 = t; f0 < total; f0 += 8 * 256) {
      V v[8];
      int cc[8], ee[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        cc[i] = c;
        ee[i] = e;
        if (f0 + 256 * i < total) v[i] = vsrc[((int64_t)(c0 + c) * nb + b) * mpc + e];
        c += q;
        e += rm;
        if (e >= mpc) {
          e -= mpc;
          ++c;
        }
      }
#pragma unroll
      for (int i = 0; i < 8; ++i)
        if (f0 + 256 * i < total) tile[cc[i] * row + ee[i]] = v[i];
    }
    __syncthreads();
    if (cl < nc) {
      for (int ew = ej; ew < mpc; ew += EPI) vdst[((int64_t)ew * nb + b) * ldc + c0 + cl] = tile[cl * row + ew];
    }
    __syncthreads();
  }
}

// The same relayout through a 64 x 64 LDS tile of (centre, entry) per bin,
// both sides coalesced.  Taken for binary64 records, where it measured
// faster than the row-wise form (17.5 vs 22.4 ms at 1e6 centres, 12 bins,
// nmax 10; binary32: 9.8 vs 6.7 ms the other way round).
template <typename T>
__global__ __launch_bounds__(256) void transpose_tile_kernel(const T* __restrict__ src, T* __restrict__ dst,
                                                        int ncent, int nb, int mpc, int ldc) {
  __shared__ T tile[64][65][2];
  const int c0 = blockIdx.x * 64, b = blockIdx.y, e0 = blockIdx.z * 64;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int f = threadIdx.x + 256 * i;
    const int cl = f >> 6, el = f & 63;
    const int c = c0 + cl, e = e0 + el;
    T re = T(0), im = T(0);
    if (c < ncent && e < mpc) {
      const T* p = src + 2 * (((int64_t)c * nb + b) * mpc + e);
      re = p[0];
      im = p[1];
    }
    tile[cl][el][0] = re;
    tile[cl][el][1] = im;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int f = threadIdx.x + 256 * i;
    const int el = f >> 6, cl = f & 63;
    const int c = c0 + cl, e = e0 + el;
    if (c < ncent && e < mpc) {
      T* p = dst + 2 * (((int64_t)e * nb + b) * ldc + c);
      p[0] = tile[cl][el][0];
      p[1] = tile[cl][el][1];
    }
  }
}

template <typename T, int N, bool RED>
static int resident_blocks() {
  // persistent workgroups: as many as are resident at once
  static int resident = -1;
  if (resident < 0) {
    int per_cu = 0, dev = 0, ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, stage_a_kernel<T, N, RED>,
                                                     64 * Conf<T, N>::W, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
      ncu = 256;
    resident = per_cu * ncu;
  }
  return resident;
}

template <typename T, int N, bool RED>
static hipError_t launch_pairs(const StageAArgs& a, hipStream_t s) {
  // a multiple of the 8 XCDs (blocks are dealt round-robin to the XCDs)
  const int resident = resident_blocks<T, N, RED>();
  int nblocks = a.ncent < resident ? a.ncent : resident;
  nblocks = ((nblocks + 7) / 8) * 8;
  if (nblocks < 8) nblocks = 8;
  hipLaunchKernelGGL((stage_a_kernel<T, N, RED>), dim3(nblocks), dim3(64 * Conf<T, N>::W), 0, s, a);
  return hipGetLastError();
}

// The discrete bins (level 0) in one launch and, with the tree
// approximation, the bins on reduced catalogues in a second one (its own
// scheduling counters); then the relayout of all records.
template <typename T, int N>
hipError_t launch_n(const StageAArgs& a, hipStream_t s, int* nlaunch, hipEvent_t mid) {
  // the level of a bin never decreases with its radius, so the discrete bins
  // are a prefix of [b_lo, b_hi) and the reduced ones the rest
  int k = a.b_lo;
  while (k < a.b_hi && a.level[k] == 0) ++k;
  for (int b = k; b < a.b_hi; ++b)
    if (a.level[b] == 0) return hipErrorInvalidValue;
  const bool red = k < a.b_hi;
  StageAArgs ae = a, ar = a;
  ae.b_hi = k;
  ar.b_lo = k;
  *nlaunch = 0;
  hipError_t e = launch_pairs<T, N, false>(ae, s);
  if (e != hipSuccess) return e;
  *nlaunch = 1;
  if (red) {
    if constexpr (sizeof(T) == 4) {
      ar.work_counter = a.work_counter + 8;
      if ((e = launch_pairs<T, N, true>(ar, s)) != hipSuccess) return e;
      *nlaunch = 2;
    } else {
      return hipErrorInvalidValue;   // reduced catalogues: binary32 only
    }
  }
  if (mid != nullptr && (e = hipEventRecord(mid, s)) != hipSuccess) return e;
  const int mpc = make_layout(nord(N)).mpc;
  if constexpr (sizeof(T) == 4) {
    constexpr int CT = relayout_centres<T>();
    const size_t lds = (size_t)CT * relayout_row<T>(mpc) * 2 * sizeof(T);   // <= 61.7 KB at mpc 239
    hipLaunchKernelGGL(transpose_kernel<T>, dim3((a.ncent + CT - 1) / CT), dim3(256), lds, s,
                       reinterpret_cast<const T*>(a.rec_aos), reinterpret_cast<T*>(a.rec), a.ncent, a.nb, mpc,
                       a.ldc);
  } else {
    const dim3 grid((a.ncent + 63) / 64, a.nb, (mpc + 63) / 64);
    hipLaunchKernelGGL(transpose_tile_kernel<T>, grid, dim3(256), 0, s, reinterpret_cast<const T*>(a.rec_aos),
                       reinterpret_cast<T*>(a.rec), a.ncent, a.nb, mpc, a.ldc);
  }
  return hipGetLastError();
}

}  // namespace sa

#if defined(FPCF4_STAGE_A_N)
// One translation unit per nmax keeps the (large, fully unrolled) kernels
// compiling in parallel.
template hipError_t sa::launch_n<float, FPCF4_STAGE_A_N>(const StageAArgs&, hipStream_t, int*, hipEvent_t);
template hipError_t sa::launch_n<double, FPCF4_STAGE_A_N>(const StageAArgs&, hipStream_t, int*, hipEvent_t);
template hipError_t sa::launch_n<float, sa::PLAN3 + FPCF4_STAGE_A_N>(const StageAArgs&, hipStream_t, int*, hipEvent_t);
template hipError_t sa::launch_n<double, sa::PLAN3 + FPCF4_STAGE_A_N>(const StageAArgs&, hipStream_t, int*, hipEvent_t);
#else
namespace sa {
#define FPCF4_DECL_N(NN)                                                         \
  extern template hipError_t launch_n<float, NN>(const StageAArgs&, hipStream_t, int*, hipEvent_t); \
  extern template hipError_t launch_n<double, NN>(const StageAArgs&, hipStream_t, int*, hipEvent_t); \
  extern template hipError_t launch_n<float, PLAN3 + NN>(const StageAArgs&, hipStream_t, int*, hipEvent_t); \
  extern template hipError_t launch_n<double, PLAN3 + NN>(const StageAArgs&, hipStream_t, int*, hipEvent_t);
FPCF4_DECL_N(0) FPCF4_DECL_N(1) FPCF4_DECL_N(2) FPCF4_DECL_N(3) FPCF4_DECL_N(4)
FPCF4_DECL_N(5) FPCF4_DECL_N(6) FPCF4_DECL_N(7) FPCF4_DECL_N(8) FPCF4_DECL_N(9)
FPCF4_DECL_N(10) FPCF4_DECL_N(11) FPCF4_DECL_N(12) FPCF4_DECL_N(13) FPCF4_DECL_N(14)
FPCF4_DECL_N(15) FPCF4_DECL_N(16)
#undef FPCF4_DECL_N
}  // namespace sa

template <typename T>
hipError_t launch_stage_a(int nmax, int order, const StageAArgs& a, hipStream_t s, int* nlaunch, hipEvent_t mid) {
  switch (nmax) {
#define FPCF4_CASE(NN) \
  case NN: return order == 3 ? sa::launch_n<T, sa::PLAN3 + NN>(a, s, nlaunch, mid) : sa::launch_n<T, NN>(a, s, nlaunch, mid);
    FPCF4_CASE(0) FPCF4_CASE(1) FPCF4_CASE(2) FPCF4_CASE(3) FPCF4_CASE(4)
    FPCF4_CASE(5) FPCF4_CASE(6) FPCF4_CASE(7) FPCF4_CASE(8) FPCF4_CASE(9)
    FPCF4_CASE(10) FPCF4_CASE(11) FPCF4_CASE(12) FPCF4_CASE(13) FPCF4_CASE(14)
    FPCF4_CASE(15) FPCF4_CASE(16)
#undef FPCF4_CASE
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_stage_a<float>(int, int, const StageAArgs&, hipStream_t, int*, hipEvent_t);
template hipError_t launch_stage_a<double>(int, int, const StageAArgs&, hipStream_t, int*, hipEvent_t);
#endif

}  // namespace fpcf4
