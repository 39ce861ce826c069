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
//  * one wavefront owns one centre at a time (dynamic per-XCD queues, with
//    stealing, over a Morton-ordered centre list);
//  * for each bin the wave walks the rows of the cell grid that intersect
//    the annulus (row bounds computed lane-parallel, one row per lane); the
//    64 lanes load 64 consecutive neighbours (coalesced SoA), form r^2 in
//    binary64 without contraction and test the bin against the squared
//    edges -- the same arithmetic as the oracle, so binning is bit-exact;
//  * in-bin neighbours are compacted with a ballot into a wave-private LDS
//    ring; every full batch of 64 is consumed with all lanes busy: each
//    lane computes z, its power chain z^k and accumulates its own partial
//    sums in registers;
//  * the accumulators of a pass cover an order range [K0, K1] sized to the
//    register file; several passes cover all orders;
//  * partial sums are combined across lanes by a transposing butterfly
//    (log2 64 levels, halving the live values per level), so each lane ends
//    with complete sums of its own units; the binary32 variant folds into
//    binary64 masters every few batches (blocked summation).
#include "fpcf4_internal.hpp"

namespace fpcf4 {
namespace sa {

enum { FA = 0, FB, FC, FD, FW, FE, FV, NF };
constexpr int NSPECIAL = 15;  // P8, Q8, P4, Q4, EA4, EB4 (complex); EA0, EB0, U (real)

__host__ __device__ constexpr int kmax_f(int n, int f) {
  return (f == FA || f == FB) ? 2 * n + 3
       : (f == FC || f == FD) ? imax(2 * n + 5, n + 6)
       : (f == FE)            ? imax(2 * n + 1, n + 2)
                              : 2 * n;
}
__host__ __device__ constexpr int ktop(int n) { return imax(2 * n + 5, n + 6); }
__host__ __device__ constexpr int units_at(int n, int k) {
  int u = 0;
  for (int f = 0; f < NF; ++f)
    if (k <= kmax_f(n, f)) u += (k == 0 ? 1 : 2);
  return u;
}
__host__ __device__ constexpr int total_units(int n) {
  int u = NSPECIAL;
  for (int k = 0; k <= ktop(n); ++k) u += units_at(n, k);
  return u;
}
// Greedy split of the orders 0..ktop into passes of at most `cap` units;
// pass 0 also holds the 15 special units (orders 0, 4, 8 of the triple
// blocks, accumulated from z^4 and z^8 formed by squaring).  which: 0 = first
// order of pass p, 1 = last order of pass p, 2 = number of passes.
__host__ __device__ constexpr int greedy(int n, int cap, int p, int which) {
  int np = 0, k = 0;
  while (k <= ktop(n)) {
    int used = (np == 0) ? NSPECIAL : 0;
    const int start = k;
    while (k <= ktop(n) && (k == start || used + units_at(n, k) <= cap)) {
      used += units_at(n, k);
      ++k;
    }
    if (np == p && which < 2) return which == 0 ? start : k - 1;
    ++np;
  }
  return which == 2 ? np : -1;
}
// Fewest passes within the register budget, then the smallest cap that
// still needs no more passes (balanced passes).
__host__ __device__ constexpr int plan_cap(int n, int budget) {
  const int np = greedy(n, budget, 0, 2);
  int cap = (total_units(n) + np - 1) / np;
  while (greedy(n, cap, 0, 2) > np) ++cap;
  return cap;
}
__host__ __device__ constexpr int plan_np(int n, int budget) { return greedy(n, plan_cap(n, budget), 0, 2); }
__host__ __device__ constexpr int plan_k(int n, int budget, int p, int which) {
  return greedy(n, plan_cap(n, budget), p, which);
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
template <> struct Budget<float> { static constexpr int units = 150; static constexpr int fold = 32; };
template <> struct Budget<double> { static constexpr int units = 84; static constexpr int fold = 1 << 30; };

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

constexpr int QCAP = 128;

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

template <typename T, int N, int K0, int K1, int K>
__device__ __forceinline__ void acc_orders(T* acc, const T* val, T pr, T pi, T zr, T zi) {
  acc_fields<T, N, K0, K1, K, 0>(acc, val, pr, pi);
  if constexpr (K < K1) {
    const T tr = pr * zr - pi * zi;
    const T ti = pr * zi + pi * zr;
    acc_orders<T, N, K0, K1, K + 1>(acc, val, tr, ti, zr, zi);
  }
}

template <typename T, int E>
__device__ __forceinline__ void cpow(T zr, T zi, T& pr, T& pi) {
  pr = T(1);
  pi = T(0);
  T br = zr, bi = zi;
  int e = E;
#pragma unroll
  for (int it = 0; it < 6; ++it) {
    if (e & 1) {
      const T tr = pr * br - pi * bi;
      pi = pr * bi + pi * br;
      pr = tr;
    }
    e >>= 1;
    if (e) {
      const T tr = br * br - bi * bi;
      bi = T(2) * br * bi;
      br = tr;
    }
  }
}

template <typename T, int N, int PASS>
__global__ __launch_bounds__(256) void stage_a_kernel(StageAArgs a) {
  constexpr int BU = Budget<T>::units;
  constexpr int K0 = plan_k(N, BU, PASS, 0);
  constexpr int K1 = plan_k(N, BU, PASS, 1);
  constexpr bool P0 = (PASS == 0);
  constexpr int NUO = ubase(N, K0, K1 + 1);          // order units
  constexpr int NU = NUO + (P0 ? NSPECIAL : 0);
  constexpr int NM = (NU + 63) / 64;
  constexpr int FOLD = Budget<T>::fold;

  // queue of in-bin neighbours: separation and weights (w g1, w g2, w)
  __shared__ T q_dx[4][QCAP];
  __shared__ T q_dy[4][QCAP];
  __shared__ T q_va[4][QCAP];
  __shared__ T q_vb[4][QCAP];
  __shared__ T q_vw[4][QCAP];
  __shared__ double stage[4][NM * 64];

  const unsigned lane = lane_id();
  const int wv = threadIdx.x >> 6;
  const SortedCat& cat = a.cat;
  const Grid g = cat.g;
  const Layout L = make_layout(N);
  const int nb = a.nb;

  const int xcd0 = blockIdx.x & 7;
  int32_t* counters = a.work_counter + 8 * PASS;
  // per-wave running totals, flushed with one atomic each when the wave ends
  unsigned long long wave_pairs = 0;
  float lane_gmax = 0.f, lane_wmax = 0.f;   // lane b: maxima of bin b
  float lane_xmax = 0.f, lane_wxmax = 0.f;  // lane 0: |w g| and |w| maxima

  for (int xs = 0; xs < 8; ++xs) {
    const int xcd = (xcd0 + xs) & 7;
    const int lo = (int)(((int64_t)a.ncent * xcd) >> 3);
    const int hi = (int)(((int64_t)a.ncent * (xcd + 1)) >> 3);
    for (;;) {
      int c = 0;
      if (lane == 0) c = atomicAdd(counters + xcd, 1);
      c = __shfl(c, 0, 64);
      const int idx = lo + c;
      if (idx >= hi) break;
      const int i = a.centres[idx];
      const double xi = cat.x[i];
      const double yi = cat.y[i];

      for (int b = 0; b < nb; ++b) {
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
        unsigned head = 0, tail = 0;
        int nblk = 0;
        int cnt = 0;

        auto consume = [&](unsigned m) {
          const bool valid = lane < m;
          const unsigned e = (head + lane) & (QCAP - 1);
          T dx = T(0), dy = T(0), va = T(0), vb = T(0), vw = T(0);
          if (valid) {
            dx = q_dx[wv][e];
            dy = q_dy[wv][e];
            va = q_va[wv][e];
            vb = q_vb[wv][e];
            vw = q_vw[wv][e];
          }
          T val[NF];
          val[FA] = va;
          val[FB] = vb;
          val[FC] = va * va - vb * vb;
          val[FD] = T(2) * va * vb;
          val[FW] = vw;
          val[FE] = va * va + vb * vb;
          val[FV] = vw * vw;
          const T inv = valid ? rsq<T>(dx * dx + dy * dy) : T(0);
          const T zr = dx * inv, zi = dy * inv;
          T pr, pi;
          cpow<T, K0>(zr, zi, pr, pi);
          acc_orders<T, N, K0, K1, K0>(acc, val, pr, pi, zr, zi);
          if constexpr (P0) {
            // triple-counting blocks: T_-8, T_-4 (weight (w g)^3), M_-4, M_0
            // (weight |w g|^2 w g) and U (weight w^3)
            const T z2r = zr * zr - zi * zi, z2i = T(2) * zr * zi;
            const T z4r = z2r * z2r - z2i * z2i, z4i = T(2) * z2r * z2i;
            const T z8r = z4r * z4r - z4i * z4i, z8i = T(2) * z4r * z4i;
            const T p3 = val[FC] * va - val[FD] * vb;   // Re (w g)^3
            const T q3 = val[FC] * vb + val[FD] * va;   // Im (w g)^3
            const T ea = val[FE] * va, eb = val[FE] * vb;
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
            acc[NUO + 14] += vw * val[FV];
          }
        };

        // ---- walk the annulus: row groups of 64, one row per lane
        for (int rg = 0; rg < nrows; rg += 64) {
          int s1 = 0, t1 = 0, s2 = 0, t2 = 0;
          {
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
                  // cells entirely inside the inner circle are skipped
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
                  const int32_t* cs = cat.cell_start + (int64_t)cy * g.ncx;
                  s1 = cs[cx0];
                  t1 = cs[hx0];
                  s2 = cs[hx1 + 1];
                  t2 = cs[cx1 + 1];
                }
              }
            }
          }
          const int rend = imin(64, nrows - rg);
          // Flat walk over the row segments in batches of 64 neighbours; the
          // positions and weights of the next batch are loaded while the
          // current one is binned (and possibly consumed).
          auto find = [&](int k, int& sk, int& base, int& end) -> bool {
            for (; k < 2 * rend; ++k) {
              const int r = k >> 1;
              const int sv = __builtin_amdgcn_readlane((k & 1) ? s2 : s1, r);
              const int tv = __builtin_amdgcn_readlane((k & 1) ? t2 : t1, r);
              if (sv < tv) {
                sk = k;
                base = sv;
                end = tv;
                return true;
              }
            }
            return false;
          };
          auto fetch = [&](int bs, int en, double& px, double& py, T& pa, T& pb, T& pw) {
            const int j = bs + (int)lane;
            if (j < en) {
              px = cat.x[j];
              py = cat.y[j];
              pa = (T)cat.fa[j];
              pb = (T)cat.fb[j];
              pw = (T)cat.fw[j];
            }
          };
          int sk = 0, base = 0, end = 0;
          bool have = find(0, sk, base, end);
          double cx = 0.0, cy = 0.0;
          T ca = T(0), cb = T(0), cw = T(0);
          if (have) fetch(base, end, cx, cy, ca, cb, cw);
          while (have) {
            int nk = sk, nbase = base + 64, nend = end;
            bool nhave = true;
            if (nbase >= nend) nhave = find(sk + 1, nk, nbase, nend);
            double nx = 0.0, ny = 0.0;
            T na = T(0), nbv = T(0), nw = T(0);
            if (nhave) fetch(nbase, nend, nx, ny, na, nbv, nw);

            bool inb = false;
            double dx = 0.0, dy = 0.0;
            if (base + (int)lane < end) {
              dx = cx - xi;
              dy = cy - yi;
              const double rr = r2_exact(dx, dy);
              inb = (rr >= e2lo) && (rr < e2hi);
            }
            const unsigned long long m = __ballot(inb);
            if (inb) {
              const unsigned pos = (tail + rank_in_mask(m)) & (QCAP - 1);
              q_dx[wv][pos] = (T)dx;
              q_dy[wv][pos] = (T)dy;
              q_va[wv][pos] = ca;
              q_vb[wv][pos] = cb;
              q_vw[wv][pos] = cw;
            }
            const unsigned nadd = (unsigned)__popcll(m);
            tail += nadd;
            cnt += (int)nadd;
            if (tail - head >= 64) {
              wave_sync();
              consume(64u);
              head += 64;
              if (++nblk == FOLD) {
                fold_all<T, NU, NM>(acc, mst, lane);
#pragma unroll
                for (int u = 0; u < NU; ++u) acc[u] = T(0);
                nblk = 0;
              }
              wave_sync();
            }
            cx = nx; cy = ny; ca = na; cb = nbv; cw = nw;
            sk = nk; base = nbase; end = nend; have = nhave;
          }
        }
        if (tail != head) {
          wave_sync();
          consume(tail - head);
        }
        fold_all<T, NU, NM>(acc, mst, lane);

        // ---- epilogue: masters -> LDS -> record blocks of this pass
#pragma unroll
        for (int m = 0; m < NM; ++m) stage[wv][64 * m + lane] = mst[m];
        wave_sync();
        const double* S = stage[wv];
        T* rec = reinterpret_cast<T*>(a.rec_aos);
        float gmax = 0.f, wmax = 0.f;   // block maxima for the fp16 operand scaling
        auto su = [&](int f, int k, int part) -> double {
          if (k == 0 && part == 1) return 0.0;
          return S[uidx(N, K0, f, k) + part];
        };
        for (int e = (int)lane; e < L.mpc; e += 64) {
          double re = 0.0, im = 0.0;
          bool mine = false;
          if (e < L.offW) {                       // G_k
            const int k = e - (2 * N + 3);
            const int ko = k < 0 ? -k : k;
            if (ko >= K0 && ko <= K1) {
              mine = true;
              const double ar = su(FA, ko, 0), ai = su(FA, ko, 1);
              const double br = su(FB, ko, 0), bi = su(FB, ko, 1);
              if (k >= 0) { re = ar - bi; im = ai + br; }
              else        { re = ar + bi; im = br - ai; }
            }
          } else if (e < L.offQ) {                // W_k
            const int k = e - L.offW - 2 * N;
            const int ko = k < 0 ? -k : k;
            if (ko >= K0 && ko <= K1) {
              mine = true;
              re = su(FW, ko, 0);
              im = (k >= 0 ? 1.0 : -1.0) * su(FW, ko, 1);
            }
          } else if (e < L.offA) {                // Q_k
            const int k = e - L.offQ + L.qlo;
            const int ko = k < 0 ? -k : k;
            if (ko >= K0 && ko <= K1) {
              mine = true;
              const double cr = su(FC, ko, 0), ci = su(FC, ko, 1);
              const double dr = su(FD, ko, 0), di = su(FD, ko, 1);
              if (k >= 0) { re = cr - di; im = ci + dr; }
              else        { re = cr + di; im = dr - ci; }
            }
          } else if (e < L.offV) {                // A_k, k >= 0
            const int k = e - L.offA;
            if (k >= K0 && k <= K1) { mine = true; re = su(FE, k, 0); im = su(FE, k, 1); }
          } else if (e < L.offS) {                // V_k, k >= 0
            const int k = e - L.offV;
            if (k >= K0 && k <= K1) { mine = true; re = su(FV, k, 0); im = su(FV, k, 1); }
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
            const float m = (float)fmax(fabs(re), fabs(im));
            if (e < L.offW) gmax = fmaxf(gmax, m);
            else if (e < L.offQ) wmax = fmaxf(wmax, m);
          }
        }
        if (a.maxima != nullptr) {
#pragma unroll
          for (int d = 32; d >= 1; d >>= 1) {
            gmax = fmaxf(gmax, __shfl_xor(gmax, d, 64));
            wmax = fmaxf(wmax, __shfl_xor(wmax, d, 64));
          }
          if ((int)lane == b) {
            lane_gmax = fmaxf(lane_gmax, gmax);
            lane_wmax = fmaxf(lane_wmax, wmax);
          }
        }
        if (P0 && b == 0 && lane == 0) {
          // centre factors of this tile position
          const double fa_i = cat.fa[i], fb_i = cat.fb[i], fw_i = cat.fw[i];
          T* xg = reinterpret_cast<T*>(a.xg);
          xg[2 * idx] = (T)fa_i;
          xg[2 * idx + 1] = (T)fb_i;
          reinterpret_cast<T*>(a.xw)[idx] = (T)fw_i;
          lane_xmax = fmaxf(lane_xmax, (float)fmax(fabs(fa_i), fabs(fb_i)));
          lane_wxmax = fmaxf(lane_wxmax, (float)fabs(fw_i));
        }
        if (P0) {
          if (a.counts != nullptr && lane == 0) a.counts[(int64_t)idx * nb + b] = cnt;
          wave_pairs += (unsigned long long)cnt;
        }
        wave_sync();
      }
    }
  }
  if (P0 && a.pairs != nullptr && lane == 0 && wave_pairs) atomicAdd(a.pairs, wave_pairs);
  if (a.maxima != nullptr) {
    if ((int)lane < nb) {
      atomicMax(a.maxima + lane, __float_as_uint(lane_gmax));
      atomicMax(a.maxima + 16 + lane, __float_as_uint(lane_wmax));
    }
    if (P0 && lane == 0) {
      atomicMax(a.maxima + 32, __float_as_uint(lane_xmax));
      atomicMax(a.maxima + 33, __float_as_uint(lane_wxmax));
    }
  }
}

template <typename T, int N, int P>
hipError_t launch_passes(const StageAArgs& a, hipStream_t s, int nblocks) {
  constexpr int NP = plan_np(N, Budget<T>::units);
  if constexpr (P < NP) {
    hipLaunchKernelGGL((stage_a_kernel<T, N, P>), dim3(nblocks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_passes<T, N, P + 1>(a, s, nblocks);
  } else {
    return hipSuccess;
  }
}

// [centre][bin][entry] (as written per centre) -> [entry][bin][centre],
// through a 64 x 64 LDS tile so both sides are coalesced.
template <typename T>
__global__ __launch_bounds__(256) void transpose_kernel(const T* __restrict__ src, T* __restrict__ dst,
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

template <typename T, int N>
hipError_t launch_n(const StageAArgs& a, hipStream_t s, int* npass) {
  static_assert(plan_np(N, Budget<T>::units) <= 16, "too many passes");
  *npass = plan_np(N, Budget<T>::units);
  int nblocks = (a.ncent + 3) / 4;
  nblocks = ((nblocks + 7) / 8) * 8;
  if (nblocks > 2048) nblocks = 2048;
  if (nblocks < 8) nblocks = 8;
  hipError_t e = launch_passes<T, N, 0>(a, s, nblocks);
  if (e != hipSuccess) return e;
  const int mpc = make_layout(N).mpc;
  const dim3 grid((a.ncent + 63) / 64, a.nb, (mpc + 63) / 64);
  hipLaunchKernelGGL(transpose_kernel<T>, grid, dim3(256), 0, s, reinterpret_cast<const T*>(a.rec_aos),
                     reinterpret_cast<T*>(a.rec), a.ncent, a.nb, mpc, a.ldc);
  return hipGetLastError();
}

}  // namespace sa

#if defined(FPCF4_STAGE_A_N)
// One translation unit per nmax keeps the (large, fully unrolled) kernels
// compiling in parallel.
template hipError_t sa::launch_n<float, FPCF4_STAGE_A_N>(const StageAArgs&, hipStream_t, int*);
template hipError_t sa::launch_n<double, FPCF4_STAGE_A_N>(const StageAArgs&, hipStream_t, int*);
#else
namespace sa {
#define FPCF4_DECL_N(NN)                                                         \
  extern template hipError_t launch_n<float, NN>(const StageAArgs&, hipStream_t, int*); \
  extern template hipError_t launch_n<double, NN>(const StageAArgs&, hipStream_t, int*);
FPCF4_DECL_N(0) FPCF4_DECL_N(1) FPCF4_DECL_N(2) FPCF4_DECL_N(3) FPCF4_DECL_N(4)
FPCF4_DECL_N(5) FPCF4_DECL_N(6) FPCF4_DECL_N(7) FPCF4_DECL_N(8) FPCF4_DECL_N(9)
FPCF4_DECL_N(10) FPCF4_DECL_N(11) FPCF4_DECL_N(12) FPCF4_DECL_N(13) FPCF4_DECL_N(14)
FPCF4_DECL_N(15) FPCF4_DECL_N(16)
#undef FPCF4_DECL_N
}  // namespace sa

template <typename T>
hipError_t launch_stage_a(int nmax, const StageAArgs& a, hipStream_t s, int* npass) {
  switch (nmax) {
#define FPCF4_CASE(NN) case NN: return sa::launch_n<T, NN>(a, s, npass);
    FPCF4_CASE(0) FPCF4_CASE(1) FPCF4_CASE(2) FPCF4_CASE(3) FPCF4_CASE(4)
    FPCF4_CASE(5) FPCF4_CASE(6) FPCF4_CASE(7) FPCF4_CASE(8) FPCF4_CASE(9)
    FPCF4_CASE(10) FPCF4_CASE(11) FPCF4_CASE(12) FPCF4_CASE(13) FPCF4_CASE(14)
    FPCF4_CASE(15) FPCF4_CASE(16)
#undef FPCF4_CASE
    default: return hipErrorInvalidValue;
  }
}
template hipError_t launch_stage_a<float>(int, const StageAArgs&, hipStream_t, int*);
template hipError_t launch_stage_a<double>(int, const StageAArgs&, hipStream_t, int*);
#endif

}  // namespace fpcf4
