// Shear 3PCF multipoles from the per-centre records of stage (a): the
// order-N construction of the appendix on N-th order shear statistics,
// taken at N = 3 (beta rows (+,+,+), (-,+,+), (+,-,+), (+,+,-) for
// Gamma_0..Gamma_3, generalised x-projection zeta_0 = (phi_1 + phi_2)/2):
//
//   Upsilon_{mu,n}(b1, b2) = sum_i x_i F1_mu(i, b1; n) F2_mu(i, b2; n)
//
//   mu  x_i        F1 at Theta_1      F2 at Theta_2      same-neighbour block
//   0   w g        G_{n-3}            G_{-n-3}           Q_{-6}
//   1   conj(w g)  G_{n-1}            G_{-n-1}           Q_{-2}
//   2   w g        conj G_{-n-1}      G_{-n-3}           A_{-2} = conj A_2
//   3   w g        G_{n-3}            conj G_{n-1}       A_{-2}
//   N   w          W_n                W_{-n}             V_0
//
// (a slot with exponent coefficient c is G_c, or conj G_{-c} where its shear
// is conjugated).  The natural components are products of three projected
// shears -gamma_c e^{-2 i zeta} (Sect. 2.1), so the shear components carry a
// factor (-1)^3 that the block products above do not: the output is
// -Upsilon_mu for mu = 0..3 (the normalisation has no shear and no sign).  For distinct neighbour pairs the j = k terms, which exist
// only for Theta_1 = Theta_2, are removed:
//   Upsilon'(b, b) = Upsilon(b, b) - sum_i x_i D_mu(i, b),
// D_mu = sum_j (slot-1 weight)(slot-2 weight) e^{i (c1 + c2) phi_ij}, the
// block in the last column (c1 + c2 does not depend on n).
//
// A stage (a) record of order n4 holds G_k for k = -2 n4 - 3 .. 2 n4 - 1,
// W_k for |k| <= 2 n4, Q_-6, Q_-2, A_2 and V_0, so 3PCF multipoles up to
// |n| <= 2 n4 are read from it directly.
//
// The contraction is tiny next to stage (a) (5 (2m+1) nb^2 complex products
// per centre): one workgroup per (n, mu, centre slice), the slot values of a
// chunk of centres staged in LDS, one output (b1, b2) per thread, binary64
// throughout (the records are converted on load).  Each slice writes its own
// partial buffer; the slices are added in slice order (deterministic).
#include "fpcf4_internal.hpp"

namespace fpcf4 {
namespace {

struct Slot3 {
  bool w;      // W block (else G)
  bool conj;
  int s, o;    // order = s * n + o
};
struct Row3 {
  int x;       // centre factor: 0 = w g, 1 = conj(w g), 2 = w
  Slot3 f1, f2;
  int dfam;    // same-neighbour block: 0 = Q, 1 = A, 2 = V
  int dord;
  bool dconj;
};
__host__ __device__ constexpr Row3 row3(int mu) {
  return mu == 0 ? Row3{0, {false, false, 1, -3}, {false, false, -1, -3}, 0, -6, false}
       : mu == 1 ? Row3{1, {false, false, 1, -1}, {false, false, -1, -1}, 0, -2, false}
       : mu == 2 ? Row3{0, {false, true, -1, -1}, {false, false, -1, -3}, 1, 2, true}
       : mu == 3 ? Row3{0, {false, false, 1, -3}, {false, true, 1, -1}, 1, 2, true}
                 : Row3{2, {true, false, 1, 0}, {true, false, -1, 0}, 2, 0, false};
}

constexpr int CH3 = 32;   // centres per LDS chunk

__device__ inline int slot_entry(const Layout& L, const Slot3& f, int n) {
  const int k = f.s * n + f.o;
  return f.w ? eW(L, k) : eG(L, k);
}

template <typename T>
__device__ inline void centre_factor(const ThreeArgs& a, int x, int ci, double& xr, double& xi) {
  if (x == 2) {
    xr = (double)static_cast<const T*>(a.xw)[ci];
    xi = 0.0;
  } else {
    const T* g = static_cast<const T*>(a.xg);
    xr = (double)g[2 * ci];
    xi = (double)g[2 * ci + 1];
    if (x == 1) xi = -xi;
  }
}

// slice s of `parts` covers centres [s * per, min((s + 1) * per, ncent))
__host__ __device__ inline int slice_len(int ncent, int parts) {
  const int per = (ncent + parts - 1) / parts;
  return (per + CH3 - 1) / CH3 * CH3;
}

template <typename T>
__global__ __launch_bounds__(256) void contract3_kernel(ThreeArgs a) {
  // blockIdx.x = ni nt1 nt2 + bin tile (t1, t2): b1 in [o1, o1 + n1), b2 in
  // [o2, o2 + n2), inside the slot ranges [lo1, lo1 + nb1) and [lo2, lo2 + nb2)
  const BinTiles bt1 = bin_tiles(a.nb1), bt2 = bin_tiles(a.nb2);
  const int ntt = bt1.nt * bt2.nt;
  const int ni = (int)blockIdx.x / ntt;
  const int t12 = (int)blockIdx.x % ntt;
  const int o1 = a.lo1 + (t12 / bt2.nt) * bt1.tb, o2 = a.lo2 + (t12 % bt2.nt) * bt2.tb;
  const int n1 = min(bt1.tb, a.lo1 + a.nb1 - o1), n2 = min(bt2.tb, a.lo2 + a.nb2 - o2);
  const int mu = blockIdx.y;
  const int sl = blockIdx.z;
  const int n = ni - a.m;
  const int nb = a.nb;
  const Layout L = make_layout(a.n4);
  const Row3 r = row3(mu);
  const int e1 = slot_entry(L, r.f1, n), e2 = slot_entry(L, r.f2, n);
  const int per = slice_len(a.ncent, THREE_SLICES);
  const int c0 = sl * per;
  const int c1 = min(a.ncent, c0 + per);
  __shared__ double2 Ls[BIN_TILE_MAX][CH3 + 1];
  __shared__ double2 Rs[BIN_TILE_MAX][CH3 + 1];
  const int t = threadIdx.x;
  const bool owner = t < n1 * n2;
  const int b1 = owner ? t / n2 : 0, b2 = owner ? t % n2 : 0;
  const T* rec = static_cast<const T*>(a.rec);
  double ar = 0.0, ai = 0.0;
  for (int cb = c0; cb < c1; cb += CH3) {
    for (int q = t; q < (n1 + n2) * CH3; q += blockDim.x) {
      const int side = q >= n1 * CH3;
      const int rem = side ? q - n1 * CH3 : q;
      const int b = rem / CH3, c = rem - (rem / CH3) * CH3;
      const int ci = cb + c;
      double vr = 0.0, vi = 0.0;
      if (ci < c1) {
        const int32_t* par = side ? a.par2 : a.par1;
        const int col = par ? par[ci] : ci;
        const T* rs = side ? static_cast<const T*>(a.rec2) : rec;
        const size_t o = (((size_t)(side ? e2 : e1) * nb + (side ? o2 : o1) + b) * (side ? a.ldc2 : a.ldc) + col) * 2;
        vr = (double)rs[o];
        vi = (double)rs[o + 1];
        if (side ? r.f2.conj : r.f1.conj) vi = -vi;
        if (!side) {
          double xr, xi;
          centre_factor<T>(a, r.x, ci, xr, xi);
          const double tr = xr * vr - xi * vi;
          vi = xr * vi + xi * vr;
          vr = tr;
        }
      }
      if (side) Rs[b][c] = make_double2(vr, vi);
      else Ls[b][c] = make_double2(vr, vi);
    }
    __syncthreads();
    if (owner) {
#pragma unroll 8
      for (int c = 0; c < CH3; ++c) {
        const double2 l = Ls[b1][c], q = Rs[b2][c];
        ar = fma(l.x, q.x, ar);
        ar = fma(-l.y, q.y, ar);
        ai = fma(l.x, q.y, ai);
        ai = fma(l.y, q.x, ai);
      }
    }
    __syncthreads();
  }
  if (owner) {
    double* p = a.part + 2 * ((size_t)sl * three_elems(nb, a.m) + ((size_t)mu * a.nn + ni) * nb * nb +
                              (size_t)(o1 + b1) * nb + o2 + b2);
    p[0] = ar;
    p[1] = ai;
  }
}

// same-neighbour sums sum_i x_i D_mu(i, b) for every bin: one workgroup per
// (mu, centre slice, bin tile), centres strided over the threads, then a
// fixed-order tree reduction over the workgroup.
template <typename T>
__global__ __launch_bounds__(256) void diag3_kernel(ThreeArgs a) {
  const int mu = blockIdx.x;
  const int sl = blockIdx.y;
  const int nb = a.nb;
  const BinTiles bt = bin_tiles(a.nb1);   // bins [lo1, lo1 + nb1) of the slot-1 records
  const int ob = a.lo1 + (int)blockIdx.z * bt.tb, nbt = min(bt.tb, a.lo1 + a.nb1 - ob);
  const Layout L = make_layout(a.n4);
  const Row3 r = row3(mu);
  const int ed = r.dfam == 0 ? eQ(L, r.dord) : r.dfam == 1 ? eA(L, r.dord) : eV(L, r.dord);
  const int per = slice_len(a.ncent, THREE_SLICES);
  const int c0 = sl * per;
  const int c1 = min(a.ncent, c0 + per);
  const T* rec = static_cast<const T*>(a.rec);
  double accr[BIN_TILE_MAX], acci[BIN_TILE_MAX];
#pragma unroll
  for (int b = 0; b < BIN_TILE_MAX; ++b) accr[b] = acci[b] = 0.0;
  for (int ci = c0 + (int)threadIdx.x; ci < c1; ci += blockDim.x) {
    double xr, xi;
    centre_factor<T>(a, r.x, ci, xr, xi);
#pragma unroll
    for (int b = 0; b < BIN_TILE_MAX; ++b) {
      if (b < nbt) {
        const size_t o = (((size_t)ed * nb + ob + b) * a.ldc + ci) * 2;
        const double vr = (double)rec[o];
        const double vi = r.dconj ? -(double)rec[o + 1] : (double)rec[o + 1];
        accr[b] = fma(xr, vr, fma(-xi, vi, accr[b]));
        acci[b] = fma(xr, vi, fma(xi, vr, acci[b]));
      }
    }
  }
  __shared__ double2 red[256];
  const int t = threadIdx.x;
  double* out = a.part + 2 * ((size_t)sl * three_elems(nb, a.m) + (size_t)5 * a.nn * nb * nb +
                              (size_t)mu * nb);
#pragma unroll
  for (int b = 0; b < BIN_TILE_MAX; ++b) {
    if (b < nbt) {
      red[t] = make_double2(accr[b], acci[b]);
      __syncthreads();
      for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
          red[t].x += red[t + s].x;
          red[t].y += red[t + s].y;
        }
        __syncthreads();
      }
      if (t == 0) {
        out[2 * (ob + b)] = red[0].x;
        out[2 * (ob + b) + 1] = red[0].y;
      }
      __syncthreads();
    }
  }
}

// acc[i] += sum over slices of part[s][i], slices in order
__global__ void reduce3_kernel(const double* part, size_t elems2, double* acc) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= elems2) return;
  double v = 0.0;
  for (int s = 0; s < THREE_SLICES; ++s) v += part[(size_t)s * elems2 + i];
  acc[i] += v;
}

// out[mu][b1][b2][n] = acc[mu][n][b1][b2] - [b1 == b2] diag[mu][b1]
__global__ void finalize3_kernel(const double* acc, int nb, int m, int subtract, double* out) {
  const int nn = 2 * m + 1;
  const size_t total = (size_t)5 * nb * nb * nn;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int ni = (int)(i % nn);
  const int b2 = (int)((i / nn) % nb);
  const int b1 = (int)((i / ((size_t)nn * nb)) % nb);
  const int mu = (int)(i / ((size_t)nn * nb * nb));
  const size_t src = ((size_t)mu * nn + ni) * nb * nb + (size_t)b1 * nb + b2;
  double vr = acc[2 * src], vi = acc[2 * src + 1];
  if (subtract && b1 == b2) {
    const size_t d = (size_t)5 * nn * nb * nb + (size_t)mu * nb + b1;
    vr -= acc[2 * d];
    vi -= acc[2 * d + 1];
  }
  // (-1)^3 of the three projected shears (exact)
  const double sg = mu < 4 ? -1.0 : 1.0;
  out[2 * i] = sg * vr;
  out[2 * i + 1] = sg * vi;
}

}  // namespace

template <typename T>
hipError_t launch_three(const ThreeArgs& a, hipStream_t s) {
  if (a.ncent <= 0) return hipSuccess;
  if (a.nb < 1 || a.nb > FPCF4_NBINS_SUPPORTED || a.m < 0 || a.m > 2 * a.n4) return hipErrorInvalidValue;
  if (a.lo1 < 0 || a.nb1 < 1 || a.lo1 + a.nb1 > a.nb || a.lo2 < 0 || a.nb2 < 1 || a.lo2 + a.nb2 > a.nb)
    return hipErrorInvalidValue;
  const BinTiles bt1 = bin_tiles(a.nb1), bt2 = bin_tiles(a.nb2);
  hipLaunchKernelGGL(contract3_kernel<T>, dim3(a.nn * bt1.nt * bt2.nt, 5, THREE_SLICES), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the same-neighbour sums exist where both slots share bins and records
  if (a.lo1 == a.lo2 && a.nb1 == a.nb2 && a.rec2 == a.rec && a.par1 == nullptr && a.par2 == nullptr)
    hipLaunchKernelGGL(diag3_kernel<T>, dim3(5, THREE_SLICES, bt1.nt), dim3(256), 0, s, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t elems2 = 2 * three_elems(a.nb, a.m);
  hipLaunchKernelGGL(reduce3_kernel, dim3((unsigned)((elems2 + 255) / 256)), dim3(256), 0, s,
                     (const double*)a.part, elems2, a.acc);
  return hipGetLastError();
}
template hipError_t launch_three<float>(const ThreeArgs&, hipStream_t);
template hipError_t launch_three<double>(const ThreeArgs&, hipStream_t);

hipError_t launch_finalize3(const double* acc, int nb, int m, int subtract, double* out, hipStream_t s) {
  const size_t total = (size_t)5 * nb * nb * (2 * m + 1);
  hipLaunchKernelGGL(finalize3_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, acc, nb,
                     m, subtract, out);
  return hipGetLastError();
}

}  // namespace fpcf4
