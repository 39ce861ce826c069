// Degenerate-term sums of App. A.1 (Table 1) and the binary64 finalisation.
//
// Correction sums, binary64, accumulated over tiles.  Buffer layout per mu
// (complex):
//   P12[b][b3][n3]  nb*nb*nn   : sum_i x c12(i,b; n3) C(i,b3; n3)
//   P13[b][b2][n2]  nb*nb*nn   : sum_i x c13(i,b; n2) B(i,b2; n2)
//   P23[b1][b][s]   nb*nb*ns   : sum_i x A(i,b1; s) c23(i,b; s), s = n2+n3
//   P3[b]           nb         : sum_i x t(i,b)
// One workgroup of up to 8 waves per (mu, kind, order, bin group); each wave
// owns one equal-bin value b and all nb values of the other bin; lanes run over
// the tile's centres (records are centre-contiguous, so loads coalesce) and
// the 64 partial sums are combined at the end.
#include "factors.hpp"
#include "fpcf4_internal.hpp"

namespace fpcf4 {

struct cplx {
  double r, i;
};
__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ cplx cconj(cplx a) { return {a.r, -a.i}; }

static __host__ __device__ inline int64_t corr_mu_elems(int nb, int n) {
  const int nn = 2 * n + 1, ns = 4 * n + 1;
  return 2LL * nb * nb * nn + (int64_t)nb * nb * ns + nb;
}
size_t corr_elems(int nb, int nmax) { return (size_t)(9 * corr_mu_elems(nb, nmax)); }

template <typename T>
struct Rec {
  const T* p;
  int nb, ldc;
  __device__ __forceinline__ cplx at(int e, int b, int c) const {
    const T* q = p + 2 * (((int64_t)e * nb + b) * ldc + c);
    return {(double)q[0], (double)q[1]};
  }
};

// correction block (Q, A or V family) at order k, bin b, centre c
template <typename T>
__device__ __forceinline__ cplx corr_fam(const Rec<T>& R, const Layout& L, int fam, int k, int b, int c) {
  if (fam == C_Q) return R.at(eQ(L, k), b, c);
  const int e = fam == C_A ? eA(L, k < 0 ? -k : k) : eV(L, k < 0 ? -k : k);
  const cplx v = R.at(e, b, c);
  return k < 0 ? cconj(v) : v;
}

template <typename T>
__device__ __forceinline__ cplx fac_val(const Rec<T>& R, const Layout& L, const Fac& f, int k, int b, int c) {
  const cplx v = R.at(f.fam == F_G ? eG(L, k) : eW(L, k), b, c);
  return f.conj ? cconj(v) : v;
}

template <typename T>
__global__ __launch_bounds__(512) void corr_kernel(CorrArgs a) {
  const int nb = a.nb, n = a.nmax, nn = 2 * n + 1, ns = 4 * n + 1;
  const Layout L = make_layout(n);
  const int per_mu = 2 * nn + ns + 1;
  const int mu = blockIdx.x / per_mu;
  int r = blockIdx.x % per_mu;
  int kind, ord = 0;
  if (r < nn) { kind = 0; ord = r - n; }
  else if ((r -= nn) < nn) { kind = 1; ord = r - n; }
  else if ((r -= nn) < ns) { kind = 2; ord = r - 2 * n; }
  else { kind = 3; }
  const int lane = threadIdx.x & 63, beq = 8 * blockIdx.y + (threadIdx.x >> 6);   // wave -> equal bin
  if (beq >= nb || (kind == 3 && beq > 0)) return;
  const MuFactors F = mu_factors(mu);
  const MuCorr C = mu_corr(mu);
  const Rec<T> R{reinterpret_cast<const T*>(a.rec), nb, a.ldc};
  const T* xg = reinterpret_cast<const T*>(a.xg);
  const T* xw = reinterpret_cast<const T*>(a.xw);
  // equal-bin block (Table 1) and the remaining factor, selected by value
  const Fac ce = kind == 0 ? C.c12 : (kind == 1 ? C.c13 : C.c23);
  const int ke = kind == 0 ? ce.b * ord + ce.c : ce.a * ord + ce.c;
  const Fac fo = kind == 0 ? F.C : (kind == 1 ? F.B : F.A);
  const int ko = kind == 0 ? fo.b * ord + fo.c : fo.a * ord + fo.c;
  const int e_fo = fo.fam == F_G ? eG(L, ko) : eW(L, ko);
  const bool fo_conj = fo.conj != 0;
  const int ce_fam = ce.fam;
  const int t_entry = L.offS + C.t;
  const int xkind = F.x;

  cplx acc[16];
#pragma unroll
  for (int b = 0; b < 16; ++b) acc[b] = {0.0, 0.0};

  for (int c = lane; c < a.ncent; c += 64) {
    cplx x;
    if (xkind == X_W) x = {(double)xw[c], 0.0};
    else {
      x = {(double)xg[2 * c], (double)xg[2 * c + 1]};
      if (xkind == X_GC) x.i = -x.i;
    }
    if (kind == 3) {
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        if (b < nb) {
          const cplx v = cmul(x, R.at(t_entry, b, c));
          acc[b].r += v.r;
          acc[b].i += v.i;
        }
      }
    } else {
      const cplx e0 = cmul(x, corr_fam(R, L, ce_fam, ke, beq, c));
#pragma unroll
      for (int b = 0; b < 16; ++b) {
        if (b < nb) {
          cplx f = R.at(e_fo, b, c);
          if (fo_conj) f.i = -f.i;
          const cplx v = cmul(e0, f);
          acc[b].r += v.r;
          acc[b].i += v.i;
        }
      }
    }
  }
  // combine the 64 lane partial sums
#pragma unroll
  for (int b = 0; b < 16; ++b)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      acc[b].r += __shfl_xor(acc[b].r, d, 64);
      acc[b].i += __shfl_xor(acc[b].i, d, 64);
    }
  if (lane != 0) return;
  double* out = a.corr + 2 * (int64_t)mu * corr_mu_elems(nb, n);
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    if (b < nb) {
      int64_t o;
      if (kind == 0) o = ((int64_t)beq * nb + b) * nn + (ord + n);
      else if (kind == 1) o = (int64_t)nb * nb * nn + ((int64_t)beq * nb + b) * nn + (ord + n);
      else if (kind == 2) o = 2LL * nb * nb * nn + ((int64_t)b * nb + beq) * ns + (ord + 2 * n);
      else o = 2LL * nb * nb * nn + (int64_t)nb * nb * ns + b;
      out[2 * o] += acc[b].r;
      out[2 * o + 1] += acc[b].i;
    }
  }
}

template <typename T>
hipError_t launch_corrections(const CorrArgs& a, hipStream_t s) {
  if (a.ncent <= 0) return hipSuccess;
  const int nn = 2 * a.nmax + 1, ns = 4 * a.nmax + 1;
  const int blocks = 9 * (2 * nn + ns + 1);
  const int waves = a.nb < 8 ? a.nb : 8;
  hipLaunchKernelGGL(corr_kernel<T>, dim3(blocks, (a.nb + 7) / 8), dim3(64 * waves), 0, s, a);
  return hipGetLastError();
}
template hipError_t launch_corrections<double>(const CorrArgs&, hipStream_t);
template hipError_t launch_corrections<float>(const CorrArgs&, hipStream_t);

// out = raw - pair terms + 2 triple term (or raw when subtract == 0)
__global__ void finalize_kernel(const double* raw, const double* corr, int nb, int n, int subtract,
                                double* out) {
  const int nn = 2 * n + 1, ns = 4 * n + 1;
  const int64_t total = 9LL * nb * nb * nb * nn * nn;
  for (int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; o < total;
       o += (int64_t)gridDim.x * blockDim.x) {
    double re = raw[2 * o], im = raw[2 * o + 1];
    if (subtract) {
      int64_t t = o;
      const int n3 = (int)(t % nn) - n; t /= nn;
      const int n2 = (int)(t % nn) - n; t /= nn;
      const int b3 = (int)(t % nb); t /= nb;
      const int b2 = (int)(t % nb); t /= nb;
      const int b1 = (int)(t % nb); t /= nb;
      const int mu = (int)t;
      const double* C = corr + 2 * (int64_t)mu * corr_mu_elems(nb, n);
      if (b1 == b2) {
        const int64_t q = ((int64_t)b1 * nb + b3) * nn + (n3 + n);
        re -= C[2 * q]; im -= C[2 * q + 1];
      }
      if (b1 == b3) {
        const int64_t q = (int64_t)nb * nb * nn + ((int64_t)b1 * nb + b2) * nn + (n2 + n);
        re -= C[2 * q]; im -= C[2 * q + 1];
      }
      if (b2 == b3) {
        const int64_t q = 2LL * nb * nb * nn + ((int64_t)b1 * nb + b2) * ns + (n2 + n3 + 2 * n);
        re -= C[2 * q]; im -= C[2 * q + 1];
      }
      if (b1 == b2 && b2 == b3) {
        const int64_t q = 2LL * nb * nb * nn + (int64_t)nb * nb * ns + b1;
        re += 2.0 * C[2 * q]; im += 2.0 * C[2 * q + 1];
      }
    }
    out[2 * o] = re;
    out[2 * o + 1] = im;
  }
}

hipError_t launch_finalize(const double* raw, const double* corr, int nb, int nmax, int subtract,
                           double* out, hipStream_t s) {
  const int64_t total = 9LL * nb * nb * nb * (2 * nmax + 1) * (2 * nmax + 1);
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(finalize_kernel, dim3((int)blocks), dim3(256), 0, s, raw, corr, nb, nmax, subtract, out);
  return hipGetLastError();
}

}  // namespace fpcf4
