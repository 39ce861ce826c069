// Degenerate-term sums of App. A.1 (Table 1) and the binary64 finalisation.
//
// Correction sums, binary64, accumulated over tiles.  Buffer layout per mu
// (complex):
//   P12[b][b3][n3]  nb*nb*nn   : sum_i x c12(i,b; n3) C(i,b3; n3)
//   P13[b][b2][n2]  nb*nb*nn   : sum_i x c13(i,b; n2) B(i,b2; n2)
//   P23[b1][b][s]   nb*nb*ns   : sum_i x A(i,b1; s) c23(i,b; s), s = n2+n3
//   P3[b]           nb         : sum_i x t(i,b)
// Records are centre-contiguous, so a chunk of centres of one bin row is a
// coalesced load.
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

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int CKC = 32;   // centres per LDS chunk

// Each (mu, kind, order) is a small GEMM over the tile's centres,
//   P[b_eq, b'] = sum_c E[c, b_eq] F[c, b'],  E = x (Table 1 block), F = other factor,
// done on v_mfma_f64_16x16x4_f64 with the complex product split into real
// rows [[E_r, -E_i], [E_i, E_r]] and columns [F_r; F_i].  The triple term
// (kind 3) is the same GEMM with F = 1 in column 0.  The four waves take
// alternate K-steps of each LDS-staged chunk and are summed at the end.
template <typename T>
__global__ __launch_bounds__(256) void corr_kernel(CorrArgs a) {
  const int nb = a.nb, n = a.nmax, nn = 2 * n + 1, ns = 4 * n + 1;
  const Layout L = make_layout(n);
  const int per_mu = 2 * nn + ns + 1;
  const int lb = (int)blockIdx.x;
  const int mu = lb / per_mu;
  int r = lb % per_mu;
  int kind, ord = 0;
  if (r < nn) { kind = 0; ord = r - n; }
  else if ((r -= nn) < nn) { kind = 1; ord = r - n; }
  else if ((r -= nn) < ns) { kind = 2; ord = r - 2 * n; }
  else { kind = 3; }
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
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
  const int ncent = a.ncent;

  __shared__ cplx Es[2][16][CKC + 1];
  __shared__ cplx Fs[2][16][CKC + 1];
  __shared__ d4 red[4][2][64];

  cplx pe[2], pf[2], px[2];
  auto issue = [&](int c0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int slot = tid + 256 * h;
      const int b = slot / CKC, c = c0 + slot % CKC;
      pe[h] = pf[h] = px[h] = {0.0, 0.0};
      if (b < nb && c < ncent) {
        if (xkind == X_W) px[h] = {(double)xw[c], 0.0};
        else px[h] = {(double)xg[2 * c], (double)xg[2 * c + 1]};
        if (kind == 3) {
          pe[h] = R.at(t_entry, b, c);
          pf[h] = {b == 0 ? 1.0 : 0.0, 0.0};
        } else {
          pe[h] = corr_fam(R, L, ce_fam, ke, b, c);
          pf[h] = R.at(e_fo, b, c);
        }
      }
    }
  };
  auto commit = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int slot = tid + 256 * h;
      const int b = slot / CKC, cc = slot % CKC;
      if (b < nb) {
        cplx x = px[h];
        if (xkind == X_GC) x.i = -x.i;
        cplx f = pf[h];
        if (kind != 3 && fo_conj) f.i = -f.i;
        Es[buf][b][cc] = cmul(x, pe[h]);
        Fs[buf][b][cc] = f;
      }
    }
  };

  // A rows (part, b_eq) of this lane in the two row tiles; B column b'
  int rb[2], rp[2];
  bool rok[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int row = 16 * m + (lane & 15);
    rok[m] = row < 2 * nb;
    rp[m] = rok[m] ? row / nb : 0;
    rb[m] = rok[m] ? row % nb : 0;
  }
  const int col = lane & 15;
  const bool cok = col < nb;
  const int kq = lane >> 4;   // K index within the 4-wide step: centre kq/2, part kq%2
  d4 acc[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};

  const int nchunks = (ncent + CKC - 1) / CKC;
  issue(0);
  commit(0);
  __syncthreads();
  for (int ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunks;
    if (more) issue((ch + 1) * CKC);
#pragma unroll
    for (int q = 0; q < CKC / 8; ++q) {         // this wave's K-steps: wv, wv+4, ...
      const int ks = wv + 4 * q;
      const int cc = 2 * ks + (kq >> 1), pk = kq & 1;
      const cplx fv = Fs[buf][cok ? col : 0][cc];
      const double bv = cok ? (pk ? fv.i : fv.r) : 0.0;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const cplx ev = Es[buf][rb[m]][cc];
        const double av = rok[m] ? (rp[m] ? (pk ? ev.r : ev.i) : (pk ? -ev.i : ev.r)) : 0.0;
        acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[m], 0, 0, 0);
      }
    }
    if (more) commit(buf ^ 1);
    __syncthreads();
  }
  red[wv][0][lane] = acc[0];
  red[wv][1][lane] = acc[1];
  __syncthreads();
  if (wv != 0) return;
  double* out = a.corr + 2 * (int64_t)mu * corr_mu_elems(nb, n);
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const d4 v = red[0][m][lane] + red[1][m][lane] + red[2][m][lane] + red[3][m][lane];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * m + 4 * e + (lane >> 4);   // f64 D layout
      if (row >= 2 * nb || !cok || (kind == 3 && col != 0)) continue;
      const int part = row / nb, beq = row % nb, bo = col;
      int64_t o;
      if (kind == 0) o = ((int64_t)beq * nb + bo) * nn + (ord + n);
      else if (kind == 1) o = (int64_t)nb * nb * nn + ((int64_t)beq * nb + bo) * nn + (ord + n);
      else if (kind == 2) o = 2LL * nb * nb * nn + ((int64_t)bo * nb + beq) * ns + (ord + 2 * n);
      else o = 2LL * nb * nb * nn + (int64_t)nb * nb * ns + beq;
      out[2 * o + part] += v[e];
    }
  }
}

template <typename T>
hipError_t launch_corrections(const CorrArgs& a, hipStream_t s) {
  if (a.ncent <= 0) return hipSuccess;
  const int nn = 2 * a.nmax + 1, ns = 4 * a.nmax + 1;
  const int blocks = 9 * (2 * nn + ns + 1);
  hipLaunchKernelGGL(corr_kernel<T>, dim3(blocks), dim3(256), 0, s, a);
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
