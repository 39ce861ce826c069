// Multipoles -> bin-averaged natural components, binary64 (Sect. 2.3 and the
// multipole expansion of Sect. 3.1):
//   Ubar(T, Phi_a, Phi_b) = (2 pi)^-2 sum_{n2,n3} Upsilon_n I_n2(Phi_a) I_n3(Phi_b),
//   I_0(Phi) = |Delta Phi|, I_m(Phi) = (e^{i m Phi_up} - e^{i m Phi_low}) / (i m),
// on nphi linear angular bins of [0, 2 pi), done as two small complex
// contractions (over n2, then over n3).  Gamma_mu = Ubar_mu / Nbar.
#include "fpcf4_internal.hpp"

namespace fpcf4 {

__device__ inline void ang_int(int m, int a, int nphi, double& re, double& im) {
  const double lo = 2.0 * M_PI * a / nphi, hi = 2.0 * M_PI * (a + 1) / nphi;
  if (m == 0) {
    re = hi - lo;
    im = 0.0;
    return;
  }
  double sh, ch, sl, cl;
  sincos(m * hi, &sh, &ch);
  sincos(m * lo, &sl, &cl);
  // (e^{i m hi} - e^{i m lo}) / (i m)
  re = (sh - sl) / m;
  im = -(ch - cl) / m;
}

// table[k][a] = I_{k - nmax}(Phi_a), complex
__global__ void nat_table(int nmax, int nphi, double* table) {
  const int nn = 2 * nmax + 1;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nn * nphi; t += gridDim.x * blockDim.x) {
    double re, im;
    ang_int(t / nphi - nmax, t % nphi, nphi, re, im);
    table[2 * t] = re;
    table[2 * t + 1] = im;
  }
}

// tmp[q][a][n3] = sum_n2 ups[q][n2][n3] I_n2(a),  q = (mu, b1, b2, b3)
__global__ void nat_pass1(const double* ups, int64_t nq, int nmax, int nphi, const double* table,
                          double* tmp) {
  const int nn = 2 * nmax + 1;
  const int64_t total = nq * nphi * nn;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int n3 = (int)(t % nn);
    const int a = (int)((t / nn) % nphi);
    const int64_t q = t / ((int64_t)nn * nphi);
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < nn; ++k) {
      const double ir = table[2 * (k * nphi + a)], ii = table[2 * (k * nphi + a) + 1];
      const double ur = ups[2 * ((q * nn + k) * nn + n3)], ui = ups[2 * ((q * nn + k) * nn + n3) + 1];
      sr += ur * ir - ui * ii;
      si += ur * ii + ui * ir;
    }
    tmp[2 * t] = sr;
    tmp[2 * t + 1] = si;
  }
}

// out[q][a][b] = (2 pi)^-2 sum_n3 tmp[q][a][n3] I_n3(b)
__global__ void nat_pass2(const double* tmp, int64_t nq, int nmax, int nphi, const double* table,
                          double* out) {
  const int nn = 2 * nmax + 1;
  const double s = 1.0 / (4.0 * M_PI * M_PI);
  const int64_t total = nq * nphi * nphi;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(t % nphi);
    const int a = (int)((t / nphi) % nphi);
    const int64_t q = t / ((int64_t)nphi * nphi);
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < nn; ++k) {
      const double ir = table[2 * (k * nphi + b)], ii = table[2 * (k * nphi + b) + 1];
      const int64_t o = (q * nphi + a) * nn + k;
      const double ur = tmp[2 * o], ui = tmp[2 * o + 1];
      sr += ur * ir - ui * ii;
      si += ur * ii + ui * ir;
    }
    out[2 * t] = sr * s;
    out[2 * t + 1] = si * s;
  }
}

// gamma[mu<8] = Ubar_mu / Re(Nbar); norm = Re(Nbar); Nbar is the mu = 8 slab
__global__ void nat_divide(double* binned, int64_t per_mu, double* gamma, double* norm) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < per_mu;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double nv = binned[2 * (8 * per_mu + t)];
    norm[t] = nv;
    for (int mu = 0; mu < 8; ++mu) {
      const int64_t o = mu * per_mu + t;
      gamma[2 * o] = nv != 0.0 ? binned[2 * o] / nv : 0.0;
      gamma[2 * o + 1] = nv != 0.0 ? binned[2 * o + 1] / nv : 0.0;
    }
  }
}

// sel[mu][t][n2][n3] = ups[mu][b1][b2][b3][n2][n3] for the listed triplets
__global__ void nat_gather(const double* ups, int nb, int nmax, const int32_t* trip, int64_t ntrip,
                           double* sel) {
  const int nn = 2 * nmax + 1;
  const int64_t nn2 = (int64_t)nn * nn;
  const int64_t total = 9 * ntrip * nn2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i % nn2;
    const int64_t t = (i / nn2) % ntrip;
    const int64_t mu = i / (nn2 * ntrip);
    const int64_t q = ((mu * nb + trip[3 * t]) * nb + trip[3 * t + 1]) * nb + trip[3 * t + 2];
    sel[2 * i] = ups[2 * (q * nn2 + e)];
    sel[2 * i + 1] = ups[2 * (q * nn2 + e) + 1];
  }
}

hipError_t natural_triplets(const double* ups, int nb, int nmax, int nphi, const int32_t* trip,
                            int64_t ntrip, double* sel, double* tmp, double* binned, double* gamma,
                            double* norm, hipStream_t s) {
  const int64_t nq = 9 * ntrip;
  const int64_t per_mu = ntrip * nphi * nphi;
  double* table = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&table), (size_t)(2 * nmax + 1) * nphi * 16, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(nat_table, dim3(64), dim3(256), 0, s, nmax, nphi, table);
  hipLaunchKernelGGL(nat_gather, dim3(2048), dim3(256), 0, s, ups, nb, nmax, trip, ntrip, sel);
  hipLaunchKernelGGL(nat_pass1, dim3(2048), dim3(256), 0, s, sel, nq, nmax, nphi, table, tmp);
  hipLaunchKernelGGL(nat_pass2, dim3(2048), dim3(256), 0, s, tmp, nq, nmax, nphi, table, binned);
  hipLaunchKernelGGL(nat_divide, dim3(1024), dim3(256), 0, s, binned, per_mu, gamma, norm);
  e = hipGetLastError();
  (void)hipFreeAsync(table, s);
  return e;
}

hipError_t natural_components(const double* ups, int nb, int nmax, int nphi, double* tmp,
                              double* gamma, double* norm, hipStream_t s) {
  const int64_t nq = 9LL * nb * nb * nb;
  const int64_t per_mu = (int64_t)nb * nb * nb * nphi * nphi;
  // the binned sums of all nine correlators go to a temporary; Gamma and
  // Nbar are formed from it
  double* table = nullptr;
  hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&table), (size_t)(2 * nmax + 1) * nphi * 16, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(nat_table, dim3(64), dim3(256), 0, s, nmax, nphi, table);
  hipLaunchKernelGGL(nat_pass1, dim3(2048), dim3(256), 0, s, ups, nq, nmax, nphi, table, tmp);
  e = hipGetLastError();
  double* binned = nullptr;
  if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&binned), (size_t)(9 * per_mu) * 16, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(nat_pass2, dim3(2048), dim3(256), 0, s, tmp, nq, nmax, nphi, table, binned);
    hipLaunchKernelGGL(nat_divide, dim3(1024), dim3(256), 0, s, binned, per_mu, gamma, norm);
    e = hipGetLastError();
    (void)hipFreeAsync(binned, s);
  }
  (void)hipFreeAsync(table, s);
  return e;
}

}  // namespace fpcf4
