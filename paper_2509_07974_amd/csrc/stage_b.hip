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
//
// All three pair kinds are sums x E(b) F(b') with E the Table 1 block at the
// equal bins and F the remaining factor at the other bin (P23 stores it as
// [b'][b]), and correlators share blocks: at nmax = 10 the 9 x 84 sums of the
// buffer are 292 distinct GEMMs plus the triple terms.  make_corr_plan lists
// them; corr_kernel forms each once per centre slice, and
// corr_scatter_kernel adds the slices of every buffer entry's sum in order.
#include <algorithm>
#include <array>
#include <map>

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

// (mu, slot) with slot = kind 0 orders n3, kind 1 orders n2, kind 2 orders
// s = n2 + n3, kind 3: the kind and its order
static __host__ __device__ inline void corr_slot(int slot, int n, int& kind, int& ord) {
  const int nn = 2 * n + 1, ns = 4 * n + 1;
  ord = 0;
  if (slot < nn) { kind = 0; ord = slot - n; }
  else if ((slot -= nn) < nn) { kind = 1; ord = slot - n; }
  else if ((slot -= nn) < ns) { kind = 2; ord = slot - 2 * n; }
  else kind = 3;
}

CorrPlanHost make_corr_plan(int n) {
  const Layout L = make_layout(n);
  const int nn = 2 * n + 1, ns = 4 * n + 1, per_mu = 2 * nn + ns + 1;
  CorrPlanHost P;
  P.map.assign((size_t)9 * per_mu, -1);
  std::map<std::array<int, 5>, int> pair_id;
  std::map<std::array<int, 2>, int> triple_id;
  std::vector<CorrSum> pairs, triples;
  std::vector<std::pair<size_t, int>> triple_slots;
  for (int mu = 0; mu < FPCF4_NCORR; ++mu) {
    const MuFactors F = mu_factors(mu);
    const MuCorr C = mu_corr(mu);
    for (int slot = 0; slot < per_mu; ++slot) {
      int kind, ord;
      corr_slot(slot, n, kind, ord);
      const size_t m = (size_t)mu * per_mu + slot;
      if (kind == 3) {
        const int e = L.offS + C.t;
        const auto r = triple_id.emplace(std::array<int, 2>{F.x, e}, (int)triples.size());
        if (r.second) triples.push_back(CorrSum{(int8_t)F.x, 1, 0, 0, e, e});
        triple_slots.push_back({m, r.first->second});
        continue;
      }
      // Table 1 block at the equal bins and the remaining factor, at this order
      const Fac ce = kind == 0 ? C.c12 : (kind == 1 ? C.c13 : C.c23);
      const int ke = kind == 0 ? ce.b * ord + ce.c : ce.a * ord + ce.c;
      const Fac fo = kind == 0 ? F.C : (kind == 1 ? F.B : F.A);
      const int ko = kind == 0 ? fo.b * ord + fo.c : fo.a * ord + fo.c;
      int eidx, eflip = 0;
      if (ce.fam == C_Q) {
        eidx = eQ(L, ke);
      } else {   // A and V are sums of real weights: X_-k = conj X_k
        const int k = ke < 0 ? -ke : ke;
        eidx = ce.fam == C_A ? eA(L, k) : eV(L, k);
        eflip = ke < 0;
      }
      const int fidx = fo.fam == F_G ? eG(L, ko) : eW(L, ko);
      const std::array<int, 5> key{F.x, eidx, eflip, fidx, fo.conj};
      const auto r = pair_id.emplace(key, (int)pairs.size());
      if (r.second) pairs.push_back(CorrSum{(int8_t)F.x, 0, (int8_t)eflip, (int8_t)fo.conj, eidx, fidx});
      P.map[m] = r.first->second;
    }
  }
  P.npair = (int)pairs.size();
  for (const auto& ts : triple_slots) P.map[ts.first] = P.npair + ts.second;
  P.sums = pairs;
  P.sums.insert(P.sums.end(), triples.begin(), triples.end());
  return P;
}

typedef double d4 __attribute__((ext_vector_type(4)));
constexpr int CKC = 32;   // centres per LDS chunk

// Each distinct sum is a small GEMM over the tile's centres,
//   P[b_eq, b'] = sum_c E[c, b_eq] F[c, b'],  E = x (Table 1 block), F = other factor,
// done on v_mfma_f64_16x16x4_f64 with the complex product split into real
// rows [[E_r, -E_i], [E_i, E_r]] and columns [F_r; F_i].  The triple term
// (kind 3) is the same GEMM with F = 1 in column 0.  The four waves take
// alternate K-steps of each LDS-staged chunk and are summed at the end.  The
// centres are cut into CORR_SLICES contiguous slices (blockIdx.y), each
// written to its own binary64 partial buffer; corr_scatter_kernel adds the
// slices in a fixed order, so the sums stay deterministic.
template <typename T>
__global__ __launch_bounds__(256) void corr_kernel(CorrArgs a) {
  const int nb = a.nb;
  const int sidx = (int)blockIdx.x;
  const CorrSum cs = a.sums[sidx];
  const int kind = cs.triple ? 3 : 0;   // 3: F = 1 in column 0
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const T* xg = reinterpret_cast<const T*>(a.xg);
  const T* xw = reinterpret_cast<const T*>(a.xw);
  const int e_fo = cs.fidx;
  const bool fo_conj = cs.fconj != 0;
  const int xkind = cs.x;
  const int ncent = a.ncent;
  const int nch_all = (ncent + CKC - 1) / CKC;
  const int ch0 = (int)(((int64_t)nch_all * blockIdx.y) / gridDim.y);
  const int ch1 = (int)(((int64_t)nch_all * (blockIdx.y + 1)) / gridDim.y);
  // bin tile (blockIdx.z = te nt + tf): equal-bin rows b_eq in [oe, oe + ne),
  // other-factor columns b' in [of, of + nf); the triple term has one column
  const BinTiles bt = bin_tiles(nb);
  const int te = (int)blockIdx.z / bt.nt, tf = (int)blockIdx.z % bt.nt;
  if (kind == 3 && tf != 0) return;
  const int oe = te * bt.tb, of = tf * bt.tb;
  const int ne = imin(bt.tb, nb - oe), nf = imin(bt.tb, nb - of);

  __shared__ cplx Es[2][16][CKC + 1];
  __shared__ cplx Fs[2][16][CKC + 1];
  __shared__ d4 red[4][2][64];

  // Row pointers and conjugations of this thread's two (bin, centre) slots,
  // resolved once: per chunk a slot is three plain loads at centre c.
  const int eidx = cs.eidx;      // Table 1 block entry
  const int eflip = cs.eflip;    // conjugate (A, V at negative order)
  const T* rec = reinterpret_cast<const T*>(a.rec);
  const T* pe_row[2];
  const T* pf_row[2];
  bool slot_ok[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int b = (tid + 256 * h) / CKC;
    // a slot past ne (nf) loads a clamped row that is never read
    slot_ok[h] = b < ne || b < nf;
    const int be = b < ne ? b : 0, bf = b < nf ? b : 0;
    pe_row[h] = rec + 2 * (((int64_t)eidx * nb + oe + be) * a.ldc);
    pf_row[h] = rec + 2 * (((int64_t)e_fo * nb + of + bf) * a.ldc);
  }
  const double fone = 1.0;   // kind 3: F = 1 in column 0

  // Raw values of one chunk (two (bin, centre) slots per thread).  The loads
  // are unconditional (centre clamped to the tile), so they stay in flight
  // across the MFMAs of the current chunk; masking, conjugation and the
  // conversion to binary64 happen in commit.
  struct Regs {
    T e[2][2], f[2][2], x[2][2], w[2];
  };
  Regs ra, rbf;   // two chunks in flight: loads are issued two chunks ahead
  auto issue = [&](Regs& g, int c0) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      int c = c0 + (tid + 256 * h) % CKC;
      c = c < ncent ? c : ncent - 1;
      g.e[h][0] = pe_row[h][2 * c];
      g.e[h][1] = pe_row[h][2 * c + 1];
      g.f[h][0] = pf_row[h][2 * c];
      g.f[h][1] = pf_row[h][2 * c + 1];
      g.x[h][0] = xg[2 * c];
      g.x[h][1] = xg[2 * c + 1];
      g.w[h] = xw[c];
    }
  };
  auto commit = [&](const Regs& g, int c0, int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int slot = tid + 256 * h;
      const int b = slot / CKC, cc = slot % CKC;
      if (slot_ok[h]) {
        const bool live = c0 + cc < ncent;
        cplx x = xkind == X_W ? cplx{(double)g.w[h], 0.0} : cplx{(double)g.x[h][0], (double)g.x[h][1]};
        if (xkind == X_GC) x.i = -x.i;
        cplx e{(double)g.e[h][0], (double)g.e[h][1]};
        if (eflip) e.i = -e.i;
        cplx f{(double)g.f[h][0], (double)g.f[h][1]};
        if (kind == 3) f = {b == 0 ? fone : 0.0, 0.0};
        else if (fo_conj) f.i = -f.i;
        const cplx ex = cmul(x, e);
        Es[buf][b][cc] = live ? ex : cplx{0.0, 0.0};
        Fs[buf][b][cc] = live ? f : cplx{0.0, 0.0};
      }
    }
  };

  // A rows (part, b_eq) of this lane in the two row tiles; B column b'
  int rb[2], rp[2];
  bool rok[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const int row = 16 * m + (lane & 15);
    rok[m] = row < 2 * ne;
    rp[m] = rok[m] ? row / ne : 0;
    rb[m] = rok[m] ? row % ne : 0;
  }
  const int col = lane & 15;
  const bool cok = col < nf;
  const int kq = lane >> 4;   // K index within the 4-wide step: centre kq/2, part kq%2
  d4 acc[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};

  auto compute = [&](int buf) {
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
  };

  // chunk ch sits in LDS buffer (ch - ch0) & 1; the registers hold the next
  // one or two chunks, so every load has two chunks of compute to land
  issue(ra, ch0 * CKC);
  commit(ra, ch0 * CKC, 0);
  __syncthreads();
  if (ch0 + 1 < ch1) issue(ra, (ch0 + 1) * CKC);
  for (int ch = ch0; ch < ch1; ch += 2) {
    if (ch + 2 < ch1) issue(rbf, (ch + 2) * CKC);
    compute(0);
    if (ch + 1 < ch1) commit(ra, (ch + 1) * CKC, 1);
    __syncthreads();
    if (ch + 1 >= ch1) break;
    if (ch + 3 < ch1) issue(ra, (ch + 3) * CKC);
    compute(1);
    if (ch + 2 < ch1) commit(rbf, (ch + 2) * CKC, 0);
    __syncthreads();
  }
  red[wv][0][lane] = acc[0];
  red[wv][1][lane] = acc[1];
  __syncthreads();
  if (wv != 0) return;
  // this slice's region: pair sums [npair][nb][nb], then triple sums [nb]
  double* out = a.part + 2 * ((int64_t)blockIdx.y * 9 * corr_mu_elems(nb, a.nmax));
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    const d4 v = red[0][m][lane] + red[1][m][lane] + red[2][m][lane] + red[3][m][lane];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = 16 * m + 4 * e + (lane >> 4);   // f64 D layout
      if (row >= 2 * ne || !cok || (kind == 3 && col != 0)) continue;
      const int part = row / ne, beq = oe + row % ne, bo = of + col;
      const int64_t o = kind == 3 ? (int64_t)a.npair * nb * nb + (int64_t)(sidx - a.npair) * nb + beq
                                  : ((int64_t)sidx * nb + beq) * nb + bo;
      out[2 * o + part] = v[e];
    }
  }
}

// corr += sum over slices of the distinct sum each entry of the buffer reads,
// slice by slice (deterministic)
__global__ void corr_scatter_kernel(const double* part, const int32_t* map, int npair, int nb, int n,
                                    double* corr) {
  const int nn = 2 * n + 1, ns = 4 * n + 1, per_mu = 2 * nn + ns + 1;
  const int64_t mu_elems = corr_mu_elems(nb, n), slice = 2 * 9 * mu_elems;
  const int64_t total = 2 * 9 * mu_elems;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int p = (int)(i & 1);
    const int64_t o = i >> 1;
    const int mu = (int)(o / mu_elems);
    int64_t r = o % mu_elems;
    int slot, beq, bo = 0;
    const int64_t pq = (int64_t)nb * nb * nn;
    if (r < 2 * pq) {                        // P12 [b][b3][n3], P13 [b][b2][n2]
      const int k = (int)(r / pq);
      r %= pq;
      slot = k * nn + (int)(r % nn);
      bo = (int)((r / nn) % nb);
      beq = (int)(r / nn / nb);
    } else if ((r -= 2 * pq) < (int64_t)nb * nb * ns) {   // P23 [b1][b][s]
      slot = 2 * nn + (int)(r % ns);
      beq = (int)((r / ns) % nb);
      bo = (int)(r / ns / nb);
    } else {                                 // P3 [b]
      slot = 2 * nn + ns;
      beq = (int)(r - (int64_t)nb * nb * ns);
    }
    const int sum = map[mu * per_mu + slot];
    const int64_t src = sum < npair ? ((int64_t)sum * nb + beq) * nb + bo
                                    : (int64_t)npair * nb * nb + (int64_t)(sum - npair) * nb + beq;
    double v = corr[i];
#pragma unroll
    for (int sl = 0; sl < CORR_SLICES; ++sl) v += part[sl * slice + 2 * src + p];
    corr[i] = v;
  }
}

template <typename T>
hipError_t launch_corrections(const CorrArgs& a, hipStream_t s) {
  if (a.ncent <= 0) return hipSuccess;
  if (a.nsums <= 0 || a.npair < 0 || a.npair > a.nsums) return hipErrorInvalidValue;
  const BinTiles bt = bin_tiles(a.nb);
  hipLaunchKernelGGL(corr_kernel<T>, dim3(a.nsums, CORR_SLICES, bt.nt * bt.nt), dim3(256), 0, s, a);
  const int64_t elems = 2 * (int64_t)corr_elems(a.nb, a.nmax);
  const int64_t blocks = std::min<int64_t>((elems + 255) / 256, 1 << 16);
  hipLaunchKernelGGL(corr_scatter_kernel, dim3((int)blocks), dim3(256), 0, s, (const double*)a.part, a.map,
                     a.npair, a.nb, a.nmax, a.corr);
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
      // every kind of every mu holds its sums (filled from the distinct ones)
      auto Ck = [&](int) { return corr + 2 * (int64_t)mu * corr_mu_elems(nb, n); };
      if (b1 == b2) {
        const double* C = Ck(0);
        const int64_t q = ((int64_t)b1 * nb + b3) * nn + (n3 + n);
        re -= C[2 * q]; im -= C[2 * q + 1];
      }
      if (b1 == b3) {
        const double* C = Ck(1);
        const int64_t q = (int64_t)nb * nb * nn + ((int64_t)b1 * nb + b2) * nn + (n2 + n);
        re -= C[2 * q]; im -= C[2 * q + 1];
      }
      if (b2 == b3) {
        const double* C = Ck(2);
        const int64_t q = 2LL * nb * nb * nn + ((int64_t)b1 * nb + b2) * ns + (n2 + n3 + 2 * n);
        re -= C[2 * q]; im -= C[2 * q + 1];
      }
      if (b1 == b2 && b2 == b3) {
        const double* C = Ck(3);
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
