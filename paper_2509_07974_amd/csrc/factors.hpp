// Factor tables of the contraction and of the degenerate-term subtraction.
//
// Sect. 3.1 (the multipole equations for Upsilon_0 ... Upsilon_7 and N_n):
//   Upsilon_{mu,(n2,n3)}(T1,T2,T3) = sum_i x_i^mu A^mu(i,T1) B^mu(i,T2) C^mu(i,T3)
// with x = w gamma, its conjugate, or w, and each factor a block at order
//   k = a*n2 + b*n3 + c, optionally conjugated.
//
// App. A.1, Table 1 (double- and triple-counting corrections), read as the
// inclusion-exclusion of the quadruplet sum over distinct j, k, l:
//   Upsilon' = Upsilon - [T1=T2] sum_i x c12(T1) C(T3) - [T1=T3] sum_i x c13(T1) B(T2)
//                      - [T2=T3] sum_i x A(T1) c23(T2) + 2 [T1=T2=T3] sum_i x t(T1).
#pragma once

namespace fpcf4 {

enum { X_G = 0, X_GC = 1, X_W = 2 };        // centre factor w g, conj(w g), w
enum { F_G = 0, F_W = 1 };                  // contraction blocks
enum { C_Q = 0, C_A = 1, C_V = 2 };         // pair-correction blocks
enum { T_T8 = 0, T_T4 = 1, T_M4 = 2, T_M0 = 3, T_U = 4 };  // triple blocks (record specials)

struct Fac {
  int fam, conj, a, b, c;
};
struct MuFactors {
  int x;
  Fac A, B, C;
};
struct MuCorr {
  Fac c12, c13, c23;
  int t;
};

__host__ __device__ constexpr MuFactors mu_factors(int mu) {
  switch (mu) {
    case 0: return {X_G,  {F_G, 0, 1, 1, -3},   {F_G, 0, -1, 0, -2}, {F_G, 0, 0, -1, -3}};
    case 1: return {X_GC, {F_G, 0, 1, 1, -1},   {F_G, 0, -1, 0, -2}, {F_G, 0, 0, -1, -1}};
    case 2: return {X_G,  {F_G, 1, -1, -1, -1}, {F_G, 0, -1, 0, -2}, {F_G, 0, 0, -1, -3}};
    case 3: return {X_G,  {F_G, 0, 1, 1, -3},   {F_G, 1, 1, 0, -2},  {F_G, 0, 0, -1, -3}};
    case 4: return {X_G,  {F_G, 0, 1, 1, -3},   {F_G, 0, -1, 0, -2}, {F_G, 1, 0, 1, -1}};
    case 5: return {X_GC, {F_G, 1, -1, -1, -3}, {F_G, 0, -1, 0, -2}, {F_G, 0, 0, -1, -1}};
    case 6: return {X_GC, {F_G, 0, 1, 1, -1},   {F_G, 1, 1, 0, -2},  {F_G, 0, 0, -1, -1}};
    case 7: return {X_GC, {F_G, 0, 1, 1, -1},   {F_G, 0, -1, 0, -2}, {F_G, 1, 0, 1, -3}};
    default: return {X_W, {F_W, 0, 1, 1, 0},    {F_W, 0, -1, 0, 0},  {F_W, 0, 0, -1, 0}};
  }
}

__host__ __device__ constexpr MuCorr mu_corr(int mu) {
  switch (mu) {
    case 0: return {{C_Q, 0, 0, 1, -5}, {C_Q, 0, 1, 0, -6}, {C_Q, 0, -1, -1, -5}, T_T8};
    case 1: return {{C_Q, 0, 0, 1, -3}, {C_Q, 0, 1, 0, -2}, {C_Q, 0, -1, -1, -3}, T_T4};
    case 2: return {{C_A, 0, 0, 1, -1}, {C_A, 0, 1, 0, -2}, {C_Q, 0, -1, -1, -5}, T_M4};
    case 3: return {{C_A, 0, 0, 1, -1}, {C_Q, 0, 1, 0, -6}, {C_A, 0, -1, -1, -1}, T_M4};
    case 4: return {{C_Q, 0, 0, 1, -5}, {C_A, 0, 1, 0, -2}, {C_A, 0, -1, -1, -1}, T_M4};
    case 5: return {{C_A, 0, 0, 1, 1},  {C_A, 0, 1, 0, 2},  {C_Q, 0, -1, -1, -3}, T_M0};
    case 6: return {{C_A, 0, 0, 1, 1},  {C_Q, 0, 1, 0, -2}, {C_A, 0, -1, -1, 1},  T_M0};
    case 7: return {{C_Q, 0, 0, 1, -3}, {C_A, 0, 1, 0, 2},  {C_A, 0, -1, -1, 1},  T_M0};
    default: return {{C_V, 0, 0, 1, 0}, {C_V, 0, 1, 0, 0},  {C_V, 0, -1, -1, 0},  T_U};
  }
}

}  // namespace fpcf4
