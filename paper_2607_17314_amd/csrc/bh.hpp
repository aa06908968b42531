// Multi-centre Boys-Handy correlator (Jastrow section, eqs. bh-scaled and bh-u):
//   u(1,2) = sum_I sum_k c^{type(I)}_k [a_1I^m a_2I^n + a_2I^m a_1I^n] rbar12^o,
//   a_iI = b r_iI / (1 + b r_iI),  rbar12 = d r12 / (1 + d r12).
// The terms are regrouped for the pair kernels. With
//   csym[t][m][n][o] = sum of c^t over the terms (m, n, o) and (n, m, o),
// the nuclear part ((m, n) != (0, 0)) is, for each power o of rbar12,
//   F_o(1,2) = sum_I sum_m a_1I^m gamma_{I,o,m}(2),  gamma_{I,o,m} = sum_n csym[m][n][o] a_2I^n,
// so that grad_1 u = N + S rhat12 with
//   N = sum_o rbar^o grad_1 F_o,  grad_1 F_o = sum_I (sum_m m a_1I^{m-1} gamma_{I,o,m}) grad a_1I,
//   S = d t^2 (sum_o o rbar^{o-1} F_o + U'_ee(rbar)),
// where U_ee = sum_o cee_o rbar^o collects the (0, 0, o) terms (each carries a factor 2
// per nucleus). At r12 = 0 the rhat12 part is dropped and |grad u|^2 = |N|^2 + S^2.
#pragma once
#include "contract.hpp"

namespace xtc {

constexpr int BH_MAXNUC = 24;   // nuclei
constexpr int BH_MAXTYPE = 2;   // nucleus types
constexpr int BH_NP = 4;        // powers 0..3 of a_iI in the nuclear terms
constexpr int BH_NO = 4;        // powers 0..3 of rbar12 in the nuclear terms

struct BHTable {
  int n_nuc;
  int n_types;
  double d;
  double nuc[BH_MAXNUC][4];                      // x, y, z, b
  int type[BH_MAXNUC];
  int n_of_type[BH_MAXTYPE];
  double csym[BH_MAXTYPE][BH_NP][BH_NP][BH_NO];  // [t][m][n][o]; (0, 0, o) kept out
};

// Builds the table and the EE coefficients of the (0, 0, o) terms; validates the
// correlator (XTC_ERR_INVALID_ARG, or XTC_ERR_UNSUPPORTED beyond the limits above).
xtc_status bh_build(const xtc_correlator* corr, BHTable* T, EECoef* ee);

// a_I and grad a_I at one point (grad a_I = b t^2 (x - R_I) / r, 0 at the nucleus itself)
__device__ __forceinline__ void bh_nuc_point(const BHTable* __restrict__ T, int I, double x,
                                             double y, double z, double* out4) {
  const double dx = x - T->nuc[I][0], dy = y - T->nuc[I][1], dz = z - T->nuc[I][2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double b = T->nuc[I][3];
  const double t = 1.0 / (1.0 + b * r);
  out4[0] = b * r * t;
  const double s = r > 0.0 ? b * t * t / r : 0.0;
  out4[1] = s * dx;
  out4[2] = s * dy;
  out4[3] = s * dz;
}

__device__ __forceinline__ double bh_a(const BHTable* __restrict__ T, int I, double x, double y,
                                       double z) {
  const double dx = x - T->nuc[I][0], dy = y - T->nuc[I][1], dz = z - T->nuc[I][2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double b = T->nuc[I][3];
  return b * r / (1.0 + b * r);
}

}  // namespace xtc
