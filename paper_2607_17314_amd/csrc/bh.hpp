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

// Nuclear sums of one pair, added into F[o] and GF[o][c] (see the regrouping above), from
// the bra point's values a_I, grad a_I (a1, ax, ay, az) and the ket point's gamma_{I,o,m} (g)
__device__ __forceinline__ void bh_nuclear_terms(double a1, double ax, double ay, double az,
                                                 const double (*g)[BH_NP], double* F,
                                                 double (*GF)[3]) {
  const double a2 = a1 * a1, a3 = a2 * a1;
#pragma unroll
  for (int o = 0; o < BH_NO; ++o) {
    F[o] += g[o][0] + a1 * g[o][1] + a2 * g[o][2] + a3 * g[o][3];
    const double Dv = g[o][1] + 2.0 * a1 * g[o][2] + 3.0 * a2 * g[o][3];
    GF[o][0] += Dv * ax;
    GF[o][1] += Dv * ay;
    GF[o][2] += Dv * az;
  }
}

// grad_1 u = N + S rhat from the nuclear sums and the pair difference (dx, dy, dz) =
// r_bra - r_ket. out: d_x u, d_y u, d_z u, |grad_1 u|^2.
__device__ __forceinline__ void bh_finish(const EECoef& cf, const double* F, const double (*GF)[3],
                                          double dx, double dy, double dz, double* out) {
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double t = 1.0 / (1.0 + cf.d * r);
  const double e = cf.d * r * t;
  const double t2 = t * t;
  const double E[BH_NO] = {1.0, e, e * e, e * e * e};
  double N[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) N[c] = GF[0][c] + E[1] * GF[1][c] + E[2] * GF[2][c] + E[3] * GF[3][c];
  double q = 0.0;   // U'_ee(rbar), the pure electron-electron part
  for (int j = cf.n1 - 1; j >= 0; --j) q = q * e + cf.q1[j];
  double S = cf.d * t2 * (F[1] + 2.0 * E[1] * F[2] + 3.0 * E[2] * F[3] + q);
  if (r > 0.0) {
    const double sr = S / r;
    out[0] = N[0] + sr * dx;
    out[1] = N[1] + sr * dy;
    out[2] = N[2] + sr * dz;
    out[3] = out[0] * out[0] + out[1] * out[1] + out[2] * out[2];
  } else {
    out[0] = N[0];
    out[1] = N[1];
    out[2] = N[2];
    out[3] = N[0] * N[0] + N[1] * N[1] + N[2] * N[2] + S * S;
  }
}

// grad_1 u at one pair: TB[I][(a, da/dx, da/dy, da/dz)][slot] holds the bra point's nuclear
// values in slot gb of NBR, TK[I][o][m] = gamma_{I,o,m} of the ket point, (dx, dy, dz) =
// r_bra - r_ket.
template <int NBR>
__device__ __forceinline__ void bh_pair_channels(const EECoef& cf, int nn,
                                                 const double (*TB)[4][NBR], int gb,
                                                 const double (*TK)[BH_NO][BH_NP], double dx,
                                                 double dy, double dz, double* out) {
  double F[BH_NO] = {0.0, 0.0, 0.0, 0.0};
  double GF[BH_NO][3] = {};
  for (int I = 0; I < nn; ++I)
    bh_nuclear_terms(TB[I][0][gb], TB[I][1][gb], TB[I][2][gb], TB[I][3][gb], TK[I], F, GF);
  bh_finish(cf, F, GF, dx, dy, dz, out);
}

// gamma_{I,o,m}(g) = sum_n csym[type(I)][m][n][o] a_I(g)^n into out[o][m]
__device__ __forceinline__ void bh_ket_gamma(const BHTable* __restrict__ T, int I, double x,
                                             double y, double z, double (*out)[BH_NP]) {
  const double a = bh_a(T, I, x, y, z);
  const double A2[BH_NP] = {1.0, a, a * a, a * a * a};
  const int ty = T->type[I];
#pragma unroll
  for (int o = 0; o < BH_NO; ++o)
#pragma unroll
    for (int m = 0; m < BH_NP; ++m) {
      double s = 0.0;
#pragma unroll
      for (int n = 0; n < BH_NP; ++n) s += T->csym[ty][m][n][o] * A2[n];
      out[o][m] = s;
    }
}

}  // namespace xtc
