// Host-side regrouping of the multi-centre Boys-Handy correlator (eq. bh-u).
#include "bh.hpp"

namespace xtc {

xtc_status bh_build(const xtc_correlator* corr, BHTable* T, EECoef* ee) {
  XTC_REQUIRE(corr && corr->form == XTC_U_BH, "BH correlator expected");
  XTC_REQUIRE(corr->n_terms > 0 && corr->mno && corr->c && corr->d > 0.0, "bad BH correlator");
  XTC_REQUIRE(corr->n_nuc > 0 && corr->nuc_xyz && corr->nuc_type && corr->b,
              "BH correlator needs nuclei, their types and b");
  if (corr->n_nuc > BH_MAXNUC || corr->n_types > BH_MAXTYPE || corr->n_types < 1) {
    set_error("BH correlator: at most 24 nuclei and 2 nucleus types are supported");
    return XTC_ERR_UNSUPPORTED;
  }
  *T = BHTable{};
  *ee = EECoef{};
  T->n_nuc = corr->n_nuc;
  T->n_types = corr->n_types;
  T->d = corr->d;
  for (int t = 0; t < corr->n_types; ++t)
    XTC_REQUIRE(corr->b[t] > 0.0, "BH correlator: b must be positive");
  for (int I = 0; I < corr->n_nuc; ++I) {
    const int t = corr->nuc_type[I];
    XTC_REQUIRE(t >= 0 && t < corr->n_types, "BH correlator: nucleus type out of range");
    for (int q = 0; q < 3; ++q) T->nuc[I][q] = corr->nuc_xyz[3 * I + q];
    T->nuc[I][3] = corr->b[t];
    T->type[I] = t;
    T->n_of_type[t] += 1;
  }
  double cee[MAXQ + 1] = {0.0};
  int omax = 0;
  for (int k = 0; k < corr->n_terms; ++k) {
    const int m = corr->mno[3 * k], n = corr->mno[3 * k + 1], o = corr->mno[3 * k + 2];
    XTC_REQUIRE(m >= 0 && n >= 0 && o >= 0, "BH correlator: negative power");
    if (m == 0 && n == 0) {
      if (o > MAXQ) {
        set_error("BH correlator: electron-electron power above the supported maximum");
        return XTC_ERR_UNSUPPORTED;
      }
      // [a^0 a^0 + a^0 a^0] = 2 for every nucleus of each type
      for (int t = 0; t < corr->n_types; ++t)
        cee[o] += 2.0 * T->n_of_type[t] * corr->c[(long)t * corr->n_terms + k];
      if (o > omax) omax = o;
      continue;
    }
    if (m >= BH_NP || n >= BH_NP || o >= BH_NO) {
      set_error("BH correlator: nuclear terms need m, n, o <= 3");
      return XTC_ERR_UNSUPPORTED;
    }
    for (int t = 0; t < corr->n_types; ++t) {
      const double c = corr->c[(long)t * corr->n_terms + k];
      T->csym[t][m][n][o] += c;
      T->csym[t][n][m][o] += c;
    }
  }
  // pure electron-electron part as an EE polynomial (o = 0 carries no derivative)
  ee->d = corr->d;
  for (int o = 1; o <= omax; ++o) {
    ee->q1[o - 1] += cee[o] * o;
    if (o >= 2) {
      ee->q2[o - 2] += cee[o] * o;
      ee->q3[o - 2] += cee[o] * o * (o - 1);
    }
    if (o == 1) ee->c1 += cee[o];
  }
  ee->n1 = omax >= 1 ? omax : 0;
  ee->n2 = omax >= 2 ? omax - 1 : 0;
  ee->n3 = ee->n2;
  return XTC_OK;
}

}  // namespace xtc
