// Internal interface between the contraction driver and its stage-1 kernels.
#pragma once
#include "common.hpp"

namespace xtc {

constexpr int MAXQ = 16;

// EE correlator u = sum_k c_k rbar^{o_k}, rbar = d r t, t = 1/(1 + d r), as
// polynomials in rbar:  u' = d t^2 Q1(rbar),  (u'/r)_{o>=2} = d^2 t^3 Q2(rbar),
// u''_{o>=2} = d^2 t^4 Q3(rbar);  c1 = sum of c_k over o_k = 1.
struct EECoef {
  double d;
  double c1;
  double q1[MAXQ];
  double q2[MAXQ];
  double q3[MAXQ];
  int n1, n2, n3;
};

xtc_status ee_coefficients(const xtc_correlator* corr, EECoef* out);

// Stage 1 over one bra super-block [b0, b0 + bn): panel[ch][row][b - b0] for
// rows 0..n_mu + 1, ch = gx, gy, gz, sq (, lap). Row n_mu uses the reference
// density rho_gamma (exact field), row n_mu + 1 the ISDF density
// rhot = sum_l G_l xi_l, so that its gradient channels are H_{g,c} = sum_l G_l calG^c_{l,g}.
struct BHTable;

struct Stage1Args {
  const double* xyz; const double* w; const double* xi; const double* rho; const double* rhot;
  long n_g; int n_mu; long b0; long bn;
  double* panel; long rows_pad; long bp;
  int nch;
  const BHTable* bh = nullptr;   // device table of a BH correlator (FP64 path), or nullptr for EE
  bool rho_rows = true;          // false: the density rows n_mu, n_mu + 1 may be left unset
  const float* xi32 = nullptr;   // split path: xi in FP32 (then xi is nullptr)
  const BHTable* bh_host = nullptr;   // the host copy of *bh (split path: channel scales)
  double* pv64 = nullptr;   // FP64 path, BH form: pair-value buffer of bh_f64_pv_bytes(bp), or
                            // nullptr for the pair values made beside the products
};

xtc_status stage1_f64(const Stage1Args& a, const EECoef& cf, hipStream_t st);
xtc_status stage1_split_f16(const Stage1Args& a, const EECoef& cf, void* scratch,
                            size_t scratch_bytes, hipStream_t st);
size_t split_scratch_bytes(long n_g, int n_mu);
size_t rho_row_scratch_bytes(long bp);
// rows n_mu and n_mu + 1 of the panel in FP64 (split path); part: rho_row_scratch_bytes
xtc_status rho_row_f64(const Stage1Args& a, const EECoef& cf, double* part, hipStream_t st);
xtc_status split_prepare(const Stage1Args& a, void* scratch, hipStream_t st);
// BH form in split precision: the pair values of one launch's ket range, generated in FP64
// and stored pre-split, then the same split products. Its scratch follows the split
// operand and the density-row partials: bh_split_scratch_bytes(bp) more bytes.
size_t bh_split_scratch_bytes(long bp);
xtc_status stage1_split_bh(const Stage1Args& a, const EECoef& cf, void* scratch,
                           size_t scratch_bytes, hipStream_t st);
// BH form on the FP64 path with a pair-value buffer: the four channels of the pairs of ket
// chunks [c0, c0 + nloc) (chunks of 128 kets, nloc <= 128) in FP64 into a.pv64
size_t bh_f64_pv_bytes(long bp);
xtc_status bh_pair_values_f64(const Stage1Args& a, const EECoef& cf, long c0, long nloc,
                              hipStream_t st);

}  // namespace xtc
