// Internal interface of the fit for the contraction driver (xi~ per bra super-block
// from the factors isdf_fit keeps).
#pragma once
#include "common.hpp"

namespace xtc {

// xi (sys 0) or xi~^c (sys 1 + c) at grid points [g0, g0 + cn) from one system's kept
// factor chol_sys (XTC_CHOL_SYSTEM_DOUBLES(n_mu) doubles): the fit's own right-hand-side
// products and blocked solves, so the columns equal the fit's bit for bit.
// phimu: [4][n_orb][n_mu] at the pivots; out [n_mu][cn] (row stride ldo);
// P, R: scratch [n_mu][cn] (row stride ldr).
xtc_status fit_columns(const double* phi4, long n_g, int n_orb, const double* phimu, int n_mu,
                       int sys, const double* chol_sys, long g0, long cn, double* out, long ldo,
                       double* P, double* R, long ldr, hipStream_t st);

// out[r][m] = phi4[r][piv[m]] for r < rows (rows = 4 n_orb for phi4 [4][n_orb][n_g]).
xtc_status gather_pivot_rows(const double* phi4, long n_g, int rows, const long* piv, int n_mu,
                             double* out, hipStream_t st);

}  // namespace xtc
