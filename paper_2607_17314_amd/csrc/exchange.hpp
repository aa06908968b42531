// Internal interface of the exchange intermediates (xTC Terms 2 and 3), shared by
// xtc_exchange_terms and the fused pass of xtc_kernel_contract.
#pragma once
#include "common.hpp"

namespace xtc {

struct EECoef;

// Scratch and sizes of the X2/X3 accumulation for super-blocks of bp bra points.
// Split path: the projected rows Q = P xi over the whole grid (FP64, then cut into
// the split stage-1 operand) and a second stage-1 panel that receives R directly.
struct ExWork {
  double* phia; double* P; double* RQ; double* T; double* Xp; int2* tiles;
  void* gsplit; size_t gsplit_bytes;
  double* Qf; void* splitQ; size_t splitQ_bytes; double* panelR; long rows_padR;
  int* pex; int* ex2; int* ex3; long pex_stride;
  long npair, npl, tpart, bp, nr;
  int ntile, n_orb, n_q, n_mu, precision;
};

void ex_layout(Arena& ar, long n_g, long bp, int n_mu, int n_orb, int n_q, int precision,
               ExWork* W);
// once per call: the pair-tile table, the projector rows P and (split path) Q = P xi
// with its split stage-1 operand
xtc_status ex_prepare(ExWork& W, const double* phi_piv, const double* lq, const double* xyz,
                      const double* w, const double* xi, long n_g, hipStream_t st);
// one bra super-block [b0, b0 + bn) whose calG panel (channels 0..2, rows_pad rows of
// bp points) is ready; `first` starts the accumulation
xtc_status ex_block(ExWork& W, const EECoef& cf, const double* panel, long rows_pad,
                    const double* xyz, const double* xi, long n_g, const double* w, long b0,
                    long bn, bool first, bool want2, bool want3, hipStream_t st);
// mirror the packed q <= s accumulators into X2, X3 (zeros when no bra point was summed)
xtc_status ex_finish(ExWork& W, double* X2, double* X3, bool empty, hipStream_t st);
xtc_status check_exchange_args(const xtc_exchange* ex, int32_t n_mu);

}  // namespace xtc
