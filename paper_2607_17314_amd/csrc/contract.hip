// Driver of xtc_kernel_contract: stage 1 per bra super-block (grid-pair kernel
// tiles generated on the fly), then stage 2 on the super-block's panel
// (K-kernel section eqs. K1-isdf and K3-isdf; xTC Terms 1 and 4):
//   u1^c += (w xi~^c) calG^c^T,  u3 += (w xi) T3^T,  ulap += (w xi) TL^T,
//   D4   += sum_c (calG^c wt) calG^c^T,  D1 += (w xi) V^T,
// with wt_g = w_g sum_l G_l xi_l(g), H_gc = sum_l G_l calG^c_lg, V = sum_c H_c calG^c,
// all as FP64 MFMA GEMMs accumulated in place. The rho row of the panel gives
// the exact field A_gamma and the ISDF-free energy-scale sums.
#include <mutex>
#include "contract.hpp"
#include "plans.hpp"
#include "timing.hpp"
#include "gemm_split.hpp"
#include "bh.hpp"
#include "exchange.hpp"
#include "fit.hpp"

namespace xtc {

constexpr long SUPER_BLOCK = 16384;

xtc_status ee_coefficients(const xtc_correlator* corr, EECoef* cf) {
  *cf = EECoef{};
  cf->d = corr->d;
  int omax = 0;
  for (int k = 0; k < corr->n_terms; ++k) {
    const int* t = corr->mno + 3 * k;
    if (t[0] != 0 || t[1] != 0 || t[2] < 0) {
      set_error("EE correlator terms must be (0, 0, o) with o >= 0");
      return XTC_ERR_INVALID_ARG;
    }
    if (t[2] > omax) omax = t[2];
  }
  if (omax > MAXQ) {
    set_error("EE correlator power above the supported maximum");
    return XTC_ERR_UNSUPPORTED;
  }
  for (int k = 0; k < corr->n_terms; ++k) {
    const int o = corr->mno[3 * k + 2];
    const double c = corr->c[k];
    if (o >= 1) cf->q1[o - 1] += c * o;
    if (o >= 2) {
      cf->q2[o - 2] += c * o;
      cf->q3[o - 2] += c * o * (o - 1);
    }
    if (o == 1) cf->c1 += c;
  }
  cf->n1 = omax >= 1 ? omax : 0;
  cf->n2 = omax >= 2 ? omax - 1 : 0;
  cf->n3 = cf->n2;
  return XTC_OK;
}

__global__ void k_gather_G(const double* __restrict__ rho, const long* __restrict__ piv, int n_mu,
                           double* __restrict__ G) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n_mu) G[i] = rho[piv[i]];
}

// Per bra point of the super-block: wt = w rhot, H_c from the panel's rhot row,
// and the energy-scale partials w rho T3rho and w rho |A_gamma|^2; also copies the field.
__global__ __launch_bounds__(256) void k_point_vectors(
    const double* __restrict__ rhot, const double* __restrict__ w, const double* __restrict__ rho,
    long n_g, int n_mu, long b0, long bn, const double* __restrict__ panel, long rows_pad, long bp,
    int need_h, double* __restrict__ wt, double* __restrict__ H, double* __restrict__ e3x,
    double* __restrict__ e4x, double* __restrict__ e3, double* __restrict__ e4,
    double* __restrict__ field) {
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= bn) return;
  const long g = b0 + t;
  if (need_h) {
    wt[t] = w[g] * rhot[g];
    H[t] = panel[((long)0 * rows_pad + n_mu + 1) * bp + t];
    H[bp + t] = panel[((long)1 * rows_pad + n_mu + 1) * bp + t];
    H[2 * bp + t] = panel[((long)2 * rows_pad + n_mu + 1) * bp + t];
  }
  const double a0 = panel[((long)0 * rows_pad + n_mu) * bp + t];
  const double a1 = panel[((long)1 * rows_pad + n_mu) * bp + t];
  const double a2 = panel[((long)2 * rows_pad + n_mu) * bp + t];
  const double t3 = panel[((long)3 * rows_pad + n_mu) * bp + t];
  const double wr = w[g] * rho[g];
  e3x[t] = wr * t3;
  e4x[t] = wr * (a0 * a0 + a1 * a1 + a2 * a2);
  // ISDF energy-scale terms on the rhot row: G^T u3 G = sum_g w rhot T3rhot,
  // G^T D4 G = sum_g w rhot |H|^2 = (1/2) 2 G^T D1 G
  const double h0 = panel[((long)0 * rows_pad + n_mu + 1) * bp + t];
  const double h1 = panel[((long)1 * rows_pad + n_mu + 1) * bp + t];
  const double h2 = panel[((long)2 * rows_pad + n_mu + 1) * bp + t];
  const double t3t = panel[((long)3 * rows_pad + n_mu + 1) * bp + t];
  const double wrt = w[g] * rhot[g];
  e3[t] = wrt * t3t;
  e4[t] = wrt * (h0 * h0 + h1 * h1 + h2 * h2);
  if (field) {
    field[g] = a0;
    field[n_g + g] = a1;
    field[2 * n_g + g] = a2;
  }
}

// V[nu][g] = sum_c H_c(g) calG^c[nu][g]
__global__ __launch_bounds__(256) void k_form_V(const double* __restrict__ panel, long rows_pad,
                                                long bp, int n_mu, long bn,
                                                const double* __restrict__ H,
                                                double* __restrict__ V) {
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long)n_mu * bn) return;
  const long nu = t / bn, g = t % bn;
  V[nu * bp + g] = H[g] * panel[nu * bp + g] + H[bp + g] * panel[(rows_pad + nu) * bp + g] +
                   H[2 * bp + g] * panel[(2 * rows_pad + nu) * bp + g];
}

__global__ void k_mul(const double* __restrict__ a, const double* __restrict__ b, long n,
                      double* __restrict__ out) {
  long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}

struct ConLayout {
  long* piv; double* G; double* rhot; double* panel; double* V; double* wt; double* H; double* e3x;
  double* e4x; double* e3; double* e4; double* sums; double* red; void* split; size_t split_bytes;
  void* gsplit; size_t gsplit_bytes; BHTable* bh;
  void* gsplit2;   // second operand scratch: the u1/u3 products on the auxiliary stream
  double* pv64;    // FP64 path, BH form: the pair values of one ket launch
  // xi~ per bra super-block: the orbitals at the pivots, xi~ of the block, solve scratch
  double* phimu; double* xigb; double* fitP; double* fitR;
  long bp; long rows_pad; int nsb; int nch;
  ExWork ex;   // exchange intermediates (when requested)
};

// Width of the bra super-blocks: the whole grid rounded up to 64 points, at most SUPER_BLOCK.
static long default_bp(int64_t n_g) {
  return n_g < SUPER_BLOCK ? ((n_g + 63) / 64) * 64 : SUPER_BLOCK;
}

// bp: the super-block width, a multiple of 64 (every stage-1 and stage-2 launch of a
// super-block covers at most bp bra points, so any such width gives the same sums up to
// their order).
static ConLayout layout_con(Arena& ar, int64_t n_g, int n_mu, uint32_t channels, int precision,
                            int n_orb, int n_q, long bp, bool xig_blocks, bool dual, bool bh) {
  ConLayout C;
  C.nch = (channels & XTC_ULAP) ? 5 : 4;
  C.bp = bp;
  C.rows_pad = ((n_mu + 2 + 255) / 256) * 256;   // whole row tiles of the split kernel
  C.nsb = (int)cdiv(n_g, C.bp);
  C.piv = ar.take<long>(n_mu);
  C.G = ar.take<double>(n_mu);
  C.rhot = ar.take<double>(n_g);
  C.panel = ar.take<double>((size_t)C.nch * C.rows_pad * C.bp);
  C.V = (channels & XTC_D1) ? ar.take<double>((size_t)n_mu * C.bp) : nullptr;
  C.wt = ar.take<double>(C.bp);
  C.H = ar.take<double>(3 * (size_t)C.bp);
  C.e3x = ar.take<double>(C.bp);
  C.e4x = ar.take<double>(C.bp);
  C.e3 = ar.take<double>(C.bp);
  C.e4 = ar.take<double>(C.bp);
  C.sums = ar.take<double>(4 * (size_t)C.nsb + 4);
  C.red = ar.take<double>(1024);
  C.split_bytes = precision == XTC_SPLIT_F16
                      ? split_scratch_bytes(n_g, n_mu) + rho_row_scratch_bytes(C.bp) +
                            (bh ? bh_split_scratch_bytes(C.bp) : 0)
                      : 0;
  C.split = C.split_bytes ? (void*)ar.take<char>(C.split_bytes) : nullptr;
  // stage-2 GEMMs in split precision: the split operand tiles of one product
  C.gsplit_bytes = precision == XTC_SPLIT_F16 ? gemm_split_scratch_bytes(n_mu, n_mu, C.bp) : 0;
  C.gsplit = C.gsplit_bytes ? (void*)ar.take<char>(C.gsplit_bytes) : nullptr;
  C.gsplit2 = (dual && C.gsplit_bytes) ? (void*)ar.take<char>(C.gsplit_bytes) : nullptr;
  C.bh = ar.take<BHTable>(1);
  C.pv64 = (bh && precision == XTC_FP64) ? ar.take<double>(bh_f64_pv_bytes(C.bp) / sizeof(double))
                                         : nullptr;
  C.phimu = C.xigb = C.fitP = C.fitR = nullptr;
  if (xig_blocks && (channels & XTC_U1)) {
    C.phimu = ar.take<double>(4 * (size_t)n_orb * n_mu);
    C.xigb = ar.take<double>(3 * (size_t)n_mu * C.bp);
    C.fitP = ar.take<double>((size_t)n_mu * C.bp);
    C.fitR = ar.take<double>((size_t)n_mu * C.bp);
  }
  C.ex = ExWork{};
  if (n_q > 0) ex_layout(ar, n_g, C.bp, n_mu, n_orb, n_q, precision, &C.ex);
  return C;
}

size_t ws_contract(int64_t n_g, int n_mu, uint32_t flags, int n_orb, int n_q) {
  Arena ar(nullptr, 0);
  layout_con(ar, n_g, n_mu, flags & 0xffff, (int)((flags >> 16) & 0xff), n_orb, n_q,
             default_bp(n_g), (flags & XTC_WS_XIGRAD_BLOCKS) != 0, true,
             (flags & XTC_WS_BH) != 0);
  return ar.used;
}

// rhot[g] = sum_mu G[mu] xi[mu][g] for xi stored in FP32, summed in FP64 in mu order
__global__ __launch_bounds__(256) void k_rhot_f32(const double* __restrict__ G,
                                                  const float* __restrict__ xi, int n_mu, long n_g,
                                                  double* __restrict__ rhot) {
  const long g = (long)blockIdx.x * 256 + threadIdx.x;
  if (g >= n_g) return;
  double s = 0.0;
  for (int m = 0; m < n_mu; ++m) s += G[m] * (double)xi[(long)m * n_g + g];
  rhot[g] = s;
}

}  // namespace xtc

using namespace xtc;

static bool xig_on_the_fly(uint32_t channels, const double* xigrad) {
  return (channels & XTC_U1) && !xigrad;
}

static xtc_status check_contract_args(const xtc_grid* grid, const xtc_correlator* corr,
                                      int32_t n_mu, const void* xi, const double* xigrad,
                                      const double* rho, const int64_t* pivots,
                                      uint32_t channels, int32_t precision,
                                      const xtc_exchange* ex, const xtc_xi_source* src) {
  XTC_REQUIRE(grid && corr && xi && rho && pivots, "contract: null argument");
  XTC_REQUIRE(grid->n_g > 0 && grid->xyz && grid->w, "contract: empty grid");
  XTC_REQUIRE(n_mu > 0 && n_mu <= grid->n_g, "contract: bad n_mu");
  XTC_REQUIRE(!xig_on_the_fly(channels, xigrad) || (src && src->phi4 && src->chol && src->n_orb > 0),
              "contract: XTC_U1 needs xigrad, or the orbitals and kept factors in src");
  if (src) {
    XTC_REQUIRE(src->xi_prec == XTC_FP64 || src->xi_prec == XTC_FP32,
                "contract: src->xi_prec must be FP64 or FP32");
    if (src->xi_prec == XTC_FP32 && (precision != XTC_SPLIT_F16 || ex)) {
      set_error("contract: FP32 xi is read by the split path without exchange outputs only");
      return XTC_ERR_UNSUPPORTED;
    }
  }
  XTC_REQUIRE((channels & ~127u) == 0, "contract: unknown channel bits");
  XTC_REQUIRE(precision == XTC_FP64 || precision == XTC_SPLIT_F16, "contract: bad precision");
  XTC_REQUIRE(corr->n_terms > 0 && corr->mno && corr->c && corr->d > 0.0,
              "contract: bad correlator");
  for (int m = 0; m < n_mu; ++m)
    XTC_REQUIRE(pivots[m] >= 0 && pivots[m] < grid->n_g, "contract: pivot index out of range");
  XTC_REQUIRE(corr->form == XTC_U_EE || corr->form == XTC_U_BH, "contract: unknown correlator form");
  if (corr->form == XTC_U_BH && precision != XTC_FP64 && ex) {
    set_error("contract: the exchange outputs of the BH correlator are formed on the FP64 path only");
    return XTC_ERR_UNSUPPORTED;
  }
  if (corr->form == XTC_U_BH && (channels & XTC_ULAP)) {
    set_error("contract: the Laplacian channel is defined for the EE form only");
    return XTC_ERR_UNSUPPORTED;
  }
  return XTC_OK;
}

__global__ void k_fill_zero(double* __restrict__ x, long n) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t < n) x[t] = 0.0;
}

// The body of xtc_kernel_contract and xtc_kernel_contract_noalloc: scratch is ws (its
// bytes), the bra super-blocks are bp points wide (a multiple of 64).
static xtc_status contract_impl(const xtc_grid* grid, const xtc_correlator* corr, int32_t n_mu,
                                const void* xi_any, const double* xigrad, const double* rho,
                                const int64_t* pivots, uint32_t channels, int32_t precision,
                                int64_t bra_begin, int64_t bra_end, double* u1, double* u3,
                                double* ulap, double* D1, double* D4, double* field,
                                double* escale, const xtc_exchange* ex, const xtc_xi_source* src,
                                void* ws, size_t ws_bytes, long bp, bool dual, void* stream) {
  XTC_TRY(check_contract_args(grid, corr, n_mu, xi_any, xigrad, rho, pivots, channels, precision,
                              ex, src));
  // xi in FP64 (xi) or FP32 (xi32, split path only); xi~ stored or formed per block
  const float* xi32 = (src && src->xi_prec == XTC_FP32) ? (const float*)xi_any : nullptr;
  const double* xi = xi32 ? nullptr : (const double*)xi_any;
  const bool fly = xig_on_the_fly(channels, xigrad);
  XTC_REQUIRE(bra_begin >= 0 && bra_begin < bra_end && bra_end <= grid->n_g,
              "contract: bra range must be non-empty and inside the grid");
  if (ex) XTC_TRY(check_exchange_args(ex, n_mu));
  XTC_REQUIRE(!(channels & XTC_U1) || u1, "contract: u1 output NULL");
  XTC_REQUIRE(!(channels & XTC_U3) || u3, "contract: u3 output NULL");
  XTC_REQUIRE(!(channels & XTC_ULAP) || ulap, "contract: ulap output NULL");
  XTC_REQUIRE(!(channels & XTC_D1) || D1, "contract: D1 output NULL");
  XTC_REQUIRE(!(channels & XTC_D4) || D4, "contract: D4 output NULL");
  XTC_REQUIRE(!(channels & XTC_FIELD) || field, "contract: field output NULL");
  XTC_REQUIRE(!(channels & XTC_ESCALE) || escale, "contract: escale output NULL");
  EECoef cf;
  BHTable bt;
  const bool bh = corr->form == XTC_U_BH;
  if (bh) XTC_TRY(bh_build(corr, &bt, &cf));
  else XTC_TRY(ee_coefficients(corr, &cf));
  hipStream_t st = as_stream(stream);
  const long n_g = grid->n_g;
  Arena ar(ws, ws_bytes);
  const int n_orb_l = ex ? ex->n_orb : (fly ? src->n_orb : 0);
  ConLayout C = layout_con(ar, n_g, n_mu, channels, precision, n_orb_l, ex ? ex->n_q : 0, bp, fly,
                           dual, bh);
  XTC_TRY(need_ws(ar));
  XTC_TRY(check_weights(grid, ws, ws_bytes, st, "xtc_kernel_contract"));
  hipStream_t st2 = nullptr;
  CallEvents evs;
  if (C.gsplit2) {
    XTC_TRY(aux_stream(0, &st2));
    XTC_TRY(evs.create(2));
  }
  hipEvent_t ev_fork = evs.ev[0], ev_join = evs.ev[1];
  if (bh) XTC_HIP(hipMemcpyAsync(C.bh, &bt, sizeof(BHTable), hipMemcpyHostToDevice, st));
  XTC_HIP(hipMemcpyAsync(C.piv, pivots, sizeof(long) * n_mu, hipMemcpyHostToDevice, st));
  if (ex) XTC_TRY(ex_prepare(C.ex, ex->phi_piv, ex->lq, grid->xyz, grid->w, xi, n_g, st));
  hipLaunchKernelGGL(k_gather_G, dim3(cdiv(n_mu, 256)), dim3(256), 0, st, rho,
                     (const long*)C.piv, n_mu, C.G);
  XTC_CHECK_LAUNCH();
  if (src && src->rhot) {   // ISDF density rhot = G^T xi, given (from the fit's FP64 xi)
    XTC_HIP(hipMemcpyAsync(C.rhot, src->rhot, sizeof(double) * n_g, hipMemcpyDeviceToDevice, st));
  } else if (xi32) {
    hipLaunchKernelGGL(k_rhot_f32, dim3(cdiv(n_g, 256)), dim3(256), 0, st, (const double*)C.G,
                       xi32, n_mu, n_g, C.rhot);
    XTC_CHECK_LAUNCH();
  } else {
    GemmArgs g{};
    g.M = 1; g.N = n_g; g.K = n_mu;
    g.A = C.G; g.a_sm = 1; g.a_sk = 1;
    g.B = xi; g.b_sk = n_g; g.b_sn = 1;
    g.C = C.rhot; g.c_sm = n_g; g.c_sn = 1;
    XTC_TRY(gemm_f64(g, st));
  }
  if (fly)   // the orbitals and their gradients at the pivots, for xi~ per block
    XTC_TRY(gather_pivot_rows(src->phi4, n_g, 4 * src->n_orb, (const long*)C.piv, n_mu, C.phimu,
                              st));
  Stage1Args s1{grid->xyz, grid->w, xi, rho, C.rhot, n_g, n_mu, 0, 0, C.panel, C.rows_pad, C.bp,
                C.nch};
  s1.xi32 = xi32;
  if (bh) {
    s1.bh = C.bh;
    s1.bh_host = &bt;
    s1.pv64 = C.pv64;
  }
  if (precision == XTC_SPLIT_F16) {
    size_t tk = timing_begin(TM_SPLIT_PREP, st);
    XTC_TRY(split_prepare(s1, C.split, st));
    timing_end(tk, st);
  }
  const bool need_h = (channels & (XTC_D1 | XTC_D4)) != 0;
  if ((channels & XTC_FIELD) && (bra_begin > 0 || bra_end < n_g)) {
    // the field is written for the bra points of the range only
    hipLaunchKernelGGL(k_fill_zero, dim3(cdiv(3 * n_g, 256)), dim3(256), 0, st, field, 3 * n_g);
    XTC_CHECK_LAUNCH();
  }
  const int nsb = (int)cdiv(bra_end - bra_begin, C.bp);
  for (int sb = 0; sb < nsb; ++sb) {
    const long b0 = bra_begin + (long)sb * C.bp;
    const long bn = (bra_end - b0) < C.bp ? (bra_end - b0) : C.bp;
    s1.b0 = b0;
    s1.bn = bn;
    size_t tk = timing_begin(TM_STAGE1, st);
    if (precision == XTC_FP64) XTC_TRY(stage1_f64(s1, cf, st));
    else XTC_TRY(stage1_split_f16(s1, cf, C.split, C.split_bytes, st));
    timing_end(tk, st);
    size_t tk2 = timing_begin(TM_STAGE2, st);
    const double beta = sb == 0 ? 0.0 : 1.0;
    // split precision with the second operand scratch: the u1 and u3 products run on the
    // auxiliary stream beside the D4 and D1 products, so that each product's last partial
    // round of workgroups overlaps the next product instead of leaving the chip part idle
    const bool two = C.gsplit2 != nullptr;
    hipStream_t su = two ? st2 : st;
    if (two) {
      XTC_HIP(hipEventRecord(ev_fork, st));
      XTC_HIP(hipStreamWaitEvent(st2, ev_fork, 0));
    }
    auto nt = [&](const double* A, long a_sm, const double* s, const double* B, double* out,
                  double bet, hipStream_t ss, void* gs, const float* A32 = nullptr) {
      GemmArgs g{};
      g.M = n_mu; g.N = n_mu; g.K = bn;
      g.A = A; g.a_sm = a_sm; g.a_sk = 1;
      g.A32 = A32;
      g.s = s;
      g.B = B; g.b_sk = 1; g.b_sn = C.bp;
      g.C = out; g.c_sm = n_mu; g.c_sn = 1;
      g.beta = bet;
      return precision == XTC_SPLIT_F16 ? gemm_split_nt(g, gs, C.gsplit_bytes, ss)
                                        : gemm_f64(g, ss);
    };
    // (w xi) T^T for a panel channel, xi in FP64 or FP32
    auto nt_xi = [&](const double* B, double* out, double bet, hipStream_t ss, void* gs) {
      return xi32 ? nt(nullptr, n_g, grid->w + b0, B, out, bet, ss, gs, xi32 + b0)
                  : nt(xi + b0, n_g, grid->w + b0, B, out, bet, ss, gs);
    };
    void* gsu = two ? C.gsplit2 : C.gsplit;
    const double* wb = grid->w + b0;
    if (channels & XTC_U1)
      for (int c = 0; c < 3; ++c) {
        const double* xg = xigrad + (long)c * n_mu * n_g + b0;
        long ld = n_g;
        if (fly) {   // xi~^c of this block's columns from the kept factor of system 1 + c
          const size_t sysd = XTC_CHOL_SYSTEM_DOUBLES(n_mu);
          double* out = C.xigb + (long)c * n_mu * C.bp;
          XTC_TRY(fit_columns(src->phi4, n_g, src->n_orb, C.phimu, n_mu, 1 + c,
                              src->chol + (1 + c) * sysd, b0, bn, out, C.bp, C.fitP, C.fitR, C.bp,
                              su));
          xg = out;
          ld = C.bp;
        }
        XTC_TRY(nt(xg, ld, wb, C.panel + (long)c * C.rows_pad * C.bp, u1 + (long)c * n_mu * n_mu,
                   beta, su, gsu));
      }
    if (channels & XTC_U3) XTC_TRY(nt_xi(C.panel + 3L * C.rows_pad * C.bp, u3, beta, su, gsu));
    if (channels & XTC_ULAP) XTC_TRY(nt_xi(C.panel + 4L * C.rows_pad * C.bp, ulap, beta, su, gsu));
    hipLaunchKernelGGL(k_point_vectors, dim3(cdiv(bn, 256)), dim3(256), 0, st,
                       (const double*)C.rhot, grid->w, rho, n_g, n_mu, b0, bn,
                       (const double*)C.panel, C.rows_pad, C.bp, need_h ? 1 : 0, C.wt, C.H, C.e3x,
                       C.e4x, C.e3, C.e4, (channels & XTC_FIELD) ? field : nullptr);
    XTC_CHECK_LAUNCH();
    if (channels & XTC_D4)
      for (int c = 0; c < 3; ++c) {
        const double* Pc = C.panel + (long)c * C.rows_pad * C.bp;
        XTC_TRY(nt(Pc, C.bp, C.wt, Pc, D4, (sb == 0 && c == 0) ? 0.0 : 1.0, st, C.gsplit));
      }
    if (channels & XTC_D1) {
      hipLaunchKernelGGL(k_form_V, dim3(cdiv((long)n_mu * bn, 256)), dim3(256), 0, st,
                         (const double*)C.panel, C.rows_pad, C.bp, n_mu, bn, (const double*)C.H,
                         C.V);
      XTC_CHECK_LAUNCH();
      XTC_TRY(nt_xi(C.V, D1, beta, st, C.gsplit));
    }
    XTC_TRY(reduce_sum_f64(C.e3x, bn, C.sums + 4 * sb, C.red, st));
    XTC_TRY(reduce_sum_f64(C.e4x, bn, C.sums + 4 * sb + 1, C.red, st));
    XTC_TRY(reduce_sum_f64(C.e3, bn, C.sums + 4 * sb + 2, C.red, st));
    XTC_TRY(reduce_sum_f64(C.e4, bn, C.sums + 4 * sb + 3, C.red, st));
    if (two) {
      XTC_HIP(hipEventRecord(ev_join, st2));
      XTC_HIP(hipStreamWaitEvent(st, ev_join, 0));
    }
    timing_end(tk2, st);
    // xTC Terms 2 and 3 from the same calG panel
    if (ex)
      XTC_TRY(ex_block(C.ex, cf, C.panel, C.rows_pad, grid->xyz, xi, n_g, grid->w, b0, bn,
                       sb == 0, ex->X2 != nullptr, ex->X3 != nullptr, st));
  }
  if (ex) XTC_TRY(ex_finish(C.ex, ex->X2, ex->X3, false, st));
  if (channels & XTC_ESCALE) {
    std::vector<double> hs(4 * nsb);
    XTC_HIP(hipMemcpyAsync(hs.data(), C.sums, sizeof(double) * 4 * nsb, hipMemcpyDeviceToHost, st));
    XTC_HIP(hipStreamSynchronize(st));
    double e3x = 0.0, e4x = 0.0, e3 = 0.0, e4 = 0.0;
    for (int sb = 0; sb < nsb; ++sb) {
      e3x += hs[4 * sb];
      e4x += hs[4 * sb + 1];
      e3 += hs[4 * sb + 2];
      e4 += hs[4 * sb + 3];
    }
    escale[0] = e3;
    escale[1] = e4;
    escale[2] = 2.0 * e4;
    escale[3] = e3x;
    escale[4] = e4x;
    escale[5] = 2.0 * e4x;
  }
  return XTC_OK;
}




extern "C" xtc_status xtc_kernel_contract(const xtc_grid* grid, const xtc_correlator* corr,
                                          int32_t n_mu, const void* xi, const double* xigrad,
                                          const double* rho, const int64_t* pivots,
                                          uint32_t channels, int32_t precision, int64_t bra_begin,
                                          int64_t bra_end, double* u1,
                                          double* u3, double* ulap, double* D1, double* D4,
                                          double* field, double* escale, const xtc_exchange* ex,
                                          const xtc_xi_source* src, void* ws, size_t ws_bytes,
                                          void* stream) {
  XTC_REQUIRE(grid, "contract: null argument");
  return contract_impl(grid, corr, n_mu, xi, xigrad, rho, pivots, channels, precision, bra_begin,
                       bra_end, u1, u3, ulap, D1, D4, field, escale, ex, src, ws, ws_bytes,
                       default_bp(grid->n_g), true, stream);
}

// ---- the variant without a workspace: scratch in a file-scope device array ----------
//
// One array per device (the module's copy on that device), shared by every call of
// xtc_kernel_contract_noalloc on that device; its device address is looked up once per
// device with hipGetSymbolAddress and only that address is handed to the kernels.

static __device__ __align__(256) unsigned char scratch[XTC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

static xtc_status scratch_address(void** out) {
  int dev = -1;
  XTC_HIP(hipGetDevice(&dev));
  XTC_REQUIRE(dev >= 0 && dev < MAX_DEVICES, "contract_noalloc: device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    XTC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    XTC_REQUIRE(p != nullptr, "contract_noalloc: no device address for the static scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return XTC_OK;
}

extern "C" xtc_status xtc_kernel_contract_noalloc(
    const xtc_grid* grid, const xtc_correlator* corr, int32_t n_mu, const void* xi,
    const double* xigrad, const double* rho, const int64_t* pivots, uint32_t channels,
    int32_t precision, int64_t bra_begin, int64_t bra_end, double* u1, double* u3, double* ulap,
    double* D1, double* D4, double* field, double* escale, const xtc_exchange* ex,
    const xtc_xi_source* src, void* stream) {
  XTC_TRY(check_contract_args(grid, corr, n_mu, xi, xigrad, rho, pivots, channels, precision, ex,
                              src));
  if (ex) XTC_TRY(check_exchange_args(ex, n_mu));
  // the widest super-block (a multiple of 64, at most the regular call's) whose scratch fits
  const bool fly = xig_on_the_fly(channels, xigrad);
  const int n_orb = ex ? ex->n_orb : (fly ? src->n_orb : 0), n_q = ex ? ex->n_q : 0;
  auto need = [&](long bp) {
    Arena ar(nullptr, 0);
    layout_con(ar, grid->n_g, n_mu, channels, precision, n_orb, n_q, bp, fly, false,
               corr->form == XTC_U_BH);
    return ar.used;
  };
  long bp = default_bp(grid->n_g);
  while (bp > 64 && need(bp) > (size_t)XTC_NOALLOC_SCRATCH_BYTES) bp = ((bp / 2 + 63) / 64) * 64;
  if (need(bp) > (size_t)XTC_NOALLOC_SCRATCH_BYTES) {
    set_error("contract_noalloc: this problem needs " + std::to_string(need(bp)) +
              " bytes of scratch even with 64-point super-blocks; the static scratch holds " +
              std::to_string((size_t)XTC_NOALLOC_SCRATCH_BYTES) +
              " (use xtc_kernel_contract with a workspace)");
    return XTC_ERR_NO_WORKSPACE;
  }
  void* ptr = nullptr;
  XTC_TRY(scratch_address(&ptr));
  return contract_impl(grid, corr, n_mu, xi, xigrad, rho, pivots, channels, precision, bra_begin,
                       bra_end, u1, u3, ulap, D1, D4, field, escale, ex, src, ptr,
                       (size_t)XTC_NOALLOC_SCRATCH_BYTES, bp, false, stream);
}
