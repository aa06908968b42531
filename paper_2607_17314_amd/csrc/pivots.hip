// Interpolation-point selection: weight-scaled fixed-rank pivoted Cholesky
// (ISDF section, Alg. 1; matrix-free pivot search) for the scalar and gradient
// channels, fused by the fill-to-target rule.
//
// One pivot step = two launches:
//   k_pick   (one block)  reduces the per-block (max d, lowest index) partials,
//                         applies the rank-deficiency stop, records g*, and
//                         gathers the pivot's Cholesky row L[lambda][g*];
//   k_column (grid)       forms the new column s_g from the orbitals at g and g*
//                         (staged in LDS), subtracts sum_lambda L[lambda][g] L[lambda][g*],
//                         scales by 1/sqrt(d_g*), updates d and emits new partials.
// All state (d, L, partials, control word) lives in the workspace; the host
// only synchronises once per batch of steps to see whether the fused set is
// complete. Ties in the argmax go to the lowest grid index; the reduction
// order is fixed, so repeated runs select identical pivots.
#include <cstdio>
#include <cstdlib>
#include "common.hpp"
#include "plans.hpp"
#include "timing.hpp"

namespace xtc {

constexpr int PIV_BLOCK = 256;
constexpr double RANK_TOL = 1e-14;

struct PivCtl {
  long gstar;
  double dstar;
  double d0max;
  int step;     // pivots recorded so far in the current channel
  int stop;     // 0 running, 1 rank deficient, 2 fused target reached
  int union_n;  // |grad pivots U scalar pivots|
  int target;   // fused target (scalar channel) or 0
};

struct Cand {
  double d;
  long g;
};

__device__ __forceinline__ Cand better(Cand a, Cand b) {
  if (a.d > b.d) return a;
  if (b.d > a.d) return b;
  return a.g <= b.g ? a : b;
}

__device__ Cand block_argmax(Cand c) {
  __shared__ double sd[PIV_BLOCK / 64];
  __shared__ long sg[PIV_BLOCK / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    Cand o;
    o.d = __shfl_down(c.d, off, 64);
    o.g = __shfl_down(c.g, off, 64);
    c = better(c, o);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    sd[wave] = c.d;
    sg[wave] = c.g;
  }
  __syncthreads();
  Cand r{sd[0], sg[0]};
  for (int w = 1; w < PIV_BLOCK / 64; ++w) r = better(r, Cand{sd[w], sg[w]});
  return r;
}

// channel: 0 scalar, 1 gradient
__global__ __launch_bounds__(PIV_BLOCK) void k_diag(const double* __restrict__ phi4,
                                                    const double* __restrict__ w, long n_g,
                                                    int n_orb, int channel, double* __restrict__ d,
                                                    double* __restrict__ pd, long* __restrict__ pg) {
  long g = (long)blockIdx.x * PIV_BLOCK + threadIdx.x;
  Cand c{-1.0, 0x7fffffffffffffffL};
  if (g < n_g) {
    double n2 = 0.0, g2 = 0.0;
    for (int p = 0; p < n_orb; ++p) {
      double v = phi4[(long)p * n_g + g];
      n2 += v * v;
    }
    double dd;
    if (channel == 0) {
      dd = w[g] * w[g] * n2 * n2;
    } else {
      for (int q = 0; q < 3 * n_orb; ++q) {
        double v = phi4[(long)(n_orb + q) * n_g + g];
        g2 += v * v;
      }
      dd = w[g] * w[g] * n2 * g2;
    }
    d[g] = dd;
    c = Cand{dd, g};
  }
  c = block_argmax(c);
  if (threadIdx.x == 0) {
    pd[blockIdx.x] = c.d;
    pg[blockIdx.x] = c.g;
  }
}

__global__ __launch_bounds__(PIV_BLOCK) void k_pick(const double* __restrict__ pd,
                                                    const long* __restrict__ pg, int nparts,
                                                    PivCtl* ctl, long* __restrict__ piv,
                                                    const double* __restrict__ L, long n_g,
                                                    double* __restrict__ lstar,
                                                    unsigned char* __restrict__ mark, int mode,
                                                    int first) {
  // mode 0: gradient channel (marks its pivots); mode 1: scalar channel (fills the union)
  __shared__ int s_stop;
  __shared__ long s_g;
  __shared__ int s_step;
  Cand c{-1.0, 0x7fffffffffffffffL};
  for (int i = threadIdx.x; i < nparts; i += PIV_BLOCK) c = better(c, Cand{pd[i], pg[i]});
  c = block_argmax(c);
  if (threadIdx.x == 0) {
    if (first) {
      ctl->d0max = c.d;
      ctl->stop = 0;
      ctl->step = 0;
    }
    int stop = ctl->stop;   // 1: rank deficient, 2: fused target complete
    if (!stop && !(c.d > RANK_TOL * ctl->d0max)) stop = 1;
    int step = ctl->step;
    if (!stop) {
      piv[step] = c.g;
      ctl->gstar = c.g;
      ctl->dstar = c.d;
      ctl->step = step + 1;
      if (mode == 0) {
        mark[c.g] = 1;
      } else if (!mark[c.g]) {
        ctl->union_n += 1;
        // the completing pivot is recorded; no further column is needed
        if (ctl->union_n >= ctl->target) stop = 2;
      }
    }
    ctl->stop = stop;
    s_stop = stop;
    s_step = step;
    s_g = c.g;
  }
  __syncthreads();
  if (s_stop) return;
  const long gs = s_g;
  for (int l = threadIdx.x; l < s_step; l += PIV_BLOCK) lstar[l] = L[(long)l * n_g + gs];
}

// dot(x[i * stride], y[i]) over i < n with sixteen loads in flight and four
// accumulators combined in a fixed order (the column is memory-bound; a single
// dependent chain would leave one load outstanding per wave)
__device__ __forceinline__ double strided_dot(const double* __restrict__ x, long stride,
                                              const double* __restrict__ y, int n) {
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  int i = 0;
  for (; i + 16 <= n; i += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = x[(long)(i + u) * stride];
#pragma unroll
    for (int u = 0; u < 16; ++u) a[u & 3] += v[u] * y[i + u];
  }
  for (; i < n; ++i) a[0] += x[(long)i * stride] * y[i];
  return (a[0] + a[1]) + (a[2] + a[3]);
}

__global__ __launch_bounds__(PIV_BLOCK) void k_column(const double* __restrict__ phi4,
                                                      const double* __restrict__ w, long n_g,
                                                      int n_orb, int channel, double* __restrict__ L,
                                                      const double* __restrict__ lstar,
                                                      PivCtl* ctl, double* __restrict__ d,
                                                      double* __restrict__ pd,
                                                      long* __restrict__ pg, int lrow_in_lds) {
  // orbitals at the pivot ([4][n_orb] for channel 1, [n_orb] else), then L[.][g*]
  extern __shared__ double sphi[];
  if (ctl->stop) return;
  const int mu = ctl->step - 1;
  const long gs = ctl->gstar;
  const double inv = 1.0 / sqrt(ctl->dstar);
  const int nrows = channel == 0 ? n_orb : 4 * n_orb;
  double* sl = sphi + nrows;
  for (int i = threadIdx.x; i < nrows; i += PIV_BLOCK) sphi[i] = phi4[(long)i * n_g + gs];
  if (lrow_in_lds)
    for (int i = threadIdx.x; i < mu; i += PIV_BLOCK) sl[i] = lstar[i];
  __syncthreads();
  long g = (long)blockIdx.x * PIV_BLOCK + threadIdx.x;
  Cand c{-1.0, 0x7fffffffffffffffL};
  if (g < n_g) {
    const double a = strided_dot(phi4 + g, n_g, sphi, n_orb);
    double s;
    if (channel == 0) {
      s = w[g] * w[gs] * a * a;
    } else {
      const double bb = strided_dot(phi4 + (long)n_orb * n_g + g, n_g, sphi + n_orb, 3 * n_orb);
      s = w[g] * w[gs] * a * bb;
    }
    const double acc = lrow_in_lds ? strided_dot(L + g, n_g, sl, mu) : strided_dot(L + g, n_g, lstar, mu);
    double col = (s - acc) * inv;
    L[(long)mu * n_g + g] = col;
    double dn = d[g] - col * col;
    dn = dn > 0.0 ? dn : 0.0;
    if (g == gs) dn = 0.0;
    d[g] = dn;
    c = Cand{dn, g};
  }
  c = block_argmax(c);
  if (threadIdx.x == 0) {
    pd[blockIdx.x] = c.d;
    pg[blockIdx.x] = c.g;
  }
}

struct SelLayout {
  double* d; double* L; double* pd; long* pg; double* lstar; PivCtl* ctl;
  long* piv_g; long* piv_s; unsigned char* mark;
  int nparts;
};

static SelLayout layout_sel(Arena& ar, int64_t n_g, int n_mu) {
  SelLayout S;
  S.nparts = (int)cdiv(n_g, PIV_BLOCK);
  S.d = ar.take<double>(n_g);
  S.L = ar.take<double>((size_t)n_mu * n_g);
  S.pd = ar.take<double>(S.nparts);
  S.pg = ar.take<long>(S.nparts);
  S.lstar = ar.take<double>(n_mu + 1);
  S.ctl = ar.take<PivCtl>(1);
  S.piv_g = ar.take<long>(n_mu + 1);
  S.piv_s = ar.take<long>(n_mu + 1);
  S.mark = ar.take<unsigned char>(n_g);
  return S;
}

size_t ws_select(int64_t n_g, int n_orb, int n_mu, int mode) {
  (void)n_orb;
  (void)mode;
  Arena ar(nullptr, 0);
  layout_sel(ar, n_g, n_mu);
  return ar.used;
}

// Runs one channel; returns the number of pivots recorded.
// XTC_PROGRESS set in the environment: long host loops report their progress on stderr
// at the points where they synchronise anyway.
static bool progress_enabled() {
  static const bool on = getenv("XTC_PROGRESS") != nullptr;
  return on;
}

static xtc_status run_channel(const double* phi4, const double* w, long n_g, int n_orb, int channel,
                              int max_steps, int fill_target, SelLayout& S, long* piv_out,
                              hipStream_t st, int* n_out, int* deficient) {
  const unsigned nb = (unsigned)S.nparts;
  hipLaunchKernelGGL(k_diag, dim3(nb), dim3(PIV_BLOCK), 0, st, phi4, w, n_g, n_orb, channel, S.d,
                     S.pd, S.pg);
  XTC_CHECK_LAUNCH();
  (void)fill_target;
  PivCtl h{};
  // pivot orbitals and, up to 8192 steps, the pivot's Cholesky row in LDS
  const int lrow_in_lds = max_steps <= 8192;
  const size_t smem =
      sizeof(double) * ((channel == 0 ? n_orb : 4 * n_orb) + (lrow_in_lds ? max_steps : 0));
  const int mode = channel == 0 ? 1 : 0;
  const int batch = 64;
  int done_steps = 0;
  for (int s0 = 0; s0 < max_steps; s0 += batch) {
    int s1 = s0 + batch < max_steps ? s0 + batch : max_steps;
    for (int s = s0; s < s1; ++s) {
      hipLaunchKernelGGL(k_pick, dim3(1), dim3(PIV_BLOCK), 0, st, S.pd, S.pg, S.nparts, S.ctl,
                         piv_out, S.L, n_g, S.lstar, S.mark, mode, s == 0 ? 1 : 0);
      hipLaunchKernelGGL(k_column, dim3(nb), dim3(PIV_BLOCK), smem, st, phi4, w, n_g, n_orb,
                         channel, S.L, S.lstar, S.ctl, S.d, S.pd, S.pg, lrow_in_lds);
    }
    XTC_CHECK_LAUNCH();
    XTC_HIP(hipMemcpyAsync(&h, S.ctl, sizeof(PivCtl), hipMemcpyDeviceToHost, st));
    XTC_HIP(hipStreamSynchronize(st));
    if (progress_enabled() && h.step / 1024 != done_steps / 1024)
      fprintf(stderr, "isdf_select_points: %s channel, %d steps done\n",
              channel == 0 ? "scalar" : "gradient", h.step);
    done_steps = h.step;
    if (h.stop != 0) break;
  }
  *n_out = done_steps;
  *deficient = (h.stop == 1);
  return XTC_OK;
}

}  // namespace xtc

using namespace xtc;

xtc_status xtc_select_qr(const double* phi4, const xtc_grid* grid, int n_orb, int n_mu,
                         int64_t* pivots, int32_t* n_mu_out, double* info, Arena& ar,
                         hipStream_t st);
xtc_status xtc_select_learned(const double* phi4, const xtc_grid* grid, int n_orb, int n_occ,
                              int n_mu, int mode, const xtc_mlp* mlp, double fallback_factor,
                              int64_t* pivots, int32_t* n_mu_out, double* info, Arena& ar,
                              hipStream_t st);

xtc_status xtc_select_qr(const double* phi4, const xtc_grid* grid, int n_orb, int n_mu,
                         int64_t* pivots, int32_t* n_mu_out, double* info, Arena& ar,
                         hipStream_t st) {
  const long n_g = grid->n_g;
  const size_t mark = ar.used;
  SelLayout S = layout_sel(ar, n_g, n_mu);
  XTC_TRY(need_ws(ar));
  XTC_HIP(hipMemsetAsync(S.mark, 0, n_g, st));
  // gradient channel to ceil(n_mu / 2) pivots
  const int n_grad = (n_mu + 1) / 2;
  PivCtl init{};
  init.target = 0;
  XTC_HIP(hipMemcpyAsync(S.ctl, &init, sizeof(PivCtl), hipMemcpyHostToDevice, st));
  int ng = 0, defg = 0;
  XTC_TRY(run_channel(phi4, grid->w, n_g, n_orb, 1, n_grad, 0, S, S.piv_g, st, &ng, &defg));
  // scalar channel until the union reaches n_mu
  init.union_n = ng;
  init.target = n_mu;
  XTC_HIP(hipMemcpyAsync(S.ctl, &init, sizeof(PivCtl), hipMemcpyHostToDevice, st));
  int ns = 0, defs = 0;
  if (ng < n_mu) {
    XTC_TRY(run_channel(phi4, grid->w, n_g, n_orb, 0, n_mu, n_mu, S, S.piv_s, st, &ns, &defs));
  }
  std::vector<long> hg(ng > 0 ? ng : 1), hs(ns > 0 ? ns : 1);
  if (ng) XTC_HIP(hipMemcpyAsync(hg.data(), S.piv_g, sizeof(long) * ng, hipMemcpyDeviceToHost, st));
  if (ns) XTC_HIP(hipMemcpyAsync(hs.data(), S.piv_s, sizeof(long) * ns, hipMemcpyDeviceToHost, st));
  XTC_HIP(hipStreamSynchronize(st));
  // fused order: scalar pivots in selection order, then gradient-only pivots
  std::vector<char> in_s(n_g, 0);
  int n = 0;
  for (int i = 0; i < ns; ++i) {
    pivots[n++] = hs[i];
    in_s[hs[i]] = 1;
  }
  for (int i = 0; i < ng && n < n_mu; ++i)
    if (!in_s[hg[i]]) pivots[n++] = hg[i];
  *n_mu_out = n;
  if (info) {
    info[0] = ns;
    info[1] = ng;
  }
  ar.used = mark;
  return n < n_mu ? XTC_WARN_RANK_DEFICIENT : XTC_OK;
}

extern "C" xtc_status isdf_select_points(const double* phi4, const xtc_grid* grid, int32_t n_orb,
                                         int32_t n_occ, int32_t n_mu_target, int32_t mode,
                                         const xtc_mlp* mlp, double fallback_factor,
                                         int64_t* pivots, int32_t* n_mu_out, double* info,
                                         void* ws, size_t ws_bytes, void* stream);

extern "C" xtc_status isdf_select_points(const double* phi4, const xtc_grid* grid, int32_t n_orb,
                                         int32_t n_occ, int32_t n_mu_target, int32_t mode,
                                         const xtc_mlp* mlp, double fallback_factor,
                                         int64_t* pivots, int32_t* n_mu_out, double* info,
                                         void* ws, size_t ws_bytes, void* stream) {
  XTC_REQUIRE(phi4 && grid && pivots && n_mu_out, "isdf_select_points: null argument");
  XTC_REQUIRE(grid->n_g > 0 && grid->w, "isdf_select_points: empty grid");
  XTC_REQUIRE(n_orb > 0 && n_mu_target > 0 && n_mu_target <= grid->n_g,
              "isdf_select_points: bad sizes");
  XTC_REQUIRE(mode == XTC_SELECT_QR || mode == XTC_SELECT_LEARNED ||
                  mode == XTC_SELECT_LEARNED_JUDGED,
              "isdf_select_points: unknown mode");
  XTC_REQUIRE(mode == XTC_SELECT_QR || mlp, "isdf_select_points: learned modes need an mlp");
  if (info)
    for (int i = 0; i < 8; ++i) info[i] = 0.0;
  XTC_TRY(check_weights(grid, ws, ws_bytes, as_stream(stream), "isdf_select_points"));
  Arena ar(ws, ws_bytes);
  size_t tk = timing_begin(TM_SELECT, as_stream(stream));
  xtc_status s = mode == XTC_SELECT_QR
                     ? xtc_select_qr(phi4, grid, n_orb, n_mu_target, pivots, n_mu_out, info, ar,
                                     as_stream(stream))
                     : xtc_select_learned(phi4, grid, n_orb, n_occ, n_mu_target, mode, mlp,
                                          fallback_factor, pivots, n_mu_out, info, ar,
                                          as_stream(stream));
  timing_end(tk, as_stream(stream));
  return s;
}
