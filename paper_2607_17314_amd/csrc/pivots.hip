// Interpolation-point selection: weight-scaled fixed-rank pivoted Cholesky
// (ISDF section, Alg. 1; matrix-free pivot search) for the scalar and gradient
// channels, fused by the fill-to-target rule.
//
// The pivots are Alg. 1's greedy ones; what is reorganised is how the residual
// column of each pivot is formed. A plain step reads the orbital rows (N_orb, or
// 4 N_orb for the gradient channel) and every earlier factor row L[0..mu) at all
// grid points, so a channel of n steps streams ~n (4 N_orb + n / 2) rows of N_g
// doubles from HBM. Here the steps run in batches around a speculative candidate
// set: at a batch start with mu0 pivots, C = the 64 points of largest residual
// diagonal d (ties to the lowest index), and one set of FP64 matrix-core GEMMs
// forms their columns against every grid point,
//   R[c][g] = S(g, c) - sum_{l < mu0} L[l][g] L[l][c],
// from the orbitals at the candidates and the factor rows gathered there. Each
// step of the batch then takes the exact argmax of d over all points; while that
// pivot g* is a candidate, its factor row needs only R[g*] and the rows made in
// this batch,
//   L[mu][g] = (R[g*][g] - sum_{mu0 <= l < mu} L[l][g] L[l][g*]) / sqrt(d_g*),
// and the first pivot outside C ends the batch (the next batch's C holds it, as
// the largest d). The selected points, the stop rules and the fused order are
// those of the plain algorithm; the sums are grouped differently, so the factor
// agrees with a plain step's to rounding.
//
// One step = two launches:
//   k_pick   (one block)  reduces the per-block (max d, lowest index) partials,
//                         applies the rank-deficiency stop, ends the batch when the
//                         pivot is not a candidate, records g*, and gathers the
//                         batch's factor entries L[mu0..mu)[g*];
//   k_column (grid)       forms the new factor row from R, updates d and emits new
//                         partials.
// All state (d, L, partials, control word) lives in the workspace; the host
// synchronises once or twice per batch to see how far it went. Ties in the argmax
// go to the lowest grid index; the reduction order is fixed, so repeated runs
// select identical pivots.
#include <cstdio>
#include <cstdlib>
#include "common.hpp"
#include "plans.hpp"
#include "timing.hpp"

namespace xtc {

constexpr int PIV_BLOCK = 256;
constexpr double RANK_TOL = 1e-14;
constexpr int NCAND = 64;      // candidates per batch (one 64-row GEMM tile)
constexpr int TOP_SEG = 1024;  // entries sorted per block of the candidate search

struct PivCtl {
  long gstar;
  double dstar;
  double d0max;
  int step;     // pivots recorded so far in the current channel
  int stop;     // 0 running, 1 rank deficient, 2 fused target reached
  int union_n;  // |grad pivots U scalar pivots|
  int target;   // fused target (scalar channel) or 0
  int mu0;      // pivots recorded before the current batch
  int slot;     // candidate slot of the current pivot
  int bend;     // 1: the current batch has ended (a pivot outside its candidates)
  int stamp;    // current batch number (candidate stamps are stamp << 6 | slot)
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
                                                    unsigned char* __restrict__ mark,
                                                    const int* __restrict__ cslot, int mode,
                                                    int first) {
  // mode 0: gradient channel (marks its pivots); mode 1: scalar channel (fills the union)
  __shared__ int s_done;
  __shared__ long s_g;
  __shared__ int s_step, s_mu0;
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
    int bend = ctl->bend;   // the batch has ended
    const int step = ctl->step;
    if (!stop && !bend) {
      const int sl = cslot[c.g];
      if (!(c.d > RANK_TOL * ctl->d0max)) {
        stop = 1;
      } else if ((sl >> 6) != ctl->stamp) {
        bend = 1;            // not a candidate: the next batch starts from this point
      } else {
        piv[step] = c.g;
        ctl->gstar = c.g;
        ctl->dstar = c.d;
        ctl->slot = sl & (NCAND - 1);
        ctl->step = step + 1;
        if (mode == 0) {
          mark[c.g] = 1;
        } else if (!mark[c.g]) {
          ctl->union_n += 1;
          // the completing pivot is recorded; no further column is needed
          if (ctl->union_n >= ctl->target) stop = 2;
        }
      }
    }
    ctl->stop = stop;
    ctl->bend = bend;
    s_done = stop || bend;
    s_step = step;
    s_mu0 = ctl->mu0;
    s_g = c.g;
  }
  __syncthreads();
  if (s_done) return;
  const long gs = s_g;
  for (int l = threadIdx.x; l < s_step - s_mu0; l += PIV_BLOCK)
    lstar[l] = L[(long)(s_mu0 + l) * n_g + gs];
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

// The new factor row from the candidate's column R[slot] and the batch's earlier rows.
__global__ __launch_bounds__(PIV_BLOCK) void k_column(const double* __restrict__ R, long n_g,
                                                      double* __restrict__ L,
                                                      const double* __restrict__ lstar,
                                                      const PivCtl* __restrict__ ctl,
                                                      double* __restrict__ d,
                                                      double* __restrict__ pd,
                                                      long* __restrict__ pg) {
  __shared__ double sl[NCAND];
  if (ctl->stop || ctl->bend) return;
  const int mu = ctl->step - 1, mu0 = ctl->mu0, nb = mu - mu0;
  const long gs = ctl->gstar;
  const double inv = 1.0 / sqrt(ctl->dstar);
  const double* Rc = R + (long)ctl->slot * n_g;
  for (int i = threadIdx.x; i < nb; i += PIV_BLOCK) sl[i] = lstar[i];
  __syncthreads();
  const long g = (long)blockIdx.x * PIV_BLOCK + threadIdx.x;
  Cand c{-1.0, 0x7fffffffffffffffL};
  if (g < n_g) {
    const double acc = strided_dot(L + (long)mu0 * n_g + g, n_g, sl, nb);
    const double col = (Rc[g] - acc) * inv;
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

// --- the candidate search: the NCAND best (d, index) pairs -----------------------
// Each block sorts TOP_SEG entries (bitonic, best first: larger d, then lower index)
// and keeps its NCAND best; repeated over the outputs until one block remains.
// in_g == nullptr: the entries are d[0..n_in) with their own indices.
__global__ __launch_bounds__(256) void k_top_sort(const double* __restrict__ in_d,
                                                  const long* __restrict__ in_g, long n_in,
                                                  double* __restrict__ out_d,
                                                  long* __restrict__ out_g) {
  __shared__ double sd[TOP_SEG];
  __shared__ long sg[TOP_SEG];
  const long base = (long)blockIdx.x * TOP_SEG;
  for (int i = threadIdx.x; i < TOP_SEG; i += 256) {
    const long k = base + i;
    if (k < n_in) {
      sd[i] = in_d[k];
      sg[i] = in_g ? in_g[k] : k;
    } else {
      sd[i] = -1.0;   // below every residual diagonal (d >= 0)
      sg[i] = 0x7fffffffffffffffL;
    }
  }
  for (int k = 2; k <= TOP_SEG; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      __syncthreads();
      for (int i = threadIdx.x; i < TOP_SEG; i += 256) {
        const int p = i ^ j;
        if (p <= i) continue;
        const double di = sd[i], dp = sd[p];
        const long gi = sg[i], gp = sg[p];
        const bool p_better = dp > di || (dp == di && gp < gi);
        const bool best_first = (i & k) == 0;
        if (p_better == best_first) {
          sd[i] = dp; sg[i] = gp;
          sd[p] = di; sg[p] = gi;
        }
      }
    }
  __syncthreads();
  if (threadIdx.x < NCAND) {
    out_d[(long)blockIdx.x * NCAND + threadIdx.x] = sd[threadIdx.x];
    out_g[(long)blockIdx.x * NCAND + threadIdx.x] = sg[threadIdx.x];
  }
}

// Opens a batch: stamps the candidates, records mu0 and clears the end flag.
__global__ void k_batch_begin(const double* __restrict__ cd, const long* __restrict__ cg,
                              long n_g, int* __restrict__ cslot, int stamp,
                              long* __restrict__ cand, PivCtl* ctl) {
  const int m = threadIdx.x;
  const long g = cg[m];
  const bool ok = cd[m] >= 0.0 && g >= 0 && g < n_g;
  cand[m] = ok ? g : -1;
  if (ok) cslot[g] = (stamp << 6) | m;
  if (m == 0) {
    ctl->mu0 = ctl->step;
    ctl->bend = 0;
    ctl->stamp = stamp;
  }
}

// The orbital values and factor entries at the candidates, candidate-major:
// Ac[m][k] = phi4 row k at cand[m] (k < nrows), Lc[m][l] = L[l][cand[m]] (l < mu0),
// wc[m] = w[cand[m]]; rows of missing candidates are zero.
__global__ __launch_bounds__(256) void k_gather_cand(const double* __restrict__ phi4,
                                                     const double* __restrict__ w, long n_g,
                                                     int nrows, const double* __restrict__ L,
                                                     int mu0, int ldl,
                                                     const long* __restrict__ cand,
                                                     double* __restrict__ Ac,
                                                     double* __restrict__ Lc,
                                                     double* __restrict__ wc) {
  const long per = (long)nrows + mu0;
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= NCAND * per) return;
  const int m = (int)(i / per);
  const long k = i % per;
  const long g = cand[m];
  if (k < nrows) {
    Ac[(long)m * nrows + k] = g >= 0 ? phi4[k * n_g + g] : 0.0;
    if (k == 0) wc[m] = g >= 0 ? w[g] : 0.0;
  } else {
    const long l = k - nrows;
    Lc[(long)m * ldl + l] = g >= 0 ? L[l * n_g + g] : 0.0;
  }
}

// S(g, c) from the orbital dot products: scalar w_g w_c a^2, gradient w_g w_c a b,
// with a = R2 (gradient) or R (scalar) and b = R (gradient).
__global__ __launch_bounds__(256) void k_pair_values(double* __restrict__ R,
                                                     const double* __restrict__ R2,
                                                     const double* __restrict__ w,
                                                     const double* __restrict__ wc, long n_g,
                                                     int channel) {
  const long g = (long)blockIdx.x * 256 + threadIdx.x;
  const int m = blockIdx.y;
  if (g >= n_g) return;
  double* r = R + (long)m * n_g + g;
  if (channel == 0) {
    const double a = *r;
    *r = w[g] * wc[m] * a * a;
  } else {
    const double a = R2[(long)m * n_g + g];
    *r = w[g] * wc[m] * a * *r;
  }
}

struct SelLayout {
  double* d; double* L; double* pd; long* pg; double* lstar; PivCtl* ctl;
  long* piv_g; long* piv_s; unsigned char* mark;
  int* cslot; long* cand; double* R; double* R2; double* Ac; double* Lc; double* wc;
  double* td[2]; long* tg[2];
  int nparts, ldl;
};

static long top_entries(int64_t n_g) { return (long)cdiv(n_g, TOP_SEG) * NCAND; }

static SelLayout layout_sel(Arena& ar, int64_t n_g, int n_orb, int n_mu) {
  SelLayout S;
  S.nparts = (int)cdiv(n_g, PIV_BLOCK);
  S.ldl = n_mu > 0 ? n_mu : 1;
  S.d = ar.take<double>(n_g);
  S.L = ar.take<double>((size_t)n_mu * n_g);
  S.pd = ar.take<double>(S.nparts);
  S.pg = ar.take<long>(S.nparts);
  S.lstar = ar.take<double>(NCAND);
  S.ctl = ar.take<PivCtl>(1);
  S.piv_g = ar.take<long>(n_mu + 1);
  S.piv_s = ar.take<long>(n_mu + 1);
  S.mark = ar.take<unsigned char>(n_g);
  S.cslot = ar.take<int>(n_g);
  S.cand = ar.take<long>(NCAND);
  S.R = ar.take<double>((size_t)NCAND * n_g);
  S.R2 = ar.take<double>((size_t)NCAND * n_g);
  S.Ac = ar.take<double>((size_t)NCAND * 4 * n_orb);
  S.Lc = ar.take<double>((size_t)NCAND * S.ldl);
  S.wc = ar.take<double>(NCAND);
  for (int b = 0; b < 2; ++b) {
    S.td[b] = ar.take<double>(top_entries(n_g));
    S.tg[b] = ar.take<long>(top_entries(n_g));
  }
  return S;
}

size_t ws_select(int64_t n_g, int n_orb, int n_mu, int mode) {
  (void)mode;
  Arena ar(nullptr, 0);
  layout_sel(ar, n_g, n_orb, n_mu);
  return ar.used;
}

// XTC_PROGRESS set in the environment: long host loops report their progress on stderr
// at the points where they synchronise anyway.
static bool progress_enabled() {
  static const bool on = getenv("XTC_PROGRESS") != nullptr;
  return on;
}

// Opens a batch at the current d: candidate search, stamps, and the candidates'
// columns R against every point (GEMMs on the orbitals and the mu0 factor rows).
static xtc_status open_batch(const double* phi4, const double* w, long n_g, int n_orb,
                             int channel, int mu0, int stamp, SelLayout& S, hipStream_t st) {
  // candidate search
  long n_in = n_g;
  const double* id = S.d;
  const long* ig = nullptr;
  int b = 0;
  for (;;) {
    const unsigned nb = cdiv(n_in, TOP_SEG);
    hipLaunchKernelGGL(k_top_sort, dim3(nb), dim3(256), 0, st, id, ig, n_in, S.td[b], S.tg[b]);
    XTC_CHECK_LAUNCH();
    id = S.td[b];
    ig = S.tg[b];
    n_in = (long)nb * NCAND;
    b ^= 1;
    if (nb == 1) break;
  }
  hipLaunchKernelGGL(k_batch_begin, dim3(1), dim3(NCAND), 0, st, id, ig, n_g, S.cslot, stamp,
                     S.cand, S.ctl);
  XTC_CHECK_LAUNCH();
  const int nrows = channel == 0 ? n_orb : 4 * n_orb;
  hipLaunchKernelGGL(k_gather_cand, dim3(cdiv((long)NCAND * (nrows + mu0), 256)), dim3(256), 0, st,
                     phi4, w, n_g, nrows, S.L, mu0, S.ldl, S.cand, S.Ac, S.Lc, S.wc);
  XTC_CHECK_LAUNCH();
  // a[c][g] = sum_p phi_p(c) phi_p(g) (into R2 for the gradient channel)
  GemmArgs g{};
  g.M = NCAND; g.N = n_g; g.K = n_orb;
  g.A = S.Ac; g.a_sm = nrows; g.a_sk = 1;
  g.B = phi4; g.b_sk = n_g; g.b_sn = 1;
  g.C = channel == 0 ? S.R : S.R2; g.c_sm = n_g; g.c_sn = 1;
  XTC_TRY(gemm_f64(g, st));
  if (channel != 0) {
    // b[c][g] = sum_{x, p} d_x phi_p(c) d_x phi_p(g)
    GemmArgs h{};
    h.M = NCAND; h.N = n_g; h.K = 3L * n_orb;
    h.A = S.Ac + n_orb; h.a_sm = nrows; h.a_sk = 1;
    h.B = phi4 + (long)n_orb * n_g; h.b_sk = n_g; h.b_sn = 1;
    h.C = S.R; h.c_sm = n_g; h.c_sn = 1;
    XTC_TRY(gemm_f64(h, st));
  }
  hipLaunchKernelGGL(k_pair_values, dim3(cdiv(n_g, 256), NCAND), dim3(256), 0, st, S.R, S.R2, w,
                     S.wc, n_g, channel);
  XTC_CHECK_LAUNCH();
  if (mu0 > 0) {
    // R -= Lc L: what the mu0 earlier pivots already explain
    GemmArgs l{};
    l.M = NCAND; l.N = n_g; l.K = mu0;
    l.A = S.Lc; l.a_sm = S.ldl; l.a_sk = 1;
    l.B = S.L; l.b_sk = n_g; l.b_sn = 1;
    l.C = S.R; l.c_sm = n_g; l.c_sn = 1;
    l.alpha = -1.0; l.beta = 1.0;
    XTC_TRY(gemm_f64(l, st));
  }
  return XTC_OK;
}

// Runs one channel; returns the number of pivots recorded.
static xtc_status run_channel(const double* phi4, const double* w, long n_g, int n_orb, int channel,
                              int max_steps, SelLayout& S, long* piv_out, hipStream_t st,
                              int* n_out, int* deficient) {
  const unsigned nb = (unsigned)S.nparts;
  hipLaunchKernelGGL(k_diag, dim3(nb), dim3(PIV_BLOCK), 0, st, phi4, w, n_g, n_orb, channel, S.d,
                     S.pd, S.pg);
  XTC_CHECK_LAUNCH();
  XTC_HIP(hipMemsetAsync(S.cslot, 0, sizeof(int) * (size_t)n_g, st));
  const int mode = channel == 0 ? 1 : 0;
  PivCtl h{};
  int done = 0, stamp = 0, guess = 16;
  while (done < max_steps) {
    ++stamp;
    XTC_TRY(open_batch(phi4, w, n_g, n_orb, channel, done, stamp, S, st));
    // steps are issued in groups, with a look at the control word after each: the
    // first group is sized from the previous batch's length
    const int lim = max_steps - done < NCAND ? max_steps - done : NCAND;
    int issued = 0;
    for (;;) {
      int n = issued == 0 ? guess : 8;
      if (n > lim - issued) n = lim - issued;
      for (int i = 0; i < n; ++i) {
        const int first = done == 0 && issued == 0 && i == 0;
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(PIV_BLOCK), 0, st, S.pd, S.pg, S.nparts, S.ctl,
                           piv_out, S.L, n_g, S.lstar, S.mark, S.cslot, mode, first);
        hipLaunchKernelGGL(k_column, dim3(nb), dim3(PIV_BLOCK), 0, st, S.R, n_g, S.L, S.lstar,
                           S.ctl, S.d, S.pd, S.pg);
      }
      XTC_CHECK_LAUNCH();
      issued += n;
      XTC_HIP(hipMemcpyAsync(&h, S.ctl, sizeof(PivCtl), hipMemcpyDeviceToHost, st));
      XTC_HIP(hipStreamSynchronize(st));
      if (h.stop || h.bend || issued >= lim) break;
    }
    const int accepted = h.step - done;
    // the batch's first pick is the largest d, its first candidate: no progress and no
    // stop means the search and the argmax disagree, which only non-finite values cause
    if (accepted == 0 && h.stop == 0) {
      set_error("isdf_select_points: the pivot search made no progress (non-finite orbital "
                "values or weights?)");
      return XTC_ERR_INVALID_ARG;
    }
    guess = accepted + 4 < NCAND ? accepted + 4 : NCAND;
    if (progress_enabled() && h.step / 1024 != done / 1024)
      fprintf(stderr, "isdf_select_points: %s channel, %d steps done (%d batches)\n",
              channel == 0 ? "scalar" : "gradient", h.step, stamp);
    done = h.step;
    if (h.stop != 0) break;
  }
  *n_out = done;
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
  SelLayout S = layout_sel(ar, n_g, n_orb, n_mu);
  XTC_TRY(need_ws(ar));
  XTC_HIP(hipMemsetAsync(S.mark, 0, n_g, st));
  // gradient channel to ceil(n_mu / 2) pivots
  const int n_grad = (n_mu + 1) / 2;
  PivCtl init{};
  init.target = 0;
  XTC_HIP(hipMemcpyAsync(S.ctl, &init, sizeof(PivCtl), hipMemcpyHostToDevice, st));
  int ng = 0, defg = 0;
  XTC_TRY(run_channel(phi4, grid->w, n_g, n_orb, 1, n_grad, S, S.piv_g, st, &ng, &defg));
  // scalar channel until the union reaches n_mu
  init.union_n = ng;
  init.target = n_mu;
  XTC_HIP(hipMemcpyAsync(S.ctl, &init, sizeof(PivCtl), hipMemcpyHostToDevice, st));
  int ns = 0, defs = 0;
  if (ng < n_mu) {
    XTC_TRY(run_channel(phi4, grid->w, n_g, n_orb, 0, n_mu, S, S.piv_s, st, &ns, &defs));
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
