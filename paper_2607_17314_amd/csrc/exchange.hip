// xTC Terms 2 and 3: the exchange intermediates X2 and X3 through the low-rank
// projector (xTC section, paragraphs "Terms 2 and 3 (non-factorizable)" and
// "Low-rank projector for Terms 2 and 3"):
//   P[s a][nu]   = phi_s(r_nu) sum_t phi_t(r_nu) LQ[t][a],          gamma = LQ LQ^T,
//   R^c[s a](g)  = sum_nu P[s a][nu] calG^c_{nu,g},   Q[s a](g) = sum_nu P[s a][nu] xi_nu(g),
//   T2_{qs}(g)   = sum_{a,c} R^c[s a](g) R^c[q a](g),
//   T3^c_{qs}(g) = sum_a (Q[s a](g) R^c[q a](g) + R^c[s a](g) Q[q a](g)),
//   X2[q][s][mu] = sum_g w_g xi_mu(g) T2_{qs}(g),   X3[q][s][mu] = sum_{g,c} w_g calG^c_{mu,g} T3^c_{qs}(g).
// Both are symmetric in (q, s), so only the packed upper triangle q <= s is formed
// (pipeline section, symmetry paragraph) and mirrored at the end.
//
// Per bra super-block: stage 1 builds the calG panel (it lives only for the block);
// R and Q are FP64 MFMA GEMMs written point-major, RQ[g][R^x, R^y, R^z, Q][s a];
// per chunk of XCH points k_x_pairs stages one point's rows of two 64-orbital
// blocks in LDS and forms the pair products T[part][g][pair] (pair fastest, so the
// stores are whole lines); the chunk's contribution to X is then one GEMM for X2
// and one three-segment GEMM for X3 (the three gradient channels concatenated
// along k), in split FP16 on MFMA on the mixed path or FP64 MFMA otherwise, with
// the quadrature weight as the per-k scale and FP64 accumulation across chunks.
#include <climits>
#include "bh.hpp"
#include "contract.hpp"
#include "exchange.hpp"
#include "gemm_split.hpp"
#include "plans.hpp"
#include "timing.hpp"

namespace xtc {

constexpr long XSUPER = 16384;   // bra super-block of the standalone call
constexpr long XCH = 2048;       // bra chunk of the pair products and X GEMMs
constexpr int XOB = 64;          // orbital block of the pair kernel
constexpr int XGB = 16;          // bra points per workgroup of the pair kernel

static inline long round_to(long x, long m) { return ((x + m - 1) / m) * m; }

void ex_layout(Arena& ar, long n_g, long bp, int n_mu, int n_orb, int n_q, int precision,
               ExWork* W) {
  W->n_orb = n_orb;
  W->n_q = n_q;
  W->n_mu = n_mu;
  W->bp = bp;
  W->precision = precision;
  W->npair = (long)n_orb * (n_orb + 1) / 2;
  W->npl = round_to(W->npair, 32);
  const int nb = (int)cdiv(n_orb, XOB);
  W->ntile = nb * (nb + 1) / 2;
  const long nr = (long)n_orb * n_q;
  W->nr = nr;
  const long xch = bp < XCH ? bp : XCH;
  W->tpart = xch * W->npl;
  W->phia = ar.take<double>((size_t)n_q * n_mu);
  W->P = ar.take<double>((size_t)nr * n_mu);
  W->RQ = ar.take<double>((size_t)4 * nr * bp);
  W->T = ar.take<double>((size_t)4 * W->tpart);
  W->Xp = ar.take<double>((size_t)2 * W->npair * n_mu);
  W->tiles = ar.take<int2>(W->ntile);
  const bool split = precision == XTC_SPLIT_F16;
  W->gsplit_bytes = split ? gemm_split_seg_scratch_bytes(W->npair, n_mu, xch, 3) : 0;
  W->gsplit = W->gsplit_bytes ? (void*)ar.take<char>(W->gsplit_bytes) : nullptr;
  W->rows_padR = round_to(nr + 2, 256);
  W->Qf = split ? ar.take<double>((size_t)nr * n_g) : nullptr;
  W->splitQ_bytes = split ? split_scratch_bytes(n_g, (int)nr) + rho_row_scratch_bytes(bp) : 0;
  W->splitQ = W->splitQ_bytes ? (void*)ar.take<char>(W->splitQ_bytes) : nullptr;
  W->panelR = split ? ar.take<double>((size_t)4 * W->rows_padR * bp) : nullptr;
  // per-run exponent maxima of the pair products and the X products' A row scales
  const long nrun = cdiv(xch, XGB);
  W->pex_stride = nrun * W->npl;
  W->pex = split ? ar.take<int>((size_t)2 * W->pex_stride) : nullptr;
  W->ex2 = split ? ar.take<int>(round_to(W->npair, 128)) : nullptr;
  W->ex3 = split ? ar.take<int>(round_to(W->npair, 128)) : nullptr;
}

struct ExLayout {
  double* panel; void* split; size_t split_bytes; BHTable* bh; long bp; long rows_pad;
  ExWork W;
};

static ExLayout layout_ex(Arena& ar, int64_t n_g, int n_mu, int n_orb, int n_q, int precision) {
  ExLayout L;
  L.bp = n_g < XSUPER ? round_to(n_g, 64) : XSUPER;
  L.rows_pad = round_to(n_mu + 2, 256);
  L.panel = ar.take<double>((size_t)4 * L.rows_pad * L.bp);
  L.split_bytes = precision == XTC_SPLIT_F16
                      ? split_scratch_bytes(n_g, n_mu) + rho_row_scratch_bytes(L.bp) : 0;
  L.split = L.split_bytes ? (void*)ar.take<char>(L.split_bytes) : nullptr;
  L.bh = ar.take<BHTable>(1);
  ex_layout(ar, n_g, L.bp, n_mu, n_orb, n_q, precision, &L.W);
  return L;
}

size_t ws_exchange(int64_t n_g, int n_orb, int n_mu, int n_q, int precision) {
  Arena ar(nullptr, 0);
  layout_ex(ar, n_g, n_mu, n_orb, n_q, precision);
  return ar.used;
}

// upper-triangular tile table of the 64-orbital blocks: tile t -> (q block, s block)
__global__ void k_fill_tiles(int nb, int ntile, int2* __restrict__ tiles) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= ntile) return;
  int r = t, qb = 0;
  while (r >= nb - qb) {
    r -= nb - qb;
    ++qb;
  }
  tiles[t] = make_int2(qb, qb + r);
}

// P[(s, a)][nu] = phi_s(nu) phia[a][nu]
__global__ void k_proj_rows(const double* __restrict__ phi_piv, const double* __restrict__ phia,
                            int n_orb, int n_q, int n_mu, double* __restrict__ P) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long)n_orb * n_q * n_mu) return;
  const long nu = t % n_mu;
  const long sa = t / n_mu;
  const int s = (int)(sa / n_q), a = (int)(sa % n_q);
  P[t] = phi_piv[(long)s * n_mu + nu] * phia[(long)a * n_mu + nu];
}

__host__ __device__ inline long pair_index(int q, int s, int n_orb) {
  return (long)q * n_orb - (long)q * (q - 1) / 2 + (s - q);
}

// Pair products for a run of XGB bra points and one (q block, s block) tile of 64 x 64
// orbitals (q block <= s block). Per point, LDS holds both blocks' rows [ch][a][orbital]
// (ch = R^x, R^y, R^z, Q); thread (tq, ts) owns q = q0 + 4 tq + i and s = s0 + ts + 16 j
// (i, j < 4), so a row of 16 threads stores 16 consecutive pairs.
// RQ: [bp][4][n_orb n_q] (point-major); T: [4][xch][npl], part stride tpart.
// With pex != nullptr the kernel also records, per pair and per run of points, the
// largest binary exponent of |T2 w| (pex[0]) and of |T3^c w| over c (pex[1]); zeros
// count as INT_MIN. The split GEMM's row scales are then the maxima over the runs.

template <int NQ>
__global__ __launch_bounds__(256) void k_x_pairs(const double* __restrict__ RQ,
                                                 const int2* __restrict__ tiles, int n_orb,
                                                 int n_q, long g0, long cn, long npl, long tpart,
                                                 const double* __restrict__ w,
                                                 double* __restrict__ T, int* __restrict__ pex,
                                                 long pex_stride) {
  __shared__ double Lq[4][NQ][XOB];
  __shared__ double Ls[4][NQ][XOB];
  const int2 tl = tiles[blockIdx.x];
  const int q0 = tl.x * XOB, s0 = tl.y * XOB;
  const long nr = (long)n_orb * n_q;
  const int tq = threadIdx.x >> 4, ts = threadIdx.x & 15;
  int ex2[4][4], ex3[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) ex2[i][j] = ex3[i][j] = INT_MIN;
  const long gb = (long)blockIdx.y * XGB;
  const long ge = gb + XGB < cn ? gb + XGB : cn;
  for (long gl = gb; gl < ge; ++gl) {
    const double* src = RQ + (g0 + gl) * 4 * nr;
    __syncthreads();   // the previous point's rows are no longer read
    for (int e = threadIdx.x; e < 4 * XOB * n_q; e += 256) {
      const int ch = e / (XOB * n_q), r = e % (XOB * n_q);
      const int o = r / n_q, a = r % n_q;
      Lq[ch][a][o] = q0 + o < n_orb ? src[ch * nr + (long)(q0 + o) * n_q + a] : 0.0;
      Ls[ch][a][o] = s0 + o < n_orb ? src[ch * nr + (long)(s0 + o) * n_q + a] : 0.0;
    }
    __syncthreads();
    double t2[4][4], t3[3][4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        t2[i][j] = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) t3[c][i][j] = 0.0;
      }
    for (int a = 0; a < n_q; ++a) {
      double rq[4][4], rs[4][4];   // [ch][i], [ch][j]
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          rq[ch][i] = Lq[ch][a][4 * tq + i];
          rs[ch][i] = Ls[ch][a][ts + 16 * i];
        }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            t2[i][j] = fma(rq[c][i], rs[c][j], t2[i][j]);
            t3[c][i][j] = fma(rs[3][j], rq[c][i], fma(rs[c][j], rq[3][i], t3[c][i][j]));
          }
    }
    const double wg = pex ? w[g0 + gl] : 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = q0 + 4 * tq + i;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int s = s0 + ts + 16 * j;
        if (q <= s && s < n_orb) {
          double* out = T + gl * npl + pair_index(q, s, n_orb);
          out[0] = t2[i][j];
#pragma unroll
          for (int c = 0; c < 3; ++c) out[(1 + c) * tpart] = t3[c][i][j];
          if (pex) {
            int e;
            double v = fabs(t2[i][j] * wg);
            if (v > 0.0) {
              frexp(v, &e);
              ex2[i][j] = max(ex2[i][j], e);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              v = fabs(t3[c][i][j] * wg);
              if (v > 0.0) {
                frexp(v, &e);
                ex3[i][j] = max(ex3[i][j], e);
              }
            }
          }
        }
      }
    }
  }
  if (!pex) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = q0 + 4 * tq + i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int s = s0 + ts + 16 * j;
      if (q <= s && s < n_orb) {
        const long k = pair_index(q, s, n_orb);
        pex[(long)blockIdx.y * npl + k] = ex2[i][j];
        pex[pex_stride + (long)blockIdx.y * npl + k] = ex3[i][j];
      }
    }
  }
}

// Row scales of the split X products from the per-run exponent maxima:
// e = 15 - max_run ex (the row max times 2^e lies in [2^14, 2^15)), 0 for all-zero rows
// and for the padding rows up to rows_pad.
__global__ void k_pair_scales(const int* __restrict__ pex, long pex_stride, int nrun, long npair,
                              long npl, long rows_pad, int* __restrict__ e2,
                              int* __restrict__ e3) {
  const long k = (long)blockIdx.x * 256 + threadIdx.x;
  if (k >= rows_pad) return;
  int m2 = INT_MIN, m3 = INT_MIN;
  if (k < npair)
    for (int r = 0; r < nrun; ++r) {
      m2 = max(m2, pex[(long)r * npl + k]);
      m3 = max(m3, pex[pex_stride + (long)r * npl + k]);
    }
  e2[k] = m2 == INT_MIN ? 0 : 15 - m2;
  e3[k] = m3 == INT_MIN ? 0 : 15 - m3;
}

__global__ void k_zero(double* __restrict__ x, long n) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t < n) x[t] = 0.0;
}

// X[q][s][mu] = X[s][q][mu] = Xp[pair(q, s)][mu]
__global__ void k_unpack_sym(const double* __restrict__ Xp, int n_orb, int n_mu,
                             double* __restrict__ X) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long)n_orb * n_orb * n_mu) return;
  const long mu = t % n_mu;
  const long qs = t / n_mu;
  int q = (int)(qs / n_orb), s = (int)(qs % n_orb);
  if (q > s) {
    const int tmp = q;
    q = s;
    s = tmp;
  }
  X[t] = Xp[pair_index(q, s, n_orb) * n_mu + mu];
}

xtc_status ex_prepare(ExWork& W, const double* phi_piv, const double* lq, const double* xyz,
                      const double* w, const double* xi, long n_g, hipStream_t st) {
  const int nb = (int)cdiv(W.n_orb, XOB);
  hipLaunchKernelGGL(k_fill_tiles, dim3(cdiv(W.ntile, 256)), dim3(256), 0, st, nb, W.ntile,
                     W.tiles);
  XTC_CHECK_LAUNCH();
  const long nr = W.nr;
  GemmArgs g{};   // phia[a][nu] = sum_t LQ[t][a] phi_t(nu)
  g.M = W.n_q; g.N = W.n_mu; g.K = W.n_orb;
  g.A = lq; g.a_sm = 1; g.a_sk = W.n_q;
  g.B = phi_piv; g.b_sk = W.n_mu; g.b_sn = 1;
  g.C = W.phia; g.c_sm = W.n_mu; g.c_sn = 1;
  XTC_TRY(gemm_f64(g, st));
  hipLaunchKernelGGL(k_proj_rows, dim3(cdiv(nr * W.n_mu, 256)), dim3(256), 0, st, phi_piv,
                     (const double*)W.phia, W.n_orb, W.n_q, W.n_mu, W.P);
  XTC_CHECK_LAUNCH();
  if (W.precision == XTC_SPLIT_F16) {
    // Q[s a][g] = sum_nu P[s a][nu] xi_nu(g) over the whole grid, in FP64: the sum over
    // the pivots cancels strongly, so it is done before the split contraction
    for (long g0 = 0; g0 < n_g; g0 += 1L << 20) {
      GemmArgs q{};
      q.M = nr; q.N = (n_g - g0) < (1L << 20) ? (n_g - g0) : (1L << 20); q.K = W.n_mu;
      q.A = W.P; q.a_sm = W.n_mu; q.a_sk = 1;
      q.B = xi + g0; q.b_sk = n_g; q.b_sn = 1;
      q.C = W.Qf + g0; q.c_sm = n_g; q.c_sn = 1;
      XTC_TRY(gemm_f64(q, st));
    }
    Stage1Args sq{xyz, w, W.Qf, w, w, n_g, (int)nr, 0, 0, W.panelR, W.rows_padR, W.bp, 4};
    sq.rho_rows = false;
    XTC_TRY(split_prepare(sq, W.splitQ, st));
  }
  return XTC_OK;
}

// RQ[g][ch][sa] = panelR[ch][sa][g] (ch < 3) or Qf[sa][b0 + g] (ch 3): 64 x 64 tiles
// through LDS so that both the reads (g fastest) and the writes (sa fastest) are whole lines
__global__ __launch_bounds__(256) void k_gather_rq(const double* __restrict__ panelR,
                                                   long rows_padR, long bp,
                                                   const double* __restrict__ Qf, long n_g,
                                                   long b0, long bn, long nr,
                                                   double* __restrict__ RQ) {
  __shared__ double tile[64][65];
  const int ch = blockIdx.z;
  const long sa0 = (long)blockIdx.y * 64, g0 = (long)blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const long sa = sa0 + r, g = g0 + tx;
    double v = 0.0;
    if (sa < nr && g < bn)
      v = ch < 3 ? panelR[((long)ch * rows_padR + sa) * bp + g] : Qf[sa * n_g + b0 + g];
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const long g = g0 + r, sa = sa0 + tx;
    if (g < bn && sa < nr) RQ[(g * 4 + ch) * nr + sa] = tile[tx][r];
  }
}

xtc_status ex_block(ExWork& W, const EECoef& cf, const double* panel, long rows_pad,
                    const double* xyz, const double* xi, long n_g, const double* w, long b0,
                    long bn, bool first, bool want2, bool want3, hipStream_t st) {
  const long nr = W.nr;
  const long bp = W.bp;
  const int n_mu = W.n_mu;
  if (W.precision == XTC_SPLIT_F16) {
    // R^c_{sa}(g) = sum_g' w Q_{sa}(g') d_c u(g, g'): the split stage 1 on the projected
    // rows, so that each R row is split relative to its own scale
    Stage1Args sq{xyz, w, W.Qf, w, w, n_g, (int)nr, b0, bn, W.panelR, W.rows_padR, bp, 4};
    sq.rho_rows = false;
    size_t tk0 = timing_begin(TM_X_STAGE1, st);
    XTC_TRY(stage1_split_f16(sq, cf, W.splitQ, W.splitQ_bytes, st));
    timing_end(tk0, st);
    size_t tk1 = timing_begin(TM_X_PAIRS, st);
    hipLaunchKernelGGL(k_gather_rq, dim3(cdiv(bn, 64), cdiv(nr, 64), 4), dim3(256), 0, st,
                       (const double*)W.panelR, W.rows_padR, bp, (const double*)W.Qf, n_g, b0,
                       bn, nr, W.RQ);
    XTC_CHECK_LAUNCH();
    timing_end(tk1, st);
  }
  // FP64 path: RQ[g][ch][s a] with R^c = P calG^c (ch 0..2) and Q = P xi (ch 3)
  size_t tk1 = timing_begin(TM_X_PAIRS, st);
  for (int ch = 0; ch < 4 && W.precision == XTC_FP64; ++ch) {
    GemmArgs g{};
    g.M = nr; g.N = bn; g.K = n_mu;
    g.A = W.P; g.a_sm = n_mu; g.a_sk = 1;
    if (ch < 3) {
      g.B = panel + (long)ch * rows_pad * bp; g.b_sk = bp; g.b_sn = 1;
    } else {
      g.B = xi + b0; g.b_sk = n_g; g.b_sn = 1;
    }
    g.C = W.RQ + (long)ch * nr; g.c_sm = 1; g.c_sn = 4 * nr;
    XTC_TRY(gemm_f64(g, st));
  }
  timing_end(tk1, st);
  for (long g0 = 0; g0 < bn; g0 += XCH) {
    const long cn = (bn - g0) < XCH ? (bn - g0) : XCH;
    size_t tk2 = timing_begin(TM_X_PAIRS, st);
    dim3 gp((unsigned)W.ntile, cdiv(cn, XGB));
    const bool split = W.precision == XTC_SPLIT_F16;
    if (W.n_q <= 16)
      hipLaunchKernelGGL(k_x_pairs<16>, gp, dim3(256), 0, st, (const double*)W.RQ,
                         (const int2*)W.tiles, W.n_orb, W.n_q, g0, cn, W.npl, W.tpart, w + b0,
                         W.T, split ? W.pex : nullptr, W.pex_stride);
    else
      hipLaunchKernelGGL(k_x_pairs<32>, gp, dim3(256), 0, st, (const double*)W.RQ,
                         (const int2*)W.tiles, W.n_orb, W.n_q, g0, cn, W.npl, W.tpart, w + b0,
                         W.T, split ? W.pex : nullptr, W.pex_stride);
    XTC_CHECK_LAUNCH();
    if (split) {
      const long rp = round_to(W.npair, 128);
      hipLaunchKernelGGL(k_pair_scales, dim3(cdiv(rp, 256)), dim3(256), 0, st, (const int*)W.pex,
                         W.pex_stride, (int)cdiv(cn, XGB), W.npair, W.npl, rp, W.ex2, W.ex3);
      XTC_CHECK_LAUNCH();
    }
    timing_end(tk2, st);
    // Xp2 (+)= T2 diag(w) xi^T ;  Xp3 (+)= sum_c T3^c diag(w) calG^c^T
    const bool init = first && g0 == 0;
    const double* wc = w + b0 + g0;
    size_t tk3 = timing_begin(TM_X_GEMM, st);
    if (want2) {
      if (W.precision == XTC_SPLIT_F16) {
        SplitSeg sg{W.T, 1, W.npl, wc, xi + b0 + g0, n_g, 1};
        XTC_TRY(gemm_split_seg(W.npair, n_mu, cn, &sg, 1, W.Xp, n_mu, !init, W.gsplit,
                               W.gsplit_bytes, st, W.ex2, TM_X_MFMA));
      } else {
        GemmArgs g{};
        g.M = W.npair; g.N = n_mu; g.K = cn;
        g.A = W.T; g.a_sm = 1; g.a_sk = W.npl;
        g.s = wc;
        g.B = xi + b0 + g0; g.b_sk = 1; g.b_sn = n_g;
        g.C = W.Xp; g.c_sm = n_mu; g.c_sn = 1;
        g.beta = init ? 0.0 : 1.0;
        XTC_TRY(gemm_f64(g, st));
      }
    }
    if (want3) {
      double* X3p = W.Xp + W.npair * n_mu;
      SplitSeg sg[3];
      for (int c = 0; c < 3; ++c)
        sg[c] = SplitSeg{W.T + (1 + c) * W.tpart, 1, W.npl, wc,
                         panel + (long)c * rows_pad * bp + g0, bp, 1};
      if (W.precision == XTC_SPLIT_F16) {
        XTC_TRY(gemm_split_seg(W.npair, n_mu, cn, sg, 3, X3p, n_mu, !init, W.gsplit,
                               W.gsplit_bytes, st, W.ex3, TM_X_MFMA));
      } else {
        for (int c = 0; c < 3; ++c) {
          GemmArgs g{};
          g.M = W.npair; g.N = n_mu; g.K = cn;
          g.A = sg[c].A; g.a_sm = 1; g.a_sk = W.npl;
          g.s = wc;
          g.B = sg[c].B; g.b_sk = 1; g.b_sn = bp;
          g.C = X3p; g.c_sm = n_mu; g.c_sn = 1;
          g.beta = (init && c == 0) ? 0.0 : 1.0;
          XTC_TRY(gemm_f64(g, st));
        }
      }
    }
    timing_end(tk3, st);
  }
  return XTC_OK;
}

xtc_status ex_finish(ExWork& W, double* X2, double* X3, bool empty, hipStream_t st) {
  const long ntot = (long)W.n_orb * W.n_orb * W.n_mu;
  for (int i = 0; i < 2; ++i) {
    double* X = i == 0 ? X2 : X3;
    if (!X) continue;
    if (empty)
      hipLaunchKernelGGL(k_zero, dim3(cdiv(ntot, 256)), dim3(256), 0, st, X, ntot);
    else
      hipLaunchKernelGGL(k_unpack_sym, dim3(cdiv(ntot, 256)), dim3(256), 0, st,
                         (const double*)(W.Xp + (long)i * W.npair * W.n_mu), W.n_orb, W.n_mu, X);
    XTC_CHECK_LAUNCH();
  }
  return XTC_OK;
}

xtc_status check_exchange_args(const xtc_exchange* ex, int32_t n_mu) {
  XTC_REQUIRE(ex->phi_piv && ex->lq, "exchange: null phi_piv or lq");
  XTC_REQUIRE(ex->X2 || ex->X3, "exchange: no output requested");
  XTC_REQUIRE(ex->n_orb > 0, "exchange: n_orb must be positive");
  XTC_REQUIRE(ex->n_q > 0 && ex->n_q <= 32, "exchange: projector rank must be 1..32");
  (void)n_mu;
  return XTC_OK;
}

}  // namespace xtc

using namespace xtc;

extern "C" xtc_status xtc_exchange_terms(const xtc_grid* grid, const xtc_correlator* corr,
                                         int32_t n_mu, const double* xi, int32_t n_orb,
                                         const double* phi_piv, int32_t n_q, const double* lq,
                                         int32_t precision, int64_t bra_begin, int64_t bra_end,
                                         double* X2, double* X3, void* ws, size_t ws_bytes,
                                         void* stream) {
  XTC_REQUIRE(grid && corr && xi, "exchange: null argument");
  const xtc_exchange ex{n_orb, phi_piv, n_q, lq, X2, X3};
  XTC_TRY(check_exchange_args(&ex, n_mu));
  XTC_REQUIRE(grid->n_g > 0 && grid->xyz && grid->w, "exchange: empty grid");
  XTC_REQUIRE(n_mu > 0 && n_mu <= grid->n_g, "exchange: bad n_mu");
  XTC_REQUIRE(bra_begin >= 0 && bra_begin <= bra_end && bra_end <= grid->n_g,
              "exchange: bra range outside the grid");
  XTC_REQUIRE(precision == XTC_FP64 || precision == XTC_SPLIT_F16, "exchange: bad precision");
  XTC_REQUIRE(corr->n_terms > 0 && corr->mno && corr->c && corr->d > 0.0,
              "exchange: bad correlator");
  XTC_REQUIRE(corr->form == XTC_U_EE || corr->form == XTC_U_BH,
              "exchange: unknown correlator form");
  if (corr->form == XTC_U_BH && precision != XTC_FP64) {
    set_error("exchange: the BH correlator is evaluated on the FP64 path only");
    return XTC_ERR_UNSUPPORTED;
  }
  EECoef cf;
  BHTable bt;
  const bool bh = corr->form == XTC_U_BH;
  if (bh) XTC_TRY(bh_build(corr, &bt, &cf));
  else XTC_TRY(ee_coefficients(corr, &cf));
  hipStream_t st = as_stream(stream);
  const long n_g = grid->n_g;
  Arena ar(ws, ws_bytes);
  ExLayout L = layout_ex(ar, n_g, n_mu, n_orb, n_q, precision);
  XTC_TRY(need_ws(ar));
  XTC_TRY(check_weights(grid, ws, ws_bytes, st, "xtc_exchange_terms"));
  if (bra_end == bra_begin) {
    XTC_TRY(ex_finish(L.W, X2, X3, true, st));
    XTC_HIP(hipStreamSynchronize(st));
    return XTC_OK;
  }
  if (bh) XTC_HIP(hipMemcpyAsync(L.bh, &bt, sizeof(BHTable), hipMemcpyHostToDevice, st));
  XTC_TRY(ex_prepare(L.W, phi_piv, lq, grid->xyz, grid->w, xi, n_g, st));
  // the panel's density rows are not used here: w stands in for rho and rhot
  Stage1Args s1{grid->xyz, grid->w, xi, grid->w, grid->w, n_g, n_mu, 0, 0, L.panel,
                L.rows_pad, L.bp, 4};
  s1.rho_rows = false;
  if (bh) s1.bh = L.bh;
  if (precision == XTC_SPLIT_F16) {
    size_t tk = timing_begin(TM_SPLIT_PREP, st);
    XTC_TRY(split_prepare(s1, L.split, st));
    timing_end(tk, st);
  }
  const int nsb = (int)cdiv(bra_end - bra_begin, L.bp);
  for (int sb = 0; sb < nsb; ++sb) {
    const long b0 = bra_begin + (long)sb * L.bp;
    const long bn = (bra_end - b0) < L.bp ? (bra_end - b0) : L.bp;
    s1.b0 = b0;
    s1.bn = bn;
    size_t tk = timing_begin(TM_STAGE1, st);
    if (precision == XTC_FP64) XTC_TRY(stage1_f64(s1, cf, st));
    else XTC_TRY(stage1_split_f16(s1, cf, L.split, L.split_bytes, st));
    timing_end(tk, st);
    XTC_TRY(ex_block(L.W, cf, L.panel, L.rows_pad, grid->xyz, xi, n_g, grid->w, b0, bn, sb == 0,
                     X2 != nullptr, X3 != nullptr, st));
  }
  XTC_TRY(ex_finish(L.W, X2, X3, false, st));
  XTC_HIP(hipStreamSynchronize(st));
  return XTC_OK;
}
