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
#include "bh.hpp"
#include "contract.hpp"
#include "gemm_split.hpp"
#include "plans.hpp"
#include "timing.hpp"

namespace xtc {

constexpr long XSUPER = 16384;   // bra super-block
constexpr long XCH = 2048;       // bra chunk of the pair products and X GEMMs
constexpr int XOB = 64;          // orbital block of the pair kernel

struct ExLayout {
  double* phia; double* P; double* panel; void* split; size_t split_bytes;
  double* RQ; double* T; double* Xp; int2* tiles; void* gsplit; size_t gsplit_bytes;
  BHTable* bh; long bp; long rows_pad; long npair; long npl; long tpart; int ntile;
};

static inline long round_to(long x, long m) { return ((x + m - 1) / m) * m; }

static ExLayout layout_ex(Arena& ar, int64_t n_g, int n_mu, int n_orb, int n_q, int precision) {
  ExLayout L;
  L.bp = n_g < XSUPER ? round_to(n_g, 64) : XSUPER;
  L.rows_pad = round_to(n_mu + 2, 256);
  L.npair = (long)n_orb * (n_orb + 1) / 2;
  L.npl = round_to(L.npair, 32);
  const int nb = (int)cdiv(n_orb, XOB);
  L.ntile = nb * (nb + 1) / 2;
  const long nr = (long)n_orb * n_q;
  const long xch = L.bp < XCH ? L.bp : XCH;
  L.tpart = xch * L.npl;
  L.phia = ar.take<double>((size_t)n_q * n_mu);
  L.P = ar.take<double>((size_t)nr * n_mu);
  L.panel = ar.take<double>((size_t)4 * L.rows_pad * L.bp);
  L.split_bytes = precision == XTC_SPLIT_F16
                      ? split_scratch_bytes(n_g, n_mu) + rho_row_scratch_bytes(L.bp) : 0;
  L.split = L.split_bytes ? (void*)ar.take<char>(L.split_bytes) : nullptr;
  L.RQ = ar.take<double>((size_t)4 * nr * L.bp);
  L.T = ar.take<double>((size_t)4 * L.tpart);
  L.Xp = ar.take<double>((size_t)2 * L.npair * n_mu);
  L.tiles = ar.take<int2>(L.ntile);
  L.gsplit_bytes = precision == XTC_SPLIT_F16 ? gemm_split_seg_scratch_bytes(L.npair, n_mu, xch, 3)
                                              : 0;
  L.gsplit = L.gsplit_bytes ? (void*)ar.take<char>(L.gsplit_bytes) : nullptr;
  L.bh = ar.take<BHTable>(1);
  return L;
}

size_t ws_exchange(int64_t n_g, int n_orb, int n_mu, int n_q, int precision) {
  Arena ar(nullptr, 0);
  layout_ex(ar, n_g, n_mu, n_orb, n_q, precision);
  return ar.used;
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

// Pair products of one bra point for one (q block, s block) tile of 64 x 64
// orbitals (q block <= s block). LDS holds both blocks' rows [ch][a][orbital]
// (ch = R^x, R^y, R^z, Q); thread (tq, ts) owns q = q0 + 4 tq + i and
// s = s0 + ts + 16 j (i, j < 4), so a row of 16 threads stores 16 consecutive pairs.
// RQ: [bp][4][n_orb n_q] (point-major); T: [4][xch][npl], part stride tpart.
template <int NQ>
__global__ __launch_bounds__(256) void k_x_pairs(const double* __restrict__ RQ,
                                                 const int2* __restrict__ tiles, int n_orb,
                                                 int n_q, long g0, long npl, long tpart,
                                                 double* __restrict__ T) {
  __shared__ double Lq[4][NQ][XOB];
  __shared__ double Ls[4][NQ][XOB];
  const int2 tl = tiles[blockIdx.x];
  const int q0 = tl.x * XOB, s0 = tl.y * XOB;
  const long gl = blockIdx.y;              // point within the chunk
  const long nr = (long)n_orb * n_q;
  const double* src = RQ + (g0 + gl) * 4 * nr;
  for (int e = threadIdx.x; e < 4 * XOB * n_q; e += 256) {
    const int ch = e / (XOB * n_q), r = e % (XOB * n_q);
    const int o = r / n_q, a = r % n_q;
    Lq[ch][a][o] = q0 + o < n_orb ? src[ch * nr + (long)(q0 + o) * n_q + a] : 0.0;
    Ls[ch][a][o] = s0 + o < n_orb ? src[ch * nr + (long)(s0 + o) * n_q + a] : 0.0;
  }
  __syncthreads();
  const int tq = threadIdx.x >> 4, ts = threadIdx.x & 15;
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
      }
    }
  }
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

}  // namespace xtc

using namespace xtc;

extern "C" xtc_status xtc_exchange_terms(const xtc_grid* grid, const xtc_correlator* corr,
                                         int32_t n_mu, const double* xi, int32_t n_orb,
                                         const double* phi_piv, int32_t n_q, const double* lq,
                                         int32_t precision, int64_t bra_begin, int64_t bra_end,
                                         double* X2, double* X3, void* ws, size_t ws_bytes,
                                         void* stream) {
  XTC_REQUIRE(grid && corr && xi && phi_piv && lq, "exchange: null argument");
  XTC_REQUIRE(X2 || X3, "exchange: no output requested");
  XTC_REQUIRE(grid->n_g > 0 && grid->xyz && grid->w, "exchange: empty grid");
  XTC_REQUIRE(n_mu > 0 && n_mu <= grid->n_g && n_orb > 0, "exchange: bad sizes");
  XTC_REQUIRE(n_q > 0 && n_q <= 32, "exchange: projector rank must be 1..32");
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
  if (bh) XTC_HIP(hipMemcpyAsync(L.bh, &bt, sizeof(BHTable), hipMemcpyHostToDevice, st));
  std::vector<int2> tl;
  {
    const int nb = (int)cdiv(n_orb, XOB);
    for (int qb = 0; qb < nb; ++qb)
      for (int sb = qb; sb < nb; ++sb) tl.push_back(make_int2(qb, sb));
    XTC_HIP(hipMemcpyAsync(L.tiles, tl.data(), sizeof(int2) * tl.size(), hipMemcpyHostToDevice,
                           st));
  }
  const long nr = (long)n_orb * n_q;
  {
    // phia[a][nu] = sum_t LQ[t][a] phi_t(nu)
    GemmArgs g{};
    g.M = n_q; g.N = n_mu; g.K = n_orb;
    g.A = lq; g.a_sm = 1; g.a_sk = n_q;
    g.B = phi_piv; g.b_sk = n_mu; g.b_sn = 1;
    g.C = L.phia; g.c_sm = n_mu; g.c_sn = 1;
    XTC_TRY(gemm_f64(g, st));
  }
  hipLaunchKernelGGL(k_proj_rows, dim3(cdiv(nr * n_mu, 256)), dim3(256), 0, st, phi_piv,
                     (const double*)L.phia, n_orb, n_q, n_mu, L.P);
  XTC_CHECK_LAUNCH();
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
  const long ntot = (long)n_orb * n_orb * n_mu;
  if (bra_end == bra_begin) {
    for (double* X : {X2, X3})
      if (X) {
        hipLaunchKernelGGL(k_zero, dim3(cdiv(ntot, 256)), dim3(256), 0, st, X, ntot);
        XTC_CHECK_LAUNCH();
      }
    XTC_HIP(hipStreamSynchronize(st));
    return XTC_OK;
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
    // RQ[g][ch][s a]: R^c = P calG^c (ch 0..2) and Q = P xi (ch 3) over the block
    size_t tk1 = timing_begin(TM_X_PAIRS, st);
    for (int ch = 0; ch < 4; ++ch) {
      GemmArgs g{};
      g.M = nr; g.N = bn; g.K = n_mu;
      g.A = L.P; g.a_sm = n_mu; g.a_sk = 1;
      if (ch < 3) {
        g.B = L.panel + (long)ch * L.rows_pad * L.bp; g.b_sk = L.bp; g.b_sn = 1;
      } else {
        g.B = xi + b0; g.b_sk = n_g; g.b_sn = 1;
      }
      g.C = L.RQ + (long)ch * nr; g.c_sm = 1; g.c_sn = 4 * nr;
      XTC_TRY(gemm_f64(g, st));
    }
    timing_end(tk1, st);
    for (long g0 = 0; g0 < bn; g0 += XCH) {
      const long cn = (bn - g0) < XCH ? (bn - g0) : XCH;
      size_t tk2 = timing_begin(TM_X_PAIRS, st);
      dim3 gp((unsigned)L.ntile, (unsigned)cn);
      if (n_q <= 16)
        hipLaunchKernelGGL(k_x_pairs<16>, gp, dim3(256), 0, st, (const double*)L.RQ,
                           (const int2*)L.tiles, n_orb, n_q, g0, L.npl, L.tpart, L.T);
      else
        hipLaunchKernelGGL(k_x_pairs<32>, gp, dim3(256), 0, st, (const double*)L.RQ,
                           (const int2*)L.tiles, n_orb, n_q, g0, L.npl, L.tpart, L.T);
      XTC_CHECK_LAUNCH();
      timing_end(tk2, st);
      // Xp2 (+)= T2 diag(w) xi^T ;  Xp3 (+)= sum_c T3^c diag(w) calG^c^T
      const bool first = sb == 0 && g0 == 0;
      const double* wc = grid->w + b0 + g0;
      size_t tk3 = timing_begin(TM_X_GEMM, st);
      if (X2) {
        if (precision == XTC_SPLIT_F16) {
          SplitSeg sg{L.T, 1, L.npl, wc, xi + b0 + g0, n_g, 1};
          XTC_TRY(gemm_split_seg(L.npair, n_mu, cn, &sg, 1, L.Xp, n_mu, !first, L.gsplit,
                                 L.gsplit_bytes, st));
        } else {
          GemmArgs g{};
          g.M = L.npair; g.N = n_mu; g.K = cn;
          g.A = L.T; g.a_sm = 1; g.a_sk = L.npl;
          g.s = wc;
          g.B = xi + b0 + g0; g.b_sk = 1; g.b_sn = n_g;
          g.C = L.Xp; g.c_sm = n_mu; g.c_sn = 1;
          g.beta = first ? 0.0 : 1.0;
          XTC_TRY(gemm_f64(g, st));
        }
      }
      if (X3) {
        double* X3p = L.Xp + L.npair * n_mu;
        SplitSeg sg[3];
        for (int c = 0; c < 3; ++c)
          sg[c] = SplitSeg{L.T + (1 + c) * L.tpart, 1, L.npl, wc,
                           L.panel + (long)c * L.rows_pad * L.bp + g0, L.bp, 1};
        if (precision == XTC_SPLIT_F16) {
          XTC_TRY(gemm_split_seg(L.npair, n_mu, cn, sg, 3, X3p, n_mu, !first, L.gsplit,
                                 L.gsplit_bytes, st));
        } else {
          for (int c = 0; c < 3; ++c) {
            GemmArgs g{};
            g.M = L.npair; g.N = n_mu; g.K = cn;
            g.A = sg[c].A; g.a_sm = 1; g.a_sk = L.npl;
            g.s = wc;
            g.B = sg[c].B; g.b_sk = 1; g.b_sn = L.bp;
            g.C = X3p; g.c_sm = n_mu; g.c_sn = 1;
            g.beta = (first && c == 0) ? 0.0 : 1.0;
            XTC_TRY(gemm_f64(g, st));
          }
        }
      }
      timing_end(tk3, st);
    }
  }
  if (X2) {
    hipLaunchKernelGGL(k_unpack_sym, dim3(cdiv(ntot, 256)), dim3(256), 0, st,
                       (const double*)L.Xp, n_orb, n_mu, X2);
    XTC_CHECK_LAUNCH();
  }
  if (X3) {
    hipLaunchKernelGGL(k_unpack_sym, dim3(cdiv(ntot, 256)), dim3(256), 0, st,
                       (const double*)(L.Xp + L.npair * n_mu), n_orb, n_mu, X3);
    XTC_CHECK_LAUNCH();
  }
  // the tile table is host memory read by the copy above
  XTC_HIP(hipStreamSynchronize(st));
  return XTC_OK;
}
