// Adjoint of xtc_kernel_contract with respect to the linear correlator
// coefficients c_k (EE form u = sum_k c_k rbar^{o_k}), in FP64.
//
// All outputs are built from the stage-1 panel P[ch][row][g] = sum_g' A[row][g'] K_ch(g, g')
// (rows: w xi_mu, w rho_gamma, w rhot). Reverse mode in two parts:
//  1. stage-2 adjoints give the panel cotangent Pbar[ch][row][g] (GEMMs with the output
//     cotangents, plus the D1 term through H, whose cotangent lands on the rhot row);
//  2. dL/dc_k = sum_{g,g'} sum_ch M_ch(g,g') dK_ch(g,g')/dc_k with
//     M_ch(g,g') = sum_row Pbar[ch][row][g] A[row][g'],
//     formed tile by tile on the matrix cores (v_mfma_f64_16x16x4f64) and contracted at
//     once with the per-pair derivative basis; M is never stored.
// For the channels: dK_c/dc_k = f_k Delta_c (c = x, y, z), d|grad u|^2/dc_k = 2 u' u'_k,
// d lap u/dc_k = lap_k, with f_k, u'_k, lap_k the kernels of the unit coefficient e_k.
// The kernel tiles are regenerated from coordinates; the D cotangents add one
// recomputation of the forward panel per bra super-block.
#include "bh.hpp"
#include "contract.hpp"
#include "plans.hpp"
#include "timing.hpp"

namespace xtc {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr long GSUPER = 16384;
constexpr int GT = 64;        // bra x ket tile
constexpr int GK = 16;        // rows per LDS stage
constexpr int KSEG = 8;       // ket segments (grid y)

struct GradBasis {
  double d;
  int n;               // parameters
  int o[MAXQ];         // powers
  int omax;
  int want_d;          // also dL/dd (slot n)
  double c[MAXQ];      // the coefficients (for dL/dd)
};

// Per-pair contribution to dL/dc_k for every k, given M for the NCH channels.
template <int NCH>
__device__ __forceinline__ void pair_grad(const EECoef& cf, const GradBasis& gb, double dx,
                                          double dy, double dz, const double* m, double* dth) {
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double d = gb.d;
  const double t = 1.0 / (1.0 + d * r);
  const double e = d * r * t;
  const double t2 = t * t, t3 = t2 * t, t4 = t2 * t2;
  double p1 = 0.0;
  for (int j = cf.n1 - 1; j >= 0; --j) p1 = p1 * e + cf.q1[j];
  const double up = d * t2 * p1;                      // u' at the current coefficients
  const double sf = m[0] * dx + m[1] * dy + m[2] * dz;
  const double s3 = 2.0 * up * m[3];
  const double s4 = NCH > 4 ? m[4] : 0.0;
  double ep[MAXQ + 1];
  ep[0] = 1.0;
  for (int j = 1; j <= gb.omax; ++j) ep[j] = ep[j - 1] * e;
  double dd = 0.0;
  for (int k = 0; k < gb.n; ++k) {
    const int o = gb.o[k];
    double fk = 0.0, upk = 0.0, lapk = 0.0;
    double fd = 0.0, upd = 0.0, lapd = 0.0;   // d/dd of the unit-coefficient kernels
    if (o >= 2) {
      fk = d * d * t3 * o * ep[o - 2];
      upk = d * t2 * o * ep[o - 1];
      lapk = d * d * t4 * o * (o - 1) * ep[o - 2] - 2.0 * d * d * t3 * o * ep[o - 1] + 2.0 * fk;
      if (gb.want_d) {
        // d/dd [d^2 t^3 e^m] = d t^3 e^m (2 - 3e + m t), d/dd [d t^2 e^m] = t^2 e^m (1 - 2e + m t),
        // d/dd [d^2 t^4 e^m] = d t^4 e^m (2 - 4e + m t)   (t' = -r t^2, e' = r t^2)
        fd = o * d * t3 * ep[o - 2] * (2.0 - 3.0 * e + (o - 2) * t);
        upd = o * t2 * ep[o - 1] * (1.0 - 2.0 * e + (o - 1) * t);
        lapd = o * (o - 1) * d * t4 * ep[o - 2] * (2.0 - 4.0 * e + (o - 2) * t) -
               2.0 * o * d * t3 * ep[o - 1] * (2.0 - 3.0 * e + (o - 1) * t) + 2.0 * fd;
      }
    } else if (o == 1) {
      upk = d * t2;
      upd = t2 * (1.0 - 2.0 * e);
      if (r > 0.0) {
        fk = d * t2 / r;
        lapk = -2.0 * d * d * t3 + 2.0 * fk;
        fd = t2 * (1.0 / r - 2.0 * d * t);
        lapd = -2.0 * d * t3 * (2.0 - 3.0 * e) + 2.0 * fd;
      }
    }
    dth[k] += sf * fk + s3 * upk + s4 * lapk;
    dd += gb.c[k] * (sf * fd + s3 * upd + s4 * lapd);
  }
  if (gb.want_d) dth[gb.n] += dd;
}

// M_c(b, k) = sum_row Pbar[c][row][b] A[row][k] over the workgroup's 64 x 64 pair tile,
// rows in steps of GK through LDS. With PF the next step's tiles are loaded into registers
// while the current step's MFMAs run (the pair kernels run one wave per SIMD, so nothing
// else hides the load latency); kernels without the registers for it load in place.
template <int NCH, bool PF>
__device__ __forceinline__ void m_tiles(const double* __restrict__ Pb, long rows_pad, long bp,
                                        int n_rows, const double* __restrict__ xi,
                                        const double* __restrict__ rho,
                                        const double* __restrict__ rhot,
                                        const double* __restrict__ w, long n_g, int n_mu,
                                        long bt0, long bn, long kc, long k_hi,
                                        double (*Gs)[GK][GT + 1], double (*As)[GT + 1],
                                        d4 (&acc)[NCH][2][2]) {
  constexpr int NG = NCH * GK * GT / 256, NA = GK * GT / 256;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  double pg[NG], pa[NA];
  auto fetch = [&](int r0) {
    // Pbar tile: NCH x GK rows x 64 bra (bra contiguous in memory)
#pragma unroll
    for (int q = 0; q < NG; ++q) {
      const int e = tid + 256 * q;
      const int c = e / (GK * GT), rr = (e / GT) % GK, bb = e % GT;
      const long row = r0 + rr, b = bt0 + bb;
      pg[q] = (row < n_rows && b < bn) ? Pb[((long)c * rows_pad + row) * bp + b] : 0.0;
    }
    // A tile: GK rows x 64 ket
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      const int rr = e / GT, kk = e % GT;
      const long row = r0 + rr, g = kc + kk;
      double v = 0.0;
      if (row < n_rows && g < k_hi)
        v = w[g] * (row < n_mu ? xi[row * n_g + g] : (row == n_mu ? rho[g] : rhot[g]));
      pa[q] = v;
    }
  };
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[c][i][j] = (d4){0.0, 0.0, 0.0, 0.0};
  if (PF) fetch(0);
  for (int r0 = 0; r0 < n_rows; r0 += GK) {
    __syncthreads();
    if (PF) {
#pragma unroll
      for (int q = 0; q < NG; ++q) {
        const int e = tid + 256 * q;
        Gs[e / (GK * GT)][(e / GT) % GK][e % GT] = pg[q];
      }
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int e = tid + 256 * q;
        As[e / GT][e % GT] = pa[q];
      }
    } else {
      for (int e = tid; e < NCH * GK * GT; e += 256) {
        const int c = e / (GK * GT), rr = (e / GT) % GK, bb = e % GT;
        const long row = r0 + rr, b = bt0 + bb;
        Gs[c][rr][bb] = (row < n_rows && b < bn) ? Pb[((long)c * rows_pad + row) * bp + b] : 0.0;
      }
      for (int e = tid; e < GK * GT; e += 256) {
        const int rr = e / GT, kk = e % GT;
        const long row = r0 + rr, g = kc + kk;
        double v = 0.0;
        if (row < n_rows && g < k_hi)
          v = w[g] * (row < n_mu ? xi[row * n_g + g] : (row == n_mu ? rho[g] : rhot[g]));
        As[rr][kk] = v;
      }
    }
    __syncthreads();
    if (PF && r0 + GK < n_rows) fetch(r0 + GK);
#pragma unroll
    for (int s = 0; s < GK / 4; ++s) {
      const double b0v = As[4 * s + lk][32 * wn + li];
      const double b1v = As[4 * s + lk][32 * wn + 16 + li];
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const double a0 = Gs[c][4 * s + lk][32 * wm + li];
        const double a1 = Gs[c][4 * s + lk][32 * wm + 16 + li];
        acc[c][0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0v, acc[c][0][0], 0, 0, 0);
        acc[c][0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1v, acc[c][0][1], 0, 0, 0);
        acc[c][1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0v, acc[c][1][0], 0, 0, 0);
        acc[c][1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1v, acc[c][1][1], 0, 0, 0);
      }
    }
  }
}

template <int NCH>
__global__ __launch_bounds__(256) void k_grad_pairs(
    const double* __restrict__ Pb, long rows_pad, long bp, int n_rows,
    const double* __restrict__ xi, const double* __restrict__ rho, const double* __restrict__ rhot,
    const double* __restrict__ w, const double* __restrict__ xyz, long n_g, int n_mu, long b0,
    long bn, EECoef cf, GradBasis gb, double* __restrict__ partials) {
  __shared__ double Gs[NCH][GK][GT + 1];   // Pbar rows x bra
  __shared__ double As[GK][GT + 1];        // A rows x ket
  __shared__ double bxyz[3][GT];
  __shared__ double kxyz[3][GT];
  __shared__ double red[4][MAXQ + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  const long bt0 = (long)blockIdx.x * GT;               // bra tile origin within the block
  const long per = ((n_g + KSEG - 1) / KSEG + GT - 1) / GT * GT;
  const long k_lo = (long)blockIdx.y * per;
  const long k_hi = k_lo + per < n_g ? k_lo + per : n_g;
  if (tid < GT) {
    long b = b0 + bt0 + tid;
    if (b > b0 + bn - 1) b = b0 + bn - 1;
    bxyz[0][tid] = xyz[b];
    bxyz[1][tid] = xyz[n_g + b];
    bxyz[2][tid] = xyz[2 * n_g + b];
  }
  double dth[MAXQ + 1];
  for (int k = 0; k <= MAXQ; ++k) dth[k] = 0.0;

  for (long kc = k_lo; kc < k_hi; kc += GT) {
    __syncthreads();
    if (tid < GT) {
      long g = kc + tid;
      if (g > n_g - 1) g = n_g - 1;
      kxyz[0][tid] = xyz[g];
      kxyz[1][tid] = xyz[n_g + g];
      kxyz[2][tid] = xyz[2 * n_g + g];
    }
    d4 acc[NCH][2][2];
    m_tiles<NCH, NCH == 4>(Pb, rows_pad, bp, n_rows, xi, rho, rhot, w, n_g, n_mu, bt0, bn, kc,
                           k_hi, Gs, As, acc);
    // epilogue: the 16 pairs this lane holds, D[(l/16) + 4r][l%16] = M[bra][ket]
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int bi = 32 * wm + 16 * i + lk + 4 * r;
          const int kj = 32 * wn + 16 * j + li;
          if (bt0 + bi >= bn || kc + kj >= k_hi) continue;
          double m[NCH];
#pragma unroll
          for (int c = 0; c < NCH; ++c) m[c] = acc[c][i][j][r];
          pair_grad<NCH>(cf, gb, bxyz[0][bi] - kxyz[0][kj], bxyz[1][bi] - kxyz[1][kj],
                         bxyz[2][bi] - kxyz[2][kj], m, dth);
        }
  }
  // deterministic block reduction of the parameter partials (and dL/dd in slot n)
  const int nout = gb.n + gb.want_d;
  for (int k = 0; k < nout; ++k) {
    double v = dth[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  if (tid < nout) {
    const long blk = (long)blockIdx.y * gridDim.x + blockIdx.x;
    partials[blk * (MAXQ + 1) + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
  }
}

// --- multi-centre Boys-Handy form ---------------------------------------------------
// Per-pair adjoint for the BH correlator (see bh.hpp for N, S and csym). With the
// cotangent projections
//   r12 > 0:  V = M_vec + 2 M_sq grad u,  W = V . rhat12;
//   r12 = 0:  V = M_vec + 2 M_sq N,       W = 2 M_sq S,
// the derivative of the pair's contribution with respect to the coefficient of the
// term (m, n, o) of type t is
//   sum_{I of type t} [ (V . grad a_1I) rbar^o dP_mn + W o rbar^{o-1} d t^2 P_mn ],
//   P_mn = a_1^m a_2^n + a_1^n a_2^m,  dP_mn = m a_1^{m-1} a_2^n + n a_1^{n-1} a_2^m.
// Z[t][m][n][o] accumulates the (m, n) half of both sums; the parameter is
// Z[t][m][n][o] + Z[t][n][m][o]. The (0, 0, o) terms need only the nucleus-free sum
// Zee[o] = sum W o rbar^{o-1} d t^2 (times 2 per nucleus of the type).
// BH partial stride: [types x 64 Z][MAXQ + 1 Zee][dL/dd, dL/db_t per type]
constexpr int ZS = BH_MAXTYPE * 64 + MAXQ + 1 + 1 + BH_MAXTYPE;

template <int NT, bool LIN, bool NL>
__device__ __forceinline__ void pair_grad_bh(const EECoef& cf, const BHTable* __restrict__ T,
                                             const double (*Cs)[BH_NP][BH_NP][BH_NO],
                                             int nn, const double (*TB)[4][GT], int bi,
                                             const double (*TA)[GT], int kj, double dx, double dy,
                                             double dz, const double* m, double* z, double* zee,
                                             int omax_ee, double* znl) {
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double t = 1.0 / (1.0 + cf.d * r);
  const double e = cf.d * r * t;
  const double dedr = cf.d * t * t;
  // forward: F_o and grad F_o at this pair
  double F[BH_NO] = {0.0, 0.0, 0.0, 0.0};
  double GF[BH_NO][3] = {};
  for (int I = 0; I < nn; ++I) {
    const int ty = T->type[I];
    const double a1 = TB[I][0][bi], a2 = TA[I][kj];
    const double A1[BH_NP] = {1.0, a1, a1 * a1, a1 * a1 * a1};
    const double dA1[BH_NP] = {0.0, 1.0, 2.0 * a1, 3.0 * a1 * a1};
    const double A2[BH_NP] = {1.0, a2, a2 * a2, a2 * a2 * a2};
#pragma unroll
    for (int o = 0; o < BH_NO; ++o) {
      double f = 0.0, dv = 0.0;
#pragma unroll
      for (int mm = 0; mm < BH_NP; ++mm) {
        double g = 0.0;
#pragma unroll
        for (int n = 0; n < BH_NP; ++n) g += Cs[ty][mm][n][o] * A2[n];
        f += A1[mm] * g;
        dv += dA1[mm] * g;
      }
      F[o] += f;
      GF[o][0] += dv * TB[I][1][bi];
      GF[o][1] += dv * TB[I][2][bi];
      GF[o][2] += dv * TB[I][3][bi];
    }
  }
  const double E[BH_NO] = {1.0, e, e * e, e * e * e};
  double N[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) N[c] = GF[0][c] + E[1] * GF[1][c] + E[2] * GF[2][c] + E[3] * GF[3][c];
  double p1 = 0.0;
  for (int j = cf.n1 - 1; j >= 0; --j) p1 = p1 * e + cf.q1[j];
  const double S = dedr * (F[1] + 2.0 * E[1] * F[2] + 3.0 * E[2] * F[3] + p1);
  double V[3], W;
  if (r > 0.0) {
    const double sr = S / r;
    const double G0 = N[0] + sr * dx, G1 = N[1] + sr * dy, G2 = N[2] + sr * dz;
    V[0] = m[0] + 2.0 * m[3] * G0;
    V[1] = m[1] + 2.0 * m[3] * G1;
    V[2] = m[2] + 2.0 * m[3] * G2;
    W = (V[0] * dx + V[1] * dy + V[2] * dz) / r;
  } else {
    V[0] = m[0] + 2.0 * m[3] * N[0];
    V[1] = m[1] + 2.0 * m[3] * N[1];
    V[2] = m[2] + 2.0 * m[3] * N[2];
    W = 2.0 * m[3] * S;
  }
  const double wd = W * dedr;
  const double ES[BH_NO] = {0.0, wd, 2.0 * e * wd, 3.0 * e * e * wd};
  if (NL) {
    // d: rbar' = r t^2, (d t^2)' = t^2 (1 - 2 rbar); N' = sum_o o rbar^{o-1} rbar' grad F_o,
    // S' = (d t^2)' (F_1 + 2 rbar F_2 + 3 rbar^2 F_3 + U'_ee) + d t^2 rbar' (2 F_2 + 6 rbar F_3 + U''_ee)
    const double de_dd = r * t * t;
    const double d_dedr = t * t * (1.0 - 2.0 * e);
    double p1p = 0.0;
    for (int j = cf.n1 - 1; j >= 1; --j) p1p = p1p * e + j * cf.q1[j];
    const double inner = F[1] + 2.0 * e * F[2] + 3.0 * e * e * F[3] + p1;
    const double dS = d_dedr * inner + dedr * de_dd * (2.0 * F[2] + 6.0 * e * F[3] + p1p);
    double vdn = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c)
      vdn += V[c] * de_dd * (GF[1][c] + 2.0 * e * GF[2][c] + 3.0 * e * e * GF[3][c]);
    znl[0] += vdn + W * dS;
  }
  // electron-electron (0, 0, o) terms: W o e^{o-1} d t^2
  if (LIN) {
    double ep = 1.0;   // e^{o-1}
    for (int o = 1; o <= omax_ee; ++o) {
      zee[o] += o * ep * wd;
      ep *= e;
    }
  }
  for (int I = 0; I < nn; ++I) {
    const int ty = T->type[I];
    const double a1 = TB[I][0][bi], a2 = TA[I][kj];
    const double q = V[0] * TB[I][1][bi] + V[1] * TB[I][2][bi] + V[2] * TB[I][3][bi];
    const double A1[BH_NP] = {1.0, a1, a1 * a1, a1 * a1 * a1};
    const double dA1[BH_NP] = {0.0, 1.0, 2.0 * a1, 3.0 * a1 * a1};
    const double A2[BH_NP] = {1.0, a2, a2 * a2, a2 * a2 * a2};
    // Z[ty][mm][n][o] += (q dA1[mm] E[o] + A1[mm] ES[o]) A2[n]; ty is uniform across the wave
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
      if (tt != ty) continue;
      if (LIN) {
#pragma unroll
        for (int mm = 0; mm < BH_NP; ++mm)
#pragma unroll
          for (int o = 0; o < BH_NO; ++o) {
            const double u = q * dA1[mm] * E[o] + A1[mm] * ES[o];
#pragma unroll
            for (int n = 0; n < BH_NP; ++n) z[tt * 64 + mm * 16 + n * 4 + o] += u * A2[n];
          }
      }
      if (NL) {
        // b of this nucleus' type: a' = a (1 - a) / b, (grad a)' = (1 - 2 a) / b grad a;
        // dL/db += q sum_o rbar^o (grad F_o)'/grad a + W d t^2 sum_o o rbar^{o-1} F_o'
        const double b = T->nuc[I][3];
        const double da1 = a1 * (1.0 - a1) / b, da2 = a2 * (1.0 - a2) / b;
        const double kg = (1.0 - 2.0 * a1) / b;
        const double dA2[BH_NP] = {0.0, 1.0, 2.0 * a2, 3.0 * a2 * a2};
        const double ddA1[BH_NP] = {0.0, 0.0, 2.0, 6.0 * a1};
        double acc = 0.0;
#pragma unroll
        for (int o = 0; o < BH_NO; ++o) {
          double dF = 0.0, dG = 0.0;
#pragma unroll
          for (int mm = 0; mm < BH_NP; ++mm) {
            double g = 0.0, dg = 0.0;
#pragma unroll
            for (int n = 0; n < BH_NP; ++n) {
              g += Cs[tt][mm][n][o] * A2[n];
              dg += Cs[tt][mm][n][o] * dA2[n];
            }
            dg *= da2;
            dF += dA1[mm] * da1 * g + A1[mm] * dg;
            dG += ddA1[mm] * da1 * g + dA1[mm] * dg + kg * dA1[mm] * g;
          }
          acc += q * E[o] * dG + ES[o] * dF;
        }
        znl[1 + tt] += acc;
      }
    }
  }
}

// M tiles exactly as k_grad_pairs (four channels), then the BH per-pair adjoint: LIN the
// linear coefficients (Z and Zee), NL the derivatives with respect to d and the b of each
// nucleus type. For one nucleus type the NL part runs as a launch of its own after the LIN
// one (beside the 64 Z accumulators it spilled ~1 KB per lane; alone it spills 20 bytes)
// and writes only its entries of the partials; for two types the combined form is kept
// (the separate two-type form crashes the device compiler).
template <int NT, bool LIN, bool NL>
__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(1, 1)))
void k_grad_pairs_bh(const double* __restrict__ Pb, long rows_pad, long bp, int n_rows,
                     const double* __restrict__ xi, const double* __restrict__ rho,
                     const double* __restrict__ rhot, const double* __restrict__ w,
                     const double* __restrict__ xyz, long n_g, int n_mu, long b0, long bn,
                     EECoef cf, const BHTable* __restrict__ T, int omax_ee,
                     double* __restrict__ partials) {
  constexpr int NCH = 4;
  __shared__ double Gs[NCH][GK][GT + 1];
  __shared__ double As[GK][GT + 1];
  __shared__ double bxyz[3][GT];
  __shared__ double kxyz[3][GT];
  __shared__ double TB[BH_MAXNUC][4][GT];
  __shared__ double TA[BH_MAXNUC][GT];
  __shared__ double Cs[BH_MAXTYPE][BH_NP][BH_NP][BH_NO];
  __shared__ double red[4][ZS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int nn = T->n_nuc;
  const long bt0 = (long)blockIdx.x * GT;
  const long per = ((n_g + KSEG - 1) / KSEG + GT - 1) / GT * GT;
  const long k_lo = (long)blockIdx.y * per;
  const long k_hi = k_lo + per < n_g ? k_lo + per : n_g;
  if (tid < GT) {
    long b = b0 + bt0 + tid;
    if (b > b0 + bn - 1) b = b0 + bn - 1;
    bxyz[0][tid] = xyz[b];
    bxyz[1][tid] = xyz[n_g + b];
    bxyz[2][tid] = xyz[2 * n_g + b];
  }
  for (int e = tid; e < nn * GT; e += 256) {
    const int I = e / GT, bb = e % GT;
    long b = b0 + bt0 + bb;
    if (b > b0 + bn - 1) b = b0 + bn - 1;
    double v[4];
    bh_nuc_point(T, I, xyz[b], xyz[n_g + b], xyz[2 * n_g + b], v);
#pragma unroll
    for (int q = 0; q < 4; ++q) TB[I][q][bb] = v[q];
  }
  for (int e = tid; e < BH_MAXTYPE * BH_NP * BH_NP * BH_NO; e += 256)
    (&Cs[0][0][0][0])[e] = (&T->csym[0][0][0][0])[e];
  constexpr int NZ = LIN ? NT * 64 : 1, NZE = LIN ? MAXQ + 1 : 1, NZN = NL ? 1 + NT : 1;
  double z[NZ];
#pragma unroll
  for (int k = 0; k < NZ; ++k) z[k] = 0.0;
  double zee[NZE];
#pragma unroll
  for (int k = 0; k < NZE; ++k) zee[k] = 0.0;
  double znl[NZN];
#pragma unroll
  for (int k = 0; k < NZN; ++k) znl[k] = 0.0;

  for (long kc = k_lo; kc < k_hi; kc += GT) {
    __syncthreads();
    if (tid < GT) {
      long g = kc + tid;
      if (g > n_g - 1) g = n_g - 1;
      kxyz[0][tid] = xyz[g];
      kxyz[1][tid] = xyz[n_g + g];
      kxyz[2][tid] = xyz[2 * n_g + g];
    }
    for (int e = tid; e < nn * GT; e += 256) {
      const int I = e / GT, kk = e % GT;
      long g = kc + kk;
      if (g > n_g - 1) g = n_g - 1;
      TA[I][kk] = bh_a(T, I, xyz[g], xyz[n_g + g], xyz[2 * n_g + g]);
    }
    d4 acc[NCH][2][2];
    m_tiles<NCH, NT == 1 && LIN && !NL>(Pb, rows_pad, bp, n_rows, xi, rho, rhot, w, n_g, n_mu, bt0, bn,
                                 kc, k_hi, Gs, As, acc);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int bi = 32 * wm + 16 * i + lk + 4 * r;
          const int kj = 32 * wn + 16 * j + li;
          if (bt0 + bi >= bn || kc + kj >= k_hi) continue;
          double mv[NCH];
#pragma unroll
          for (int c = 0; c < NCH; ++c) mv[c] = acc[c][i][j][r];
          pair_grad_bh<NT, LIN, NL>(cf, T, Cs, nn, TB, bi, TA, kj, bxyz[0][bi] - kxyz[0][kj],
                           bxyz[1][bi] - kxyz[1][kj], bxyz[2][bi] - kxyz[2][kj], mv, z, zee,
                           omax_ee, znl);
        }
  }
  // deterministic block reduction: [NT * 64 Z entries][MAXQ + 1 Zee entries][1 + NT nonlinear]
  __syncthreads();
  constexpr int K0 = LIN ? 0 : NT * 64 + MAXQ + 1;
  constexpr int K1 = NL ? NT * 64 + MAXQ + 1 + 1 + NT : NT * 64 + MAXQ + 1;
#pragma unroll
  for (int k = K0; k < K1; ++k) {
    double v = k < NT * 64 ? z[LIN ? k : 0]
                           : (k < NT * 64 + MAXQ + 1 ? zee[LIN ? k - NT * 64 : 0]
                                                     : znl[NL ? k - NT * 64 - MAXQ - 1 : 0]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wave][k] = v;
  }
  __syncthreads();
  const long blk = (long)blockIdx.y * gridDim.x + blockIdx.x;
  // LIN writes every entry (those past its range as 0); NL alone writes only its own
  for (int k = (LIN ? 0 : K0) + tid; k < (LIN ? ZS : K1); k += 256) {
    const double v = k < K1 ? (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]) : 0.0;
    partials[blk * ZS + k] = v;
  }
}

// dtheta[p] = scale_p (Zsum[i1_p] + Zsum[i2_p]) (i2 < 0: one term)
struct BHParamMap {
  int i1, i2;
  double scale;
};

__global__ void k_bh_params(const double* __restrict__ zsum, const BHParamMap* __restrict__ map,
                            int n, double* __restrict__ out) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= n) return;
  const BHParamMap q = map[p];
  out[p] = q.scale * (zsum[q.i1] + (q.i2 >= 0 ? zsum[q.i2] : 0.0));
}

__global__ void k_sum_partials(const double* __restrict__ partials, long nblk, int n, int stride,
                               double* __restrict__ out) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (long b = 0; b < nblk; ++b) s += partials[b * stride + k];
  out[k] = s;
}

__global__ void k_sym(const double* __restrict__ a, long n, double* __restrict__ s) {
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= n * n) return;
  long i = t / n, j = t % n;
  s[t] = a[t] + a[j * n + i];
}

__global__ void k_gather_G2(const double* __restrict__ rho, const long* __restrict__ piv, int n_mu,
                            double* __restrict__ G) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n_mu) G[i] = rho[piv[i]];
}

__global__ void k_fill_rows(double* __restrict__ Pb, long rows_pad, long bp, int nch, int n_mu,
                            long b0, long bn, const double* __restrict__ gfield, long n_g) {
  // rho row: field cotangent (channels x, y, z), 0 for the other channels; rhot row: 0
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= bn) return;
  for (int c = 0; c < nch; ++c) {
    Pb[((long)c * rows_pad + n_mu) * bp + t] = (c < 3 && gfield) ? gfield[c * n_g + b0 + t] : 0.0;
    Pb[((long)c * rows_pad + n_mu + 1) * bp + t] = 0.0;
  }
}

// D1 term: Pbar^c[nu][g] += Pd[nu][g] H_c(g); Pbar^c[rhot row][g] = sum_nu Pd[nu][g] F^c[nu][g]
__global__ void k_d1_terms(double* __restrict__ Pb, const double* __restrict__ F,
                           const double* __restrict__ Pd, long rows_pad, long bp, int n_mu,
                           long bn) {
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= bn) return;
  for (int c = 0; c < 3; ++c) {
    const double H = F[((long)c * rows_pad + n_mu + 1) * bp + t];
    double hb = 0.0;
    for (int nu = 0; nu < n_mu; ++nu) {
      const double p = Pd[(long)nu * bp + t];
      Pb[((long)c * rows_pad + nu) * bp + t] += p * H;
      hb += p * F[((long)c * rows_pad + nu) * bp + t];
    }
    Pb[((long)c * rows_pad + n_mu + 1) * bp + t] = hb;
  }
}

__global__ void k_mul_vec(const double* __restrict__ a, const double* __restrict__ b, long n,
                          double* __restrict__ out) {
  long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}

struct GradLayout {
  long* piv; double* G; double* rhot; double* wt; double* F; double* Pb; double* Pd; double* S4;
  double* partials; BHTable* bh; double* zsum; BHParamMap* pmap;
  long bp; long rows_pad; int nsb; int nch; long nblk;
};

static GradLayout layout_grad(Arena& ar, int64_t n_g, int n_mu, int n_params, uint32_t flags) {
  GradLayout L;
  L.nch = (flags & 1) ? 5 : 4;               // bit 0: Laplacian cotangent present
  L.bp = n_g < GSUPER ? ((n_g + 63) / 64) * 64 : GSUPER;
  L.rows_pad = ((n_mu + 2 + 63) / 64) * 64;
  L.nsb = (int)cdiv(n_g, L.bp);
  L.nblk = (long)cdiv(L.bp, GT) * KSEG;
  L.piv = ar.take<long>(n_mu);
  L.G = ar.take<double>(n_mu);
  L.rhot = ar.take<double>(n_g);
  L.wt = ar.take<double>(n_g);
  L.F = ar.take<double>(4 * (size_t)L.rows_pad * L.bp);
  L.Pb = ar.take<double>((size_t)L.nch * L.rows_pad * L.bp);
  L.Pd = ar.take<double>((size_t)n_mu * L.bp);
  L.S4 = ar.take<double>((size_t)n_mu * n_mu);
  // per-block partial sums; the stride fits the BH parameter table (the EE form uses MAXQ)
  L.partials = ar.take<double>((size_t)L.nsb * L.nblk * ZS);
  L.bh = ar.take<BHTable>(1);
  L.zsum = ar.take<double>(ZS);
  L.pmap = ar.take<BHParamMap>(n_params > 0 ? n_params : 1);
  return L;
}

size_t ws_grad(int64_t n_g, int n_mu, int n_params, uint32_t flags) {
  Arena ar(nullptr, 0);
  layout_grad(ar, n_g, n_mu, n_params, flags);
  return ar.used;
}

}  // namespace xtc

using namespace xtc;

extern "C" xtc_status xtc_grad(const xtc_grid* grid, const xtc_correlator* corr, int32_t n_mu,
                               const double* xi, const double* xigrad, const double* rho,
                               const int64_t* pivots, int64_t bra_begin, int64_t bra_end,
                               const double* gu1, const double* gu3,
                               const double* gulap, const double* gD1, const double* gD4,
                               const double* gfield, double* dtheta, double* dd, void* ws,
                               size_t ws_bytes, void* stream) {
  XTC_REQUIRE(grid && corr && xi && rho && pivots && dtheta, "xtc_grad: null argument");
  XTC_REQUIRE(grid->n_g > 0 && grid->xyz && grid->w, "xtc_grad: empty grid");
  XTC_REQUIRE(bra_begin >= 0 && bra_begin < bra_end && bra_end <= grid->n_g,
              "xtc_grad: bra range must be non-empty and inside the grid");
  XTC_REQUIRE(n_mu > 0 && n_mu <= grid->n_g, "xtc_grad: bad n_mu");
  XTC_REQUIRE(!gu1 || xigrad, "xtc_grad: the u1 cotangent needs xigrad");
  XTC_REQUIRE(corr->n_terms > 0 && corr->mno && corr->c && corr->d > 0.0,
              "xtc_grad: bad correlator");
  XTC_REQUIRE(corr->form == XTC_U_EE || corr->form == XTC_U_BH, "xtc_grad: unknown correlator form");
  const bool bh = corr->form == XTC_U_BH;
  XTC_REQUIRE(bh || corr->n_terms <= MAXQ, "xtc_grad: too many EE terms");
  for (int m = 0; m < n_mu; ++m)
    XTC_REQUIRE(pivots[m] >= 0 && pivots[m] < grid->n_g, "xtc_grad: pivot index out of range");
  if (bh && gulap) {
    set_error("xtc_grad: the Laplacian channel is defined for the EE form only");
    return XTC_ERR_UNSUPPORTED;
  }

  EECoef cf;
  BHTable bt;
  int omax_ee = 0;
  const int n_params = bh ? corr->n_types * corr->n_terms : corr->n_terms;
  std::vector<BHParamMap> pmap;
  if (bh) {
    XTC_TRY(bh_build(corr, &bt, &cf));
    omax_ee = cf.n1;
    // parameter p = type * n_terms + k -> entries of the summed [types x 64 Z][Zee] table
    const int nz = bt.n_types * 64;
    for (int t = 0; t < corr->n_types; ++t)
      for (int k = 0; k < corr->n_terms; ++k) {
        const int m = corr->mno[3 * k], n = corr->mno[3 * k + 1], o = corr->mno[3 * k + 2];
        BHParamMap q;
        if (m == 0 && n == 0) {
          q.i1 = nz + o;
          q.i2 = -1;
          q.scale = 2.0 * bt.n_of_type[t];
        } else {
          q.i1 = t * 64 + m * 16 + n * 4 + o;
          q.i2 = t * 64 + n * 16 + m * 4 + o;
          q.scale = 1.0;
        }
        pmap.push_back(q);
      }
  } else {
    XTC_TRY(ee_coefficients(corr, &cf));
  }
  GradBasis gb{};   // EE form only (at most MAXQ terms)
  gb.d = corr->d;
  if (!bh) {
    gb.n = corr->n_terms;
    gb.want_d = dd ? 1 : 0;
    for (int k = 0; k < gb.n; ++k) {
      gb.o[k] = corr->mno[3 * k + 2];
      gb.c[k] = corr->c[k];
      if (gb.o[k] > gb.omax) gb.omax = gb.o[k];
    }
  }
  hipStream_t st = as_stream(stream);
  const long n_g = grid->n_g;
  Arena ar(ws, ws_bytes);
  GradLayout L = layout_grad(ar, n_g, n_mu, n_params, gulap ? 1u : 0u);
  XTC_TRY(need_ws(ar));
  XTC_TRY(check_weights(grid, ws, ws_bytes, st, "xtc_grad"));
  if (bh) {
    XTC_HIP(hipMemcpyAsync(L.bh, &bt, sizeof(BHTable), hipMemcpyHostToDevice, st));
    XTC_HIP(hipMemcpyAsync(L.pmap, pmap.data(), sizeof(BHParamMap) * pmap.size(),
                           hipMemcpyHostToDevice, st));
  }
  size_t tk = timing_begin(TM_GRAD, st);
  XTC_HIP(hipMemcpyAsync(L.piv, pivots, sizeof(long) * n_mu, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_gather_G2, dim3(cdiv(n_mu, 256)), dim3(256), 0, st, rho, (const long*)L.piv,
                     n_mu, L.G);
  {
    GemmArgs g{};   // rhot = G^T xi
    g.M = 1; g.N = n_g; g.K = n_mu;
    g.A = L.G; g.a_sm = 1; g.a_sk = 1;
    g.B = xi; g.b_sk = n_g; g.b_sn = 1;
    g.C = L.rhot; g.c_sm = n_g; g.c_sn = 1;
    XTC_TRY(gemm_f64(g, st));
  }
  hipLaunchKernelGGL(k_mul_vec, dim3(cdiv(n_g, 256)), dim3(256), 0, st, grid->w,
                     (const double*)L.rhot, n_g, L.wt);
  XTC_CHECK_LAUNCH();
  if (gD4) {
    hipLaunchKernelGGL(k_sym, dim3(cdiv((long)n_mu * n_mu, 256)), dim3(256), 0, st, gD4, (long)n_mu,
                       L.S4);
    XTC_CHECK_LAUNCH();
  }
  const bool need_fwd = gD1 || gD4;
  Stage1Args s1{grid->xyz, grid->w, xi, rho, L.rhot, n_g, n_mu, 0, 0, L.F, L.rows_pad, L.bp, 4};
  if (bh) s1.bh = L.bh;
  // bra super-blocks of the range; the ket sums always cover the whole grid
  const int nsb = (int)cdiv(bra_end - bra_begin, L.bp);
  for (int sb = 0; sb < nsb; ++sb) {
    const long b0 = bra_begin + (long)sb * L.bp;
    const long bn = (bra_end - b0) < L.bp ? (bra_end - b0) : L.bp;
    if (need_fwd) {
      s1.b0 = b0;
      s1.bn = bn;
      XTC_TRY(stage1_f64(s1, cf, st));
    }
    // Pbar for rows 0..n_mu-1 of every channel
    auto tn = [&](const double* cot, const double* B, long b_sk, const double* sn, double* C,
                  double beta) {
      GemmArgs g{};   // C[nu][g] = sn[g] sum_mu cot[mu][nu] B[mu][g] + beta C
      g.M = n_mu; g.N = bn; g.K = n_mu;
      g.A = cot; g.a_sm = 1; g.a_sk = n_mu;
      g.B = B; g.b_sk = b_sk; g.b_sn = 1;
      g.sn = sn;
      g.C = C; g.c_sm = L.bp; g.c_sn = 1;
      g.beta = beta;
      return gemm_f64(g, st);
    };
    const double* wb = grid->w + b0;
    for (int c = 0; c < L.nch; ++c) {
      double* Pc = L.Pb + (long)c * L.rows_pad * L.bp;
      bool have = false;
      const double* cot = nullptr;
      const double* B = nullptr;
      if (c < 3 && gu1) { cot = gu1 + (long)c * n_mu * n_mu; B = xigrad + (long)c * n_mu * n_g + b0; }
      if (c == 3 && gu3) { cot = gu3; B = xi + b0; }
      if (c == 4 && gulap) { cot = gulap; B = xi + b0; }
      if (cot) {
        XTC_TRY(tn(cot, B, n_g, wb, Pc, 0.0));
        have = true;
      }
      if (c < 3 && gD4) {
        GemmArgs g{};   // += wt (S4 F^c)
        g.M = n_mu; g.N = bn; g.K = n_mu;
        g.A = L.S4; g.a_sm = n_mu; g.a_sk = 1;
        g.B = L.F + (long)c * L.rows_pad * L.bp; g.b_sk = L.bp; g.b_sn = 1;
        g.sn = L.wt + b0;
        g.C = Pc; g.c_sm = L.bp; g.c_sn = 1;
        g.beta = have ? 1.0 : 0.0;
        XTC_TRY(gemm_f64(g, st));
        have = true;
      }
      if (!have) XTC_HIP(hipMemsetAsync(Pc, 0, sizeof(double) * L.rows_pad * L.bp, st));
    }
    hipLaunchKernelGGL(k_fill_rows, dim3(cdiv(bn, 256)), dim3(256), 0, st, L.Pb, L.rows_pad, L.bp,
                       L.nch, n_mu, b0, bn, gfield, n_g);
    XTC_CHECK_LAUNCH();
    if (gD1) {
      XTC_TRY(tn(gD1, xi + b0, n_g, wb, L.Pd, 0.0));   // Pd = w (gD1^T xi)
      hipLaunchKernelGGL(k_d1_terms, dim3(cdiv(bn, 256)), dim3(256), 0, st, L.Pb,
                         (const double*)L.F, (const double*)L.Pd, L.rows_pad, L.bp, n_mu, bn);
      XTC_CHECK_LAUNCH();
    }
    dim3 gridp(cdiv(bn, GT), KSEG);
    const int stride = bh ? ZS : MAXQ + 1;
    double* part = L.partials + (long)sb * L.nblk * stride;
    if (bh) {
#define XTC_LAUNCH_BH(NTV, LINV, NLV)                                                           \
  hipLaunchKernelGGL((k_grad_pairs_bh<NTV, LINV, NLV>), gridp, dim3(256), 0, st,                 \
                     (const double*)L.Pb, L.rows_pad, L.bp, n_mu + 2, xi, rho,                   \
                     (const double*)L.rhot, grid->w, grid->xyz, n_g, n_mu, b0, bn, cf,           \
                     (const BHTable*)L.bh, omax_ee, part)
      if (bt.n_types == 1) {
        XTC_LAUNCH_BH(1, true, false);
        if (dd) {   // the nonlinear parameters in a launch of their own (after the linear one)
          XTC_CHECK_LAUNCH();
          XTC_LAUNCH_BH(1, false, true);
        }
      } else if (!dd) {
        XTC_LAUNCH_BH(2, true, false);
      } else {
        XTC_LAUNCH_BH(2, true, true);
      }
#undef XTC_LAUNCH_BH
    }
    else if (L.nch == 4)
      hipLaunchKernelGGL(k_grad_pairs<4>, gridp, dim3(256), 0, st, (const double*)L.Pb, L.rows_pad,
                         L.bp, n_mu + 2, xi, rho, (const double*)L.rhot, grid->w, grid->xyz, n_g,
                         n_mu, b0, bn, cf, gb, part);
    else
      hipLaunchKernelGGL(k_grad_pairs<5>, gridp, dim3(256), 0, st, (const double*)L.Pb, L.rows_pad,
                         L.bp, n_mu + 2, xi, rho, (const double*)L.rhot, grid->w, grid->xyz, n_g,
                         n_mu, b0, bn, cf, gb, part);
    XTC_CHECK_LAUNCH();
    // unused block slots of a short last super-block stay zero
    if ((long)gridp.x * KSEG < L.nblk)
      XTC_HIP(hipMemsetAsync(part + (long)gridp.x * KSEG * stride, 0,
                             sizeof(double) * (L.nblk - (long)gridp.x * KSEG) * stride, st));
  }
  if (bh) {
    hipLaunchKernelGGL(k_sum_partials, dim3(cdiv(ZS, 256)), dim3(256), 0, st,
                       (const double*)L.partials, (long)nsb * L.nblk, ZS, ZS, L.zsum);
    XTC_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_bh_params, dim3(cdiv(n_params, 256)), dim3(256), 0, st,
                       (const double*)L.zsum, (const BHParamMap*)L.pmap, n_params, dtheta);
    if (dd)
      XTC_HIP(hipMemcpyAsync(dd, L.zsum + bt.n_types * 64 + MAXQ + 1,
                             sizeof(double) * (1 + bt.n_types), hipMemcpyDeviceToDevice, st));
  } else {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, st, (const double*)L.partials,
                       (long)nsb * L.nblk, gb.n + gb.want_d, MAXQ + 1, L.zsum);
    XTC_CHECK_LAUNCH();
    XTC_HIP(hipMemcpyAsync(dtheta, L.zsum, sizeof(double) * gb.n, hipMemcpyDeviceToDevice, st));
    if (dd) XTC_HIP(hipMemcpyAsync(dd, L.zsum + gb.n, sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  XTC_CHECK_LAUNCH();
  timing_end(tk, st);
  return XTC_OK;
}
