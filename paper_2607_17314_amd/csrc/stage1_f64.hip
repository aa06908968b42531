// Stage 1 of the grid-pair contraction in FP64 (K-kernel section: the
// doubly-blocked grid sums, each auxiliary vector used once per grid pair):
//   panel[ch][row][g] = sum_g' A[row][g'] K_ch(g, g'),  A = [w xi ; w rho ; w rhot]
// with the kernel channels K = (d_x u, d_y u, d_z u, |grad u|^2 [, lap u])
// generated in registers for every (bra g, ket g') pair and never written to
// HBM.
//
// Workgroup tile: 64 rows x 64 bra points, 256 threads = 4 waves in 2 x 2,
// each wave 32 rows x 32 bra points per channel. Ket chunks of 16 points:
//   * each thread loads 4 elements of the 64 x 16 A tile (scaled by w) and
//     generates the NCH channels of 4 (bra, ket) pairs in FP64,
//   * both go to LDS, then every wave runs 4 k-steps of
//     v_mfma_f64_16x16x4f64 per channel and sub-tile.
// The kernel tile is generated once per workgroup and reused by all 64 rows.
#include "bh.hpp"
#include "stage1_split.hpp"
#include "timing.hpp"

namespace xtc {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double horner(const double* q, int n, double x) {
  double r = 0.0;
  for (int j = n - 1; j >= 0; --j) r = r * x + q[j];
  return r;
}

template <int NCH>
__device__ __forceinline__ void ee_channels(const EECoef& cf, double dx, double dy, double dz,
                                            double* out) {
  const double r2 = dx * dx + dy * dy + dz * dz;
  const double r = sqrt(r2);
  const double t = 1.0 / (1.0 + cf.d * r);
  const double e = cf.d * r * t;
  const double t2 = t * t, t3 = t2 * t;
  const double p1 = horner(cf.q1, cf.n1, e);
  const double up = cf.d * t2 * p1;
  double f = cf.d * cf.d * t3 * horner(cf.q2, cf.n2, e);
  if (cf.c1 != 0.0 && r > 0.0) f += cf.c1 * cf.d * t2 / r;
  out[0] = f * dx;
  out[1] = f * dy;
  out[2] = f * dz;
  out[3] = up * up;
  if (NCH > 4) {
    double upp = cf.d * cf.d * t2 * t2 * horner(cf.q3, cf.n3, e) - 2.0 * cf.d * cf.d * t3 * p1;
    if (cf.c1 != 0.0 && r == 0.0) upp += 2.0 * cf.d * cf.d * t3 * cf.c1;
    out[NCH - 1] = upp + 2.0 * f;
  }
}

template <int NCH>
__global__ __launch_bounds__(256) void k_stage1_f64(const double* __restrict__ xyz,
                                                    const double* __restrict__ w,
                                                    const double* __restrict__ xi,
                                                    const double* __restrict__ rho,
                                                    const double* __restrict__ rhot, long n_g,
                                                    int n_mu, long b0, long bn, EECoef cf,
                                                    double* __restrict__ panel, long rows_pad,
                                                    long bp) {
  constexpr int KC = 16;
  __shared__ double As[64][KC + 1];
  __shared__ double Bs[NCH][KC][65];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long m0 = (long)blockIdx.y * 64;
  const long nb0 = (long)blockIdx.x * 64;
  const int gb = tid & 63;
  const int gk = tid >> 6;
  long bra = b0 + nb0 + gb;
  if (bra > b0 + bn - 1) bra = b0 + bn - 1;
  const double xb = xyz[bra], yb = xyz[n_g + bra], zb = xyz[2 * n_g + bra];

  d4 acc[NCH][2][2];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[c][i][j] = (d4){0.0, 0.0, 0.0, 0.0};

  const int li = lane & 15, lk = lane >> 4;
  for (long k0 = 0; k0 < n_g; k0 += KC) {
    double ra[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = tid + 256 * j;
      const int row = e >> 4, kk = e & 15;
      const long g = k0 + kk, rr = m0 + row;
      double v = 0.0;
      if (g < n_g && rr <= n_mu + 1)
        v = w[g] * (rr < n_mu ? xi[rr * n_g + g] : (rr == n_mu ? rho[g] : rhot[g]));
      ra[j] = v;
    }
    double ch[4][NCH];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      long g = k0 + 4 * gk + q;
      if (g > n_g - 1) g = n_g - 1;
      ee_channels<NCH>(cf, xb - xyz[g], yb - xyz[n_g + g], zb - xyz[2 * n_g + g], ch[q]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = tid + 256 * j;
      As[e >> 4][e & 15] = ra[j];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < NCH; ++c) Bs[c][4 * gk + q][gb] = ch[q][c];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const double a0 = As[32 * wm + li][4 * s + lk];
      const double a1 = As[32 * wm + 16 + li][4 * s + lk];
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const double bb0 = Bs[c][4 * s + lk][32 * wn + li];
        const double bb1 = Bs[c][4 * s + lk][32 * wn + 16 + li];
        acc[c][0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bb0, acc[c][0][0], 0, 0, 0);
        acc[c][0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bb1, acc[c][0][1], 0, 0, 0);
        acc[c][1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bb0, acc[c][1][0], 0, 0, 0);
        acc[c][1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bb1, acc[c][1][1], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const long row = m0 + 32 * wm + 16 * i + lk + 4 * r;   // D[(l/16) + 4r][l%16]
          const long col = nb0 + 32 * wn + 16 * j + li;
          if (row <= n_mu + 1 && col < bn) panel[((long)c * rows_pad + row) * bp + col] = acc[c][i][j][r];
        }
}

// BH form (four channels): per pair, from the workgroup's LDS tables of
//   TB[I][a, grad a][bra]  (the 64 bra points, filled once) and
//   TK[ket][I][o][m] = gamma_{I,o,m}(ket)  (per ket chunk),
// the nuclear sums F_o and grad F_o, then N, S and the channels (bh_pair_channels).

// Same MFMA structure as k_stage1_f64 (four channels), with the BH tables in LDS and RT
// rows per workgroup (64 or 128): the generated pair channels, whose nuclear sums dominate
// the work, are reused by all RT rows, so RT = 128 halves the generation per row. Each
// wave holds RT/2 rows x 32 bra points per channel.
constexpr int BH_ROW_TILE = 128;

template <int RT>
__global__ __launch_bounds__(256) void k_stage1_f64_bh(
    const double* __restrict__ xyz, const double* __restrict__ w, const double* __restrict__ xi,
    const double* __restrict__ rho, const double* __restrict__ rhot, long n_g, int n_mu, long b0,
    long bn, EECoef cf, const BHTable* __restrict__ T, double* __restrict__ panel, long rows_pad,
    long bp) {
  constexpr int KC = 16, NCH = 4;
  constexpr int MI = RT / 32;            // 16-row sub-tiles per wave
  constexpr int NA = RT * KC / 256;      // A elements loaded per thread per chunk
  __shared__ double As[RT][KC + 1];
  __shared__ double Bs[NCH][KC][65];
  __shared__ double TB[BH_MAXNUC][4][64];
  __shared__ double TK[KC][BH_MAXNUC][BH_NO][BH_NP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long m0 = (long)blockIdx.y * RT;
  const long nb0 = (long)blockIdx.x * 64;
  const int gb = tid & 63;
  const int gk = tid >> 6;
  const int nn = T->n_nuc;
  long bra = b0 + nb0 + gb;
  if (bra > b0 + bn - 1) bra = b0 + bn - 1;
  const double xb = xyz[bra], yb = xyz[n_g + bra], zb = xyz[2 * n_g + bra];
  for (int e = tid; e < nn * 64; e += 256) {
    const int I = e / 64, bb = e % 64;
    long b = b0 + nb0 + bb;
    if (b > b0 + bn - 1) b = b0 + bn - 1;
    double v[4];
    bh_nuc_point(T, I, xyz[b], xyz[n_g + b], xyz[2 * n_g + b], v);
#pragma unroll
    for (int q = 0; q < 4; ++q) TB[I][q][bb] = v[q];
  }

  d4 acc[NCH][MI][2];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[c][i][j] = (d4){0.0, 0.0, 0.0, 0.0};

  const int li = lane & 15, lk = lane >> 4;
  for (long k0 = 0; k0 < n_g; k0 += KC) {
    double ra[NA];
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int e = tid + 256 * j;
      const int row = e >> 4, kk = e & 15;
      const long g = k0 + kk, rr = m0 + row;
      double v = 0.0;
      if (g < n_g && rr <= n_mu + 1)
        v = w[g] * (rr < n_mu ? xi[rr * n_g + g] : (rr == n_mu ? rho[g] : rhot[g]));
      ra[j] = v;
    }
    // ket tables of this chunk (the previous chunk's generation has passed the
    // barrier before its MFMA phase, so TK is free)
    for (int e = tid; e < KC * nn; e += 256) {
      const int kk = e / nn, I = e % nn;
      long g = k0 + kk;
      if (g > n_g - 1) g = n_g - 1;
      bh_ket_gamma(T, I, xyz[g], xyz[n_g + g], xyz[2 * n_g + g], TK[kk][I]);
    }
    __syncthreads();
    double ch[4][NCH];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = 4 * gk + q;
      long g = k0 + kk;
      if (g > n_g - 1) g = n_g - 1;
      bh_pair_channels<64>(cf, nn, TB, gb, TK[kk], xb - xyz[g], yb - xyz[n_g + g],
                           zb - xyz[2 * n_g + g], ch[q]);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NA; ++j) {
      const int e = tid + 256 * j;
      As[e >> 4][e & 15] = ra[j];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < NCH; ++c) Bs[c][4 * gk + q][gb] = ch[q][c];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      double av[MI];
#pragma unroll
      for (int i = 0; i < MI; ++i) av[i] = As[(RT / 2) * wm + 16 * i + li][4 * s + lk];
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const double bb0 = Bs[c][4 * s + lk][32 * wn + li];
        const double bb1 = Bs[c][4 * s + lk][32 * wn + 16 + li];
#pragma unroll
        for (int i = 0; i < MI; ++i) {
          acc[c][i][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bb0, acc[c][i][0], 0, 0, 0);
          acc[c][i][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bb1, acc[c][i][1], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const long row = m0 + (RT / 2) * wm + 16 * i + lk + 4 * r;   // D[(l/16) + 4r][l%16]
          const long col = nb0 + 32 * wn + 16 * j + li;
          if (row <= n_mu + 1 && col < bn) panel[((long)c * rows_pad + row) * bp + col] = acc[c][i][j][r];
        }
}

// BH form with its pair values made beforehand (k_bh_pairs_f64, FP64, once per pair and
// ket launch instead of once per row tile): the FP64 products of k_stage1_f64 over the
// 16-ket steps of one launch, kets [kbeg, kbeg + 16 nsteps), the B tile read from the buffer
// (pv64[tile][step][q][c][gk][gb], the pair (bra gb, ket 4 gk + q)) and the next step's A
// and B loaded into registers while the current step's MFMAs run. first: the panel is
// written, else added to.
__global__ __launch_bounds__(256) void k_stage1_f64_pv(const double* __restrict__ w,
                                                       const double* __restrict__ xi,
                                                       const double* __restrict__ rho,
                                                       const double* __restrict__ rhot, long n_g,
                                                       int n_mu, long bn,
                                                       const double* __restrict__ pv64,
                                                       long nsteps, long kbeg,
                                                       double* __restrict__ panel, long rows_pad,
                                                       long bp, int first) {
  constexpr int KC = 16, NCH = 4;
  __shared__ double As[64][KC + 1];
  __shared__ double Bs[NCH][KC][65];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long m0 = (long)blockIdx.y * 64;
  const long nb0 = (long)blockIdx.x * 64;
  const int gb = tid & 63, gk = tid >> 6;
  const double* pb = pv64 + (long)blockIdx.x * nsteps * 4096 + gk * 64 + gb;
  d4 acc[NCH][2][2];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[c][i][j] = (d4){0.0, 0.0, 0.0, 0.0};
  double ra[4], ch[4][NCH];
  auto load = [&](long sidx) {
    const long k0 = kbeg + 16 * sidx;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = tid + 256 * j;
      const int row = e >> 4, kk = e & 15;
      const long g = k0 + kk, rr = m0 + row;
      double v = 0.0;
      if (g < n_g && rr <= n_mu + 1)
        v = w[g] * (rr < n_mu ? xi[rr * n_g + g] : (rr == n_mu ? rho[g] : rhot[g]));
      ra[j] = v;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < NCH; ++c) ch[q][c] = pb[sidx * 4096 + (q * 4 + c) * 256];
  };
  load(0);
  const int li = lane & 15, lk = lane >> 4;
  for (long sidx = 0; sidx < nsteps; ++sidx) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int e = tid + 256 * j;
      As[e >> 4][e & 15] = ra[j];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int c = 0; c < NCH; ++c) Bs[c][4 * gk + q][gb] = ch[q][c];
    __builtin_amdgcn_s_waitcnt(0xc07f);   // the tile's LDS stores done before the barrier
    __syncthreads();
    if (sidx + 1 < nsteps) load(sidx + 1);
    __builtin_amdgcn_sched_barrier(0);   // the loads stay ahead of the MFMAs
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const double a0 = As[32 * wm + li][4 * s + lk];
      const double a1 = As[32 * wm + 16 + li][4 * s + lk];
#pragma unroll
      for (int c = 0; c < NCH; ++c) {
        const double bb0 = Bs[c][4 * s + lk][32 * wn + li];
        const double bb1 = Bs[c][4 * s + lk][32 * wn + 16 + li];
        acc[c][0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bb0, acc[c][0][0], 0, 0, 0);
        acc[c][0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, bb1, acc[c][0][1], 0, 0, 0);
        acc[c][1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bb0, acc[c][1][0], 0, 0, 0);
        acc[c][1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, bb1, acc[c][1][1], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const long row = m0 + 32 * wm + 16 * i + lk + 4 * r;   // D[(l/16) + 4r][l%16]
          const long col = nb0 + 32 * wn + 16 * j + li;
          if (row <= n_mu + 1 && col < bn) {
            double* p = panel + ((long)c * rows_pad + row) * bp + col;
            *p = first ? acc[c][i][j][r] : *p + acc[c][i][j][r];
          }
        }
}

xtc_status stage1_f64(const Stage1Args& a, const EECoef& cf, hipStream_t st) {
  if (a.bh && a.pv64) {
    XTC_REQUIRE(a.nch == 4, "BH correlator: the Laplacian channel is defined for the EE form only");
    const long nch = (a.n_g + SKC - 1) / SKC;
    for (long c0 = 0; c0 < nch; c0 += SMED) {
      const long nloc = SMED < nch - c0 ? SMED : nch - c0;
      size_t tk = timing_begin(TM_S1_PAIRS, st);
      XTC_TRY(bh_pair_values_f64(a, cf, c0, nloc, st));
      timing_end(tk, st);
      tk = timing_begin(TM_S1_KERNEL, st);
      hipLaunchKernelGGL(k_stage1_f64_pv, dim3(cdiv(a.bn, 64), cdiv(a.n_mu + 2, 64)), dim3(256), 0,
                         st, a.w, a.xi, a.rho, a.rhot, a.n_g, a.n_mu, a.bn, (const double*)a.pv64,
                         nloc * 8, c0 * SKC, a.panel, a.rows_pad, a.bp, c0 == 0 ? 1 : 0);
      timing_end(tk, st);
      XTC_CHECK_LAUNCH();
    }
    return XTC_OK;
  }
  dim3 grid(cdiv(a.bn, 64), cdiv(a.n_mu + 2, 64));
  const size_t tk = timing_begin(TM_S1_KERNEL, st);
  if (a.bh) {
    XTC_REQUIRE(a.nch == 4, "BH correlator: the Laplacian channel is defined for the EE form only");
    dim3 gbh(cdiv(a.bn, 64), cdiv(a.n_mu + 2, BH_ROW_TILE));
    hipLaunchKernelGGL(k_stage1_f64_bh<BH_ROW_TILE>, gbh, dim3(256), 0, st, a.xyz, a.w, a.xi, a.rho,
                       a.rhot, a.n_g, a.n_mu, a.b0, a.bn, cf, a.bh, a.panel, a.rows_pad, a.bp);
  } else if (a.nch == 4)
    hipLaunchKernelGGL(k_stage1_f64<4>, grid, dim3(256), 0, st, a.xyz, a.w, a.xi, a.rho, a.rhot, a.n_g,
                       a.n_mu, a.b0, a.bn, cf, a.panel, a.rows_pad, a.bp);
  else
    hipLaunchKernelGGL(k_stage1_f64<5>, grid, dim3(256), 0, st, a.xyz, a.w, a.xi, a.rho, a.rhot, a.n_g,
                       a.n_mu, a.b0, a.bn, cf, a.panel, a.rows_pad, a.bp);
  timing_end(tk, st);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

}  // namespace xtc
