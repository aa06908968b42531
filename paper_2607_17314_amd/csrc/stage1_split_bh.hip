// Stage 1 of the grid-pair contraction for the multi-centre (BH) correlator in split
// precision (K-kernel section, eqs. K1-isdf and K3-isdf, with the kernel of eq. bh-u):
//   panel[ch][row][g] = sum_g' A[row][g'] K_ch(g, g'),  A = [w xi ; w rho ; w rhot].
// The EE pair kernel makes its kernel values in registers beside the MFMAs (~50 FP32
// operations per pair). The BH values cost ~40 FP64 operations per nucleus and pair (the
// nuclear sums F_o and grad F_o), which beside the MFMAs of one 256-row tile would be made
// again for every row tile. Here they are made once per pair and launch:
//   1. k_bh_pairs (vector FP64): the four channels of every (bra, ket) pair of a bra
//      tile and a ket chunk, scaled by a power of two and split into FP16 (hi, lo), stored
//      in the MFMA B-fragment order of the split pair kernel; the same FP64 values feed
//      the two density rows (rows n_mu and n_mu + 1), summed in FP64 per bra point;
//   2. k_stage1_split_pv: the split products A_hi K_hi + A_hi K_lo + A_lo K_hi with
//      v_mfma_f32_32x32x16_f16, the pair values streamed from the buffer through LDS
//      (double-buffered, one ket chunk ahead), FP32 accumulation over a pair of chunks,
//      an FP32 medium sum over the launch, FP64 in the panel, scales removed exactly.
// The A operand and its per-row exponents are the split operand of the EE path. The FP64
// path of the BH form takes its pair values from k_bh_pairs_f64 below (the same tables and
// sums, the values stored unscaled in FP64 for k_stage1_f64_pv).
#include <algorithm>
#include <type_traits>
#include "bh.hpp"
#include "stage1_split.hpp"
#include "timing.hpp"

namespace xtc {

// The kernel's own LDS writes completed (lgkmcnt(0)) before a barrier: the barrier alone is
// not relied on to order them with other waves' reads that follow it.
#define XTC_LDS_DONE() __builtin_amdgcn_s_waitcnt(0xc07f)
#define XTC_FENCE() __builtin_amdgcn_sched_barrier(0)

constexpr int GCH = 8;                // ket chunks per generation workgroup
constexpr int PV_CHUNK = 8 * 4 * 2 * 64;   // h8 per (bra tile, ket chunk): [ks][ch][hl][lane]

size_t bh_split_scratch_bytes(long bp) {
  return (size_t)cdiv(bp, SB) * SMED * PV_CHUNK * sizeof(h8) + 256;
}

// Channel exponents: |grad_1 u| <= |N| + |S| with a, rbar in [0, 1), |grad a| <= b, t <= 1:
//   |F_o| <= sum_I sum_{m,n} |csym[m][n][o]|,  |grad F_o| <= sum_I b_I sum_{m,n} m |csym[m][n][o]|,
//   |N| <= sum_o |grad F_o|,  |S| <= d (sum_o o |F_o| + sum_j |q1_j|).
// 2^eg bounds the gradient channels and 2^es the squared norm below 2^14, as on the EE path.
static void bh_split_exponents(const BHTable& T, const EECoef& cf, int* eg, int* es) {
  double Fb[BH_NO] = {}, Gb[BH_NO] = {};
  for (int I = 0; I < T.n_nuc; ++I) {
    const int t = T.type[I];
    for (int o = 0; o < BH_NO; ++o)
      for (int m = 0; m < BH_NP; ++m)
        for (int n = 0; n < BH_NP; ++n) {
          const double c = fabs(T.csym[t][m][n][o]);
          Fb[o] += c;
          Gb[o] += m * c * T.nuc[I][3];
        }
  }
  double N = 0.0, S = 0.0;
  for (int o = 0; o < BH_NO; ++o) {
    N += Gb[o];
    S += o * Fb[o];
  }
  for (int j = 0; j < cf.n1; ++j) S += fabs(cf.q1[j]);
  S *= cf.d;
  int ex = 0;
  if (N + S > 0.0) frexp(N + S, &ex);   // N + S < 2^ex
  *eg = 14 - ex;
  *es = 14 - 2 * ex;
}

// gamma_{I,o,m} of one ket point (see bh.hpp) from the workgroup's LDS copies of the
// nuclei (x, y, z, b) and of csym
__device__ __forceinline__ void ket_gamma_lds(const double (*NU)[4], const int* __restrict__ ty,
                                              const double* CS, int I, double x, double y,
                                              double z, double* out) {
  const double dx = x - NU[I][0], dy = y - NU[I][1], dz = z - NU[I][2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double a = NU[I][3] * r / (1.0 + NU[I][3] * r);
  const double A2[BH_NP] = {1.0, a, a * a, a * a * a};
  const double* c = CS + ty[I] * (BH_NP * BH_NP * BH_NO);   // [m][n][o]
#pragma unroll
  for (int o = 0; o < BH_NO; ++o)
#pragma unroll
    for (int m = 0; m < BH_NP; ++m) {
      double v = 0.0;
#pragma unroll
      for (int n = 0; n < BH_NP; ++n) v += c[(m * BH_NP + n) * BH_NO + o] * A2[n];
      out[o * BH_NP + m] = v;
    }
}

// Doubles per ket in the LDS ket tables: the 16 kets of a wave read at once sit 2 doubles
// (4 banks) apart modulo the 64 banks, instead of all in one bank.
__host__ __device__ constexpr int bh_ket_stride(int nn) { return nn * BH_NO * BH_NP + 2; }

// LDS tables of the pair-value kernels, in doubles: bra tables [nn][a, grad a][32 bras],
// ket tables [16 kets][bh_ket_stride(nn)], csym [t][m][n][o], nuclei [BH_MAXNUC][x, y, z, b]
__host__ __device__ constexpr long bh_tables_lds_doubles(int nn) {
  return (long)nn * 4 * SB + 16L * bh_ket_stride(nn) + BH_MAXTYPE * BH_NP * BH_NP * BH_NO +
         4L * BH_MAXNUC;
}

// LDS of k_bh_pairs: the tables, then the staged half-precision fragments (two k-steps'
// worth, 2 x 4096 halves)
__host__ __device__ constexpr long bh_pairs_lds_doubles(int nn) {
  return bh_tables_lds_doubles(nn) + 2 * 4096 / 4;
}

struct BHLds {
  double (*TB)[4][SB];   // bra tables of the 32-bra tile
  double* TK;            // ket tables of the current 16-ket step
  double* CS;            // csym
  double (*NU)[4];       // nuclei
  int ks;                // doubles per ket in TK
};

__device__ __forceinline__ BHLds bh_lds(double* sm, int nn) {
  BHLds L;
  L.TB = (double(*)[4][SB])sm;
  L.ks = bh_ket_stride(nn);
  L.TK = sm + nn * 4 * SB;
  L.CS = L.TK + 16 * L.ks;
  L.NU = (double(*)[4])(L.CS + BH_MAXTYPE * BH_NP * BH_NP * BH_NO);
  return L;
}

// csym, the nuclei and the bra tables of bra tile bt (bras past the range repeat its last
// point); followed by a barrier before any use
__device__ __forceinline__ void bh_fill_bra_tables(const BHLds& L, const BHTable* __restrict__ T,
                                                   const double* __restrict__ xyz, long n_g,
                                                   long b0, long bn, long bt, int nn, int tid) {
  for (int e = tid; e < BH_MAXTYPE * BH_NP * BH_NP * BH_NO; e += 256)
    L.CS[e] = (&T->csym[0][0][0][0])[e];
  for (int e = tid; e < 4 * nn; e += 256) L.NU[e / 4][e % 4] = T->nuc[e / 4][e % 4];
  const long blast = b0 + bn - 1;
  for (int e = tid; e < nn * SB; e += 256) {
    const int I = e / SB, bb = e % SB;
    long b = b0 + bt * SB + bb;
    if (b > blast) b = blast;
    double v[4];
    bh_nuc_point(T, I, xyz[b], xyz[n_g + b], xyz[2 * n_g + b], v);
#pragma unroll
    for (int q = 0; q < 4; ++q) L.TB[I][q][bb] = v[q];
  }
  XTC_LDS_DONE();
}

// the ket tables of kets k0 .. k0 + 15 (kets past the grid repeat its last point); between
// barriers
__device__ __forceinline__ void bh_fill_ket_tables(const BHLds& L, const BHTable* __restrict__ T,
                                                   const double* __restrict__ xyz, long n_g,
                                                   long k0, int nn, int tid) {
  for (int e = tid; e < 16 * nn; e += 256) {
    long g = k0 + e / nn;
    if (g > n_g - 1) g = n_g - 1;
    ket_gamma_lds(L.NU, T->type, L.CS, e % nn, xyz[g], xyz[n_g + g], xyz[2 * n_g + g],
                  L.TK + (e / nn) * L.ks + (e % nn) * BH_NO * BH_NP);
  }
  XTC_LDS_DONE();
}

// the nuclear sums of the pairs (bra 2 q2 + v, ket kk), v = 0, 1, in one pass over the
// nuclei: each ket-table entry is read from LDS once for the two bras
__device__ __forceinline__ void bh_two_pairs(const BHLds& L, int nn, int q2, int kk,
                                             double (&F)[2][BH_NO], double (&GF)[2][BH_NO][3]) {
  const double(*tk)[BH_NO][BH_NP] = (const double(*)[BH_NO][BH_NP])(L.TK + kk * L.ks);
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int o = 0; o < BH_NO; ++o) {
      F[v][o] = 0.0;
      GF[v][o][0] = GF[v][o][1] = GF[v][o][2] = 0.0;
    }
  for (int I = 0; I < nn; ++I) {
    double gk[BH_NO][BH_NP];
#pragma unroll
    for (int o = 0; o < BH_NO; ++o)
#pragma unroll
      for (int m = 0; m < BH_NP; ++m) gk[o][m] = tk[I][o][m];
#pragma unroll
    for (int v = 0; v < 2; ++v)
      bh_nuclear_terms(L.TB[I][0][2 * q2 + v], L.TB[I][1][2 * q2 + v], L.TB[I][2][2 * q2 + v],
                       L.TB[I][3][2 * q2 + v], gk, F[v], GF[v]);
  }
}

// One workgroup: bra tile blockIdx.x (32 points) x the GCH ket chunks of group blockIdx.y
// of the launch. Per k-step (16 kets) the ket tables gamma_{I,o,m} go to LDS, then thread
// (ket kk = tid % 16, bra pair q = tid / 16) makes the pairs (bra 2 q + v, ket kk), v = 0, 1:
// each ket table read from LDS serves two pairs. The split values are staged in LDS in the
// B-fragment order (slot L = bra + 32 (kk / 8), element kk % 8) and copied out, 16 bytes per
// lane, during the next k-step. The density-row sums of each bra are added over the
// workgroup in a fixed order and written (first launch) or added (later launches) to
// part[group][8][bp].
__global__ __launch_bounds__(256) void k_bh_pairs(
    const double* __restrict__ xyz, const double* __restrict__ w, const double* __restrict__ rho,
    const double* __restrict__ rhot, long n_g, long b0, long bn, long c0, long nloc, EECoef cf,
    const BHTable* __restrict__ T, int eg, int es, h8* __restrict__ pv,
    double* __restrict__ part, long bp, int first) {
  extern __shared__ double sm[];
  const int nn = T->n_nuc;
  const BHLds L = bh_lds(sm, nn);
  h8* ST = (h8*)(sm + bh_tables_lds_doubles(nn));   // [2][512] h8
  _Float16* STh = (_Float16*)ST;
  const int tid = threadIdx.x, kk = tid & 15, q2 = tid >> 4;
  const long bt = blockIdx.x;
  const long blast = b0 + bn - 1;
  bh_fill_bra_tables(L, T, xyz, n_g, b0, bn, bt, nn, tid);
  double xb[2], yb[2], zb[2];
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    long b = b0 + bt * SB + 2 * q2 + v;
    if (b > blast) b = blast;
    xb[v] = xyz[b];
    yb[v] = xyz[n_g + b];
    zb[v] = xyz[2 * n_g + b];
  }
  const double sg = ldexp(1.0, eg), ss = ldexp(1.0, es);
  double s[2][4] = {}, h[2][4] = {};
  const long cl0 = (long)blockIdx.y * GCH;
  const long cl1 = cl0 + GCH < nloc ? cl0 + GCH : nloc;
  long prev = -1;   // pv index of the staged k-step's first fragment
  for (long cl = cl0; cl < cl1; ++cl) {
    for (int j = 0; j < 8; ++j) {
      const long k0 = (c0 + cl) * SKC + 16 * j;
      __syncthreads();   // TK free again; the previous k-step's staging complete
      if (prev >= 0) {
        const h8* src = ST + ((j + 7) & 1) * 512;   // the buffer of the previous k-step
        pv[prev + tid] = src[tid];
        pv[prev + 256 + tid] = src[256 + tid];
      }
      bh_fill_ket_tables(L, T, xyz, n_g, k0, nn, tid);
      __syncthreads();
      const long g = k0 + kk;
      const long gc = g < n_g ? g : n_g - 1;   // padding kets: finite values, zero weight
      const double kx = xyz[gc], ky = xyz[n_g + gc], kz = xyz[2 * n_g + gc];
      const double a = g < n_g ? w[g] * rho[g] : 0.0, at = g < n_g ? w[g] * rhot[g] : 0.0;
      unsigned pk[2][4];   // per bra and channel: (hi, lo) halves of the scaled value
      double F[2][BH_NO], GF[2][BH_NO][3];
      bh_two_pairs(L, nn, q2, kk, F, GF);
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        double o[4];
        bh_finish(cf, F[v], GF[v], xb[v] - kx, yb[v] - ky, zb[v] - kz, o);
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          s[v][c] = fma(a, o[c], s[v][c]);
          h[v][c] = fma(at, o[c], h[v][c]);
          const double x = o[c] * (c < 3 ? sg : ss);
          const _Float16 hi = (_Float16)(float)x;
          const _Float16 lo = (_Float16)(float)(x - (double)hi);
          pk[v][c] = (unsigned)__builtin_bit_cast(unsigned short, hi) |
                     ((unsigned)__builtin_bit_cast(unsigned short, lo) << 16);
        }
      }
      // lanes kk = 2p and 2p + 1 (adjacent lanes) trade values so that each writes whole
      // 32-bit words: the even lane elements (2p, 2p + 1) of bra 2 q, the odd lane those of
      // bra 2 q + 1
      const bool odd = kk & 1;
      unsigned* dw = (unsigned*)(STh + (j & 1) * 4096);
      const int bw = 2 * q2 + (odd ? 1 : 0);
      const int slot = bw + 32 * (kk >> 3);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const unsigned mine = odd ? pk[1][c] : pk[0][c];
        const unsigned other = (unsigned)__shfl_xor((int)(odd ? pk[0][c] : pk[1][c]), 1);
        const unsigned e0 = odd ? other : mine, e1 = odd ? mine : other;   // kets 2p, 2p + 1
        dw[(((c * 2 + 0) * 64 + slot) * 8 + (kk & 6)) / 2] = (e0 & 0xffffu) | (e1 << 16);
        dw[(((c * 2 + 1) * 64 + slot) * 8 + (kk & 6)) / 2] = (e0 >> 16) | (e1 & 0xffff0000u);
      }
      XTC_LDS_DONE();
      prev = (bt * nloc + cl) * PV_CHUNK + j * 512;
    }
  }
  __syncthreads();
  pv[prev + tid] = ST[512 + tid];   // the last k-step (j = 7) staged in buffer 1
  pv[prev + 256 + tid] = ST[512 + 256 + tid];
  __syncthreads();
  double* red = sm;   // [8 sums][32 bras][16 kets], over the tables and the staging
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      red[(c * SB + 2 * q2 + v) * 16 + kk] = s[v][c];
      red[((4 + c) * SB + 2 * q2 + v) * 16 + kk] = h[v][c];
    }
  XTC_LDS_DONE();
  __syncthreads();
  const int qq = tid >> 5, bb = tid & 31;
  double v = 0.0;
#pragma unroll
  for (int c = 0; c < 16; ++c) v += red[(qq * SB + bb) * 16 + c];
  const long tb = bt * SB + bb;
  if (tb < bn) {
    double* p = part + ((long)blockIdx.y * 8 + qq) * bp + tb;
    *p = first ? v : *p + v;
  }
}

// The FP64 path's pair values (the BH form): the same tables and nuclear sums as k_bh_pairs,
// the four channels stored unscaled in FP64 for k_stage1_f64_pv, per 16-ket step s of the
// launch and 64-bra tile t: pv64[t][s][q][c][gk][gb] for the pair (bra gb, ket 4 gk + q).
// The grid covers whole 64-bra tiles (two 32-bra halves; bras past the range repeat its
// last point).
__global__ __launch_bounds__(256) void k_bh_pairs_f64(const double* __restrict__ xyz, long n_g,
                                                      long b0, long bn, long c0, long nloc,
                                                      EECoef cf, const BHTable* __restrict__ T,
                                                      double* __restrict__ pv64) {
  extern __shared__ double sm[];
  const int nn = T->n_nuc;
  const BHLds L = bh_lds(sm, nn);
  const int tid = threadIdx.x, kk = tid & 15, q2 = tid >> 4;
  const long bt = blockIdx.x;
  const long blast = b0 + bn - 1;
  bh_fill_bra_tables(L, T, xyz, n_g, b0, bn, bt, nn, tid);
  double xb[2], yb[2], zb[2];
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    long b = b0 + bt * SB + 2 * q2 + v;
    if (b > blast) b = blast;
    xb[v] = xyz[b];
    yb[v] = xyz[n_g + b];
    zb[v] = xyz[2 * n_g + b];
  }
  const long nsteps = nloc * 8;
  const long cl0 = (long)blockIdx.y * GCH;
  const long cl1 = cl0 + GCH < nloc ? cl0 + GCH : nloc;
  // this thread's slot in a step: bra 64 (bt % 2) + 2 q2 + v of tile bt / 2, ket 4 gk + q
  double* dst = pv64 + (bt >> 1) * nsteps * 4096 + (kk & 3) * 1024 + (kk >> 2) * 64 +
                (bt & 1) * 32 + 2 * q2;
  for (long cl = cl0; cl < cl1; ++cl) {
    for (int j = 0; j < 8; ++j) {
      const long k0 = (c0 + cl) * SKC + 16 * j;
      __syncthreads();
      bh_fill_ket_tables(L, T, xyz, n_g, k0, nn, tid);
      __syncthreads();
      long g = k0 + kk;
      if (g > n_g - 1) g = n_g - 1;   // padding kets: finite values; their A is zero
      const double kx = xyz[g], ky = xyz[n_g + g], kz = xyz[2 * n_g + g];
      double F[2][BH_NO], GF[2][BH_NO][3];
      bh_two_pairs(L, nn, q2, kk, F, GF);
      double* d = dst + (cl * 8 + j) * 4096;
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        double o[4];
        bh_finish(cf, F[v], GF[v], xb[v] - kx, yb[v] - ky, zb[v] - kz, o);
#pragma unroll
        for (int c = 0; c < 4; ++c) d[c * 256 + v] = o[c];
      }
    }
  }
}

size_t bh_f64_pv_bytes(long bp) {
  return (size_t)cdiv(bp, 64) * SMED * 8 * 4096 * sizeof(double) + 256;
}

xtc_status bh_pair_values_f64(const Stage1Args& a, const EECoef& cf, long c0, long nloc,
                              hipStream_t st) {
  XTC_REQUIRE(a.bh && a.bh_host && a.pv64, "FP64 BH stage 1: no correlator table or buffer");
  XTC_REQUIRE(nloc >= 1 && nloc <= SMED && a.bn <= a.bp, "FP64 BH stage 1: bad launch range");
  const int nn = a.bh_host->n_nuc;
  const size_t lds = sizeof(double) * (size_t)bh_tables_lds_doubles(nn);
  hipLaunchKernelGGL(k_bh_pairs_f64, dim3(2 * cdiv(a.bn, 64), cdiv(nloc, GCH)), dim3(256), lds, st,
                     a.xyz, a.n_g, a.b0, a.bn, c0, nloc, cf, a.bh, a.pv64);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

// rows n_mu (rho_gamma) and n_mu + 1 (ISDF density) of the panel from the group sums
__global__ __launch_bounds__(256) void k_bh_rho_rows(const double* __restrict__ part, int ngrp,
                                                     long bn, int n_mu, double* __restrict__ panel,
                                                     long rows_pad, long bp) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= bn) return;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double v = 0.0;
    for (int g = 0; g < ngrp; ++g) v += part[((long)g * 8 + q) * bp + t];
    panel[((long)(q & 3) * rows_pad + n_mu + (q >> 2)) * bp + t] = v;
  }
}

// Tile groups of the split-product launch: PV_GR row tiles x PV_GB bra tiles per XCD at a
// time (32 workgroups, one per CU of the XCD), which share PV_GR row tiles of A and PV_GB
// bra tiles of pair values in its L2. A is read two k-steps ahead of its use and the pair
// values a whole chunk ahead, so the groups favour sharing A.
constexpr int PV_GR = 2, PV_GB = 16;

// The split products over ket chunks [c0, c1) with the pair values from pv. 8 waves over a
// tile of 256 rows (wave v: rows 32 v .. 32 v + 31) x 32 bra points. grouped: the grid has
// nrt x nbt_grid workgroups (nrt a multiple of PV_GR, nbt_grid of PV_GB, nrt nbt_grid of
// 8 PV_GR PV_GB; tiles past nbt exit at once), and XCD x (ids are dealt to the 8 XCDs in
// turn) takes the consecutive tile groups [x, x + 1) nwg / 8 in order; otherwise the row
// tiles of one bra tile are consecutive.
__global__ __attribute__((amdgpu_flat_work_group_size(512, 512), amdgpu_waves_per_eu(2, 2)))
void k_stage1_split_pv(const h8* __restrict__ At, const int* __restrict__ sA, long nks,
                       const h8* __restrict__ pv, int nrt, int nbt, int nbt_grid, int grouped,
                       long nloc, int eg, int es, double* __restrict__ panel, long rows_pad_panel,
                       long bp, long c0, long c1, int first_flush) {
  extern __shared__ h8 Bs[];   // [2 buf][8 ksteps][4 ch][2 hl][64 lanes]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long nwg = (long)nrt * nbt_grid, id = blockIdx.x;
  long rt, bt;
  if (grouped) {
    const long lid = (id % 8) * (nwg / 8) + id / 8;
    const long blk = lid / (PV_GR * PV_GB), wq = lid % (PV_GR * PV_GB);
    const long nrb = nrt / PV_GR;
    rt = (blk % nrb) * PV_GR + wq % PV_GR;
    bt = (blk / nrb) * PV_GB + wq / PV_GR;
  } else {
    const long lid = (nwg % 8 == 0) ? (id % 8) * (nwg / 8) + id / 8 : id;
    rt = lid % nrt;
    bt = lid / nrt;
  }
  if (bt >= nbt) return;   // padding of the grouped grid (whole workgroup, before any barrier)
  const long row0 = rt * SR, nb0 = bt * SB;
  const h8* Aw = At + (row0 / 32 + wave) * nks * 128 + lane;
  const h8* Bt = pv + bt * nloc * PV_CHUNK + tid;
  const long last_ks = nks - 1;
#pragma unroll
  for (int i = 0; i < 8; ++i) Bs[i * 512 + tid] = Bt[i * 512];
  // A operand pipeline: loaded three k-steps ahead (ks + 1 .. ks + 3 in flight while ks is used)
  h8 a0[2], a1[2], a2[2];
  {
    const long s0 = c0 * 8, s1 = c0 * 8 + 1 < last_ks ? c0 * 8 + 1 : last_ks;
    const long s2 = c0 * 8 + 2 < last_ks ? c0 * 8 + 2 : last_ks;
    a0[0] = Aw[s0 * 128];
    a0[1] = Aw[s0 * 128 + 64];
    a1[0] = Aw[s1 * 128];
    a1[1] = Aw[s1 * 128 + 64];
    a2[0] = Aw[s2 * 128];
    a2[1] = Aw[s2 * 128 + 64];
  }
  f16x med[4], acc[4];
#pragma unroll
  for (int ch = 0; ch < 4; ++ch)
#pragma unroll
    for (int r = 0; r < 16; ++r) med[ch][r] = 0.0f;
  const f16x zero = {};
  __syncthreads();
  auto chunk = [&](long c, auto zero_tag) {
    constexpr bool ZERO = decltype(zero_tag)::value;
    const int buf = (int)((c - c0) & 1);
    const h8* Bb = Bs + buf * PV_CHUNK + lane;
    // the next chunk's pair values (this chunk's again after the launch's last chunk, into
    // the buffer nobody reads any more), issued before this chunk's A loads without a
    // branch, so that the waits for A count exactly and the wait for them at the chunk's end
    // leaves the A loads in flight
    const long cn = c + 1 < c1 ? c + 1 - c0 : c - c0;
    const h8* Bn = Bt + cn * PV_CHUNK;
    h8 nx[8], bh[4], bl[4];
#pragma unroll
    for (int i = 0; i < 8; ++i) nx[i] = Bn[i * 512];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      bh[ch] = Bb[(ch * 2 + 0) * 64];
      bl[ch] = Bb[(ch * 2 + 1) * 64];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      long ks3 = c * 8 + j + 3;
      if (ks3 > last_ks) ks3 = last_ks;
      h8 a3[2];
      a3[0] = Aw[ks3 * 128];
      a3[1] = Aw[ks3 * 128 + 64];
      // scheduling fences keep the loads issued ahead of their uses (unfenced, the
      // scheduler sinks them towards the MFMAs and every k-step waits on memory)
      XTC_FENCE();
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
        acc[ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[1], bh[ch],
                                                         (ZERO && j == 0) ? zero : acc[ch], 0, 0, 0);
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
        acc[ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[0], bh[ch], acc[ch], 0, 0, 0);
      XTC_FENCE();
      if (j < 7) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) bh[ch] = Bb[(((j + 1) * 4 + ch) * 2 + 0) * 64];
      }
      XTC_FENCE();
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
        acc[ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[0], bl[ch], acc[ch], 0, 0, 0);
      XTC_FENCE();
      if (j < 7) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) bl[ch] = Bb[(((j + 1) * 4 + ch) * 2 + 1) * 64];
      }
      XTC_FENCE();
      a0[0] = a1[0];
      a0[1] = a1[1];
      a1[0] = a2[0];
      a1[1] = a2[1];
      a2[0] = a3[0];
      a2[1] = a3[1];
    }
    h8* Bo = Bs + (buf ^ 1) * PV_CHUNK + tid;
#pragma unroll
    for (int i = 0; i < 8; ++i) Bo[i * 512] = nx[i];
    __syncthreads();
  };
  // chunks in pairs (every launch covers an even number): the MFMA accumulator sums
  // 256 kets before it is added to the FP32 medium sum
  for (long c = c0; c < c1; c += 2) {
    chunk(c, std::true_type{});
    chunk(c + 1, std::false_type{});
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) med[ch] += acc[ch];
  }
  // med -> FP64 panel, scales removed exactly: lane l holds rows 8 q + 4 (l / 32) + rr of
  // its wave's block (register 4 q + rr) and bra column l % 32
  const long col = nb0 + (lane & 31);
  const long rbase = row0 + 32 * wave + 4 * (lane >> 5);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const long rq = rbase + 8 * q;
    const int4 e4 = *(const int4*)(sA + rq);
    const int ev[4] = {e4.x, e4.y, e4.z, e4.w};
    double* p = panel + rq * bp + col;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr)
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        double v = ldexp((double)med[ch][4 * q + rr], -(ev[rr] + (ch < 3 ? eg : es)));
        double* pe = p + ((long)ch * rows_pad_panel + rr) * bp;
        if (!first_flush) v += *pe;
        *pe = v;
      }
  }
}

xtc_status stage1_split_bh(const Stage1Args& a, const EECoef& cf, void* scratch, size_t bytes,
                           hipStream_t st) {
  XTC_REQUIRE(a.bh && a.bh_host, "split BH stage 1: no correlator table");
  const size_t off_part = split_scratch_bytes(a.n_g, a.n_mu);
  const size_t off_pv = off_part + rho_row_scratch_bytes(a.bp);
  XTC_REQUIRE(bytes >= off_pv + bh_split_scratch_bytes(a.bp),
              "split BH stage 1: scratch smaller than its pair-value buffer");
  SplitLayout S = split_layout(scratch, a.n_g, a.n_mu);
  const int nbt = (int)cdiv(a.bn, SB);
  // whole 256-row tiles and 32-column bra tiles are written
  XTC_REQUIRE(a.rows_pad >= S.rows_pad && a.bp >= (long)nbt * SB,
              "split BH stage 1: panel smaller than its tiles");
  double* part = (double*)((char*)scratch + off_part);
  h8* pv = (h8*)((char*)scratch + off_pv);
  int eg = 0, es = 0;
  bh_split_exponents(*a.bh_host, cf, &eg, &es);
  const int nn = a.bh_host->n_nuc;
  const size_t lds_gen = sizeof(double) * (size_t)std::max(bh_pairs_lds_doubles(nn), 8L * SB * 16);
  const size_t lds_pv = sizeof(h8) * 2 * PV_CHUNK;
  const int nrt = (int)(S.rows_pad / SR);
  const long nchunks = S.n_g_pad / SKC;
  const int grouped = nrt % PV_GR == 0 ? 1 : 0;
  int nbt_grid = nbt;
  if (grouped) {   // whole tile groups, and as many workgroups on each of the 8 XCDs
    nbt_grid = (int)cdiv(nbt, PV_GB) * PV_GB;
    while (((long)nrt * nbt_grid) % (8 * PV_GR * PV_GB) != 0) nbt_grid += PV_GB;
  }
  for (long c0 = 0; c0 < nchunks; c0 += SMED) {
    const long nloc = SMED < nchunks - c0 ? SMED : nchunks - c0;
    size_t tk = timing_begin(TM_S1_PAIRS, st);
    hipLaunchKernelGGL(k_bh_pairs, dim3(nbt, cdiv(nloc, GCH)), dim3(256), lds_gen, st, a.xyz, a.w,
                       a.rho, a.rhot, a.n_g, a.b0, a.bn, c0, nloc, cf, a.bh, eg, es, pv, part,
                       a.bp, c0 == 0 ? 1 : 0);
    timing_end(tk, st);
    XTC_CHECK_LAUNCH();
    tk = timing_begin(TM_S1_KERNEL, st);
    hipLaunchKernelGGL(k_stage1_split_pv, dim3((unsigned)nrt * nbt_grid), dim3(512), lds_pv, st,
                       (const h8*)S.A, (const int*)S.sA, S.nks, (const h8*)pv, nrt, nbt, nbt_grid,
                       grouped, nloc, eg, es, a.panel, a.rows_pad, a.bp, c0, c0 + nloc,
                       c0 == 0 ? 1 : 0);
    timing_end(tk, st);
    XTC_CHECK_LAUNCH();
  }
  const int ngrp = (int)cdiv(SMED < nchunks ? SMED : nchunks, GCH);
  hipLaunchKernelGGL(k_bh_rho_rows, dim3(cdiv(a.bn, 256)), dim3(256), 0, st, (const double*)part,
                     ngrp, a.bn, a.n_mu, a.panel, a.rows_pad, a.bp);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

}  // namespace xtc
