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
// The A operand and its per-row exponents are the split operand of the EE path.
#include <algorithm>
#include <type_traits>
#include "bh.hpp"
#include "stage1_split.hpp"
#include "timing.hpp"

namespace xtc {

typedef _Float16 h2 __attribute__((ext_vector_type(2)));

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

// One workgroup: bra tile blockIdx.x (32 points) x the GCH ket chunks of group blockIdx.y
// of the launch. Per k-step (16 kets) the ket tables gamma_{I,o,m} go to LDS, then thread
// (slot L = tid % 64, wave v) makes the pairs of slot L's bra and kets 8 (L / 32) + 2 v + u,
// u = 0, 1: elements 2 v, 2 v + 1 of slot L's B fragments, stored as (hi, hi) and (lo, lo)
// half pairs. The density-row sums of each bra slot are added over the workgroup in a
// fixed order and written (first launch) or added (later launches) to part[group][8][bp].
__global__ __launch_bounds__(256) void k_bh_pairs(
    const double* __restrict__ xyz, const double* __restrict__ w, const double* __restrict__ rho,
    const double* __restrict__ rhot, long n_g, long b0, long bn, long c0, long nloc, EECoef cf,
    const BHTable* __restrict__ T, int eg, int es, h8* __restrict__ pv,
    double* __restrict__ part, long bp, int first) {
  extern __shared__ double sm[];
  const int nn = T->n_nuc;
  double(*TB)[4][SB] = (double(*)[4][SB])sm;   // [nn][a, grad a][bra slot]
  double* TK = sm + nn * 4 * SB;                // [16 kets][nn][BH_NO][BH_NP]
  const int tid = threadIdx.x, L = tid & 63, wv = tid >> 6, gb = L & 31;
  const long bt = blockIdx.x;
  const long blast = b0 + bn - 1;
  for (int e = tid; e < nn * SB; e += 256) {
    const int I = e / SB, bb = e % SB;
    long b = b0 + bt * SB + bb;
    if (b > blast) b = blast;
    double v[4];
    bh_nuc_point(T, I, xyz[b], xyz[n_g + b], xyz[2 * n_g + b], v);
#pragma unroll
    for (int q = 0; q < 4; ++q) TB[I][q][bb] = v[q];
  }
  long b = b0 + bt * SB + gb;
  if (b > blast) b = blast;
  const double xb = xyz[b], yb = xyz[n_g + b], zb = xyz[2 * n_g + b];
  const double sg = ldexp(1.0, eg), ss = ldexp(1.0, es);
  double s[4] = {0.0, 0.0, 0.0, 0.0}, h[4] = {0.0, 0.0, 0.0, 0.0};
  const long cl0 = (long)blockIdx.y * GCH;
  const long cl1 = cl0 + GCH < nloc ? cl0 + GCH : nloc;
  const int kq = 8 * (L >> 5) + 2 * wv;
  for (long cl = cl0; cl < cl1; ++cl) {
    h8* dst = pv + (bt * nloc + cl) * PV_CHUNK + L;
    for (int j = 0; j < 8; ++j) {
      const long k0 = (c0 + cl) * SKC + 16 * j;
      __syncthreads();   // the previous k-step's readers of TK are done (and TB is written)
      for (int e = tid; e < 16 * nn; e += 256) {
        long g = k0 + e / nn;
        if (g > n_g - 1) g = n_g - 1;
        bh_ket_gamma(T, e % nn, xyz[g], xyz[n_g + g], xyz[2 * n_g + g],
                     (double(*)[BH_NP])(TK + (long)e * BH_NO * BH_NP));
      }
      __syncthreads();
      double o[2][4];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int kk = kq + u;
        const long g = k0 + kk;
        const long gc = g < n_g ? g : n_g - 1;   // padding kets: finite values, zero weight
        bh_pair_channels<SB>(cf, nn, TB, gb,
                             (const double(*)[BH_NO][BH_NP])(TK + (long)kk * nn * BH_NO * BH_NP),
                             xb - xyz[gc], yb - xyz[n_g + gc], zb - xyz[2 * n_g + gc], o[u]);
        if (g < n_g) {
          const double a = w[g] * rho[g], at = w[g] * rhot[g];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            s[q] = fma(a, o[u][q], s[q]);
            h[q] = fma(at, o[u][q], h[q]);
          }
        }
      }
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        const double sc = ch < 3 ? sg : ss;
        const double v0 = o[0][ch] * sc, v1 = o[1][ch] * sc;
        const _Float16 h0 = (_Float16)(float)v0, h1 = (_Float16)(float)v1;
        const _Float16 l0 = (_Float16)(float)(v0 - (double)h0);
        const _Float16 l1 = (_Float16)(float)(v1 - (double)h1);
        ((h2*)(dst + ((j * 4 + ch) * 2 + 0) * 64))[wv] = (h2){h0, h1};
        ((h2*)(dst + ((j * 4 + ch) * 2 + 1) * 64))[wv] = (h2){l0, l1};
      }
    }
  }
  __syncthreads();
  double* red = sm;   // [8 sums][8 contributors][SB]
  const int ctb = 2 * wv + (L >> 5);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    red[(q * 8 + ctb) * SB + gb] = s[q];
    red[((4 + q) * 8 + ctb) * SB + gb] = h[q];
  }
  __syncthreads();
  const int q = tid >> 5, bb = tid & 31;
  double v = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) v += red[(q * 8 + c) * SB + bb];
  const long tb = bt * SB + bb;
  if (tb < bn) {
    double* p = part + ((long)blockIdx.y * 8 + q) * bp + tb;
    *p = first ? v : *p + v;
  }
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

// The split products over ket chunks [c0, c1) with the pair values from pv. 8 waves over a
// tile of 256 rows (wave v: rows 32 v .. 32 v + 31) x 32 bra points; workgroup ids are
// mapped so that the row tiles of one bra tile, which read the same pair values, run on
// one XCD (ids are dealt to the 8 XCDs in turn).
__global__ __attribute__((amdgpu_flat_work_group_size(512, 512), amdgpu_waves_per_eu(2, 2)))
void k_stage1_split_pv(const h8* __restrict__ At, const int* __restrict__ sA, long nks,
                       const h8* __restrict__ pv, int nrt, int nbt, long nloc, int eg, int es,
                       double* __restrict__ panel, long rows_pad_panel, long bp, long c0, long c1,
                       int first_flush) {
  extern __shared__ h8 Bs[];   // [2 buf][8 ksteps][4 ch][2 hl][64 lanes]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long nwg = (long)nrt * nbt, id = blockIdx.x;
  const long lid = (nwg % 8 == 0) ? (id % 8) * (nwg / 8) + id / 8 : id;
  const long row0 = (lid % nrt) * SR, bt = lid / nrt, nb0 = bt * SB;
  const h8* Aw = At + (row0 / 32 + wave) * nks * 128 + lane;
  const h8* Bt = pv + bt * nloc * PV_CHUNK + tid;
  const long last_ks = nks - 1;
#pragma unroll
  for (int i = 0; i < 8; ++i) Bs[i * 512 + tid] = Bt[i * 512];
  h8 a0[2], a1[2];
  {
    const long s0 = c0 * 8, s1 = c0 * 8 + 1 < last_ks ? c0 * 8 + 1 : last_ks;
    a0[0] = Aw[s0 * 128];
    a0[1] = Aw[s0 * 128 + 64];
    a1[0] = Aw[s1 * 128];
    a1[1] = Aw[s1 * 128 + 64];
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
    const bool more = c + 1 < c1;
    const h8* Bn = Bt + (c + 1 - c0) * PV_CHUNK;
    h8 nx[8], bh[4], bl[4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      bh[ch] = Bb[(ch * 2 + 0) * 64];
      bl[ch] = Bb[(ch * 2 + 1) * 64];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      long ks2 = c * 8 + j + 2;
      if (ks2 > last_ks) ks2 = last_ks;
      h8 a2[2];
      a2[0] = Aw[ks2 * 128];
      a2[1] = Aw[ks2 * 128 + 64];
      if (more) nx[j] = Bn[j * 512];
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
        acc[ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[1], bh[ch],
                                                         (ZERO && j == 0) ? zero : acc[ch], 0, 0, 0);
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
        acc[ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[0], bh[ch], acc[ch], 0, 0, 0);
      if (j < 7) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) bh[ch] = Bb[(((j + 1) * 4 + ch) * 2 + 0) * 64];
      }
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
        acc[ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[0], bl[ch], acc[ch], 0, 0, 0);
      if (j < 7) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) bl[ch] = Bb[(((j + 1) * 4 + ch) * 2 + 1) * 64];
      }
      a0[0] = a1[0];
      a0[1] = a1[1];
      a1[0] = a2[0];
      a1[1] = a2[1];
    }
    if (more) {
      h8* Bo = Bs + (buf ^ 1) * PV_CHUNK + tid;
#pragma unroll
      for (int i = 0; i < 8; ++i) Bo[i * 512] = nx[i];
    }
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
  const size_t lds_gen = sizeof(double) * (size_t)std::max(nn * (4 * SB + 16 * BH_NO * BH_NP),
                                                           8 * 8 * SB);
  const size_t lds_pv = sizeof(h8) * 2 * PV_CHUNK;
  const int nrt = (int)(S.rows_pad / SR);
  const long nchunks = S.n_g_pad / SKC;
  for (long c0 = 0; c0 < nchunks; c0 += SMED) {
    const long nloc = SMED < nchunks - c0 ? SMED : nchunks - c0;
    size_t tk = timing_begin(TM_S1_PAIRS, st);
    hipLaunchKernelGGL(k_bh_pairs, dim3(nbt, cdiv(nloc, GCH)), dim3(256), lds_gen, st, a.xyz, a.w,
                       a.rho, a.rhot, a.n_g, a.b0, a.bn, c0, nloc, cf, a.bh, eg, es, pv, part,
                       a.bp, c0 == 0 ? 1 : 0);
    timing_end(tk, st);
    XTC_CHECK_LAUNCH();
    tk = timing_begin(TM_S1_KERNEL, st);
    hipLaunchKernelGGL(k_stage1_split_pv, dim3((unsigned)nrt * nbt), dim3(512), lds_pv, st,
                       (const h8*)S.A, (const int*)S.sA, S.nks, (const h8*)pv, nrt, nbt, nloc, eg,
                       es, a.panel, a.rows_pad, a.bp, c0, c0 + nloc, c0 == 0 ? 1 : 0);
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
