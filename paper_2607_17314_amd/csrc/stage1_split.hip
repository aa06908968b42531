// Stage 1 of the grid-pair contraction with FP16 split products on the
// CDNA4 matrix cores:
//   panel[ch][row][g] = sum_g' A[row][g'] K_ch(g, g'),  A = [w xi ; w rho].
// Both operands are split into an FP16 pair, x ~= x_hi + x_lo, after a
// power-of-two scaling (A per row, K per channel), and every product is taken
// as A_hi K_hi + A_hi K_lo + A_lo K_hi with v_mfma_f32_32x32x16_f16 (the
// dropped A_lo K_lo term is 2^-22 relative). Accumulation is three-level:
// the MFMA accumulator over a pair of 128-point ket chunks, an FP32 medium
// sum over the chunks of one launch, then FP64 in the output panel; the scales
// are removed exactly on flush.
//
// Workgroup: 8 waves (two per SIMD) over a tile of 256 rows x 32 bra points.
// Per ket chunk every thread generates the 4 kernel channels of one (bra, ket)
// pair per k-step in FP32 (pair differences formed in double-float, so close
// pairs keep their relative accuracy), in three stages placed beside the three
// MFMA groups of the k-step, and writes the split values to LDS in the MFMA
// B-operand layout (double-buffered, 128 KB). The A operand streams from a
// pre-split, MFMA-native tiled copy in HBM two k-steps ahead; scheduling fences
// keep those loads from sinking towards their uses. The ket range is cut into
// launches of SMED chunks so that the workgroups resident at one time walk the
// same stretch of A and share it in L2.
//
// MFMA 32x32x16 f16 layouts (measured on gfx950), lane l, element e, register r:
//   A[l % 32][8 (l / 32) + e]   B[8 (l / 32) + e][l % 32]
//   D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
#include <type_traits>
#include "stage1_split.hpp"
#include "timing.hpp"

namespace xtc {

#ifndef SPLIT_WAVES
#define SPLIT_WAVES 8          // waves per workgroup (4 or 8)
#endif

// Pair-kernel coefficients in FP32 with d and the power-of-two channel scales
// folded in: U = t^2 Q1f(rbar) = 2^(es/2) u', F = t^3 Q2f(rbar) (+ c1f t^2 / r) = 2^eg u'/r.
struct SplitCoef {
  float d;
  float c1;         // c1 d 2^eg (the o = 1 term of u'/r)
  float q1[MAXQ];   // q1 d 2^(es/2)
  float q2[MAXQ];   // q2 d^2 2^eg
  int eg, es;       // channel exponents; es is even
};

size_t split_scratch_bytes(long n_g, int n_mu) {
  Arena ar(nullptr, 0);
  long rows_pad = ((n_mu + SR - 1) / SR) * SR;
  long n_g_pad = ((n_g + 2 * SKC - 1) / (2 * SKC)) * (2 * SKC);
  ar.take<h8>((size_t)(rows_pad / 32) * (n_g_pad / 16) * 2 * 64);
  ar.take<int>(rows_pad);
  ar.take<float>(6 * (size_t)n_g_pad);
  return ar.used + 256;
}

// --- preparation --------------------------------------------------------------

// w xi in FP64 from xi stored in FP64 or FP32 (T)
template <class T>
__device__ __forceinline__ double a_value(const double* __restrict__ w, const T* __restrict__ xi,
                                          long n_g, int n_mu, long row, long g) {
  if (g >= n_g || row >= n_mu) return 0.0;
  return w[g] * (double)xi[row * n_g + g];
}

// one block per row: exponent s with max |A_row| 2^s in [2^14, 2^15)
template <class T>
__global__ __launch_bounds__(256) void k_row_scale(const double* __restrict__ w,
                                                   const T* __restrict__ xi, long n_g,
                                                   int n_mu, int* __restrict__ sA) {
  __shared__ double red[256];
  const long row = blockIdx.x;
  double m = 0.0;
  for (long g = threadIdx.x; g < n_g; g += 256) m = fmax(m, fabs(a_value(w, xi, n_g, n_mu, row, g)));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int e = 0;
    if (red[0] > 0.0) {
      int ex;
      frexp(red[0], &ex);          // red = f 2^ex, f in [0.5, 1)
      e = 15 - ex;                 // red 2^e in [2^14, 2^15)
    }
    sA[row] = e;
  }
}

// one thread per (row block, k-step, lane): 8 consecutive ket values, split
template <class T>
__global__ __launch_bounds__(256) void k_split_A(const double* __restrict__ w,
                                                 const T* __restrict__ xi, long n_g,
                                                 int n_mu, const int* __restrict__ sA, long nks,
                                                 long nrb, h8* __restrict__ At) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= nrb * nks * 64) return;
  const int lane = (int)(t % 64);
  const long ks = (t / 64) % nks;
  const long rb = t / (64 * nks);
  const long row = rb * 32 + (lane % 32);
  const long k0 = ks * 16 + 8 * (lane / 32);
  const double sc = ldexp(1.0, sA[row]);
  h8 hi, lo;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const double v = a_value(w, xi, n_g, n_mu, row, k0 + e) * sc;
    const float vf = (float)v;
    const _Float16 h = (_Float16)vf;
    hi[e] = h;
    lo[e] = (_Float16)((float)(v - (double)(float)h));
  }
  const long base = ((rb * nks + ks) * 2) * 64 + lane;
  At[base] = hi;
  At[base + 64] = lo;
}

__global__ __launch_bounds__(256) void k_split_coords(const double* __restrict__ xyz, long n_g,
                                                      long n_g_pad, float* __restrict__ kc) {
  const long g = (long)blockIdx.x * 256 + threadIdx.x;
  if (g >= n_g_pad) return;
  const long src = g < n_g ? g : n_g - 1;   // padding repeats the last point (its A is zero)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double v = xyz[c * n_g + src];
    const float h = (float)v;
    kc[c * n_g_pad + g] = h;
    kc[(3 + c) * n_g_pad + g] = (float)(v - (double)h);
  }
}

xtc_status split_prepare(const Stage1Args& a, void* scratch, hipStream_t st) {
  SplitLayout S = split_layout(scratch, a.n_g, a.n_mu);
  XTC_HIP(hipMemsetAsync(S.sA, 0, sizeof(int) * S.rows_pad, st));
  const long nrb = S.rows_pad / 32;
  if (a.xi32) {
    hipLaunchKernelGGL(k_row_scale<float>, dim3(a.n_mu), dim3(256), 0, st, a.w, a.xi32, a.n_g,
                       a.n_mu, S.sA);
    XTC_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_split_A<float>, dim3(cdiv(nrb * S.nks * 64, 256)), dim3(256), 0, st, a.w,
                       a.xi32, a.n_g, a.n_mu, (const int*)S.sA, S.nks, nrb, S.A);
  } else {
    hipLaunchKernelGGL(k_row_scale<double>, dim3(a.n_mu), dim3(256), 0, st, a.w, a.xi, a.n_g,
                       a.n_mu, S.sA);
    XTC_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_split_A<double>, dim3(cdiv(nrb * S.nks * 64, 256)), dim3(256), 0, st, a.w,
                       a.xi, a.n_g, a.n_mu, (const int*)S.sA, S.nks, nrb, S.A);
  }
  XTC_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_split_coords, dim3(cdiv(S.n_g_pad, 256)), dim3(256), 0, st, a.xyz, a.n_g,
                     S.n_g_pad, S.kc);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

// --- the pair kernel ------------------------------------------------------------

// Horner with a compile-time degree bound; coefficients beyond the true degree are 0.
template <int N>
__device__ __forceinline__ float hornerf(const float* q, float x) {
  float r = q[N - 1];
#pragma unroll
  for (int j = N - 2; j >= 0; --j) r = r * x + q[j];
  return r;
}

// The four scaled channels of one pair, (d_x u, d_y u, d_z u) 2^eg and |grad u|^2 2^es,
// in three stages so that each can be placed beside its own group of MFMAs:
//   A: r from the pair difference (formed in double-float, so close pairs keep
//      their relative accuracy);
//   B: t = 1/(1 + d r), rbar = d r t, U = sqrt(2^es) u' and F = 2^eg u'/r, with d and
//      the channel scales folded into the polynomial coefficients;
//   C: the channels F dx, F dy, F dz, U^2.
// EVEN: every power o_k is even (no o = 1 term), so Q1(e) = e P1(e^2), Q2(e) = P2(e^2)
// with compacted coefficients (q1[i] of e^(2i+1), q2[i] of e^(2i)).
struct PairState {
  float dx, dy, dz, r;
  float U, F;
};

__device__ __forceinline__ void pair_stage_a(PairState& p, float bxh, float bxl, float byh,
                                             float byl, float bzh, float bzl, const float (&c)[6]) {
  p.dx = (bxh - c[0]) + (bxl - c[3]);
  p.dy = (byh - c[1]) + (byl - c[4]);
  p.dz = (bzh - c[2]) + (bzl - c[5]);
  p.r = __builtin_amdgcn_sqrtf(p.dx * p.dx + p.dy * p.dy + p.dz * p.dz);   // v_sqrt_f32, 1 ulp
}

template <bool EVEN, int NQ>
__device__ __forceinline__ void pair_stage_b(PairState& p, const SplitCoef& k) {
  const float dr = k.d * p.r;
  const float t = __builtin_amdgcn_rcpf(1.0f + dr);
  const float e = dr * t;
  const float t2 = t * t;
  if (EVEN) {
    const float e2 = e * e;
    p.U = t2 * e * hornerf<NQ>(k.q1, e2);
    p.F = t2 * t * hornerf<NQ>(k.q2, e2);
  } else {
    p.U = t2 * hornerf<MAXQ>(k.q1, e);
    float f = t2 * t * hornerf<MAXQ>(k.q2, e);
    if (k.c1 != 0.0f && p.r > 0.0f) f += k.c1 * t2 / p.r;
    p.F = f;
  }
}

__device__ __forceinline__ void pair_stage_c(const PairState& p, float (&o)[4]) {
  o[0] = p.F * p.dx;
  o[1] = p.F * p.dy;
  o[2] = p.F * p.dz;
  o[3] = p.U * p.U;
}

// One k-step's MFMA group and the VALU work placed beside it: the scheduler is
// told to alternate one MFMA with `nv` vector instructions, and fences keep the
// loads issued ahead of the group from sinking towards their uses.
#define XTC_INTERLEAVE(nmfma, nv)                                        \
  do {                                                                   \
    _Pragma("unroll") for (int i_ = 0; i_ < (nmfma); ++i_) {             \
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);                 \
      __builtin_amdgcn_sched_group_barrier(0x002, (nv), 0);              \
    }                                                                    \
  } while (0)
#define XTC_FENCE() __builtin_amdgcn_sched_barrier(0)

// Workgroup of NW waves (4 or 8) over a tile of 256 rows x 32 bra points: wave w
// owns NB = 8 / NW consecutive 32-row blocks and, for the generation, the NX = 8 / NW
// k-steps NX w .. NX w + NX - 1 of the next chunk (one pair of each per k-step).
template <bool EVEN, int NQ, int NW>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * NW, 64 * NW),
                          amdgpu_waves_per_eu(NW / 4, NW / 4)))
void k_stage1_split(const h8* __restrict__ At, const int* __restrict__ sA,
                    const float* __restrict__ kc, long n_g_pad, long nks,
                    const double* __restrict__ xyz, long n_g, int n_mu, long b0, long bn,
                    SplitCoef k, double* __restrict__ panel, long rows_pad_panel, long bp,
                    long c0, long c1, int first_flush) {
  constexpr int NB = 8 / NW, NX = 8 / NW, NT = 64 * NW;
  constexpr int NCV = (6 * SKC + NT - 1) / NT;   // coordinate floats loaded per thread
  extern __shared__ h8 Bs[];   // [2 buf][8 ksteps][4 ch][2 hl][64 lanes], then coordinates
  float* Kc = (float*)(Bs + 2 * 8 * 8 * 64);   // [2 buf][6][SKC]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long row0 = (long)blockIdx.y * SR;
  const long nb0 = (long)blockIdx.x * SB;
  long bra = b0 + nb0 + (lane & 31);
  if (bra > b0 + bn - 1) bra = b0 + bn - 1;
  const double bx = xyz[bra], by = xyz[n_g + bra], bz = xyz[2 * n_g + bra];
  const float bxh = (float)bx, byh = (float)by, bzh = (float)bz;
  const float bxl = (float)(bx - (double)bxh), byl = (float)(by - (double)byh),
              bzl = (float)(bz - (double)bzh);
  // this wave's 32-row blocks of the pre-split A
  const h8* Aw = At + ((row0 / 32) + NB * wave) * nks * 128 + lane;
  const long Ab = nks * 128;                   // stride between consecutive blocks
  const long nchunks = n_g_pad / SKC;
  const long last_ks = nks - 1;

  // Generation: lane slot `lane` of k-step jx is bra lane & 31, ket 16 jx + 8 (lane / 32) + e.
  // Pair e of this wave's k-steps is made during k-step e of the current chunk; the
  // half fragments (e = 0..3, then 4..7) go to the other LDS buffer after k-steps 3 and 7.
  const int kofs = 16 * NX * wave + 8 * (lane >> 5);
  auto read_coords = [&](const float* kcb, int e, float (&c)[NX][6]) {
#pragma unroll
    for (int x = 0; x < NX; ++x)
#pragma unroll
      for (int q = 0; q < 6; ++q) c[x][q] = kcb[q * SKC + kofs + 16 * x + e];
  };
  typedef _Float16 h4 __attribute__((ext_vector_type(4)));
  auto put = [&](h4 (&fr)[NX][4][2], int x, const float (&o)[4], int e) {
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      const _Float16 h = (_Float16)o[ch];
      fr[x][ch][0][e & 3] = h;
      fr[x][ch][1][e & 3] = (_Float16)(o[ch] - (float)h);
    }
  };
  auto store_half = [&](int buf, h4 (&fr)[NX][4][2], int half) {
    h4* B4 = (h4*)Bs;
#pragma unroll
    for (int x = 0; x < NX; ++x)
#pragma unroll
      for (int ch = 0; ch < 4; ++ch)
#pragma unroll
        for (int hl = 0; hl < 2; ++hl)
          B4[2 * ((((long)buf * 8 + NX * wave + x) * 8 + ch * 2 + hl) * 64 + lane) + half] =
              fr[x][ch][hl];
  };
  // coordinates of chunk c: 6 x SKC floats, NCV per thread
  auto load_coords = [&](long c, float (&v)[NCV]) {
    const long cc = c < nchunks ? c : nchunks - 1;
#pragma unroll
    for (int i = 0; i < NCV; ++i) {
      const int q = tid + NT * i;
      v[i] = q < 6 * SKC ? kc[(long)(q / SKC) * n_g_pad + cc * SKC + (q % SKC)] : 0.0f;
    }
  };
  auto store_coords = [&](int cb, const float (&v)[NCV]) {
#pragma unroll
    for (int i = 0; i < NCV; ++i) {
      const int q = tid + NT * i;
      if (q < 6 * SKC) Kc[cb * 6 * SKC + q] = v[i];
    }
  };

  f16x med[NB][4], acc[NB][4];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
#pragma unroll
      for (int r = 0; r < 16; ++r) med[b][ch][r] = 0.0f;

  // med -> FP64 panel with the scales removed exactly. The panel holds every row of
  // the tile (rows at and past n_mu come out zero, the two density rows are written
  // afterwards) and every column of the last bra tile, so the writes need no
  // predicate; each lane's rows come in groups of four consecutive rows, whose
  // exponents are one 16-byte load and whose 16 panel values are loaded together.
  const long col = nb0 + (lane & 31);
  auto flush = [&](bool first) {
    // the row base goes through an opaque move so that the addresses below are
    // formed here and not hoisted, as live registers, out of the chunk loop
    long rbase = row0 + 32 * NB * wave + 4 * (lane >> 5);
    asm volatile("" : "+v"(rbase));
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const long rq = rbase + 32 * b + 8 * q;
        const int4 e4 = *(const int4*)(sA + rq);
        const int ev[4] = {e4.x, e4.y, e4.z, e4.w};
        double* p = panel + rq * bp + col;
        double v[4][4];
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
          for (int ch = 0; ch < 4; ++ch)
            v[rr][ch] = ldexp((double)med[b][ch][4 * q + rr], -(ev[rr] + (ch < 3 ? k.eg : k.es)));
        if (!first) {
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
#pragma unroll
            for (int ch = 0; ch < 4; ++ch) v[rr][ch] += p[((long)ch * rows_pad_panel + rr) * bp];
        }
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
#pragma unroll
          for (int ch = 0; ch < 4; ++ch) p[((long)ch * rows_pad_panel + rr) * bp] = v[rr][ch];
      }
  };

  // chunk c's fragments live in LDS buffer c & 1 and its coordinates in Kc buffer c & 1
  {
    float v[NCV];
    load_coords(c0, v);
    store_coords((int)(c0 & 1), v);
    load_coords(c0 + 1, v);
    store_coords((int)((c0 + 1) & 1), v);
    __syncthreads();
    const float* kcb = Kc + (c0 & 1) * 6 * SKC;
    h4 fr[NX][4][2];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float c[NX][6];
      read_coords(kcb, e, c);
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        PairState p;
        pair_stage_a(p, bxh, bxl, byh, byl, bzh, bzl, c[x]);
        pair_stage_b<EVEN, NQ>(p, k);
        float o[4];
        pair_stage_c(p, o);
        put(fr, x, o, e);
      }
      if (e == 3) store_half((int)(c0 & 1), fr, 0);
    }
    store_half((int)(c0 & 1), fr, 1);
  }
  __syncthreads();
  // A operand pipeline: k-steps ks and ks + 1 in flight while ks is used
  h8 a0[NB][2], a1[NB][2];
  {
    const long s0 = c0 * 8, s1 = c0 * 8 + 1 < last_ks ? c0 * 8 + 1 : last_ks;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      a0[b][0] = Aw[b * Ab + s0 * 128];
      a0[b][1] = Aw[b * Ab + s0 * 128 + 64];
      a1[b][0] = Aw[b * Ab + s1 * 128];
      a1[b][1] = Aw[b * Ab + s1 * 128 + 64];
    }
  }
  const f16x zero = {};
  // One chunk: 8 k-steps of MFMAs on buffer c & 1 while the next chunk's fragments
  // are generated into the other buffer. ZERO starts the chunk-pair accumulator.
  auto chunk = [&](long c, auto zero_tag) {
    constexpr bool ZERO = decltype(zero_tag)::value;
    const int buf = (int)(c & 1);
    const h8* Bb = Bs + (long)buf * 8 * 8 * 64 + lane;
    const float* kcb = Kc + ((c + 1) & 1) * 6 * SKC;   // coordinates of chunk c + 1
    float cv[NCV];
    load_coords(c + 2, cv);                            // for the generation during chunk c + 1
    h4 fr[NX][4][2];
    h8 bh[4], bl[4];
    float cn[NX][6];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      bh[ch] = Bb[(ch * 2 + 0) * 64];
      bl[ch] = Bb[(ch * 2 + 1) * 64];
    }
    read_coords(kcb, 0, cn);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      // loads issued ahead: A two k-steps on
      long ks2 = c * 8 + j + 2;
      if (ks2 > last_ks) ks2 = last_ks;
      h8 a2[NB][2];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        a2[b][0] = Aw[b * Ab + ks2 * 128];
        a2[b][1] = Aw[b * Ab + ks2 * 128 + 64];
      }
      PairState p[NX];
      // the k-step's MFMA issue takes precedence over the other wave's vector work on
      // this SIMD (measured faster, with the 1 : 4-5 interleave below)
      __builtin_amdgcn_s_setprio(1);
      XTC_FENCE();
      // group 1: A_lo K_hi beside stage A of this k-step's pairs
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
          acc[b][ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
              a0[b][1], bh[ch], (ZERO && j == 0) ? zero : acc[b][ch], 0, 0, 0);
#pragma unroll
      for (int x = 0; x < NX; ++x) pair_stage_a(p[x], bxh, bxl, byh, byl, bzh, bzl, cn[x]);
      XTC_INTERLEAVE(4 * NB, 4);
      XTC_FENCE();
      // the next k-step's pair coordinates, as soon as stage A has used this one's: LDS
      // reads return in order, so issued ahead of the next K_hi and K_lo they never hold
      // up a wait for those
      if (j < 7) read_coords(kcb, j + 1, cn);
      XTC_FENCE();
      // group 2: A_hi K_hi beside stage B
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
          acc[b][ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[b][0], bh[ch], acc[b][ch], 0, 0, 0);
#pragma unroll
      for (int x = 0; x < NX; ++x) pair_stage_b<EVEN, NQ>(p[x], k);
      XTC_INTERLEAVE(4 * NB, 5);
      XTC_FENCE();
      // the next k-step's K_hi, now that group 2 has read bh
      if (j < 7) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) bh[ch] = Bb[(((j + 1) * 4 + ch) * 2 + 0) * 64];
      }
      XTC_FENCE();
      // group 3: A_hi K_lo beside stage C and the fragment packing
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
          acc[b][ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[b][0], bl[ch], acc[b][ch], 0, 0, 0);
#pragma unroll
      for (int x = 0; x < NX; ++x) {
        float o[4];
        pair_stage_c(p[x], o);
        put(fr, x, o, j);
      }
      XTC_INTERLEAVE(4 * NB, 5);
      XTC_FENCE();
      // the next k-step's K_lo
      if (j < 7) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch) bl[ch] = Bb[(((j + 1) * 4 + ch) * 2 + 1) * 64];
      }
      __builtin_amdgcn_s_setprio(0);
      if (j == 3) store_half(buf ^ 1, fr, 0);
      XTC_FENCE();
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        a0[b][0] = a1[b][0];
        a0[b][1] = a1[b][1];
        a1[b][0] = a2[b][0];
        a1[b][1] = a2[b][1];
      }
    }
    store_half(buf ^ 1, fr, 1);
    store_coords(c & 1, cv);                           // chunk c + 2 into the freed buffer
    __syncthreads();
  };
  // chunks in pairs (the range has even length): the MFMA accumulator sums a pair
  // of chunks (256 ket points) before it is added to the FP32 medium sum
  for (long c = c0; c < c1; c += 2) {
    chunk(c, std::true_type{});
    chunk(c + 1, std::false_type{});
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) med[b][ch] += acc[b][ch];
  }
  flush(first_flush != 0);
}

// Every power even (and no o = 1 term): Q1 has odd powers of rbar only, Q2 even ones.
static bool even_powers(const EECoef& cf) {
  if (cf.c1 != 0.0) return false;
  for (int j = 0; j < MAXQ; ++j) {
    if (j % 2 == 0 && cf.q1[j] != 0.0) return false;
    if (j % 2 == 1 && cf.q2[j] != 0.0) return false;
  }
  return true;
}

static void split_coef(const EECoef& cf, SplitCoef* k, bool even) {
  *k = SplitCoef{};
  // |grad u| = |u'| <= d sum |c o| (t <= 1, rbar <= 1); pick 2^eg with bound 2^eg <= 2^14
  double bg = 0.0;
  for (int j = 0; j < MAXQ; ++j) bg += fabs(cf.q1[j]);
  bg *= cf.d;
  if (cf.c1 != 0.0) bg += fabs(cf.c1) * cf.d;
  int ex = 0;
  if (bg > 0.0) frexp(bg, &ex);        // bg < 2^ex
  k->eg = 14 - ex;                     // |grad u| 2^eg < 2^14
  k->es = 14 - 2 * ex;                 // |grad u|^2 <= bg^2 < 2^(2 ex), so |grad u|^2 2^es < 2^14
  const double sg = ldexp(1.0, k->eg), sh = ldexp(1.0, k->es / 2);
  k->d = (float)cf.d;
  k->c1 = (float)(cf.c1 * cf.d * sg);
  for (int j = 0; j < MAXQ; ++j) {
    const double a1 = cf.q1[j] * cf.d * sh, a2 = cf.q2[j] * cf.d * cf.d * sg;
    if (even) {
      if (j % 2 == 1) k->q1[j / 2] = (float)a1;   // e^j = e * (e^2)^(j/2)
      else k->q2[j / 2] = (float)a2;
    } else {
      k->q1[j] = (float)a1;
      k->q2[j] = (float)a2;
    }
  }
}

xtc_status stage1_split_f16(const Stage1Args& a, const EECoef& cf, void* scratch, size_t bytes,
                            hipStream_t st) {
  if (a.nch != 4) {
    set_error("split precision: the Laplacian channel is evaluated by the FP64 path only");
    return XTC_ERR_UNSUPPORTED;
  }
  if (a.bh) return stage1_split_bh(a, cf, scratch, bytes, st);
  SplitLayout S = split_layout(scratch, a.n_g, a.n_mu);
  // the kernel writes whole 256-row tiles and whole 32-column bra tiles
  XTC_REQUIRE(a.rows_pad >= S.rows_pad && a.bp >= ((a.bn + SB - 1) / SB) * SB,
              "split stage 1: panel smaller than its tiles");
  SplitCoef k;
  const bool even = even_powers(cf);
  split_coef(cf, &k, even);
  dim3 grid(cdiv(a.bn, SB), (unsigned)(S.rows_pad / SR));
  const size_t smem = sizeof(h8) * 2 * 8 * 8 * 64 + sizeof(float) * 2 * 6 * SKC;
  // compacted even-power polynomials of degree < 4 (powers up to 8) use the short form
  bool short_even = even;
  for (int j = 4; j < MAXQ / 2; ++j)
    if (k.q1[j] != 0.0f || k.q2[j] != 0.0f) short_even = false;
  // one launch per run of SMED chunks: the workgroups of a launch walk the same
  // stretch of A together, so its lines are shared in each L2
  const long nchunks = S.n_g_pad / SKC;
  for (long c0 = 0; c0 < nchunks; c0 += SMED) {
    const long c1 = c0 + SMED < nchunks ? c0 + SMED : nchunks;
    const int first = c0 == 0;
#define XTC_LAUNCH_SPLIT(EV, NQV)                                                              \
  hipLaunchKernelGGL((k_stage1_split<EV, NQV, SPLIT_WAVES>), grid, dim3(64 * SPLIT_WAVES), smem, st, (const h8*)S.A, \
                     (const int*)S.sA, (const float*)S.kc, S.n_g_pad, S.nks, a.xyz, a.n_g,    \
                     a.n_mu, a.b0, a.bn, k, a.panel, a.rows_pad, a.bp, c0, c1, first)
    const size_t tk = timing_begin(TM_S1_KERNEL, st);
    if (short_even) XTC_LAUNCH_SPLIT(true, 4);
    else if (even) XTC_LAUNCH_SPLIT(true, MAXQ / 2);
    else XTC_LAUNCH_SPLIT(false, MAXQ);
    timing_end(tk, st);
    XTC_CHECK_LAUNCH();
  }
#undef XTC_LAUNCH_SPLIT
  // the rho row (exact field and the ISDF-free energy-scale sums) in FP64
  if (!a.rho_rows) return XTC_OK;
  double* part = (double*)((char*)scratch + split_scratch_bytes(a.n_g, a.n_mu));
  return rho_row_f64(a, cf, part, st);
}

}  // namespace xtc
