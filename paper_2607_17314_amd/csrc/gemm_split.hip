// Split-precision NT GEMM on the CDNA4 matrix cores, for stage 2 of the
// contraction (the dense Xi / K-panel products):
//   C[m][n] (+)= sum_k A[m][k] s[k] B[n][k],
// A and B FP64 with k contiguous, C FP64 row-major.
//
// Each operand is first cut into FP16 pairs, x 2^e ~= x_hi + x_lo, with one
// power-of-two exponent e per row (row max scaled into [2^14, 2^15)), and stored
// in the MFMA-native tiled layout [row block of 32][k-step of 16][hi, lo][lane],
// lane l holding row 32 rb + l % 32, k = 16 ks + 8 (l / 32) + 0..7. That layout is
// the A operand of v_mfma_f32_32x32x16_f16 for A and, read as [n][k], its B
// operand for B, so both stream from HBM straight into registers.
// Every product is A_hi B_hi + A_hi B_lo + A_lo B_hi; the MFMA accumulator sums a
// pair of 128-point k-chunks, an FP32 medium sum takes the rest of the k range,
// and the exponents are removed exactly in the FP64 epilogue.
//
// Workgroup 256 threads = 4 waves over a 128 x 128 tile of C; wave (wm, wn) owns
// the 64 x 64 sub-tile = 2 x 2 MFMA blocks. The k-step ahead is loaded while the
// current one is multiplied; scheduling fences keep those loads in place.
#include "common.hpp"
#include "gemm_split.hpp"

namespace xtc {

typedef _Float16 g8 __attribute__((ext_vector_type(8)));
typedef float g16 __attribute__((ext_vector_type(16)));

constexpr int ST = 128;     // C tile (M and N)
constexpr int SK2 = 256;    // k padding: a pair of 128-point chunks

struct SplitTiles {
  g8* t;
  int* e;
};

static long round_up(long x, long m) { return ((x + m - 1) / m) * m; }

size_t gemm_split_scratch_bytes(long M, long N, long K) {
  const long Mp = round_up(M, ST), Np = round_up(N, ST), Kp = round_up(K, SK2);
  Arena ar(nullptr, 0);
  ar.take<g8>((size_t)(Mp / 32) * (Kp / 16) * 128);
  ar.take<int>(Mp);
  ar.take<g8>((size_t)(Np / 32) * (Kp / 16) * 128);
  ar.take<int>(Np);
  return ar.used + 256;
}

// one block per padded row: e with max_k |x[r][k] s[k]| 2^e in [2^14, 2^15); 0 for
// rows past `rows` and for all-zero rows
__global__ __launch_bounds__(256) void k_row_exp(const double* __restrict__ X, long ld, long rows,
                                                 long K, const double* __restrict__ s,
                                                 int* __restrict__ e) {
  __shared__ double red[256];
  const long r = blockIdx.x;
  double m = 0.0;
  if (r < rows)
    for (long k = threadIdx.x; k < K; k += 256) {
      double v = X[r * ld + k];
      if (s) v *= s[k];
      m = fmax(m, fabs(v));
    }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int ex = 0, out = 0;
    if (red[0] > 0.0) {
      frexp(red[0], &ex);   // red = f 2^ex, f in [0.5, 1)
      out = 15 - ex;
    }
    e[r] = out;
  }
}

// one thread per (row block, k-step, lane): 8 consecutive k of one row, split
__global__ __launch_bounds__(256) void k_split_tiles(const double* __restrict__ X, long ld,
                                                     long rows, long K, const double* __restrict__ s,
                                                     const int* __restrict__ e, long nrb, long nks,
                                                     g8* __restrict__ T) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= nrb * nks * 64) return;
  const int lane = (int)(t % 64);
  const long ks = (t / 64) % nks;
  const long rb = t / (64 * nks);
  const long r = rb * 32 + (lane % 32);
  const long k0 = ks * 16 + 8 * (lane / 32);
  const double sc = ldexp(1.0, e[r]);
  g8 hi, lo;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const long k = k0 + q;
    double v = 0.0;
    if (r < rows && k < K) {
      v = X[r * ld + k];
      if (s) v *= s[k];
    }
    v *= sc;
    const _Float16 h = (_Float16)(float)v;
    hi[q] = h;
    lo[q] = (_Float16)(float)(v - (double)(float)h);
  }
  const long base = ((rb * nks + ks) * 2) * 64 + lane;
  T[base] = hi;
  T[base + 64] = lo;
}

#define XTC_GFENCE() __builtin_amdgcn_sched_barrier(0)

__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2, 2)))
void k_gemm_split_nt(const g8* __restrict__ At, const int* __restrict__ eA,
                     const g8* __restrict__ Bt, const int* __restrict__ eB, long M, long N,
                     long nks, double* __restrict__ C, long ldc, int accumulate) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long m0 = (long)blockIdx.y * ST + 64 * wm, n0 = (long)blockIdx.x * ST + 64 * wn;
  const g8* Aw = At + (m0 / 32) * nks * 128 + lane;
  const g8* Bw = Bt + (n0 / 32) * nks * 128 + lane;
  const long blk = nks * 128;   // stride between consecutive row blocks
  const long nchunks = nks / 8;

  g16 acc[2][2], med[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) med[i][j][r] = 0.0f;

  // operands of one k-step: [block][hi, lo]
  g8 a0[2][2], b0[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    a0[i][0] = Aw[i * blk];
    a0[i][1] = Aw[i * blk + 64];
    b0[i][0] = Bw[i * blk];
    b0[i][1] = Bw[i * blk + 64];
  }
  const g16 zero = {};
  auto chunk = [&](long c, auto zero_tag) {
    constexpr bool ZERO = decltype(zero_tag)::value;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      long ks1 = c * 8 + j + 1;
      if (ks1 > nks - 1) ks1 = nks - 1;
      g8 a1[2][2], b1[2][2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a1[i][0] = Aw[i * blk + ks1 * 128];
        a1[i][1] = Aw[i * blk + ks1 * 128 + 64];
        b1[i][0] = Bw[i * blk + ks1 * 128];
        b1[i][1] = Bw[i * blk + ks1 * 128 + 64];
      }
      XTC_GFENCE();
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[i][q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
              a0[i][1], b0[q][0], (ZERO && j == 0) ? zero : acc[i][q], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[i][q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[i][0], b0[q][0], acc[i][q], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int q = 0; q < 2; ++q)
          acc[i][q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0[i][0], b0[q][1], acc[i][q], 0, 0, 0);
      XTC_GFENCE();
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          a0[i][h] = a1[i][h];
          b0[i][h] = b1[i][h];
        }
    }
  };
  for (long c = 0; c < nchunks; c += 2) {
    chunk(c, std::true_type{});
    chunk(c + 1, std::false_type{});
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int q = 0; q < 2; ++q) med[i][q] += acc[i][q];
  }
  // epilogue: D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] of each 32 x 32 block
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const long n = n0 + 32 * q + (lane & 31);
    if (n >= N) continue;
    const int en = eB[n];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long m = m0 + 32 * i + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (m < M) {
          const double v = ldexp((double)med[i][q][r], -(eA[m] + en));
          double* p = C + m * ldc + n;
          *p = accumulate ? *p + v : v;
        }
      }
  }
}

xtc_status gemm_split_nt(const GemmArgs& g, void* scratch, size_t bytes, hipStream_t st) {
  XTC_REQUIRE(g.a_sk == 1 && g.b_sk == 1 && g.c_sn == 1,
              "split GEMM: operands need k contiguous and C row-major");
  XTC_REQUIRE(g.alpha == 1.0 && (g.beta == 0.0 || g.beta == 1.0) && g.D == nullptr &&
                  g.epi == EPI_NONE && g.sn == nullptr && !g.lower_only,
              "split GEMM: only C = A s B^T or C += A s B^T");
  XTC_REQUIRE(bytes >= gemm_split_scratch_bytes(g.M, g.N, g.K), "split GEMM: scratch too small");
  if (g.M <= 0 || g.N <= 0) return XTC_OK;
  const long Mp = round_up(g.M, ST), Np = round_up(g.N, ST), Kp = round_up(g.K, SK2);
  const long nks = Kp / 16;
  Arena ar(scratch, bytes);
  g8* At = ar.take<g8>((size_t)(Mp / 32) * nks * 128);
  int* eA = ar.take<int>(Mp);
  g8* Bt = ar.take<g8>((size_t)(Np / 32) * nks * 128);
  int* eB = ar.take<int>(Np);
  hipLaunchKernelGGL(k_row_exp, dim3(Mp), dim3(256), 0, st, g.A, g.a_sm, g.M, g.K, g.s, eA);
  XTC_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_split_tiles, dim3(cdiv((Mp / 32) * nks * 64, 256)), dim3(256), 0, st, g.A,
                     g.a_sm, g.M, g.K, g.s, (const int*)eA, Mp / 32, nks, At);
  XTC_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_row_exp, dim3(Np), dim3(256), 0, st, g.B, g.b_sn, g.N, g.K,
                     (const double*)nullptr, eB);
  XTC_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_split_tiles, dim3(cdiv((Np / 32) * nks * 64, 256)), dim3(256), 0, st, g.B,
                     g.b_sn, g.N, g.K, (const double*)nullptr, (const int*)eB, Np / 32, nks, Bt);
  XTC_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_gemm_split_nt, dim3(Np / ST, Mp / ST), dim3(256), 0, st, (const g8*)At,
                     (const int*)eA, (const g8*)Bt, (const int*)eB, g.M, g.N, nks, g.C, g.c_sm,
                     g.beta == 1.0 ? 1 : 0);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

}  // namespace xtc
