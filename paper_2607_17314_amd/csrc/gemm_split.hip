// Split-precision NT GEMM on the CDNA4 matrix cores, for stage 2 of the
// contraction (the dense Xi / K-panel products) and the exchange intermediates:
//   C[m][n] (+)= sum_seg sum_k A_seg[m][k] s_seg[k] B_seg[n][k],
// A FP64 with k or m contiguous, B FP64 with k contiguous, C FP64 row-major. The
// segments (up to four products summed) are concatenated along k.
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
#include "timing.hpp"

namespace xtc {

typedef _Float16 g8 __attribute__((ext_vector_type(8)));
typedef float g16 __attribute__((ext_vector_type(16)));

constexpr int ST = 128;     // C tile (M and N)
constexpr int SK2 = 256;    // k padding: a pair of 128-point chunks

static long round_up(long x, long m) { return ((x + m - 1) / m) * m; }

// k-steps of one segment and of the concatenation (a whole number of chunk pairs)
static long seg_steps(long K) { return round_up(K, 16) / 16; }
static long total_steps(long K, int nseg) { return round_up(seg_steps(K) * nseg, SK2 / 16); }

size_t gemm_split_seg_scratch_bytes(long M, long N, long K, int nseg) {
  const long Mp = round_up(M, ST), Np = round_up(N, ST), nks = total_steps(K, nseg);
  Arena ar(nullptr, 0);
  ar.take<g8>((size_t)(Mp / 32) * nks * 128);
  ar.take<int>(Mp);
  ar.take<g8>((size_t)(Np / 32) * nks * 128);
  ar.take<int>(Np);
  return ar.used + 256;
}

size_t gemm_split_scratch_bytes(long M, long N, long K) {
  return gemm_split_seg_scratch_bytes(M, N, K, 1);
}

// One operand over its segments: value(r, k) = X[seg][r sm + k sk] s[seg][k], X in FP64
// or (Xf set) FP32.
struct SegOperand {
  const double* X[SPLIT_MAXSEG];
  const float* Xf[SPLIT_MAXSEG];
  const double* s[SPLIT_MAXSEG];
  long sm, sk;
  long K;
  int nseg;
};

__device__ inline double seg_value(const SegOperand& o, int seg, long r, long k) {
  const long i = r * o.sm + k * o.sk;
  double v = o.Xf[seg] ? (double)o.Xf[seg][i] : o.X[seg][i];
  if (o.s[seg]) v *= o.s[seg][k];
  return v;
}

__device__ inline int exp_of_max(double m) {
  int ex = 0;
  if (m > 0.0) {
    frexp(m, &ex);   // m = f 2^ex, f in [0.5, 1)
    return 15 - ex;
  }
  return 0;
}

// k contiguous (sk 1): one block per padded row; e with max |value| 2^e in [2^14, 2^15),
// 0 for rows past `rows` and for all-zero rows
__global__ __launch_bounds__(256) void k_row_exp(SegOperand o, long rows, int* __restrict__ e) {
  __shared__ double red[256];
  const long r = blockIdx.x;
  double m = 0.0;
  if (r < rows)
    for (int sg = 0; sg < o.nseg; ++sg) {
      const double* X = o.X[sg] ? o.X[sg] + r * o.sm : nullptr;
      const double* sc = o.s[sg];
      // FP64 rows that start on a 16-byte boundary: two values per load (the maximum does
      // not depend on the order it is taken in)
      if (X && !o.Xf[sg] && ((uintptr_t)X & 15) == 0 && (!sc || ((uintptr_t)sc & 15) == 0)) {
        const long K2 = o.K / 2;
        for (long k = threadIdx.x; k < K2; k += 256) {
          double2 v = ((const double2*)X)[k];
          if (sc) {
            const double2 t = ((const double2*)sc)[k];
            v.x *= t.x;
            v.y *= t.y;
          }
          m = fmax(m, fmax(fabs(v.x), fabs(v.y)));
        }
        if ((o.K & 1) && threadIdx.x == 0) m = fmax(m, fabs(seg_value(o, sg, r, o.K - 1)));
      } else {
        for (long k = threadIdx.x; k < o.K; k += 256) m = fmax(m, fabs(seg_value(o, sg, r, k)));
      }
    }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) e[r] = exp_of_max(red[0]);
}

// rows contiguous (sm 1): one thread per padded row, the k loop reads whole lines
__global__ __launch_bounds__(256) void k_col_exp(SegOperand o, long rows, long rows_pad,
                                                 int* __restrict__ e) {
  const long r = (long)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows_pad) return;
  double m = 0.0;
  if (r < rows)
    for (int sg = 0; sg < o.nseg; ++sg)
      for (long k = 0; k < o.K; ++k) m = fmax(m, fabs(seg_value(o, sg, r, k)));
  e[r] = exp_of_max(m);
}

// one thread per (row block, k-step, lane): 8 consecutive k of one row, split;
// k-step ks covers segment ks / nks_seg; steps past the last segment are zero
__global__ __launch_bounds__(256) void k_split_tiles(SegOperand o, long rows,
                                                     const int* __restrict__ e, long nrb, long nks,
                                                     long nks_seg, g8* __restrict__ T) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= nrb * nks * 64) return;
  const int lane = (int)(t % 64);
  const long ks = (t / 64) % nks;
  const long rb = t / (64 * nks);
  const long r = rb * 32 + (lane % 32);
  const int sg = (int)(ks / nks_seg);
  const long k0 = (ks % nks_seg) * 16 + 8 * (lane / 32);
  const double sc = ldexp(1.0, e[r]);
  g8 hi, lo;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const long k = k0 + q;
    double v = 0.0;
    if (r < rows && sg < o.nseg && k < o.K) v = seg_value(o, sg, r, k);
    v *= sc;
    const _Float16 h = (_Float16)(float)v;
    hi[q] = h;
    lo[q] = (_Float16)(float)(v - (double)(float)h);
  }
  const long base = ((rb * nks + ks) * 2) * 64 + lane;
  T[base] = hi;
  T[base + 64] = lo;
}

// The same split for a k-contiguous operand (sk 1), whose eight values per thread are one
// contiguous run of a row: loaded as 16-byte vectors where the run is aligned and whole.
__device__ __forceinline__ void load8(const double* p, double (&v)[8]) {
  const double2* q = (const double2*)p;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 t = q[i];
    v[2 * i] = t.x;
    v[2 * i + 1] = t.y;
  }
}
__device__ __forceinline__ void load8(const float* p, double (&v)[8]) {
  const float4* q = (const float4*)p;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float4 t = q[i];
    v[4 * i] = t.x;
    v[4 * i + 1] = t.y;
    v[4 * i + 2] = t.z;
    v[4 * i + 3] = t.w;
  }
}

__global__ __launch_bounds__(256) void k_split_tiles_k1(SegOperand o, long rows,
                                                        const int* __restrict__ e, long nrb,
                                                        long nks, long nks_seg,
                                                        g8* __restrict__ T) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= nrb * nks * 64) return;
  const int lane = (int)(t % 64);
  const long ks = (t / 64) % nks;
  const long rb = t / (64 * nks);
  const long r = rb * 32 + (lane % 32);
  const int sg = (int)(ks / nks_seg);
  const long k0 = (ks % nks_seg) * 16 + 8 * (lane / 32);
  double v[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (r < rows && sg < o.nseg && k0 < o.K) {
    const long off = r * o.sm + k0;
    const bool whole = k0 + 8 <= o.K;
    if (o.Xf[sg]) {
      const float* p = o.Xf[sg] + off;
      if (whole && ((uintptr_t)p & 15) == 0) load8(p, v);
      else
        for (int q = 0; q < 8; ++q) v[q] = k0 + q < o.K ? (double)p[q] : 0.0;
    } else {
      const double* p = o.X[sg] + off;
      if (whole && ((uintptr_t)p & 15) == 0) load8(p, v);
      else
        for (int q = 0; q < 8; ++q) v[q] = k0 + q < o.K ? p[q] : 0.0;
    }
    if (o.s[sg]) {
      double sv[8];
      const double* ps = o.s[sg] + k0;
      if (whole && ((uintptr_t)ps & 15) == 0) load8(ps, sv);
      else
        for (int q = 0; q < 8; ++q) sv[q] = k0 + q < o.K ? ps[q] : 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] *= sv[q];
    }
  }
  const double sc = ldexp(1.0, e[r]);
  g8 hi, lo;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const double x = v[q] * sc;
    const _Float16 h = (_Float16)(float)x;
    hi[q] = h;
    lo[q] = (_Float16)(float)(x - (double)(float)h);
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

// split both operands of C (+)= sum_seg A_seg diag(s_seg) B_seg^T and run the MFMA kernel
static xtc_status split_operand(const SegOperand& o, long rows, long rows_pad, long nks,
                                long nks_seg, int* e, g8* T, hipStream_t st, bool have_e) {
  if (have_e) {
  } else if (o.sk == 1) {
    hipLaunchKernelGGL(k_row_exp, dim3(rows_pad), dim3(256), 0, st, o, rows, e);
  } else {
    hipLaunchKernelGGL(k_col_exp, dim3(cdiv(rows_pad, 256)), dim3(256), 0, st, o, rows, rows_pad,
                       e);
  }
  XTC_CHECK_LAUNCH();
  if (o.sk == 1) {
    hipLaunchKernelGGL(k_split_tiles_k1, dim3(cdiv((rows_pad / 32) * nks * 64, 256)), dim3(256), 0,
                       st, o, rows, (const int*)e, rows_pad / 32, nks, nks_seg, T);
    XTC_CHECK_LAUNCH();
    return XTC_OK;
  }
  hipLaunchKernelGGL(k_split_tiles, dim3(cdiv((rows_pad / 32) * nks * 64, 256)), dim3(256), 0, st,
                     o, rows, (const int*)e, rows_pad / 32, nks, nks_seg, T);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

xtc_status gemm_split_seg(long M, long N, long K, const SplitSeg* seg, int nseg, double* C,
                          long ldc, bool accumulate, void* scratch, size_t bytes, hipStream_t st,
                          const int* eA_given, int timing_category) {
  XTC_REQUIRE(nseg >= 1 && nseg <= SPLIT_MAXSEG, "split GEMM: 1 to 4 segments");
  XTC_REQUIRE(bytes >= gemm_split_seg_scratch_bytes(M, N, K, nseg), "split GEMM: scratch too small");
  SegOperand a{}, b{};
  a.sm = seg[0].a_sm; a.sk = seg[0].a_sk; a.K = K; a.nseg = nseg;
  b.sm = seg[0].b_sn; b.sk = seg[0].b_sk; b.K = K; b.nseg = nseg;
  XTC_REQUIRE(a.sk == 1 || a.sm == 1, "split GEMM: A needs k or m contiguous");
  XTC_REQUIRE(b.sk == 1, "split GEMM: B needs k contiguous");
  for (int i = 0; i < nseg; ++i) {
    XTC_REQUIRE((seg[i].A != nullptr) != (seg[i].Af != nullptr) && seg[i].B,
                "split GEMM: null segment operand");
    XTC_REQUIRE(seg[i].a_sm == a.sm && seg[i].a_sk == a.sk && seg[i].b_sn == b.sm &&
                    seg[i].b_sk == b.sk,
                "split GEMM: segments need one layout");
    a.X[i] = seg[i].A; a.Xf[i] = seg[i].Af; a.s[i] = seg[i].s;
    b.X[i] = seg[i].B; b.Xf[i] = nullptr; b.s[i] = nullptr;
  }
  if (M <= 0 || N <= 0) return XTC_OK;
  const long Mp = round_up(M, ST), Np = round_up(N, ST);
  const long nks_seg = seg_steps(K), nks = total_steps(K, nseg);
  Arena ar(scratch, bytes);
  g8* At = ar.take<g8>((size_t)(Mp / 32) * nks * 128);
  int* eA = ar.take<int>(Mp);
  g8* Bt = ar.take<g8>((size_t)(Np / 32) * nks * 128);
  int* eB = ar.take<int>(Np);
  if (eA_given) eA = const_cast<int*>(eA_given);
  XTC_TRY(split_operand(a, M, Mp, nks, nks_seg, eA, At, st, eA_given != nullptr));
  XTC_TRY(split_operand(b, N, Np, nks, nks_seg, eB, Bt, st, false));
  const size_t tk = timing_category >= 0 ? timing_begin(timing_category, st) : (size_t)-1;
  hipLaunchKernelGGL(k_gemm_split_nt, dim3(Np / ST, Mp / ST), dim3(256), 0, st, (const g8*)At,
                     (const int*)eA, (const g8*)Bt, (const int*)eB, M, N, nks, C, ldc,
                     accumulate ? 1 : 0);
  timing_end(tk, st);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

xtc_status gemm_split_nt(const GemmArgs& g, void* scratch, size_t bytes, hipStream_t st) {
  XTC_REQUIRE(g.b_sk == 1 && g.c_sn == 1, "split GEMM: B needs k contiguous and C row-major");
  XTC_REQUIRE(g.alpha == 1.0 && (g.beta == 0.0 || g.beta == 1.0) && g.D == nullptr &&
                  g.epi == EPI_NONE && g.sn == nullptr && !g.lower_only,
              "split GEMM: only C = A s B^T or C += A s B^T");
  SplitSeg sg{g.A, g.a_sm, g.a_sk, g.s, g.B, g.b_sn, g.b_sk, g.A32};
  return gemm_split_seg(g.M, g.N, g.K, &sg, 1, g.C, g.c_sm, g.beta == 1.0, scratch, bytes, st);
}

}  // namespace xtc
