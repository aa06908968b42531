// Generic FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4f64) and small
// deterministic reductions. Used by the orbital GEMM, the fit (Gram, RHS,
// Cholesky updates, blocked triangular solves) and stage 2 of the contraction.
//
// Tile 64 x 64 x 16, 256 threads = 4 wave64s arranged 2 x 2; each wave owns a
// 32 x 32 sub-tile = 2 x 2 MFMA blocks of 16 x 16. Operands are staged through
// LDS k-major (row stride 65 doubles, so k-contiguous staging writes hit
// distinct banks); the next k-tile is prefetched into registers while the
// current one is multiplied.
//
// MFMA 16x16x4 f64 register layout (per lane l of the wave):
//   A operand: A[l % 16][l / 16]      B operand: B[l / 16][l % 16]
//   D (4 doubles): D[(l / 16) + 4 r][l % 16], r = 0..3  (measured on gfx950)
#include "common.hpp"

namespace xtc {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int GT = 64;    // tile M and N
constexpr int GK = 16;    // tile K
constexpr int LDS_LD = GT + 1;

template <bool A_KCONT, bool B_KCONT>
__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs g) {
  __shared__ double As[GK][LDS_LD];
  __shared__ double Bs[GK][LDS_LD];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // Tile order: the M tile runs fastest, so the workgroups that read the same
  // column panel of B run at the same time, and consecutive workgroup ids (which
  // the hardware deals to the 8 XCDs in turn) are spread so that each XCD takes a
  // contiguous run of tiles and shares those panels in its own L2.
  const long n_mt = (g.M + GT - 1) / GT, n_tiles = n_mt * ((g.N + GT - 1) / GT);
  const long per_xcd = (n_tiles + 7) / 8;
  const long t = (long)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (t >= n_tiles) return;   // the whole workgroup, before any barrier
  const long m0 = (t % n_mt) * GT;
  const long n0 = (t / n_mt) * GT;
  if (g.lower_only && m0 + GT - 1 < n0) return;

  double ra[4], rb[4];
  auto load = [&](long k0) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int e = tid + 256 * j;
      int mm, kk;
      if (A_KCONT) { kk = e % GK; mm = e / GK; } else { mm = e % GT; kk = e / GT; }
      long m = m0 + mm, k = k0 + kk;
      double v = 0.0;
      if (m < g.M && k < g.K) {
        v = g.A[m * g.a_sm + k * g.a_sk];
        if (g.s) v *= g.s[k];
      }
      ra[j] = v;
      int nn;
      if (B_KCONT) { kk = e % GK; nn = e / GK; } else { nn = e % GT; kk = e / GT; }
      long n = n0 + nn;
      k = k0 + kk;
      rb[j] = (n < g.N && k < g.K) ? g.B[k * g.b_sk + n * g.b_sn] : 0.0;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int e = tid + 256 * j;
      int mm, kk;
      if (A_KCONT) { kk = e % GK; mm = e / GK; } else { mm = e % GT; kk = e / GT; }
      As[kk][mm] = ra[j];
      int nn;
      if (B_KCONT) { kk = e % GK; nn = e / GK; } else { nn = e % GT; kk = e / GT; }
      Bs[kk][nn] = rb[j];
    }
  };

  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = (d4){0.0, 0.0, 0.0, 0.0};

  const int li = lane & 15, lk = lane >> 4;
  load(0);
  for (long k0 = 0; k0 < g.K; k0 += GK) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + GK < g.K) load(k0 + GK);
#pragma unroll
    for (int s = 0; s < GK / 4; ++s) {
      double a0 = As[4 * s + lk][32 * wm + li];
      double a1 = As[4 * s + lk][32 * wm + 16 + li];
      double b0 = Bs[4 * s + lk][32 * wn + li];
      double b1 = Bs[4 * s + lk][32 * wn + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        long m = m0 + 32 * wm + 16 * bi + lk + 4 * r;
        long n = n0 + 32 * wn + 16 * bj + li;
        if (m >= g.M || n >= g.N) continue;
        double v = g.alpha * acc[bi][bj][r];
        if (g.sn) v *= g.sn[n];
        if (g.beta != 0.0) {
          const double* D = g.D ? g.D : g.C;
          v += g.beta * D[m * g.c_sm + n * g.c_sn];
        }
        if (g.epi == EPI_MUL_E) v *= g.E[m * g.e_sm + n * g.e_sn];
        else if (g.epi == EPI_SQUARE) v *= v;
        g.C[m * g.c_sm + n * g.c_sn] = v;
      }
}

xtc_status gemm_f64(const GemmArgs& g, hipStream_t st) {
  XTC_REQUIRE(g.A32 == nullptr, "gemm_f64: FP32 operands are for the split GEMM only");
  if (g.M <= 0 || g.N <= 0) return XTC_OK;
  if (g.K <= 0) {
    set_error("gemm_f64: K must be positive");
    return XTC_ERR_INVALID_ARG;
  }
  const long n_tiles = ((g.M + GT - 1) / GT) * ((g.N + GT - 1) / GT);
  const long n_wg = 8 * ((n_tiles + 7) / 8);
  if (n_wg > 0x7fffffffL) {
    set_error("gemm_f64: too many tiles for one launch");
    return XTC_ERR_INVALID_ARG;
  }
  const dim3 grid((unsigned)n_wg);
  bool ak = (g.a_sk == 1), bk = (g.b_sk == 1);
  if (ak && bk) hipLaunchKernelGGL((k_gemm_f64<true, true>), grid, dim3(256), 0, st, g);
  else if (ak && !bk) hipLaunchKernelGGL((k_gemm_f64<true, false>), grid, dim3(256), 0, st, g);
  else if (!ak && bk) hipLaunchKernelGGL((k_gemm_f64<false, true>), grid, dim3(256), 0, st, g);
  else hipLaunchKernelGGL((k_gemm_f64<false, false>), grid, dim3(256), 0, st, g);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

// ---------------------------------------------------------------------------
// Deterministic FP64 sum: 256-thread blocks, each block sums a contiguous
// stretch in a fixed shuffle/LDS tree; a second single-block pass sums the
// partials in order.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__device__ double block_sum_256(double v) {
  __shared__ double part[4];
  v = wave_sum(v);
  int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) part[wave] = v;
  __syncthreads();
  double r = (part[0] + part[1]) + (part[2] + part[3]);
  return r;
}

__global__ __launch_bounds__(256) void k_reduce_stage(const double* x, long n, long per_block,
                                                      double* out) {
  long b0 = (long)blockIdx.x * per_block;
  long b1 = b0 + per_block < n ? b0 + per_block : n;
  double v = 0.0;
  for (long i = b0 + threadIdx.x; i < b1; i += 256) v += x[i];
  v = block_sum_256(v);
  if (threadIdx.x == 0) out[blockIdx.x] = v;
}

xtc_status reduce_sum_f64(const double* x, long n, double* out, double* scratch, hipStream_t st) {
  // scratch must hold 1024 doubles
  long per = (n + 1023) / 1024;
  if (per < 256) per = 256;
  unsigned nb = cdiv(n, per);
  if (nb == 0) nb = 1;
  hipLaunchKernelGGL(k_reduce_stage, dim3(nb), dim3(256), 0, st, x, n, per, scratch);
  XTC_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_reduce_stage, dim3(1), dim3(256), 0, st, (const double*)scratch, (long)nb,
                     (long)nb, out);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

}  // namespace xtc
