// Stage 1 of the grid-pair contraction with FP16 split products on the
// CDNA4 matrix cores:
//   panel[ch][row][g] = sum_g' A[row][g'] K_ch(g, g'),  A = [w xi ; w rho].
// Both operands are split into an FP16 pair, x ~= x_hi + x_lo, after a
// power-of-two scaling (A per row, K per channel), and every product is taken
// as A_hi K_hi + A_hi K_lo + A_lo K_hi with v_mfma_f32_32x32x16_f16 (the
// dropped A_lo K_lo term is 2^-22 relative). Accumulation is three-level:
// the MFMA accumulator over a 128-point ket chunk, an FP32 sum of 64 chunks,
// then FP64 in the output panel; the scales are removed exactly on flush.
//
// Workgroup: 512 threads = 8 waves, tile 256 rows x 32 bra points; wave w owns
// rows 32w..32w+31. Per ket chunk each thread generates the 4 kernel channels
// of 8 (bra, ket) pairs in FP32 (pair differences formed in double-float, so
// close pairs keep their relative accuracy) and writes them, split, to LDS
// directly in the MFMA B-operand layout (double-buffered, 128 KB); the A
// operand streams from a pre-split, MFMA-native tiled copy in HBM.
//
// MFMA 32x32x16 f16 layouts (measured on gfx950), lane l, element e, register r:
//   A[l % 32][8 (l / 32) + e]   B[8 (l / 32) + e][l % 32]
//   D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
#include "contract.hpp"

namespace xtc {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f16x __attribute__((ext_vector_type(16)));

constexpr int SR = 256;        // rows per workgroup
constexpr int SB = 32;         // bra points per workgroup
constexpr int SKC = 128;       // ket points per chunk (8 k-steps of 16)
constexpr int SMED = 64;       // chunks per FP32 medium sum (then FP64)

struct SplitCoef {
  float d;
  float c1;
  float q1[MAXQ];
  float q2[MAXQ];
  int n1, n2;
  float sg;     // 2^(channel scale) for the gradient channels
  float ss;     // 2^(channel scale) for |grad u|^2
  int eg, es;   // the exponents
};

struct SplitLayout {
  h8* A;            // [rows_pad / 32][nks][2][64]
  int* sA;          // [rows_pad] per-row exponent
  float* kc;        // [6][n_g_pad]: x_hi, y_hi, z_hi, x_lo, y_lo, z_lo
  long rows_pad;    // multiple of SR
  long n_g_pad;     // multiple of SKC
  long nks;         // n_g_pad / 16
};

static SplitLayout split_layout(void* base, long n_g, int n_mu) {
  SplitLayout S;
  S.rows_pad = ((n_mu + SR - 1) / SR) * SR;
  S.n_g_pad = ((n_g + SKC - 1) / SKC) * SKC;
  S.nks = S.n_g_pad / 16;
  Arena ar(base, (size_t)-1);
  S.A = ar.take<h8>((size_t)(S.rows_pad / 32) * S.nks * 2 * 64);
  S.sA = ar.take<int>(S.rows_pad);
  S.kc = ar.take<float>(6 * (size_t)S.n_g_pad);
  return S;
}

size_t split_scratch_bytes(long n_g, int n_mu) {
  Arena ar(nullptr, 0);
  long rows_pad = ((n_mu + SR - 1) / SR) * SR;
  long n_g_pad = ((n_g + SKC - 1) / SKC) * SKC;
  ar.take<h8>((size_t)(rows_pad / 32) * (n_g_pad / 16) * 2 * 64);
  ar.take<int>(rows_pad);
  ar.take<float>(6 * (size_t)n_g_pad);
  return ar.used + 256;
}

size_t rho_row_scratch_bytes(long bp);

// --- preparation --------------------------------------------------------------

__device__ __forceinline__ double a_value(const double* __restrict__ w, const double* __restrict__ xi,
                                          const double* __restrict__ rho, long n_g, int n_mu,
                                          long row, long g) {
  (void)rho;
  if (g >= n_g || row >= n_mu) return 0.0;
  return w[g] * xi[row * n_g + g];
}

// one block per row: exponent s with max |A_row| 2^s in [2^14, 2^15)
__global__ __launch_bounds__(256) void k_row_scale(const double* __restrict__ w,
                                                   const double* __restrict__ xi,
                                                   const double* __restrict__ rho, long n_g,
                                                   int n_mu, int* __restrict__ sA) {
  __shared__ double red[256];
  const long row = blockIdx.x;
  double m = 0.0;
  for (long g = threadIdx.x; g < n_g; g += 256) m = fmax(m, fabs(a_value(w, xi, rho, n_g, n_mu, row, g)));
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
__global__ __launch_bounds__(256) void k_split_A(const double* __restrict__ w,
                                                 const double* __restrict__ xi,
                                                 const double* __restrict__ rho, long n_g,
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
    const double v = a_value(w, xi, rho, n_g, n_mu, row, k0 + e) * sc;
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
  hipLaunchKernelGGL(k_row_scale, dim3(a.n_mu), dim3(256), 0, st, a.w, a.xi, a.rho, a.n_g,
                     a.n_mu, S.sA);
  XTC_CHECK_LAUNCH();
  const long nrb = S.rows_pad / 32;
  hipLaunchKernelGGL(k_split_A, dim3(cdiv(nrb * S.nks * 64, 256)), dim3(256), 0, st, a.w, a.xi,
                     a.rho, a.n_g, a.n_mu, (const int*)S.sA, S.nks, nrb, S.A);
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

// Four scaled channels of one pair: (d_x u, d_y u, d_z u) 2^eg and |grad u|^2 2^es.
// EVEN: every power o_k is even (no o = 1 term), so Q1(e) = e P1(e^2), Q2(e) = P2(e^2)
// with the coefficients of q1, q2 stored compacted (q1[i] = coef of e^(2i+1), q2[i] of e^(2i)).
template <bool EVEN, int NQ>
__device__ __forceinline__ void split_channels(const SplitCoef& k, float dx, float dy, float dz,
                                               float* o) {
  const float r2 = dx * dx + dy * dy + dz * dz;
  const float r = __builtin_amdgcn_sqrtf(r2);   // v_sqrt_f32, 1 ulp
  const float dr = k.d * r;
  const float t = __builtin_amdgcn_rcpf(1.0f + dr);
  const float e = dr * t;
  const float t2 = t * t;
  float up, f;
  if (EVEN) {
    const float e2 = e * e;
    up = k.d * t2 * e * hornerf<NQ>(k.q1, e2);
    f = k.d * k.d * t2 * t * hornerf<NQ>(k.q2, e2);
  } else {
    up = k.d * t2 * hornerf<MAXQ>(k.q1, e);
    f = k.d * k.d * t2 * t * hornerf<MAXQ>(k.q2, e);
    if (k.c1 != 0.0f && r > 0.0f) f += k.c1 * k.d * t2 / r;
  }
  const float fs = f * k.sg;
  o[0] = fs * dx;
  o[1] = fs * dy;
  o[2] = fs * dz;
  o[3] = up * up * k.ss;
}

template <bool EVEN, int NQ>
__global__ __launch_bounds__(512) void k_stage1_split(const h8* __restrict__ At,
                                                      const int* __restrict__ sA,
                                                      const float* __restrict__ kc, long n_g_pad,
                                                      long nks, const double* __restrict__ xyz,
                                                      long n_g, int n_mu, long b0, long bn,
                                                      SplitCoef k, double* __restrict__ panel,
                                                      long rows_pad_panel, long bp) {
  extern __shared__ h8 Bs[];   // [2][8 ksteps][4 ch][2 hl][64 lanes], then coordinates
  // ket coordinates of a chunk, double-buffered: [2][6][SKC] floats after the fragments
  float* Kc = (float*)(Bs + 2 * 8 * 8 * 64);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long row0 = (long)blockIdx.y * SR;
  const long nb0 = (long)blockIdx.x * SB;
  // generation role: k-step j of the chunk, destination lane ld
  const int gj = tid >> 6, ld = tid & 63;
  long bra = b0 + nb0 + (ld & 31);
  if (bra > b0 + bn - 1) bra = b0 + bn - 1;
  const double bx = xyz[bra], by = xyz[n_g + bra], bz = xyz[2 * n_g + bra];
  const float bxh = (float)bx, byh = (float)by, bzh = (float)bz;
  const float bxl = (float)(bx - (double)bxh), byl = (float)(by - (double)byh),
              bzl = (float)(bz - (double)bzh);
  const long rb = (row0 / 32) + wave;          // this wave's 32-row block
  const h8* Aw = At + rb * nks * 2 * 64 + lane;
  const long nchunks = n_g_pad / SKC;

  // One pair of the next chunk is generated per k-step of the current chunk, so the
  // vector units work in the shadow of the matrix-core instructions; the fragments
  // are written to the other LDS buffer after the chunk's last k-step. Ket
  // coordinates come from LDS, loaded from HBM one chunk earlier still.
  const int kofs = 16 * gj + 8 * (ld >> 5);
  auto gen_pair = [&](const float* kcb, int e, h8 (&fr)[4][2]) {
    const int g = kofs + e;
    const float dx = (bxh - kcb[g]) + (bxl - kcb[3 * SKC + g]);
    const float dy = (byh - kcb[SKC + g]) + (byl - kcb[4 * SKC + g]);
    const float dz = (bzh - kcb[2 * SKC + g]) + (bzl - kcb[5 * SKC + g]);
    float o[4];
    split_channels<EVEN, NQ>(k, dx, dy, dz, o);
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      const _Float16 h = (_Float16)o[ch];
      fr[ch][0][e] = h;
      fr[ch][1][e] = (_Float16)(o[ch] - (float)h);
    }
  };
  auto store_frags = [&](int buf, h8 (&fr)[4][2]) {
    h8* dst = Bs + ((long)(buf * 8 + gj) * 8) * 64 + ld;
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      dst[(ch * 2 + 0) * 64] = fr[ch][0];
      dst[(ch * 2 + 1) * 64] = fr[ch][1];
    }
  };
  // coordinates of chunk c: 6 x SKC floats = 768, two per thread (threads 0..383)
  auto load_coords = [&](long c, float& v0, float& v1) {
    v0 = v1 = 0.0f;
    if (tid < 384 && c < nchunks) {
      const int q = tid * 2, comp = q / SKC, off = q % SKC;
      const float* src = kc + (long)comp * n_g_pad + c * SKC + off;
      v0 = src[0];
      v1 = src[1];
    }
  };
  auto store_coords = [&](int cb, float v0, float v1) {
    if (tid < 384) {
      Kc[cb * 6 * SKC + tid * 2] = v0;
      Kc[cb * 6 * SKC + tid * 2 + 1] = v1;
    }
  };

  f16x med[4], acc[4];
#pragma unroll
  for (int ch = 0; ch < 4; ++ch)
#pragma unroll
    for (int r = 0; r < 16; ++r) med[ch][r] = 0.0f;

  // rows and scales owned by this lane (16 rows of one column)
  const long col = nb0 + (lane & 31);
  auto flush = [&](bool first) {
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
      const int ek = ch < 3 ? k.eg : k.es;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long row = row0 + 32 * wave + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (row < n_mu && col < bn) {
          const double v = ldexp((double)med[ch][r], -(sA[row] + ek));
          double* p = panel + ((long)ch * rows_pad_panel + row) * bp + col;
          *p = first ? v : *p + v;
        }
        med[ch][r] = 0.0f;
      }
    }
  };

  {
    float v0, v1;
    load_coords(0, v0, v1);
    store_coords(0, v0, v1);
    load_coords(1, v0, v1);
    store_coords(1, v0, v1);
    __syncthreads();
    h8 fr[4][2];
#pragma unroll
    for (int e = 0; e < 8; ++e) gen_pair(Kc, e, fr);
    store_frags(0, fr);
  }
  __syncthreads();
  bool first_flush = true;
  const long last_ks = nks - 1;
  h8 a0h = Aw[0], a0l = Aw[64];
  for (long c = 0; c < nchunks; ++c) {
    const int buf = (int)(c & 1);
    const bool more = c + 1 < nchunks;
    const h8* Bb = Bs + (long)buf * 8 * 8 * 64 + lane;
    const float* kcb = Kc + ((c + 1) & 1) * 6 * SKC;   // coordinates of chunk c + 1
    float cv0, cv1;
    load_coords(c + 2, cv0, cv1);                      // for the generation during chunk c + 1
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[ch][r] = 0.0f;
    h8 fr[4][2];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      long ks1 = c * 8 + j + 1;                        // A one k-step ahead
      if (ks1 > last_ks) ks1 = last_ks;
      const h8 a1h = Aw[ks1 * 128];
      const h8 a1l = Aw[ks1 * 128 + 64];
      h8 b[4];
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) b[ch] = Bb[((j * 4 + ch) * 2 + 0) * 64];
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) acc[ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0l, b[ch], acc[ch], 0, 0, 0);
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) acc[ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0h, b[ch], acc[ch], 0, 0, 0);
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) b[ch] = Bb[((j * 4 + ch) * 2 + 1) * 64];
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) acc[ch] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a0h, b[ch], acc[ch], 0, 0, 0);
      if (more) gen_pair(kcb, j, fr);
      a0h = a1h;
      a0l = a1l;
    }
    if (more) store_frags(buf ^ 1, fr);
    store_coords(c & 1, cv0, cv1);                     // chunk c + 2 into the freed buffer
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) med[ch] += acc[ch];
    if ((c + 1) % SMED == 0 || c + 1 == nchunks) {
      flush(first_flush);
      first_flush = false;
    }
    __syncthreads();
  }
}

// Every power even (and no o = 1 term): Q1 has odd powers of rbar only, Q2 even ones.
// The two density rows of the panel in FP64 on the vector units: row n_mu with
// rho_gamma (field A_gamma and T3rho) and row n_mu + 1 with the ISDF density
// rhot (H_{g,c}, which as a sum over N_mu split-precision rows would cancel):
// one thread per bra point and ket segment; the segments' partial sums are added
// in a fixed order by k_rho_row_sum.
constexpr int RHO_SEG = 16;

__global__ __launch_bounds__(256) void k_rho_row(const double* __restrict__ xyz,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ rho,
                                                 const double* __restrict__ rhot, long n_g,
                                                 long b0, long bn, EECoef cf,
                                                 double* __restrict__ part) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  const long seg = blockIdx.y;
  const long per = (n_g + RHO_SEG - 1) / RHO_SEG;
  const long k0 = seg * per, k1 = k0 + per < n_g ? k0 + per : n_g;
  long b = b0 + t;
  if (b > b0 + bn - 1) b = b0 + bn - 1;
  const double bx = xyz[b], by = xyz[n_g + b], bz = xyz[2 * n_g + b];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, h0 = 0.0, h1 = 0.0, h2 = 0.0, h3 = 0.0;
  for (long g = k0; g < k1; ++g) {
    const double dx = bx - xyz[g], dy = by - xyz[n_g + g], dz = bz - xyz[2 * n_g + g];
    const double r = sqrt(dx * dx + dy * dy + dz * dz);
    const double tt = 1.0 / (1.0 + cf.d * r);
    const double e = cf.d * r * tt;
    const double t2 = tt * tt;
    double p1 = 0.0, p2 = 0.0;
    for (int j = cf.n1 - 1; j >= 0; --j) p1 = p1 * e + cf.q1[j];
    for (int j = cf.n2 - 1; j >= 0; --j) p2 = p2 * e + cf.q2[j];
    const double up = cf.d * t2 * p1;
    double f = cf.d * cf.d * t2 * tt * p2;
    if (cf.c1 != 0.0 && r > 0.0) f += cf.c1 * cf.d * t2 / r;
    const double a = w[g] * rho[g];
    const double at = w[g] * rhot[g];
    const double fx = f * dx, fy = f * dy, fz = f * dz, sq = up * up;
    s0 += a * fx;
    s1 += a * fy;
    s2 += a * fz;
    s3 += a * sq;
    h0 += at * fx;
    h1 += at * fy;
    h2 += at * fz;
    h3 += at * sq;
  }
  if (t < bn) {
    double* p = part + (seg * 8) * bn + t;
    p[0] = s0;
    p[bn] = s1;
    p[2 * bn] = s2;
    p[3 * bn] = s3;
    p[4 * bn] = h0;
    p[5 * bn] = h1;
    p[6 * bn] = h2;
    p[7 * bn] = h3;
  }
}

__global__ __launch_bounds__(256) void k_rho_row_sum(const double* __restrict__ part, long bn,
                                                     int n_mu, double* __restrict__ panel,
                                                     long rows_pad, long bp) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= bn) return;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    double v = 0.0;
    for (int sgm = 0; sgm < RHO_SEG; ++sgm) v += part[(sgm * 8 + q) * bn + t];
    panel[((long)(q & 3) * rows_pad + n_mu + (q >> 2)) * bp + t] = v;
  }
}

size_t rho_row_scratch_bytes(long bp) { return sizeof(double) * RHO_SEG * 8 * (size_t)bp + 256; }

xtc_status rho_row_f64(const Stage1Args& a, const EECoef& cf, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_rho_row, dim3(cdiv(a.bn, 256), RHO_SEG), dim3(256), 0, st, a.xyz, a.w, a.rho,
                     a.rhot, a.n_g, a.b0, a.bn, cf, part);
  XTC_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_rho_row_sum, dim3(cdiv(a.bn, 256)), dim3(256), 0, st, (const double*)part,
                     a.bn, a.n_mu, a.panel, a.rows_pad, a.bp);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

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
  k->d = (float)cf.d;
  k->c1 = (float)cf.c1;
  for (int j = 0; j < MAXQ; ++j) {
    if (even) {
      if (j % 2 == 1) k->q1[j / 2] = (float)cf.q1[j];   // e^j = e * (e^2)^(j/2)
      else k->q2[j / 2] = (float)cf.q2[j];
    } else {
      k->q1[j] = (float)cf.q1[j];
      k->q2[j] = (float)cf.q2[j];
    }
  }
  k->n1 = cf.n1;
  k->n2 = cf.n2;
  // |grad u| = |u'| <= d sum |c o| (t <= 1, rbar <= 1); pick 2^eg with bound 2^eg <= 2^14
  double bg = 0.0;
  for (int j = 0; j < MAXQ; ++j) bg += fabs(cf.q1[j]);
  bg *= cf.d;
  if (cf.c1 != 0.0) bg += fabs(cf.c1) * cf.d;
  int ex = 0;
  if (bg > 0.0) frexp(bg, &ex);        // bg < 2^ex
  k->eg = 14 - ex;                     // |grad u| 2^eg < 2^14
  k->es = 14 - 2 * ex;                 // |grad u|^2 <= bg^2 < 2^(2 ex), so |grad u|^2 2^es < 2^14
  k->sg = (float)ldexp(1.0, k->eg);
  k->ss = (float)ldexp(1.0, k->es);
}

xtc_status stage1_split_f16(const Stage1Args& a, const EECoef& cf, void* scratch, size_t bytes,
                            hipStream_t st) {
  (void)bytes;
  if (a.nch != 4) {
    set_error("split precision: the Laplacian channel is evaluated by the FP64 path only");
    return XTC_ERR_UNSUPPORTED;
  }
  SplitLayout S = split_layout(scratch, a.n_g, a.n_mu);
  SplitCoef k;
  const bool even = even_powers(cf);
  split_coef(cf, &k, even);
  dim3 grid(cdiv(a.bn, SB), (unsigned)(S.rows_pad / SR));
  const size_t smem = sizeof(h8) * 2 * 8 * 8 * 64 + sizeof(float) * 2 * 6 * SKC;
  // compacted even-power polynomials of degree < 4 (powers up to 8) use the short form
  bool short_even = even;
  for (int j = 4; j < MAXQ / 2; ++j)
    if (k.q1[j] != 0.0f || k.q2[j] != 0.0f) short_even = false;
#define XTC_LAUNCH_SPLIT(EV, NQV)                                                              \
  hipLaunchKernelGGL((k_stage1_split<EV, NQV>), grid, dim3(512), smem, st, (const h8*)S.A,     \
                     (const int*)S.sA, (const float*)S.kc, S.n_g_pad, S.nks, a.xyz, a.n_g,    \
                     a.n_mu, a.b0, a.bn, k, a.panel, a.rows_pad, a.bp)
  if (short_even) XTC_LAUNCH_SPLIT(true, 4);
  else if (even) XTC_LAUNCH_SPLIT(true, MAXQ / 2);
  else XTC_LAUNCH_SPLIT(false, MAXQ);
#undef XTC_LAUNCH_SPLIT
  XTC_CHECK_LAUNCH();
  // the rho row (exact field and the ISDF-free energy-scale sums) in FP64
  double* part = (double*)((char*)scratch + split_scratch_bytes(a.n_g, a.n_mu));
  return rho_row_f64(a, cf, part, st);
}

}  // namespace xtc
