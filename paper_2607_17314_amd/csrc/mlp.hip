// Learned interpolation-point proposer: features, MLP forward, weighted-BCE
// gradient, Adam, top-K candidates by score, and the learned selection modes of
// isdf_select_points (candidate-restricted fused pivoting plus the residual judge).
// The network is tiny (8 -> 64 -> 64 -> 1); every point is one thread, with the
// weights in LDS. Reductions over points are fixed-order, so results are
// bitwise repeatable.
#include "common.hpp"
#include "plans.hpp"
#include "timing.hpp"

namespace xtc {

constexpr int NF = 8;
constexpr int HMAX = 128;
constexpr double FEPS = 1e-30;

__host__ __device__ static inline int mlp_nparams(int h) { return NF * h + h + h * h + h + h + 1; }

// ---------------------------------------------------------------- features
__global__ __launch_bounds__(256) void k_features(const double* __restrict__ phi4,
                                                  const double* __restrict__ xyz,
                                                  const double* __restrict__ w, long n_g, int n_orb,
                                                  int n_occ, const double* __restrict__ nuc,
                                                  int n_nuc, float* __restrict__ f, long ld) {
  const long g = (long)blockIdx.x * 256 + threadIdx.x;
  if (g >= n_g) return;
  double n2 = 0.0, g2 = 0.0, rho = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int p = 0; p < n_orb; ++p) {
    const double v = phi4[(long)p * n_g + g];
    const double dx = phi4[(long)(n_orb + p) * n_g + g];
    const double dy = phi4[(long)(2 * n_orb + p) * n_g + g];
    const double dz = phi4[(long)(3 * n_orb + p) * n_g + g];
    n2 += v * v;
    g2 += dx * dx + dy * dy + dz * dz;
    if (p < n_occ) {
      rho += v * v;
      gx += 2.0 * v * dx;
      gy += 2.0 * v * dy;
      gz += 2.0 * v * dz;
    }
  }
  double d0 = 1e300, d1 = 1e300, d2 = 1e300;   // three smallest distances
  const double x = xyz[g], y = xyz[n_g + g], z = xyz[2 * n_g + g];
  for (int a = 0; a < n_nuc; ++a) {
    const double ex = x - nuc[3 * a], ey = y - nuc[3 * a + 1], ez = z - nuc[3 * a + 2];
    const double d = sqrt(ex * ex + ey * ey + ez * ez);
    if (d < d0) { d2 = d1; d1 = d0; d0 = d; }
    else if (d < d1) { d2 = d1; d1 = d; }
    else if (d < d2) { d2 = d; }
  }
  if (n_nuc < 2) d1 = d0;
  if (n_nuc < 3) d2 = d1;
  const double v[NF] = {w[g], n2, g2, rho, sqrt(gx * gx + gy * gy + gz * gz), d0, d1, d2};
#pragma unroll
  for (int k = 0; k < NF; ++k) f[k * ld + g] = (float)log(v[k] + FEPS);
}

// ---------------------------------------------------------------- network
struct MlpDev {
  const float* p; const float* shift; const float* scale; int h;
};

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

__device__ void load_weights(const MlpDev& m, float* sw) {
  const int np = mlp_nparams(m.h);
  for (int i = threadIdx.x; i < np; i += blockDim.x) sw[i] = m.p[i];
  if (threadIdx.x < NF) {
    sw[np + threadIdx.x] = m.shift[threadIdx.x];
    sw[np + NF + threadIdx.x] = m.scale[threadIdx.x];
  }
  __syncthreads();
}

// forward for one point; a1 (h) returned in registers-backed local array
__device__ __forceinline__ float point_forward(const float* sw, int h, const float* x, float* a1,
                                               float* z1) {
  const float* W1 = sw;
  const float* b1 = W1 + NF * h;
  const float* W2 = b1 + h;
  const float* b2 = W2 + h * h;
  const float* W3 = b2 + h;
  const float b3 = W3[h];
  for (int i = 0; i < h; ++i) {
    float z = b1[i];
#pragma unroll
    for (int k = 0; k < NF; ++k) z += W1[i * NF + k] * x[k];
    z1[i] = z;
    a1[i] = silu(z);
  }
  float s = b3;
  for (int j = 0; j < h; ++j) {
    float z = b2[j];
    for (int i = 0; i < h; ++i) z += W2[j * h + i] * a1[i];
    s += W3[j] * silu(z);
  }
  return s;
}

__device__ __forceinline__ void load_point(const float* __restrict__ f, long ld, long i,
                                           const float* sw, int np, float* x) {
#pragma unroll
  for (int k = 0; k < NF; ++k) x[k] = (f[k * ld + i] - sw[np + k]) / sw[np + NF + k];
}

__global__ __launch_bounds__(256) void k_mlp_forward(MlpDev m, const float* __restrict__ f, long ld,
                                                     long n, float* __restrict__ logits) {
  extern __shared__ float sw[];
  load_weights(m, sw);
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int np = mlp_nparams(m.h);
  float x[NF], a1[HMAX], z1[HMAX];
  load_point(f, ld, i, sw, np, x);
  logits[i] = point_forward(sw, m.h, x, a1, z1);
}

// BF16 MFMA inference of the 8 -> 64 -> 64 -> 1 network (v_mfma_f32_32x32x16_bf16, FP32
// accumulation; biases and SiLU in FP32). Each wave takes tiles of 32 points. Every layer
// is a product of the weights (A operand: rows = output units, k = input units) with the
// activations (B operand: k = input units, columns = points), so layer 1's accumulator
// feeds layer 2 without a transpose: lane l (point l % 32, half h = l / 32) holds the
// units 32 mb + 8 q + 4 h + t (q, t = 0..3) of row block mb, and layer 2 takes input unit
// u(s) = 32 (j / 2) + 16 (j % 2) + 8 (e / 4) + 4 h + e % 4 as its k slot s = 16 j + 8 h + e
// (a permutation of the summation index, applied to W2's columns).
// MFMA 32x32x16 layouts (as measured for the FP16 form on gfx950), lane l, element e,
// register r: A[l % 32][8 (l / 32) + e], B[8 (l / 32) + e][l % 32],
// D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32].
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float mf16 __attribute__((ext_vector_type(16)));
constexpr int BF_H = 64;   // the hidden width the BF16 kernel serves

__global__ __launch_bounds__(256) void k_mlp_forward_bf16(MlpDev m, const float* __restrict__ f,
                                                          long ld, long n,
                                                          float* __restrict__ logits) {
  extern __shared__ float sw[];
  load_weights(m, sw);
  const int np = mlp_nparams(BF_H);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 31, half = lane >> 5;
  const float* W1 = sw;
  const float* b1 = W1 + NF * BF_H;
  const float* W2 = b1 + BF_H;
  const float* b2 = W2 + BF_H * BF_H;
  const float* W3 = b2 + BF_H;
  const float b3 = W3[BF_H];
  bf8 a1f[2], a2f[2][4];
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      a1f[mb][e] = (__bf16)(half == 0 ? W1[(32 * mb + col) * NF + e] : 0.0f);
#pragma unroll
  for (int mb = 0; mb < 2; ++mb)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int u = 32 * (j / 2) + 16 * (j % 2) + 8 * (e / 4) + 4 * half + (e % 4);
        a2f[mb][j][e] = (__bf16)W2[(32 * mb + col) * BF_H + u];
      }
  const mf16 zero = {};
  const long ntile = (n + 31) / 32;
  for (long t = (long)blockIdx.x * 4 + wave; t < ntile; t += (long)gridDim.x * 4) {
    const long p = t * 32 + col;
    bf8 xb;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      float v = 0.0f;
      if (half == 0 && p < n) v = (f[e * ld + p] - sw[np + e]) / sw[np + NF + e];
      xb[e] = (__bf16)v;
    }
    mf16 z1[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) z1[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1f[mb], xb, zero, 0, 0, 0);
    bf8 hb[4];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int unit = 32 * mb + 8 * (r / 4) + 4 * half + r % 4;
        hb[2 * mb + r / 8][r % 8] = (__bf16)silu(z1[mb][r] + b1[unit]);
      }
    mf16 z2[2] = {zero, zero};
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        z2[mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2f[mb][j], hb[j], z2[mb], 0, 0, 0);
    float s = 0.0f;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int v = 32 * mb + 8 * (r / 4) + 4 * half + r % 4;
        s += W3[v] * silu(z2[mb][r] + b2[v]);
      }
    s += __shfl_xor(s, 32, 64);
    if (half == 0 && p < n) logits[p] = s + b3;
  }
}

static xtc_status launch_forward(const xtc_mlp* mlp, const float* feats, long ld, long n,
                                 float* logits, hipStream_t st) {
  MlpDev m{mlp->params, mlp->feat_shift, mlp->feat_scale, mlp->hidden};
  const size_t smem = sizeof(float) * (mlp_nparams(mlp->hidden) + 2 * NF);
  if (mlp->bf16) {
    XTC_REQUIRE(mlp->hidden == BF_H, "mlp: BF16 inference is built for 64 hidden units");
    const long tiles = (n + 31) / 32;
    long blocks = (tiles + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_mlp_forward_bf16, dim3((unsigned)blocks), dim3(256), smem, st, m, feats,
                       ld, n, logits);
  } else {
    hipLaunchKernelGGL(k_mlp_forward, dim3(cdiv(n, 256)), dim3(256), smem, st, m, feats, ld, n,
                       logits);
  }
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

// per-point backward quantities, point-major: rec[i] = {x[8], a1[h], d1[h], a2[h], d2[h], ds, loss}
__global__ __launch_bounds__(256) void k_mlp_point_grad(MlpDev m, const float* __restrict__ f,
                                                        long ld, long n,
                                                        const float* __restrict__ y, float pw,
                                                        float* __restrict__ rec, int stride) {
  extern __shared__ float sw[];
  load_weights(m, sw);
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int h = m.h, np = mlp_nparams(h);
  const float* W2 = sw + NF * h + h;
  const float* b2 = W2 + h * h;
  const float* W3 = b2 + h;
  float x[NF], a1[HMAX], z1[HMAX];
  load_point(f, ld, i, sw, np, x);
  const float s = point_forward(sw, h, x, a1, z1);
  const float yi = y[i];
  const float sig = 1.0f / (1.0f + expf(-s));
  // softplus(t) = max(t, 0) + log1p(exp(-|t|))
  const float spn = fmaxf(-s, 0.0f) + log1pf(expf(-fabsf(s)));
  const float spp = fmaxf(s, 0.0f) + log1pf(expf(-fabsf(s)));
  const float li = pw * yi * spn + (1.0f - yi) * spp;
  const float ds = (-pw * yi * (1.0f - sig) + (1.0f - yi) * sig) / (float)n;
  float* r = rec + i * stride;
#pragma unroll
  for (int k = 0; k < NF; ++k) r[k] = x[k];
  float d1[HMAX];
  for (int k = 0; k < h; ++k) d1[k] = 0.0f;
  for (int j = 0; j < h; ++j) {
    float z = b2[j];
    for (int k = 0; k < h; ++k) z += W2[j * h + k] * a1[k];
    const float a2 = silu(z);
    const float d2 = W3[j] * ds * dsilu(z);
    r[NF + 2 * h + j] = a2;
    r[NF + 3 * h + j] = d2;
    for (int k = 0; k < h; ++k) d1[k] += W2[j * h + k] * d2;
  }
  for (int k = 0; k < h; ++k) {
    r[NF + k] = a1[k];
    r[NF + h + k] = d1[k] * dsilu(z1[k]);
  }
  r[NF + 4 * h] = ds;
  r[NF + 4 * h + 1] = li / (float)n;
}

// one thread per parameter (and one for the loss): fixed-order sum over points
__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ rec, int stride, long n,
                                                    int h, float* __restrict__ grad,
                                                    float* __restrict__ loss) {
  const int np = mlp_nparams(h);
  const int q = blockIdx.x * 256 + threadIdx.x;
  if (q > np) return;
  // offsets within a record
  const int X = 0, A1 = NF, D1 = NF + h, A2 = NF + 2 * h, D2 = NF + 3 * h, DS = NF + 4 * h;
  int oa, ob;   // grad = sum_i rec[oa] * (ob < 0 ? 1 : rec[ob])
  if (q == np) { oa = DS + 1; ob = -1; }
  else if (q < NF * h) { oa = D1 + q / NF; ob = X + q % NF; }                 // W1[i][k]
  else if (q < NF * h + h) { oa = D1 + (q - NF * h); ob = -1; }              // b1
  else if (q < NF * h + h + h * h) { const int t = q - NF * h - h; oa = D2 + t / h; ob = A1 + t % h; }
  else if (q < NF * h + 2 * h + h * h) { oa = D2 + (q - NF * h - h - h * h); ob = -1; }   // b2
  else if (q < NF * h + 3 * h + h * h) { oa = DS; ob = A2 + (q - NF * h - 2 * h - h * h); } // W3
  else { oa = DS; ob = -1; }                                                  // b3
  float s = 0.0f;
  for (long i = 0; i < n; ++i) {
    const float* r = rec + i * stride;
    s += r[oa] * (ob < 0 ? 1.0f : r[ob]);
  }
  if (q == np) *loss = s;
  else grad[q] = s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- top-K
__device__ __forceinline__ unsigned fkey(float s) {
  unsigned u = __float_as_uint(s);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);   // order-preserving
}

struct SelState {
  unsigned lo, hi;        // bisection bounds on the key threshold
  unsigned long long cnt; // count of keys >= mid (scratch)
  unsigned thr;
  long above, need_eq;
};

__global__ __launch_bounds__(256) void k_count_ge(const float* __restrict__ s, long n,
                                                  const SelState* st, int use_mid, unsigned thr_in,
                                                  unsigned* __restrict__ block_cnt) {
  __shared__ unsigned c[256];
  const unsigned thr = use_mid ? (unsigned)(((unsigned long long)st->lo + st->hi + 1) / 2) : thr_in;
  unsigned k = 0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256)
    k += fkey(s[i]) >= thr;
  c[threadIdx.x] = k;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) c[threadIdx.x] += c[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) block_cnt[blockIdx.x] = c[0];
}

// largest threshold T with count(key >= T) >= K: bisection over [lo, hi]
__global__ void k_bisect(SelState* st, const unsigned* __restrict__ block_cnt, int nb, long K) {
  unsigned long long tot = 0;
  for (int b = 0; b < nb; ++b) tot += block_cnt[b];
  const unsigned mid = (unsigned)(((unsigned long long)st->lo + st->hi + 1) / 2);
  if (st->lo < st->hi) {
    if ((long)tot >= K) st->lo = mid;
    else st->hi = mid - 1;
  }
}

__global__ void k_finish_thr(SelState* st, const unsigned* __restrict__ block_cnt, int nb, long K) {
  // block_cnt holds count(key >= thr + 1) = count(key > thr)
  unsigned long long tot = 0;
  for (int b = 0; b < nb; ++b) tot += block_cnt[b];
  st->thr = st->lo;
  st->above = (long)tot;
  st->need_eq = K - (long)tot;
}

// selection flags in index order: sel = key > T or (key == T and rank among ties < need_eq)
__global__ __launch_bounds__(256) void k_eq_counts(const float* __restrict__ s, long n,
                                                   const SelState* st, unsigned* __restrict__ bc) {
  __shared__ unsigned c[256];
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  c[threadIdx.x] = (i < n && fkey(s[i]) == st->thr) ? 1u : 0u;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) c[threadIdx.x] += c[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bc[blockIdx.x] = c[0];
}

__global__ void k_excl_scan(unsigned* __restrict__ bc, int nb) {
  if (threadIdx.x) return;
  unsigned run = 0;
  for (int b = 0; b < nb; ++b) {
    const unsigned v = bc[b];
    bc[b] = run;
    run += v;
  }
}

__device__ unsigned block_excl_scan(unsigned v, unsigned* tot) {
  __shared__ unsigned sc[256];
  sc[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const unsigned t = threadIdx.x >= (unsigned)o ? sc[threadIdx.x - o] : 0u;
    __syncthreads();
    sc[threadIdx.x] += t;
    __syncthreads();
  }
  const unsigned incl = sc[threadIdx.x];
  *tot = sc[255];
  __syncthreads();
  return incl - v;
}

// candidates: the top K by score (ties to the lowest index) and every stride-th point
__global__ __launch_bounds__(256) void k_sel_flags(const float* __restrict__ s, long n,
                                                   const SelState* st,
                                                   const unsigned* __restrict__ eq_off,
                                                   long stride, unsigned char* __restrict__ sel,
                                                   unsigned* __restrict__ sel_cnt) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  const unsigned key = i < n ? fkey(s[i]) : 0u;
  const unsigned eq = (i < n && key == st->thr) ? 1u : 0u;
  unsigned tot;
  const unsigned r = block_excl_scan(eq, &tot) + eq_off[blockIdx.x];
  const unsigned f = (i < n) && (key > st->thr || (eq && (long)r < st->need_eq) ||
                                 (stride > 0 && i % stride == 0));
  if (i < n) sel[i] = (unsigned char)f;
  unsigned tot2;
  block_excl_scan(f, &tot2);
  if (threadIdx.x == 0) sel_cnt[blockIdx.x] = tot2;
}

// total of the per-block counts (before their exclusive scan) into st->cnt
__global__ void k_sum_counts(SelState* st, const unsigned* __restrict__ bc, int nb) {
  if (threadIdx.x) return;
  unsigned long long t = 0;
  for (int b = 0; b < nb; ++b) t += bc[b];
  st->cnt = t;
}

__global__ __launch_bounds__(256) void k_scatter_sel(const unsigned char* __restrict__ sel, long n,
                                                     const unsigned* __restrict__ off,
                                                     long* __restrict__ out) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  const unsigned f = i < n ? sel[i] : 0u;
  unsigned tot;
  const unsigned r = block_excl_scan(f, &tot) + off[blockIdx.x];
  if (f) out[r] = i;
}

__global__ void k_gather_sub(const double* __restrict__ phi4, const double* __restrict__ w, long n_g,
                             int rows, const long* __restrict__ idx, long K,
                             double* __restrict__ sub, double* __restrict__ wsub) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long)rows * K) return;
  const long r = t / K, j = t % K;
  sub[t] = phi4[r * n_g + idx[j]];
  if (r == 0) wsub[j] = w[idx[j]];
}

}  // namespace xtc

using namespace xtc;

// ---------------------------------------------------------------- entry points
extern "C" xtc_status xtc_mlp_features(const double* phi4, const xtc_grid* grid, int32_t n_orb,
                                       int32_t n_occ, int32_t n_nuc, const double* nuc_xyz,
                                       float* feats, void* ws, size_t ws_bytes, void* stream) {
  XTC_REQUIRE(phi4 && grid && feats && (n_nuc == 0 || nuc_xyz), "xtc_mlp_features: null argument");
  XTC_REQUIRE(grid->n_g > 0 && grid->xyz && grid->w && n_orb > 0 && n_occ >= 0 && n_occ <= n_orb &&
                  n_nuc >= 1 && n_nuc <= 4096,
              "xtc_mlp_features: bad sizes");
  hipStream_t st = as_stream(stream);
  Arena ar(ws, ws_bytes);
  double* nuc = ar.take<double>(3 * (size_t)n_nuc);
  XTC_TRY(need_ws(ar));
  XTC_TRY(check_weights(grid, ws, ws_bytes, st, "xtc_mlp_features"));
  XTC_HIP(hipMemcpyAsync(nuc, nuc_xyz, sizeof(double) * 3 * n_nuc, hipMemcpyHostToDevice, st));
  XTC_HIP(hipStreamSynchronize(st));
  hipLaunchKernelGGL(k_features, dim3(cdiv(grid->n_g, 256)), dim3(256), 0, st, phi4, grid->xyz,
                     grid->w, grid->n_g, n_orb, n_occ, (const double*)nuc, n_nuc, feats,
                     (long)grid->n_g);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

static xtc_status check_mlp(const xtc_mlp* m) {
  XTC_REQUIRE(m && m->params && m->feat_shift && m->feat_scale, "mlp: null argument");
  XTC_REQUIRE(m->in_dim == NF && m->hidden >= 1 && m->hidden <= HMAX, "mlp: bad shape");
  XTC_REQUIRE(m->bf16 == 0 || m->bf16 == 1, "mlp: bf16 must be 0 or 1");
  if (m->bf16 && m->hidden != BF_H) {
    set_error("mlp: BF16 inference is built for 64 hidden units");
    return XTC_ERR_UNSUPPORTED;
  }
  return XTC_OK;
}

extern "C" xtc_status xtc_mlp_forward(const xtc_mlp* mlp, const float* feats, int64_t ld, int64_t n,
                                      float* logits, void* stream) {
  XTC_TRY(check_mlp(mlp));
  XTC_REQUIRE(feats && logits && n > 0 && ld >= n, "xtc_mlp_forward: bad arguments");
  return launch_forward(mlp, feats, (long)ld, (long)n, logits, as_stream(stream));
}

static inline int rec_stride(int h) { return NF + 4 * h + 2; }

extern "C" xtc_status xtc_mlp_loss_grad(const xtc_mlp* mlp, const float* feats, int64_t ld,
                                        int64_t n, const float* labels, float pos_weight,
                                        float* loss, float* grad, void* ws, size_t ws_bytes,
                                        void* stream) {
  XTC_TRY(check_mlp(mlp));
  XTC_REQUIRE(feats && labels && loss && grad && n > 0 && ld >= n, "xtc_mlp_loss_grad: bad arguments");
  hipStream_t st = as_stream(stream);
  Arena ar(ws, ws_bytes);
  const int stride = rec_stride(mlp->hidden);
  float* rec = ar.take<float>((size_t)n * stride);
  XTC_TRY(need_ws(ar));
  MlpDev m{mlp->params, mlp->feat_shift, mlp->feat_scale, mlp->hidden};
  const size_t smem = sizeof(float) * (mlp_nparams(mlp->hidden) + 2 * NF);
  size_t tk = timing_begin(TM_MLP, st);
  hipLaunchKernelGGL(k_mlp_point_grad, dim3(cdiv(n, 256)), dim3(256), smem, st, m, feats, (long)ld,
                     (long)n, labels, pos_weight, rec, stride);
  XTC_CHECK_LAUNCH();
  const int np = mlp_nparams(mlp->hidden);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(cdiv(np + 1, 256)), dim3(256), 0, st, (const float*)rec,
                     stride, (long)n, mlp->hidden, grad, loss);
  XTC_CHECK_LAUNCH();
  timing_end(tk, st);
  return XTC_OK;
}

extern "C" xtc_status xtc_adam_step(float* params, const float* grad, float* m, float* v, int32_t n,
                                    float lr, float beta1, float beta2, float eps, int32_t t,
                                    void* stream) {
  XTC_REQUIRE(params && grad && m && v && n > 0 && t >= 1, "xtc_adam_step: bad arguments");
  const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(cdiv(n, 256)), dim3(256), 0, as_stream(stream), params, grad, m, v,
                     n, lr, beta1, beta2, eps, c1, c2);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

namespace xtc {

size_t ws_features(int64_t n_g) { (void)n_g; return 3 * 4096 * sizeof(double) + 256; }
size_t ws_mlp_grad(int64_t n, int hidden) { return (size_t)n * rec_stride(hidden) * sizeof(float) + 256; }

struct LearnLayout {
  float* feats; float* logits; SelState* sst; unsigned* bc; unsigned* bc2; unsigned char* sel;
  long* cand; double* sub; double* wsub; double* nuc; int nb; long K;
};

// K: the largest candidate count (the top K by score plus the coverage points)
static LearnLayout layout_learn(Arena& ar, int64_t n_g, int n_orb, long K) {
  LearnLayout L;
  L.K = K;
  L.nb = (int)cdiv(n_g, 256);
  L.feats = ar.take<float>((size_t)NF * n_g);
  L.logits = ar.take<float>(n_g);
  L.sst = ar.take<SelState>(1);
  L.bc = ar.take<unsigned>(L.nb);
  L.bc2 = ar.take<unsigned>(L.nb);
  L.sel = ar.take<unsigned char>(n_g);
  L.cand = ar.take<long>(K);
  L.sub = ar.take<double>(4 * (size_t)n_orb * K);
  L.wsub = ar.take<double>(K);
  L.nuc = ar.take<double>(3 * 4096);
  return L;
}

// top-K by score and every stride-th point; candidate indices ascending in L.cand, their
// number returned in *count
static xtc_status top_k(LearnLayout& L, long n, long K, long stride, hipStream_t st,
                        long* count) {
  SelState init{};
  init.lo = 0u;
  init.hi = 0xffffffffu;
  XTC_HIP(hipMemcpyAsync(L.sst, &init, sizeof(SelState), hipMemcpyHostToDevice, st));
  const int nbc = L.nb < 1024 ? L.nb : 1024;
  for (int it = 0; it < 32; ++it) {
    hipLaunchKernelGGL(k_count_ge, dim3(nbc), dim3(256), 0, st, (const float*)L.logits, n,
                       (const SelState*)L.sst, 1, 0u, L.bc);
    hipLaunchKernelGGL(k_bisect, dim3(1), dim3(1), 0, st, L.sst, (const unsigned*)L.bc, nbc, K);
  }
  XTC_CHECK_LAUNCH();
  // count(key > thr): one more pass at thr + 1, read on the device
  SelState h{};
  XTC_HIP(hipMemcpyAsync(&h, L.sst, sizeof(SelState), hipMemcpyDeviceToHost, st));
  XTC_HIP(hipStreamSynchronize(st));
  if (h.lo == 0xffffffffu) {
    XTC_HIP(hipMemsetAsync(L.bc, 0, sizeof(unsigned) * nbc, st));
  } else {
    hipLaunchKernelGGL(k_count_ge, dim3(nbc), dim3(256), 0, st, (const float*)L.logits, n,
                       (const SelState*)L.sst, 0, h.lo + 1u, L.bc);
  }
  hipLaunchKernelGGL(k_finish_thr, dim3(1), dim3(1), 0, st, L.sst, (const unsigned*)L.bc, nbc, K);
  hipLaunchKernelGGL(k_eq_counts, dim3(L.nb), dim3(256), 0, st, (const float*)L.logits, n,
                     (const SelState*)L.sst, L.bc2);
  hipLaunchKernelGGL(k_excl_scan, dim3(1), dim3(1), 0, st, L.bc2, L.nb);
  hipLaunchKernelGGL(k_sel_flags, dim3(L.nb), dim3(256), 0, st, (const float*)L.logits, n,
                     (const SelState*)L.sst, (const unsigned*)L.bc2, stride, L.sel, L.bc);
  hipLaunchKernelGGL(k_sum_counts, dim3(1), dim3(1), 0, st, L.sst, (const unsigned*)L.bc, L.nb);
  hipLaunchKernelGGL(k_excl_scan, dim3(1), dim3(1), 0, st, L.bc, L.nb);
  hipLaunchKernelGGL(k_scatter_sel, dim3(L.nb), dim3(256), 0, st, (const unsigned char*)L.sel, n,
                     (const unsigned*)L.bc, L.cand);
  XTC_CHECK_LAUNCH();
  SelState fin{};
  XTC_HIP(hipMemcpyAsync(&fin, L.sst, sizeof(SelState), hipMemcpyDeviceToHost, st));
  XTC_HIP(hipStreamSynchronize(st));
  *count = (long)fin.cnt;
  return XTC_OK;
}

}  // namespace xtc

// defined in pivots.hip / fit.hip
xtc_status xtc_select_qr(const double* phi4, const xtc_grid* grid, int n_orb, int n_mu,
                         int64_t* pivots, int32_t* n_mu_out, double* info, Arena& ar,
                         hipStream_t st);
namespace xtc {
xtc_status fit_scalar_residual(const double* phi4, const xtc_grid* grid, int n_orb,
                               const int64_t* pivots, int n_mu, Arena& ar, hipStream_t st,
                               double* rel);
size_t ws_learned(int64_t n_g, int n_orb, int n_mu, double kappa, long stride);
xtc_status fit_residuals(const double* phi4, const xtc_grid* grid, int n_orb,
                         const int64_t* pivots, int n_mu, Arena& ar, hipStream_t st, double* rel);
}

// candidates at most: ceil(kappa n_mu) by score plus ceil(n_g / stride) coverage points
static long max_candidates(int64_t n_g, int n_mu, double kappa, long stride) {
  long K = (long)ceil(kappa * n_mu);
  if (K < n_mu) K = n_mu;
  if (stride > 0) K += (n_g + stride - 1) / stride;
  return K > n_g ? n_g : K;
}

size_t xtc::ws_learned(int64_t n_g, int n_orb, int n_mu, double kappa, long stride) {
  Arena ar(nullptr, 0);
  layout_learn(ar, n_g, n_orb, max_candidates(n_g, n_mu, kappa, stride));
  return ar.used;
}

xtc_status xtc_select_learned(const double* phi4, const xtc_grid* grid, int n_orb, int n_occ,
                              int n_mu, int mode, const xtc_mlp* mlp, double fallback_factor,
                              int64_t* pivots, int32_t* n_mu_out, double* info, Arena& ar,
                              hipStream_t st) {
  XTC_TRY(check_mlp(mlp));
  XTC_REQUIRE(mlp->n_nuc >= 1 && mlp->n_nuc <= 4096 && mlp->nuc_xyz, "learned selection: nuclei");
  XTC_REQUIRE(mlp->kappa >= 1.0, "learned selection: kappa must be >= 1");
  XTC_REQUIRE(mlp->stride >= 0, "learned selection: stride must be >= 0");
  const long n_g = grid->n_g;
  long K = (long)ceil(mlp->kappa * n_mu);
  if (K > n_g) K = n_g;
  LearnLayout L = layout_learn(ar, n_g, n_orb, max_candidates(n_g, n_mu, mlp->kappa, mlp->stride));
  XTC_TRY(need_ws(ar));
  // features -> logits -> candidates
  XTC_HIP(hipMemcpyAsync(L.nuc, mlp->nuc_xyz, sizeof(double) * 3 * mlp->n_nuc,
                         hipMemcpyHostToDevice, st));
  XTC_HIP(hipStreamSynchronize(st));
  hipLaunchKernelGGL(k_features, dim3(cdiv(n_g, 256)), dim3(256), 0, st, phi4, grid->xyz, grid->w,
                     n_g, n_orb, n_occ, (const double*)L.nuc, mlp->n_nuc, L.feats, n_g);
  XTC_CHECK_LAUNCH();
  XTC_TRY(launch_forward(mlp, L.feats, n_g, n_g, L.logits, st));
  long nc = 0;
  XTC_TRY(top_k(L, n_g, K, mlp->stride, st, &nc));
  hipLaunchKernelGGL(k_gather_sub, dim3(cdiv(4L * n_orb * nc, 256)), dim3(256), 0, st, phi4, grid->w,
                     n_g, 4 * n_orb, (const long*)L.cand, nc, L.sub, L.wsub);
  XTC_CHECK_LAUNCH();
  // fused pivoting restricted to the candidates
  xtc_grid sub{nc, nullptr, L.wsub};
  std::vector<int64_t> local(n_mu);
  int32_t n_loc = 0;
  xtc_status s = xtc_select_qr(L.sub, &sub, n_orb, n_mu, local.data(), &n_loc, info, ar, st);
  if (s < 0) return s;
  std::vector<long> cand(nc);
  XTC_HIP(hipMemcpyAsync(cand.data(), L.cand, sizeof(long) * nc, hipMemcpyDeviceToHost, st));
  XTC_HIP(hipStreamSynchronize(st));
  for (int i = 0; i < n_loc; ++i) pivots[i] = cand[local[i]];
  *n_mu_out = n_loc;
  if (info) {
    info[2] = 0.0;
    info[6] = (double)nc;
  }
  if (mode != XTC_SELECT_LEARNED_JUDGED) return s;
  // judge: the mean of the four relative fit residuals (scalar and the three gradient
  // components) of the proposal over the whole grid
  auto mean4 = [](const double* r) { return 0.25 * ((r[0] + r[1]) + (r[2] + r[3])); };
  double rl4[4] = {0, 0, 0, 0};
  XTC_TRY(xtc::fit_residuals(phi4, grid, n_orb, pivots, n_loc, ar, st, rl4));
  const double r_l = mean4(rl4);
  double r_ref;
  std::vector<int64_t> qr(n_mu);
  int32_t n_qr = 0;
  if (mlp->judge == 1) {
    double qinfo[8] = {0};
    xtc_status sq = xtc_select_qr(phi4, grid, n_orb, n_mu, qr.data(), &n_qr, qinfo, ar, st);
    if (sq < 0) return sq;
    double rq4[4] = {0, 0, 0, 0};
    XTC_TRY(xtc::fit_residuals(phi4, grid, n_orb, qr.data(), n_qr, ar, st, rq4));
    r_ref = mean4(rq4);
  } else {
    r_ref = exp(mlp->ref_a + mlp->ref_b * log((double)n_mu / (double)n_orb));
  }
  if (info) {
    info[3] = r_l;
    info[4] = r_ref;
  }
  if (r_l <= fallback_factor * r_ref && n_loc == n_mu) return s;
  // fall back to the QR selection
  if (mlp->judge != 1) {
    double qinfo[8] = {0};
    xtc_status sq = xtc_select_qr(phi4, grid, n_orb, n_mu, qr.data(), &n_qr, qinfo, ar, st);
    if (sq < 0) return sq;
    if (info) { info[0] = qinfo[0]; info[1] = qinfo[1]; }
  }
  for (int i = 0; i < n_qr; ++i) pivots[i] = qr[i];
  *n_mu_out = n_qr;
  if (info) info[2] = 1.0;
  return XTC_WARN_FALLBACK;
}
