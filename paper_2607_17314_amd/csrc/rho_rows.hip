// The two density rows of the stage-1 panel in FP64 for the split path (the split
// pair kernel leaves them out): rows n_mu (rho_gamma) and n_mu + 1 (the ISDF density).
#include "contract.hpp"

namespace xtc {

// The two density rows of the panel in FP64 on the vector units: row n_mu with
// rho_gamma (field A_gamma and T3rho) and row n_mu + 1 with the ISDF density
// rhot (H_{g,c}, which as a sum over N_mu split-precision rows would cancel).
// Each thread takes two bra points and one ket segment (the ket values are
// wave-uniform, so they come through the scalar cache); the segments' partial
// sums are added in a fixed order by k_rho_row_sum. 1/sqrt and 1/(1 + d r) start
// from the hardware estimates and take two Newton steps (about one ulp; FP64
// division and square root would each expand to a longer correctly-rounded
// sequence), and the polynomials have a compile-time length NQ (coefficients
// past the true degree are zero).
constexpr int RHO_SEG = 32;

template <int NQ>
__device__ __forceinline__ double horner_fixed(const double (&q)[NQ], double x) {
  double r = q[NQ - 1];
#pragma unroll
  for (int j = NQ - 2; j >= 0; --j) r = fma(r, x, q[j]);
  return r;
}

// r = |d| and 1/r (0 and 0 at r = 0) from r2 = |d|^2
__device__ __forceinline__ void sqrt_rsqrt(double r2, double& r, double& rinv) {
  double y = __builtin_amdgcn_rsq(r2);            // ~1/sqrt(r2)
  double g = r2 * y, h = 0.5 * y;                  // g ~ sqrt(r2), h ~ 1/(2 sqrt(r2))
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-h, g, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
  }
  const bool zero = !(r2 > 0.0);
  r = zero ? 0.0 : g;
  rinv = zero ? 0.0 : 2.0 * h;
}

__device__ __forceinline__ double recip(double x) {   // x >= 1
  double y = __builtin_amdgcn_rcp(x);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
  }
  return y;
}

template <int NQ, bool C1>
__global__ __launch_bounds__(256) void k_rho_row(const double* __restrict__ xyz,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ rho,
                                                 const double* __restrict__ rhot, long n_g,
                                                 long b0, long bn, EECoef cf,
                                                 double* __restrict__ part) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;   // bra points 2t, 2t + 1
  const long seg = blockIdx.y;
  const long per = (n_g + RHO_SEG - 1) / RHO_SEG;
  const long k0 = seg * per, k1 = k0 + per < n_g ? k0 + per : n_g;
  double q1[NQ], q2[NQ];
#pragma unroll
  for (int j = 0; j < NQ; ++j) {
    q1[j] = j < cf.n1 ? cf.q1[j] : 0.0;
    q2[j] = j < cf.n2 ? cf.q2[j] : 0.0;
  }
  const double d = cf.d, c1d = cf.c1 * cf.d, dd = cf.d * cf.d;
  double bx[2], by[2], bz[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    long b = b0 + 2 * t + u;
    if (b > b0 + bn - 1) b = b0 + bn - 1;
    bx[u] = xyz[b];
    by[u] = xyz[n_g + b];
    bz[u] = xyz[2 * n_g + b];
  }
  double s[2][4] = {}, h[2][4] = {};
  for (long g = k0; g < k1; ++g) {
    const double kx = xyz[g], ky = xyz[n_g + g], kz = xyz[2 * n_g + g];
    const double a = w[g] * rho[g];
    const double at = w[g] * rhot[g];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const double dx = bx[u] - kx, dy = by[u] - ky, dz = bz[u] - kz;
      double r, rinv;
      sqrt_rsqrt(fma(dx, dx, fma(dy, dy, dz * dz)), r, rinv);
      const double tt = recip(fma(d, r, 1.0));
      const double e = d * r * tt;
      const double t2 = tt * tt;
      const double up = d * t2 * horner_fixed(q1, e);
      double f = dd * t2 * tt * horner_fixed(q2, e);
      if (C1) f = fma(c1d * t2, rinv, f);   // the o = 1 term; 0 at r = 0
      const double fx = f * dx, fy = f * dy, fz = f * dz, sq = up * up;
      s[u][0] = fma(a, fx, s[u][0]);
      s[u][1] = fma(a, fy, s[u][1]);
      s[u][2] = fma(a, fz, s[u][2]);
      s[u][3] = fma(a, sq, s[u][3]);
      h[u][0] = fma(at, fx, h[u][0]);
      h[u][1] = fma(at, fy, h[u][1]);
      h[u][2] = fma(at, fz, h[u][2]);
      h[u][3] = fma(at, sq, h[u][3]);
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const long tb = 2 * t + u;
    if (tb < bn) {
      double* p = part + (seg * 8) * bn + tb;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        p[q * bn] = s[u][q];
        p[(4 + q) * bn] = h[u][q];
      }
    }
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
  const dim3 grid(cdiv((a.bn + 1) / 2, 256), RHO_SEG);
  const int nq = cf.n1 > cf.n2 ? cf.n1 : cf.n2;
#define XTC_LAUNCH_RHO(NQV, C1V)                                                           \
  hipLaunchKernelGGL((k_rho_row<NQV, C1V>), grid, dim3(256), 0, st, a.xyz, a.w, a.rho, a.rhot, \
                     a.n_g, a.b0, a.bn, cf, part)
  const bool c1 = cf.c1 != 0.0;
  if (nq <= 4) {
    if (c1) XTC_LAUNCH_RHO(4, true); else XTC_LAUNCH_RHO(4, false);
  } else if (nq <= 8) {
    if (c1) XTC_LAUNCH_RHO(8, true); else XTC_LAUNCH_RHO(8, false);
  } else {
    if (c1) XTC_LAUNCH_RHO(MAXQ, true); else XTC_LAUNCH_RHO(MAXQ, false);
  }
#undef XTC_LAUNCH_RHO
  XTC_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_rho_row_sum, dim3(cdiv(a.bn, 256)), dim3(256), 0, st, (const double*)part,
                     a.bn, a.n_mu, a.panel, a.rows_pad, a.bp);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

}  // namespace xtc
