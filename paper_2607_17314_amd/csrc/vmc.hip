// Reference-variance optimisation of the correlator by variational Monte Carlo (the
// VMC section): Metropolis sampling of the reference determinant |Phi_0|^2, the local
// energy of the Slater-Jastrow trial function with its parameter derivatives (eq. Eloc),
// and the Newton step with Gauss-Newton curvature on the clipped variance (eqs. var-loss,
// gn).
//
// Walkers are independent, so the sampler and the local energy give each walker one
// 64-lane workgroup (a single wave): the wave holds the walker's electrons, its two
// inverse Slater matrices and the AO row of the current point in LDS, evaluates the AOs
// lane-parallel over shells and the occupied orbitals lane-parallel over (orbital,
// AO slice), and keeps the inverses current with Sherman-Morrison updates. No state
// crosses walkers, so one launch runs every sweep. The Gauss-Newton step is one
// workgroup: its sums over the walkers are block reductions for a few parameters and
// walker tiles staged in LDS for more, all in a fixed order, then a Cholesky solve in
// LDS.
#include <cmath>
#include "common.hpp"
#include "plans.hpp"
#include "timing.hpp"

namespace xtc {

constexpr int VMC_MAX_OCC = 32;      // electrons per spin
constexpr int VMC_MAX_L = 6;
constexpr int VMC_MAX_TERMS = 12;    // EE terms of the local-energy kernel
constexpr int VMC_MAX_THETA = 128;   // parameters of the Gauss-Newton step
constexpr int VMC_GN_THREADS = 512;
constexpr int GN_FEW = 16;   // up to this many parameters the GN sums are block reductions

// Basis tables as the kernels hold them (staged into LDS at kernel start): per shell the
// centre {x, y, z, 0} and {l, first primitive, end primitive, first AO}; per primitive
// {exponent, coefficient}. The Cartesian component factors are folded into the orbital
// coefficients (C'[a][k] = comp_a C[a][k]), so the AO rows below omit them.
struct VmcBasis {
  const double* cen;   // [n_cent][4]: the distinct shell centres (x, y, z, 0)
  const int* shi;      // [n_shell][2]: l | centre << 3 | n_prim << 15, first primitive | first AO << 15
  const double* prim;  // [n_prim][2]
  int n_shell, n_prim, n_ao, n_cent;
};

struct VmcDev {
  VmcBasis b;
  const double* C;      // [n_occ][n_ao] (orbital-major), component factors folded in
  const double* nuc;    // [n_nuc][4]: x, y, z, Z
  int n_occ, n_nuc;
  double e_nuc;
};

struct EECoefV {
  int n;
  double d;
  int o[VMC_MAX_TERMS];
  double c[VMC_MAX_TERMS];
};

// x^n for 0 <= n <= NMAX by a fixed-length predicated product (no register tables
// indexed by lane-varying exponents).
template <int NMAX>
__device__ __forceinline__ double vmc_ipow_to(double x, int n) {
  double r = 1.0;
#pragma unroll
  for (int q = 0; q < NMAX; ++q) r = q < n ? r * x : r;
  return r;
}
__device__ __forceinline__ double vmc_ipow(double x, int n) {   // Cartesian powers, n <= l + 1
  return vmc_ipow_to<VMC_MAX_L + 1>(x, n);
}

// The Cartesian functions of one shell of angular momentum L (compile time, so every
// power below is a fixed product, the same left-to-right product as at run time).
template <int L, bool LAP>
__device__ __forceinline__ void vmc_shell_l(double x, double y, double z, double r2, double g0,
                                            double g1, double g2, int n_ao, int a, double* chi) {
#pragma unroll
  for (int i = L; i >= 0; --i) {
    const double xi = vmc_ipow(x, i);
#pragma unroll
    for (int j = L - i; j >= 0; --j, ++a) {
      const int k = L - i - j;
      const double yj = vmc_ipow(y, j), zk = vmc_ipow(z, k);
      const double P = xi * yj * zk;
      chi[a] = P * g0;
      if (LAP) {
        const double xm = i > 0 ? vmc_ipow(x, i - 1) : 0.0;
        const double ym = j > 0 ? vmc_ipow(y, j - 1) : 0.0;
        const double zm = k > 0 ? vmc_ipow(z, k - 1) : 0.0;
        chi[n_ao + a] = yj * zk * (i * xm * g0 + 2.0 * xi * x * g1);
        chi[2 * n_ao + a] = xi * zk * (j * ym * g0 + 2.0 * yj * y * g1);
        chi[3 * n_ao + a] = xi * yj * (k * zm * g0 + 2.0 * zk * z * g1);
        double lapP = 0.0;
        if (i >= 2) lapP += i * (i - 1) * vmc_ipow(x, i - 2) * yj * zk;
        if (j >= 2) lapP += j * (j - 1) * xi * vmc_ipow(y, j - 2) * zk;
        if (k >= 2) lapP += k * (k - 1) * xi * yj * vmc_ipow(z, k - 2);
        chi[4 * n_ao + a] = g0 * lapP + P * ((4.0 * L + 6.0) * g1 + 4.0 * r2 * g2);
      }
    }
  }
}

// AO rows (without the component factor) of shell s at the point p, written to chi[a]
// and, with LAP, chi[n_ao * q + a] for q = 1..4 (gradient, Laplacian). chi = P g(s),
// P = x^i y^j z^k, g = sum c e^{-alpha r^2}: d_x chi = (i x^{i-1} g + 2 x^{i+1} g') y^j z^k,
// lap chi = g lap P + P (4 l g' + 6 g' + 4 r^2 g''), primes in s = r^2. Tables in LDS.
template <bool LAP>
__device__ void vmc_shell(const double* cen, const int* shi, const double* prim, int n_ao, int s,
                          double px, double py, double pz, double* chi) {
  const unsigned w0 = (unsigned)shi[2 * s], w1 = (unsigned)shi[2 * s + 1];
  const int l = (int)(w0 & 7u), c = (int)((w0 >> 3) & 4095u);
  const int p0 = (int)(w1 & 32767u), p1 = p0 + (int)(w0 >> 15);
  const int a = (int)(w1 >> 15);
  const double x = px - cen[4 * c], y = py - cen[4 * c + 1], z = pz - cen[4 * c + 2];
  const double r2 = x * x + y * y + z * z;
  double g0 = 0.0, g1 = 0.0, g2 = 0.0;
  for (int p = p0; p < p1; ++p) {
    const double al = prim[2 * p];
    const double e = prim[2 * p + 1] * exp(-al * r2);
    g0 += e;
    if (LAP) {
      g1 -= al * e;
      g2 += al * al * e;
    }
  }
  switch (l) {   // one straight-line body per angular momentum
    case 0: vmc_shell_l<0, LAP>(x, y, z, r2, g0, g1, g2, n_ao, a, chi); break;
    case 1: vmc_shell_l<1, LAP>(x, y, z, r2, g0, g1, g2, n_ao, a, chi); break;
    case 2: vmc_shell_l<2, LAP>(x, y, z, r2, g0, g1, g2, n_ao, a, chi); break;
    case 3: vmc_shell_l<3, LAP>(x, y, z, r2, g0, g1, g2, n_ao, a, chi); break;
    case 4: vmc_shell_l<4, LAP>(x, y, z, r2, g0, g1, g2, n_ao, a, chi); break;
    case 5: vmc_shell_l<5, LAP>(x, y, z, r2, g0, g1, g2, n_ao, a, chi); break;
    default: vmc_shell_l<6, LAP>(x, y, z, r2, g0, g1, g2, n_ao, a, chi); break;
  }
}

// Copies the basis tables into LDS (the caller synchronises before use).
__device__ __forceinline__ void vmc_stage(const VmcBasis& b, double* cen, int* shi,
                                          double* prim) {
  for (int i = threadIdx.x; i < 4 * b.n_cent; i += 64) cen[i] = b.cen[i];
  for (int i = threadIdx.x; i < 2 * b.n_shell; i += 64) shi[i] = b.shi[i];
  for (int i = threadIdx.x; i < 2 * b.n_prim; i += 64) prim[i] = b.prim[i];
}

// All AOs of the point p into chi (lanes over shells); the caller synchronises.
template <bool LAP>
__device__ __forceinline__ void vmc_aos(const VmcBasis& b, const double* cen, const int* shi,
                                        const double* prim, double px, double py, double pz,
                                        double* chi) {
  for (int s = threadIdx.x; s < b.n_shell; s += 64)
    vmc_shell<LAP>(cen, shi, prim, b.n_ao, s, px, py, pz, chi);
}

// out[q * ostride + k] = sum_a chi[q * n_ao + a] C[a][k], q < NQ, k < n_occ: lanes as
// (k, slice) with P = 64 / n_occ slices; slice sl sums the contiguous AOs
// [sl B, sl B + B), B = ceil(n_ao / P), in order (the coefficients orbital-major, so both
// operands of a batch of eight are read at fixed offsets from one base); partial sums in
// part[64 * NQ], added in slice order.
template <int NQ>
__device__ __forceinline__ void vmc_orbitals(const VmcDev& v, const double* chi, double* part,
                                             double* out, int ostride) {
  const int n = v.n_occ, n_ao = v.b.n_ao;
  const int P = 64 / n;
  const int lane = threadIdx.x;
  const int k = lane / P, sl = lane - k * P;
  double acc[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
  if (k < n) {
    const int B = (n_ao + P - 1) / P;
    const int a0 = sl * B, a1 = a0 + B < n_ao ? a0 + B : n_ao;
    const double* ck = v.C + (long)k * n_ao;
    int a = a0;
    for (; a + 8 <= a1; a += 8) {
      double cv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) cv[u] = ck[a + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += chi[q * n_ao + a + u] * cv[u];
      }
    }
    for (; a < a1; ++a) {
      const double cak = ck[a];
#pragma unroll
      for (int q = 0; q < NQ; ++q) acc[q] += chi[q * n_ao + a] * cak;
    }
  }
#pragma unroll
  for (int q = 0; q < NQ; ++q) part[q * 64 + lane] = acc[q];
  __syncthreads();
  if (lane < n) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = 0.0;
      for (int t = 0; t < P; ++t) s += part[q * 64 + lane * P + t];
      out[q * ostride + lane] = s;
    }
  }
  __syncthreads();
}

// In-place Gauss-Jordan inverse with partial pivoting of the n x n matrix in the left half
// of aug [n][2n] (row-major); the inverse ends in the right half. Returns false (uniformly)
// when a pivot is exactly zero.
__device__ bool vmc_invert(double* aug, int n, double* fac, int* piv) {
  const int lane = threadIdx.x;
  const int w = 2 * n;
  for (int r = lane; r < n * w; r += 64) {
    const int i = r / w, c = r - i * w;
    if (c >= n) aug[r] = (c - n == i) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int p = 0; p < n; ++p) {
    if (lane == 0) {
      int best = p;
      double bv = fabs(aug[p * w + p]);
      for (int r = p + 1; r < n; ++r) {
        const double v = fabs(aug[r * w + p]);
        if (v > bv) { bv = v; best = r; }
      }
      piv[0] = bv > 0.0 ? best : -1;
    }
    __syncthreads();
    const int pr = piv[0];
    if (pr < 0) return false;
    if (pr != p) {
      for (int c = lane; c < w; c += 64) {
        const double t = aug[p * w + c];
        aug[p * w + c] = aug[pr * w + c];
        aug[pr * w + c] = t;
      }
      __syncthreads();
    }
    const double inv = 1.0 / aug[p * w + p];
    __syncthreads();
    for (int c = lane; c < w; c += 64) aug[p * w + c] *= inv;
    for (int r = lane; r < n; r += 64) fac[r] = aug[r * w + p];
    __syncthreads();
    for (int e = lane; e < n * w; e += 64) {
      const int r = e / w, c = e - r * w;
      if (r != p) aug[e] -= fac[r] * aug[p * w + c];
    }
    __syncthreads();
  }
  return true;
}

// r + s * e with the product and the sum rounded separately (no fused multiply-add).
__device__ __forceinline__ double vmc_step(double r, double s, double e) {
#pragma clang fp contract(off)
  const double m = s * e;
  return r + m;
}

// ---------------------------------------------------------------------------------------
// Sampler: n_sweeps sweeps of single-electron moves, electrons in index order.
// LDS (doubles): shell centres [n_cent][4], primitives [n_prim][2], Ainv [2][n][n],
// aug [n][2n] for the starting inverses, whose space then holds the sweep's draws
// [n_el][4] (eta_x, eta_y, eta_z, u), phin [n], wv [n] and fac [n]; chi [n_ao], part [64]
// (also the inversion's scratch), R [n_el][3]; then ints: shell records [n_shell][2], piv.
__global__ __launch_bounds__(64) void k_vmc_sweeps(VmcDev v, double* __restrict__ R, long n_w,
                                                   int n_sweeps, double step,
                                                   const double* __restrict__ normals,
                                                   const double* __restrict__ uniforms,
                                                   long long* __restrict__ accepted) {
  extern __shared__ double lds[];
  const int n = v.n_occ, n_el = 2 * n, lane = threadIdx.x;
  const long w = blockIdx.x;
  double* cen = lds;
  double* prim = cen + 4 * v.b.n_cent;
  double* Ainv = prim + 2 * v.b.n_prim;
  double* aug = Ainv + 2 * n * n;
  double* dr = aug;   // after the starting inverses
  double* phin = dr + 4 * n_el;
  double* wv = phin + n;
  double* fac = wv + n;
  double* chi = aug + (2 * n * n > 11 * n ? 2 * n * n : 11 * n);
  double* part = chi + v.b.n_ao;
  double* Rs = part + 64;
  int* shi = (int*)(Rs + 3 * n_el);
  int* piv = shi + 2 * v.b.n_shell;
  for (int e = lane; e < 3 * n_el; e += 64) Rs[e] = R[w * 3 * n_el + e];
  vmc_stage(v.b, cen, shi, prim);
  __syncthreads();
  // inverse Slater matrices of the starting configuration
  for (int sp = 0; sp < 2; ++sp) {
    for (int ii = 0; ii < n; ++ii) {
      const int e = sp * n + ii;
      vmc_aos<false>(v.b, cen, shi, prim, Rs[3 * e], Rs[3 * e + 1], Rs[3 * e + 2], chi);
      __syncthreads();
      vmc_orbitals<1>(v, chi, part, aug + ii * 2 * n, 0);
    }
    if (!vmc_invert(aug, n, part, piv)) {   // part: free between orbital rows
      if (lane == 0) accepted[w] = -1;
      return;   // uniform over the (single-wave) workgroup
    }
    for (int e = lane; e < n * n; e += 64) {
      const int k = e / n, i = e - k * n;
      Ainv[sp * n * n + e] = aug[k * 2 * n + n + i];
    }
    __syncthreads();
  }
  long long acc = 0;
  // A sweep's draws (one record per electron) are loaded one sweep ahead by lanes
  // 0 .. n_el - 1 (vector loads, straight from HBM) and staged in LDS at the sweep's start.
  double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
  auto fetch = [&](int s) {
    if (lane < n_el) {
      const long di = ((long)s * n_el + lane) * n_w + w;
      q0 = normals[3 * di];
      q1 = normals[3 * di + 1];
      q2 = normals[3 * di + 2];
      q3 = uniforms[di];
    }
  };
  if (n_sweeps > 0) fetch(0);
  for (int s = 0; s < n_sweeps; ++s) {
    if (lane < n_el) {
      dr[4 * lane] = q0;
      dr[4 * lane + 1] = q1;
      dr[4 * lane + 2] = q2;
      dr[4 * lane + 3] = q3;
    }
    __syncthreads();
    if (s + 1 < n_sweeps) fetch(s + 1);
    for (int e = 0; e < n_el; ++e) {
      const int sp = e / n, ii = e - sp * n;
      const double u = dr[4 * e + 3];
      // r' = r + step * eta, rounded as two separate operations
      const double px = vmc_step(Rs[3 * e], step, dr[4 * e]);
      const double py = vmc_step(Rs[3 * e + 1], step, dr[4 * e + 1]);
      const double pz = vmc_step(Rs[3 * e + 2], step, dr[4 * e + 2]);
      vmc_aos<false>(v.b, cen, shi, prim, px, py, pz, chi);
      __syncthreads();
      vmc_orbitals<1>(v, chi, part, phin, 0);
      double* Ai = Ainv + sp * n * n;
      // wv[j] = sum_k phi_k(r') Ainv[k][j]; the determinant ratio is wv[ii]
      if (lane < n) {
        double t = 0.0;
#pragma unroll 8
        for (int k = 0; k < n; ++k) t += phin[k] * Ai[k * n + lane];
        wv[lane] = t;
      }
      __syncthreads();
      const double ratio = wv[ii];
      if (u < ratio * ratio) {
        // Sherman-Morrison for row ii of A replaced by phi(r'):
        // Ainv[k][j] -= Ainv[k][ii] (wv[j] - delta_{j ii}) / ratio
        if (lane < n) fac[lane] = Ai[lane * n + ii];
        __syncthreads();
        const double rinv = 1.0 / ratio;
        for (int q = lane; q < n * n; q += 64) {
          const int k = q / n, j = q - k * n;
          Ai[q] = (j == ii) ? fac[k] * rinv : Ai[q] - fac[k] * wv[j] * rinv;
        }
        if (lane == 0) {
          Rs[3 * e] = px;
          Rs[3 * e + 1] = py;
          Rs[3 * e + 2] = pz;
        }
        ++acc;
      }
      __syncthreads();
    }
  }
  for (int e = lane; e < 3 * n_el; e += 64) R[w * 3 * n_el + e] = Rs[e];
  if (lane == 0) accepted[w] = acc;
}

// ---------------------------------------------------------------------------------------
// The Slater part of a walker's local energy: A5[q][e][k] = (phi_k, d_x, d_y, d_z, lap)
// of the occupied orbitals at electron e, and the two inverse spin blocks Ainv[sp][k][i].
// Returns false (uniformly) when a determinant is exactly singular.
__device__ bool vmc_slater(const VmcDev& v, const double* cen, const int* shi, const double* prim,
                           const double* Rs, double* A5, double* aug, double* Ainv, double* chi,
                           double* part, double* fac, int* piv) {
  const int n = v.n_occ, n_el = 2 * n, lane = threadIdx.x;
  for (int e = 0; e < n_el; ++e) {
    vmc_aos<true>(v.b, cen, shi, prim, Rs[3 * e], Rs[3 * e + 1], Rs[3 * e + 2], chi);
    __syncthreads();
    vmc_orbitals<5>(v, chi, part, A5 + e * n, n_el * n);
  }
  for (int sp = 0; sp < 2; ++sp) {
    for (int q = lane; q < n * n; q += 64) {
      const int i = q / n, k = q - i * n;
      aug[i * 2 * n + k] = A5[(sp * n + i) * n + k];
    }
    __syncthreads();
    if (!vmc_invert(aug, n, fac, piv)) return false;
    for (int q = lane; q < n * n; q += 64) {
      const int k = q / n, i = q - k * n;
      Ainv[sp * n * n + q] = aug[k * 2 * n + n + i];
    }
    __syncthreads();
  }
  return true;
}

// D_i = grad_i Phi_0 / Phi_0 and S_i = lap_i Phi_0 / Phi_0 for electron i (Jacobi).
__device__ __forceinline__ void vmc_ratios(const VmcDev& v, const double* A5, const double* Ainv,
                                           int i, double& Dx, double& Dy, double& Dz,
                                           double& S) {
  const int n = v.n_occ, n_el = 2 * n, sp = i / n, ii = i - sp * n;
  const double* Ai = Ainv + sp * n * n;
  Dx = Dy = Dz = S = 0.0;
  for (int k = 0; k < n; ++k) {
    const double a = Ai[k * n + ii];
    Dx += A5[(n_el + i) * n + k] * a;
    Dy += A5[(2 * n_el + i) * n + k] * a;
    Dz += A5[(3 * n_el + i) * n + k] * a;
    S += A5[(4 * n_el + i) * n + k] * a;
  }
}

// ---------------------------------------------------------------------------------------
// Local energy and its parameter derivatives, one walker per workgroup.
// LDS (doubles): shell centres [n_cent][4], primitives [n_prim][2], A5 [5][n_el][n],
// aug [n][2n], Ainv [2][n][n], chi [5][n_ao], part [5][64], fac [n], R [n_el][3], red [64];
// then ints: shell records [n_shell][2], piv.
__global__ __launch_bounds__(64) void k_vmc_energy(VmcDev v, EECoefV cf,
                                                   const double* __restrict__ R, long n_w,
                                                   double* __restrict__ E,
                                                   double* __restrict__ dE) {
  extern __shared__ double lds[];
  const int n = v.n_occ, n_el = 2 * n, lane = threadIdx.x;
  const long w = blockIdx.x;
  const int nth = cf.n + 1;
  double* cen = lds;
  double* prim = cen + 4 * v.b.n_cent;
  double* A5 = prim + 2 * v.b.n_prim;
  double* aug = A5 + 5 * n_el * n;
  double* Ainv = aug + 2 * n * n;
  double* chi = Ainv + 2 * n * n;
  double* part = chi + 5 * v.b.n_ao;
  double* fac = part + 5 * 64;
  double* Rs = fac + n;
  double* red = Rs + 3 * n_el;
  int* shi = (int*)(red + 64);
  int* piv = shi + 2 * v.b.n_shell;
  for (int e = lane; e < 3 * n_el; e += 64) Rs[e] = R[w * 3 * n_el + e];
  vmc_stage(v.b, cen, shi, prim);
  __syncthreads();
  if (!vmc_slater(v, cen, shi, prim, Rs, A5, aug, Ainv, chi, part, fac, piv)) {
    // exactly singular reference determinant: no local energy
    if (lane == 0) {
      E[w] = __builtin_nan("");
      if (dE)
        for (int p = 0; p < nth; ++p) dE[w * nth + p] = __builtin_nan("");
    }
    return;
  }
  // per electron (lane i): Slater ratios, Jastrow sums, potential
  double ekin = 0.0, pot = 0.0;
  double dEp[VMC_MAX_TERMS + 1];
#pragma unroll
  for (int p = 0; p <= VMC_MAX_TERMS; ++p) dEp[p] = 0.0;
  if (lane < n_el) {
    const int i = lane;
    double Dx, Dy, Dz, S;
    vmc_ratios(v, A5, Ainv, i, Dx, Dy, Dz, S);
    const double xi = Rs[3 * i], yi = Rs[3 * i + 1], zi = Rs[3 * i + 2];
    double Gx = 0.0, Gy = 0.0, Gz = 0.0, Lj = 0.0;
    double gk[VMC_MAX_TERMS + 1][3], lk[VMC_MAX_TERMS + 1];
#pragma unroll
    for (int p = 0; p <= VMC_MAX_TERMS; ++p) gk[p][0] = gk[p][1] = gk[p][2] = lk[p] = 0.0;
    const double d = cf.d;
    for (int j = 0; j < n_el; ++j) {
      if (j == i) continue;
      const double dx = xi - Rs[3 * j], dy = yi - Rs[3 * j + 1], dz = zi - Rs[3 * j + 2];
      const double r = sqrt(dx * dx + dy * dy + dz * dz);
      const double rinv = 1.0 / r;
      if (j > i) pot += rinv;
      const double t = 1.0 / (1.0 + d * r);
      const double e = d * r * t;
      const double t2 = t * t, t3 = t2 * t, t4 = t2 * t2;
      double up = 0.0, upp = 0.0, upd = 0.0, uppd = 0.0;
#pragma unroll
      for (int k = 0; k < VMC_MAX_TERMS; ++k) {
        if (k < cf.n) {
          const int o = cf.o[k];
          // e^{o-1}, e^{o-2} (o >= 1; terms with o = 0 are constant and drop out)
          double em1 = 1.0, em2 = 1.0;
          for (int q = 0; q < o - 2; ++q) em2 *= e;
          em1 = o >= 2 ? em2 * e : 1.0;
          if (o == 0) continue;
          // f' = o e^{o-1} d t^2, f'' = o (o-1) e^{o-2} d^2 t^4 - 2 o e^{o-1} d^2 t^3
          const double fp = o * em1 * d * t2;
          const double fpp = (o >= 2 ? o * (o - 1) * em2 * d * d * t4 : 0.0) -
                             2.0 * o * em1 * d * d * t3;
          // d/dd: [d t^2 e^m]' = t^2 e^m (1 - 2e + m t); [d^2 t^4 e^m]' = d t^4 e^m
          // (2 - 4e + m t); [d^2 t^3 e^m]' = d t^3 e^m (2 - 3e + m t)
          const double fpd = o * t2 * em1 * (1.0 - 2.0 * e + (o - 1) * t);
          const double fppd = (o >= 2 ? o * (o - 1) * d * t4 * em2 * (2.0 - 4.0 * e + (o - 2) * t) : 0.0) -
                              2.0 * o * d * t3 * em1 * (2.0 - 3.0 * e + (o - 1) * t);
          const double c = cf.c[k];
          up += c * fp;
          upp += c * fpp;
          upd += c * fpd;
          uppd += c * fppd;
          const double s = fp * rinv;
          gk[k][0] += s * dx;
          gk[k][1] += s * dy;
          gk[k][2] += s * dz;
          lk[k] += fpp + 2.0 * s;
        }
      }
      const double s = up * rinv;
      Gx += s * dx;
      Gy += s * dy;
      Gz += s * dz;
      Lj += upp + 2.0 * s;
      const double sd = upd * rinv;
      gk[VMC_MAX_TERMS][0] += sd * dx;
      gk[VMC_MAX_TERMS][1] += sd * dy;
      gk[VMC_MAX_TERMS][2] += sd * dz;
      lk[VMC_MAX_TERMS] += uppd + 2.0 * sd;
    }
    for (int I = 0; I < v.n_nuc; ++I) {
      const double dx = xi - v.nuc[4 * I], dy = yi - v.nuc[4 * I + 1], dz = zi - v.nuc[4 * I + 2];
      pot -= v.nuc[4 * I + 3] / sqrt(dx * dx + dy * dy + dz * dz);
    }
    // lap_i Psi / Psi = lap J + |grad J|^2 + 2 grad J . D + S
    ekin = -0.5 * (Lj + Gx * Gx + Gy * Gy + Gz * Gz + 2.0 * (Gx * Dx + Gy * Dy + Gz * Dz) + S);
    const double hx = Gx + Dx, hy = Gy + Dy, hz = Gz + Dz;
#pragma unroll
    for (int p = 0; p <= VMC_MAX_TERMS; ++p)
      dEp[p] = -0.5 * (lk[p] + 2.0 * (hx * gk[p][0] + hy * gk[p][1] + hz * gk[p][2]));
  }
  // fixed-order sums over the electrons (lanes)
  auto lane_sum = [&](double x) {
    red[lane] = x;
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
      if (lane < h) red[lane] += red[lane + h];
      __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
  };
  const double Etot = lane_sum(ekin + pot);
  if (lane == 0) E[w] = Etot + v.e_nuc;
  if (dE) {
    for (int p = 0; p < cf.n; ++p) {
      double x = 0.0;
#pragma unroll
      for (int q = 0; q < VMC_MAX_TERMS; ++q)
        if (q == p) x = dEp[q];
      const double s = lane_sum(x);
      if (lane == 0) dE[w * nth + p] = s;
    }
    const double s = lane_sum(dEp[VMC_MAX_TERMS]);
    if (lane == 0) dE[w * nth + cf.n] = s;
  }
}

// ---------------------------------------------------------------------------------------
// Local energy of the BH correlator (eq. bh-u) and its derivatives in every parameter.
// u(r_i, r_j) = sum_I sum_k c[type I][k] (a_i^m a_j^n + a_j^m a_i^n) e^o with a = a(r_.I),
// e = rbar(r_ij). For electron i, per (j, I) and with P(a_i) = a_i^m a_j^n + a_j^m a_i^n:
//   grad_i f = c [P_a e^o grad a_i + P o e^{o-1} grad e],
//   lap_i f  = c [P_aa e^o |grad a_i|^2 + P_a e^o lap a_i + 2 P_a o e^{o-1} grad a_i . grad e
//                + P (o (o-1) e^{o-2} |grad e|^2 + o e^{o-1} lap e)],
// s = x r / (1 + x r): s' = x t^2, s'' = -2 x^2 t^3, grad s = (s'/r) (r - R), lap s = s'' + 2 s'/r;
// in x: ds = r t^2, ds' = t^2 (1 - 2 s), ds'' = x t^3 (6 s - 4).
constexpr int VMC_BH_MAXNUC = 24, VMC_BH_MAXTYPE = 2, VMC_BH_MAXTERM = 64, VMC_BH_MAXO = 12;
// per (electron, nucleus): a, da/db, ga, dga/db, la, dla/db, r - R (3), a^2, a^3
constexpr int VMC_BH_TA = 6;
constexpr int VMC_BH_NO = VMC_BH_MAXO + 1;

struct VmcBH {
  const double* nuc;   // [n_nuc][4]: x, y, z, type
  const double* bt;    // [n_types]
  const double* c;     // [n_types][n_terms]
  const int* mno;      // [n_terms][3]
  const double* cs;    // [n_types][4][4][13]: coefficients summed per (min(m,n), max(m,n), o)
  const int* on;       // [n_types][4][4]: 1 + the largest o with a coefficient (0: none)
  const int* gst;      // [n_types][11]: start of each (m <= n) group's terms in gtm
  const int* gtm;      // [n_types][VMC_BH_MAXTERM]: term k | o << 8, grouped by (m <= n)
  int n_nuc, n_types, n_terms;
  double d;
};

// value and derivative in one seeded parameter (forward mode)
struct Dl {
  double v, d;
};
__device__ __forceinline__ Dl operator+(Dl a, Dl b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dl operator*(Dl a, Dl b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dl operator*(double s, Dl a) { return {s * a.v, s * a.d}; }
__device__ __forceinline__ Dl operator*(Dl a, double s) { return {a.v * s, a.d * s}; }
__device__ __forceinline__ Dl operator+(Dl a, double s) { return {a.v + s, a.d}; }
// the type of a product or sum of a T and a U (a dual when either is one)
template <class T, class U> struct DlJoin { typedef Dl type; };
template <> struct DlJoin<double, double> { typedef double type; };
template <class T> __device__ __forceinline__ T vmc_mk(double v, double d);
template <> __device__ __forceinline__ double vmc_mk<double>(double v, double) { return v; }
template <> __device__ __forceinline__ Dl vmc_mk<Dl>(double v, double d) { return {v, d}; }
template <class T> __device__ __forceinline__ T vmc_zero() { return vmc_mk<T>(0.0, 0.0); }

// The partners j = j0, j0 + js, ... of electron i: their share of grad_i J and lap_i J. The derivative in one parameter `seed` (0: d,
// 1 + t: b_t) rides along as a dual number: d moves only the pair quantities (e and its
// derivatives, type TE), b_t only the nuclear ones (a and its derivatives, type TN), so
// each seed makes just one side dual; TR joins the two. TA: the per-(electron, nucleus)
// table in LDS.
template <class TE, class TN, class TR = typename DlJoin<TE, TN>::type>
__device__ void vmc_bh_jastrow(const VmcBH& bh, const double* TA, const double* Rs, int n_el,
                               int i, int seed, int j0, int js, TR& Gx, TR& Gy, TR& Gz, TR& L) {
  Gx = Gy = Gz = L = vmc_zero<TR>();
  const double d = bh.d;
  const int nn = bh.n_nuc;
  for (int j = j0; j < n_el; j += js) {   // the partners j0, j0 + js, ...
    if (j == i) continue;
    const double dx = Rs[3 * i] - Rs[3 * j], dy = Rs[3 * i + 1] - Rs[3 * j + 1],
                 dz = Rs[3 * i + 2] - Rs[3 * j + 2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz), rinv = 1.0 / r;
    const double t = 1.0 / (1.0 + d * r), e = d * r * t, e1 = d * t * t, e2 = -2.0 * d * d * t * t * t;
    const bool sd = seed == 0;
    const double de = r * t * t, de1 = t * t * (1.0 - 2.0 * e), de2 = d * t * t * t * (6.0 * e - 4.0);
    const TE E = vmc_mk<TE>(e, sd ? de : 0.0);
    const TE ge = vmc_mk<TE>(e1 * rinv, sd ? de1 * rinv : 0.0);
    const TE le = vmc_mk<TE>(e2 + 2.0 * e1 * rinv, sd ? de2 + 2.0 * de1 * rinv : 0.0);
    const TE ge2 = (r * r) * (ge * ge);
    for (int ty = 0; ty < bh.n_types; ++ty) {
      // the o-sums of each (m <= n) group depend on the pair and the nucleus type only:
      // W[g] = (q(e), q'(e), q''(e)) for q(e) = sum_o c_o e^o, formed once per type by
      // Horner's rule with its first two derivatives (a rolled loop: the kernel's code
      // stays small)
      TE W[10][3];
#pragma unroll
      for (int m = 0, g = 0; m < 4; ++m) {
#pragma unroll
        for (int n = m; n < 4; ++n, ++g) {
          const int on = bh.on[(ty * 4 + m) * 4 + n];
          const double* cw = bh.cs + ((ty * 4 + m) * 4 + n) * VMC_BH_NO;
          TE q0 = vmc_zero<TE>(), q1 = q0, q2 = q0;   // q, q', q''/2
          for (int o = on - 1; o >= 0; --o) {   // wave-uniform bound
            q2 = q2 * E + q1;
            q1 = q1 * E + q0;
            q0 = q0 * E + cw[o];
          }
          W[g][0] = q0;
          W[g][1] = q1;
          W[g][2] = 2.0 * q2;
        }
      }
      const bool sb = seed == 1 + ty;
      for (int I = 0; I < nn; ++I) {
        if ((int)bh.nuc[4 * I + 3] != ty) continue;   // wave-uniform
        const double* ti = TA + ((long)i * nn + I) * VMC_BH_TA;
        const double* tj = TA + ((long)j * nn + I) * VMC_BH_TA;
        const TN A = vmc_mk<TN>(ti[0], sb ? ti[1] : 0.0);
        const TN Aj = vmc_mk<TN>(tj[0], sb ? tj[1] : 0.0);
        const TN GA = vmc_mk<TN>(ti[2], sb ? ti[3] : 0.0);
        const TN LA = vmc_mk<TN>(ti[4], sb ? ti[5] : 0.0);
        const double Dix = Rs[3 * i] - bh.nuc[4 * I], Diy = Rs[3 * i + 1] - bh.nuc[4 * I + 1],
                     Diz = Rs[3 * i + 2] - bh.nuc[4 * I + 2];
        TN pa[4], pj[4];
        pa[0] = pj[0] = vmc_mk<TN>(1.0, 0.0);
#pragma unroll
        for (int q = 1; q < 4; ++q) {
          pa[q] = pa[q - 1] * A;
          pj[q] = pj[q - 1] * Aj;
        }
        // P = a^m a'^n + a'^m a^n is symmetric in (m, n), hence the grouping by m <= n
        TR S1 = vmc_zero<TR>(), S2 = S1, S3 = S1, S4 = S1, S5 = S1;
#pragma unroll
        for (int m = 0, g = 0; m < 4; ++m) {
#pragma unroll
          for (int n = m; n < 4; ++n, ++g) {
            if (bh.on[(ty * 4 + m) * 4 + n] == 0) continue;   // wave-uniform
            const TN P = m == n ? 2.0 * (pa[m] * pj[m]) : pa[m] * pj[n] + pj[m] * pa[n];
            TN Pa = vmc_zero<TN>(), Paa = Pa;
            if (m >= 1) Pa = Pa + (double)m * (pa[m - 1] * pj[n]);
            if (n >= 1) Pa = Pa + (double)n * (pj[m] * pa[n - 1]);
            if (m >= 2) Paa = Paa + (double)(m * (m - 1)) * (pa[m - 2] * pj[n]);
            if (n >= 2) Paa = Paa + (double)(n * (n - 1)) * (pj[m] * pa[n - 2]);
            S1 = S1 + Pa * W[g][0];
            S2 = S2 + P * W[g][1];
            S3 = S3 + Paa * W[g][0];
            S4 = S4 + Pa * W[g][1];
            S5 = S5 + P * W[g][2];
          }
        }
        // grad a = GA (r_i - R_I), grad e = ge (r_i - r_j)
        const double dd = Dix * dx + Diy * dy + Diz * dz, di2 = Dix * Dix + Diy * Diy + Diz * Diz;
        const TN ga2 = di2 * (GA * GA);
        const TR gage = dd * (GA * ge);
        Gx = Gx + Dix * (S1 * GA) + dx * (S2 * ge);
        Gy = Gy + Diy * (S1 * GA) + dy * (S2 * ge);
        Gz = Gz + Diz * (S1 * GA) + dz * (S2 * ge);
        L = L + S3 * ga2 + S1 * LA + 2.0 * (S4 * gage) + S5 * ge2 + S2 * le;
      }
    }
  }
}

__device__ __forceinline__ double vmc_wave_sum(double x) {   // fixed butterfly order
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Pass 2: dE/dc[t][k] = -1/2 sum_i sum_{j != i} sum_{I of type t} [lap_i f + 2 h_i . grad_i f]
// for the unit kernel f of term k, h_i = grad_i J + grad_i Phi_0 / Phi_0. Lanes over the
// ordered electron pairs (i, j). Per pair and nucleus type, the nuclear sums of each
// (m <= n) group, Y0 = sum_I Paa |grad a|^2 + Pa (lap a + 2 h.grad a),
// Y1 = sum_I Pa ga (r_i - R_I).(r_i - r_j) (grad a = ga (r_i - R_I), grad e = ge (r_i - r_j))
// and Y2 = sum_I P, serve every term of the group: a term of power o contributes
// E0 Y0 + E1 (2 ge Y1 + (le + 2 h.grad e) Y2) + E2 |grad e|^2 Y2 with E0 = e^o,
// E1 = o e^(o-1), E2 = o (o-1) e^(o-2). Each term's pair values are summed over the wave
// (fixed order) and lane 0 adds them to acc[t][k] in LDS, pair block by pair block.
__device__ void vmc_bh_dc_pairs(const VmcBH& bh, const double* TA, const double* Rs,
                                const double* H, int n_el, double* acc) {
  const int lane = threadIdx.x, nn = bh.n_nuc, np = n_el * (n_el - 1);
  const double d = bh.d;
  for (int q0 = 0; q0 < np; q0 += 64) {   // wave-uniform
    const int q = q0 + lane;
    const bool live = q < np;
    const int qq = live ? q : 0;
    const int i = qq / (n_el - 1), jj = qq - i * (n_el - 1), j = jj + (jj >= i ? 1 : 0);
    const double hx = H[4 * i], hy = H[4 * i + 1], hz = H[4 * i + 2];
    const double dx = Rs[3 * i] - Rs[3 * j], dy = Rs[3 * i + 1] - Rs[3 * j + 1],
                 dz = Rs[3 * i + 2] - Rs[3 * j + 2];
    const double r = sqrt(dx * dx + dy * dy + dz * dz), rinv = 1.0 / r;
    const double t = 1.0 / (1.0 + d * r), e = d * r * t, e1 = d * t * t,
                 e2 = -2.0 * d * d * t * t * t;
    const double ge = e1 * rinv, le = e2 + 2.0 * e1 * rinv, ge2 = e1 * e1;
    const double hge = ge * (hx * dx + hy * dy + hz * dz);
    for (int ty = 0; ty < bh.n_types; ++ty) {
      double Y[10][3];
#pragma unroll
      for (int g = 0; g < 10; ++g) Y[g][0] = Y[g][1] = Y[g][2] = 0.0;
      for (int I = 0; I < nn; ++I) {
        if ((int)bh.nuc[4 * I + 3] != ty) continue;   // wave-uniform
        const double* ti = TA + ((long)i * nn + I) * VMC_BH_TA;
        const double* tj = TA + ((long)j * nn + I) * VMC_BH_TA;
        const double ga = ti[2], la = ti[4];
        const double Dix = Rs[3 * i] - bh.nuc[4 * I], Diy = Rs[3 * i + 1] - bh.nuc[4 * I + 1],
                     Diz = Rs[3 * i + 2] - bh.nuc[4 * I + 2];
        const double di2 = Dix * Dix + Diy * Diy + Diz * Diz, dd = Dix * dx + Diy * dy + Diz * dz;
        const double u0 = ga * ga * di2, u1 = la + 2.0 * ga * (hx * Dix + hy * Diy + hz * Diz),
                     u2 = ga * dd;
        double pa[4], pj[4];
        pa[0] = pj[0] = 1.0;
#pragma unroll
        for (int k = 1; k < 4; ++k) {
          pa[k] = pa[k - 1] * ti[0];
          pj[k] = pj[k - 1] * tj[0];
        }
#pragma unroll
        for (int m = 0, g = 0; m < 4; ++m) {
#pragma unroll
          for (int n = m; n < 4; ++n, ++g) {
            if (bh.on[(ty * 4 + m) * 4 + n] == 0) continue;   // wave-uniform
            const double P = m == n ? 2.0 * (pa[m] * pj[m]) : pa[m] * pj[n] + pj[m] * pa[n];
            double Pa = 0.0, Paa = 0.0;
            if (m >= 1) Pa += m * (pa[m - 1] * pj[n]);
            if (n >= 1) Pa += n * (pj[m] * pa[n - 1]);
            if (m >= 2) Paa += (m * (m - 1)) * (pa[m - 2] * pj[n]);
            if (n >= 2) Paa += (n * (n - 1)) * (pj[m] * pa[n - 2]);
            Y[g][0] += Paa * u0 + Pa * u1;
            Y[g][1] += Pa * u2;
            Y[g][2] += P;
          }
        }
      }
#pragma unroll
      for (int g = 0; g < 10; ++g) {
        const int x1 = bh.gst[ty * 11 + g + 1];
        for (int x = bh.gst[ty * 11 + g]; x < x1; ++x) {   // wave-uniform
          const int ko = bh.gtm[ty * VMC_BH_MAXTERM + x], k = ko & 255, o = ko >> 8;
          const double eo2 = vmc_ipow_to<VMC_BH_MAXO>(e, o >= 2 ? o - 2 : 0);
          const double eo1 = o >= 2 ? eo2 * e : 1.0, eo = o >= 2 ? eo1 * e : (o == 1 ? e : 1.0);
          const double E1 = o >= 1 ? o * eo1 : 0.0, E2 = o >= 2 ? (o * (o - 1)) * eo2 : 0.0;
          const double val = eo * Y[g][0] + E1 * (2.0 * ge * Y[g][1] + (le + 2.0 * hge) * Y[g][2]) +
                             E2 * ge2 * Y[g][2];
          const double sum = vmc_wave_sum(live ? val : 0.0);
          if (lane == 0) acc[ty * bh.n_terms + k] += sum;
        }
      }
    }
  }
}

// LDS (doubles): A5 [5][n_el][n], Ainv [2][n][n], fac [n], R [n_el][3], red [64],
// H [n_el][4] (h_i, then spare), the nuclei [n_nuc][4] (read in every pair's nuclear
// loop), pass 2's sums [2][64], the partner-group partial sums [64][8], then one region
// used twice: during the Slater part
// shell centres [n_cent][4], primitives [n_prim][2], aug [n][2n], chi [5][n_ao],
// part [5][64] and the ints (shell records [n_shell][2], piv); after it the
// per-(electron, nucleus) table TA [n_el][n_nuc][6]. Sharing the region keeps a
// walker's LDS small enough for four workgroups per CU at H20.
__global__ __launch_bounds__(64) void k_vmc_energy_bh(VmcDev v, VmcBH bh_in,
                                                      const double* __restrict__ R, long n_w,
                                                      double* __restrict__ E,
                                                      double* __restrict__ dE) {
  extern __shared__ double lds[];
  const int n = v.n_occ, n_el = 2 * n, lane = threadIdx.x;
  const long w = blockIdx.x;
  const int nlin = bh_in.n_types * bh_in.n_terms, nth = nlin + 1 + bh_in.n_types;
  const int nn = bh_in.n_nuc;
  double* A5 = lds;
  double* Ainv = A5 + 5 * n_el * n;
  double* fac = Ainv + 2 * n * n;
  double* Rs = fac + n;
  double* red = Rs + 3 * n_el;
  double* H = red + 64;
  double* nuc = H + 4 * n_el;
  double* acc = nuc + 4 * nn;   // pass 2's sums [n_types][n_terms]
  double* PJ = acc + VMC_BH_MAXTYPE * VMC_BH_MAXTERM;   // partner-group partial sums [64][8]
  double* cen = PJ + 64 * 8;    // the shared region
  double* prim = cen + 4 * v.b.n_cent;
  double* aug = prim + 2 * v.b.n_prim;
  double* chi = aug + 2 * n * n;
  double* part = chi + 5 * v.b.n_ao;
  int* shi = (int*)(part + 5 * 64);
  int* piv = shi + 2 * v.b.n_shell;
  double* TA = cen;
  for (int e = lane; e < 3 * n_el; e += 64) Rs[e] = R[w * 3 * n_el + e];
  for (int e = lane; e < 4 * nn; e += 64) nuc[e] = bh_in.nuc[e];
  VmcBH bh = bh_in;
  bh.nuc = nuc;
  vmc_stage(v.b, cen, shi, prim);
  __syncthreads();
  if (!vmc_slater(v, cen, shi, prim, Rs, A5, aug, Ainv, chi, part, fac, piv)) {
    if (lane == 0) {
      E[w] = __builtin_nan("");
      if (dE)
        for (int p = 0; p < nth; ++p) dE[w * nth + p] = __builtin_nan("");
    }
    return;
  }
  __syncthreads();   // the Slater part's tables are dead: TA takes their place
  // the per-(electron, nucleus) table: a, da/db, (a'/r), d(a'/r)/db, lap a, d lap a/db
  for (int q = lane; q < n_el * nn; q += 64) {
    const int e = q / nn, I = q - e * nn;
    const double Dx = Rs[3 * e] - bh.nuc[4 * I], Dy = Rs[3 * e + 1] - bh.nuc[4 * I + 1],
                 Dz = Rs[3 * e + 2] - bh.nuc[4 * I + 2];
    const double r = sqrt(Dx * Dx + Dy * Dy + Dz * Dz), rinv = 1.0 / r;
    const double b = bh.bt[(int)bh.nuc[4 * I + 3]];
    const double t = 1.0 / (1.0 + b * r), a = b * r * t, a1 = b * t * t, a2 = -2.0 * b * b * t * t * t;
    const double da = r * t * t, da1 = t * t * (1.0 - 2.0 * a), da2 = b * t * t * t * (6.0 * a - 4.0);
    double* o = TA + (long)q * VMC_BH_TA;
    o[0] = a;
    o[1] = da;
    o[2] = a1 * rinv;
    o[3] = da1 * rinv;
    o[4] = a2 + 2.0 * a1 * rinv;
    o[5] = da2 + 2.0 * da1 * rinv;
  }
  __syncthreads();
  auto lane_sum = [&](double x) {
    red[lane] = x;
    __syncthreads();
    for (int h = 32; h > 0; h >>= 1) {
      if (lane < h) red[lane] += red[lane + h];
      __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
  };
  // Passes 1 and 3 put the lanes over (electron i, partner group gj): the partners of i
  // are split into NG strided groups, each lane sums its group, and lane i adds the
  // groups' partial sums in order.
  const int NG = 64 / n_el, gi = lane % n_el, gj = lane / n_el;
  // pass 1: local energy; h_i = grad_i J + D_i to LDS
  if (gj < NG) {
    double gx, gy, gz, l;
    vmc_bh_jastrow<double, double>(bh, TA, Rs, n_el, gi, -1, gj, NG, gx, gy, gz, l);
    double* o = PJ + 8 * (gj * n_el + gi);
    o[0] = gx;
    o[1] = gy;
    o[2] = gz;
    o[3] = l;
  }
  __syncthreads();
  double ekin = 0.0, pot = 0.0, Dx = 0.0, Dy = 0.0, Dz = 0.0, Gx = 0.0, Gy = 0.0, Gz = 0.0;
  if (lane < n_el) {
    const int i = lane;
    double S, L = 0.0;
    vmc_ratios(v, A5, Ainv, i, Dx, Dy, Dz, S);
    for (int g = 0; g < NG; ++g) {
      const double* o = PJ + 8 * (g * n_el + i);
      Gx += o[0];
      Gy += o[1];
      Gz += o[2];
      L += o[3];
    }
    ekin = -0.5 * (L + Gx * Gx + Gy * Gy + Gz * Gz + 2.0 * (Gx * Dx + Gy * Dy + Gz * Dz) + S);
    const double xi = Rs[3 * i], yi = Rs[3 * i + 1], zi = Rs[3 * i + 2];
    for (int j = i + 1; j < n_el; ++j) {
      const double ax = xi - Rs[3 * j], ay = yi - Rs[3 * j + 1], az = zi - Rs[3 * j + 2];
      pot += 1.0 / sqrt(ax * ax + ay * ay + az * az);
    }
    for (int I = 0; I < v.n_nuc; ++I) {
      const double ax = xi - v.nuc[4 * I], ay = yi - v.nuc[4 * I + 1], az = zi - v.nuc[4 * I + 2];
      pot -= v.nuc[4 * I + 3] / sqrt(ax * ax + ay * ay + az * az);
    }
    H[4 * i] = Gx + Dx;
    H[4 * i + 1] = Gy + Dy;
    H[4 * i + 2] = Gz + Dz;
    H[4 * i + 3] = 0.0;
  }
  const double Etot = lane_sum(ekin + pot);
  if (lane == 0) E[w] = Etot + v.e_nuc;
  if (!dE) return;   // uniform
  // pass 2: the linear coefficients
  for (int p = lane; p < nlin; p += 64) acc[p] = 0.0;
  __syncthreads();
  vmc_bh_dc_pairs(bh, TA, Rs, H, n_el, acc);
  __syncthreads();
  for (int p = lane; p < nlin; p += 64) dE[w * nth + p] = -0.5 * acc[p];
  // pass 3: d and each b_t in forward mode
  for (int sd = 0; sd <= bh.n_types; ++sd) {
    if (gj < NG) {
      Dl gx, gy, gz, l;
      if (sd == 0) vmc_bh_jastrow<Dl, double>(bh, TA, Rs, n_el, gi, sd, gj, NG, gx, gy, gz, l);
      else vmc_bh_jastrow<double, Dl>(bh, TA, Rs, n_el, gi, sd, gj, NG, gx, gy, gz, l);
      double* o = PJ + 8 * (gj * n_el + gi);
      o[0] = gx.v;
      o[1] = gx.d;
      o[2] = gy.v;
      o[3] = gy.d;
      o[4] = gz.v;
      o[5] = gz.d;
      o[6] = l.v;
      o[7] = l.d;
    }
    __syncthreads();
    double x = 0.0;
    if (lane < n_el) {
      Dl gx = {0.0, 0.0}, gy = gx, gz = gx, l = gx;
      for (int g = 0; g < NG; ++g) {
        const double* o = PJ + 8 * (g * n_el + lane);
        gx = gx + Dl{o[0], o[1]};
        gy = gy + Dl{o[2], o[3]};
        gz = gz + Dl{o[4], o[5]};
        l = l + Dl{o[6], o[7]};
      }
      x = -0.5 * (l.d + 2.0 * ((gx.v + Dx) * gx.d + (gy.v + Dy) * gy.d + (gz.v + Dz) * gz.d));
    }
    const double s = lane_sum(x);
    if (lane == 0) dE[w * nth + nlin + sd] = s;
  }
}

// ---------------------------------------------------------------------------------------
// Gauss-Newton step (eq. gn) on the clipped variance (eq. var-loss), one workgroup of
// VMC_GN_THREADS threads.
__device__ double gn_block_sum(double x, double* red) {
  const int t = threadIdx.x;
  red[t] = x;
  __syncthreads();
  for (int h = VMC_GN_THREADS / 2; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

struct GnShared {
  double red[VMC_GN_THREADS];
  double dm[VMC_MAX_THETA], dmad[VMC_MAX_THETA], mdt[VMC_MAX_THETA], grad[VMC_MAX_THETA];
  double C[VMC_MAX_THETA * VMC_MAX_THETA];
  double x[VMC_MAX_THETA];
};

__global__ __launch_bounds__(VMC_GN_THREADS) void k_vmc_gn(const double* __restrict__ E,
                                                           const double* __restrict__ dE, long N,
                                                           int nth, double lam, double eta,
                                                           double* __restrict__ delta,
                                                           double* __restrict__ stats) {
  __shared__ GnShared sh;
  const int t = threadIdx.x;
  const double inv_n = 1.0 / (double)N;
  double a = 0.0;
  for (long k = t; k < N; k += VMC_GN_THREADS) a += E[k];
  const double m = gn_block_sum(a, sh.red) * inv_n;
  a = 0.0;
  for (long k = t; k < N; k += VMC_GN_THREADS) a += fabs(E[k] - m);
  const double mad = gn_block_sum(a, sh.red) * inv_n;
  const double lo = m - 5.0 * mad, hi = m + 5.0 * mad;
  a = 0.0;
  double ncl = 0.0;
  for (long k = t; k < N; k += VMC_GN_THREADS) {
    const double e = E[k];
    a += e < lo ? lo : (e > hi ? hi : e);
    ncl += (e < lo || e > hi) ? 1.0 : 0.0;
  }
  const double mean = gn_block_sum(a, sh.red) * inv_n;
  const double nclip = gn_block_sum(ncl, sh.red);
  a = 0.0;
  for (long k = t; k < N; k += VMC_GN_THREADS) {
    const double e = E[k];
    const double r = (e < lo ? lo : (e > hi ? hi : e)) - mean;
    a += r * r;
  }
  const double var = gn_block_sum(a, sh.red) / (double)(N - 1);
  if (nth <= GN_FEW) {
    // few parameters: each sum is one block reduction over the walkers
    // derivatives of m and of the MAD, then of the clipped energies
    for (int p = 0; p < nth; ++p) {
      a = 0.0;
      for (long k = t; k < N; k += VMC_GN_THREADS) a += dE[k * nth + p];
      const double s = gn_block_sum(a, sh.red);
      if (t == 0) sh.dm[p] = s * inv_n;
    }
    __syncthreads();
    for (int p = 0; p < nth; ++p) {
      a = 0.0;
      for (long k = t; k < N; k += VMC_GN_THREADS) {
        const double df = E[k] - m;
        const double sg = df > 0.0 ? 1.0 : (df < 0.0 ? -1.0 : 0.0);
        a += sg * (dE[k * nth + p] - sh.dm[p]);
      }
      const double s = gn_block_sum(a, sh.red);
      if (t == 0) sh.dmad[p] = s * inv_n;
    }
    __syncthreads();
    auto dclip = [&](long k, int p) {
      const double e = E[k];
      if (e < lo) return sh.dm[p] - 5.0 * sh.dmad[p];
      if (e > hi) return sh.dm[p] + 5.0 * sh.dmad[p];
      return dE[k * nth + p];
    };
    for (int p = 0; p < nth; ++p) {
      a = 0.0;
      for (long k = t; k < N; k += VMC_GN_THREADS) a += dclip(k, p);
      const double s = gn_block_sum(a, sh.red);
      if (t == 0) sh.mdt[p] = s * inv_n;
    }
    __syncthreads();
    // residual r_k = Et_k - mean, dr_kp = dEt_kp - mean_k(dEt_kp)
    for (int p = 0; p < nth; ++p) {
      a = 0.0;
      for (long k = t; k < N; k += VMC_GN_THREADS) {
        const double e = E[k];
        const double r = (e < lo ? lo : (e > hi ? hi : e)) - mean;
        a += (dclip(k, p) - sh.mdt[p]) * r;
      }
      const double s = gn_block_sum(a, sh.red);
      if (t == 0) sh.grad[p] = 2.0 * s / (double)(N - 1);
    }
    for (int p = 0; p < nth; ++p) {
      for (int q = 0; q <= p; ++q) {
        a = 0.0;
        for (long k = t; k < N; k += VMC_GN_THREADS)
          a += (dclip(k, p) - sh.mdt[p]) * (dclip(k, q) - sh.mdt[q]);
        const double s = gn_block_sum(a, sh.red);
        if (t == 0) {
          const double c = s * inv_n + (p == q ? lam : 0.0);
          sh.C[p * nth + q] = c;
          sh.C[q * nth + p] = c;
        }
      }
    }
  } else {
    // The parameter sums run in walker order over tiles of tk walkers: a tile's dE rows are
    // staged in the space of C (not needed until the end) and its energies in red; one
    // thread per parameter column, and up to GN_BLK blocks of C per thread, a block being the
    // four entries (p, q0 .. q0 + 3), q0 a multiple of 4 not above p (one read of row p
    // serves four products).
    constexpr int GN_NBLK = VMC_MAX_THETA * (VMC_MAX_THETA / 4 + 1) / 2 + VMC_MAX_THETA;
    constexpr int GN_BLK = (GN_NBLK + VMC_GN_THREADS - 1) / VMC_GN_THREADS;
    const int tk = VMC_MAX_THETA * VMC_MAX_THETA / nth < VMC_GN_THREADS
                       ? VMC_MAX_THETA * VMC_MAX_THETA / nth : VMC_GN_THREADS;
    double* tile = sh.C;
    double* te = sh.red;
    auto stage = [&](long k0, int nk) {
      __syncthreads();   // the previous tile's readers are done
      for (int e = t; e < nk * nth; e += VMC_GN_THREADS) tile[e] = dE[k0 * nth + e];
      for (int e = t; e < nk; e += VMC_GN_THREADS) te[e] = E[k0 + e];
      __syncthreads();
    };
    auto tile_len = [&](long k0) { return (int)(N - k0 < tk ? N - k0 : tk); };
    // Column sums over the walkers: thread t takes column t % nth and the walkers of
    // segment t / nth (every S-th walker of each tile, S = threads / nth); the S partial
    // sums of a column are then added in segment order (fixed).
    const int S = VMC_GN_THREADS / nth, ccol = t % nth, cseg = t / nth;
    auto combine = [&](double a) {   // returns the column total on threads t < nth
      __syncthreads();
      te[t] = cseg < S ? a : 0.0;
      __syncthreads();
      double tot = 0.0;
      if (t < nth)
        for (int g = 0; g < S; ++g) tot += te[g * nth + t];
      return tot;
    };
    auto colsum = [&](auto f) {
      double a = 0.0;
      for (long k0 = 0; k0 < N; k0 += tk) {
        const int nk = tile_len(k0);
        stage(k0, nk);
        if (cseg < S)
          for (int kk = cseg; kk < nk; kk += S) a += f(kk, tile[kk * nth + ccol]);
      }
      return combine(a);
    };
    // derivatives of m and of the MAD, then of the clipped energies
    double a1 = colsum([&](int, double x) { return x; });
    if (t < nth) sh.dm[t] = a1 * inv_n;
    a1 = colsum([&](int kk, double x) {   // sh.dm is visible after the first tile's barrier
      const double df = te[kk] - m;
      return (df > 0.0 ? 1.0 : (df < 0.0 ? -1.0 : 0.0)) * (x - sh.dm[ccol]);
    });
    if (t < nth) sh.dmad[t] = a1 * inv_n;
    a1 = colsum([&](int kk, double x) {
      const double e = te[kk];
      return e < lo ? sh.dm[ccol] - 5.0 * sh.dmad[ccol]
                    : (e > hi ? sh.dm[ccol] + 5.0 * sh.dmad[ccol] : x);
    });
    if (t < nth) sh.mdt[t] = a1 * inv_n;
    // residual r_k = Et_k - mean and dr_kp = dEt_kp - mean_k(dEt_kp): the gradient and C
    int nblk = 0;   // blocks (p, q0), p-major
    for (int pp = 0; pp < nth; ++pp) nblk += pp / 4 + 1;
    const int nu = t < nblk ? (nblk - t + VMC_GN_THREADS - 1) / VMC_GN_THREADS : 0;
    double cacc[GN_BLK][4];
    int cp[GN_BLK], cq[GN_BLK];   // row p and first column q0 of this thread's blocks
  #pragma unroll
    for (int u = 0; u < GN_BLK; ++u) {
      const int x = t + u * VMC_GN_THREADS;
      int pp = 0, first = 0;
      while (pp < nth && first + pp / 4 + 1 <= x) first += pp++ / 4 + 1;
      cp[u] = x < nblk ? pp : 0;
      cq[u] = x < nblk ? 4 * (x - first) : 0;
      cacc[u][0] = cacc[u][1] = cacc[u][2] = cacc[u][3] = 0.0;
    }
    a1 = 0.0;
    for (long k0 = 0; k0 < N; k0 += tk) {
      const int nk = tile_len(k0);
      stage(k0, nk);
      for (int e = t; e < nk * nth; e += VMC_GN_THREADS) {   // centred clipped derivatives
        const int kk = e / nth, p = e - kk * nth;
        const double ev = te[kk];
        const double v = ev < lo ? sh.dm[p] - 5.0 * sh.dmad[p]
                                 : (ev > hi ? sh.dm[p] + 5.0 * sh.dmad[p] : tile[e]);
        tile[e] = v - sh.mdt[p];
      }
      __syncthreads();
      if (cseg < S)
        for (int kk = cseg; kk < nk; kk += S) {
          const double e0 = te[kk];
          a1 += tile[kk * nth + ccol] * ((e0 < lo ? lo : (e0 > hi ? hi : e0)) - mean);
        }
      if (nu > 0)
        for (int kk = 0; kk < nk; ++kk) {
          const double* row = tile + kk * nth;
  #pragma unroll
          for (int u = 0; u < GN_BLK; ++u)   // the first test is block-uniform
            if (u * VMC_GN_THREADS < nblk && u < nu) {
              const double a = row[cp[u]];
  #pragma unroll
              for (int jq = 0; jq < 4; ++jq) {   // columns past the row's end are clamped, then dropped
                const int q = cq[u] + jq < nth ? cq[u] + jq : nth - 1;
                cacc[u][jq] += a * row[q];
              }
            }
        }
    }
    a1 = combine(a1);
    if (t < nth) sh.grad[t] = 2.0 * a1 / (double)(N - 1);
    __syncthreads();   // the tile space becomes C
  #pragma unroll
    for (int u = 0; u < GN_BLK; ++u)
      if (t + u * VMC_GN_THREADS < nblk) {
  #pragma unroll
        for (int jq = 0; jq < 4; ++jq) {
          const int pp = cp[u], qq = cq[u] + jq;
          if (qq > pp) continue;   // q <= p < nth
          const double c = cacc[u][jq] * inv_n + (pp == qq ? lam : 0.0);
          sh.C[pp * nth + qq] = c;
          sh.C[qq * nth + pp] = c;
        }
      }
  }
  __syncthreads();
  if (t == 0) {
    // Cholesky C = L L^T in place (lower), then L y = grad, L^T x = y, delta = -eta x
    double info = 0.0;
    for (int j = 0; j < nth && info == 0.0; ++j) {
      double s = sh.C[j * nth + j];
      for (int k = 0; k < j; ++k) s -= sh.C[j * nth + k] * sh.C[j * nth + k];
      if (!(s > 0.0)) {
        info = j + 1;
        break;
      }
      const double ljj = sqrt(s);
      sh.C[j * nth + j] = ljj;
      for (int i = j + 1; i < nth; ++i) {
        double v = sh.C[i * nth + j];
        for (int k = 0; k < j; ++k) v -= sh.C[i * nth + k] * sh.C[j * nth + k];
        sh.C[i * nth + j] = v / ljj;
      }
    }
    if (info == 0.0) {
      for (int i = 0; i < nth; ++i) {
        double v = sh.grad[i];
        for (int k = 0; k < i; ++k) v -= sh.C[i * nth + k] * sh.x[k];
        sh.x[i] = v / sh.C[i * nth + i];
      }
      for (int i = nth - 1; i >= 0; --i) {
        double v = sh.x[i];
        for (int k = i + 1; k < nth; ++k) v -= sh.C[k * nth + i] * sh.x[k];
        sh.x[i] = v / sh.C[i * nth + i];
      }
      for (int i = 0; i < nth; ++i) delta[i] = -eta * sh.x[i];
    } else {
      for (int i = 0; i < nth; ++i) delta[i] = __builtin_nan("");
    }
    stats[0] = m;
    stats[1] = mad;
    stats[2] = mean;
    stats[3] = var;
    stats[4] = nclip;
    stats[5] = info;
  }
}

// ---------------------------------------------------------------------------------------
// C'[k][a] = comp[a] C[a][k] (stored orbital-major)
__global__ __launch_bounds__(256) void k_vmc_scale_c(const double* __restrict__ C,
                                                     const double* __restrict__ comp, long n_ao,
                                                     int n_occ, double* __restrict__ Cs) {
  const long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n_ao * n_occ) return;
  const long a = i / n_occ, k = i - a * n_occ;
  Cs[k * n_ao + a] = comp[a] * C[i];   // orbital-major
}

struct VmcLayout {
  double* cen; int* shi; double* prim; double* comp; double* nuc; double* Cs;
  double* bh;    // BH correlator: nuclei [24][4], b [2], c [2][64]
  int* bh_mno;   // [64][3]
};

static VmcLayout layout_vmc(Arena& ar, int n_shell, int n_prim, int n_ao, int n_occ, int n_nuc) {
  VmcLayout L;
  L.cen = ar.take<double>(4 * (size_t)n_shell);
  L.shi = ar.take<int>(2 * (size_t)n_shell);
  L.prim = ar.take<double>(2 * (size_t)n_prim);
  L.comp = ar.take<double>(n_ao);
  L.nuc = ar.take<double>(4 * (size_t)(n_nuc > 0 ? n_nuc : 1));
  L.Cs = ar.take<double>((size_t)n_ao * n_occ);
  L.bh = ar.take<double>(4 * VMC_BH_MAXNUC + VMC_BH_MAXTYPE + VMC_BH_MAXTYPE * VMC_BH_MAXTERM +
                         VMC_BH_MAXTYPE * 16 * VMC_BH_NO);
  L.bh_mno = ar.take<int>(3 * VMC_BH_MAXTERM + VMC_BH_MAXTYPE * 16 + VMC_BH_MAXTYPE * 11 +
                          VMC_BH_MAXTYPE * VMC_BH_MAXTERM);
  return L;
}

size_t ws_vmc(int n_ao) {
  Arena ar(nullptr, 0);
  const int na = n_ao > 0 ? n_ao : 1;
  layout_vmc(ar, 4096, 16384, na, VMC_MAX_OCC, 4096);
  return ar.used;
}

static size_t lds_tables(const VmcBasis& b) {
  return sizeof(double) * (4 * (size_t)b.n_cent + 2 * (size_t)b.n_prim) +
         sizeof(int) * 2 * (size_t)b.n_shell;
}

static size_t lds_sweeps(const VmcBasis& b, int n) {
  const int n_el = 2 * n;
  const size_t shared = 2 * (size_t)n * n > 11 * (size_t)n ? 2 * (size_t)n * n : 11 * (size_t)n;
  return lds_tables(b) + sizeof(double) * (2 * (size_t)n * n + shared + b.n_ao + 64 + 3 * n_el) +
         sizeof(int) * n + 16;
}

static size_t lds_energy_bh(const VmcBasis& b, int n, int n_nuc) {
  const int n_el = 2 * n;
  const size_t keep = sizeof(double) * (5 * (size_t)n_el * n + 2 * (size_t)n * n + n +
                                        3 * n_el + 64 + 4 * n_el + 4 * (size_t)n_nuc +
                                        VMC_BH_MAXTYPE * VMC_BH_MAXTERM + 64 * 8);
  const size_t slater = lds_tables(b) + sizeof(double) * (2 * (size_t)n * n + 5 * (size_t)b.n_ao +
                                                          5 * 64) + sizeof(int) * n;
  const size_t table = sizeof(double) * (size_t)n_el * n_nuc * VMC_BH_TA;
  return keep + (slater > table ? slater : table) + 16;
}

static size_t lds_energy(const VmcBasis& b, int n) {
  const int n_el = 2 * n;
  return lds_tables(b) + sizeof(double) * (5 * (size_t)n_el * n + 4 * (size_t)n * n +
                                           5 * (size_t)b.n_ao + 5 * 64 + n + 3 * n_el + 64) + 16;
}

constexpr size_t VMC_LDS_MAX = 160 * 1024;

// Validates the system, uploads its tables and folds the component factors into the
// orbital coefficients; the stream is synchronised before return (host staging ends).
static xtc_status vmc_upload(const xtc_vmc_system* sy, Arena& ar, hipStream_t st, VmcDev* out,
                             VmcLayout* lay = nullptr) {
  const xtc_basis* basis = sy->basis;
  XTC_REQUIRE(basis && sy->C_occ, "vmc: null basis or orbital coefficients");
  XTC_REQUIRE(sy->n_occ >= 1 && sy->n_occ <= VMC_MAX_OCC, "vmc: n_occ must be in 1..32");
  XTC_REQUIRE(basis->n_shell > 0 && basis->n_atom > 0 && basis->n_atom <= 4096 &&
                  basis->n_shell <= 4096,
              "vmc: bad basis sizes");
  XTC_REQUIRE(basis->atom_xyz && basis->shell_center && basis->shell_l &&
                  basis->shell_prim_start && basis->prim_exp && basis->prim_coef &&
                  basis->comp_factor,
              "vmc: null basis table");
  XTC_REQUIRE(sy->n_nuc >= 0 && sy->n_nuc <= 4096 && (sy->n_nuc == 0 || (sy->nuc_xyz && sy->nuc_charge)),
              "vmc: bad nuclei");
  const int ns = basis->n_shell;
  // distinct shell centres in order of first use (at most one per shell)
  std::vector<double> cen;
  std::vector<int> cid((size_t)basis->n_atom, -1);
  std::vector<int> shi(2 * (size_t)ns);
  int n_ao = 0, n_cent = 0;
  for (int s = 0; s < ns; ++s) {
    const int l = basis->shell_l[s];
    const int c = basis->shell_center[s];
    XTC_REQUIRE(l >= 0 && l <= VMC_MAX_L, "vmc: angular momentum out of range");
    XTC_REQUIRE(c >= 0 && c < basis->n_atom, "vmc: shell centre out of range");
    XTC_REQUIRE(basis->shell_prim_start[s + 1] > basis->shell_prim_start[s],
                "vmc: shell without primitives");
    if (cid[c] < 0) {
      cid[c] = n_cent++;
      for (int q = 0; q < 3; ++q) cen.push_back(basis->atom_xyz[3 * c + q]);
      cen.push_back(0.0);
    }
    // two words per shell: l (3 bits) | centre (12) | primitive count (15), and
    // first primitive (15) | first AO (17)
    const unsigned np = (unsigned)(basis->shell_prim_start[s + 1] - basis->shell_prim_start[s]);
    XTC_REQUIRE(basis->shell_prim_start[s] < 32768 && np < 32768 && n_ao < 131072,
                "vmc: basis too large for the packed shell records");
    shi[2 * s] = (int)((unsigned)l | ((unsigned)cid[c] << 3) | (np << 15));
    shi[2 * s + 1] = (int)((unsigned)basis->shell_prim_start[s] | ((unsigned)n_ao << 15));
    n_ao += (l + 1) * (l + 2) / 2;
  }
  const int n_prim = basis->shell_prim_start[ns];
  XTC_REQUIRE(basis->shell_prim_start[0] == 0 && n_prim <= 16384, "vmc: bad primitive table");
  XTC_REQUIRE(n_ao == basis->n_ao, "vmc: n_ao does not match the shells");
  VmcLayout L = layout_vmc(ar, ns, n_prim, n_ao, sy->n_occ, sy->n_nuc);
  XTC_TRY(need_ws(ar));
  std::vector<double> prim(2 * (size_t)n_prim);
  for (int p = 0; p < n_prim; ++p) {
    prim[2 * p] = basis->prim_exp[p];
    prim[2 * p + 1] = basis->prim_coef[p];
  }
  std::vector<double> nuc(4 * (size_t)(sy->n_nuc > 0 ? sy->n_nuc : 1), 0.0);
  for (int I = 0; I < sy->n_nuc; ++I) {
    for (int c = 0; c < 3; ++c) nuc[4 * I + c] = sy->nuc_xyz[3 * I + c];
    nuc[4 * I + 3] = sy->nuc_charge[I];
  }
  XTC_HIP(hipMemcpyAsync(L.cen, cen.data(), sizeof(double) * cen.size(), hipMemcpyHostToDevice, st));
  XTC_HIP(hipMemcpyAsync(L.shi, shi.data(), sizeof(int) * shi.size(), hipMemcpyHostToDevice, st));
  XTC_HIP(hipMemcpyAsync(L.prim, prim.data(), sizeof(double) * prim.size(), hipMemcpyHostToDevice, st));
  XTC_HIP(hipMemcpyAsync(L.comp, basis->comp_factor, sizeof(double) * n_ao, hipMemcpyHostToDevice, st));
  XTC_HIP(hipMemcpyAsync(L.nuc, nuc.data(), sizeof(double) * nuc.size(), hipMemcpyHostToDevice, st));
  const long nc = (long)n_ao * sy->n_occ;
  hipLaunchKernelGGL(k_vmc_scale_c, dim3(cdiv(nc, 256)), dim3(256), 0, st, sy->C_occ,
                     (const double*)L.comp, (long)n_ao, sy->n_occ, L.Cs);
  XTC_CHECK_LAUNCH();
  XTC_HIP(hipStreamSynchronize(st));   // host staging vectors end with this call
  VmcDev v;
  v.b = VmcBasis{L.cen, L.shi, L.prim, ns, n_prim, n_ao, n_cent};
  v.C = L.Cs;
  v.nuc = L.nuc;
  v.n_occ = sy->n_occ;
  v.n_nuc = sy->n_nuc;
  v.e_nuc = sy->e_nuc;
  *out = v;
  if (lay) *lay = L;
  return XTC_OK;
}

// The BH local energy: validates the correlator, uploads its table and launches
// k_vmc_energy_bh. dE: [n_walkers][n_types n_terms + 1 + n_types] or NULL.
static xtc_status vmc_local_energy_bh(const xtc_vmc_system* sys, const xtc_correlator* corr,
                                      int64_t n_walkers, const double* R, double* E, double* dE,
                                      void* ws, size_t ws_bytes, void* stream) {
  XTC_REQUIRE(corr->n_nuc >= 1 && corr->n_nuc <= VMC_BH_MAXNUC && corr->nuc_xyz && corr->nuc_type,
              "xtc_vmc_local_energy: BH needs 1..24 nuclei");
  XTC_REQUIRE(corr->n_types >= 1 && corr->n_types <= VMC_BH_MAXTYPE && corr->b && corr->c,
              "xtc_vmc_local_energy: BH needs 1..2 nucleus types");
  XTC_REQUIRE(corr->n_terms >= 1 && corr->n_terms <= VMC_BH_MAXTERM && corr->mno,
              "xtc_vmc_local_energy: BH needs 1..64 terms");
  XTC_REQUIRE(corr->d > 0.0 && std::isfinite(corr->d), "xtc_vmc_local_energy: d must be > 0");
  for (int t = 0; t < corr->n_types; ++t)
    XTC_REQUIRE(corr->b[t] > 0.0 && std::isfinite(corr->b[t]), "xtc_vmc_local_energy: b must be > 0");
  for (int k = 0; k < corr->n_terms; ++k) {
    const int m = corr->mno[3 * k], n = corr->mno[3 * k + 1], o = corr->mno[3 * k + 2];
    XTC_REQUIRE(m >= 0 && m <= 3 && n >= 0 && n <= 3 && o >= 0 && o <= VMC_BH_MAXO,
                "xtc_vmc_local_energy: BH terms need 0 <= m, n <= 3 and 0 <= o <= 12");
  }
  for (int I = 0; I < corr->n_nuc; ++I)
    XTC_REQUIRE(corr->nuc_type[I] >= 0 && corr->nuc_type[I] < corr->n_types,
                "xtc_vmc_local_energy: nucleus type out of range");
  const int nparam = corr->n_types * corr->n_terms + 1 + corr->n_types;
  XTC_REQUIRE(nparam <= VMC_MAX_THETA, "xtc_vmc_local_energy: more than 128 parameters");
  hipStream_t st = as_stream(stream);
  Arena ar(ws, ws_bytes);
  VmcDev v;
  VmcLayout L;
  XTC_TRY(vmc_upload(sys, ar, st, &v, &L));
  const size_t lds = lds_energy_bh(v.b, v.n_occ, corr->n_nuc);
  XTC_REQUIRE(lds <= VMC_LDS_MAX, "xtc_vmc_local_energy: system too large for the walker's LDS");
  std::vector<double> tab(4 * VMC_BH_MAXNUC + VMC_BH_MAXTYPE + VMC_BH_MAXTYPE * VMC_BH_MAXTERM +
                              VMC_BH_MAXTYPE * 16 * VMC_BH_NO, 0.0);
  std::vector<int> itab(3 * VMC_BH_MAXTERM + VMC_BH_MAXTYPE * 16 + VMC_BH_MAXTYPE * 11 +
                            VMC_BH_MAXTYPE * VMC_BH_MAXTERM, 0);
  for (int I = 0; I < corr->n_nuc; ++I) {
    for (int c = 0; c < 3; ++c) tab[4 * I + c] = corr->nuc_xyz[3 * I + c];
    tab[4 * I + 3] = corr->nuc_type[I];
  }
  double* bt = tab.data() + 4 * VMC_BH_MAXNUC;
  double* cc = bt + VMC_BH_MAXTYPE;
  double* cs = cc + VMC_BH_MAXTYPE * VMC_BH_MAXTERM;
  int* on = itab.data() + 3 * VMC_BH_MAXTERM;
  int* gst = on + VMC_BH_MAXTYPE * 16;
  int* gtm = gst + VMC_BH_MAXTYPE * 11;
  for (int k = 0; k < 3 * corr->n_terms; ++k) itab[k] = corr->mno[k];
  for (int t = 0; t < corr->n_types; ++t) {
    bt[t] = corr->b[t];
    for (int k = 0; k < corr->n_terms; ++k) {
      const double c = corr->c[t * corr->n_terms + k];
      cc[t * corr->n_terms + k] = c;
      const int m = corr->mno[3 * k], n = corr->mno[3 * k + 1], o = corr->mno[3 * k + 2];
      const int lo = m < n ? m : n, hi = m < n ? n : m;
      cs[((t * 4 + lo) * 4 + hi) * VMC_BH_NO + o] += c;
      int& top = on[(t * 4 + lo) * 4 + hi];
      if (o + 1 > top) top = o + 1;
    }
    // the terms of each (m <= n) group, groups in the kernel's order (0,0), (0,1), ..., (3,3)
    int x = 0;
    for (int lo = 0, g = 0; lo < 4; ++lo)
      for (int hi = lo; hi < 4; ++hi, ++g) {
        gst[t * 11 + g] = x;
        for (int k = 0; k < corr->n_terms; ++k) {
          const int m = corr->mno[3 * k], n = corr->mno[3 * k + 1], o = corr->mno[3 * k + 2];
          if ((m < n ? m : n) == lo && (m < n ? n : m) == hi) gtm[t * VMC_BH_MAXTERM + x++] = k | (o << 8);
        }
      }
    gst[t * 11 + 10] = x;
  }
  XTC_HIP(hipMemcpyAsync(L.bh, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice, st));
  XTC_HIP(hipMemcpyAsync(L.bh_mno, itab.data(), sizeof(int) * itab.size(), hipMemcpyHostToDevice, st));
  XTC_HIP(hipStreamSynchronize(st));   // host staging vector ends with this call
  if (n_walkers == 0) return XTC_OK;
  const double* cdev = L.bh + 4 * VMC_BH_MAXNUC + VMC_BH_MAXTYPE;
  const int* on_dev = L.bh_mno + 3 * VMC_BH_MAXTERM;
  VmcBH bh{L.bh, L.bh + 4 * VMC_BH_MAXNUC, cdev, L.bh_mno, cdev + VMC_BH_MAXTYPE * VMC_BH_MAXTERM,
           on_dev, on_dev + VMC_BH_MAXTYPE * 16, on_dev + VMC_BH_MAXTYPE * 16 + VMC_BH_MAXTYPE * 11,
           corr->n_nuc, corr->n_types, corr->n_terms, corr->d};
  size_t tk = timing_begin(TM_VMC_ENERGY, st);
  hipLaunchKernelGGL(k_vmc_energy_bh, dim3((unsigned)n_walkers), dim3(64), lds, st, v, bh, R,
                     (long)n_walkers, E, dE);
  XTC_CHECK_LAUNCH();
  timing_end(tk, st);
  return XTC_OK;
}

}  // namespace xtc

using namespace xtc;

extern "C" xtc_status xtc_vmc_sample(const xtc_vmc_system* sys, int64_t n_walkers, double* R,
                                     int32_t n_sweeps, double step, const double* normals,
                                     const double* uniforms, int64_t* accepted, void* ws,
                                     size_t ws_bytes, void* stream) {
  XTC_REQUIRE(sys && (n_walkers == 0 || (R && accepted)), "xtc_vmc_sample: null argument");
  XTC_REQUIRE(n_walkers >= 0 && n_walkers <= (int64_t)1 << 31, "xtc_vmc_sample: bad n_walkers");
  XTC_REQUIRE(n_sweeps >= 0, "xtc_vmc_sample: n_sweeps < 0");
  XTC_REQUIRE(n_sweeps == 0 || (normals && uniforms), "xtc_vmc_sample: null draws");
  XTC_REQUIRE(std::isfinite(step), "xtc_vmc_sample: step not finite");
  hipStream_t st = as_stream(stream);
  Arena ar(ws, ws_bytes);
  VmcDev v;
  XTC_TRY(vmc_upload(sys, ar, st, &v));
  const size_t lds = lds_sweeps(v.b, v.n_occ);
  XTC_REQUIRE(lds <= VMC_LDS_MAX, "xtc_vmc_sample: basis too large for the walker's LDS");
  if (n_walkers == 0) return XTC_OK;
  size_t tk = timing_begin(TM_VMC_SAMPLE, st);
  hipLaunchKernelGGL(k_vmc_sweeps, dim3((unsigned)n_walkers), dim3(64), lds, st, v, R,
                     (long)n_walkers, n_sweeps, step, normals, uniforms, (long long*)accepted);
  XTC_CHECK_LAUNCH();
  timing_end(tk, st);
  return XTC_OK;
}

extern "C" xtc_status xtc_vmc_local_energy(const xtc_vmc_system* sys, const xtc_correlator* corr,
                                           int64_t n_walkers, const double* R, double* E,
                                           double* dE, void* ws, size_t ws_bytes, void* stream) {
  XTC_REQUIRE(sys && corr && (n_walkers == 0 || (R && E)), "xtc_vmc_local_energy: null argument");
  XTC_REQUIRE(n_walkers >= 0 && n_walkers <= (int64_t)1 << 31, "xtc_vmc_local_energy: bad n_walkers");
  if (corr->form == XTC_U_BH) return vmc_local_energy_bh(sys, corr, n_walkers, R, E, dE, ws, ws_bytes,
                                                          stream);
  XTC_REQUIRE(corr->form == XTC_U_EE, "xtc_vmc_local_energy: unknown correlator form");
  XTC_REQUIRE(corr->n_terms >= 1 && corr->n_terms <= VMC_MAX_TERMS && corr->mno && corr->c,
              "xtc_vmc_local_energy: EE correlator needs 1..12 terms");
  XTC_REQUIRE(corr->d > 0.0 && std::isfinite(corr->d), "xtc_vmc_local_energy: d must be > 0");
  EECoefV cf;
  cf.n = corr->n_terms;
  cf.d = corr->d;
  for (int k = 0; k < VMC_MAX_TERMS; ++k) {
    cf.o[k] = k < cf.n ? corr->mno[3 * k + 2] : 0;
    cf.c[k] = k < cf.n ? corr->c[k] : 0.0;
    XTC_REQUIRE(k >= cf.n || (corr->mno[3 * k] == 0 && corr->mno[3 * k + 1] == 0 &&
                              cf.o[k] >= 0 && cf.o[k] <= 64),
                "xtc_vmc_local_energy: EE terms are (0, 0, o) with 0 <= o <= 64");
  }
  hipStream_t st = as_stream(stream);
  Arena ar(ws, ws_bytes);
  VmcDev v;
  XTC_TRY(vmc_upload(sys, ar, st, &v));
  const size_t lds = lds_energy(v.b, v.n_occ);
  XTC_REQUIRE(lds <= VMC_LDS_MAX, "xtc_vmc_local_energy: basis too large for the walker's LDS");
  if (n_walkers == 0) return XTC_OK;
  size_t tk = timing_begin(TM_VMC_ENERGY, st);
  hipLaunchKernelGGL(k_vmc_energy, dim3((unsigned)n_walkers), dim3(64), lds, st, v, cf, R,
                     (long)n_walkers, E, dE);
  XTC_CHECK_LAUNCH();
  timing_end(tk, st);
  return XTC_OK;
}

extern "C" xtc_status xtc_vmc_gn_step(int64_t n_walkers, int32_t n_params, const double* E,
                                      const double* dE, double lambda, double eta, double* delta,
                                      double* stats, void* stream) {
  XTC_REQUIRE(E && dE && delta && stats, "xtc_vmc_gn_step: null argument");
  XTC_REQUIRE(n_walkers >= 2, "xtc_vmc_gn_step: need at least two walkers");
  XTC_REQUIRE(n_params >= 1 && n_params <= VMC_MAX_THETA, "xtc_vmc_gn_step: n_params must be in 1..128");
  XTC_REQUIRE(lambda >= 0.0 && std::isfinite(lambda) && std::isfinite(eta),
              "xtc_vmc_gn_step: lambda must be >= 0 and finite, eta finite");
  hipStream_t st = as_stream(stream);
  size_t tk = timing_begin(TM_VMC_GN, st);
  hipLaunchKernelGGL(k_vmc_gn, dim3(1), dim3(VMC_GN_THREADS), 0, st, E, dE, (long)n_walkers,
                     n_params, lambda, eta, delta, stats);
  XTC_CHECK_LAUNCH();
  timing_end(tk, st);
  return XTC_OK;
}
