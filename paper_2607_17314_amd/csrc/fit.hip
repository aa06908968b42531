// ISDF fit of the auxiliary vectors (ISDF section, eq. isdf-rho and its normal
// equations; auxiliary-fit robustness). Per system (scalar, then x, y, z):
//   Gram      A = (Phi_mu^T Phi_mu) o (Phi_mu^T Phi_mu) or (dPhi_mu^T dPhi_mu)_c o G, FP64 MFMA GEMMs
//   Cholesky  blocked right-looking FP64 factorisation (64-wide panels); the
//             diagonal block is factored and inverted in LDS by one workgroup,
//             panel and trailing updates are GEMMs; on a non-positive pivot the
//             adaptive Tikhonov retry re-factors A + shift_k I
//   RHS       per grid chunk: P = Phi_mu^T Phi, B = P o P or (dPhi_mu^T dPhi)_c o P
//   solves    blocked forward and backward substitution as GEMMs with the
//             inverted diagonal blocks; the weighted residual
//             sum_g w^2 (|m_g|^2 - |L^{-1} B(g)|^2) falls out of the forward solve.
// The fit is column-separable in g, so the grid is processed in chunks and the
// workspace does not grow with n_g beyond one chunk.
#include "common.hpp"
#include "fit.hpp"
#include "plans.hpp"
#include "timing.hpp"

namespace xtc {

constexpr int NB = 64;
constexpr long FIT_CHUNK = 65536;

__global__ void k_gather_piv(const double* __restrict__ phi4, long n_g, int rows,
                             const long* __restrict__ piv, int n_mu, double* __restrict__ out) {
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  long total = (long)rows * n_mu;
  if (t >= total) return;
  int r = (int)(t / n_mu), m = (int)(t % n_mu);
  out[t] = phi4[(long)r * n_g + piv[m]];
}

// Factor the NB x NB diagonal block at (j0, j0) of the n x n matrix a (row-major,
// lower triangle used) in LDS, write L_jj back (upper part zeroed) and its
// inverse to linv [NB][NB]; a non-positive or non-finite pivot sets *fail.
// One workgroup of 256 threads as 16 x 16. The factorisation runs column by column
// (right-looking, the trailing update spread over the 16 x 16 threads); the inverse
// goes by 16 x 16 blocks: the four diagonal blocks first (one column per thread),
// then the blocks below the diagonal by block diagonals,
//   X_IJ = -inv(L_II) sum_{J <= K < I} L_IK X_KJ,
// so that its longest dependent chain is ~300 products instead of ~NB^2 / 2.
constexpr int PB = 16;   // inverse block

__global__ __launch_bounds__(256) void k_potrf_diag(double* __restrict__ a, long n, long j0,
                                                    int nb, double* __restrict__ linv,
                                                    int* __restrict__ fail) {
  static_assert(NB == 4 * PB, "the inverse works on 4 x 4 blocks of 16");
  __shared__ double s[NB][NB + 1];
  __shared__ double sinv[NB][NB + 1];
  __shared__ double tmp[NB][NB + 1];
  __shared__ double rdiag[NB];
  __shared__ int bad;
  const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
  if (t == 0) bad = 0;
  for (int e = t; e < NB * NB; e += 256) {
    const int i = e / NB, k = e % NB;
    s[i][k] = (i < nb && k < nb && k <= i) ? a[(j0 + i) * n + j0 + k] : 0.0;
    sinv[i][k] = 0.0;
  }
  // padding rows and columns past nb: unit diagonal, so the blocked inverse stays regular
  if (t < NB && t >= nb) s[t][t] = 1.0;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (t == 0) {
      double v = s[j][j];
      if (!(v > 0.0) || !isfinite(v)) {
        bad = 1;
        v = 1.0;
      }
      const double d = sqrt(v);
      s[j][j] = d;
      rdiag[j] = 1.0 / d;
    }
    __syncthreads();
    const double rj = rdiag[j];
    for (int i = j + 1 + t; i < nb; i += 256) s[i][j] *= rj;
    __syncthreads();
    // trailing update of (i, k), j < k <= i < nb
    for (int i = j + 1 + ty; i < nb; i += 16) {
      const double sij = s[i][j];
      for (int k = j + 1 + tx; k <= i; k += 16) s[i][k] -= sij * s[k][j];
    }
    __syncthreads();
  }
  for (int i = t; i < NB; i += 256)
    if (i >= nb) rdiag[i] = 1.0;
  __syncthreads();
  // diagonal blocks: thread (block b = ty / 4 .. , column) -- 64 threads, one column each
  if (t < NB) {
    const int b = t / PB, c = t;
    const int r0 = b * PB;
    for (int i = c; i < r0 + PB; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) v -= s[i][k] * sinv[k][c];
      sinv[i][c] = v * rdiag[i];
    }
  }
  __syncthreads();
  // block diagonals d = 1, 2, 3: T_IJ = sum_{J <= K < I} L_IK X_KJ, then X_IJ = -inv(L_II) T_IJ
  for (int d = 1; d < 4; ++d) {
    for (int J = 0; J + d < 4; ++J) {
      const int I = J + d;
      const int r = I * PB + ty, c = J * PB + tx;
      double v = 0.0;
      for (int k = J * PB; k < I * PB; ++k) v += s[r][k] * sinv[k][c];
      tmp[r][c] = v;
    }
    __syncthreads();
    for (int J = 0; J + d < 4; ++J) {
      const int I = J + d;
      const int r = I * PB + ty, c = J * PB + tx;
      double v = 0.0;
      for (int k = I * PB; k <= r; ++k) v += sinv[r][k] * tmp[k][c];
      sinv[r][c] = -v;
    }
    __syncthreads();
  }
  for (int e = t; e < NB * NB; e += 256) {
    const int i = e / NB, k = e % NB;
    linv[e] = (i < nb && k < nb) ? sinv[i][k] : 0.0;
    if (i < nb && k < nb) a[(j0 + i) * n + j0 + k] = (k <= i) ? s[i][k] : 0.0;
  }
  if (t == 0 && bad) *fail = 1;
}

__global__ void k_diag_extract(const double* __restrict__ a, long n, double* __restrict__ dg) {
  long i = (long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dg[i] = a[i * n + i];
}

__global__ void k_restore_shift(const double* __restrict__ src, double* __restrict__ dst, long n,
                                double shift) {
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= n * n) return;
  long i = t / n, k = t % n;
  dst[t] = src[t] + ((i == k) ? shift : 0.0);
}

__global__ void k_square(double* __restrict__ x, long n) {
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t < n) x[t] = x[t] * x[t];
}

__global__ void k_copy_rows(const double* __restrict__ src, long lds, double* __restrict__ dst,
                            long ldd, int rows, long cols) {
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= (long)rows * cols) return;
  long r = t / cols, c = t % cols;
  dst[r * ldd + c] = src[r * lds + c];
}

// per grid point of a chunk: w^2 (|m_g|^2 - |y_g|^2) and w^2 |m_g|^2, channel c (-1 scalar)
__global__ void k_resid(const double* __restrict__ phi4, const double* __restrict__ w, long n_g,
                        int n_orb, int comp, long g0, long cn, const double* __restrict__ y,
                        long ldy, int n_mu, double* __restrict__ r_out,
                        double* __restrict__ m_out) {
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= cn) return;
  long g = g0 + t;
  double n2 = 0.0;
  for (int p = 0; p < n_orb; ++p) {
    double v = phi4[(long)p * n_g + g];
    n2 += v * v;
  }
  double m2;
  if (comp < 0) {
    m2 = n2 * n2;
  } else {
    double g2 = 0.0;
    for (int p = 0; p < n_orb; ++p) {
      double v = phi4[(long)((1 + comp) * n_orb + p) * n_g + g];
      g2 += v * v;
    }
    m2 = n2 * g2;
  }
  double yy = 0.0;
  for (int m = 0; m < n_mu; ++m) {
    double v = y[(long)m * ldy + t];
    yy += v * v;
  }
  double ww = w[g] * w[g];
  r_out[t] = ww * (m2 - yy);
  m_out[t] = ww * m2;
}

// Chunks of grid columns are independent in the right-hand sides and the solves, so
// isdf_fit runs them in up to FIT_LANES lanes (the caller's stream and auxiliary ones),
// each with its own scratch: P, R, rtmp, mtmp and red below are lane 0's, Px[l], ... lane l's.
constexpr int FIT_LANES = 1 + AUX_STREAMS;

struct FitLayout {
  long* piv; double* phimu; double* G; double* A; double* Asave; double* linv; double* P;
  double* R; double* rtmp; double* mtmp; double* red; double* sums; int* fail; double* dg;
  double* Px[FIT_LANES]; double* Rx[FIT_LANES]; double* rtx[FIT_LANES]; double* mtx[FIT_LANES];
  double* redx[FIT_LANES];
  long chunk; int nblk; int nchunks; int lanes;
};

static FitLayout layout_fit(Arena& ar, int64_t n_g, int n_orb, int n_mu, bool lanes = false) {
  FitLayout F;
  F.chunk = n_g < FIT_CHUNK ? n_g : FIT_CHUNK;
  F.nblk = (int)cdiv(n_mu, NB);
  F.nchunks = (int)cdiv(n_g, F.chunk);
  F.lanes = lanes ? (F.nchunks < FIT_LANES ? F.nchunks : FIT_LANES) : 1;
  F.piv = ar.take<long>(n_mu);
  F.phimu = ar.take<double>(4 * (size_t)n_orb * n_mu);
  F.G = ar.take<double>((size_t)n_mu * n_mu);
  F.A = ar.take<double>((size_t)n_mu * n_mu);
  F.Asave = ar.take<double>((size_t)n_mu * n_mu);
  F.linv = ar.take<double>((size_t)F.nblk * NB * NB);
  F.P = ar.take<double>((size_t)n_mu * F.chunk);
  F.R = ar.take<double>((size_t)n_mu * F.chunk);
  F.rtmp = ar.take<double>(F.chunk);
  F.mtmp = ar.take<double>(F.chunk);
  F.red = ar.take<double>(1024);
  F.sums = ar.take<double>(2 * (size_t)F.nchunks + 2);
  F.fail = ar.take<int>(1);
  F.dg = ar.take<double>(n_mu);
  F.Px[0] = F.P; F.Rx[0] = F.R; F.rtx[0] = F.rtmp; F.mtx[0] = F.mtmp; F.redx[0] = F.red;
  for (int l = 1; l < F.lanes; ++l) {
    F.Px[l] = ar.take<double>((size_t)n_mu * F.chunk);
    F.Rx[l] = ar.take<double>((size_t)n_mu * F.chunk);
    F.rtx[l] = ar.take<double>(F.chunk);
    F.mtx[l] = ar.take<double>(F.chunk);
    F.redx[l] = ar.take<double>(1024);
  }
  return F;
}

size_t ws_fit(int64_t n_g, int n_orb, int n_mu, uint32_t what) {
  (void)what;
  Arena ar(nullptr, 0);
  layout_fit(ar, n_g, n_orb, n_mu, true);
  ar.take<double>(n_mu);   // rho at the pivots, when rhot is asked for
  return ar.used;
}

// Blocked Cholesky of F.A (n x n) in place; returns 0 on success, 1 on failure.
static xtc_status cholesky(FitLayout& F, long n, hipStream_t st, int* failed) {
  XTC_HIP(hipMemsetAsync(F.fail, 0, sizeof(int), st));
  for (int b = 0; b < F.nblk; ++b) {
    long j0 = (long)b * NB;
    int nb = (int)((n - j0) < NB ? (n - j0) : NB);
    hipLaunchKernelGGL(k_potrf_diag, dim3(1), dim3(256), 0, st, F.A, n, j0, nb,
                       F.linv + (long)b * NB * NB, F.fail);
    XTC_CHECK_LAUNCH();
    long rest = n - j0 - nb;
    if (rest <= 0) continue;
    GemmArgs p{};   // L21 = A21 Linv_jj^T (in place)
    p.M = rest; p.N = nb; p.K = nb;
    p.A = F.A + (j0 + nb) * n + j0; p.a_sm = n; p.a_sk = 1;
    p.B = F.linv + (long)b * NB * NB; p.b_sk = 1; p.b_sn = NB;
    p.C = F.A + (j0 + nb) * n + j0; p.c_sm = n; p.c_sn = 1;
    XTC_TRY(gemm_f64(p, st));
    GemmArgs u{};   // A22 -= L21 L21^T (lower tiles)
    u.M = rest; u.N = rest; u.K = nb;
    u.A = F.A + (j0 + nb) * n + j0; u.a_sm = n; u.a_sk = 1;
    u.B = F.A + (j0 + nb) * n + j0; u.b_sk = 1; u.b_sn = n;
    u.C = F.A + (j0 + nb) * n + j0 + nb; u.c_sm = n; u.c_sn = 1;
    u.alpha = -1.0; u.beta = 1.0; u.lower_only = true;
    XTC_TRY(gemm_f64(u, st));
  }
  int h = 0;
  XTC_HIP(hipMemcpyAsync(&h, F.fail, sizeof(int), hipMemcpyDeviceToHost, st));
  XTC_HIP(hipStreamSynchronize(st));
  *failed = h;
  return XTC_OK;
}

// A lower Cholesky factor L (row-major n x n, lower triangle used) with the inverses of
// its NB x NB diagonal blocks, as the blocked solves below use it.
struct Factor {
  const double* L; const double* linv; long n; int nblk;
};

// Forward substitution L Y = R for the columns of a chunk (R: [n][cn], row stride ldr, used
// as scratch); Y goes to out (row stride ldo).
static xtc_status solve_chunk(const Factor& f, long cn, double* R, long ldr, double* out, long ldo,
                              hipStream_t st) {
  const long n = f.n;
  // forward: Y_i = Linv_ii (R_i - L_i,<i Y_<i), Y stored in out
  for (int b = 0; b < f.nblk; ++b) {
    long i0 = (long)b * NB;
    long nb = (n - i0) < NB ? (n - i0) : NB;
    if (i0 > 0) {
      GemmArgs g{};
      g.M = nb; g.N = cn; g.K = i0;
      g.A = f.L + i0 * n; g.a_sm = n; g.a_sk = 1;
      g.B = out; g.b_sk = ldo; g.b_sn = 1;
      g.C = R + i0 * ldr; g.c_sm = ldr; g.c_sn = 1;
      g.alpha = -1.0; g.beta = 1.0;
      XTC_TRY(gemm_f64(g, st));
    }
    GemmArgs d{};
    d.M = nb; d.N = cn; d.K = nb;
    d.A = f.linv + (long)b * NB * NB; d.a_sm = NB; d.a_sk = 1;
    d.B = R + i0 * ldr; d.b_sk = ldr; d.b_sn = 1;
    d.C = out + i0 * ldo; d.c_sm = ldo; d.c_sn = 1;
    XTC_TRY(gemm_f64(d, st));
  }
  return XTC_OK;
}

// Back substitution L^T X = Y in place in out (row stride ldo); R [n][cn] (row stride ldr)
// is scratch.
static xtc_status back_chunk(const Factor& f, long cn, double* R, long ldr, double* out, long ldo,
                             hipStream_t st) {
  const long n = f.n;
  for (int b = f.nblk - 1; b >= 0; --b) {
    long i0 = (long)b * NB;
    long nb = (n - i0) < NB ? (n - i0) : NB;
    long i1 = i0 + nb;
    if (i1 < n) {
      GemmArgs g{};   // R_i = Y_i - L_{>i,i}^T X_{>i}
      g.M = nb; g.N = cn; g.K = n - i1;
      g.A = f.L + i1 * n + i0; g.a_sm = 1; g.a_sk = n;
      g.B = out + i1 * ldo; g.b_sk = ldo; g.b_sn = 1;
      g.C = R + i0 * ldr; g.c_sm = ldr; g.c_sn = 1;
      g.alpha = -1.0; g.beta = 1.0;   // R_i holds a copy of Y_i (below)
      hipLaunchKernelGGL(k_copy_rows, dim3(cdiv(nb * cn, 256)), dim3(256), 0, st,
                         (const double*)(out + i0 * ldo), ldo, R + i0 * ldr, ldr, (int)nb, cn);
      XTC_CHECK_LAUNCH();
      XTC_TRY(gemm_f64(g, st));
    } else {
      hipLaunchKernelGGL(k_copy_rows, dim3(cdiv(nb * cn, 256)), dim3(256), 0, st,
                         (const double*)(out + i0 * ldo), ldo, R + i0 * ldr, ldr, (int)nb, cn);
      XTC_CHECK_LAUNCH();
    }
    GemmArgs d{};   // X_i = Linv_ii^T R_i
    d.M = nb; d.N = cn; d.K = nb;
    d.A = f.linv + (long)b * NB * NB; d.a_sm = 1; d.a_sk = NB;
    d.B = R + i0 * ldr; d.b_sk = ldr; d.b_sn = 1;
    d.C = out + i0 * ldo; d.c_sm = ldo; d.c_sn = 1;
    XTC_TRY(gemm_f64(d, st));
  }
  return XTC_OK;
}

static Factor factor_of(const FitLayout& F, long n) { return Factor{F.A, F.linv, n, F.nblk}; }

// The right-hand side of one system for grid points [g0, g0 + cn) into R (row stride ldr),
// with P (row stride ldr) as scratch: B = P o P (scalar, comp -1) or (dPhi_mu^T dPhi)_c o P,
// P = Phi_mu^T Phi. phimu: [4][n_orb][n_mu], the orbitals and gradients at the pivots.
static xtc_status rhs_chunk(const double* phi4, long n_g, int n_orb, const double* phimu, long n,
                            int comp, long g0, long cn, double* P, double* R, long ldr,
                            hipStream_t st) {
  GemmArgs p{};   // P = Phi_mu^T Phi (chunk)
  p.M = n; p.N = cn; p.K = n_orb;
  p.A = phimu; p.a_sm = 1; p.a_sk = n;
  p.B = phi4 + g0; p.b_sk = n_g; p.b_sn = 1;
  p.C = P; p.c_sm = ldr; p.c_sn = 1;
  XTC_TRY(gemm_f64(p, st));
  GemmArgs r{};   // B = P o P or (dPhi_mu^T dPhi)_c o P
  r.M = n; r.N = cn; r.K = n_orb;
  const double* ph = phimu + (long)(comp < 0 ? 0 : (1 + comp)) * n_orb * n;
  r.A = ph; r.a_sm = 1; r.a_sk = n;
  r.B = phi4 + (long)(comp < 0 ? 0 : (1 + comp)) * n_orb * n_g + g0; r.b_sk = n_g; r.b_sn = 1;
  r.C = R; r.c_sm = ldr; r.c_sn = 1;
  r.epi = EPI_MUL_E; r.E = P; r.e_sm = ldr; r.e_sn = 1;
  return gemm_f64(r, st);
}

__global__ void k_to_f32(const double* __restrict__ src, long lds, float* __restrict__ dst,
                         long ldd, long rows, long cols) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= rows * cols) return;
  const long r = t / cols, c = t % cols;
  dst[r * ldd + c] = (float)src[r * lds + c];
}

// Cholesky of F.A with the adaptive Tikhonov retry; F.Asave receives the unshifted A.
// *k_used = -1 (no shift) or the shift index; XTC_ERR_NOT_SPD after the last retry.
static xtc_status chol_jitter(FitLayout& F, long n, hipStream_t st, int* k_used) {
  XTC_HIP(hipMemcpyAsync(F.Asave, F.A, sizeof(double) * n * n, hipMemcpyDeviceToDevice, st));
  int failed = 0;
  XTC_TRY(cholesky(F, n, st, &failed));
  *k_used = -1;
  if (!failed) return XTC_OK;
  hipLaunchKernelGGL(k_diag_extract, dim3(cdiv(n, 256)), dim3(256), 0, st, (const double*)F.Asave,
                     n, F.dg);
  std::vector<double> hd(n);
  XTC_HIP(hipMemcpyAsync(hd.data(), F.dg, sizeof(double) * n, hipMemcpyDeviceToHost, st));
  XTC_HIP(hipStreamSynchronize(st));
  double mean = 0.0;
  for (long i = 0; i < n; ++i) mean += hd[i];
  mean /= (double)n;
  for (int k = 0; k < 9; ++k) {
    const double shift = 1e-14 * pow(10.0, k) * mean;
    hipLaunchKernelGGL(k_restore_shift, dim3(cdiv(n * n, 256)), dim3(256), 0, st,
                       (const double*)F.Asave, F.A, n, shift);
    XTC_CHECK_LAUNCH();
    XTC_TRY(cholesky(F, n, st, &failed));
    if (!failed) {
      *k_used = k;
      return XTC_OK;
    }
  }
  set_error("isdf_fit: Gram matrix not positive definite after the last Tikhonov shift");
  return XTC_ERR_NOT_SPD;
}

// Relative weighted fit residuals of a pivot set in the four systems (scalar, x, y, z; the
// judge of the learned selection): per system the Gram, its Cholesky with the retry, and per
// grid chunk the right-hand side, the forward solve and the residual sums; xi is not formed.
// Uses (and releases) arena space after ar.used.
xtc_status fit_residuals(const double* phi4, const xtc_grid* grid, int n_orb,
                         const int64_t* pivots, int n_mu, Arena& ar, hipStream_t st, double* rel) {
  const size_t mark = ar.used;
  const long n_g = grid->n_g;
  FitLayout F = layout_fit(ar, n_g, n_orb, n_mu);
  XTC_TRY(need_ws(ar));
  XTC_HIP(hipMemcpyAsync(F.piv, pivots, sizeof(long) * n_mu, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_gather_piv, dim3(cdiv(4L * n_orb * n_mu, 256)), dim3(256), 0, st, phi4,
                     n_g, 4 * n_orb, (const long*)F.piv, n_mu, F.phimu);
  XTC_CHECK_LAUNCH();
  const long n = n_mu;
  {
    GemmArgs g{};   // G = Phi_mu^T Phi_mu
    g.M = n; g.N = n; g.K = n_orb;
    g.A = F.phimu; g.a_sm = 1; g.a_sk = n;
    g.B = F.phimu; g.b_sk = n; g.b_sn = 1;
    g.C = F.G; g.c_sm = n; g.c_sn = 1;
    XTC_TRY(gemm_f64(g, st));
  }
  for (int sys = 0; sys < 4; ++sys) {
    const int comp = sys - 1;
    GemmArgs g{};
    g.M = n; g.N = n; g.K = n_orb;
    const double* ph = F.phimu + (long)sys * n_orb * n;
    g.A = ph; g.a_sm = 1; g.a_sk = n;
    g.B = ph; g.b_sk = n; g.b_sn = 1;
    g.C = F.A; g.c_sm = n; g.c_sn = 1;
    g.epi = EPI_MUL_E; g.E = F.G; g.e_sm = n; g.e_sn = 1;
    XTC_TRY(gemm_f64(g, st));
    int k = -1;
    XTC_TRY(chol_jitter(F, n, st, &k));
    for (int c = 0; c < F.nchunks; ++c) {
      const long g0 = (long)c * F.chunk;
      const long cn = (n_g - g0) < F.chunk ? (n_g - g0) : F.chunk;
      XTC_TRY(rhs_chunk(phi4, n_g, n_orb, F.phimu, n, comp, g0, cn, F.P, F.R, F.chunk, st));
      XTC_TRY(solve_chunk(factor_of(F, n), cn, F.R, F.chunk, F.P, F.chunk, st));  // Y into F.P
      hipLaunchKernelGGL(k_resid, dim3(cdiv(cn, 256)), dim3(256), 0, st, phi4, grid->w, n_g, n_orb,
                         comp, g0, cn, (const double*)F.P, F.chunk, n_mu, F.rtmp, F.mtmp);
      XTC_CHECK_LAUNCH();
      XTC_TRY(reduce_sum_f64(F.rtmp, cn, F.sums + 2 * c, F.red, st));
      XTC_TRY(reduce_sum_f64(F.mtmp, cn, F.sums + 2 * c + 1, F.red, st));
    }
    std::vector<double> hs(2 * F.nchunks);
    XTC_HIP(hipMemcpyAsync(hs.data(), F.sums, sizeof(double) * 2 * F.nchunks,
                           hipMemcpyDeviceToHost, st));
    XTC_HIP(hipStreamSynchronize(st));
    double rs = 0.0, ms = 0.0;
    for (int c = 0; c < F.nchunks; ++c) {
      rs += hs[2 * c];
      ms += hs[2 * c + 1];
    }
    rel[sys] = ms > 0.0 ? rs / ms : 0.0;
  }
  ar.used = mark;
  return XTC_OK;
}

size_t ws_fit_residual(int64_t n_g, int n_orb, int n_mu) {
  Arena ar(nullptr, 0);
  layout_fit(ar, n_g, n_orb, n_mu);
  return ar.used;
}

// Copies the factor of one system (L, then the inverted diagonal blocks) to dst.
static xtc_status keep_factor(const FitLayout& F, long n, double* dst, hipStream_t st) {
  XTC_HIP(hipMemcpyAsync(dst, F.A, sizeof(double) * n * n, hipMemcpyDeviceToDevice, st));
  XTC_HIP(hipMemcpyAsync(dst + n * n, F.linv, sizeof(double) * F.nblk * NB * NB,
                         hipMemcpyDeviceToDevice, st));
  return XTC_OK;
}

// xi (sys 0) or xi~^c (sys 1 + c) at grid points [g0, g0 + cn) from a factor kept by
// isdf_fit (XTC_FIT_KEEP_CHOL): the same right-hand-side GEMMs and blocked solves as the
// fit, so the columns equal the fit's bit for bit. phimu: [4][n_orb][n_mu] at the pivots;
// out [n_mu][cn] (row stride ldo); P, R: scratch [n_mu][cn] (row stride ldr).
xtc_status fit_columns(const double* phi4, long n_g, int n_orb, const double* phimu, int n_mu,
                       int sys, const double* chol_sys, long g0, long cn, double* out, long ldo,
                       double* P, double* R, long ldr, hipStream_t st) {
  const long n = n_mu;
  const Factor f{chol_sys, chol_sys + n * n, n, (int)cdiv(n, NB)};
  XTC_TRY(rhs_chunk(phi4, n_g, n_orb, phimu, n, sys - 1, g0, cn, P, R, ldr, st));
  XTC_TRY(solve_chunk(f, cn, R, ldr, out, ldo, st));
  return back_chunk(f, cn, R, ldr, out, ldo, st);
}

xtc_status gather_pivot_rows(const double* phi4, long n_g, int rows, const long* piv, int n_mu,
                             double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_gather_piv, dim3(cdiv((long)rows * n_mu, 256)), dim3(256), 0, st, phi4, n_g,
                     rows, piv, n_mu, out);
  XTC_CHECK_LAUNCH();
  return XTC_OK;
}

}  // namespace xtc

using namespace xtc;

__global__ void k_gather_rho(const double* __restrict__ rho, const long* __restrict__ piv,
                             int n_mu, double* __restrict__ G) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n_mu) G[i] = rho[piv[i]];
}

extern "C" xtc_status isdf_fit(const double* phi4, const xtc_grid* grid, int32_t n_orb,
                               const int64_t* pivots, int32_t n_mu, uint32_t what,
                               int32_t xi_prec, void* xi, double* xigrad, double* chol,
                               const double* rho, double* rhot, double* info, void* ws,
                               size_t ws_bytes, void* stream) {
  XTC_REQUIRE(phi4 && grid && pivots, "isdf_fit: null argument");
  XTC_REQUIRE(grid->n_g > 0 && grid->w, "isdf_fit: empty grid");
  XTC_REQUIRE(n_orb > 0 && n_mu > 0 && n_mu <= grid->n_g, "isdf_fit: bad sizes");
  XTC_REQUIRE(!(what & XTC_FIT_XI) || xi, "isdf_fit: xi requested but NULL");
  XTC_REQUIRE(!(what & XTC_FIT_XIGRAD) || xigrad, "isdf_fit: xigrad requested but NULL");
  XTC_REQUIRE(!(what & XTC_FIT_KEEP_CHOL) || chol, "isdf_fit: factors requested but chol NULL");
  XTC_REQUIRE(what & (XTC_FIT_XI | XTC_FIT_XIGRAD | XTC_FIT_KEEP_CHOL),
              "isdf_fit: nothing requested");
  XTC_REQUIRE((what & ~7u) == 0, "isdf_fit: unknown bits in what");
  XTC_REQUIRE(xi_prec == XTC_FP64 || xi_prec == XTC_FP32, "isdf_fit: xi_prec must be FP64 or FP32");
  XTC_REQUIRE(!rhot || (rho && (what & XTC_FIT_XI)), "isdf_fit: rhot needs rho and XTC_FIT_XI");
  const long n_g = grid->n_g;
  for (int m = 0; m < n_mu; ++m)
    XTC_REQUIRE(pivots[m] >= 0 && pivots[m] < n_g, "isdf_fit: pivot index out of range");
  hipStream_t st = as_stream(stream);
  Arena ar(ws, ws_bytes);
  FitLayout F = layout_fit(ar, n_g, n_orb, n_mu, true);
  CallEvents evs;
  if (F.lanes > 1) XTC_TRY(evs.create(F.lanes));
  double* Grho = rhot ? ar.take<double>(n_mu) : nullptr;   // rho at the pivots
  XTC_TRY(need_ws(ar));
  XTC_TRY(check_weights(grid, ws, ws_bytes, st, "isdf_fit"));
  size_t tk = timing_begin(TM_FIT, st);
  XTC_HIP(hipMemcpyAsync(F.piv, pivots, sizeof(long) * n_mu, hipMemcpyHostToDevice, st));
  if (rhot) {
    hipLaunchKernelGGL(k_gather_rho, dim3(cdiv(n_mu, 256)), dim3(256), 0, st, rho,
                       (const long*)F.piv, n_mu, Grho);
    XTC_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(k_gather_piv, dim3(cdiv(4L * n_orb * n_mu, 256)), dim3(256), 0, st, phi4,
                     n_g, 4 * n_orb, (const long*)F.piv, n_mu, F.phimu);
  XTC_CHECK_LAUNCH();
  const long n = n_mu;
  const size_t sys_doubles = XTC_CHOL_SYSTEM_DOUBLES(n_mu);
  // G = Phi_mu^T Phi_mu
  {
    GemmArgs g{};
    g.M = n; g.N = n; g.K = n_orb;
    g.A = F.phimu; g.a_sm = 1; g.a_sk = n;
    g.B = F.phimu; g.b_sk = n; g.b_sn = 1;
    g.C = F.G; g.c_sm = n; g.c_sn = 1;
    XTC_TRY(gemm_f64(g, st));
  }
  double jit[4] = {-1, -1, -1, -1}, rel[4] = {0, 0, 0, 0};
  bool any_jitter = false;
  const bool keep = (what & XTC_FIT_KEEP_CHOL) != 0;
  for (int sys = 0; sys < 4; ++sys) {
    const int comp = sys - 1;   // -1 scalar, 0..2 gradient component
    const bool solve = sys == 0 ? (what & XTC_FIT_XI) != 0 : (what & XTC_FIT_XIGRAD) != 0;
    if (!solve && !keep) continue;
    // Gram of this system
    {
      GemmArgs g{};
      g.M = n; g.N = n; g.K = n_orb;
      const double* ph = F.phimu + (long)(sys == 0 ? 0 : (1 + comp)) * n_orb * n;
      g.A = ph; g.a_sm = 1; g.a_sk = n;
      g.B = ph; g.b_sk = n; g.b_sn = 1;
      g.C = F.A; g.c_sm = n; g.c_sn = 1;
      g.epi = EPI_MUL_E; g.E = F.G; g.e_sm = n; g.e_sn = 1;
      XTC_TRY(gemm_f64(g, st));
    }
    int k = -1;
    XTC_TRY(chol_jitter(F, n, st, &k));
    if (k >= 0) {
      jit[sys] = k;
      any_jitter = true;
    }
    if (keep) XTC_TRY(keep_factor(F, n, chol + sys * sys_doubles, st));
    if (!solve) continue;
    // the FP64 solution of a chunk goes straight into the output, or (FP32 xi) into P first;
    // chunk c runs in lane c % lanes (lane 0 on the caller's stream), forked from and
    // joined back into it with events
    const bool f32 = sys == 0 && xi_prec == XTC_FP32;
    hipStream_t ls[FIT_LANES] = {st};
    if (F.lanes > 1) {
      XTC_HIP(hipEventRecord(evs.ev[0], st));
      for (int l = 1; l < F.lanes; ++l) {
        XTC_TRY(aux_stream(l - 1, &ls[l]));
        XTC_HIP(hipStreamWaitEvent(ls[l], evs.ev[0], 0));
      }
    }
    for (int c = 0; c < F.nchunks; ++c) {
      const int l = c % F.lanes;
      hipStream_t sl = ls[l];
      long g0 = (long)c * F.chunk;
      long cn = (n_g - g0) < F.chunk ? (n_g - g0) : F.chunk;
      double* out = f32 ? F.Px[l] : (sys == 0 ? (double*)xi : xigrad + (long)comp * n * n_g) + g0;
      const long ldo = f32 ? F.chunk : n_g;
      XTC_TRY(rhs_chunk(phi4, n_g, n_orb, F.phimu, n, comp, g0, cn, F.Px[l], F.Rx[l], F.chunk, sl));
      XTC_TRY(solve_chunk(factor_of(F, n), cn, F.Rx[l], F.chunk, out, ldo, sl));
      hipLaunchKernelGGL(k_resid, dim3(cdiv(cn, 256)), dim3(256), 0, sl, phi4, grid->w, n_g,
                         n_orb, comp, g0, cn, (const double*)out, ldo, n_mu, F.rtx[l], F.mtx[l]);
      XTC_CHECK_LAUNCH();
      XTC_TRY(reduce_sum_f64(F.rtx[l], cn, F.sums + 2 * c, F.redx[l], sl));
      XTC_TRY(reduce_sum_f64(F.mtx[l], cn, F.sums + 2 * c + 1, F.redx[l], sl));
      XTC_TRY(back_chunk(factor_of(F, n), cn, F.Rx[l], F.chunk, out, ldo, sl));
      if (sys == 0 && rhot) {   // ISDF density from the FP64 solution (the product the
        GemmArgs g{};           // contraction forms from FP64 xi, element for element)
        g.M = 1; g.N = cn; g.K = n;
        g.A = Grho; g.a_sm = 1; g.a_sk = 1;
        g.B = out; g.b_sk = ldo; g.b_sn = 1;
        g.C = rhot + g0; g.c_sm = n_g; g.c_sn = 1;
        XTC_TRY(gemm_f64(g, sl));
      }
      if (f32) {
        hipLaunchKernelGGL(k_to_f32, dim3(cdiv(n * cn, 256)), dim3(256), 0, sl, (const double*)out,
                           ldo, (float*)xi + g0, n_g, n, cn);
        XTC_CHECK_LAUNCH();
      }
    }
    for (int l = 1; l < F.lanes; ++l) {
      XTC_HIP(hipEventRecord(evs.ev[l], ls[l]));
      XTC_HIP(hipStreamWaitEvent(st, evs.ev[l], 0));
    }
    std::vector<double> hs(2 * F.nchunks);
    XTC_HIP(hipMemcpyAsync(hs.data(), F.sums, sizeof(double) * 2 * F.nchunks,
                           hipMemcpyDeviceToHost, st));
    XTC_HIP(hipStreamSynchronize(st));
    double rs = 0.0, ms = 0.0;
    for (int c = 0; c < F.nchunks; ++c) {
      rs += hs[2 * c];
      ms += hs[2 * c + 1];
    }
    rel[sys] = ms > 0.0 ? rs / ms : 0.0;
  }
  timing_end(tk, st);
  XTC_HIP(hipStreamSynchronize(st));
  if (info) {
    for (int i = 0; i < 4; ++i) {
      info[i] = jit[i];
      info[4 + i] = rel[i];
    }
  }
  return any_jitter ? XTC_WARN_JITTER : XTC_OK;
}
