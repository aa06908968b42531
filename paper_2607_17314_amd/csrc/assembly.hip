// Four-index assembly of the transcorrelated two-body corrections and the xTC
// one-body pieces from the ISDF intermediates (K-kernel section, eq.
// K-recombine-final with eqs. K1-isdf and K3-isdf; xTC section, eq.
// delta-u-dx-kernels and the final assembly; Hamiltonian assembly section, eqs.
// xtc-deltah, xtc-fock, xtc-const).
//
// With the pair factors C_mu(p,r) = phi_p phi_r (r_mu) (symmetric in p, r) and
// A^c_mu(p,r) = phi_p d_c phi_r - phi_r d_c phi_p (r_mu) (antisymmetric):
//   K1 - K1swap + K3 = sum_nu PK_nu(p,r) C_nu(q,s),  PK_nu = sum_mu [sum_c A^c_mu u1^c_{mu nu} + C_mu u3_{mu nu}]
//   C D C - C X      = sum_nu PU_nu(p,r) C_nu(q,s) - sum_mu C_mu(p,r) X_mu(q,s),  PU_nu = sum_mu C_mu D_{mu nu}
// and P12 T^{pq}_{rs} = T^{pq}_{rs} + T^{qp}_{sr}, so every output is
//   out[(p,r),(q,s)] = a sum_nu [P(p,r) C(q,s) + C(p,r) P(q,s)] + b sum_mu [C(p,r) X(q,s) + X(p,r) C(q,s)]
// with (P, a, b) = (PK, 1/2, 0) for K, (PU, -1, 1) for dU and (PW = PK/2 + PU, -1, 1) for
// W = -K + dU: one FP64 MFMA product over four k-segments per output panel
// (k_asm_panel), written once. The one-body pieces need only partial traces over the
// occupied orbitals, formed from the same factors without the four-index tensors.
#include "common.hpp"
#include "plans.hpp"
#include "timing.hpp"

namespace xtc {

typedef double d4v __attribute__((ext_vector_type(4)));

struct AsmLayout {
  double* F4;    // [A^x, A^y, A^z, C][n_mu][n_orb^2]
  double* Xm;    // [n_mu][n_orb^2] = X2 + X3 transposed (or nullptr)
  double* PK; double* PU; double* PW;   // [n_mu][n_orb^2] each (when requested)
  double* U4;    // [4][n_mu][n_mu] stacked right factors of the projection GEMMs
  double* vec;   // [3][n_mu]: g, pi, chi of the one-body traces
  double* J; double* Kx;   // [n_orb][n_orb] one-body partial traces
  double* dhd;   // [n_orb] diagonal of dh
  long nn;       // n_orb^2
};

static AsmLayout layout_asm(Arena& ar, int n_orb, int n_mu, uint32_t outputs, bool one_body) {
  AsmLayout L{};
  L.nn = (long)n_orb * n_orb;
  const size_t blk = (size_t)n_mu * L.nn;
  L.F4 = ar.take<double>(4 * blk);
  L.Xm = ar.take<double>(blk);
  if (outputs & XTC_ASM_K) L.PK = ar.take<double>(blk);
  if (outputs & XTC_ASM_DU) L.PU = ar.take<double>(blk);
  if (outputs & XTC_ASM_W) L.PW = ar.take<double>(blk);
  L.U4 = ar.take<double>((size_t)4 * n_mu * n_mu);
  L.vec = ar.take<double>((size_t)3 * n_mu);
  if (one_body) {
    L.J = ar.take<double>(L.nn);
    L.Kx = ar.take<double>(L.nn);
    L.dhd = ar.take<double>(n_orb);
  }
  return L;
}

size_t ws_assembly(int n_orb, int n_mu, uint32_t outputs) {
  Arena ar(nullptr, 0);
  layout_asm(ar, n_orb, n_mu, outputs, false);
  return ar.used;
}

size_t ws_one_body(int n_orb, int n_mu) {
  Arena ar(nullptr, 0);
  layout_asm(ar, n_orb, n_mu, XTC_ASM_DU | XTC_ASM_W, true);
  return ar.used;
}

// F4[c][mu][p n + r] = A^c_mu(p,r) (c < 3), F4[3][mu][p n + r] = C_mu(p,r)
__global__ void k_pair_factors(const double* __restrict__ phi4, int n, int n_mu,
                               double* __restrict__ F4) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  const long nn = (long)n * n;
  if (t >= (long)n_mu * nn) return;
  const long pr = t % nn;
  const int mu = (int)(t / nn);
  const int p = (int)(pr / n), r = (int)(pr % n);
  const long sp = (long)p * n_mu + mu, sr = (long)r * n_mu + mu, comp = (long)n * n_mu;
  const double fp = phi4[sp], fr = phi4[sr];
  const long blk = (long)n_mu * nn;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    F4[c * blk + t] = fp * phi4[(1 + c) * comp + sr] - fr * phi4[(1 + c) * comp + sp];
  F4[3 * blk + t] = fp * fr;
}

// U4[seg][mu][nu] = s1 * M1[seg] + s2 * M2 (a scaled copy, M2 only in the last segment)
__global__ void k_stack_u(const double* __restrict__ u1, const double* __restrict__ u3,
                          const double* __restrict__ Da, const double* __restrict__ Db, int n_mu,
                          double su, double s3, double sa, double sb, double* __restrict__ U4) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  const long m2 = (long)n_mu * n_mu;
  if (t >= 4 * m2) return;
  const int seg = (int)(t / m2);
  const long i = t % m2;
  double v;
  if (seg < 3) {
    v = su * u1[seg * m2 + i];
  } else {
    v = s3 * u3[i];
    if (Da) v += sa * Da[i];
    if (Db) v += sb * Db[i];
  }
  U4[t] = v;
}

// Xm[mu][q n + s] = X2[q][s][mu] + X3[q][s][mu] (64 x 64 tiles through LDS)
__global__ __launch_bounds__(256) void k_x_transpose(const double* __restrict__ X2,
                                                     const double* __restrict__ X3, long nn,
                                                     int n_mu, double* __restrict__ Xm) {
  __shared__ double tile[64][65];
  const long qs0 = (long)blockIdx.x * 64;
  const int mu0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const long qs = qs0 + r;
    const int mu = mu0 + tx;
    double v = 0.0;
    if (qs < nn && mu < n_mu) {
      const long i = qs * n_mu + mu;
      if (X2) v += X2[i];
      if (X3) v += X3[i];
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int mu = mu0 + r;
    const long qs = qs0 + tx;
    if (mu < n_mu && qs < nn) Xm[(long)mu * nn + qs] = tile[tx][r];
  }
}

// The panel product: out[m][n] = sum_seg coef[seg] sum_k R[seg][k][m_off + m] S[seg][k][n],
// every operand k-major ([k][ld], the m or n index contiguous), K = kseg per segment.
// 128 x 128 tile of out per workgroup, 4 waves of 64 x 64 (4 x 4 blocks of
// v_mfma_f64_16x16x4f64), k-tiles of 16 through LDS with the next tile prefetched in
// registers. The k loop runs over (segment, k-tile) pairs, so the segment, its
// pointers and coefficient are uniform per tile; a segment's last tile is zero-padded.
// Launch order: a 1-D grid of 8 x ceil(tiles / 8) workgroups; the hardware deals them
// round-robin to the 8 XCDs, so workgroup id goes to XCD id % 8, and each XCD takes a
// contiguous run of output tiles with the M tile fastest. The workgroups that share an
// N tile (the large, panel-independent operand S) then run together on one XCD and read
// it through that XCD's L2 instead of each streaming it from HBM.
struct AsmSegs {
  const double* R[4];
  const double* S[4];
  double coef[4];
  int nseg;
  long kseg, ld, m_off;
};

constexpr int AT = 128, AK = 16, ALD = AT + 2;

__global__ __attribute__((amdgpu_flat_work_group_size(256, 256), amdgpu_waves_per_eu(2, 2)))
void k_asm_panel(AsmSegs sg, long M, long N, double* __restrict__ out, long ldc) {
  __shared__ double As[AK][ALD];
  __shared__ double Bs[AK][ALD];
  const long n_mt = (M + AT - 1) / AT, n_tiles = n_mt * ((N + AT - 1) / AT);
  const long per_xcd = (n_tiles + 7) / 8;
  const long logical = (long)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (logical >= n_tiles) return;   // the whole workgroup, before any barrier
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const long m0 = (logical % n_mt) * AT, n0 = (logical / n_mt) * AT;
  const int tps = (int)((sg.kseg + AK - 1) / AK);   // k-tiles per segment
  const int ntiles = tps * sg.nseg;
  const int ld = (int)sg.ld;                          // n_orb^2 < 2^31
  const int mlim = (int)(M - m0 < AT ? M - m0 : AT), nlim = (int)(N - n0 < AT ? N - n0 : AT);
  double ra[8], rb[8];
  auto load = [&](int t) {
    const int s = t / tps;
    const int k0 = (t - s * tps) * AK;
    const int kl = (int)sg.kseg - k0;                 // rows left in this segment
    const double* Rt = sg.R[s] + (long)k0 * sg.ld + sg.m_off + m0;
    const double* St = sg.S[s] + (long)k0 * sg.ld + n0;
    const double c = sg.coef[s];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      const int mm = e & (AT - 1), kk = e >> 7;
      const bool kin = kk < kl;
      ra[j] = (kin && mm < mlim) ? c * Rt[kk * ld + mm] : 0.0;
      rb[j] = (kin && mm < nlim) ? St[kk * ld + mm] : 0.0;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = tid + 256 * j;
      As[e >> 7][e & (AT - 1)] = ra[j];
      Bs[e >> 7][e & (AT - 1)] = rb[j];
    }
  };
  d4v acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (d4v){0.0, 0.0, 0.0, 0.0};
  const int li = lane & 15, lk = lane >> 4;
  load(0);
  for (int t = 0; t < ntiles; ++t) {
    __syncthreads();
    stash();
    __syncthreads();
    if (t + 1 < ntiles) load(t + 1);
#pragma unroll
    for (int s = 0; s < AK / 4; ++s) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        a[i] = As[4 * s + lk][64 * wm + 16 * i + li];
        b[i] = Bs[4 * s + lk][64 * wn + 16 * i + li];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  // D[(l / 16) + 4 r][l % 16] of each 16 x 16 block
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long m = m0 + 64 * wm + 16 * i + lk + 4 * r;
        const long n = n0 + 64 * wn + 16 * j + li;
        if (m < M && n < N) out[m * ldc + n] = acc[i][j][r];
      }
}

// g[k] = sum_o C_k(o,o); pi[k] = sum_o P_k(o,o); chi[k] = sum_o X_k(o,o) (o < n_occ)
__global__ void k_occ_diag(const double* __restrict__ C, const double* __restrict__ P,
                           const double* __restrict__ Xm, int n, int n_occ, int n_mu,
                           double* __restrict__ vec) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n_mu) return;
  const long nn = (long)n * n;
  double g = 0.0, pi = 0.0, chi = 0.0;
  for (int o = 0; o < n_occ; ++o) {
    const long i = (long)k * nn + (long)o * n + o;
    g += C[i];
    pi += P[i];
    chi += Xm[i];
  }
  vec[k] = g;
  vec[n_mu + k] = pi;
  vec[2 * n_mu + k] = chi;
}

__global__ void k_one_body_mix(const double* __restrict__ J, const double* __restrict__ Kx,
                               long nn, double cj, double ck, const double* __restrict__ base,
                               double* __restrict__ out) {
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= nn) return;
  out[t] = (base ? base[t] : 0.0) + cj * J[t] + ck * Kx[t];
}

__global__ void k_diag(const double* __restrict__ M, int n, double* __restrict__ d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) d[i] = M[(long)i * n + i];
}

static xtc_status check_asm(const xtc_assembly* a) {
  XTC_REQUIRE(a, "assembly: null argument");
  XTC_REQUIRE(a->n_orb > 0 && a->n_mu > 0, "assembly: bad sizes");
  XTC_REQUIRE(a->phi4_piv && a->u1 && a->u3 && a->D1 && a->D4,
              "assembly: null phi4_piv, u1, u3, D1 or D4");
  XTC_REQUIRE((long)a->n_orb * a->n_orb <= (1L << 31), "assembly: n_orb too large");
  return XTC_OK;
}

// The factors every panel reads (see the file comment).
static xtc_status prepare(const xtc_assembly* a, uint32_t outputs, const AsmLayout& L,
                          hipStream_t st) {
  const int n = a->n_orb, n_mu = a->n_mu;
  const long nn = L.nn, blk = (long)n_mu * nn;
  hipLaunchKernelGGL(k_pair_factors, dim3(cdiv(blk, 256)), dim3(256), 0, st, a->phi4_piv, n, n_mu,
                     L.F4);
  XTC_CHECK_LAUNCH();
  hipLaunchKernelGGL(k_x_transpose, dim3(cdiv(nn, 64), cdiv(n_mu, 64)), dim3(256), 0, st, a->X2,
                     a->X3, nn, n_mu, L.Xm);
  XTC_CHECK_LAUNCH();
  const long m2 = (long)n_mu * n_mu;
  // P[nu][pr] = sum_seg sum_mu U4[seg][mu][nu] F4[seg][mu][pr]   (segments 0..3 of F4)
  auto project = [&](double* P, int seg0, int nseg) {
    GemmArgs g{};
    g.M = n_mu; g.N = nn; g.K = (long)nseg * n_mu;
    g.A = L.U4 + (long)seg0 * m2; g.a_sm = 1; g.a_sk = n_mu;
    g.B = L.F4 + (long)seg0 * blk; g.b_sk = nn; g.b_sn = 1;
    g.C = P; g.c_sm = nn; g.c_sn = 1;
    return gemm_f64(g, st);
  };
  const unsigned gs = cdiv(4 * m2, 256);
  if (outputs & XTC_ASM_K) {
    hipLaunchKernelGGL(k_stack_u, dim3(gs), dim3(256), 0, st, a->u1, a->u3, (const double*)nullptr,
                       (const double*)nullptr, n_mu, 1.0, 1.0, 0.0, 0.0, L.U4);
    XTC_CHECK_LAUNCH();
    XTC_TRY(project(L.PK, 0, 4));
  }
  if (outputs & XTC_ASM_DU) {
    hipLaunchKernelGGL(k_stack_u, dim3(gs), dim3(256), 0, st, a->u1, a->u3, a->D4, a->D1, n_mu,
                       0.0, 0.0, 1.0, 2.0, L.U4);
    XTC_CHECK_LAUNCH();
    XTC_TRY(project(L.PU, 3, 1));
  }
  if (outputs & XTC_ASM_W) {
    hipLaunchKernelGGL(k_stack_u, dim3(gs), dim3(256), 0, st, a->u1, a->u3, a->D4, a->D1, n_mu,
                       0.5, 0.5, 1.0, 2.0, L.U4);
    XTC_CHECK_LAUNCH();
    XTC_TRY(project(L.PW, 0, 4));
  }
  return XTC_OK;
}

static AsmSegs segs_for(const AsmLayout& L, const double* P, double a, double b, bool has_x,
                        int n_mu) {
  AsmSegs s{};
  const double* C = L.F4 + 3L * n_mu * L.nn;
  s.R[0] = P; s.S[0] = C; s.coef[0] = a;
  s.R[1] = C; s.S[1] = P; s.coef[1] = a;
  s.nseg = 2;
  if (has_x) {
    s.R[2] = C; s.S[2] = L.Xm; s.coef[2] = b;
    s.R[3] = L.Xm; s.S[3] = C; s.coef[3] = b;
    s.nseg = 4;
  }
  s.kseg = n_mu;
  s.ld = L.nn;
  return s;
}

// Partial traces of out = a P12[sum P C] + b P12[sum C X]-type tensors:
//   J[p][q] = sum_o out[(p,q),(o,o)],  Kx[p][q] = sum_o out[(p,o),(o,q)]
static xtc_status partial_traces(const AsmLayout& L, const double* P, double a, double b,
                                 bool has_x, int n, int n_occ, int n_mu, hipStream_t st) {
  const long nn = L.nn;
  const double* C = L.F4 + 3L * n_mu * nn;
  hipLaunchKernelGGL(k_occ_diag, dim3(cdiv(n_mu, 256)), dim3(256), 0, st, C, P,
                     (const double*)L.Xm, n, n_occ, n_mu, L.vec);
  XTC_CHECK_LAUNCH();
  const double* g = L.vec;
  const double* pi = L.vec + n_mu;
  const double* chi = L.vec + 2 * n_mu;
  // J = a (P g + C pi) + b (C chi + X g), as products [n^2 x n_mu] [n_mu x 1]
  struct Term { const double* M; const double* v; double c; };
  const Term jt[4] = {{P, g, a}, {C, pi, a}, {C, chi, b}, {L.Xm, g, b}};
  const int njt = has_x ? 4 : 2;
  for (int i = 0; i < njt; ++i) {
    GemmArgs q{};
    q.M = nn; q.N = 1; q.K = n_mu;
    q.A = jt[i].M; q.a_sm = 1; q.a_sk = nn;
    q.B = jt[i].v; q.b_sk = 1; q.b_sn = 1;
    q.C = L.J; q.c_sm = 1; q.c_sn = 1;
    q.alpha = jt[i].c;
    q.beta = i == 0 ? 0.0 : 1.0;
    XTC_TRY(gemm_f64(q, st));
  }
  // Kx = sum_o [a (P(p,o) C(o,q) + C(p,o) P(o,q)) + b (C(p,o) X(o,q) + X(p,o) C(o,q))]
  struct Pair { const double* L; const double* R; double c; };
  const Pair kt[4] = {{P, C, a}, {C, P, a}, {C, L.Xm, b}, {L.Xm, C, b}};
  const int nkt = has_x ? 4 : 2;
  bool first = true;
  for (int o = 0; o < n_occ; ++o)
    for (int i = 0; i < nkt; ++i) {
      GemmArgs q{};
      q.M = n; q.N = n; q.K = n_mu;
      q.A = kt[i].L + o; q.a_sm = n; q.a_sk = nn;            // A[p][k] = L_k(p, o)
      q.B = kt[i].R + (long)o * n; q.b_sk = nn; q.b_sn = 1;  // B[k][q] = R_k(o, q)
      q.C = L.Kx; q.c_sm = n; q.c_sn = 1;
      q.alpha = kt[i].c;
      q.beta = first ? 0.0 : 1.0;
      first = false;
      XTC_TRY(gemm_f64(q, st));
    }
  return XTC_OK;
}

}  // namespace xtc

using namespace xtc;

extern "C" xtc_status xtc_assembly_prepare(const xtc_assembly* a, uint32_t outputs, void* ws,
                                           size_t ws_bytes, void* stream) {
  XTC_TRY(check_asm(a));
  XTC_REQUIRE(outputs != 0 && (outputs & ~7u) == 0, "assembly: outputs must be a mask of K, DU, W");
  Arena ar(ws, ws_bytes);
  AsmLayout L = layout_asm(ar, a->n_orb, a->n_mu, outputs, false);
  XTC_TRY(need_ws(ar));
  return prepare(a, outputs, L, as_stream(stream));
}

extern "C" xtc_status xtc_assembly_panel(const xtc_assembly* a, uint32_t outputs, int32_t p0,
                                         int32_t p1, double* K, double* dU, double* W, void* ws,
                                         size_t ws_bytes, void* stream) {
  XTC_TRY(check_asm(a));
  XTC_REQUIRE(outputs != 0 && (outputs & ~7u) == 0, "assembly: outputs must be a mask of K, DU, W");
  XTC_REQUIRE(0 <= p0 && p0 <= p1 && p1 <= a->n_orb, "assembly: panel outside the orbital range");
  XTC_REQUIRE(!(outputs & XTC_ASM_K) || K, "assembly: K output NULL");
  XTC_REQUIRE(!(outputs & XTC_ASM_DU) || dU, "assembly: dU output NULL");
  XTC_REQUIRE(!(outputs & XTC_ASM_W) || W, "assembly: W output NULL");
  Arena ar(ws, ws_bytes);
  AsmLayout L = layout_asm(ar, a->n_orb, a->n_mu, outputs, false);
  XTC_TRY(need_ws(ar));
  if (p1 == p0) return XTC_OK;
  hipStream_t st = as_stream(stream);
  const int n = a->n_orb;
  const bool has_x = a->X2 || a->X3;
  const long M = (long)(p1 - p0) * n, N = L.nn;
  const long n_tiles = (long)cdiv(N, AT) * cdiv(M, AT);
  XTC_REQUIRE(n_tiles <= 0x7fffffffL, "assembly: panel too large for one launch");
  dim3 grid((unsigned)(8 * ((n_tiles + 7) / 8)));
  struct Out { uint32_t bit; const double* P; double a, b; bool x; double* dst; };
  const Out outs[3] = {{XTC_ASM_K, L.PK, 0.5, 0.0, false, K},
                       {XTC_ASM_DU, L.PU, -1.0, 1.0, has_x, dU},
                       {XTC_ASM_W, L.PW, -1.0, 1.0, has_x, W}};
  for (const Out& o : outs) {
    if (!(outputs & o.bit)) continue;
    AsmSegs s = segs_for(L, o.P, o.a, o.b, o.x, a->n_mu);
    s.m_off = (long)p0 * n;
    const size_t tk = timing_begin(TM_ASM_PANEL, st);
    hipLaunchKernelGGL(k_asm_panel, grid, dim3(256), 0, st, s, M, N, o.dst, N);
    timing_end(tk, st);
    XTC_CHECK_LAUNCH();
  }
  return XTC_OK;
}

extern "C" xtc_status xtc_one_body(const xtc_assembly* a, int32_t n_occ, double e_nuc, double* dh,
                                   double* f, double* e0, void* ws, size_t ws_bytes,
                                   void* stream) {
  XTC_TRY(check_asm(a));
  XTC_REQUIRE(n_occ > 0 && n_occ <= a->n_orb, "one-body: bad n_occ");
  XTC_REQUIRE(dh || f || e0, "one-body: no output requested");
  Arena ar(ws, ws_bytes);
  AsmLayout L = layout_asm(ar, a->n_orb, a->n_mu, XTC_ASM_DU | XTC_ASM_W, true);
  XTC_TRY(need_ws(ar));
  hipStream_t st = as_stream(stream);
  const int n = a->n_orb;
  const bool has_x = a->X2 || a->X3;
  XTC_TRY(prepare(a, XTC_ASM_DU | XTC_ASM_W, L, st));
  // dh = -1/2 (2 J[dU] - Kx[dU])   (eq. xtc-deltah)
  XTC_TRY(partial_traces(L, L.PU, -1.0, 1.0, has_x, n, n_occ, a->n_mu, st));
  double* dhb = dh ? dh : L.J;   // dh is needed for f and E0 even when not returned
  const unsigned gb = cdiv(L.nn, 256);
  if (!dh) {
    // keep J, Kx of dU apart from the buffers reused below
    hipLaunchKernelGGL(k_one_body_mix, dim3(gb), dim3(256), 0, st, (const double*)L.J,
                       (const double*)L.Kx, L.nn, -1.0, 0.5, (const double*)nullptr, L.Kx);
    XTC_CHECK_LAUNCH();
    dhb = L.Kx;
  } else {
    hipLaunchKernelGGL(k_one_body_mix, dim3(gb), dim3(256), 0, st, (const double*)L.J,
                       (const double*)L.Kx, L.nn, -1.0, 0.5, (const double*)nullptr, dh);
    XTC_CHECK_LAUNCH();
  }
  if (e0) {
    hipLaunchKernelGGL(k_diag, dim3(cdiv(n, 256)), dim3(256), 0, st, (const double*)dhb, n, L.dhd);
    XTC_CHECK_LAUNCH();
    std::vector<double> d(n);
    XTC_HIP(hipMemcpyAsync(d.data(), L.dhd, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    XTC_HIP(hipStreamSynchronize(st));
    double tr = 0.0;
    for (int i = 0; i < n_occ; ++i) tr += d[i];
    *e0 = -2.0 / 3.0 * tr + e_nuc;   // eq. xtc-const
  }
  if (f) {
    // the dh buffer must survive the W traces: copy it into f first
    hipLaunchKernelGGL(k_one_body_mix, dim3(gb), dim3(256), 0, st, (const double*)dhb,
                       (const double*)dhb, L.nn, 1.0, 0.0, (const double*)nullptr, f);
    XTC_CHECK_LAUNCH();
    // f = dh + 2 J[W] - Kx[W]   (eq. xtc-fock)
    XTC_TRY(partial_traces(L, L.PW, -1.0, 1.0, has_x, n, n_occ, a->n_mu, st));
    hipLaunchKernelGGL(k_one_body_mix, dim3(gb), dim3(256), 0, st, (const double*)L.J,
                       (const double*)L.Kx, L.nn, 2.0, -1.0, (const double*)f, f);
    XTC_CHECK_LAUNCH();
  }
  return XTC_OK;
}
