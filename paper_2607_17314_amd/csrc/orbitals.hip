// Orbital and orbital-gradient values on the grid (Alg. 2, grid step).
// One thread per grid point evaluates every AO value and Cartesian gradient of
// a grid chunk into an SoA buffer ao4[4][n_ao][chunk]; the MO values follow as
// four FP64 MFMA GEMMs phi4[c] = C_mo^T ao4[c]; rho_gamma is a per-point sum
// over the occupied orbitals.
#include "common.hpp"
#include "plans.hpp"
#include "timing.hpp"

namespace xtc {

constexpr int ORB_CHUNK = 32768;
constexpr int MAX_L = 6;

struct BasisDev {
  const double* atom_xyz;
  const int* shell_center;
  const int* shell_l;
  const int* shell_prim_start;
  const double* prim_exp;
  const double* prim_coef;
  const double* comp;
  int n_shell, n_ao;
};

__global__ __launch_bounds__(256) void k_eval_ao(BasisDev b, const double* __restrict__ xyz,
                                                 long n_g, long g0, long chunk,
                                                 double* __restrict__ ao4) {
  long t = (long)blockIdx.x * 256 + threadIdx.x;
  if (t >= chunk) return;
  long g = g0 + t;
  if (g >= n_g) return;
  const double px = xyz[g], py = xyz[n_g + g], pz = xyz[2 * n_g + g];
  const long plane = (long)b.n_ao * chunk;
  int a = 0;
  for (int s = 0; s < b.n_shell; ++s) {
    const int cen = b.shell_center[s];
    const int l = b.shell_l[s];
    const double x = px - b.atom_xyz[3 * cen], y = py - b.atom_xyz[3 * cen + 1],
                 z = pz - b.atom_xyz[3 * cen + 2];
    const double r2 = x * x + y * y + z * z;
    double rad = 0.0, drad = 0.0;
    for (int p = b.shell_prim_start[s]; p < b.shell_prim_start[s + 1]; ++p) {
      double e = b.prim_coef[p] * exp(-b.prim_exp[p] * r2);
      rad += e;
      drad -= 2.0 * b.prim_exp[p] * e;
    }
    double xp[MAX_L + 2], yp[MAX_L + 2], zp[MAX_L + 2];
    xp[0] = yp[0] = zp[0] = 1.0;
    for (int n = 1; n <= l + 1; ++n) {
      xp[n] = xp[n - 1] * x;
      yp[n] = yp[n - 1] * y;
      zp[n] = zp[n - 1] * z;
    }
    for (int i = l; i >= 0; --i) {
      for (int j = l - i; j >= 0; --j, ++a) {
        const int k = l - i - j;
        const double f = b.comp[a];
        const double ang = xp[i] * yp[j] * zp[k];
        const long o = (long)a * chunk + t;
        ao4[o] = f * ang * rad;
        const double dxi = i > 0 ? i * xp[i - 1] : 0.0;
        const double dyj = j > 0 ? j * yp[j - 1] : 0.0;
        const double dzk = k > 0 ? k * zp[k - 1] : 0.0;
        ao4[plane + o] = f * yp[j] * zp[k] * (dxi * rad + xp[i + 1] * drad);
        ao4[2 * plane + o] = f * xp[i] * zp[k] * (dyj * rad + yp[j + 1] * drad);
        ao4[3 * plane + o] = f * xp[i] * yp[j] * (dzk * rad + zp[k + 1] * drad);
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_density(const double* __restrict__ phi, long n_g,
                                                 int n_occ, double* __restrict__ rho) {
  long g = (long)blockIdx.x * 256 + threadIdx.x;
  if (g >= n_g) return;
  double s = 0.0;
  for (int i = 0; i < n_occ; ++i) {
    double v = phi[(long)i * n_g + g];
    s += v * v;
  }
  rho[g] = s;
}

struct OrbLayout {
  double* atom_xyz; int* ints; double* prim; double* comp; double* ao4;
  long chunk;
};

static OrbLayout layout_orb(Arena& ar, int64_t n_g, int n_ao, int n_atom, int n_shell, int n_prim) {
  OrbLayout L;
  L.chunk = n_g < ORB_CHUNK ? n_g : ORB_CHUNK;
  L.atom_xyz = ar.take<double>(3 * (size_t)n_atom);
  L.ints = ar.take<int>(3 * (size_t)n_shell + 1);
  L.prim = ar.take<double>(2 * (size_t)n_prim);
  L.comp = ar.take<double>(n_ao);
  L.ao4 = ar.take<double>(4 * (size_t)n_ao * L.chunk);
  return L;
}

size_t ws_eval_orbitals(int64_t n_g, int n_orb, int n_ao) {
  (void)n_orb;
  Arena ar(nullptr, 0);
  // basis tables are tiny; reserve generously for up to 4096 shells / primitives / atoms
  layout_orb(ar, n_g, n_ao, 4096, 4096, 16384);
  return ar.used;
}

}  // namespace xtc

using namespace xtc;

extern "C" xtc_status xtc_eval_orbitals(const xtc_basis* basis, const xtc_grid* grid,
                                        const double* C_mo, int32_t n_orb, int32_t n_occ,
                                        double* phi4, double* rho, void* ws, size_t ws_bytes,
                                        void* stream) {
  XTC_REQUIRE(basis && grid && C_mo && phi4, "xtc_eval_orbitals: null argument");
  XTC_REQUIRE(grid->n_g > 0 && grid->xyz, "xtc_eval_orbitals: empty grid");
  XTC_REQUIRE(n_orb > 0 && n_occ >= 0 && n_occ <= n_orb, "xtc_eval_orbitals: bad n_orb/n_occ");
  XTC_REQUIRE(basis->n_shell > 0 && basis->n_atom > 0 && basis->n_atom <= 4096 &&
                  basis->n_shell <= 4096,
              "xtc_eval_orbitals: bad basis sizes");
  XTC_REQUIRE(basis->atom_xyz && basis->shell_center && basis->shell_l &&
                  basis->shell_prim_start && basis->prim_exp && basis->prim_coef &&
                  basis->comp_factor,
              "xtc_eval_orbitals: null basis table");
  int n_ao = 0;
  for (int s = 0; s < basis->n_shell; ++s) {
    int l = basis->shell_l[s];
    XTC_REQUIRE(l >= 0 && l <= MAX_L, "xtc_eval_orbitals: angular momentum out of range");
    XTC_REQUIRE(basis->shell_center[s] >= 0 && basis->shell_center[s] < basis->n_atom,
                "xtc_eval_orbitals: shell centre out of range");
    XTC_REQUIRE(basis->shell_prim_start[s + 1] > basis->shell_prim_start[s],
                "xtc_eval_orbitals: shell without primitives");
    n_ao += (l + 1) * (l + 2) / 2;
  }
  int n_prim = basis->shell_prim_start[basis->n_shell];
  XTC_REQUIRE(basis->shell_prim_start[0] == 0 && n_prim <= 16384,
              "xtc_eval_orbitals: bad primitive table");
  XTC_REQUIRE(n_ao == basis->n_ao, "xtc_eval_orbitals: n_ao does not match the shells");
  hipStream_t st = as_stream(stream);
  Arena ar(ws, ws_bytes);
  OrbLayout L = layout_orb(ar, grid->n_g, n_ao, basis->n_atom, basis->n_shell, n_prim);
  XTC_TRY(need_ws(ar));

  std::vector<int> ints(3 * basis->n_shell + 1);
  for (int s = 0; s < basis->n_shell; ++s) {
    ints[s] = basis->shell_center[s];
    ints[basis->n_shell + s] = basis->shell_l[s];
  }
  for (int s = 0; s <= basis->n_shell; ++s) ints[2 * basis->n_shell + s] = basis->shell_prim_start[s];
  std::vector<double> prim(2 * (size_t)n_prim);
  for (int p = 0; p < n_prim; ++p) {
    prim[p] = basis->prim_exp[p];
    prim[n_prim + p] = basis->prim_coef[p];
  }
  XTC_HIP(hipMemcpyAsync(L.atom_xyz, basis->atom_xyz, sizeof(double) * 3 * basis->n_atom,
                         hipMemcpyHostToDevice, st));
  XTC_HIP(hipMemcpyAsync(L.ints, ints.data(), sizeof(int) * ints.size(), hipMemcpyHostToDevice, st));
  XTC_HIP(hipMemcpyAsync(L.prim, prim.data(), sizeof(double) * prim.size(), hipMemcpyHostToDevice, st));
  XTC_HIP(hipMemcpyAsync(L.comp, basis->comp_factor, sizeof(double) * n_ao, hipMemcpyHostToDevice, st));
  XTC_HIP(hipStreamSynchronize(st));   // host staging vectors end with this call
  BasisDev b{L.atom_xyz, L.ints, L.ints + basis->n_shell, L.ints + 2 * basis->n_shell,
             L.prim, L.prim + n_prim, L.comp, basis->n_shell, n_ao};
  const long n_g = grid->n_g;
  size_t tk = timing_begin(TM_ORBITALS, st);
  for (long g0 = 0; g0 < n_g; g0 += L.chunk) {
    long cn = (n_g - g0) < L.chunk ? (n_g - g0) : L.chunk;
    hipLaunchKernelGGL(k_eval_ao, dim3(cdiv(cn, 256)), dim3(256), 0, st, b, grid->xyz, n_g, g0,
                       L.chunk, L.ao4);
    XTC_CHECK_LAUNCH();
    for (int c = 0; c < 4; ++c) {
      GemmArgs g{};
      g.M = n_orb; g.N = cn; g.K = n_ao;
      g.A = C_mo; g.a_sm = 1; g.a_sk = n_orb;
      g.B = L.ao4 + (long)c * n_ao * L.chunk; g.b_sk = L.chunk; g.b_sn = 1;
      g.s = nullptr;
      g.C = phi4 + (long)c * n_orb * n_g + g0; g.c_sm = n_g; g.c_sn = 1;
      XTC_TRY(gemm_f64(g, st));
    }
  }
  if (rho) {
    hipLaunchKernelGGL(k_density, dim3(cdiv(n_g, 256)), dim3(256), 0, st, phi4, n_g, n_occ, rho);
    XTC_CHECK_LAUNCH();
  }
  timing_end(tk, st);
  return XTC_OK;
}
