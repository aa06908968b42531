// Shared host/device helpers of libisdfxtc: status handling, workspace carving,
// launch checks. Internal header; the public ABI is include/isdf_xtc.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <math.h>
#include <string>
#include <vector>
#include "isdf_xtc.h"

namespace xtc {

void set_error(const std::string& msg);

// A failed HIP call maps to XTC_ERR_HIP with the runtime's message recorded.
#define XTC_HIP(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::xtc::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));         \
      return XTC_ERR_HIP;                                                          \
    }                                                                              \
  } while (0)

#define XTC_CHECK_LAUNCH() XTC_HIP(hipGetLastError())

#define XTC_REQUIRE(cond, msg)                                                     \
  do {                                                                             \
    if (!(cond)) {                                                                 \
      ::xtc::set_error(msg);                                                       \
      return XTC_ERR_INVALID_ARG;                                                  \
    }                                                                              \
  } while (0)

#define XTC_TRY(expr)                                                              \
  do {                                                                             \
    xtc_status s_ = (expr);                                                        \
    if (s_ < 0) return s_;                                                         \
  } while (0)

// Bump allocator over the caller's workspace; every region is 256-byte aligned.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  bool dry = false;   // size-only pass (base may be null)
  Arena(void* p, size_t n) : base((char*)p), cap(n), dry(p == nullptr) {}
  template <class T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    if (dry || used > cap) return nullptr;
    return (T*)(base + off);
  }
  bool ok() const { return !dry && used <= cap; }
};

inline xtc_status need_ws(const Arena& a) {
  if (a.used > a.cap || a.base == nullptr) {
    set_error("workspace too small: need " + std::to_string(a.used) + " bytes, have " +
              std::to_string(a.cap));
    return XTC_ERR_NO_WORKSPACE;
  }
  return XTC_OK;
}

inline unsigned cdiv(long a, long b) { return (unsigned)((a + b - 1) / b); }

inline hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// ---------------------------------------------------------------------------
// Generic FP64 GEMM (MFMA 16x16x4, tile 64x64x16):
//   C[m, n] = alpha * sn[n] * sum_k A[m, k] s[k] B[k, n]   (+ beta * D[m, n])
// then an optional epilogue: C <- C * E[m, n] (Hadamard) or C <- C * C.
// Strides are in elements; A/B may be k- or m/n-contiguous.
enum Epilogue { EPI_NONE = 0, EPI_MUL_E = 1, EPI_SQUARE = 2 };

struct GemmArgs {
  long M, N, K;
  const double* A; long a_sm, a_sk;
  const double* B; long b_sk, b_sn;
  const double* s;            // per-k scale or nullptr
  double* C; long c_sm, c_sn;
  double alpha = 1.0;
  double beta = 0.0;
  const double* D = nullptr;  // beta term source (same strides as C); nullptr -> C
  int epi = EPI_NONE;
  const double* E = nullptr; long e_sm = 0, e_sn = 0;
  bool lower_only = false;    // skip tiles strictly above the diagonal (m < n)
  const double* sn = nullptr; // per-column scale of the product: alpha * sn[n] * (A B)[m, n]
  const float* A32 = nullptr; // split GEMM only: A in FP32 (then A is nullptr)
};

xtc_status gemm_f64(const GemmArgs& g, hipStream_t st);

// Rejects quadrature weights that are negative, NaN or infinite (XTC_ERR_INVALID_ARG):
// one small kernel over grid->w with an integer flag in the first bytes of the caller's
// workspace, then a synchronisation of the stream to read the flag. Called before any
// other launch of the calls that take a grid.
xtc_status check_weights(const xtc_grid* grid, void* ws, size_t ws_bytes, hipStream_t st,
                         const char* who);

// Deterministic FP64 sum of x[0..n) (fixed two-level tree); result to *out (device).
xtc_status reduce_sum_f64(const double* x, long n, double* out, double* scratch, hipStream_t st);

// Auxiliary stream idx (0 .. AUX_STREAMS - 1) of the current device: created on first use
// with default priority and hipStreamNonBlocking (not synchronised with the legacy
// default stream), kept until the process ends; work on it is ordered with the caller's
// stream by events only.
constexpr int AUX_STREAMS = 2;
xtc_status aux_stream(int idx, hipStream_t* out);

// Events owned by one call (fork and joins), destroyed when it returns.
struct CallEvents {
  hipEvent_t ev[1 + AUX_STREAMS] = {};
  xtc_status create(int n);
  ~CallEvents();
};

}  // namespace xtc
