// Operand layout and tile sizes shared by the split-precision stage-1 kernels (the
// EE pair kernel, which generates its kernel values in registers, and the BH pair
// kernels, which read them from a buffer of pre-split pair values).
#pragma once
#include "contract.hpp"

namespace xtc {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f16x __attribute__((ext_vector_type(16)));

constexpr int SR = 256;        // rows per workgroup
constexpr int SB = 32;         // bra points per workgroup
constexpr int SKC = 128;       // ket points per chunk (8 k-steps of 16)
constexpr int SMED = 128;      // chunks per launch: FP32 medium sum, then FP64

// The split operand in the scratch (split_prepare writes it): A = w xi scaled per row by
// 2^sA and split into FP16 (hi, lo) pairs, in MFMA A-fragment order per 32-row block and
// k-step; the ket coordinates as FP32 (hi, lo) pairs.
struct SplitLayout {
  h8* A;            // [rows_pad / 32][nks][2][64]
  int* sA;          // [rows_pad] per-row exponent
  float* kc;        // [6][n_g_pad]: x_hi, y_hi, z_hi, x_lo, y_lo, z_lo
  long rows_pad;    // multiple of SR
  long n_g_pad;     // multiple of 2 SKC
  long nks;         // n_g_pad / 16
};

inline SplitLayout split_layout(void* base, long n_g, int n_mu) {
  SplitLayout S;
  S.rows_pad = ((n_mu + SR - 1) / SR) * SR;
  S.n_g_pad = ((n_g + 2 * SKC - 1) / (2 * SKC)) * (2 * SKC);   // an even number of chunks
  S.nks = S.n_g_pad / 16;
  Arena ar(base, (size_t)-1);
  S.A = ar.take<h8>((size_t)(S.rows_pad / 32) * S.nks * 2 * 64);
  S.sA = ar.take<int>(S.rows_pad);
  S.kc = ar.take<float>(6 * (size_t)S.n_g_pad);
  return S;
}

}  // namespace xtc
