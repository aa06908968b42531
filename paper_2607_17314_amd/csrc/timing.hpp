// Internal hooks of xtc_timing (see include/isdf_xtc.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace xtc {
enum { TM_STAGE1 = 0, TM_STAGE2 = 1, TM_SELECT = 2, TM_FIT = 3, TM_ORBITALS = 4, TM_GRAD = 5,
       TM_MLP = 6, TM_SPLIT_PREP = 7, TM_S1_KERNEL = 8, TM_X_PAIRS = 9,
       TM_X_GEMM = 10, TM_X_STAGE1 = 11, TM_X_MFMA = 12,
       TM_ASM_PANEL = 13, TM_VMC_SAMPLE = 14, TM_VMC_ENERGY = 15, TM_VMC_GN = 16,
       TM_S1_PAIRS = 17 };
size_t timing_begin(int cat, hipStream_t st);
void timing_end(size_t tok, hipStream_t st);
}  // namespace xtc
