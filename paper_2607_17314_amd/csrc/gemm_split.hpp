// Split-precision (FP16 hi/lo on MFMA) NT GEMM used by stage 2 of the contraction.
#pragma once
#include <type_traits>
#include "common.hpp"

namespace xtc {

// C = A diag(s) B^T (beta 0) or C += A diag(s) B^T (beta 1); A [M][K] (a_sk 1, row
// stride a_sm), B [N][K] (b_sk 1, row stride b_sn), C row-major (c_sn 1, stride c_sm).
// scratch: gemm_split_scratch_bytes(M, N, K) bytes of device memory.
xtc_status gemm_split_nt(const GemmArgs& g, void* scratch, size_t bytes, hipStream_t st);
size_t gemm_split_scratch_bytes(long M, long N, long K);

}  // namespace xtc
