// Split-precision (FP16 hi/lo on MFMA) NT GEMM used by stage 2 of the contraction
// and by the exchange intermediates.
#pragma once
#include <type_traits>
#include "common.hpp"

namespace xtc {

constexpr int SPLIT_MAXSEG = 4;

// One product of a segmented GEMM: A(m, k) = A[m a_sm + k a_sk] (k or m contiguous),
// s[k] an optional per-k scale, B(n, k) = B[n b_sn + k] (k contiguous).
struct SplitSeg {
  const double* A; long a_sm, a_sk;
  const double* s;
  const double* B; long b_sn, b_sk;
  const float* Af = nullptr;   // A in FP32 instead (then A is nullptr)
};

// C (+)= sum_seg A_seg diag(s_seg) B_seg^T over nseg (1..4) segments of K each, one
// MFMA launch with one FP32 medium sum over the concatenated k range; C row-major
// with row stride ldc. scratch: gemm_split_seg_scratch_bytes(M, N, K, nseg) bytes.
// eA: nullptr, or the A row scales already known (device, M rounded up to 128 entries:
// max_k |A(m, k) s(k)| 2^eA[m] in [2^14, 2^15), 0 for zero and padding rows).
xtc_status gemm_split_seg(long M, long N, long K, const SplitSeg* seg, int nseg, double* C,
                          long ldc, bool accumulate, void* scratch, size_t bytes, hipStream_t st,
                          const int* eA = nullptr, int timing_category = -1);
size_t gemm_split_seg_scratch_bytes(long M, long N, long K, int nseg);

// C = A diag(s) B^T (beta 0) or C += A diag(s) B^T (beta 1); A [M][K] with k or m
// contiguous, B [N][K] (b_sk 1, row stride b_sn), C row-major (c_sn 1, stride c_sm).
// scratch: gemm_split_scratch_bytes(M, N, K) bytes of device memory.
xtc_status gemm_split_nt(const GemmArgs& g, void* scratch, size_t bytes, hipStream_t st);
size_t gemm_split_scratch_bytes(long M, long N, long K);

}  // namespace xtc
