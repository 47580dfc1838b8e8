// Complex GEMM on CDNA4 matrix cores: C[b] (=|+=) op(A[b]) * op(B[b]).
#pragma once

#include "common.h"

namespace ephw {

// All sizes, leading dimensions, strides and offsets count complex elements.
// Operands are interleaved complex (T re, T im), T = double (prec 0) or float
// (prec 1).  "trans" means the operand is stored transposed (A as [K][M],
// B as [N][K]); "conj" conjugates it on load.  Batch b uses
//   A + (offA ? offA[b] : b * strideA), likewise for B and C.
struct GemmParams {
  int64_t M = 0, N = 0, K = 0, batch = 1;
  const void* A = nullptr;
  int64_t lda = 0, strideA = 0;
  const int64_t* offA = nullptr;
  const void* A_lo = nullptr;  // FP32 only: low part of a split A (same layout)
  const void* B = nullptr;
  int64_t ldb = 0, strideB = 0;
  const int64_t* offB = nullptr;
  void* C = nullptr;
  int64_t ldc = 0, strideC = 0;
  const int64_t* offC = nullptr;
  bool transA = false, conjA = false, transB = false, conjB = false;
  bool accumulate = false;
  int64_t batch_base = 0;  // internal: first batch index of this launch
};

// prec: 0 = complex128 on FP64 MFMA, 1 = complex64 on FP32 MFMA
ephw_status cgemm(int prec, const GemmParams& p, hipStream_t stream);

// Many independent GEMMs C = A B (row-major, no transposes) in one persistent
// launch: `grid` workgroups stride over the concatenated tile lists.  Each
// problem picks its tile shape with `cfg` (0 = large, 1 = small).
struct GroupProblem {
  int64_t M = 0, N = 0, K = 0;
  const void* A = nullptr;
  int64_t lda = 0;
  const void* B = nullptr;
  int64_t ldb = 0;
  void* C = nullptr;
  int64_t ldc = 0;
  int32_t cfg = 0;
  int64_t tiles_m = 0, tiles_n = 0, tile_base = 0;  // set by cgemm_grouped_layout
};
void cgemm_tile_shape(int prec, int cfg, int* bm, int* bn);
// fills tiles_m/tiles_n/tile_base of every problem; returns the total tile count
int64_t cgemm_grouped_layout(int prec, GroupProblem* probs, int n);
ephw_status cgemm_grouped(int prec, const GroupProblem* d_probs, int n, int64_t total_tiles, int grid,
                          hipStream_t stream);

}  // namespace ephw
