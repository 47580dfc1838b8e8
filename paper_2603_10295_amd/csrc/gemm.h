// Complex GEMM on CDNA4 matrix cores: C[b] (=|+=) op(A[b]) * op(B[b]).
#pragma once

#include "common.h"

namespace ephw {

// Weighted |C|^2 epilogue for the loss L = sum w |g|^2 (SplitMix64 weights).
// layout 0: batch b is (il, iq, nu) = (b / (qb nm), (b / nm) % qb, b % nm)
// (k point k0 + il, q point q0 + iq, mode nu) and C's row m and column n are
// band indices.  layout 1: batch b is the pair (il, iq) = (b / qb, b % qb),
// row r of C is (nu, n) = (r / nw, r % nw) and column m is the other band.
// Every workgroup writes the sum of w |c|^2 over its tile to
// partial[b * tiles_per_batch + tile].  With grad_scale the stored value is
// 2 w c (the gradient of L with respect to g) instead of c.
struct LossEpilogue {
  bool on = false;
  bool store = true;        // also store C (plain or scaled)
  bool grad_scale = false;
  int layout = 0;
  uint64_t seed = 0;
  int64_t nk = 0;           // size of the k set (element index stride)
  int nm = 0, nw = 0, qb = 0;
  int64_t q0 = 0, k0 = 0;
  double* partial = nullptr;
};

// Band rotations fused into the epilogue of the Eq. (10) Re-sum GEMM (FP32,
// 128x128 tiles, no transposes, Nw of 4 or 8 so that every Nw x Nw block of a
// (q, nu) lies inside one wave's 64 columns).  C = W[k][(q, nu, m', n')] with
// row r the k point r of the set and column c = (q, nu, m', n') of the batch;
// instead of storing W the tile forms g_nu(k,q) = V(k+q)^dagger W_nu V(k)
// (Eq. (7)'s band factors, U = V^dagger) and applies the epilogues:
//   EPHW_OUT_G        g stored [q][k][nu][m][n]
//   EPHW_OUT_BAND_SUM T_nu = sum_mn |g|^2 stored [q][k][nu]
//   EPHW_OUT_LOSS     sum of w |g|^2 over the tile -> loss_partial[tile]
//   lw_partial        linewidth terms of every element (the weights of
//                     ephw_linewidth) summed over the (q, nu, m) of a column
//                     group -> lw_partial[group][k][n], cgemm_band_lw_groups
//                     groups of 64 or 128 columns
struct BandEpilogue {
  bool on = false;
  int nw = 0, nm = 0;
  int64_t nk = 0;                 // k points of the set (rows of C; stride of kq_index, g_out, band_sum)
  int64_t q_global0 = 0;          // position of the batch's first q in the caller's list (loss index)
  const void* Vk = nullptr;       // [nk][nw][nw] c64, eigenvector columns V(k)
  const void* Vkq = nullptr;      // [qb][nk][nw][nw] c64 V(k+q), or NULL: taken through kq_index
  const int32_t* kq_index = nullptr;  // [qb][nk], offset to the batch
  uint32_t flags = 0;             // EPHW_OUT_G / EPHW_OUT_BAND_SUM / EPHW_OUT_LOSS
  void* g_out = nullptr;          // [qb][nk][nm][nw][nw] c64, offset to the batch
  double* band_sum = nullptr;     // [qb][nk][nm], offset to the batch
  double* loss_partial = nullptr; // [tiles of the launch]
  uint64_t loss_seed = 0;
  double* lw_partial = nullptr;   // [groups][nk][nw], or NULL: no linewidth terms
  const double* eps_k = nullptr;  // [nk][nw]
  const double* eps_kq = nullptr; // [qb][nk][nw]
  const double* omega = nullptr;  // [qb][nm]
  LwParams lw;
  uint32_t* status = nullptr;     // kStatusIndex for an index outside [0, nk)
};

// All sizes, leading dimensions, strides and offsets count complex elements.
// Operands are interleaved complex (T re, T im), T = double (prec 0) or float
// (prec 1).  "trans" means the operand is stored transposed (A as [K][M],
// B as [N][K]); "conj" conjugates it on load.  Batch b is decomposed as
// b = (i0 * n1 + i1) * n2 + i2 and uses
//   A + (offA ? offA[b] : i0 * strideA + i1 * strideA1 + i2 * strideA2),
// likewise for B and C (n1 = n2 = 1 gives the plain stride b * strideA).
struct GemmParams {
  int64_t M = 0, N = 0, K = 0, batch = 1;
  const void* A = nullptr;
  int64_t lda = 0, strideA = 0;
  const int64_t* offA = nullptr;
  const void* B = nullptr;
  int64_t ldb = 0, strideB = 0;
  const int64_t* offB = nullptr;
  void* C = nullptr;
  int64_t ldc = 0, strideC = 0;
  const int64_t* offC = nullptr;
  bool transA = false, conjA = false, transB = false, conjB = false;
  bool accumulate = false;
  // FP32 only: K-blocked accumulation (fresh accumulators every 32 k, block
  // sums added in FP32), the compensated form of EPHW_FP32_COMP
  bool compensated = false;
  int64_t n1 = 1, n2 = 1;
  int64_t strideA1 = 0, strideA2 = 0, strideB1 = 0, strideB2 = 0, strideC1 = 0, strideC2 = 0;
  // tblock > 0: C is stored in blocks of tblock rows, each block transposed:
  // element (r, c) goes to (r / tblock) * ldc + c * tblock + r % tblock
  // (ldc is then the block stride).
  int64_t tblock = 0;
  LossEpilogue loss;
  BandEpilogue band;
  int64_t batch_base = 0;  // internal: first batch index of this launch
};
// whether cgemm can run the fused band epilogue for this Re-sum shape (FP32,
// nw 4 or 8; always on 128x128 tiles, ceil(M/128) * ceil(N/128) of them);
// otherwise the caller stores W and rotates
bool cgemm_band_fusable(int prec, int64_t M, int64_t N, int nw, int64_t lda, int64_t ldb);
// column groups of the fused epilogue's linewidth partials for N columns
int64_t cgemm_band_lw_groups(int nw, int nm, int64_t N);
// workgroup tiles per batch entry of a GEMM (size of the loss partial block)
int64_t cgemm_tiles(int prec, int64_t M, int64_t N);

// prec: 0 = complex128 on FP64 MFMA, 1 = complex64 on FP32 MFMA
ephw_status cgemm(int prec, const GemmParams& p, hipStream_t stream);

// Many independent GEMMs C = A B (row-major, no transposes) in one persistent
// launch: `grid` workgroups take tiles of the concatenated tile lists from a
// work queue (per-XCD ranges, then the others).  All
// problems of one launch share a tile configuration `cfg` (0 = large,
// 1 = small 64x64).
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
  int32_t flat = 0;   // set by cgemm_grouped_layout: both operands' extents fit 32-bit byte offsets
};
void cgemm_tile_shape(int prec, int cfg, int* bm, int* bn);
// workgroups of the grouped kernel one CU holds at once (its persistent grid
// is this times the CU count)
int cgemm_grouped_blocks_per_cu(int prec, int cfg);
// whether the grouped kernel can address operands with these leading dimensions
bool cgemm_grouped_fits(int prec, int64_t lda, int64_t ldb);
// fills tiles_m/tiles_n/tile_base of every problem; returns the total tile count
int64_t cgemm_grouped_layout(int prec, GroupProblem* probs, int n);
// `queue` points at kGroupQueues ints that must be zero when the launch
// starts (cgemm_grouped_reset zeroes many with one kernel, so a captured graph
// holds no memset node); the launch leaves them nonzero.
constexpr int kGroupQueues = 8;
ephw_status cgemm_grouped(int prec, int cfg, const GroupProblem* d_probs, int n, int64_t total_tiles, int grid,
                          int* queue, hipStream_t stream);
ephw_status cgemm_grouped_reset(int* queues, int count, hipStream_t stream);

}  // namespace ephw
