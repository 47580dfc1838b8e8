// Complex GEMM on gfx950 matrix cores (v_mfma_f64_16x16x4_f64 /
// v_mfma_f32_16x16x4_f32).
//
// The phase sums of Eqs. (9) and (10) are dense complex contractions, so they
// run here.  A complex product is four real MFMAs on planar (re, im) tiles:
//   Cr += Ar Br - Ai Bi,  Ci += Ar Bi + Ai Br
// with the sign folded into a negated copy of Ai held in a register.
//
// Tiling: a workgroup of WM x WN waves owns a BM x BN tile of C; each wave
// owns a (BM/WM) x (BN/WN) sub-tile made of 16x16 MFMA blocks.  K advances
// in BK-wide slabs staged through LDS as [k][m] / [k][n] planes, so the lane
// reads of every MFMA (16 consecutive m or n per k row) are conflict-free.
// Global loads of the next slab are issued into registers before the MFMAs of
// the current one (single LDS buffer, register prefetch).
//
// Workgroup order: hardware hands workgroups to the 8 XCDs round-robin, each
// XCD with its own L2.  The tile index is remapped so that consecutive tiles
// land on one XCD, then grouped GROUP_M tile-rows at a time so that an XCD's
// concurrent tiles share A row-panels and B column-panels in its L2.
#include "gemm.h"

namespace ephw {
namespace {

template <typename T>
struct Mfma;
// Both instructions take A[i][k] from lane i + 16 k and B[k][j] from lane
// j + 16 k.  They differ in where the 16x16 result lands: the f32 form gives
// lane group g = lane/16 the four consecutive rows 4g..4g+3 (register v holds
// row 4g + v), the f64 form gives it rows g, g+4, g+8, g+12 (row g + 4v).
template <>
struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
};
template <>
struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
};

constexpr int kGroupM = 8;
constexpr int kXcds = 8;

// bijection on [0, n): workgroup id -> logical tile, consecutive logical tiles on one XCD
__device__ __forceinline__ int64_t xcd_remap(int64_t id, int64_t n) {
  const int64_t xcd = id % kXcds, local = id / kXcds;
  const int64_t q = n / kXcds, r = n % kXcds;
  return (xcd < r) ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

template <typename T, int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, bool SPLIT>
__global__ void __launch_bounds__(64 * WM * WN)
    cgemm_kernel(GemmParams p, int64_t tiles_m, int64_t tiles_n) {
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 16, FN = TN / 16;
  constexpr int PAD = (sizeof(T) == 4) ? 4 : 2;
  constexpr int NA = SPLIT ? 4 : 2;
  constexpr int AE = BM * BK / NT, BE = BK * BN / NT;
  static_assert(BM * BK % NT == 0 && BK * BN % NT == 0, "tile not divisible by threads");
  static_assert(TM % 16 == 0 && TN % 16 == 0 && BK % 4 == 0, "bad tile");
  using V4 = typename Mfma<T>::v4;

  __shared__ T As[NA][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

  // --- tile coordinates ---------------------------------------------------
  const int64_t ntiles = tiles_m * tiles_n;
  const int64_t logical = xcd_remap(blockIdx.x, ntiles);
  const int64_t per_group = (int64_t)kGroupM * tiles_n;
  const int64_t group = logical / per_group;
  const int64_t first_m = group * kGroupM;
  const int64_t gsize = (tiles_m - first_m) < kGroupM ? (tiles_m - first_m) : kGroupM;
  const int64_t in_group = logical % per_group;
  const int64_t tm = first_m + in_group % gsize;
  const int64_t tn = in_group / gsize;
  const int64_t m0 = tm * BM, n0 = tn * BN;

  const int64_t b = p.batch_base + blockIdx.y;
  const T* A = static_cast<const T*>(p.A) + 2 * (p.offA ? p.offA[b] : b * p.strideA);
  const T* Alo = SPLIT ? static_cast<const T*>(p.A_lo) + 2 * (p.offA ? p.offA[b] : b * p.strideA)
                       : nullptr;
  const T* B = static_cast<const T*>(p.B) + 2 * (p.offB ? p.offB[b] : b * p.strideB);
  T* C = static_cast<T*>(p.C) + 2 * (p.offC ? p.offC[b] : b * p.strideC);
  const int64_t M = p.M, N = p.N, K = p.K;
  const T sa = p.conjA ? T(-1) : T(1);
  const T sb = p.conjB ? T(-1) : T(1);

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;

  // --- register staging -----------------------------------------------------
  T ra[AE][2], rb[BE][2], rl[SPLIT ? AE : 1][2];

  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      const int e = tid + i * NT;
      int mm, kk;
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      T re = 0, im = 0, lre = 0, lim = 0;
      if (gm < M && gk < K) {
        const int64_t off = TA ? gk * p.lda + gm : gm * p.lda + gk;
        re = A[2 * off];
        im = A[2 * off + 1];
        if (SPLIT) { lre = Alo[2 * off]; lim = Alo[2 * off + 1]; }
      }
      ra[i][0] = re;
      ra[i][1] = im;
      if (SPLIT) { rl[i][0] = lre; rl[i][1] = lim; }
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      const int e = tid + i * NT;
      int nn, kk;
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }
      const int64_t gn = n0 + nn, gk = k0 + kk;
      T re = 0, im = 0;
      if (gn < N && gk < K) {
        const int64_t off = TB ? gn * p.ldb + gk : gk * p.ldb + gn;
        re = B[2 * off];
        im = B[2 * off + 1];
      }
      rb[i][0] = re;
      rb[i][1] = im;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      const int e = tid + i * NT;
      int mm, kk;
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }
      As[0][kk][mm] = ra[i][0];
      As[1][kk][mm] = sa * ra[i][1];
      if (SPLIT) { As[2][kk][mm] = rl[i][0]; As[3][kk][mm] = sa * rl[i][1]; }
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      const int e = tid + i * NT;
      int nn, kk;
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }
      Bs[0][kk][nn] = rb[i][0];
      Bs[1][kk][nn] = sb * rb[i][1];
    }
  };

  V4 acc_r[FM][FN], acc_i[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      acc_r[i][j] = V4{0, 0, 0, 0};
      acc_i[i][j] = V4{0, 0, 0, 0};
    }

  const int lrow = lane >> 4;   // k row inside one MFMA (0..3)
  const int lcol = lane & 15;   // m (A) or n (B) inside one 16-block

  load(0);
  stash();
  __syncthreads();
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + lrow;
      T ar[FM], ai[FM], nai[FM], br[FN], bi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ar[i] = As[0][kr][wm * TM + i * 16 + lcol];
        ai[i] = As[1][kr][wm * TM + i * 16 + lcol];
        nai[i] = -ai[i];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        br[j] = Bs[0][kr][wn * TN + j * 16 + lcol];
        bi[j] = Bs[1][kr][wn * TN + j * 16 + lcol];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc_r[i][j] = Mfma<T>::op(ar[i], br[j], acc_r[i][j]);
          acc_r[i][j] = Mfma<T>::op(nai[i], bi[j], acc_r[i][j]);
          acc_i[i][j] = Mfma<T>::op(ar[i], bi[j], acc_i[i][j]);
          acc_i[i][j] = Mfma<T>::op(ai[i], br[j], acc_i[i][j]);
        }
      if (SPLIT) {
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          ar[i] = As[2][kr][wm * TM + i * 16 + lcol];
          ai[i] = As[3][kr][wm * TM + i * 16 + lcol];
          nai[i] = -ai[i];
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            acc_r[i][j] = Mfma<T>::op(ar[i], br[j], acc_r[i][j]);
            acc_r[i][j] = Mfma<T>::op(nai[i], bi[j], acc_r[i][j]);
            acc_i[i][j] = Mfma<T>::op(ar[i], bi[j], acc_i[i][j]);
            acc_i[i][j] = Mfma<T>::op(ai[i], br[j], acc_i[i][j]);
          }
      }
    }
    __syncthreads();
    if (more) {
      stash();
      __syncthreads();
    }
  }

  // --- epilogue: lane holds column lcol of every block, rows per Mfma<T>::row --
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      const int64_t col = n0 + wn * TN + j * 16 + lcol;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * TM + i * 16 + Mfma<T>::row(lrow, v);
        if (row < M && col < N) {
          T* c = C + 2 * (row * p.ldc + col);
          T re = acc_r[i][j][v], im = acc_i[i][j][v];
          if (p.accumulate) { re += c[0]; im += c[1]; }
          c[0] = re;
          c[1] = im;
        }
      }
    }
}

template <typename T, int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, bool SPLIT>
ephw_status launch(const GemmParams& p0, hipStream_t stream) {
  const int64_t tiles_m = ceil_div(p0.M, BM), tiles_n = ceil_div(p0.N, BN);
  const int64_t ntiles = tiles_m * tiles_n;
  if (ntiles > 0x7fffffff) {
    set_error("cgemm: too many tiles");
    return EPHW_EUNSUPPORTED;
  }
  GemmParams p = p0;
  for (int64_t b0 = 0; b0 < p0.batch; b0 += 65535) {
    const int64_t nb = (p0.batch - b0) < 65535 ? (p0.batch - b0) : 65535;
    p.batch_base = b0;
    hipLaunchKernelGGL((cgemm_kernel<T, BM, BN, BK, WM, WN, TA, TB, SPLIT>),
                       dim3((unsigned)ntiles, (unsigned)nb), dim3(64 * WM * WN), 0, stream, p,
                       tiles_m, tiles_n);
    EPHW_CHECK_LAUNCH();
  }
  return EPHW_OK;
}

template <typename T, int BM, int BN, int BK, int WM, int WN, bool SPLIT>
ephw_status dispatch_trans(const GemmParams& p, hipStream_t s) {
  if (!p.transA && !p.transB) return launch<T, BM, BN, BK, WM, WN, false, false, SPLIT>(p, s);
  if (p.transA && !p.transB) return launch<T, BM, BN, BK, WM, WN, true, false, SPLIT>(p, s);
  if (!p.transA && p.transB) return launch<T, BM, BN, BK, WM, WN, false, true, SPLIT>(p, s);
  return launch<T, BM, BN, BK, WM, WN, true, true, SPLIT>(p, s);
}

}  // namespace

ephw_status cgemm(int prec, const GemmParams& p, hipStream_t stream) {
  if (p.M <= 0 || p.N <= 0 || p.batch <= 0) return EPHW_OK;
  if (p.K <= 0) {
    set_error("cgemm: K must be positive");
    return EPHW_EINVAL;
  }
  if (prec == 0) {
    if (p.A_lo) {
      set_error("cgemm: split A is an FP32 feature");
      return EPHW_EINVAL;
    }
    return dispatch_trans<double, 128, 64, 16, 2, 2, false>(p, stream);
  }
  if (p.A_lo) return dispatch_trans<float, 128, 128, 16, 2, 2, true>(p, stream);
  return dispatch_trans<float, 128, 128, 16, 2, 2, false>(p, stream);
}

}  // namespace ephw
