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

// One GEMM problem as seen by a tile: operand pointers already offset to the
// batch entry, sizes and leading dimensions in complex elements.
template <typename T>
struct TileJob {
  const T* A;
  const T* Alo;
  const T* B;
  T* C;
  int64_t M, N, K, lda, ldb, ldc;
  T sa, sb;          // -1 conjugates the operand's imaginary part
  bool accumulate;
  LossEpilogue loss;          // loss.on false: plain store
  int64_t batch;              // batch index (for the loss epilogue)
  int64_t tile, ntiles;       // tile index within the batch entry, tiles per entry
};

__device__ __forceinline__ double splitmix_weight(uint64_t seed, uint64_t index) {
  // SplitMix64 (Steele, Lea & Flood 2014): index-th output for `seed`
  uint64_t z = seed + (index + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return 0.5 + (double)(z >> 40) * 0x1p-24;
}

template <typename T, int BM, int BN, int BK, int WM, int WN, bool SPLIT>
struct TileShape {
  static constexpr int NT = 64 * WM * WN;
  static constexpr int PAD = (sizeof(T) == 4) ? 4 : 2;
  static constexpr int NA = SPLIT ? 4 : 2;
  static constexpr size_t a_elems = (size_t)NA * BK * (BM + PAD);
  static constexpr size_t b_elems = (size_t)2 * BK * (BN + PAD);
  static constexpr size_t smem_elems = a_elems + b_elems;
};

// Computes the BM x BN tile at (m0, n0) of job j with the workgroup's
// NT threads; `smem` holds TileShape::smem_elems values of T.
template <typename T, int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, bool SPLIT>
__device__ __forceinline__ void gemm_tile(const TileJob<T>& j, int64_t m0, int64_t n0, T* smem) {
  using S = TileShape<T, BM, BN, BK, WM, WN, SPLIT>;
  constexpr int NT = S::NT;
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 16, FN = TN / 16;
  constexpr int PAD = S::PAD;
  constexpr int AE = BM * BK / NT, BE = BK * BN / NT;
  constexpr int LA = BM + PAD, LB = BN + PAD;   // LDS row lengths
  static_assert(BM * BK % NT == 0 && BK * BN % NT == 0, "tile not divisible by threads");
  static_assert(TM % 16 == 0 && TN % 16 == 0 && BK % 4 == 0, "bad tile");
  using V4 = typename Mfma<T>::v4;
  // planes: As[0] re, As[1] im (conj applied), As[2]/As[3] low parts; Bs[0] re, Bs[1] im
  T* As = smem;
  T* Bs = smem + S::a_elems;
  auto AS = [&](int plane, int k, int m) -> T& { return As[(plane * BK + k) * LA + m]; };
  auto BS = [&](int plane, int k, int n) -> T& { return Bs[(plane * BK + k) * LB + n]; };

  const T* A = j.A;
  const T* Alo = j.Alo;
  const T* B = j.B;
  const int64_t M = j.M, N = j.N, K = j.K;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;

  T ra[AE][2], rb[BE][2], rl[SPLIT ? AE : 1][2];

  // Branch-free loads: an out-of-range element reads element 0 (always
  // valid) and is then replaced by zero, so the loop body is straight-line.
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      const int e = tid + i * NT;
      int mm, kk;
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }
      const int64_t gm = m0 + mm, gk = k0 + kk;
      const bool ok = gm < M && gk < K;
      const int64_t off = ok ? (TA ? gk * j.lda + gm : gm * j.lda + gk) : 0;
      const T re = A[2 * off], im = A[2 * off + 1];
      ra[i][0] = ok ? re : T(0);
      ra[i][1] = ok ? im : T(0);
      if (SPLIT) {
        const T lre = Alo[2 * off], lim = Alo[2 * off + 1];
        rl[i][0] = ok ? lre : T(0);
        rl[i][1] = ok ? lim : T(0);
      }
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      const int e = tid + i * NT;
      int nn, kk;
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }
      const int64_t gn = n0 + nn, gk = k0 + kk;
      const bool ok = gn < N && gk < K;
      const int64_t off = ok ? (TB ? gn * j.ldb + gk : gk * j.ldb + gn) : 0;
      const T re = B[2 * off], im = B[2 * off + 1];
      rb[i][0] = ok ? re : T(0);
      rb[i][1] = ok ? im : T(0);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < AE; ++i) {
      const int e = tid + i * NT;
      int mm, kk;
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }
      AS(0, kk, mm) = ra[i][0];
      AS(1, kk, mm) = j.sa * ra[i][1];
      if (SPLIT) { AS(2, kk, mm) = rl[i][0]; AS(3, kk, mm) = j.sa * rl[i][1]; }
    }
#pragma unroll
    for (int i = 0; i < BE; ++i) {
      const int e = tid + i * NT;
      int nn, kk;
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }
      BS(0, kk, nn) = rb[i][0];
      BS(1, kk, nn) = j.sb * rb[i][1];
    }
  };

  V4 acc_r[FM][FN], acc_i[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int jj = 0; jj < FN; ++jj) {
      acc_r[i][jj] = V4{0, 0, 0, 0};
      acc_i[i][jj] = V4{0, 0, 0, 0};
    }

  const int lrow = lane >> 4;   // k row inside one MFMA (0..3); also the lane group
  const int lcol = lane & 15;   // m (A) or n (B) inside one 16-block

  // One BK slab of MFMAs from LDS.  The four real products of every block are
  // issued product by product across all blocks, so consecutive MFMAs never
  // depend on each other.
  auto compute = [&]() {
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + lrow;
      T ar[FM], ai[FM], nai[FM], br[FN], bi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ar[i] = AS(0, kr, wm * TM + i * 16 + lcol);
        ai[i] = AS(1, kr, wm * TM + i * 16 + lcol);
        nai[i] = -ai[i];
      }
#pragma unroll
      for (int jj = 0; jj < FN; ++jj) {
        br[jj] = BS(0, kr, wn * TN + jj * 16 + lcol);
        bi[jj] = BS(1, kr, wn * TN + jj * 16 + lcol);
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int jj = 0; jj < FN; ++jj) acc_r[i][jj] = Mfma<T>::op(ar[i], br[jj], acc_r[i][jj]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int jj = 0; jj < FN; ++jj) acc_i[i][jj] = Mfma<T>::op(ar[i], bi[jj], acc_i[i][jj]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int jj = 0; jj < FN; ++jj) acc_r[i][jj] = Mfma<T>::op(nai[i], bi[jj], acc_r[i][jj]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int jj = 0; jj < FN; ++jj) acc_i[i][jj] = Mfma<T>::op(ai[i], br[jj], acc_i[i][jj]);
      if (SPLIT) {
#pragma unroll
        for (int i = 0; i < FM; ++i) {
          ar[i] = AS(2, kr, wm * TM + i * 16 + lcol);
          ai[i] = AS(3, kr, wm * TM + i * 16 + lcol);
          nai[i] = -ai[i];
        }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int jj = 0; jj < FN; ++jj) {
            acc_r[i][jj] = Mfma<T>::op(ar[i], br[jj], acc_r[i][jj]);
            acc_i[i][jj] = Mfma<T>::op(ar[i], bi[jj], acc_i[i][jj]);
          }
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int jj = 0; jj < FN; ++jj) {
            acc_r[i][jj] = Mfma<T>::op(nai[i], bi[jj], acc_r[i][jj]);
            acc_i[i][jj] = Mfma<T>::op(ai[i], br[jj], acc_i[i][jj]);
          }
      }
    }
  };

  // K loop: the next slab is fetched into registers while the current one is
  // multiplied; the last slab is peeled so the loop body has no branches.
  load(0);
  stash();
  __syncthreads();
  const int64_t nslab = (K + BK - 1) / BK;
  for (int64_t sl = 1; sl < nslab; ++sl) {
    load(sl * BK);
    compute();
    __syncthreads();
    stash();
    __syncthreads();
  }
  compute();

  // --- epilogue: lane holds column lcol of every block, rows per Mfma<T>::row --
  if (!j.loss.on) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int jj = 0; jj < FN; ++jj) {
        const int64_t col = n0 + wn * TN + jj * 16 + lcol;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = m0 + wm * TM + i * 16 + Mfma<T>::row(lrow, v);
          if (row < M && col < N) {
            T* c = j.C + 2 * (row * j.ldc + col);
            T re = acc_r[i][jj][v], im = acc_i[i][jj][v];
            if (j.accumulate) { re += c[0]; im += c[1]; }
            c[0] = re;
            c[1] = im;
          }
        }
      }
    return;
  }
  // weighted |c|^2: element index ((((q nk + k) nm + nu) nw + m) nw + n)
  const LossEpilogue& L = j.loss;
  const int64_t il = j.batch / ((int64_t)L.qb * L.nm);
  const int64_t iq = (j.batch / L.nm) % L.qb;
  const int64_t nu = j.batch % L.nm;
  const uint64_t base =
      (((uint64_t)(L.q0 + iq) * (uint64_t)L.nk + (uint64_t)(L.k0 + il)) * (uint64_t)L.nm + (uint64_t)nu) *
      (uint64_t)L.nw * (uint64_t)L.nw;
  double part = 0.0;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int jj = 0; jj < FN; ++jj) {
      const int64_t col = n0 + wn * TN + jj * 16 + lcol;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * TM + i * 16 + Mfma<T>::row(lrow, v);
        if (row < M && col < N) {
          const T re = acc_r[i][jj][v], im = acc_i[i][jj][v];
          const double w = splitmix_weight(L.seed, base + (uint64_t)(row * L.nw + col));
          part += w * ((double)re * (double)re + (double)im * (double)im);
          if (L.store) {
            T* c = j.C + 2 * (row * j.ldc + col);
            if (L.grad_scale) {
              c[0] = (T)(2.0 * w) * re;
              c[1] = (T)(2.0 * w) * im;
            } else {
              c[0] = re;
              c[1] = im;
            }
          }
        }
      }
    }
  // workgroup sum in a fixed order: waves through LDS (free after the K loop)
  for (int off = 32; off > 0; off >>= 1) part += __shfl_down(part, off, 64);
  double* red = reinterpret_cast<double*>(smem);
  __syncthreads();
  if (lane == 0) red[wave] = part;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int w = 0; w < WM * WN; ++w) tot += red[w];
    L.partial[j.batch * j.ntiles + j.tile] = tot;
  }
  __syncthreads();
}

// tile (tm, tn) of logical tile index t: groups of kGroupM tile-rows
__device__ __forceinline__ void tile_coords(int64_t t, int64_t tiles_m, int64_t tiles_n, int64_t* tm,
                                            int64_t* tn) {
  const int64_t per_group = (int64_t)kGroupM * tiles_n;
  const int64_t group = t / per_group;
  const int64_t first_m = group * kGroupM;
  const int64_t gsize = (tiles_m - first_m) < kGroupM ? (tiles_m - first_m) : kGroupM;
  const int64_t in_group = t % per_group;
  *tm = first_m + in_group % gsize;
  *tn = in_group / gsize;
}

template <typename T>
__device__ __forceinline__ TileJob<T> job_of(const GemmParams& p, int64_t b) {
  const int64_t i2 = b % p.n2, i1 = (b / p.n2) % p.n1, i0 = b / (p.n1 * p.n2);
  const int64_t oa = p.offA ? p.offA[b] : i0 * p.strideA + i1 * p.strideA1 + i2 * p.strideA2;
  const int64_t ob = p.offB ? p.offB[b] : i0 * p.strideB + i1 * p.strideB1 + i2 * p.strideB2;
  const int64_t oc = p.offC ? p.offC[b] : i0 * p.strideC + i1 * p.strideC1 + i2 * p.strideC2;
  TileJob<T> j;
  j.A = static_cast<const T*>(p.A) + 2 * oa;
  j.Alo = p.A_lo ? static_cast<const T*>(p.A_lo) + 2 * oa : nullptr;
  j.B = static_cast<const T*>(p.B) + 2 * ob;
  j.C = static_cast<T*>(p.C) + 2 * oc;
  j.M = p.M;
  j.N = p.N;
  j.K = p.K;
  j.lda = p.lda;
  j.ldb = p.ldb;
  j.ldc = p.ldc;
  j.sa = p.conjA ? T(-1) : T(1);
  j.sb = p.conjB ? T(-1) : T(1);
  j.accumulate = p.accumulate;
  j.loss = p.loss;
  j.batch = b;
  j.tile = 0;
  j.ntiles = 1;
  return j;
}

template <typename T, int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, bool SPLIT>
__global__ void __launch_bounds__(64 * WM * WN)
    cgemm_kernel(GemmParams p, int64_t tiles_m, int64_t tiles_n) {
  using S = TileShape<T, BM, BN, BK, WM, WN, SPLIT>;
  __shared__ T smem[S::smem_elems];
  const int64_t logical = xcd_remap(blockIdx.x, tiles_m * tiles_n);
  int64_t tm, tn;
  tile_coords(logical, tiles_m, tiles_n, &tm, &tn);
  TileJob<T> j = job_of<T>(p, p.batch_base + blockIdx.y);
  j.tile = tm * tiles_n + tn;
  j.ntiles = tiles_m * tiles_n;
  gemm_tile<T, BM, BN, BK, WM, WN, TA, TB, SPLIT>(j, tm * BM, tn * BN, smem);
}

// Tile shapes of the grouped kernel: cfg 0 is the shape of the plain kernel,
// cfg 1 a 64x64 tile for small problems.  Both use 4 waves.
template <typename T>
struct GroupCfg;
template <>
struct GroupCfg<float> {
  using L = TileShape<float, 128, 128, 16, 2, 2, false>;
  using S = TileShape<float, 64, 64, 16, 2, 2, false>;
  static constexpr int LM = 128, LN = 128;
};
template <>
struct GroupCfg<double> {
  using L = TileShape<double, 128, 64, 16, 2, 2, false>;
  using S = TileShape<double, 64, 64, 16, 2, 2, false>;
  static constexpr int LM = 128, LN = 64;
};

template <typename T>
__global__ void __launch_bounds__(256)
    cgemm_grouped_kernel(const GroupProblem* __restrict__ probs, int n, int64_t total) {
  using G = GroupCfg<T>;
  constexpr size_t kSmem = G::L::smem_elems > G::S::smem_elems ? G::L::smem_elems : G::S::smem_elems;
  __shared__ T smem[kSmem];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (probs[mid].tile_base <= t) lo = mid; else hi = mid - 1;
    }
    const GroupProblem& P = probs[lo];
    int64_t tm, tn;
    tile_coords(t - P.tile_base, P.tiles_m, P.tiles_n, &tm, &tn);
    TileJob<T> j;
    j.A = static_cast<const T*>(P.A);
    j.Alo = nullptr;
    j.B = static_cast<const T*>(P.B);
    j.C = static_cast<T*>(P.C);
    j.M = P.M;
    j.N = P.N;
    j.K = P.K;
    j.lda = P.lda;
    j.ldb = P.ldb;
    j.ldc = P.ldc;
    j.sa = T(1);
    j.sb = T(1);
    j.accumulate = false;
    j.loss = LossEpilogue();
    j.batch = 0;
    j.tile = 0;
    j.ntiles = 1;
    if (P.cfg == 0)
      gemm_tile<T, G::LM, G::LN, 16, 2, 2, false, false, false>(j, tm * G::LM, tn * G::LN, smem);
    else
      gemm_tile<T, 64, 64, 16, 2, 2, false, false, false>(j, tm * 64, tn * 64, smem);
    __syncthreads();
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

int64_t cgemm_tiles(int prec, int64_t M, int64_t N) {
  return prec == 0 ? ceil_div(M, 128) * ceil_div(N, 64) : ceil_div(M, 128) * ceil_div(N, 128);
}

void cgemm_tile_shape(int prec, int cfg, int* bm, int* bn) {
  if (cfg != 0) {
    *bm = 64;
    *bn = 64;
  } else if (prec == 0) {
    *bm = 128;
    *bn = 64;
  } else {
    *bm = 128;
    *bn = 128;
  }
}

int64_t cgemm_grouped_layout(int prec, GroupProblem* probs, int n) {
  int64_t base = 0;
  for (int i = 0; i < n; ++i) {
    int bm, bn;
    cgemm_tile_shape(prec, probs[i].cfg, &bm, &bn);
    probs[i].tiles_m = (probs[i].M > 0 && probs[i].K > 0) ? ceil_div(probs[i].M, bm) : 0;
    probs[i].tiles_n = (probs[i].N > 0 && probs[i].K > 0) ? ceil_div(probs[i].N, bn) : 0;
    probs[i].tile_base = base;
    base += probs[i].tiles_m * probs[i].tiles_n;
  }
  return base;
}

ephw_status cgemm_grouped(int prec, const GroupProblem* d_probs, int n, int64_t total_tiles, int grid,
                          hipStream_t stream) {
  if (n <= 0 || total_tiles <= 0) return EPHW_OK;
  if (grid <= 0) grid = 1;
  if (prec == 0)
    hipLaunchKernelGGL(cgemm_grouped_kernel<double>, dim3(grid), dim3(256), 0, stream, d_probs, n, total_tiles);
  else
    hipLaunchKernelGGL(cgemm_grouped_kernel<float>, dim3(grid), dim3(256), 0, stream, d_probs, n, total_tiles);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

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
