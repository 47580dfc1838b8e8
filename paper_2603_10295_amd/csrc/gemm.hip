// Complex GEMM on gfx950 matrix cores (v_mfma_f64_16x16x4_f64 /
// v_mfma_f32_16x16x4_f32).
//
// The phase sums of Eqs. (9) and (10) are dense complex contractions, so they
// run here.  A complex product is four real MFMAs on the (re, im) parts:
//   Cr += Ar Br - Ai Bi,  Ci += Ar Bi + Ai Br
// with the sign folded into a negated copy of Ai held in a register.
//
// Tiling: a workgroup of WM x WN waves owns a BM x BN tile of C; each wave
// owns a (BM/WM) x (BN/WN) sub-tile made of 16x16 MFMA blocks.  K advances
// in BK-deep slabs: 16-byte buffer loads bring slab s+1 into registers while
// slab s is multiplied out of one of two LDS stages, then the registers are
// written to the other stage (one barrier per slab).  LDS holds complex
// values interleaved, [k][m] and [k][n], so each MFMA operand pair is one
// 8- or 16-byte read and the 16 lanes of a row read consecutive addresses.
// FP32: 128x128x16 tiles at two waves per SIMD (register budget 256);
// FP64: 64x64x8 tiles; outputs 129..224 wide use 64x224 tiles.
//
// Workgroup order: hardware hands workgroups to the 8 XCDs round-robin, each
// XCD with its own L2.  The tile index is remapped so that consecutive tiles
// land on one XCD, then grouped GROUP_M tile-rows at a time so that an XCD's
// concurrent tiles share A row-panels and B column-panels in its L2.
#include "gemm.h"
#include "mfma.h"

namespace ephw {
namespace {

constexpr int kGroupM = 8;
constexpr int kXcds = 8;
static_assert(kGroupQueues == kXcds, "one grouped-GEMM work queue per XCD");

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
  const T* B;
  T* C;
  int64_t M, N, K, lda, ldb, ldc;
  T sa, sb;          // -1 conjugates the operand's imaginary part
  bool accumulate;
  int64_t tblock;             // > 0: block-transposed C (see GemmParams)
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

// 16-byte global chunks: two complex floats or one complex double.
template <typename T>
struct Chunk;
template <>
struct Chunk<float> {
  static constexpr int CPC = 2;   // complex values per chunk
  typedef float v4 __attribute__((ext_vector_type(4)));
  typedef float v2 __attribute__((ext_vector_type(2)));
};
template <>
struct Chunk<double> {
  static constexpr int CPC = 1;
  typedef double v4 __attribute__((ext_vector_type(2)));
  typedef double v2 __attribute__((ext_vector_type(2)));
};

// Buffer resource over `bytes` bytes from `base` (clamped to the 32-bit
// range field).  Loads past the end return zero, which pads the M, N and
// (for the operand whose rows run along K) K tails of a tile for free.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  const uint64_t p = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)p);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(p >> 32));
  uint32_t n = bytes <= 0 ? 0u : (bytes >= 0xffffffffll ? 0xffffffffu : (uint32_t)bytes);
  n = __builtin_amdgcn_readfirstlane(n);
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo), (short)0, (int)n,
                                           0x00020000);
}

template <typename T>
__device__ __forceinline__ typename Chunk<T>::v4 load_chunk(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(typename Chunk<T>::v4, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
}

template <int N>
struct IntC {
  static constexpr int value = N;
};

template <typename T, int BM, int BN, int BK, int WM, int WN>
struct TileShape {
  static constexpr int NT = 64 * WM * WN;
  static constexpr int PADC = (sizeof(T) == 4) ? 2 : 1;  // complex values of padding per LDS row
  static constexpr int LA = BM + PADC, LB = BN + PADC;
  // one pipeline stage: an A slab [BK][LA] and a B slab [BK][LB], complex T
  static constexpr size_t stage_elems = (size_t)2 * BK * (LA + LB);
  static constexpr size_t smem_elems = 2 * stage_elems;   // two stages
};

// Fused band rotation of the FP32 128x128 Re-sum tile (see BandEpilogue).
// Wave (wm, wn) holds W for 64 k points (rows) and 64 columns, i.e. 64/Nw^2
// whole (q, nu) blocks of Nw x Nw.  Its rows go through LDS in two halves of
// 32 k points (the wave's own 32 x 65 complex region; the K loop's stages are
// free by then).  Two lanes share a k point and split its 64/Nw rows (b, m')
// into four-row groups: Nw = 8, one block, rows 4s..4s+3; Nw = 4, blocks
// 2s, 2s+1, all four rows (s = lane parity).  Per half:
//   1. T_b[m'][:] = W_b[m'][:] V(k) for the lane's rows, written over them in
//      LDS; V(k) is read once per half, row by row (both lanes of the k point
//      read the same rows);
//   2. after a wave-level wait, g_b[m][:] = sum_m' conj(V(k+q_b)[m'][m]) T_b[m'][:]
//      for the lane's output rows (the same four-row groups), T_b rows from
//      LDS and V(k+q_b) rows (the lane's four columns) from global memory;
//   3. the epilogues of the lane's rows: g stored (four contiguous rows),
//      |g|^2 of a block summed over its lanes (band sum), w |g|^2 into the
//      lane's loss sum, linewidth weights times |g|^2 summed per band n over
//      the k point's rows and stored per wave column.
// Sums run in a fixed order (shuffles and a fixed wave order), so the results
// are deterministic.
template <int NW>
__device__ __forceinline__ void band_epilogue(const TileJob<float>& j, const BandEpilogue& B, int64_t m0, int64_t n0,
                                              typename Mfma<float>::v4 (&acc_r)[4][4],
                                              typename Mfma<float>::v4 (&acc_i)[4][4], float* smem) {
  static_assert(NW == 4 || NW == 8, "four-row groups of whole blocks");
  constexpr int TM = 64, TN = 64, HR = 32, LDW = TN + 1;
  constexpr int NW2 = NW * NW, NB = 8 / NW, MR = 4;   // blocks per lane, rows per block group
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % 2, wn = wave / 2;
  const int lrow = lane >> 4, lcol = lane & 15;
  float* wl = smem + wave * (HR * LDW * 2);
  const int kl = lane >> 1, sb = lane & 1;               // k point within the half, lane of the pair
  const int64_t cw0 = n0 + wn * TN;                      // first column of the wave
  const int64_t E = (int64_t)B.nm * NW2;
  const bool want_g = (B.flags & EPHW_OUT_G) != 0, want_t = (B.flags & EPHW_OUT_BAND_SUM) != 0;
  const bool want_l = (B.flags & EPHW_OUT_LOSS) != 0, want_w = B.lw_partial != nullptr;
  const float* Vk = static_cast<const float*>(B.Vk);
  const float* Vkq = static_cast<const float*>(B.Vkq);
  // the lane's blocks: column offset in the wave, first row, (q, nu), validity
  int bcol[NB], brow0[NB], bnu[NB];
  int64_t bq[NB];
  bool bok[NB];
  double bom[NB], bnb[NB];
  bool blw[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int blk = NW == 8 ? 0 : 2 * sb + i;
    brow0[i] = NW == 8 ? MR * sb : 0;
    bcol[i] = blk * NW2;
    const int64_t c0 = cw0 + bcol[i];
    bok[i] = c0 < j.N;
    bq[i] = bok[i] ? c0 / E : 0;
    bnu[i] = bok[i] ? (int)((c0 - bq[i] * E) / NW2) : 0;
    bom[i] = 0.0;
    bnb[i] = 0.0;
    blw[i] = false;
    if (want_w && bok[i]) {
      bom[i] = B.omega[bq[i] * B.nm + bnu[i]];
      blw[i] = bom[i] > 0.0 && bom[i] >= B.lw.omega_min;   // omega = 0: no zero-point amplitude
      if (blw[i]) bnb[i] = 1.0 / expm1(bom[i] * B.lw.inv_t);
    }
  }
  double lsum = 0.0;
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    if (h == 0)
      __syncthreads();   // every wave is done with the K loop's LDS stages
    else
      wave_sync();       // this wave is done with the first half's rows
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = ii * 16 + Mfma<float>::row(lrow, v), col = jj * 16 + lcol;
          const float re = h == 0 ? acc_r[ii][jj][v] : acc_r[2 + ii][jj][v];
          const float im = h == 0 ? acc_i[ii][jj][v] : acc_i[2 + ii][jj][v];
          *reinterpret_cast<float2*>(wl + 2 * (row * LDW + col)) = make_float2(re, im);
        }
    wave_sync();
    const int64_t k = m0 + wm * TM + h * HR + kl;
    const bool kok = k < j.M;
    float* krow = wl + 2 * (kl * LDW);
    // V(k+q_b) of the lane's blocks: the index is read now, ahead of its use
    const float* vqb[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      if (Vkq) {
        vqb[i] = Vkq + 2 * ((bq[i] * B.nk + (kok ? k : 0)) * NW2);
      } else {
        int64_t id = (kok && bok[i]) ? B.kq_index[bq[i] * B.nk + k] : 0;
        if (id < 0 || id >= B.nk) {
          atomicOr(B.status, kStatusIndex);
          id = 0;
        }
        vqb[i] = Vk + 2 * id * NW2;
      }
    }
    // 1. T = W V(k) for the lane's rows (b, m'), written over them
    if (kok) {
      cplx<float> t[NB][MR][NW];
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int r = 0; r < MR; ++r)
#pragma unroll
          for (int n = 0; n < NW; ++n) t[i][r][n] = cplx<float>{0.f, 0.f};
      const float* vk = Vk + 2 * k * NW2;
      // one V(k) row per iteration, the next row's loads in flight meanwhile
      // (unrolling would hoist every row's loads and spill the accumulators of
      // the second half)
      float4 cur[NW / 2], nxt[NW / 2];
#pragma unroll
      for (int n = 0; n < NW; n += 2) cur[n / 2] = *reinterpret_cast<const float4*>(vk + 2 * n);
#pragma unroll 1
      for (int a = 0; a < NW; ++a) {
        const int an = a + 1 < NW ? a + 1 : a;
#pragma unroll
        for (int n = 0; n < NW; n += 2) nxt[n / 2] = *reinterpret_cast<const float4*>(vk + 2 * (an * NW + n));
        cplx<float> vr[NW];
#pragma unroll
        for (int n = 0; n < NW; n += 2) {
          vr[n] = cplx<float>{cur[n / 2].x, cur[n / 2].y};
          vr[n + 1] = cplx<float>{cur[n / 2].z, cur[n / 2].w};
        }
#pragma unroll
        for (int i = 0; i < NB; ++i)
#pragma unroll
          for (int r = 0; r < MR; ++r) {
            const float2 x = *reinterpret_cast<const float2*>(krow + 2 * (bcol[i] + (brow0[i] + r) * NW + a));
#pragma unroll
            for (int n = 0; n < NW; ++n) cfma(t[i][r][n], cplx<float>{x.x, x.y}, vr[n]);
          }
#pragma unroll
        for (int n = 0; n < NW / 2; ++n) cur[n] = nxt[n];
      }
      // every W value of the lane's rows has been read (the loop above is
      // this lane's only reader of them): write T over them
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int r = 0; r < MR; ++r)
#pragma unroll
          for (int n = 0; n < NW; ++n)
            *reinterpret_cast<float2*>(krow + 2 * (bcol[i] + (brow0[i] + r) * NW + n)) =
                make_float2(t[i][r][n].re, t[i][r][n].im);
    }
    wave_sync();
    // 2. g_b[m][:] = sum_m' conj(V(k+q_b)[m'][m]) T_b[m'][:] for the lane's rows m
    cplx<float> g[NB][MR][NW];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int r = 0; r < MR; ++r)
#pragma unroll
        for (int n = 0; n < NW; ++n) g[i][r][n] = cplx<float>{0.f, 0.f};
    if (kok) {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        if (!bok[i]) continue;
        const float* vq = vqb[i];
        // V(k+q)[a][m] for the lane's four columns m (16-byte aligned: m0 is 0 or 4),
        // the next row's in flight meanwhile
        float4 c01 = *reinterpret_cast<const float4*>(vq + 2 * brow0[i]);
        float4 c23 = *reinterpret_cast<const float4*>(vq + 2 * (brow0[i] + 2));
#pragma unroll 1
        for (int a = 0; a < NW; ++a) {
          const int an = a + 1 < NW ? a + 1 : a;
          const float4 n01 = *reinterpret_cast<const float4*>(vq + 2 * (an * NW + brow0[i]));
          const float4 n23 = *reinterpret_cast<const float4*>(vq + 2 * (an * NW + brow0[i] + 2));
          const cplx<float> c[MR] = {{c01.x, c01.y}, {c01.z, c01.w}, {c23.x, c23.y}, {c23.z, c23.w}};
#pragma unroll
          for (int n = 0; n < NW; ++n) {
            const float2 tv = *reinterpret_cast<const float2*>(krow + 2 * (bcol[i] + a * NW + n));
#pragma unroll
            for (int r = 0; r < MR; ++r) cfmac(g[i][r][n], c[r], cplx<float>{tv.x, tv.y});
          }
          c01 = n01;
          c23 = n23;
        }
      }
    }
    // the g rows go back to LDS over the lane's own rows once every lane has
    // read its T rows, so that the epilogues below hold one row at a time
    wave_sync();
    if (kok) {
#pragma unroll
      for (int i = 0; i < NB; ++i)
#pragma unroll
        for (int r = 0; r < MR; ++r)
#pragma unroll
          for (int n = 0; n < NW; ++n)
            *reinterpret_cast<float2*>(krow + 2 * (bcol[i] + (brow0[i] + r) * NW + n)) =
                make_float2(g[i][r][n].re, g[i][r][n].im);
    }
    // 3. epilogues (the shuffles run on every lane; rows outside the tile add zero)
    double lw[NW];
#pragma unroll
    for (int n = 0; n < NW; ++n) lw[n] = 0.0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const bool act = kok && bok[i];
      const int64_t pair = bq[i] * B.nk + k;                   // (q, k) within the batch
      const int64_t eoff = (int64_t)bnu[i] * NW2 + (int64_t)brow0[i] * NW;
      const uint64_t base = ((uint64_t)(B.q_global0 + bq[i]) * (uint64_t)B.nk + (uint64_t)k) * (uint64_t)E +
                            (uint64_t)eoff;
      float* go = static_cast<float*>(B.g_out) + 2 * (pair * E + eoff);
      double rs = 0.0;
#pragma unroll 1
      for (int r = 0; r < MR; ++r) {
        const float* gr = krow + 2 * (bcol[i] + (brow0[i] + r) * NW);
        float4 gv[NW / 2];
#pragma unroll
        for (int n = 0; n < NW; n += 2) {
          const float2 a = *reinterpret_cast<const float2*>(gr + 2 * n);
          const float2 b = *reinterpret_cast<const float2*>(gr + 2 * n + 2);
          gv[n / 2] = act ? make_float4(a.x, a.y, b.x, b.y) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
        if (act && want_g) {
#pragma unroll
          for (int n = 0; n < NW; n += 2) *reinterpret_cast<float4*>(go + 2 * (r * NW + n)) = gv[n / 2];
        }
        double g2[NW];
#pragma unroll
        for (int n = 0; n < NW; n += 2) {
          const float4 v = gv[n / 2];
          g2[n] = (double)v.x * (double)v.x + (double)v.y * (double)v.y;
          g2[n + 1] = (double)v.z * (double)v.z + (double)v.w * (double)v.w;
        }
#pragma unroll
        for (int n = 0; n < NW; ++n) rs += g2[n];
        if (act && want_l) {
#pragma unroll
          for (int n = 0; n < NW; ++n) lsum += splitmix_weight(B.loss_seed, base + (uint64_t)(r * NW + n)) * g2[n];
        }
        if (act && want_w && blw[i]) {
          const double em = B.eps_kq[pair * NW + brow0[i] + r];
          const double fm = fermi_occ(em, B.lw);
          const double wa = (bnb[i] + fm) * B.lw.gnorm / (2.0 * bom[i]);
          const double we = (bnb[i] + 1.0 - fm) * B.lw.gnorm / (2.0 * bom[i]);
#pragma unroll
          for (int n = 0; n < NW; ++n) {
            const double en = B.eps_k[k * NW + n];
            const double a = (en - em + bom[i]) * B.lw.inv_sigma, b = (en - em - bom[i]) * B.lw.inv_sigma;
            lw[n] += (wa * gauss_exp<float>(a) + we * gauss_exp<float>(b)) * g2[n];
          }
        }
      }
      if (want_t) {
        // Nw = 8: the block's rows are split over the lane pair; Nw = 4: one lane holds the block
        double tv = rs;
        if (NW == 8) tv += __shfl_xor(tv, 1, 64);
        if (act && (NW == 4 || sb == 0)) B.band_sum[pair * B.nm + bnu[i]] = tv;
      }
    }
    if (want_w) {
      // sum over the k point's rows: the lane pair holds all of them
#pragma unroll
      for (int n = 0; n < NW; ++n) lw[n] += __shfl_xor(lw[n], 1, 64);
      if (kok && cw0 < j.N) {
        double* dst = B.lw_partial + ((cw0 / TN) * B.nk + k) * NW;
#pragma unroll
        for (int n = 0; n < NW; ++n)
          if ((n & 1) == sb) dst[n] = lw[n];
      }
    }
  }
  if (want_l) {
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off, 64);
    double* red = reinterpret_cast<double*>(smem);
    __syncthreads();
    if (lane == 0) red[wave] = lsum;
    __syncthreads();
    if (tid == 0) B.loss_partial[j.tile] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// The same rotations for Nw = 8 when every tile's 128 columns are the two
// modes (nu0, nu0 + 1) of one q (Nm even), on the matrix cores.  Per k point:
//   T = W V(k) with the two modes' W rows stacked (16 rows (nu, m') x 8 bands,
//   both modes share V(k)); g_nu^T = T_nu^T conj(V(k+q)) with rows (nu, n).
// Each complex product is one 16x16 real MFMA product with K = 16 in the
// real embedding [X_re X_im] [[Y_re, Y_im], [-Y_im, Y_re]] = [Z_re Z_im]
// (four v_mfma_f32_16x16x4_f32), so the two rotations of a k point are
// eight MFMAs (1.6 % of the tile's main loop).  The operands come from the
// tile's W rows staged in LDS (both modes' waves), V(k) and V(k+q) from
// global memory (two complex values per lane and k point); the transpose
// between the products and the final store go through the k point's LDS
// rows.  A wave takes 16 k points per half, KI of them per iteration as
// independent MFMA chains.
__device__ __forceinline__ float emb_b(int j_hi, bool c_lo, float re, float im, bool conj_b) {
  // element (j, c) of the real embedding of Y (conj_b: of conj(Y)) given
  // Y[j mod 8][c mod 8] = re + i im: j < 8 rows give (Re, Im) by column half,
  // j >= 8 rows (-Im, Re)
  const float yi = conj_b ? -im : im;
  if (!j_hi) return c_lo ? re : yi;
  return c_lo ? -yi : re;
}

// exp(-x^2/2) and the Fermi occupation 1/(exp(x)+1) on the hardware exp2
// (v_exp_f32, about 1 ulp): the fused epilogue's per-element weights
__device__ __forceinline__ float gauss_fast(float x) {
  return __builtin_amdgcn_exp2f(-0.72134752044448170368f * x * x);   // 0.5 log2(e)
}
__device__ __forceinline__ float fermi_fast(float x) {
  const float z = __builtin_amdgcn_exp2f(-1.44269504088896340736f * fabsf(x));   // exp(-|x|)
  return x > 0.f ? z / (1.f + z) : 1.f / (1.f + z);
}

__device__ __forceinline__ void band_epilogue_mfma8(const TileJob<float>& j, const BandEpilogue& B, int64_t m0,
                                                    int64_t n0, typename Mfma<float>::v4 (&acc_r)[4][4],
                                                    typename Mfma<float>::v4 (&acc_i)[4][4], float* smem) {
  using V4 = typename Mfma<float>::v4;
  constexpr int TM = 64, TN = 64, HR = 32, LDW = TN + 1, KI = 4;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % 2, wn = wave / 2;
  const int lrow = lane >> 4, lcol = lane & 15;
  const int g4 = lane >> 4, c16 = lane & 15, cc = c16 & 7;
  const bool c_lo = c16 < 8;
  const int64_t E = (int64_t)B.nm * 64;
  const int64_t ql = n0 / E;                               // the tile's q (its columns lie in one q)
  const int nu0 = (int)((n0 - ql * E) / 64);              // first of its two modes
  const bool want_g = (B.flags & EPHW_OUT_G) != 0, want_t = (B.flags & EPHW_OUT_BAND_SUM) != 0;
  const bool want_l = (B.flags & EPHW_OUT_LOSS) != 0, want_w = B.lw_partial != nullptr;
  const float* Vk = static_cast<const float*>(B.Vk);
  const float* Vkq = static_cast<const float*>(B.Vkq);
  auto region = [&](int wm_, int nu_l) { return smem + (nu_l * 2 + wm_) * (HR * LDW * 2); };
  // linewidth: the lane's mode in the second product's output is nu0 + g4 / 2
  double om = 0.0, nbose = 0.0, amp0 = 0.0;
  bool lw_mode = false;
  if (want_w) {
    om = B.omega[ql * B.nm + nu0 + g4 / 2];
    lw_mode = om > 0.0 && om >= B.lw.omega_min;
    if (lw_mode) {
      nbose = 1.0 / expm1(om * B.lw.inv_t);
      amp0 = B.lw.gnorm / (2.0 * om);
    }
  }
  const float inv_sigma_f = (float)B.lw.inv_sigma;
  double lsum = 0.0;
  float* wl = smem + wave * (HR * LDW * 2);
  const int wsrc = wave >> 1, ksub = wave & 1;             // rows of wave-row wsrc, 16-row half ksub
#pragma unroll 1
  for (int h = 0; h < 2; ++h) {
    __syncthreads();   // the K loop's stages / the previous half's rows are done with
#pragma unroll
    for (int ii = 0; ii < 2; ++ii)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = ii * 16 + Mfma<float>::row(lrow, v), col = jj * 16 + lcol;
          const float re = h == 0 ? acc_r[ii][jj][v] : acc_r[2 + ii][jj][v];
          const float im = h == 0 ? acc_i[ii][jj][v] : acc_i[2 + ii][jj][v];
          *reinterpret_cast<float2*>(wl + 2 * (row * LDW + col)) = make_float2(re, im);
        }
    __syncthreads();   // both modes' rows of every k point are staged
#pragma unroll 1
    for (int it = 0; it < 16; it += KI) {
      int kl[KI];
      int64_t k[KI];
      bool kok[KI];
#pragma unroll
      for (int u = 0; u < KI; ++u) {
        kl[u] = ksub * 16 + it + u;
        k[u] = m0 + wsrc * TM + h * HR + kl[u];
        kok[u] = k[u] < j.M;
      }
      // operands of the first product: V(k)[g][cc], V(k)[4+g][cc]; W rows
      V4 acc[KI];
      float2 v0[KI], v1[KI], u0[KI], u1[KI];
#pragma unroll
      for (int u = 0; u < KI; ++u) {
        const int64_t kk = kok[u] ? k[u] : 0;
        const float* vk = Vk + 2 * kk * 64;
        v0[u] = *reinterpret_cast<const float2*>(vk + 2 * (g4 * 8 + cc));
        v1[u] = *reinterpret_cast<const float2*>(vk + 2 * ((4 + g4) * 8 + cc));
        const float* vq;
        if (Vkq) {
          vq = Vkq + 2 * ((ql * B.nk + kk) * 64);
        } else {
          int64_t id = kok[u] ? B.kq_index[ql * B.nk + kk] : 0;
          if (id < 0 || id >= B.nk) {
            atomicOr(B.status, kStatusIndex);
            id = 0;
          }
          vq = Vk + 2 * id * 64;
        }
        u0[u] = *reinterpret_cast<const float2*>(vq + 2 * (g4 * 8 + cc));
        u1[u] = *reinterpret_cast<const float2*>(vq + 2 * ((4 + g4) * 8 + cc));
        acc[u] = V4{0.f, 0.f, 0.f, 0.f};
      }
      // T = W V(k): A[(nu, m')][(part, n')] = W_part[nu][m'][n'], lane row c16
#pragma unroll
      for (int u = 0; u < KI; ++u) {
        const float* wr = region(wsrc, c16 >> 3) + 2 * (kl[u] * LDW + (c16 & 7) * 8);
        const float2 w0 = *reinterpret_cast<const float2*>(wr + 2 * g4);
        const float2 w1 = *reinterpret_cast<const float2*>(wr + 2 * (4 + g4));
        const float a[4] = {w0.x, w1.x, w0.y, w1.y};
        const float b[4] = {emb_b(0, c_lo, v0[u].x, v0[u].y, false), emb_b(0, c_lo, v1[u].x, v1[u].y, false),
                            emb_b(1, c_lo, v0[u].x, v0[u].y, false), emb_b(1, c_lo, v1[u].x, v1[u].y, false)};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) acc[u] = Mfma<float>::op(a[s4], b[s4], acc[u]);
      }
      wave_sync();   // every lane has read its W operands
      // T rows back to the k point's LDS rows: lane holds T_part[nu][m'][n],
      // nu = g4 / 2, m' = 4 (g4 % 2) + i, part = c16 / 8, n = cc
#pragma unroll
      for (int u = 0; u < KI; ++u) {
        float* tr = region(wsrc, g4 >> 1) + 2 * (kl[u] * LDW);
#pragma unroll
        for (int i = 0; i < 4; ++i) tr[2 * ((4 * (g4 & 1) + i) * 8 + cc) + (c16 >> 3)] = acc[u][i];
        acc[u] = V4{0.f, 0.f, 0.f, 0.f};
      }
      wave_sync();
      // g^T = T^T conj(V(k+q)): A[(nu, n)][(part, m')] = T_part[nu][m'][n], lane row c16
#pragma unroll
      for (int u = 0; u < KI; ++u) {
        const float* tr = region(wsrc, c16 >> 3) + 2 * (kl[u] * LDW);
        const int n = c16 & 7;
        const float a[4] = {tr[2 * (g4 * 8 + n)], tr[2 * ((4 + g4) * 8 + n)], tr[2 * (g4 * 8 + n) + 1],
                            tr[2 * ((4 + g4) * 8 + n) + 1]};
        const float b[4] = {emb_b(0, c_lo, u0[u].x, u0[u].y, true), emb_b(0, c_lo, u1[u].x, u1[u].y, true),
                            emb_b(1, c_lo, u0[u].x, u0[u].y, true), emb_b(1, c_lo, u1[u].x, u1[u].y, true)};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) acc[u] = Mfma<float>::op(a[s4], b[s4], acc[u]);
      }
      wave_sync();   // every lane has read its T operands
      // lane holds part c16 / 8 of g_nu[m][n], nu = nu0 + g4 / 2, n = 4 (g4 % 2) + i, m = cc
#pragma unroll
      for (int u = 0; u < KI; ++u) {
        const int nul = g4 >> 1;
        double vsq[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) vsq[i] = (double)acc[u][i] * (double)acc[u][i];
        const int64_t pair = ql * B.nk + k[u];
        if (want_g) {
          float* gr = region(wsrc, nul) + 2 * (kl[u] * LDW);
#pragma unroll
          for (int i = 0; i < 4; ++i) gr[2 * (cc * 8 + 4 * (g4 & 1) + i) + (c16 >> 3)] = acc[u][i];
        }
        if (want_t) {
          double tv = (vsq[0] + vsq[1]) + (vsq[2] + vsq[3]);
#pragma unroll
          for (int off = 1; off < 32; off <<= 1) tv += __shfl_xor(tv, off, 64);
          if (kok[u] && (lane & 31) == 0) B.band_sum[pair * B.nm + nu0 + nul] = tv;
        }
        if (want_l && kok[u]) {
          const uint64_t base = ((uint64_t)(B.q_global0 + ql) * (uint64_t)B.nk + (uint64_t)k[u]) * (uint64_t)E +
                                (uint64_t)(nu0 + nul) * 64u + (uint64_t)cc * 8u + (uint64_t)(4 * (g4 & 1));
#pragma unroll
          for (int i = 0; i < 4; ++i) lsum += splitmix_weight(B.loss_seed, base + (uint64_t)i) * vsq[i];
        }
        if (want_w) {
          // |g|^2 of the lane's four elements: the other part sits in lane c16 ^ 8
          double s2[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float o = __shfl_xor(acc[u][i], 8, 64);
            s2[i] = vsq[i] + (double)o * (double)o;
          }
          // the lane pair (c16, c16 ^ 8) splits the two terms: absorption
          // (N + f_m) G(e_n - e_m + omega) on c16 < 8, emission (N + 1 - f_m)
          // G(e_n - e_m - omega) on c16 >= 8
          double lw[4] = {0.0, 0.0, 0.0, 0.0};
          if (kok[u] && lw_mode) {
            // c64 data: occupation and Gaussians from the hardware exp2 in
            // FP32 (relative error near 1e-7, below the data's own); the energy
            // differences in FP64
            const double em = B.eps_kq[pair * 8 + cc];
            const double fm = (double)fermi_fast((float)((em - B.lw.mu) * B.lw.inv_t));
            const double amp = (c_lo ? nbose + fm : nbose + 1.0 - fm) * amp0;
            const double sh = (c_lo ? om : -om) - em;
            const double2 e01 = *reinterpret_cast<const double2*>(B.eps_k + k[u] * 8 + 4 * (g4 & 1));
            const double2 e23 = *reinterpret_cast<const double2*>(B.eps_k + k[u] * 8 + 4 * (g4 & 1) + 2);
            const double en[4] = {e01.x, e01.y, e23.x, e23.y};
#pragma unroll
            for (int i = 0; i < 4; ++i)
              lw[i] = amp * (double)gauss_fast((float)(en[i] + sh) * inv_sigma_f) * s2[i];
          }
          // sum over m, both terms and both modes for each band n: halve the
          // four values over lane bits 0 and 1, then add over bits 2, 3 and 5
          const int b0 = lane & 1, b1 = (lane >> 1) & 1;
          double l2[2];
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            const double mine = b0 ? lw[2 + jj] : lw[jj];
            const double other = b0 ? lw[jj] : lw[2 + jj];
            l2[jj] = mine + __shfl_xor(other, 1, 64);
          }
          double v = b1 ? l2[1] : l2[0];
          v += __shfl_xor(b1 ? l2[0] : l2[1], 2, 64);
          v += __shfl_xor(v, 4, 64);
          v += __shfl_xor(v, 8, 64);
          v += __shfl_xor(v, 32, 64);
          // lanes c16 < 4 of groups 0 and 1 hold band n = 4 g4 + 2 b0 + b1
          if (kok[u] && c16 < 4 && g4 < 2)
            B.lw_partial[((n0 / 128) * B.nk + k[u]) * 8 + 4 * g4 + 2 * b0 + b1] = v;
        }
      }
      if (want_g) {
        wave_sync();   // the k points' g blocks are complete in LDS
        // each k point's two modes are 128 consecutive complex values of g:
        // lane l stores values 2l, 2l + 1 (mode l / 32)
#pragma unroll
        for (int u = 0; u < KI; ++u) {
          if (!kok[u]) continue;
          const float* gr = region(wsrc, lane >> 5) + 2 * (kl[u] * LDW + 2 * (lane & 31));
          const float2 x0 = *reinterpret_cast<const float2*>(gr);
          const float2 x1 = *reinterpret_cast<const float2*>(gr + 2);
          float* go = static_cast<float*>(B.g_out) + 2 * ((ql * B.nk + k[u]) * E + (int64_t)nu0 * 64 + 2 * lane);
          *reinterpret_cast<float4*>(go) = make_float4(x0.x, x0.y, x1.x, x1.y);
        }
      }
      wave_sync();   // the next k points' rows are other rows; keep the order simple
    }
  }
  if (want_l) {
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off, 64);
    double* red = reinterpret_cast<double*>(smem);
    __syncthreads();
    if (lane == 0) red[wave] = lsum;
    __syncthreads();
    if (tid == 0) B.loss_partial[j.tile] = (red[0] + red[1]) + (red[2] + red[3]);
  }
}

// Computes the BM x BN tile at (m0, n0) of job j with the workgroup's
// NT threads; `smem` holds TileShape::smem_elems values of T.
//
// Pipeline: global loads of slab s+1 go to registers (16-byte buffer loads)
// while slab s is multiplied from one LDS stage; the registers are then
// written to the other stage, so each slab costs one barrier.  LDS keeps
// complex values interleaved, laid out [k][m] and [k][n], so one 8- or
// 16-byte read gives a lane its (re, im) operand pair.
// KBLK > 0: K-blocked accumulation, a fresh accumulator every KBLK slabs
// (the compensated FP32 form, see the K loop)
// FLAT: both operands' whole extents fit 32-bit byte offsets from the
// tile's origin (checked at launch), so one buffer resource per operand
// serves every slab and a slab only adds a uniform offset
template <typename T, int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, int KBLK, int BANDNW = 0,
          bool FLAT = false>
__device__ __forceinline__ void gemm_tile(const TileJob<T>& j, int64_t m0, int64_t n0, T* smem,
                                          const BandEpilogue* band = nullptr) {
  using S = TileShape<T, BM, BN, BK, WM, WN>;
  using C = Chunk<T>;
  using V4 = typename C::v4;
  using V2 = typename C::v2;
  using Acc = typename Mfma<T>::v4;
  constexpr int NT = S::NT, CPC = C::CPC;
  constexpr int TM = BM / WM, TN = BN / WN;
  constexpr int FM = TM / 16, FN = TN / 16;
  constexpr int LA = S::LA, LB = S::LB;
  constexpr int CS = 2 * (int)sizeof(T);               // bytes per complex value
  // global slab rows: A is [BM][BK] (TA: [BK][BM]), B is [BK][BN] (TB: [BN][BK])
  constexpr int A_RC = (TA ? BM : BK) / CPC;           // chunks per slab row
  constexpr int B_RC = (TB ? BK : BN) / CPC;
  constexpr int AC = BM * BK / CPC / NT;               // chunks per thread
  constexpr int BC = BK * BN / CPC / NT;
  // Row-group mode (NT a multiple of the chunks per row): a thread's chunks
  // share one slab column and sit RSTEP rows apart, so one 32-bit lane offset
  // serves all of them with one buffer base per row group.  Otherwise each
  // chunk has its own offset from the slab base.
  constexpr bool A_GRP = NT % A_RC == 0, B_GRP = NT % B_RC == 0;
  constexpr int A_RSTEP = A_GRP ? NT / A_RC : 0, B_RSTEP = B_GRP ? NT / B_RC : 0;
  // a whole number of waves per slab row: the row is wave-uniform and goes
  // into the base, leaving only the in-row chunk offset per lane
  constexpr bool A_WROW = A_GRP && A_RC % 64 == 0, B_WROW = B_GRP && B_RC % 64 == 0;
  static_assert(TM % 16 == 0 && TN % 16 == 0 && BK % 4 == 0, "bad tile");
  static_assert(AC * NT * CPC == BM * BK && BC * NT * CPC == BK * BN, "tile not divisible by threads");

  const int64_t M = j.M, N = j.N, K = j.K;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % WM, wn = wave / WM;
  const int lrow = lane >> 4;   // k row inside one MFMA (0..3); also the lane group
  const int lcol = lane & 15;   // m (A) or n (B) inside one 16-block

  // slab row and chunk of a thread's i-th chunk
  auto a_pos = [&](int i, int& r, int& ch) {
    const int c = A_GRP ? tid : tid + i * NT;
    r = c / A_RC + (A_GRP ? i * A_RSTEP : 0);
    ch = c % A_RC;
  };
  auto b_pos = [&](int i, int& r, int& ch) {
    const int c = B_GRP ? tid : tid + i * NT;
    r = c / B_RC + (B_GRP ? i * B_RSTEP : 0);
    ch = c % B_RC;
  };
  const int64_t a_row0 = A_WROW ? (int64_t)(tid / A_RC) * j.lda : 0;   // wave-uniform part
  const int64_t b_row0 = B_WROW ? (int64_t)(tid / B_RC) * j.ldb : 0;
  const uint32_t a_off0 =
      (uint32_t)(((A_WROW ? 0 : (int64_t)(tid / A_RC) * j.lda) + (tid % A_RC) * CPC) * CS);
  const uint32_t b_off0 =
      (uint32_t)(((B_WROW ? 0 : (int64_t)(tid / B_RC) * j.ldb) + (tid % B_RC) * CPC) * CS);
  const int64_t a_ext = TA ? (K - 1) * j.lda + M : (M - 1) * j.lda + K;   // complex values from A
  const int64_t b_ext = TB ? (N - 1) * j.ldb + K : (K - 1) * j.ldb + N;

  V4 ra[AC], rb[BC];

  static_assert(!FLAT || (A_GRP && B_GRP), "the flat loader addresses chunks by row group");
  const int64_t ao0 = TA ? m0 : m0 * j.lda, bo0 = TB ? n0 * j.ldb : n0;
  const __amdgpu_buffer_rsrc_t rsa = make_rsrc(j.A + 2 * ao0, FLAT ? (a_ext - ao0) * CS : 0);
  const __amdgpu_buffer_rsrc_t rsb = make_rsrc(j.B + 2 * bo0, FLAT ? (b_ext - bo0) * CS : 0);
  const uint32_t a_row_bytes = (uint32_t)(a_row0 * CS), b_row_bytes = (uint32_t)(b_row0 * CS);
  auto load = [&](int64_t k0) {
    if constexpr (FLAT) {
      const uint32_t ka = (uint32_t)((TA ? k0 * j.lda : k0) * CS);
      const uint32_t kb = (uint32_t)((TB ? k0 : k0 * j.ldb) * CS);
#pragma unroll
      for (int i = 0; i < AC; ++i)
        ra[i] = load_chunk<T>(rsa, a_off0 + a_row_bytes + (uint32_t)((int64_t)i * A_RSTEP * j.lda * CS) + ka);
#pragma unroll
      for (int i = 0; i < BC; ++i)
        rb[i] = load_chunk<T>(rsb, b_off0 + b_row_bytes + (uint32_t)((int64_t)i * B_RSTEP * j.ldb * CS) + kb);
      return;
    }
    const int64_t ao = TA ? k0 * j.lda + m0 : m0 * j.lda + k0;
    const int64_t bo = TB ? n0 * j.ldb + k0 : k0 * j.ldb + n0;
#pragma unroll
    for (int i = 0; i < AC; ++i) {
      if (A_GRP) {  // one resource per row group
        const int64_t o = ao + (int64_t)i * A_RSTEP * j.lda + a_row0;
        ra[i] = load_chunk<T>(make_rsrc(j.A + 2 * o, (a_ext - o) * CS), a_off0);
      } else {
        int r, ch;
        a_pos(i, r, ch);
        const uint32_t off = (uint32_t)(((int64_t)r * j.lda + ch * CPC) * CS);
        ra[i] = load_chunk<T>(make_rsrc(j.A + 2 * ao, (a_ext - ao) * CS), off);
      }
    }
#pragma unroll
    for (int i = 0; i < BC; ++i) {
      if (B_GRP) {
        const int64_t o = bo + (int64_t)i * B_RSTEP * j.ldb + b_row0;
        rb[i] = load_chunk<T>(make_rsrc(j.B + 2 * o, (b_ext - o) * CS), b_off0);
      } else {
        int r, ch;
        b_pos(i, r, ch);
        const uint32_t off = (uint32_t)(((int64_t)r * j.ldb + ch * CPC) * CS);
        rb[i] = load_chunk<T>(make_rsrc(j.B + 2 * bo, (b_ext - bo) * CS), off);
      }
    }
  };

  // registers -> LDS stage of the slab at k0; conjugation is applied here,
  // and the K tail where K runs along a row (the next row's values must not
  // enter).  The tail is masked here rather than right after the loads: a
  // select on the loaded registers would make the wave wait for the loads at
  // the top of the slab instead of after its MFMAs.
  auto stash = [&](T* st, int64_t k0) {
    const int64_t klim = K - k0;
    if (!TA && klim < BK) {
#pragma unroll
      for (int i = 0; i < AC; ++i) {
        int r, ch;
        a_pos(i, r, ch);
#pragma unroll
        for (int e = 0; e < CPC; ++e)
          if (ch * CPC + e >= klim) {
            ra[i][2 * e] = T(0);
            ra[i][2 * e + 1] = T(0);
          }
      }
    }
    if (TB && klim < BK) {
#pragma unroll
      for (int i = 0; i < BC; ++i) {
        int r, ch;
        b_pos(i, r, ch);
#pragma unroll
        for (int e = 0; e < CPC; ++e)
          if (ch * CPC + e >= klim) {
            rb[i][2 * e] = T(0);
            rb[i][2 * e + 1] = T(0);
          }
      }
    }
    T* As = st;
    T* Bs = st + 2 * BK * LA;
#pragma unroll
    for (int i = 0; i < AC; ++i) {
      V4 v = ra[i];
#pragma unroll
      for (int e = 0; e < CPC; ++e) v[2 * e + 1] *= j.sa;
      int r, ch;
      a_pos(i, r, ch);
      if (TA) {  // slab row r is k; the chunk holds CPC consecutive m
        *reinterpret_cast<V4*>(As + 2 * (r * LA + ch * CPC)) = v;
      } else {   // slab row r is m; the chunk holds CPC consecutive k
#pragma unroll
        for (int e = 0; e < CPC; ++e)
          *reinterpret_cast<V2*>(As + 2 * ((ch * CPC + e) * LA + r)) = V2{v[2 * e], v[2 * e + 1]};
      }
    }
#pragma unroll
    for (int i = 0; i < BC; ++i) {
      V4 v = rb[i];
#pragma unroll
      for (int e = 0; e < CPC; ++e) v[2 * e + 1] *= j.sb;
      int r, ch;
      b_pos(i, r, ch);
      if (!TB) {  // slab row r is k; the chunk holds CPC consecutive n
        *reinterpret_cast<V4*>(Bs + 2 * (r * LB + ch * CPC)) = v;
      } else {    // slab row r is n; the chunk holds CPC consecutive k
#pragma unroll
        for (int e = 0; e < CPC; ++e)
          *reinterpret_cast<V2*>(Bs + 2 * ((ch * CPC + e) * LB + r)) = V2{v[2 * e], v[2 * e + 1]};
      }
    }
  };

  Acc acc_r[FM][FN], acc_i[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int jj = 0; jj < FN; ++jj) {
      acc_r[i][jj] = Acc{0, 0, 0, 0};
      acc_i[i][jj] = Acc{0, 0, 0, 0};
    }

  // One BK slab of MFMAs from an LDS stage.  The four real products of every
  // block are issued product by product across all blocks, so consecutive
  // MFMAs never depend on each other.  NBL (compile time) column blocks of
  // the wave are multiplied and K steps from kmax on are skipped: the
  // one-wave-column tiles (WN = 1) leave out a column block that lies wholly
  // past N and the K steps of the last slab past K (their operands are the
  // zeros of the padded loads, so skipping them changes nothing).
  auto compute = [&](const T* st, auto nbl, int kmax) {
    constexpr int NBL = decltype(nbl)::value;
    const T* As = st;
    const T* Bs = st + 2 * BK * LA;
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      if (kk >= kmax) break;
      const int kr = kk + lrow;
      V2 a[FM], b[NBL];
      T nai[FM];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        a[i] = *reinterpret_cast<const V2*>(As + 2 * (kr * LA + wm * TM + i * 16 + lcol));
        nai[i] = -a[i][1];
      }
#pragma unroll
      for (int jj = 0; jj < NBL; ++jj)
        b[jj] = *reinterpret_cast<const V2*>(Bs + 2 * (kr * LB + wn * TN + jj * 16 + lcol));
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int jj = 0; jj < NBL; ++jj) acc_r[i][jj] = Mfma<T>::op(a[i][0], b[jj][0], acc_r[i][jj]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int jj = 0; jj < NBL; ++jj) acc_i[i][jj] = Mfma<T>::op(a[i][0], b[jj][1], acc_i[i][jj]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int jj = 0; jj < NBL; ++jj) acc_r[i][jj] = Mfma<T>::op(nai[i], b[jj][1], acc_r[i][jj]);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int jj = 0; jj < NBL; ++jj) acc_i[i][jj] = Mfma<T>::op(a[i][1], b[jj][0], acc_i[i][jj]);
    }
  };
  // the skipping form: FP32 tiles with one wave column (all waves then skip
  // the same blocks, so no wave waits for another at the slab barrier)
  constexpr bool SKIP = sizeof(T) == 4 && WN == 1 && FN > 1 && KBLK == 0 && BANDNW == 0;
  const bool last_col_dead = SKIP && n0 + (FN - 1) * 16 >= N;

  // K-blocked accumulation (the compensated FP32 form): the MFMA
  // accumulators start from zero every KBLK slabs and each block's partial
  // sum is added into a second set of registers.  One accumulator summing
  // all K products in order picks up a rounding error that grows with the
  // size of the running sum; over K = 1000 that is the dominant error of the
  // FP32 phase sums, well above the rounding of the phases themselves.
  Acc sum_r[KBLK ? FM : 1][KBLK ? FN : 1], sum_i[KBLK ? FM : 1][KBLK ? FN : 1];
  if constexpr (KBLK > 0) {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int jj = 0; jj < FN; ++jj) {
        sum_r[i][jj] = Acc{0, 0, 0, 0};
        sum_i[i][jj] = Acc{0, 0, 0, 0};
      }
  }
  auto fold = [&]() {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int jj = 0; jj < FN; ++jj) {
        sum_r[i][jj] += acc_r[i][jj];
        sum_i[i][jj] += acc_i[i][jj];
        acc_r[i][jj] = Acc{0, 0, 0, 0};
        acc_i[i][jj] = Acc{0, 0, 0, 0};
      }
  };

  // K loop: one barrier per slab (see the pipeline note above)
  const int64_t nslab = (K + BK - 1) / BK;
  // (the skipping tiles run one K loop per column-block count; a branch
  // between two compute forms inside one loop made the compiler spill)
  auto kloop = [&](auto nbl) {
    load(0);
    stash(smem, 0);
    __syncthreads();
    for (int64_t sl = 0; sl < nslab; ++sl) {
      const bool more = sl + 1 < nslab;
      if (more) load((sl + 1) * BK);
      // the K steps of the last slab past K are skipped where columns are
      const int kmax = SKIP ? (int)(K - sl * BK < BK ? K - sl * BK : BK) : BK;
      compute(smem + (sl & 1) * S::stage_elems, nbl, kmax);
      if constexpr (KBLK > 0) {
        if ((sl + 1) % KBLK == 0) fold();
      }
      if (more) stash(smem + ((sl + 1) & 1) * S::stage_elems, (sl + 1) * BK);
      __syncthreads();
    }
  };
  if constexpr (SKIP) {
    if (last_col_dead)
      kloop(IntC<(SKIP ? FN - 1 : FN)>{});
    else
      kloop(IntC<FN>{});
  } else if constexpr (sizeof(T) == 4 && KBLK == 0 && BANDNW == 0) {
    // FP32 without a fused epilogue: the last slab peeled off, so that its K
    // steps past K are skipped without a test in the main loop (with the
    // fused band epilogues the peeled copy made the compiler spill more)
    load(0);
    stash(smem, 0);
    __syncthreads();
    for (int64_t sl = 0; sl + 1 < nslab; ++sl) {
      load((sl + 1) * BK);
      compute(smem + (sl & 1) * S::stage_elems, IntC<FN>{}, BK);
      stash(smem + ((sl + 1) & 1) * S::stage_elems, (sl + 1) * BK);
      __syncthreads();
    }
    if (nslab > 0) {
      const int64_t sl = nslab - 1;
      compute(smem + (sl & 1) * S::stage_elems, IntC<FN>{}, (int)(K - sl * BK));
      __syncthreads();
    }
  } else {
    load(0);
    stash(smem, 0);
    __syncthreads();
    for (int64_t sl = 0; sl < nslab; ++sl) {
      const bool more = sl + 1 < nslab;
      if (more) load((sl + 1) * BK);
      compute(smem + (sl & 1) * S::stage_elems, IntC<FN>{}, BK);
      if constexpr (KBLK > 0) {
        if ((sl + 1) % KBLK == 0) fold();
      }
      if (more) stash(smem + ((sl + 1) & 1) * S::stage_elems, (sl + 1) * BK);
      __syncthreads();
    }
  }
  if constexpr (KBLK > 0) {
    // the last (partial) block, then the blocked sum back into the accumulators
    // the epilogues read
    if (nslab % KBLK != 0) fold();
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int jj = 0; jj < FN; ++jj) {
        acc_r[i][jj] = sum_r[i][jj];
        acc_i[i][jj] = sum_i[i][jj];
      }
  }

  if constexpr (BANDNW > 0) {
    static_assert(sizeof(T) == 4 && BM == 128 && BN == 128 && WM == 2 && WN == 2 && KBLK == 0,
                  "the band epilogue runs on the FP32 128x128 tile");
    // BANDNW: 4 or 8 the rotations on VALU; 16 the Nw = 8 rotations on MFMA
    if constexpr (BANDNW == 16)
      band_epilogue_mfma8(j, *band, m0, n0, acc_r, acc_i, smem);
    else
      band_epilogue<BANDNW>(j, *band, m0, n0, acc_r, acc_i, smem);
    return;
  }
  // --- epilogue: lane holds column lcol of every block, rows per Mfma<T>::row --
  double part = 0.0;
  const LossEpilogue& L = j.loss;
  if constexpr (sizeof(T) == 8) {
    // FP64: offsets per element (the 64x224 FP64 tiles sit at the register
    // limit; hoisting the row offsets out of the column loop spills there)
    const int64_t tb = j.tblock;
    auto c_index = [&](int64_t row, int64_t col) -> int64_t {
      return tb > 0 ? (row / tb) * j.ldc + col * tb + row % tb : row * j.ldc + col;
    };
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
              V2* c = reinterpret_cast<V2*>(j.C + 2 * c_index(row, col));
              V2 val{acc_r[i][jj][v], acc_i[i][jj][v]};
              if (j.accumulate) val += *c;
              *c = val;
            }
          }
        }
      return;
    }
    // weighted |c|^2: element index ((((q nk + k) nm + nu) nw + m) nw + n)
    const int64_t per_q = L.layout == 0 ? (int64_t)L.qb * L.nm : (int64_t)L.qb;
    const int64_t il = j.batch / per_q;
    const int64_t iq = L.layout == 0 ? (j.batch / L.nm) % L.qb : j.batch % L.qb;
    const int64_t nu = L.layout == 0 ? j.batch % L.nm : 0;
    const uint64_t nw2 = (uint64_t)L.nw * (uint64_t)L.nw;
    const uint64_t base =
        (((uint64_t)(L.q0 + iq) * (uint64_t)L.nk + (uint64_t)(L.k0 + il)) * (uint64_t)L.nm + (uint64_t)nu) * nw2;
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
            const uint64_t el = L.layout == 0
                                    ? (uint64_t)(row * L.nw + col)
                                    : (uint64_t)(row / L.nw) * nw2 + (uint64_t)col * L.nw + (uint64_t)(row % L.nw);
            const double w = splitmix_weight(L.seed, base + el);
            part += w * ((double)re * (double)re + (double)im * (double)im);
            if (L.store) {
              T* c = j.C + 2 * c_index(row, col);
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
  } else {
    // C offset of element (row, col) = row_off(row) + col * cstep: the row part
    // takes one division per row of the lane, not one per element
    const int64_t tb = j.tblock;
    const int64_t cstep = tb > 0 ? tb : 1;
    auto row_off = [&](int64_t row) -> int64_t {
      if (tb > 0) {
        const int64_t blk = row / tb;
        return blk * j.ldc + (row - blk * tb);
      }
      return row * j.ldc;
    };
    if (!j.loss.on) {
      if constexpr (sizeof(T) == 4) {
        // Block-transposed FP32 output: the four rows 4g..4g+3 of a lane are
        // consecutive in C (rows of one Nw block, Nw a multiple of 4), so the
        // lane stores them as two 16-byte chunks.
        if (tb > 0 && tb % 4 == 0 && j.ldc % 4 == 0 && (reinterpret_cast<uintptr_t>(j.C) & 31) == 0 &&
            !j.accumulate) {
#pragma unroll
          for (int i = 0; i < FM; ++i) {
            const int64_t row0 = m0 + wm * TM + i * 16 + Mfma<T>::row(lrow, 0);
            const int64_t ro = row_off(row0);
            const bool all4 = row0 + 3 < M;
#pragma unroll
            for (int jj = 0; jj < FN; ++jj) {
              const int64_t col = n0 + wn * TN + jj * 16 + lcol;
              if (col >= N) continue;
              T* c = j.C + 2 * (ro + col * cstep);
              if (all4) {
                reinterpret_cast<V4*>(c)[0] = V4{acc_r[i][jj][0], acc_i[i][jj][0], acc_r[i][jj][1], acc_i[i][jj][1]};
                reinterpret_cast<V4*>(c)[1] = V4{acc_r[i][jj][2], acc_i[i][jj][2], acc_r[i][jj][3], acc_i[i][jj][3]};
              } else {
#pragma unroll
                for (int v = 0; v < 4; ++v)
                  if (row0 + v < M) reinterpret_cast<V2*>(c)[v] = V2{acc_r[i][jj][v], acc_i[i][jj][v]};
              }
            }
          }
          return;
        }
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t row = m0 + wm * TM + i * 16 + Mfma<T>::row(lrow, v);
          if (row >= M) continue;
          const int64_t ro = row_off(row);
#pragma unroll
          for (int jj = 0; jj < FN; ++jj) {
            const int64_t col = n0 + wn * TN + jj * 16 + lcol;
            if (col < N) {
              V2* c = reinterpret_cast<V2*>(j.C + 2 * (ro + col * cstep));
              V2 val{acc_r[i][jj][v], acc_i[i][jj][v]};
              if (j.accumulate) val += *c;
              *c = val;
            }
          }
        }
      return;
    }
    // weighted |c|^2: element index ((((q nk + k) nm + nu) nw + m) nw + n)
    const int64_t per_q = L.layout == 0 ? (int64_t)L.qb * L.nm : (int64_t)L.qb;
    const int64_t il = j.batch / per_q;
    const int64_t iq = L.layout == 0 ? (j.batch / L.nm) % L.qb : j.batch % L.qb;
    const int64_t nu = L.layout == 0 ? j.batch % L.nm : 0;
    const uint64_t nw2 = (uint64_t)L.nw * (uint64_t)L.nw;
    const uint64_t base =
        (((uint64_t)(L.q0 + iq) * (uint64_t)L.nk + (uint64_t)(L.k0 + il)) * (uint64_t)L.nm + (uint64_t)nu) * nw2;
    // element index of (row, col) = base + ebase(row) + col * estep
    const uint64_t estep = L.layout == 0 ? 1 : (uint64_t)L.nw;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t row = m0 + wm * TM + i * 16 + Mfma<T>::row(lrow, v);
        if (row >= M) continue;
        const int64_t ro = L.store ? row_off(row) : 0;
        uint64_t eb;
        if (L.layout == 0) {
          eb = (uint64_t)row * L.nw;
        } else {
          const int64_t b = row / L.nw;
          eb = (uint64_t)b * nw2 + (uint64_t)(row - b * L.nw);
        }
        eb += base;
#pragma unroll
        for (int jj = 0; jj < FN; ++jj) {
          const int64_t col = n0 + wn * TN + jj * 16 + lcol;
          if (col < N) {
            const T re = acc_r[i][jj][v], im = acc_i[i][jj][v];
            const double w = splitmix_weight(L.seed, eb + (uint64_t)col * estep);
            part += w * ((double)re * (double)re + (double)im * (double)im);
            if (L.store) {
              T* c = j.C + 2 * (ro + col * cstep);
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
  j.tblock = p.tblock;
  j.loss = p.loss;
  j.batch = b;
  j.tile = 0;
  j.ntiles = 1;
  return j;
}

// OCC: waves per SIMD the register allocation must leave room for
template <typename T, int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, int KBLK, int OCC, int BANDNW = 0,
          bool FLAT = false>
__global__ void __launch_bounds__(64 * WM * WN) __attribute__((amdgpu_waves_per_eu(OCC)))
    cgemm_kernel(GemmParams p, int64_t tiles_m, int64_t tiles_n) {
  using S = TileShape<T, BM, BN, BK, WM, WN>;
  __shared__ T smem[S::smem_elems];
  const int64_t logical = xcd_remap(blockIdx.x, tiles_m * tiles_n);
  int64_t tm, tn;
  tile_coords(logical, tiles_m, tiles_n, &tm, &tn);
  TileJob<T> j = job_of<T>(p, p.batch_base + blockIdx.y);
  j.tile = tm * tiles_n + tn;
  j.ntiles = tiles_m * tiles_n;
  gemm_tile<T, BM, BN, BK, WM, WN, TA, TB, KBLK, BANDNW, FLAT>(j, tm * BM, tn * BN, smem, &p.band);
}

// Tile shapes of the grouped kernel: cfg 0 is the default tile of the plain
// kernel (FP32 128x128, FP64 64x64), cfg 1 a 64x64 tile for small problems.
// Both use 4 waves.
template <typename T>
struct GroupCfg;
template <>
struct GroupCfg<float> {
  static constexpr int LM = 128, LN = 128, LK = 16, SM = 64, SN = 64, SK = 16;
};
template <>
struct GroupCfg<double> {
  static constexpr int LM = 64, LN = 64, LK = 8, SM = 64, SN = 64, SK = 8;
};

// One launch serves problems of one tile configuration (CFG), so each
// instance gets the register budget of its own tile.
// Work queue of the grouped kernel: the tile list is cut into kXcds
// contiguous ranges, one per XCD, each with a counter in `queue` (zeroed
// before the launch).  A workgroup takes tiles from its own XCD's range in
// order (neighbouring tiles share A and B panels in that XCD's L2) and, once
// that range is used up, from the other ranges; so workgroups that draw cheap
// tiles (small K) take more of them.  Every range is handed out exactly once
// and every workgroup stops after finding all ranges used up.
__device__ __forceinline__ int64_t queue_lo(int q, int64_t total) { return (int64_t)q * total / kXcds; }

__device__ __forceinline__ int64_t queue_grab(int* __restrict__ queue, int64_t total, int& q, int& tried) {
  while (tried < kXcds) {
    const int64_t t = queue_lo(q, total) + atomicAdd(&queue[q], 1);
    if (t < queue_lo(q + 1, total)) return t;
    q = (q + 1) % kXcds;
    ++tried;
  }
  return -1;
}

template <typename T, int CFG>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    cgemm_grouped_kernel(const GroupProblem* __restrict__ probs, int n, int64_t total, int* __restrict__ queue) {
  using G = GroupCfg<T>;
  constexpr int BM = CFG == 0 ? G::LM : G::SM, BN = CFG == 0 ? G::LN : G::SN, BK = CFG == 0 ? G::LK : G::SK;
  using Sh = TileShape<T, BM, BN, BK, 2, 2>;
  __shared__ T smem[Sh::smem_elems];
  __shared__ int64_t s_next;
  int q = blockIdx.x % kXcds, tried = 0;   // used by thread 0 only
  if (threadIdx.x == 0) s_next = queue_grab(queue, total, q, tried);
  __syncthreads();
  int64_t t = s_next;
  while (t >= 0) {
    __syncthreads();   // every thread has read s_next
    // the next grab from the current range is issued now and resolved after
    // the tile, so its latency hides behind the tile's loads
    int pending = 0;
    if (threadIdx.x == 0 && tried < kXcds) pending = atomicAdd(&queue[q], 1);
    // problem index: how many problems start at or before tile t, less one
    // (one parallel load per 64 problems and a ballot per wave)
    int lo = -1;
    {
      const int lane = threadIdx.x & 63;
      int cnt = 0;
      for (int i0 = 0; i0 < n; i0 += 64) {
        const bool le = (i0 + lane < n) && probs[i0 + lane].tile_base <= t;
        cnt += __popcll(__ballot(le));
      }
      lo = cnt - 1;
    }
    const GroupProblem P = probs[lo];
    int64_t tm, tn;
    tile_coords(t - P.tile_base, P.tiles_m, P.tiles_n, &tm, &tn);
    TileJob<T> j;
    j.A = static_cast<const T*>(P.A);
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
    j.tblock = 0;
    j.loss = LossEpilogue();
    j.batch = 0;
    j.tile = 0;
    j.ntiles = 1;
    // the flat loader where the problem's operand extents allow it (the same
    // condition as for a plain launch); the per-row-group buffer resources else
    constexpr int kCpc = Chunk<T>::CPC;
    constexpr bool kFlatTile = 256 % (BK / kCpc) == 0 && 256 % (BN / kCpc) == 0;
    if (kFlatTile && P.flat)
      gemm_tile<T, BM, BN, BK, 2, 2, false, false, 0, 0, kFlatTile>(j, tm * BM, tn * BN, smem);
    else
      gemm_tile<T, BM, BN, BK, 2, 2, false, false, 0>(j, tm * BM, tn * BN, smem);
    if (threadIdx.x == 0) {
      int64_t nt = -1;
      if (tried < kXcds) {
        nt = queue_lo(q, total) + pending;
        if (nt >= queue_lo(q + 1, total)) {
          q = (q + 1) % kXcds;
          ++tried;
          nt = queue_grab(queue, total, q, tried);
        }
      }
      s_next = nt;
    }
    __syncthreads();
    t = s_next;
  }
}

__global__ void zero_ints_kernel(int* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// The buffer loads address a row group of RSTEP operand rows with 32-bit
// byte offsets from one base.
template <typename T, int BM, int BN, int BK, int WM, int WN, bool TA, bool TB>
bool lane_offsets_fit(int64_t lda, int64_t ldb) {
  constexpr int CPC = Chunk<T>::CPC, NT = 64 * WM * WN;
  constexpr int a_rc = (TA ? BM : BK) / CPC, b_rc = (TB ? BK : BN) / CPC;
  // rows a lane offset spans: none (wave-uniform row), a row group, or the whole slab
  constexpr int64_t a_rows = NT % a_rc == 0 ? (a_rc % 64 == 0 ? 0 : NT / a_rc) : (TA ? BK : BM);
  constexpr int64_t b_rows = NT % b_rc == 0 ? (b_rc % 64 == 0 ? 0 : NT / b_rc) : (TB ? BN : BK);
  constexpr int64_t cs = 2 * sizeof(T);
  const int64_t lim = ((int64_t)1 << 32) - 1024;
  return lda >= 0 && ldb >= 0 && (a_rows * lda + BM + BK) * cs < lim && (b_rows * ldb + BN + BK) * cs < lim;
}

template <typename T, int BM, int BN, int BK, int WM, int WN, bool TA, bool TB, int KBLK, int OCC, int BANDNW = 0>
ephw_status launch(const GemmParams& p0, hipStream_t stream) {
  const int64_t tiles_m = ceil_div(p0.M, BM), tiles_n = ceil_div(p0.N, BN);
  const int64_t ntiles = tiles_m * tiles_n;
  if (ntiles > 0x7fffffff) {
    set_error("cgemm: too many tiles");
    return EPHW_EUNSUPPORTED;
  }
  if (!lane_offsets_fit<T, BM, BN, BK, WM, WN, TA, TB>(p0.lda, p0.ldb)) {
    set_error("cgemm: leading dimension too large for 32-bit lane offsets");
    return EPHW_EUNSUPPORTED;
  }
  GemmParams p = p0;
  // the flat loader (untransposed operands, tiles whose threads load whole
  // row groups) when both operands' whole extents (per batch entry) fit
  // 32-bit byte offsets
  constexpr int kCpc = Chunk<T>::CPC, kNt = 64 * WM * WN;
  constexpr bool kFlatTile = !TA && !TB && kNt % (BK / kCpc) == 0 && kNt % (BN / kCpc) == 0;
  bool flat = false;
  if constexpr (kFlatTile) {
    constexpr int64_t cs = 2 * (int64_t)sizeof(T), lim = ((int64_t)1 << 32) - 4096;
    const int64_t a_ext = TA ? (p0.K - 1) * p0.lda + p0.M : (p0.M - 1) * p0.lda + p0.K;
    const int64_t b_ext = TB ? (p0.N - 1) * p0.ldb + p0.K : (p0.K - 1) * p0.ldb + p0.N;
    flat = (a_ext + BM + BK) * cs < lim && (b_ext + BN + BK) * cs < lim;
  }
  for (int64_t b0 = 0; b0 < p0.batch; b0 += 65535) {
    const int64_t nb = (p0.batch - b0) < 65535 ? (p0.batch - b0) : 65535;
    p.batch_base = b0;
    if (flat)
      hipLaunchKernelGGL((cgemm_kernel<T, BM, BN, BK, WM, WN, TA, TB, KBLK, OCC, BANDNW, kFlatTile>),
                         dim3((unsigned)ntiles, (unsigned)nb), dim3(64 * WM * WN), 0, stream, p, tiles_m, tiles_n);
    else
      hipLaunchKernelGGL((cgemm_kernel<T, BM, BN, BK, WM, WN, TA, TB, KBLK, OCC, BANDNW>),
                         dim3((unsigned)ntiles, (unsigned)nb), dim3(64 * WM * WN), 0, stream, p, tiles_m, tiles_n);
    EPHW_CHECK_LAUNCH();
  }
  return EPHW_OK;
}

// ---------------------------------------------------------------------------
// Few-row GEMM (M <= MB): C[M][N] (+)= op(A)[M][K] B[K][N] with B row-major
// and N large, e.g. the Eq. (9) sum of a small q batch (B = g(Re,Rp)) or
// dL/dg += Pq^H Gbar.  Such a product is a stream over B and C: each thread
// owns two adjacent columns (FP32; one for FP64), op(A) is staged in LDS in
// K chunks and read as a broadcast, and the M accumulators of each column
// stay in registers.  A 128-row MFMA tile would spend most of its work on
// padding rows here.
constexpr int kSkinnyThreads = 256, kSkinnyKC = 128;

template <typename T, int MB>
__global__ void __launch_bounds__(kSkinnyThreads) cgemm_skinny_kernel(GemmParams p) {
  constexpr int CPC = Chunk<T>::CPC;
  using V4 = typename Chunk<T>::v4;
  __shared__ T sa[2 * MB * kSkinnyKC];
  const TileJob<T> j = job_of<T>(p, p.batch_base + blockIdx.y);
  const int64_t n0 = ((int64_t)blockIdx.x * kSkinnyThreads + threadIdx.x) * CPC;
  const bool col_ok = n0 < j.N;
  const bool pair_ok = CPC == 1 || n0 + 1 < j.N;
  cplx<T> acc[MB][CPC];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int c = 0; c < CPC; ++c) acc[m][c] = cplx<T>{0, 0};
  for (int64_t k0 = 0; k0 < j.K; k0 += kSkinnyKC) {
    const int kc = (int)((j.K - k0) < kSkinnyKC ? (j.K - k0) : kSkinnyKC);
    __syncthreads();
    for (int i = threadIdx.x; i < MB * kc; i += kSkinnyThreads) {
      const int m = i / kc, kk = i % kc;
      T re = 0, im = 0;
      if (m < j.M) {
        const int64_t off = p.transA ? (k0 + kk) * j.lda + m : (int64_t)m * j.lda + k0 + kk;
        re = j.A[2 * off];
        im = j.sa * j.A[2 * off + 1];
      }
      sa[2 * (kk * MB + m)] = re;
      sa[2 * (kk * MB + m) + 1] = im;
    }
    __syncthreads();
    if (col_ok) {
      const T* brow = j.B + 2 * (k0 * j.ldb + n0);
#pragma unroll 4
      for (int kk = 0; kk < kc; ++kk) {
        T bv[2 * CPC];
        if (pair_ok) {
          const V4 v = *reinterpret_cast<const V4*>(brow + 2 * (int64_t)kk * j.ldb);
#pragma unroll
          for (int e = 0; e < 2 * CPC; ++e) bv[e] = v[e];
        } else {
          bv[0] = brow[2 * (int64_t)kk * j.ldb];
          bv[1] = brow[2 * (int64_t)kk * j.ldb + 1];
#pragma unroll
          for (int e = 2; e < 2 * CPC; ++e) bv[e] = 0;
        }
        const T* ar = sa + 2 * kk * MB;
#pragma unroll
        for (int m = 0; m < MB; ++m) {
          const cplx<T> a{ar[2 * m], ar[2 * m + 1]};
#pragma unroll
          for (int c = 0; c < CPC; ++c) cfma(acc[m][c], a, cplx<T>{bv[2 * c], bv[2 * c + 1]});
        }
      }
    }
  }
  if (!col_ok) return;
#pragma unroll
  for (int m = 0; m < MB; ++m) {
    if (m >= j.M) break;
#pragma unroll
    for (int c = 0; c < CPC; ++c) {
      if (c == 1 && !pair_ok) break;
      T* cp = j.C + 2 * ((int64_t)m * j.ldc + n0 + c);
      cplx<T> v = acc[m][c];
      if (j.accumulate) {
        v.re += cp[0];
        v.im += cp[1];
      }
      cp[0] = v.re;
      cp[1] = v.im;
    }
  }
}

template <typename T, int MB>
ephw_status launch_skinny(const GemmParams& p0, hipStream_t stream) {
  constexpr int CPC = Chunk<T>::CPC;
  const int64_t blocks = ceil_div(p0.N, (int64_t)kSkinnyThreads * CPC);
  if (blocks > 0x7fffffff) {
    set_error("cgemm: too many columns");
    return EPHW_EUNSUPPORTED;
  }
  GemmParams p = p0;
  for (int64_t b0 = 0; b0 < p0.batch; b0 += 65535) {
    const int64_t nb = (p0.batch - b0) < 65535 ? (p0.batch - b0) : 65535;
    p.batch_base = b0;
    hipLaunchKernelGGL((cgemm_skinny_kernel<T, MB>), dim3((unsigned)blocks, (unsigned)nb), dim3(kSkinnyThreads), 0,
                       stream, p);
    EPHW_CHECK_LAUNCH();
  }
  return EPHW_OK;
}

template <typename T>
ephw_status dispatch_skinny(const GemmParams& p, hipStream_t s) {
  if (p.M <= 4) return launch_skinny<T, 4>(p, s);
  if (p.M <= 8) return launch_skinny<T, 8>(p, s);
  return launch_skinny<T, 16>(p, s);
}

template <typename T, int BM, int BN, int BK, int WM, int WN, int KBLK, int OCC>
ephw_status dispatch_trans(const GemmParams& p, hipStream_t s) {
  if (!p.transA && !p.transB) return launch<T, BM, BN, BK, WM, WN, false, false, KBLK, OCC>(p, s);
  if (p.transA && !p.transB) return launch<T, BM, BN, BK, WM, WN, true, false, KBLK, OCC>(p, s);
  if (!p.transA && p.transB) return launch<T, BM, BN, BK, WM, WN, false, true, KBLK, OCC>(p, s);
  return launch<T, BM, BN, BK, WM, WN, true, true, KBLK, OCC>(p, s);
}

}  // namespace

// Tile shape of the plain kernel (no split A): the default tile, or a 64 x 224
// tile where it pads the output by at least 10% less (the band and mode
// rotations of systems with 129..224 bands or modes, e.g. 200 x 200 blocks
// pad to 256 x 224 instead of 256 x 256).
void plain_shape(int prec, int64_t M, int64_t N, int* bm, int* bn) {
  const int dm = prec == 0 ? 64 : 128, dn = prec == 0 ? 64 : 128;
  const double pad_d = (double)(ceil_div(M, dm) * dm) * (double)(ceil_div(N, dn) * dn);
  const double pad_w = (double)(ceil_div(M, 64) * 64) * (double)(ceil_div(N, 224) * 224);
  // FP32 only: 64x64 tiles for outputs that the 128x128 tile would mostly pad
  // (e.g. the Nw-wide band rotations of a few bands)
  const double pad_s = (double)(ceil_div(M, 64) * 64) * (double)(ceil_div(N, 64) * 64);
  if (prec != 0 && pad_s < 0.5 * pad_d && pad_s < 0.5 * pad_w) {
    *bm = 64;
    *bn = 64;
    return;
  }
  const bool wide = pad_w < 0.9 * pad_d;
  *bm = wide ? 64 : dm;
  *bn = wide ? 224 : dn;
}

int64_t cgemm_tiles(int prec, int64_t M, int64_t N) {
  int bm, bn;
  plain_shape(prec, M, N, &bm, &bn);
  return ceil_div(M, bm) * ceil_div(N, bn);
}

void cgemm_tile_shape(int prec, int cfg, int* bm, int* bn) {
  if (prec == 0) {
    *bm = cfg != 0 ? GroupCfg<double>::SM : GroupCfg<double>::LM;
    *bn = cfg != 0 ? GroupCfg<double>::SN : GroupCfg<double>::LN;
  } else {
    *bm = cfg != 0 ? GroupCfg<float>::SM : GroupCfg<float>::LM;
    *bn = cfg != 0 ? GroupCfg<float>::SN : GroupCfg<float>::LN;
  }
}

template <typename T>
bool grouped_fits(int64_t lda, int64_t ldb) {
  using G = GroupCfg<T>;
  return lane_offsets_fit<T, G::LM, G::LN, G::LK, 2, 2, false, false>(lda, ldb) &&
         lane_offsets_fit<T, G::SM, G::SN, G::SK, 2, 2, false, false>(lda, ldb);
}

int cgemm_grouped_blocks_per_cu(int prec, int cfg) {
  int n = 0;
  hipError_t e;
  if (prec == 0)
    e = cfg == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cgemm_grouped_kernel<double, 0>, 256, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cgemm_grouped_kernel<double, 1>, 256, 0);
  else
    e = cfg == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cgemm_grouped_kernel<float, 0>, 256, 0)
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cgemm_grouped_kernel<float, 1>, 256, 0);
  return (e == hipSuccess && n > 0) ? n : 1;
}

bool cgemm_grouped_fits(int prec, int64_t lda, int64_t ldb) {
  return prec == 0 ? grouped_fits<double>(lda, ldb) : grouped_fits<float>(lda, ldb);
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
    const int64_t cs = prec == 0 ? 16 : 8, lim = ((int64_t)1 << 32) - 4096, bk = 16;
    const int64_t a_ext = (probs[i].M - 1) * probs[i].lda + probs[i].K;
    const int64_t b_ext = (probs[i].K - 1) * probs[i].ldb + probs[i].N;
    probs[i].flat = (a_ext + bm + bk) * cs < lim && (b_ext + bn + bk) * cs < lim;
  }
  return base;
}

ephw_status cgemm_grouped(int prec, int cfg, const GroupProblem* d_probs, int n, int64_t total_tiles, int grid,
                          int* queue, hipStream_t stream) {
  if (n <= 0 || total_tiles <= 0) return EPHW_OK;
  if (grid <= 0) grid = 1;
  if (total_tiles > 0x7fffffffll) {
    set_error("cgemm_grouped: too many tiles");
    return EPHW_EUNSUPPORTED;
  }
  if (prec == 0) {
    if (cfg == 0)
      hipLaunchKernelGGL((cgemm_grouped_kernel<double, 0>), dim3(grid), dim3(256), 0, stream, d_probs, n, total_tiles,
                         queue);
    else
      hipLaunchKernelGGL((cgemm_grouped_kernel<double, 1>), dim3(grid), dim3(256), 0, stream, d_probs, n, total_tiles,
                         queue);
  } else {
    if (cfg == 0)
      hipLaunchKernelGGL((cgemm_grouped_kernel<float, 0>), dim3(grid), dim3(256), 0, stream, d_probs, n, total_tiles,
                         queue);
    else
      hipLaunchKernelGGL((cgemm_grouped_kernel<float, 1>), dim3(grid), dim3(256), 0, stream, d_probs, n, total_tiles,
                         queue);
  }
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status cgemm_grouped_reset(int* queues, int count, hipStream_t stream) {
  if (count <= 0) return EPHW_OK;
  hipLaunchKernelGGL(zero_ints_kernel, dim3((unsigned)ceil_div(count, 256)), dim3(256), 0, stream, queues, count);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

template <typename T, int BM, int BN, int BK, int WM, int WN>
bool fits_any(const GemmParams& p) {
  if (!p.transA && !p.transB) return lane_offsets_fit<T, BM, BN, BK, WM, WN, false, false>(p.lda, p.ldb);
  if (p.transA && !p.transB) return lane_offsets_fit<T, BM, BN, BK, WM, WN, true, false>(p.lda, p.ldb);
  if (!p.transA && p.transB) return lane_offsets_fit<T, BM, BN, BK, WM, WN, false, true>(p.lda, p.ldb);
  return lane_offsets_fit<T, BM, BN, BK, WM, WN, true, true>(p.lda, p.ldb);
}

// The fused epilogue always runs on the 128x128 tile (whatever tile the
// padding rule would pick for a plain store): it saves the W round trip
// through HBM and the separate band-rotation pass, more than any padding.
bool cgemm_band_fusable(int prec, int64_t M, int64_t N, int nw, int64_t lda, int64_t ldb) {
  if (prec != 1 || (nw != 4 && nw != 8) || M <= 0 || N <= 0) return false;
  return ceil_div(M, 128) * ceil_div(N, 128) <= 0x7fffffff &&
         lane_offsets_fit<float, 128, 128, 16, 2, 2, false, false>(lda, ldb);
}

// the MFMA form (Nw = 8, even Nm) sums a tile's two modes into one group of
// 128 columns; the VALU forms write one group per wave's 64 columns
int64_t cgemm_band_lw_groups(int nw, int nm, int64_t N) {
  return (nw == 8 && nm % 2 == 0) ? ceil_div(N, 128) : ceil_div(N, 64);
}

ephw_status cgemm(int prec, const GemmParams& p, hipStream_t stream) {
  if (p.M <= 0 || p.N <= 0 || p.batch <= 0) return EPHW_OK;
  if (p.band.on) {
    const BandEpilogue& b = p.band;
    if (!cgemm_band_fusable(prec, p.M, p.N, b.nw, p.lda, p.ldb) || p.compensated || p.transA || p.transB || p.conjA ||
        p.conjB || p.accumulate || p.loss.on || p.tblock != 0 || p.batch != 1 || p.M != b.nk ||
        p.N % ((int64_t)b.nm * b.nw * b.nw) != 0 || !b.Vk || (!b.Vkq && !b.kq_index)) {
      set_error("cgemm: this product cannot take the fused band epilogue");
      return EPHW_EUNSUPPORTED;
    }
    if ((b.flags & EPHW_OUT_G) && reinterpret_cast<uintptr_t>(b.g_out) % 16 != 0) {
      set_error("cgemm: the fused band epilogue stores g in 16-byte chunks (g must be 16-byte aligned)");
      return EPHW_EINVAL;
    }
    // Nw = 8 with an even mode count: every tile holds two whole modes of one
    // q, which the MFMA form of the rotations needs
    if (b.nw == 8 && b.nm % 2 == 0) return launch<float, 128, 128, 16, 2, 2, false, false, 0, 2, 16>(p, stream);
    return b.nw == 8 ? launch<float, 128, 128, 16, 2, 2, false, false, 0, 2, 8>(p, stream)
                     : launch<float, 128, 128, 16, 2, 2, false, false, 0, 2, 4>(p, stream);
  }
  if (p.K <= 0) {
    set_error("cgemm: K must be positive");
    return EPHW_EINVAL;
  }
  if (p.compensated) {
    if (prec == 0) {
      set_error("cgemm: K-blocked accumulation is an FP32 form");
      return EPHW_EINVAL;
    }
    // eight waves of 64 x 32 outputs: the second set of accumulators fits the
    // register budget of two waves per SIMD
    return dispatch_trans<float, 128, 128, 16, 2, 4, 2, 2>(p, stream);
  }
  // few rows, many columns, B read straight: a stream over B and C
  // (FP32 reads two complex values per 16-byte load: rows must start on 16 bytes)
  if (p.M <= 16 && p.N >= 16384 && !p.transB && !p.conjB && !p.loss.on && p.tblock == 0 &&
      (prec == 0 || (p.ldb % 2 == 0 && p.strideB % 2 == 0 && p.strideB1 % 2 == 0 && p.strideB2 % 2 == 0 &&
                     !p.offB && reinterpret_cast<uintptr_t>(p.B) % 16 == 0)))
    return prec == 0 ? dispatch_skinny<double>(p, stream) : dispatch_skinny<float>(p, stream);
  int bm, bn;
  plain_shape(prec, p.M, p.N, &bm, &bn);
  // the 64x224 tile addresses a whole slab from one base; very long rows
  // (e.g. g(Re,Rp) as the B operand) take the default tile instead
  bool wide = bn == 224 && (prec == 0 ? fits_any<double, 64, 224, 16, 2, 2>(p) : fits_any<float, 64, 224, 16, 4, 1>(p));
  const bool small = prec != 0 && bm == 64 && bn == 64 && fits_any<float, 64, 64, 16, 2, 2>(p);
  if (prec != 0 && bm == 64 && bn == 64 && !small && p.loss.on) {
    set_error("cgemm: leading dimension too large for the 64x64 tile's 32-bit lane offsets");
    return EPHW_EUNSUPPORTED;
  }
  if (bn == 224 && !wide && p.loss.on) {
    // the loss partials are sized by cgemm_tiles for the wide tile
    set_error("cgemm: loss epilogue with leading dimensions too large for the 64x224 tile");
    return EPHW_EUNSUPPORTED;
  }
  if (prec == 0) {
    if (wide) return dispatch_trans<double, 64, 224, 16, 2, 2, false, 1>(p, stream);
    return dispatch_trans<double, 64, 64, 8, 2, 2, false, 2>(p, stream);
  }
  if (wide) return dispatch_trans<float, 64, 224, 16, 4, 1, false, 2>(p, stream);
  if (small) return dispatch_trans<float, 64, 64, 16, 2, 2, false, 4>(p, stream);
  return dispatch_trans<float, 128, 128, 16, 2, 2, false, 2>(p, stream);
}

}  // namespace ephw
