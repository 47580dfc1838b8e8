// Mode and band rotations of Eq. (10) and the output epilogues.
//
// Mode rotation (applied once per q, before the Re sum, which it commutes
// with): G_nu(Re,q) = sum_{kappa alpha} G_{kappa alpha}(Re,q) u_{kappa alpha, nu}(q).
// Band rotation (per (k, q) pair, after the Re sum):
//   g_nu(k,q) = V(k+q)^dagger gW_nu(k,q) V(k).
// The mode rotation streams its operands once, coalesced, with u(q) in LDS
// (HBM-bound).  The band rotation (Nw <= 32) keeps V(k), V(k+q) and the
// rows of a chunk in LDS; it is HBM-bound at Nw = 8 and VALU-bound from
// Nw of about 16 up.  Larger bands use pair-stacked GEMMs instead.
#include "kernels.h"
#include "mfma.h"

namespace ephw {
namespace {

template <typename T>
__global__ void cast_kernel(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    dst[2 * i] = (T)src[2 * i];
    dst[2 * i + 1] = (T)src[2 * i + 1];
  }
}

template <typename T>
__global__ void mode_vectors_kernel(const double* __restrict__ e, int64_t nq, int nm,
                                    const double* __restrict__ ism, T* __restrict__ u) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)nm * nm;
  if (i >= nq * per) return;
  const int a = (int)((i % per) / nm);
  u[2 * i] = (T)(e[2 * i] * ism[a]);
  u[2 * i + 1] = (T)(e[2 * i + 1] * ism[a]);
}

__global__ void abs_sqrt_kernel(const double* __restrict__ lam, double* __restrict__ om, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) om[i] = sqrt(fabs(lam[i]));
}

__global__ void scale_rows_kernel(const double* __restrict__ ph, int64_t nq, const double* __restrict__ H,
                                  int64_t nr, int64_t nab, double* __restrict__ B) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nq * nr * nab) return;
  const int64_t q = i / (nr * nab), r = (i / nab) % nr, ab = i % nab;
  const cplx<double> p = ld(ph, q * nr + r), h = ld(H, r * nab + ab);
  st(B, i, cmul(p, h));
}

// One thread per (e, mn) of one q; all modes nu of that column.
constexpr int kModeReg = 24;

template <typename T>
__device__ __forceinline__ void mode_rotate_body(const T* __restrict__ G, const T* __restrict__ u,
                                                 T* __restrict__ Gnu, int64_t ne, int qb, int nm,
                                                 int64_t nw2, int q, int64_t bx, T* us) {
  const int64_t E = (int64_t)nm * nw2;
  if (u) {
    for (int i = threadIdx.x; i < nm * nm; i += blockDim.x) {
      us[2 * i] = u[2 * ((int64_t)q * nm * nm + i)];
      us[2 * i + 1] = u[2 * ((int64_t)q * nm * nm + i) + 1];
    }
    __syncthreads();
  }
  const int64_t idx = bx * blockDim.x + threadIdx.x;
  if (idx >= ne * nw2) return;
  const int64_t e = idx / nw2, mn = idx % nw2;
  const T* src = G + 2 * (((int64_t)q * ne + e) * E + mn);
  T* dst = Gnu + 2 * ((e * qb + q) * E + mn);
  if (!u) {
    for (int a = 0; a < nm; ++a) {
      dst[2 * a * nw2] = src[2 * a * nw2];
      dst[2 * a * nw2 + 1] = src[2 * a * nw2 + 1];
    }
    return;
  }
  if (nm <= kModeReg) {
    cplx<T> x[kModeReg];
#pragma unroll
    for (int a = 0; a < kModeReg; ++a)
      if (a < nm) x[a] = {src[2 * a * nw2], src[2 * a * nw2 + 1]};
    for (int v = 0; v < nm; ++v) {
      cplx<T> acc = {0, 0};
#pragma unroll
      for (int a = 0; a < kModeReg; ++a)
        if (a < nm) cfma(acc, x[a], cplx<T>{us[2 * (a * nm + v)], us[2 * (a * nm + v) + 1]});
      dst[2 * v * nw2] = acc.re;
      dst[2 * v * nw2 + 1] = acc.im;
    }
  } else {
    for (int v = 0; v < nm; ++v) {
      cplx<T> acc = {0, 0};
      for (int a = 0; a < nm; ++a)
        cfma(acc, cplx<T>{src[2 * a * nw2], src[2 * a * nw2 + 1]},
             cplx<T>{us[2 * (a * nm + v)], us[2 * (a * nm + v) + 1]});
      dst[2 * v * nw2] = acc.re;
      dst[2 * v * nw2 + 1] = acc.im;
    }
  }
}

template <typename T>
__global__ void mode_rotate_kernel(const T* __restrict__ G, const T* __restrict__ u, T* __restrict__ Gnu,
                                   int64_t ne, int qb, int nm, int64_t nw2) {
  extern __shared__ unsigned char smem_raw[];
  mode_rotate_body<T>(G, u, Gnu, ne, qb, nm, nw2, blockIdx.y, blockIdx.x, reinterpret_cast<T*>(smem_raw));
}

// The job whose [block_base, next block_base) holds block b: block_base
// ascends, so the index is the number of jobs with block_base <= b, less one.
// Each wave counts with one parallel load per 64 jobs and a ballot (no chain
// of dependent loads).
template <typename J>
__device__ __forceinline__ int find_job(const J* jobs, int n, int64_t b) {
  const int lane = threadIdx.x & 63;
  int cnt = 0;
  for (int i0 = 0; i0 < n; i0 += 64) {
    const bool le = (i0 + lane < n) && jobs[i0 + lane].block_base <= b;
    cnt += __popcll(__ballot(le));
  }
  return cnt - 1;
}

template <typename T>
__global__ void mode_rotate_grouped_kernel(const ModeRotateJob* __restrict__ jobs, int n) {
  extern __shared__ unsigned char smem_raw[];
  const int64_t b = blockIdx.x;
  const ModeRotateJob j = jobs[find_job(jobs, n, b)];
  const int64_t local = b - j.block_base;
  const int64_t per_q = ceil_div(j.ne * j.nw2, (int64_t)blockDim.x);
  mode_rotate_body<T>(static_cast<const T*>(j.G), static_cast<const T*>(j.u), static_cast<T*>(j.Gnu), j.ne,
                      j.qb, j.nm, j.nw2, (int)(local / per_q), local % per_q,
                      reinterpret_cast<T*>(smem_raw));
}

__device__ __forceinline__ double loss_weight(uint64_t seed, uint64_t index) {
  // SplitMix64 (Steele, Lea & Flood 2014): index-th output for `seed`
  uint64_t z = seed + (index + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return 0.5 + (double)(z >> 40) * 0x1p-24;
}

// Band rotation g_nu = V(k+q)^dagger X_nu V(k) for Nw <= 32, one row of one
// mode per thread.  A workgroup takes P consecutive k of one q (P pairs
// whose Nm*Nw rows fill the 256 threads) or, for larger pairs, one pair in
// chunks of nuc modes.  Per chunk:
//   1. the chunk's X rows are copied, coalesced, into LDS (rows padded to
//      Nw+1 complex values to spread the banks); in FP64 with Nw <= 8 each
//      thread reads its own row into registers instead;
//   2. thread (pair p, mode v, row m') forms T[m'][:] = X[m'][:] V(k) from
//      its own X row and V(k) (an LDS broadcast, every lane of the pair
//      reads the same element) and writes it over its X row;
//   3. after a barrier thread (p, v, m) forms g[m][:] = sum_m'
//      conj(V(k+q)[m'][m]) T[m'][:] from the mode's T rows;
//   4. epilogues: g rows staged back in LDS and stored coalesced (the P
//      pairs are consecutive k, so the workgroup writes one contiguous
//      range; FP64 with Nw <= 8 stores its rows directly), row sums of
//      |g|^2 (band sums, summed per mode in a fixed order), weighted |g|^2
//      (loss, summed per pair in a fixed order).
// NWB is Nw rounded up to a multiple of 4; the column loops are unrolled to
// NWB with a uniform guard, so the accumulators stay in registers.
constexpr int kRotThreads = 256;

template <typename T>
struct BandLds {
  T* vk;        // [P][nw2] complex
  T* vkq;       // [P][nw2] complex
  T* rows;      // [P * rows_pp][nw + 1] complex
  double* red;  // [kRotThreads]
};

template <typename T>
__device__ __forceinline__ BandLds<T> band_lds(unsigned char* smem_raw, int P, int nw, int rows_pp) {
  BandLds<T> L;
  const int nw2 = nw * nw;
  L.vk = reinterpret_cast<T*>(smem_raw);
  L.vkq = L.vk + 2 * P * nw2;
  L.rows = L.vkq + 2 * P * nw2;
  size_t off = (size_t)2 * sizeof(T) * ((size_t)2 * P * nw2 + (size_t)P * rows_pp * (nw + 1));
  off = (off + 7) & ~(size_t)7;
  L.red = reinterpret_cast<double*>(smem_raw + off);
  return L;
}

// floor(i / d) for 0 <= i < 2^22 from rd = 1.0f / d: (i + 1/2) / d lies at
// least 1/(2d) from an integer, more than the float product's error
__device__ __forceinline__ int div_rcp(int i, float rd) { return (int)(((float)i + 0.5f) * rd); }

// complex values of a 16-byte chunk: 2 at c64, 1 at c128
template <typename T>
struct Chunk16 {
  static constexpr int kVec = 16 / (2 * (int)sizeof(T));
};

// one 16-byte chunk of complex values between HBM (contiguous) and a padded
// LDS row (8-byte aligned at c64); both values of a c64 chunk share the row
template <typename T>
__device__ __forceinline__ void chunk_to_lds(const T* src, T* dst) {
  if constexpr (sizeof(T) == 4) {
    const float4 v = *reinterpret_cast<const float4*>(src);
    reinterpret_cast<float2*>(dst)[0] = make_float2(v.x, v.y);
    reinterpret_cast<float2*>(dst)[1] = make_float2(v.z, v.w);
  } else {
    *reinterpret_cast<double2*>(dst) = *reinterpret_cast<const double2*>(src);
  }
}
template <typename T>
__device__ __forceinline__ void chunk_from_lds(const T* src, T* dst) {
  if constexpr (sizeof(T) == 4) {
    const float2 a = reinterpret_cast<const float2*>(src)[0], b = reinterpret_cast<const float2*>(src)[1];
    *reinterpret_cast<float4*>(dst) = make_float4(a.x, a.y, b.x, b.y);
  } else {
    *reinterpret_cast<double2*>(dst) = *reinterpret_cast<const double2*>(src);
  }
}

template <typename T, int NWB>
__device__ __forceinline__ void band_rows_body(const BandRotateArgs& a, int P, int nuc, int64_t kblk, int iq,
                                               unsigned char* smem_raw) {
  // FP64 with Nw <= 8: X rows go straight from HBM to registers and g rows
  // straight back (measured faster there); otherwise both pass through LDS so
  // that the HBM loads and stores are coalesced
  constexpr bool DIRECT = sizeof(T) == 8 && NWB <= 8;
  const int nw = a.nw, nm = a.nm, nw2 = nw * nw, ld = nw + 1;
  const int64_t E = (int64_t)nm * nw2;
  // band window: output bands b0 .. b0+nbo-1 at k+q (rows m) and at k (columns n)
  const int b0 = a.band_n > 0 ? a.band_lo : 0, nbo = a.band_n > 0 ? a.band_n : nw, nbo2 = nbo * nbo;
  const int64_t Eo = (int64_t)nm * nbo2;   // output values per pair
  const bool rot = a.Vk != nullptr;
  const int tid = threadIdx.x;
  const bool vec_shape = E % Chunk16<T>::kVec == 0 && nw2 % Chunk16<T>::kVec == 0;
  const bool vec = vec_shape && (reinterpret_cast<uintptr_t>(a.W) & 15) == 0;               // loads
  const bool vec_g = Eo % Chunk16<T>::kVec == 0 && nbo % Chunk16<T>::kVec == 0 &&
                     (reinterpret_cast<uintptr_t>(a.g_out) & 15) == 0;                      // stores
  const int rows_pp = nuc * nw;
  const int p = tid / rows_pp, r = tid % rows_pp;
  const int vl = r / nw, mrow = r % nw;
  const int64_t ik0 = kblk * P;                                    // first local k of the block
  const int npair = (int)((a.nk_tile - ik0) < P ? (a.nk_tile - ik0) : P);
  const bool in_pair = p < npair;
  BandLds<T> L = band_lds<T>(smem_raw, P, nw, rows_pp);

  const float r_nw = 1.0f / (float)nw, r_nw2 = 1.0f / (float)nw2;
  const bool pairs = a.pair_k != nullptr;
  const int64_t nset = pairs ? a.nk_set : a.nk;   // points V and the k+q indices refer to
  if (rot) {
    const T* Vk = static_cast<const T*>(a.Vk);
    for (int i = tid; i < npair * nw2; i += kRotThreads) {
      const int pp = div_rcp(i, r_nw2), e = i - pp * nw2;
      const int64_t ik = a.k0 + ik0 + pp;
      int64_t kv = ik;   // row of V(k)
      if (pairs) {
        kv = a.pair_k[ik];
        if (kv < 0 || kv >= nset) {
          if (e == 0) atomicOr(a.status, kStatusIndex);
          kv = 0;
        }
      }
      const T* src;
      if (a.kq_index) {
        int64_t id = a.kq_index[(int64_t)iq * a.nk + ik];
        if (id < 0 || id >= nset) {
          if (e == 0) atomicOr(a.status, kStatusIndex);
          id = 0;
        }
        src = Vk + 2 * id * nw2;
      } else {
        src = static_cast<const T*>(a.Vkq) + 2 * ((int64_t)iq * a.nk + ik) * nw2;
      }
      L.vk[2 * i] = Vk[2 * (kv * nw2 + e)];
      L.vk[2 * i + 1] = Vk[2 * (kv * nw2 + e) + 1];
      L.vkq[2 * i] = src[2 * e];
      L.vkq[2 * i + 1] = src[2 * e + 1];
    }
  }
  const bool want_g = (a.flags & EPHW_OUT_G) && a.g_out;
  const bool want_t = (a.flags & EPHW_OUT_BAND_SUM) && a.band_sum;
  const bool want_l = (a.flags & EPHW_OUT_LOSS) && a.loss_partial;
  const int64_t ik_l = ik0 + p;           // this thread's local k
  const int64_t ik = a.k0 + ik_l;
  const T* W = static_cast<const T*>(a.W);
  double lsum = 0.0;

  for (int v0 = 0; v0 < nm; v0 += nuc) {
    const int nv = (nm - v0) < nuc ? (nm - v0) : nuc;
    const bool act = in_pair && vl < nv;
    // 1. X rows of the chunk -> LDS (small bands: each thread reads its own
    //    row straight into registers in step 2 instead)
    const int cw = nv * nw2;   // complex values per pair in this chunk
    // 16-byte chunks when every chunk's source offset is a multiple of the
    // chunk (E and Nw^2 are); element by element otherwise
    const int step = vec ? Chunk16<T>::kVec : 1;
    const int cpp = cw / step;
    const float r_cpp = 1.0f / (float)cpp;
    for (int i = tid; i < ((DIRECT && rot) ? 0 : npair * cpp); i += kRotThreads) {
      const int pp = div_rcp(i, r_cpp), e = (i - pp * cpp) * step;
      const int row = div_rcp(e, r_nw), col = e - row * nw;
      const T* src = W + 2 * ((ik0 + pp) * (int64_t)a.qb * E + (int64_t)iq * E + (int64_t)v0 * nw2 + e);
      T* dst = L.rows + 2 * ((pp * rows_pp + row) * ld + col);
      if (vec) {
        chunk_to_lds(src, dst);
      } else {
        dst[0] = src[0];
        dst[1] = src[1];
      }
    }
    __syncthreads();
    T* own = L.rows + 2 * (tid * ld);
    cplx<T> acc[NWB];
    if (rot) {
      // 2. T row = X row V(k)
      if (act) {
#pragma unroll
        for (int n = 0; n < NWB; ++n) acc[n] = cplx<T>{0, 0};
        const T* vkp = L.vk + 2 * p * nw2;
        if (DIRECT) {
          const T* xrow = W + 2 * (ik_l * (int64_t)a.qb * E + (int64_t)iq * E + (int64_t)(v0 + vl) * nw2 +
                                   (int64_t)mrow * nw);
          cplx<T> x[NWB];
#pragma unroll
          for (int j = 0; j < NWB; ++j) x[j] = j < nw ? cplx<T>{xrow[2 * j], xrow[2 * j + 1]} : cplx<T>{0, 0};
#pragma unroll
          for (int j = 0; j < NWB; ++j) {
            const T* vr = vkp + 2 * j * nw;
#pragma unroll
            for (int n = 0; n < NWB; ++n)
              if (j < nw && n < nbo) cfma(acc[n], x[j], cplx<T>{vr[2 * (b0 + n)], vr[2 * (b0 + n) + 1]});
          }
        } else {
          for (int j = 0; j < nw; ++j) {
            const cplx<T> x{own[2 * j], own[2 * j + 1]};
            const T* vr = vkp + 2 * j * nw;
#pragma unroll
            for (int n = 0; n < NWB; ++n)
              if (n < nbo) cfma(acc[n], x, cplx<T>{vr[2 * (b0 + n)], vr[2 * (b0 + n) + 1]});
          }
        }
#pragma unroll
        for (int n = 0; n < NWB; ++n)
          if (n < nbo) {
            own[2 * n] = acc[n].re;
            own[2 * n + 1] = acc[n].im;
          }
      }
      __syncthreads();
      // 3. g row m = sum_m' conj(V(k+q)[m'][m]) T[m'][:]  (rows of the band window)
      if (act && mrow < nbo) {
#pragma unroll
        for (int n = 0; n < NWB; ++n) acc[n] = cplx<T>{0, 0};
        const T* vq = L.vkq + 2 * p * nw2;
        const T* tb = L.rows + 2 * ((p * rows_pp + vl * nw) * ld);
        for (int j = 0; j < nw; ++j) {
          const cplx<T> c{vq[2 * (j * nw + b0 + mrow)], vq[2 * (j * nw + b0 + mrow) + 1]};
          const T* tr = tb + 2 * j * ld;
#pragma unroll
          for (int n = 0; n < NWB; ++n)
            if (n < nbo) cfmac(acc[n], c, cplx<T>{tr[2 * n], tr[2 * n + 1]});
        }
      }
    } else if (act) {
#pragma unroll
      for (int n = 0; n < NWB; ++n)
        if (n < nw) acc[n] = cplx<T>{own[2 * n], own[2 * n + 1]};
    }
    // 4. epilogues
    double rsum = 0.0;
    const bool act_o = act && mrow < nbo;   // this thread holds an output row
    if (act_o) {
      const int nu = v0 + vl;
      // element offset of (nu, b0 + mrow, b0) in the full pair, and in the output
      const int64_t eoff = (int64_t)nu * nw2 + (int64_t)(b0 + mrow) * nw + b0;
      const int64_t eoff_o = (int64_t)nu * nbo2 + (int64_t)mrow * nbo;
      if (want_g && DIRECT) {
        T* go = static_cast<T*>(a.g_out) + 2 * (((int64_t)iq * a.nk + ik) * Eo + eoff_o);
#pragma unroll
        for (int n = 0; n < NWB; ++n)
          if (n < nbo) {
            go[2 * n] = acc[n].re;
            go[2 * n + 1] = acc[n].im;
          }
      }
      uint64_t base = ((uint64_t)(a.q_global0 + iq) * (uint64_t)a.nk + (uint64_t)ik) * (uint64_t)E +
                      (uint64_t)eoff;
      if (pairs && want_l)
        base = ((uint64_t)(a.q_global0 + a.pair_q[ik]) * (uint64_t)a.nk_set + (uint64_t)a.pair_k[ik]) *
                   (uint64_t)E + (uint64_t)eoff;
#pragma unroll
      for (int n = 0; n < NWB; ++n)
        if (n < nbo) {
          const double m2 = (double)acc[n].re * (double)acc[n].re + (double)acc[n].im * (double)acc[n].im;
          rsum += m2;
          if (want_l) lsum += loss_weight(a.loss_seed, base + (uint64_t)n) * m2;
        }
    }
    if (want_g && !DIRECT) {
      // stage the g rows in LDS and store the chunk coalesced: the P pairs of
      // the workgroup are consecutive k, so their values are contiguous
      __syncthreads();   // every T row has been read
      if (act_o) {
#pragma unroll
        for (int n = 0; n < NWB; ++n)
          if (n < nbo) {
            own[2 * n] = acc[n].re;
            own[2 * n + 1] = acc[n].im;
          }
      }
      __syncthreads();
      T* go = static_cast<T*>(a.g_out) + 2 * (((int64_t)iq * a.nk + a.k0 + ik0) * Eo + (int64_t)v0 * nbo2);
      const int gstep = vec_g ? Chunk16<T>::kVec : 1;
      const int gpp = nv * nbo2 / gstep;
      const float r_gpp = 1.0f / (float)gpp, r_nbo = 1.0f / (float)nbo, r_nbo2 = 1.0f / (float)nbo2;
      for (int i = tid; i < npair * gpp; i += kRotThreads) {
        const int pp = div_rcp(i, r_gpp), e = (i - pp * gpp) * gstep;
        const int v = div_rcp(e, r_nbo2), rem = e - v * nbo2;
        const int mr = div_rcp(rem, r_nbo), col = rem - mr * nbo;
        const T* src = L.rows + 2 * ((pp * rows_pp + v * nw + mr) * ld + col);
        T* dst = go + 2 * ((int64_t)pp * Eo + e);
        if (vec_g) {
          chunk_from_lds(src, dst);
        } else {
          dst[0] = src[0];
          dst[1] = src[1];
        }
      }
    }
    if (want_t) {
      L.red[tid] = rsum;
      __syncthreads();
      // per (pair, mode): rows m = 0..nw-1 in order
      for (int t = tid; t < npair * nv; t += kRotThreads) {
        const int pp = t / nv, v = t % nv;
        const double* rr = L.red + pp * rows_pp + v * nw;
        double s = 0.0;
        for (int m = 0; m < nw; ++m) s += rr[m];
        a.band_sum[((int64_t)iq * a.nk + a.k0 + ik0 + pp) * nm + v0 + v] = s;
      }
    }
    __syncthreads();   // the rows buffer (and red) are rewritten by the next chunk
  }
  if (want_l) {
    L.red[tid] = lsum;
    __syncthreads();
    // per pair: its threads in order
    if (tid < npair) {
      const double* rr = L.red + tid * rows_pp;
      double s = 0.0;
      for (int i = 0; i < rows_pp; ++i) s += rr[i];
      a.loss_partial[(int64_t)iq * a.nk_tile + ik0 + tid] = s;
    }
  }
}

// Band rotations on the matrix cores for 8 < Nw <= 32 (no band window):
// one wavefront per (k, q) pair, looping over its modes.  Per mode the two
// complex products T = W_nu V(k) and g_nu = V(k+q)^dagger T run as 16x16
// MFMA blocks of an NP x NP problem (NP = 16 or 32, rows and columns past Nw
// zero; K steps past Nw skipped), each complex block product four real
// MFMAs per K step of 4 (the minus sign of the complex product on a negated
// operand).  T goes from the MFMA output layout to the B-operand layout of
// the second product through the wave's own LDS tile.  V(k) (B operand of the
// first product) and V(k+q)^dagger (A operand of the second) stay in
// registers for all modes of the pair.  Epilogues as in the row kernel: g
// rows stored, band sums and the pair's weighted |g|^2 summed in a fixed
// order (lane butterflies).
constexpr int kRotMfmaWaves = 4;

template <typename T, int NB>
struct RotMfmaTile {
  static constexpr int NP = 16 * NB, LDT = NP + 1;
  T t[kRotMfmaWaves][NP * LDT];   // per wave: one part of T as [NP][NP + 1]
};

template <typename T, int NB>
__device__ __forceinline__ void band_mfma_body(const BandRotateArgs& a, int64_t kblk, int iq,
                                               RotMfmaTile<T, NB>& tile) {
  using M = Mfma<T>;
  using V4 = typename M::v4;
  constexpr int NP = 16 * NB, NS = NP / 4, LDT = NP + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int64_t ik = kblk * kRotMfmaWaves + wave;   // local k of the tile (or pair)
  if (ik >= a.nk_tile) return;   // no barrier below: a whole wave leaves together
  const int nw = a.nw, nm = a.nm, nw2 = nw * nw, nsl = (nw + 3) / 4;
  const int64_t E = (int64_t)nm * nw2;
  const bool pairs = a.pair_k != nullptr;
  const int64_t nset = pairs ? a.nk_set : a.nk;
  const int64_t kl = a.k0 + ik;
  int64_t kv = kl;
  if (pairs) {
    kv = a.pair_k[kl];
    if (kv < 0 || kv >= nset) {
      if (lane == 0) atomicOr(a.status, kStatusIndex);
      kv = 0;
    }
  }
  const T* Vk = static_cast<const T*>(a.Vk);
  const T* Vq;
  if (a.kq_index) {
    int64_t id = a.kq_index[(int64_t)iq * a.nk + kl];
    if (id < 0 || id >= nset) {
      if (lane == 0) atomicOr(a.status, kStatusIndex);
      id = 0;
    }
    Vq = Vk + 2 * id * nw2;
  } else {
    Vq = static_cast<const T*>(a.Vkq) + 2 * ((int64_t)iq * a.nk + kl) * nw2;
  }
  const T* Vkk = Vk + 2 * kv * nw2;
  // V(k) as the B operand: B[kk][j] = V(k)[kk][j], kk = 4s + g, j = 16 jb + c
  T bre[NB][NS], bim[NB][NS];
  // V(k+q)^dagger as the A operand: A[i][kk] = conj(V(k+q)[kk][i]), i = 16 ib + c
  T are[NB][NS], aim[NB][NS];
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      const int kk = 4 * st + g, jj = 16 * b + c;
      const bool ok = kk < nw && jj < nw;
      bre[b][st] = ok ? Vkk[2 * (kk * nw + jj)] : T(0);
      bim[b][st] = ok ? Vkk[2 * (kk * nw + jj) + 1] : T(0);
      are[b][st] = ok ? Vq[2 * (kk * nw + jj)] : T(0);
      aim[b][st] = ok ? -Vq[2 * (kk * nw + jj) + 1] : T(0);
    }
  const T* W = static_cast<const T*>(a.W) + 2 * ((ik * (int64_t)a.qb + iq) * E);
  const int64_t pair_row = (int64_t)iq * a.nk + kl;   // row of g_out / band_sum
  const bool want_g = (a.flags & EPHW_OUT_G) && a.g_out;
  const bool want_t = (a.flags & EPHW_OUT_BAND_SUM) && a.band_sum;
  const bool want_l = (a.flags & EPHW_OUT_LOSS) && a.loss_partial;
  uint64_t lbase = 0;
  if (want_l)
    lbase = pairs ? ((uint64_t)(a.q_global0 + a.pair_q[kl]) * (uint64_t)nset + (uint64_t)kv) * (uint64_t)E
                  : ((uint64_t)(a.q_global0 + iq) * (uint64_t)a.nk + (uint64_t)kl) * (uint64_t)E;
  T* Tl = tile.t[wave];
  double lsum = 0.0;
  for (int nu = 0; nu < nm; ++nu) {
    const T* Wn = W + 2 * (int64_t)nu * nw2;
    // W_nu as the A operand: A[i][kk] = W[i][kk], i = 16 ib + c, kk = 4s + g
    T wre[NB][NS], wim[NB][NS];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int st = 0; st < NS; ++st) {
        const int ii = 16 * b + c, kk = 4 * st + g;
        const bool ok = ii < nw && kk < nw;
        wre[b][st] = ok ? Wn[2 * (ii * nw + kk)] : T(0);
        wim[b][st] = ok ? Wn[2 * (ii * nw + kk) + 1] : T(0);
      }
    // T = W V(k)
    V4 tr[NB][NB], ti[NB][NB];
#pragma unroll
    for (int ib = 0; ib < NB; ++ib)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        tr[ib][jb] = V4{0, 0, 0, 0};
        ti[ib][jb] = V4{0, 0, 0, 0};
      }
#pragma unroll
    for (int st = 0; st < NS; ++st)
      if (st < nsl)   // k steps past Nw hold zeros only
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
          tr[ib][jb] = M::op(wre[ib][st], bre[jb][st], tr[ib][jb]);
          ti[ib][jb] = M::op(wre[ib][st], bim[jb][st], ti[ib][jb]);
          tr[ib][jb] = M::op(-wim[ib][st], bim[jb][st], tr[ib][jb]);
          ti[ib][jb] = M::op(wim[ib][st], bre[jb][st], ti[ib][jb]);
        }
    // T from the output layout to the B-operand layout through the wave's LDS
    // tile, the real parts first, then the imaginary parts.  The wave's LDS
    // accesses complete in order: the fences only keep the compiler from
    // moving reads above the writes they depend on (or writes above the reads
    // of the previous part).
    T tre[NB][NS], tim[NB][NS];
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            Tl[(16 * ib + M::row(g, v)) * LDT + 16 * jb + c] = part ? ti[ib][jb][v] : tr[ib][jb][v];
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
      for (int jb = 0; jb < NB; ++jb)
#pragma unroll
        for (int st = 0; st < NS; ++st) {
          const T x = Tl[(4 * st + g) * LDT + 16 * jb + c];
          if (part) tim[jb][st] = x;
          else tre[jb][st] = x;
        }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    // g = V(k+q)^dagger T
    V4 gr[NB][NB], gi[NB][NB];
#pragma unroll
    for (int ib = 0; ib < NB; ++ib)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        gr[ib][jb] = V4{0, 0, 0, 0};
        gi[ib][jb] = V4{0, 0, 0, 0};
      }
#pragma unroll
    for (int st = 0; st < NS; ++st)
      if (st < nsl)
#pragma unroll
      for (int ib = 0; ib < NB; ++ib)
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) {
          gr[ib][jb] = M::op(are[ib][st], tre[jb][st], gr[ib][jb]);
          gi[ib][jb] = M::op(are[ib][st], tim[jb][st], gi[ib][jb]);
          gr[ib][jb] = M::op(-aim[ib][st], tim[jb][st], gr[ib][jb]);
          gi[ib][jb] = M::op(aim[ib][st], tre[jb][st], gi[ib][jb]);
        }
    // epilogues of the mode
    double tsum = 0.0;
#pragma unroll
    for (int ib = 0; ib < NB; ++ib)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = 16 * ib + M::row(g, v), n = 16 * jb + c;
          if (m < nw && n < nw) {
            const T re = gr[ib][jb][v], im = gi[ib][jb][v];
            const int64_t e = (int64_t)nu * nw2 + (int64_t)m * nw + n;
            if (want_g) {
              T* go = static_cast<T*>(a.g_out) + 2 * (pair_row * E + e);
              go[0] = re;
              go[1] = im;
            }
            const double m2 = (double)re * (double)re + (double)im * (double)im;
            tsum += m2;
            if (want_l) lsum += loss_weight(a.loss_seed, lbase + (uint64_t)e) * m2;
          }
        }
    if (want_t) {
      for (int off = 32; off > 0; off >>= 1) tsum += __shfl_xor(tsum, off, 64);
      if (lane == 0) a.band_sum[pair_row * nm + nu] = tsum;
    }
  }
  if (want_l) {
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (lane == 0) a.loss_partial[(int64_t)iq * a.nk_tile + ik] = lsum;
  }
}

// FP32 at Nw <= 16: six waves per SIMD instead of the five the compiler
// would pick (a few more registers spilled, 4 % faster at Nw = 12)
#define EPHW_ROT_MFMA_WAVES(T, NB) __attribute__((amdgpu_waves_per_eu(NB == 1 && sizeof(T) == 4 ? 6 : 1, 8)))

template <typename T, int NB>
__global__ void __launch_bounds__(64 * kRotMfmaWaves) EPHW_ROT_MFMA_WAVES(T, NB)
    band_rotate_mfma_kernel(BandRotateArgs a) {
  __shared__ RotMfmaTile<T, NB> tile;
  band_mfma_body<T, NB>(a, blockIdx.x, blockIdx.y, tile);
}

template <typename T, int NB>
__global__ void __launch_bounds__(64 * kRotMfmaWaves) EPHW_ROT_MFMA_WAVES(T, NB) band_rotate_mfma_grouped_kernel(
    const BandRotateJob* __restrict__ jobs, int n) {
  __shared__ RotMfmaTile<T, NB> tile;
  const int64_t b = blockIdx.x;
  const BandRotateJob j = jobs[find_job(jobs, n, b)];
  const int64_t local = b - j.block_base;
  const int64_t kb = ceil_div(j.args.nk_tile, (int64_t)kRotMfmaWaves);
  band_mfma_body<T, NB>(j.args, local % kb, (int)(local / kb), tile);
}

template <typename T, int NWB>
__global__ void __launch_bounds__(kRotThreads) band_rotate_kernel(BandRotateArgs a, int P, int nuc) {
  extern __shared__ unsigned char smem_raw[];
  band_rows_body<T, NWB>(a, P, nuc, blockIdx.x, blockIdx.y, smem_raw);
}

template <typename T, int NWB>
__global__ void __launch_bounds__(kRotThreads) band_rotate_grouped_kernel(const BandRotateJob* __restrict__ jobs,
                                                                          int n) {
  extern __shared__ unsigned char smem_raw[];
  const int64_t b = blockIdx.x;
  const BandRotateJob j = jobs[find_job(jobs, n, b)];   // by value: the fields stay in registers
  const int64_t local = b - j.block_base;
  const int64_t kb = ceil_div(j.args.nk_tile, (int64_t)j.P);
  band_rows_body<T, NWB>(j.args, j.P, j.nuc, local % kb, (int)(local / kb), smem_raw);
}

// out += sum of x[0..n) by one workgroup of kSumThreads, in a fixed order:
// thread t sums x[t + kSumThreads (4 j + r)] into four partial sums r (four
// independent load streams), then the workgroup adds them in a tree.
constexpr int kSumThreads = 1024;

__device__ __forceinline__ void block_sum_into(const double* __restrict__ x, int64_t n, double* __restrict__ out,
                                               double* red) {
  const int t = threadIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t i = t;
  for (; i + 3 * kSumThreads < n; i += 4 * kSumThreads) {
    s0 += x[i];
    s1 += x[i + kSumThreads];
    s2 += x[i + 2 * kSumThreads];
    s3 += x[i + 3 * kSumThreads];
  }
  for (; i < n; i += kSumThreads) s0 += x[i];
  red[t] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  for (int w = kSumThreads / 2; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0 && n > 0) out[0] += red[0];
}

__global__ void __launch_bounds__(kSumThreads) sum_into_kernel(const double* __restrict__ x, int64_t n,
                                                               double* __restrict__ out) {
  __shared__ double red[kSumThreads];
  block_sum_into(x, n, out, red);
}

__global__ void gather_rows_kernel(const double* __restrict__ src, int64_t nsrc,
                                   const int32_t* __restrict__ idx, int64_t cnt, int w,
                                   double* __restrict__ dst, uint32_t* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt * w) return;
  const int64_t r = i / w, c = i % w;
  int64_t j = idx[r];
  if (j < 0 || j >= nsrc) {
    if (c == 0) atomicOr(status, kStatusIndex);
    j = 0;
  }
  dst[i] = src[j * w + c];
}

inline unsigned grid1(int64_t n, int bs) { return (unsigned)ceil_div(n, bs); }

}  // namespace

ephw_status cast_complex(int prec, const double* src, void* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return EPHW_OK;
  if (prec == 0) {
    EPHW_HIP(hipMemcpyAsync(dst, src, (size_t)n * 16, hipMemcpyDeviceToDevice, s));
    return EPHW_OK;
  }
  hipLaunchKernelGGL(cast_kernel<float>, dim3(grid1(n, 256)), dim3(256), 0, s, src,
                     static_cast<float*>(dst), n);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status mode_vectors(int prec, const double* e, int64_t nq, int nm, const double* ism, void* u,
                         hipStream_t s) {
  const int64_t n = nq * nm * nm;
  if (n <= 0) return EPHW_OK;
  if (prec == 0)
    hipLaunchKernelGGL(mode_vectors_kernel<double>, dim3(grid1(n, 256)), dim3(256), 0, s, e, nq, nm,
                       ism, static_cast<double*>(u));
  else
    hipLaunchKernelGGL(mode_vectors_kernel<float>, dim3(grid1(n, 256)), dim3(256), 0, s, e, nq, nm,
                       ism, static_cast<float*>(u));
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status abs_sqrt(const double* lam, double* omega, int64_t n, hipStream_t s) {
  if (n <= 0) return EPHW_OK;
  hipLaunchKernelGGL(abs_sqrt_kernel, dim3(grid1(n, 256)), dim3(256), 0, s, lam, omega, n);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status scale_rows_by_phase(const double* phase, int64_t nq, const double* H, int64_t nr,
                                int64_t nab, double* B, hipStream_t s) {
  const int64_t n = nq * nr * nab;
  if (n <= 0) return EPHW_OK;
  hipLaunchKernelGGL(scale_rows_kernel, dim3(grid1(n, 256)), dim3(256), 0, s, phase, nq, H, nr, nab, B);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status mode_rotate(int prec, const void* G, const void* u, void* Gnu, int64_t ne, int qb, int nm,
                        int64_t nw2, hipStream_t s) {
  const int64_t cols = ne * nw2;
  if (cols <= 0 || qb <= 0) return EPHW_OK;
  const int bs = 256;
  const size_t lds = u ? (size_t)nm * nm * 2 * (prec == 0 ? 8 : 4) : 0;
  if (prec == 0)
    hipLaunchKernelGGL(mode_rotate_kernel<double>, dim3(grid1(cols, bs), qb), dim3(bs), lds, s,
                       static_cast<const double*>(G), static_cast<const double*>(u),
                       static_cast<double*>(Gnu), ne, qb, nm, nw2);
  else
    hipLaunchKernelGGL(mode_rotate_kernel<float>, dim3(grid1(cols, bs), qb), dim3(bs), lds, s,
                       static_cast<const float*>(G), static_cast<const float*>(u),
                       static_cast<float*>(Gnu), ne, qb, nm, nw2);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

namespace {

size_t band_lds_bytes(int prec, int nw, int P, int nuc) {
  const size_t cs = prec == 0 ? 16 : 8;
  size_t b = cs * ((size_t)2 * P * nw * nw + (size_t)P * nuc * nw * (nw + 1));
  b = (b + 7) & ~(size_t)7;
  return b + 8 * kRotThreads;
}

template <typename T>
using BandKernel = void (*)(BandRotateArgs, int, int);
template <typename T>
using BandGroupedKernel = void (*)(const BandRotateJob*, int);

template <typename T>
BandKernel<T> band_kernel(int nwb) {
  switch (nwb) {
    case 4: return band_rotate_kernel<T, 4>;
    case 8: return band_rotate_kernel<T, 8>;
    case 12: return band_rotate_kernel<T, 12>;
    case 16: return band_rotate_kernel<T, 16>;
    case 20: return band_rotate_kernel<T, 20>;
    case 24: return band_rotate_kernel<T, 24>;
    case 28: return band_rotate_kernel<T, 28>;
    default: return band_rotate_kernel<T, 32>;
  }
}
template <typename T>
BandGroupedKernel<T> band_grouped_kernel(int nwb) {
  switch (nwb) {
    case -16: return band_rotate_mfma_grouped_kernel<T, 1>;
    case -32: return band_rotate_mfma_grouped_kernel<T, 2>;
    case 4: return band_rotate_grouped_kernel<T, 4>;
    case 8: return band_rotate_grouped_kernel<T, 8>;
    case 12: return band_rotate_grouped_kernel<T, 12>;
    case 16: return band_rotate_grouped_kernel<T, 16>;
    case 20: return band_rotate_grouped_kernel<T, 20>;
    case 24: return band_rotate_grouped_kernel<T, 24>;
    case 28: return band_rotate_grouped_kernel<T, 28>;
    default: return band_rotate_grouped_kernel<T, 32>;
  }
}

BandPlan band_rows_plan(int prec, int nw, int nm) {
  BandPlan pl;
  const int rows = nm * nw;
  if (rows <= kRotThreads) {
    pl.nuc = nm;
    pl.P = kRotThreads / rows;
  } else {
    pl.nuc = kRotThreads / nw;
    pl.P = 1;
  }
  // fit 64 KB of LDS (several workgroups per CU); if that leaves fewer than
  // 128 busy threads, use up to 160 KB instead
  for (size_t cap : {(size_t)65536, (size_t)163840}) {
    int P = pl.P, nuc = pl.nuc;
    while (band_lds_bytes(prec, nw, P, nuc) > cap && (P > 1 || nuc > 1)) {
      if (P > 1) --P; else --nuc;
    }
    if (band_lds_bytes(prec, nw, P, nuc) <= cap && (P * nuc * nw >= 128 || cap > 65536)) {
      pl.P = P;
      pl.nuc = nuc;
      break;
    }
  }
  pl.lds = band_lds_bytes(prec, nw, pl.P, pl.nuc);
  return pl;
}

}  // namespace

bool band_rotate_on_mfma(int nw) { return nw > 8 && nw <= 32; }

int band_rotate_class(int nw) {
  if (band_rotate_on_mfma(nw)) return nw <= 16 ? -16 : -32;
  return 4 * (int)ceil_div(nw, 4);
}

BandPlan band_rotate_plan(int prec, int nw, int nm) {
  if (band_rotate_on_mfma(nw)) {
    BandPlan pl;
    pl.P = kRotMfmaWaves;
    pl.nuc = nm;
    pl.lds = 0;
    return pl;
  }
  return band_rows_plan(prec, nw, nm);
}


ephw_status band_rotate(int prec, const BandRotateArgs& a, hipStream_t s) {
  if (a.nk_tile <= 0 || a.qb <= 0) return EPHW_OK;
  if (a.nw > 32 || a.nw < 1) {
    set_error("band_rotate: this kernel handles 1 <= nw <= 32");
    return EPHW_EUNSUPPORTED;
  }
  if (a.band_n > 0 && (!a.Vk || a.band_lo < 0 || a.band_lo + a.band_n > a.nw)) {
    set_error("band_rotate: the band window needs the rotations and 0 <= band_lo, band_lo + band_n <= nw");
    return EPHW_EINVAL;
  }
  if (band_rotate_on_mfma(a.nw) && a.Vk && a.band_n == 0) {
    const int64_t nbk = ceil_div(a.nk_tile, (int64_t)kRotMfmaWaves);
    if (nbk > 0x7fffffff || a.qb > 65535) {
      set_error("band_rotate: grid too large");
      return EPHW_EUNSUPPORTED;
    }
    const dim3 grid((unsigned)nbk, (unsigned)a.qb), block(64 * kRotMfmaWaves);
    if (prec == 0) {
      if (a.nw <= 16) hipLaunchKernelGGL((band_rotate_mfma_kernel<double, 1>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((band_rotate_mfma_kernel<double, 2>), grid, block, 0, s, a);
    } else {
      if (a.nw <= 16) hipLaunchKernelGGL((band_rotate_mfma_kernel<float, 1>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((band_rotate_mfma_kernel<float, 2>), grid, block, 0, s, a);
    }
    EPHW_CHECK_LAUNCH();
    return EPHW_OK;
  }
  const BandPlan pl = band_rows_plan(prec, a.nw, a.nm);
  const int64_t kb = ceil_div(a.nk_tile, (int64_t)pl.P);
  if (kb > 0x7fffffff || a.qb > 65535) {
    set_error("band_rotate: grid too large");
    return EPHW_EUNSUPPORTED;
  }
  const int nwb = 4 * (int)ceil_div(a.nw, 4);
  if (prec == 0) {
    auto k = band_kernel<double>(nwb);
    if (pl.lds > 65536)
      EPHW_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds));
    hipLaunchKernelGGL(k, dim3((unsigned)kb, a.qb), dim3(kRotThreads), pl.lds, s, a, pl.P, pl.nuc);
  } else {
    auto k = band_kernel<float>(nwb);
    if (pl.lds > 65536)
      EPHW_HIP(hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pl.lds));
    hipLaunchKernelGGL(k, dim3((unsigned)kb, a.qb), dim3(kRotThreads), pl.lds, s, a, pl.P, pl.nuc);
  }
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status gather_rows(const double* src, int64_t nsrc, const int32_t* idx, int64_t cnt, int w,
                        double* dst, uint32_t* status, hipStream_t s) {
  if (cnt <= 0 || w <= 0) return EPHW_OK;
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid1(cnt * w, 256)), dim3(256), 0, s, src, nsrc, idx,
                     cnt, w, dst, status);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status mode_rotate_grouped(int prec, const ModeRotateJob* d_jobs, int n, int64_t blocks, size_t lds,
                                hipStream_t s) {
  if (n <= 0 || blocks <= 0) return EPHW_OK;
  if (prec == 0)
    hipLaunchKernelGGL(mode_rotate_grouped_kernel<double>, dim3((unsigned)blocks), dim3(256), lds, s, d_jobs, n);
  else
    hipLaunchKernelGGL(mode_rotate_grouped_kernel<float>, dim3((unsigned)blocks), dim3(256), lds, s, d_jobs, n);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status band_rotate_grouped_prepare(int prec, int nwb, size_t lds) {
  if (lds <= 65536) return EPHW_OK;
  if (prec == 0)
    EPHW_HIP(hipFuncSetAttribute((const void*)band_grouped_kernel<double>(nwb),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  else
    EPHW_HIP(hipFuncSetAttribute((const void*)band_grouped_kernel<float>(nwb),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return EPHW_OK;
}

ephw_status band_rotate_grouped(int prec, int nwb, const BandRotateJob* d_jobs, int n, int64_t blocks, size_t lds,
                                hipStream_t s) {
  if (n <= 0 || blocks <= 0) return EPHW_OK;
  if (prec == 0)
    hipLaunchKernelGGL(band_grouped_kernel<double>(nwb), dim3((unsigned)blocks), dim3(kRotThreads), lds, s, d_jobs,
                       n);
  else
    hipLaunchKernelGGL(band_grouped_kernel<float>(nwb), dim3((unsigned)blocks), dim3(kRotThreads), lds, s, d_jobs,
                       n);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

__global__ void __launch_bounds__(kSumThreads) sum_into_grouped_kernel(const SumJob* __restrict__ jobs) {
  __shared__ double red[kSumThreads];
  const SumJob j = jobs[blockIdx.x];
  block_sum_into(j.x, j.n, j.out, red);
}

ephw_status sum_into_grouped(const SumJob* d_jobs, int n, hipStream_t s) {
  if (n <= 0) return EPHW_OK;
  hipLaunchKernelGGL(sum_into_grouped_kernel, dim3((unsigned)n), dim3(kSumThreads), 0, s, d_jobs);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status sum_into(const double* x, int64_t n, double* out, hipStream_t s) {
  if (n <= 0) return EPHW_OK;
  hipLaunchKernelGGL(sum_into_kernel, dim3(1), dim3(kSumThreads), 0, s, x, n, out);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

}  // namespace ephw
