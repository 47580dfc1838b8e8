// Mode and band rotations of Eq. (10) and the output epilogues.
//
// Mode rotation (applied once per q, before the Re sum, which it commutes
// with): G_nu(Re,q) = sum_{kappa alpha} G_{kappa alpha}(Re,q) u_{kappa alpha, nu}(q).
// Band rotation (per (k, q) pair, after the Re sum):
//   g_nu(k,q) = V(k+q)^dagger gW_nu(k,q) V(k).
// Both are bandwidth-bound at the sizes of the stock workloads: the kernels
// stream their operands once, coalesced, with the small matrices in LDS.
#include "kernels.h"

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

// find the job whose [block_base, next block_base) holds block b
template <typename J>
__device__ __forceinline__ int find_job(const J* jobs, int n, int64_t b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block_base <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <typename T>
__global__ void mode_rotate_grouped_kernel(const ModeRotateJob* __restrict__ jobs, int n) {
  extern __shared__ unsigned char smem_raw[];
  const int64_t b = blockIdx.x;
  const ModeRotateJob& j = jobs[find_job(jobs, n, b)];
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

// One workgroup per (k, q) pair.  LDS: V(k), V(k+q), then chunks of nu
// matrices: X (the Re sums) and Tmp = X V(k).
constexpr int kRotThreads = 256;

template <typename T>
__device__ __forceinline__ void band_rotate_body(const BandRotateArgs& a, int nuc, int64_t ik_local,
                                                 int iq, unsigned char* smem_raw) {
  const int nw = a.nw, nm = a.nm;
  const int nw2 = nw * nw;
  const int64_t ik = a.k0 + ik_local;   // global k index
  const int64_t E = (int64_t)nm * nw2;
  const bool rot = a.Vk != nullptr;
  T* vk = reinterpret_cast<T*>(smem_raw);            // [nw][nw]
  T* vkq = vk + 2 * nw2;                              // [nw][nw]
  T* xs = vkq + 2 * nw2;                              // [nuc][nw][nw]
  T* ts = xs + 2 * nuc * nw2;                         // [nuc][nw][nw]
  double* m2s = reinterpret_cast<double*>(ts + 2 * nuc * nw2);  // [nuc][nw][nw] |y|^2
  double* red = m2s + nuc * nw2;                      // [kRotThreads/64]
  const int tid = threadIdx.x;

  if (rot) {
    const T* Vk = static_cast<const T*>(a.Vk);
    int64_t jk;
    const T* src;
    if (a.kq_index) {
      int64_t id = a.kq_index[(int64_t)iq * a.nk + ik];
      if (id < 0 || id >= a.nk) {
        if (tid == 0) atomicOr(a.status, kStatusIndex);
        id = 0;
      }
      jk = id;
      src = Vk + 2 * jk * nw2;
    } else {
      src = static_cast<const T*>(a.Vkq) + 2 * ((int64_t)iq * a.nk + ik) * nw2;
    }
    for (int i = tid; i < nw2; i += kRotThreads) {
      vk[2 * i] = Vk[2 * (ik * nw2 + i)];
      vk[2 * i + 1] = Vk[2 * (ik * nw2 + i) + 1];
      vkq[2 * i] = src[2 * i];
      vkq[2 * i + 1] = src[2 * i + 1];
    }
  }
  const T* W = static_cast<const T*>(a.W) + 2 * (ik_local * (int64_t)a.qb * E + (int64_t)iq * E);
  T* gout = a.g_out ? static_cast<T*>(a.g_out) + 2 * (((int64_t)iq * a.nk + ik) * E) : nullptr;
  const bool want_g = (a.flags & EPHW_OUT_G) && gout;
  const bool want_t = (a.flags & EPHW_OUT_BAND_SUM) && a.band_sum;
  const bool want_l = (a.flags & EPHW_OUT_LOSS) && a.loss_partial;
  const uint64_t pair_base =
      ((uint64_t)(a.q_global0 + iq) * (uint64_t)a.nk + (uint64_t)ik) * (uint64_t)E;
  double lsum = 0.0;

  for (int v0 = 0; v0 < nm; v0 += nuc) {
    const int nv = (nm - v0) < nuc ? (nm - v0) : nuc;
    __syncthreads();
    for (int i = tid; i < nv * nw2; i += kRotThreads) {
      xs[2 * i] = W[2 * ((int64_t)v0 * nw2 + i)];
      xs[2 * i + 1] = W[2 * ((int64_t)v0 * nw2 + i) + 1];
    }
    __syncthreads();
    if (rot) {
      // Tmp[v][m'][n] = sum_n' X[v][m'][n'] V(k)[n'][n]
      for (int i = tid; i < nv * nw2; i += kRotThreads) {
        const int v = i / nw2, r = (i / nw) % nw, c = i % nw;
        cplx<T> acc = {0, 0};
        const T* xr = xs + 2 * (v * nw2 + r * nw);
        for (int j = 0; j < nw; ++j)
          cfma(acc, cplx<T>{xr[2 * j], xr[2 * j + 1]}, cplx<T>{vk[2 * (j * nw + c)], vk[2 * (j * nw + c) + 1]});
        ts[2 * i] = acc.re;
        ts[2 * i + 1] = acc.im;
      }
      __syncthreads();
    }
    // Y[v][m][n] = sum_m' conj(V(k+q)[m'][m]) Tmp[v][m'][n]
    for (int i = tid; i < nv * nw2; i += kRotThreads) {
      const int v = i / nw2, r = (i / nw) % nw, c = i % nw;
      cplx<T> y;
      if (rot) {
        y = {0, 0};
        const T* tc = ts + 2 * (v * nw2 + c);
        for (int j = 0; j < nw; ++j)
          cfmac(y, cplx<T>{vkq[2 * (j * nw + r)], vkq[2 * (j * nw + r) + 1]},
                cplx<T>{tc[2 * j * nw], tc[2 * j * nw + 1]});
      } else {
        y = {xs[2 * i], xs[2 * i + 1]};
      }
      const int64_t eidx = (int64_t)v0 * nw2 + i;
      if (want_g) {
        gout[2 * eidx] = y.re;
        gout[2 * eidx + 1] = y.im;
      }
      const double m2 = (double)y.re * (double)y.re + (double)y.im * (double)y.im;
      if (want_t) m2s[i] = m2;
      if (want_l) lsum += loss_weight(a.loss_seed, pair_base + (uint64_t)eidx) * m2;
    }
    if (want_t) {
      __syncthreads();
      // fixed-order sum of |y|^2 over (m, n) for every mode of the chunk
      for (int v = tid; v < nv; v += kRotThreads) {
        const double* m2 = m2s + v * nw2;
        double s = 0.0;
        for (int i = 0; i < nw2; ++i) s += m2[i];
        a.band_sum[((int64_t)iq * a.nk + ik) * nm + v0 + v] = s;
      }
    }
  }
  if (want_l) {
    double* wred = red;
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off, 64);
    __syncthreads();
    if ((tid & 63) == 0) wred[tid >> 6] = lsum;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < kRotThreads / 64; ++w) s += wred[w];
      a.loss_partial[(int64_t)iq * a.nk_tile + ik_local] = s;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kRotThreads) band_rotate_kernel(BandRotateArgs a, int nuc) {
  extern __shared__ unsigned char smem_raw[];
  band_rotate_body<T>(a, nuc, blockIdx.x, blockIdx.y, smem_raw);
}

template <typename T>
__global__ void __launch_bounds__(kRotThreads) band_rotate_grouped_kernel(const BandRotateJob* __restrict__ jobs,
                                                                          int n) {
  extern __shared__ unsigned char smem_raw[];
  const int64_t b = blockIdx.x;
  const BandRotateJob& j = jobs[find_job(jobs, n, b)];
  const int64_t local = b - j.block_base;
  band_rotate_body<T>(j.args, j.nuc, local % j.args.nk_tile, (int)(local / j.args.nk_tile), smem_raw);
}

__global__ void sum_into_kernel(const double* __restrict__ x, int64_t n, double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] += red[0];
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

int band_rotate_modes_per_chunk(int prec, int nw, int nm, size_t* lds_bytes) {
  const size_t esz = 2 * (prec == 0 ? 8 : 4);
  const size_t nw2 = (size_t)nw * nw;
  const size_t fixed = esz * 2 * nw2 + 8 * (kRotThreads / 64);
  const size_t per_mode = (2 * esz + 8) * nw2;
  int nuc = fixed + per_mode <= 65536 ? (int)((65536 - fixed) / per_mode) : 1;
  if (nuc > nm) nuc = nm;
  if (lds_bytes) *lds_bytes = fixed + per_mode * (size_t)nuc;
  return nuc;
}

ephw_status band_rotate(int prec, const BandRotateArgs& a, hipStream_t s) {
  if (a.nk_tile <= 0 || a.qb <= 0) return EPHW_OK;
  if (a.nw > 32) {
    set_error("band_rotate: this kernel handles nw <= 32");
    return EPHW_EUNSUPPORTED;
  }
  const size_t esz = 2 * (prec == 0 ? 8 : 4);
  const int nw2 = a.nw * a.nw;
  // chunk of modes so that V(k), V(k+q), X, Tmp and |y|^2 fit in 64 KB of LDS
  const size_t fixed = esz * 2 * nw2 + 8 * (kRotThreads / 64);
  const size_t per_mode = (2 * esz + 8) * nw2;
  int nuc = fixed + per_mode <= 65536 ? (int)((65536 - fixed) / per_mode) : 1;
  if (nuc > a.nm) nuc = a.nm;
  const size_t lds = fixed + per_mode * (size_t)nuc;
  if (lds > 65536) {
    // large FP64 bands: use the bigger LDS of gfx950 (160 KB per workgroup)
    if (prec == 0)
      EPHW_HIP(hipFuncSetAttribute((const void*)band_rotate_kernel<double>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    else
      EPHW_HIP(hipFuncSetAttribute((const void*)band_rotate_kernel<float>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  }
  if (a.nk_tile > 0x7fffffff || a.qb > 65535) {
    set_error("band_rotate: grid too large");
    return EPHW_EUNSUPPORTED;
  }
  if (prec == 0)
    hipLaunchKernelGGL(band_rotate_kernel<double>, dim3((unsigned)a.nk_tile, a.qb), dim3(kRotThreads), lds,
                       s, a, nuc);
  else
    hipLaunchKernelGGL(band_rotate_kernel<float>, dim3((unsigned)a.nk_tile, a.qb), dim3(kRotThreads), lds,
                       s, a, nuc);
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

ephw_status band_rotate_grouped_prepare(int prec, size_t lds) {
  if (lds <= 65536) return EPHW_OK;
  if (prec == 0)
    EPHW_HIP(hipFuncSetAttribute((const void*)band_rotate_grouped_kernel<double>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  else
    EPHW_HIP(hipFuncSetAttribute((const void*)band_rotate_grouped_kernel<float>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  return EPHW_OK;
}

ephw_status band_rotate_grouped(int prec, const BandRotateJob* d_jobs, int n, int64_t blocks, size_t lds,
                                hipStream_t s) {
  if (n <= 0 || blocks <= 0) return EPHW_OK;
  if (prec == 0)
    hipLaunchKernelGGL(band_rotate_grouped_kernel<double>, dim3((unsigned)blocks), dim3(kRotThreads), lds, s,
                       d_jobs, n);
  else
    hipLaunchKernelGGL(band_rotate_grouped_kernel<float>, dim3((unsigned)blocks), dim3(kRotThreads), lds, s,
                       d_jobs, n);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

__global__ void sum_into_grouped_kernel(const SumJob* __restrict__ jobs) {
  __shared__ double red[256];
  const SumJob& j = jobs[blockIdx.x];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < j.n; i += 256) s += j.x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && j.n > 0) j.out[0] += red[0];
}

ephw_status sum_into_grouped(const SumJob* d_jobs, int n, hipStream_t s) {
  if (n <= 0) return EPHW_OK;
  hipLaunchKernelGGL(sum_into_grouped_kernel, dim3((unsigned)n), dim3(256), 0, s, d_jobs);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status sum_into(const double* x, int64_t n, double* out, hipStream_t s) {
  if (n <= 0) return EPHW_OK;
  hipLaunchKernelGGL(sum_into_kernel, dim3(1), dim3(256), 0, s, x, n, out);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

}  // namespace ephw
