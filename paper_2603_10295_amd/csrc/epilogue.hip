// Gauge-invariant |g|^2 of every pair (the epilogue behind the comparison of
// interpolated matrix elements): eigenvectors of (near-)degenerate
// eigenvalues are defined only up to a unitary mixing inside their block, so
// |g_{mn nu}|^2 is gauge free only once summed over the blocks of m (bands at
// k+q), n (bands at k) and nu (modes at q).  Element (nu, m, n) of the output
// is that block sum, written to every element of the block.  A block is a run
// of ascending eigenvalues whose consecutive gaps are at most
// rel_tol * max(1, max |value|) of their list.
//
// One 64-lane wavefront per pair: the lanes first find each index's block
// bounds (kept in LDS), then sum |g|^2 over the block of each element.
//
// The same file holds a downstream reduction of |g|^2 over q, the
// phonon-limited linewidth of each state (below).
#include "kernels.h"

namespace ephw {
namespace {

constexpr int kDegWaves = 4;  // pairs (wavefronts) per workgroup

__device__ double list_tol(const double* v, int n, double rel_tol) {
  double m = 1.0;
  for (int i = 0; i < n; ++i) m = fmax(m, fabs(v[i]));
  return rel_tol * m;
}

__device__ void block_bounds(const double* v, int n, double tol, int i, int* lo, int* hi) {
  int a = i, b = i;
  while (a > 0 && v[a] - v[a - 1] <= tol) --a;
  while (b < n - 1 && v[b + 1] - v[b] <= tol) ++b;
  lo[i] = a;
  hi[i] = b;
}

template <typename T>
__global__ void __launch_bounds__(64 * kDegWaves)
    degenerate_sums_kernel(const T* __restrict__ g, int64_t npairs, int64_t nk, int nm, int nw,
                           const double* __restrict__ eps_kq, const double* __restrict__ eps_k,
                           const double* __restrict__ lam, double rel_tol, double* __restrict__ out) {
  extern __shared__ int dlds[];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t pair = (int64_t)blockIdx.x * kDegWaves + wave;   // q-major
  if (pair >= npairs) return;
  const int64_t iq = pair / nk, ik = pair - iq * nk;
  int* lo_m = dlds + wave * (4 * nw + 2 * nm);
  int* hi_m = lo_m + nw;
  int* lo_n = hi_m + nw;
  int* hi_n = lo_n + nw;
  int* lo_v = hi_n + nw;
  int* hi_v = lo_v + nm;
  const double* em = eps_kq + pair * nw;
  const double* en = eps_k + ik * nw;
  const double* ev = lam + iq * nm;
  const double tm = list_tol(em, nw, rel_tol), tn = list_tol(en, nw, rel_tol), tv = list_tol(ev, nm, rel_tol);
  for (int i = lane; i < nw; i += 64) {
    block_bounds(em, nw, tm, i, lo_m, hi_m);
    block_bounds(en, nw, tn, i, lo_n, hi_n);
  }
  for (int i = lane; i < nm; i += 64) block_bounds(ev, nm, tv, i, lo_v, hi_v);
  wave_sync();
  const int nw2 = nw * nw;
  const int64_t E = (int64_t)nm * nw2;
  const T* gp = g + 2 * pair * E;
  double* op = out + pair * E;
  for (int64_t e = lane; e < E; e += 64) {
    const int nu = (int)(e / nw2), rem = (int)(e - (int64_t)nu * nw2), m = rem / nw, n = rem - m * nw;
    double s = 0.0;
    for (int v = lo_v[nu]; v <= hi_v[nu]; ++v)
      for (int a = lo_m[m]; a <= hi_m[m]; ++a)
        for (int b = lo_n[n]; b <= hi_n[n]; ++b) {
          const int64_t i = ((int64_t)v * nw + a) * nw + b;
          const double x = (double)gp[2 * i], y = (double)gp[2 * i + 1];
          s += x * x + y * y;
        }
    op[e] = s;
  }
}

// Phonon-limited linewidth of the states n at k (imaginary part of the
// Fan-Migdal self-energy, Gaussian broadening):
//   gamma[k][n] += scale * sum over q, nu (omega >= omega_min), m of
//     |g_mn nu|^2 / (2 omega) [ (N + f_m) G(e_n - e_m + omega) + (N + 1 - f_m) G(e_n - e_m - omega) ]
// N Bose, f_m Fermi at e_m(k+q), G a normalised Gaussian of width sigma.
// One workgroup per k; for Nw > 32 thread (row group rg, band n) sums column
// n over the rows (q, nu, m) rg, rg + G, ..., then the row groups are added
// in order.
constexpr int kLwThreads = 256;

template <typename T>
__global__ void __launch_bounds__(kLwThreads)
    linewidth_kernel(const T* __restrict__ g, int64_t nq, int64_t nk, int nm, int nw,
                     const double* __restrict__ eps_k, const double* __restrict__ eps_kq,
                     const double* __restrict__ omega, LwParams p, double* __restrict__ gamma) {
  __shared__ double red[kLwThreads];
  const int64_t ik = blockIdx.x;
  const int groups = kLwThreads / nw > 0 ? kLwThreads / nw : 1;
  const int tid = threadIdx.x, rg = tid / nw, n = tid % nw;
  const bool act = rg < groups;
  double acc = 0.0;
  if (act) {
    const double en = eps_k[ik * nw + n];
    const int64_t rows = nq * nm * nw;   // (q, nu, m)
    for (int64_t r = rg; r < rows; r += groups) {
      const int64_t iq = r / ((int64_t)nm * nw);
      const int rem = (int)(r - iq * nm * nw), nu = rem / nw, m = rem - nu * nw;
      const double om = omega[iq * nm + nu];
      if (!(om > 0.0) || om < p.omega_min) continue;   // omega = 0: no zero-point amplitude
      const double em = eps_kq[(iq * nk + ik) * nw + m];
      const double nb = 1.0 / expm1(om * p.inv_t);
      const double fm = fermi_occ(em, p);
      const double a = (en - em + om) * p.inv_sigma, b = (en - em - om) * p.inv_sigma;
      const double w = ((nb + fm) * gauss_exp<T>(a) + (nb + 1.0 - fm) * gauss_exp<T>(b)) * p.gnorm / (2.0 * om);
      const int64_t i = ((iq * nk + ik) * nm + nu) * (int64_t)nw * nw + (int64_t)m * nw + n;
      const double x = (double)g[2 * i], y = (double)g[2 * i + 1];
      acc += w * (x * x + y * y);
    }
  }
  red[tid] = act ? acc : 0.0;
  __syncthreads();
  if (tid < nw) {
    double s = 0.0;
    for (int j = 0; j < groups; ++j) s += red[j * nw + tid];
    gamma[ik * nw + tid] += p.scale * s;
  }
}

// Nw <= 32: thread per row (q, nu, m) with the NWB column sums in registers,
// so the occupations N and f_m cost one evaluation per row instead of one per
// element; per-column sums are added across the workgroup in a fixed order
// (butterfly within each wave, then the waves in turn).
template <typename T, int NWB>
__global__ void __launch_bounds__(kLwThreads)
    linewidth_rows_kernel(const T* __restrict__ g, int64_t nq, int64_t nk, int nm, int nw,
                          const double* __restrict__ eps_k, const double* __restrict__ eps_kq,
                          const double* __restrict__ omega, LwParams p, double* __restrict__ gamma) {
  __shared__ double red[kLwThreads / 64];
  const int64_t ik = blockIdx.x;
  const int tid = threadIdx.x;
  const bool vec16 = (nw % 2 == 0) && (reinterpret_cast<uintptr_t>(g) & 15) == 0;
  double en[NWB], acc[NWB];
#pragma unroll
  for (int n = 0; n < NWB; ++n) {
    en[n] = n < nw ? eps_k[ik * nw + n] : 0.0;
    acc[n] = 0.0;
  }
  const int64_t rows = nq * nm * nw;   // (q, nu, m)
  for (int64_t r = tid; r < rows; r += kLwThreads) {
    const int64_t iq = r / ((int64_t)nm * nw);
    const int rem = (int)(r - iq * nm * nw), nu = rem / nw, m = rem - nu * nw;
    const double om = omega[iq * nm + nu];
    if (!(om > 0.0) || om < p.omega_min) continue;   // omega = 0: no zero-point amplitude
    const double em = eps_kq[(iq * nk + ik) * nw + m];
    const double nb = 1.0 / expm1(om * p.inv_t);
    const double fm = fermi_occ(em, p);
    const double wa = (nb + fm) * p.gnorm / (2.0 * om), we = (nb + 1.0 - fm) * p.gnorm / (2.0 * om);
    const T* row = g + 2 * ((((iq * nk + ik) * nm + nu) * (int64_t)nw + m) * nw);
    double g2[NWB];
    if constexpr (sizeof(T) == 4) {
      if (vec16) {
        // even Nw, 16-byte aligned rows: two complex values per load
#pragma unroll
        for (int n = 0; n < NWB; n += 2) {
          if (n < nw) {
            const float4 v = *reinterpret_cast<const float4*>(row + 2 * n);
            g2[n] = (double)v.x * v.x + (double)v.y * v.y;
            g2[n + 1] = (double)v.z * v.z + (double)v.w * v.w;
          }
        }
      } else {
#pragma unroll
        for (int n = 0; n < NWB; ++n)
          if (n < nw) g2[n] = (double)row[2 * n] * row[2 * n] + (double)row[2 * n + 1] * row[2 * n + 1];
      }
    } else {
#pragma unroll
      for (int n = 0; n < NWB; ++n)
        if (n < nw) g2[n] = (double)row[2 * n] * row[2 * n] + (double)row[2 * n + 1] * row[2 * n + 1];
    }
#pragma unroll
    for (int n = 0; n < NWB; ++n) {
      if (n < nw) {
        const double a = (en[n] - em + om) * p.inv_sigma, b = (en[n] - em - om) * p.inv_sigma;
        acc[n] += (wa * gauss_exp<T>(a) + we * gauss_exp<T>(b)) * g2[n];
      }
    }
  }
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int n = 0; n < NWB; ++n) {
    if (n >= nw) break;   // nw is uniform: every thread leaves together
    double v = acc[n];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < kLwThreads / 64; ++w) s += red[w];
      gamma[ik * nw + n] += p.scale * s;
    }
    __syncthreads();
  }
}

template <typename T>
using LwKernel = void (*)(const T*, int64_t, int64_t, int, int, const double*, const double*, const double*,
                          LwParams, double*);

template <typename T>
LwKernel<T> lw_rows_kernel(int nw) {
  switch ((nw + 3) / 4) {
    case 1: return linewidth_rows_kernel<T, 4>;
    case 2: return linewidth_rows_kernel<T, 8>;
    case 3: return linewidth_rows_kernel<T, 12>;
    case 4: return linewidth_rows_kernel<T, 16>;
    case 5: return linewidth_rows_kernel<T, 20>;
    case 6: return linewidth_rows_kernel<T, 24>;
    case 7: return linewidth_rows_kernel<T, 28>;
    case 8: return linewidth_rows_kernel<T, 32>;
    default: return linewidth_kernel<T>;
  }
}

constexpr int64_t kColChunk = 16;     // columns per partial sum
constexpr int64_t kColChunksMax = 64; // chunks held in the scratch (more: chunks of more columns)

__global__ void column_chunk_sums_kernel(const double* __restrict__ x, int64_t ncol, int64_t n, int64_t chunk,
                                         double* __restrict__ part) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.y * chunk;
  if (i >= n) return;
  const int64_t c1 = c0 + chunk < ncol ? c0 + chunk : ncol;
  double s = 0.0;
  for (int64_t c = c0; c < c1; ++c) s += x[c * n + i];
  part[blockIdx.y * n + i] = s;
}

__global__ void add_chunk_sums_kernel(const double* __restrict__ part, int64_t nchunk, int64_t n, double scale,
                                      double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t c = 0; c < nchunk; ++c) s += part[c * n + i];
  out[i] += scale * s;
}

}  // namespace

size_t column_sum_scratch(int64_t n) { return (size_t)kColChunksMax * (size_t)n * sizeof(double); }

ephw_status add_column_sums(const double* x, int64_t ncol, int64_t n, double scale, double* out, double* scratch,
                            hipStream_t s) {
  if (n <= 0 || ncol <= 0) return EPHW_OK;
  int64_t chunk = kColChunk;
  while (ceil_div(ncol, chunk) > kColChunksMax) chunk *= 2;
  const int64_t nchunk = ceil_div(ncol, chunk);
  const unsigned gx = (unsigned)ceil_div(n, (int64_t)256);
  hipLaunchKernelGGL(column_chunk_sums_kernel, dim3(gx, (unsigned)nchunk), dim3(256), 0, s, x, ncol, n, chunk,
                     scratch);
  EPHW_CHECK_LAUNCH();
  hipLaunchKernelGGL(add_chunk_sums_kernel, dim3(gx), dim3(256), 0, s, scratch, nchunk, n, scale, out);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status linewidth(int prec, const void* g, int64_t nq, int64_t nk, int nm, int nw, const double* eps_k,
                      const double* eps_kq, const double* omega, double temperature, double mu, double sigma,
                      double omega_min, int64_t nq_total, double* gamma, hipStream_t s) {
  if (nq == 0 || nk == 0) return EPHW_OK;
  if (nk > 0x7fffffff) {
    set_error("ephw_linewidth: more than 2^31 k points");
    return EPHW_EUNSUPPORTED;
  }
  const LwParams p = lw_params(temperature, mu, sigma, omega_min, nq_total);
  if (prec == 0)
    hipLaunchKernelGGL(lw_rows_kernel<double>(nw), dim3((unsigned)nk), dim3(kLwThreads), 0, s,
                       static_cast<const double*>(g), nq, nk, nm, nw, eps_k, eps_kq, omega, p, gamma);
  else
    hipLaunchKernelGGL(lw_rows_kernel<float>(nw), dim3((unsigned)nk), dim3(kLwThreads), 0, s,
                       static_cast<const float*>(g), nq, nk, nm, nw, eps_k, eps_kq, omega, p, gamma);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status degenerate_sums(int prec, const void* g, int64_t nq, int64_t nk, int nm, int nw,
                            const double* eps_kq, const double* eps_k, const double* lam, double rel_tol,
                            double* out, hipStream_t s) {
  const int64_t npairs = nq * nk;
  if (npairs == 0) return EPHW_OK;
  const int64_t grid = ceil_div(npairs, kDegWaves);
  if (grid > 0x7fffffff) {
    set_error("ephw_degenerate_sums: too many pairs for one launch");
    return EPHW_EUNSUPPORTED;
  }
  const size_t lds = (size_t)kDegWaves * (4 * (size_t)nw + 2 * (size_t)nm) * sizeof(int);
  if (prec == EPHW_FP64)
    hipLaunchKernelGGL(degenerate_sums_kernel<double>, dim3((unsigned)grid), dim3(64 * kDegWaves), lds, s,
                       static_cast<const double*>(g), npairs, nk, nm, nw, eps_kq, eps_k, lam, rel_tol, out);
  else
    hipLaunchKernelGGL(degenerate_sums_kernel<float>, dim3((unsigned)grid), dim3(64 * kDegWaves), lds, s,
                       static_cast<const float*>(g), npairs, nk, nm, nw, eps_kq, eps_k, lam, rel_tol, out);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

}  // namespace ephw
