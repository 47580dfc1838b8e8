// Internal helpers shared by the libephw HIP sources (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/ephw.h"

namespace ephw {

// ---------------------------------------------------------------------------
// complex values in registers
// ---------------------------------------------------------------------------
template <typename T>
struct cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
template <typename T>
__device__ __forceinline__ cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T>
__device__ __forceinline__ void cfma(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.re = fma(a.re, b.re, fma(-a.im, b.im, acc.re));
  acc.im = fma(a.re, b.im, fma(a.im, b.re, acc.im));
}
// acc += conj(a) * b
template <typename T>
__device__ __forceinline__ void cfmac(cplx<T>& acc, cplx<T> a, cplx<T> b) {
  acc.re = fma(a.re, b.re, fma(a.im, b.im, acc.re));
  acc.im = fma(a.re, b.im, fma(-a.im, b.re, acc.im));
}

template <typename T>
__device__ __forceinline__ cplx<T> ld(const T* p, int64_t i) {
  return {p[2 * i], p[2 * i + 1]};
}
template <typename T>
__device__ __forceinline__ void st(T* p, int64_t i, cplx<T> v) {
  p[2 * i] = v.re;
  p[2 * i + 1] = v.im;
}

// A wavefront that owns its LDS region alone needs only its own LDS
// operations complete before it reads what other lanes wrote, never a
// workgroup barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// ---------------------------------------------------------------------------
// phonon-limited linewidth weights (the downstream reduction of stored or
// freshly rotated matrix elements): parameters and occupations
// ---------------------------------------------------------------------------
struct LwParams {
  double inv_t = 0, mu = 0, inv_sigma = 0, gnorm = 0, omega_min = 0, scale = 0;
};

inline LwParams lw_params(double temperature, double mu, double sigma, double omega_min, int64_t nq_total) {
  LwParams p;
  p.inv_t = 1.0 / temperature;
  p.mu = mu;
  p.inv_sigma = 1.0 / sigma;
  p.gnorm = 1.0 / (sigma * 2.5066282746310005024);   // 1 / (sigma sqrt(2 pi))
  p.omega_min = omega_min;
  p.scale = 3.14159265358979323846 / (double)nq_total;
  return p;
}

// exp(-x^2/2) of a scaled energy difference: in FP32 for c64 matrix elements
// (a weight error near 1e-7, below the data's own), FP64 otherwise
template <typename T>
__device__ __forceinline__ double gauss_exp(double x) {
  if constexpr (sizeof(T) == 4) {
    const float f = (float)x;
    return (double)expf(-0.5f * f * f);
  } else {
    return exp(-0.5 * x * x);
  }
}

__device__ __forceinline__ double fermi_occ(double e, const LwParams& p) {
  const double x = (e - p.mu) * p.inv_t;
  const double z = exp(-fabs(x));
  return x > 0.0 ? z / (1.0 + z) : 1.0 / (1.0 + z);
}

// ---------------------------------------------------------------------------
// device status word bits (context-wide, read by ephw_ctx_check)
// ---------------------------------------------------------------------------
enum : uint32_t { kStatusNoConv = 1u, kStatusIndex = 2u };
// Jacobi sweeps before an eigensolve reports kStatusNoConv: the context's
// second device word holds the limit (default kDefaultSweeps)
constexpr int kDefaultSweeps = 40;
constexpr int kMaxSweepLimit = 1000;
__device__ __forceinline__ int sweep_limit(const uint32_t* status) { return (int)status[1]; }

// ---------------------------------------------------------------------------
// host-side error plumbing
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);

#define EPHW_HIP(expr)                                                              \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::ephw::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));         \
      return EPHW_EDEVICE;                                                          \
    }                                                                               \
  } while (0)

#define EPHW_TRY(expr)                  \
  do {                                  \
    ephw_status s_ = (expr);            \
    if (s_ != EPHW_OK) return s_;       \
  } while (0)

#define EPHW_CHECK_LAUNCH() EPHW_HIP(hipGetLastError())

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace ephw
