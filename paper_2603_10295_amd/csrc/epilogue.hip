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

}  // namespace

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
