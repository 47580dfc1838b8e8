// Phase factors w_R exp(2 pi i p.R) of Eq. (7), generated on the device.
//
// p is fractional (FP64) and R integer, so p.R is formed in FP64 and reduced
// to (-1/2, 1/2] by subtracting its nearest integer before sincospi; the
// reduced argument keeps full FP64 accuracy however large |R| is.  For the
// FP32 forms the FP64 phase is rounded to a (hi, lo) pair of floats.
#include "kernels.h"

namespace ephw {
namespace {

template <typename T>
__global__ void phase_kernel(const double* __restrict__ pts, int64_t n, const int32_t* __restrict__ R,
                             const double* __restrict__ w, int64_t nr, T* __restrict__ out,
                             T* __restrict__ out_lo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * nr) return;
  const int64_t i = idx / nr, r = idx % nr;
  const double t = pts[3 * i] * (double)R[3 * r] + pts[3 * i + 1] * (double)R[3 * r + 1] +
                   pts[3 * i + 2] * (double)R[3 * r + 2];
  const double red = t - rint(t);
  double sn, cs;
  sincospi(2.0 * red, &sn, &cs);
  if (w) {
    const double wr = w[r];
    sn *= wr;
    cs *= wr;
  }
  const T hr = (T)cs, hi = (T)sn;
  out[2 * idx] = hr;
  out[2 * idx + 1] = hi;
  if (out_lo) {
    out_lo[2 * idx] = (T)(cs - (double)hr);
    out_lo[2 * idx + 1] = (T)(sn - (double)hi);
  }
}

}  // namespace

ephw_status phase_matrix(int prec, const double* pts, int64_t n, const int32_t* R, const double* w,
                         int64_t nr, void* out, void* out_lo, hipStream_t s) {
  const int64_t total = n * nr;
  if (total <= 0) return EPHW_OK;
  const int bs = 256;
  const int64_t grid = ceil_div(total, bs);
  if (prec == 0) {
    hipLaunchKernelGGL(phase_kernel<double>, dim3((unsigned)grid), dim3(bs), 0, s, pts, n, R, w, nr,
                       static_cast<double*>(out), static_cast<double*>(out_lo));
  } else {
    hipLaunchKernelGGL(phase_kernel<float>, dim3((unsigned)grid), dim3(bs), 0, s, pts, n, R, w, nr,
                       static_cast<float*>(out), static_cast<float*>(out_lo));
  }
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

}  // namespace ephw
