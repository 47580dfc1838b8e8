// Phase factors w_R exp(2 pi i p.R) of Eq. (7), generated on the device.
//
// p is fractional (FP64) and R integer, so p.R is formed in FP64 and reduced
// to (-1/2, 1/2] by subtracting its nearest integer before sincospi; the
// reduced argument keeps full FP64 accuracy however large |R| is.  The FP32
// forms take the FP64 phase rounded to complex64.
#include "kernels.h"

namespace ephw {
namespace {

template <typename T>
__global__ void phase_kernel(const double* __restrict__ pts, int64_t n, const int32_t* __restrict__ R,
                             const double* __restrict__ w, int64_t nr, T* __restrict__ out) {
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
  out[2 * idx] = (T)cs;
  out[2 * idx + 1] = (T)sn;
}

}  // namespace

ephw_status phase_matrix(int prec, const double* pts, int64_t n, const int32_t* R, const double* w,
                         int64_t nr, void* out, hipStream_t s) {
  const int64_t total = n * nr;
  if (total <= 0) return EPHW_OK;
  const int bs = 256;
  const int64_t grid = ceil_div(total, bs);
  if (prec == 0) {
    hipLaunchKernelGGL(phase_kernel<double>, dim3((unsigned)grid), dim3(bs), 0, s, pts, n, R, w, nr,
                       static_cast<double*>(out));
  } else {
    hipLaunchKernelGGL(phase_kernel<float>, dim3((unsigned)grid), dim3(bs), 0, s, pts, n, R, w, nr,
                       static_cast<float*>(out));
  }
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

}  // namespace ephw
