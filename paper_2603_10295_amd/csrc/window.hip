// Energy-window prescreening of k and q points (the pre-screening the paper
// applies before interpolating: matrix elements whose states lie outside an
// energy window are not computed).  A k point is active when one of its bands
// lies in [e_lo, e_hi]; a pair (k, q) when both k and k+q are; a q point when
// it has an active pair.  The screen compacts the active k and q points (in
// ascending order), maps each selected pair's k+q grid index into the
// compacted k list and marks the pairs whose k+q is active, so that Eq. (7)
// then runs on the compacted sets only.  ephw_window_pairs goes one step
// further and lists the kept pairs themselves (CSR by q), the input of
// ephw_interpolate_pairs, which computes nothing for the pairs it drops.
#include "internal.h"

namespace ephw {
namespace {

constexpr int kScanThreads = 1024;

__global__ void band_window_flags_kernel(const double* __restrict__ eps, int64_t n, int nw, double lo, double hi,
                                         int32_t* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int f = 0;
  for (int b = 0; b < nw; ++b) {
    const double e = eps[i * nw + b];
    f |= (e >= lo && e <= hi) ? 1 : 0;
  }
  flag[i] = f;
}

// q flag: some k is active with k+q active; k+q indices outside [0, nk) are
// reported through the status word
__global__ void q_window_flags_kernel(const int32_t* __restrict__ kq, int64_t nq, int64_t nk,
                                      const int32_t* __restrict__ kflag, int32_t* __restrict__ qflag,
                                      uint32_t* status) {
  const int64_t iq = blockIdx.x;
  int f = 0;
  for (int64_t ik = threadIdx.x; ik < nk; ik += blockDim.x) {
    const int32_t j = kq[iq * nk + ik];
    if (j < 0 || j >= nk) {
      atomicOr(status, kStatusIndex);
      continue;
    }
    f |= kflag[ik] & kflag[j];
  }
  f = __syncthreads_or(f);
  if (threadIdx.x == 0) qflag[iq] = f ? 1 : 0;
}

// one workgroup: sel[c] = index of the c-th set flag (ascending), map[i] = c
// or -1, *count = number of set flags.  Each thread scans a contiguous chunk.
__global__ void __launch_bounds__(kScanThreads)
    compact_kernel(const int32_t* __restrict__ flag, int64_t n, int32_t* __restrict__ sel, int32_t* __restrict__ map,
                   int64_t* __restrict__ count) {
  __shared__ int64_t part[kScanThreads];
  const int t = threadIdx.x;
  const int64_t chunk = (n + kScanThreads - 1) / kScanThreads;
  const int64_t b = t * chunk, e = (b + chunk) < n ? (b + chunk) : n;
  int64_t c = 0;
  for (int64_t i = b; i < e; ++i) c += flag[i] != 0;
  part[t] = c;
  __syncthreads();
  // exclusive scan of the per-thread counts (Hillis-Steele in LDS)
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t pos = part[t] - c;
  for (int64_t i = b; i < e; ++i) {
    if (flag[i]) {
      sel[pos] = (int32_t)i;
      map[i] = (int32_t)pos;
      ++pos;
    } else {
      map[i] = -1;
    }
  }
  if (t == kScanThreads - 1) *count = part[t];
}

__global__ void gather_points_kernel(const double* __restrict__ pts, const int32_t* __restrict__ sel, int64_t n,
                                     double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * n) return;
  out[i] = pts[3 * (int64_t)sel[i / 3] + i % 3];
}

// rows r of the selected q, columns c of the selected k
__global__ void window_pairs_kernel(const int32_t* __restrict__ kq, int64_t nk, const int32_t* __restrict__ q_sel,
                                    const int32_t* __restrict__ k_sel, const int32_t* __restrict__ kmap, int64_t nqs,
                                    int64_t nks, int32_t* __restrict__ kq_sel, uint8_t* __restrict__ mask) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nqs * nks) return;
  const int64_t r = i / nks, c = i % nks;
  const int32_t j = kq[(int64_t)q_sel[r] * nk + k_sel[c]];
  const int32_t m = (j >= 0 && j < nk) ? kmap[j] : -1;
  kq_sel[i] = m >= 0 ? m : 0;
  if (mask) mask[i] = m >= 0 ? 1 : 0;
}

int64_t grid_of(int64_t n, int t) { return (n + t - 1) / t; }

// Pair lists (CSR by q) of the pairs whose k and k+q both have a band in the
// window.  One workgroup per q; each thread takes a contiguous run of k.
constexpr int kPairThreads = 256;

__device__ __forceinline__ bool pair_kept(const int32_t* __restrict__ kq_row, const int32_t* __restrict__ kflag,
                                          int64_t nk, int64_t ik, uint32_t* status, int32_t* j_out) {
  const int32_t j = kq_row[ik];
  if (j < 0 || j >= nk) {
    atomicOr(status, kStatusIndex);
    return false;
  }
  *j_out = j;
  return kflag[ik] && kflag[j];
}

__global__ void __launch_bounds__(kPairThreads)
    pair_count_kernel(const int32_t* __restrict__ kq, int64_t nk, const int32_t* __restrict__ kflag,
                      int64_t* __restrict__ count, uint32_t* status) {
  __shared__ int64_t part[kPairThreads];
  const int64_t iq = blockIdx.x;
  const int32_t* row = kq + iq * nk;
  int64_t c = 0;
  for (int64_t ik = threadIdx.x; ik < nk; ik += kPairThreads) {
    int32_t j;
    c += pair_kept(row, kflag, nk, ik, status, &j) ? 1 : 0;
  }
  part[threadIdx.x] = c;
  __syncthreads();
  for (int w = kPairThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) count[iq] = part[0];
}

// start[i] = sum of count[0..i) for i = 0..n (one workgroup)
__global__ void __launch_bounds__(kScanThreads)
    exclusive_scan_kernel(const int64_t* __restrict__ count, int64_t n, int64_t* __restrict__ start) {
  __shared__ int64_t part[kScanThreads];
  const int t = threadIdx.x;
  const int64_t chunk = (n + kScanThreads - 1) / kScanThreads;
  const int64_t b = t * chunk, e = (b + chunk) < n ? (b + chunk) : n;
  int64_t c = 0;
  for (int64_t i = b; i < e; ++i) c += count[i];
  part[t] = c;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t pos = part[t] - c;
  for (int64_t i = b; i < e; ++i) {
    start[i] = pos;
    pos += count[i];
  }
  if (t == kScanThreads - 1) start[n] = part[t];
}

// the kept pairs of q in ascending k: pair_k = k, pair_kq = index of k+q
__global__ void __launch_bounds__(kPairThreads)
    pair_fill_kernel(const int32_t* __restrict__ kq, int64_t nk, const int32_t* __restrict__ kflag,
                     const int64_t* __restrict__ start, int32_t* __restrict__ pair_k, int32_t* __restrict__ pair_kq,
                     uint32_t* status) {
  __shared__ int64_t part[kPairThreads];
  const int64_t iq = blockIdx.x;
  const int32_t* row = kq + iq * nk;
  const int t = threadIdx.x;
  const int64_t chunk = (nk + kPairThreads - 1) / kPairThreads;
  const int64_t b = t * chunk, e = (b + chunk) < nk ? (b + chunk) : nk;
  int64_t c = 0;
  for (int64_t ik = b; ik < e; ++ik) {
    int32_t j;
    c += pair_kept(row, kflag, nk, ik, status, &j) ? 1 : 0;
  }
  part[t] = c;
  __syncthreads();
  for (int off = 1; off < kPairThreads; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t pos = start[iq] + part[t] - c;
  for (int64_t ik = b; ik < e; ++ik) {
    int32_t j;
    if (pair_kept(row, kflag, nk, ik, status, &j)) {
      pair_k[pos] = (int32_t)ik;
      pair_kq[pos] = j;
      ++pos;
    }
  }
}

}  // namespace
}  // namespace ephw

using namespace ephw;

extern "C" {

ephw_status ephw_window_screen(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index, double e_lo,
                               double e_hi, double* k_out, int64_t* nk_out, double* q_out, int64_t* nq_out,
                               int32_t* kq_out, uint8_t* pair_mask, void* stream) {
  if (!ks || nq < 0 || (nq > 0 && (!q || !kq_index)) || !k_out || !nk_out || !nq_out ||
      (nq > 0 && (!q_out || !kq_out)) || !(e_lo <= e_hi)) {
    set_error("ephw_window_screen: invalid argument");
    return EPHW_EINVAL;
  }
  ephw_system* s = ks->sys;
  hipStream_t st = as_stream(stream);
  const int64_t nk = ks->nk;
  if (nk == 0) {
    *nk_out = 0;
    *nq_out = 0;
    return EPHW_OK;
  }
  if (nk > 0x7fffffff || nq > 0x7fffffff) {
    set_error("ephw_window_screen: more than 2^31 points");
    return EPHW_EUNSUPPORTED;
  }
  // workspace: k flags, k map, k selection, q flags, q map, q selection, two counts
  const size_t ints = (size_t)3 * nk + (size_t)3 * nq;
  EPHW_TRY(ws_need(s, WS_WINDOW, ints * 4 + 16 + 256));
  char* base = static_cast<char*>(wsp(s, WS_WINDOW));
  int64_t* counts = reinterpret_cast<int64_t*>(base);
  int32_t* kflag = reinterpret_cast<int32_t*>(base + 256);
  int32_t* kmap = kflag + nk;
  int32_t* ksel = kmap + nk;
  int32_t* qflag = ksel + nk;
  int32_t* qmap = qflag + nq;
  int32_t* qsel = qmap + nq;

  hipLaunchKernelGGL(band_window_flags_kernel, dim3((unsigned)grid_of(nk, 256)), dim3(256), 0, st, ks->eps, nk,
                     s->nw, e_lo, e_hi, kflag);
  EPHW_CHECK_LAUNCH();
  hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(kScanThreads), 0, st, kflag, nk, ksel, kmap, counts);
  EPHW_CHECK_LAUNCH();
  if (nq > 0) {
    hipLaunchKernelGGL(q_window_flags_kernel, dim3((unsigned)nq), dim3(256), 0, st, kq_index, nq, nk, kflag, qflag,
                       s->ctx->status);
    EPHW_CHECK_LAUNCH();
    hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(kScanThreads), 0, st, qflag, nq, qsel, qmap, counts + 1);
    EPHW_CHECK_LAUNCH();
  }
  int64_t h[2] = {0, 0};
  EPHW_HIP(hipMemcpyAsync(h, counts, sizeof(h), hipMemcpyDeviceToHost, st));
  EPHW_HIP(hipStreamSynchronize(st));
  const int64_t nks = h[0], nqs = nq > 0 ? h[1] : 0;
  *nk_out = nks;
  *nq_out = nqs;
  if (nks > 0) {
    hipLaunchKernelGGL(gather_points_kernel, dim3((unsigned)grid_of(3 * nks, 256)), dim3(256), 0, st, ks->k, ksel,
                       nks, k_out);
    EPHW_CHECK_LAUNCH();
  }
  if (nqs > 0 && nks > 0) {
    hipLaunchKernelGGL(gather_points_kernel, dim3((unsigned)grid_of(3 * nqs, 256)), dim3(256), 0, st, q, qsel, nqs,
                       q_out);
    EPHW_CHECK_LAUNCH();
    hipLaunchKernelGGL(window_pairs_kernel, dim3((unsigned)grid_of(nqs * nks, 256)), dim3(256), 0, st, kq_index, nk,
                       qsel, ksel, kmap, nqs, nks, kq_out, pair_mask);
    EPHW_CHECK_LAUNCH();
  }
  return EPHW_OK;
}

ephw_status ephw_window_pairs(ephw_kset* ks, const int32_t* kq_index, int64_t nq, double e_lo, double e_hi,
                             int64_t* pair_start, int32_t* pair_k, int32_t* pair_kq, int64_t capacity,
                             void* stream) {
  if (!ks || nq < 0 || (nq > 0 && !kq_index) || !pair_start || capacity < 0 || !(e_lo <= e_hi)) {
    set_error("ephw_window_pairs: invalid argument");
    return EPHW_EINVAL;
  }
  ephw_system* s = ks->sys;
  hipStream_t st = as_stream(stream);
  const int64_t nk = ks->nk;
  if (nq == 0 || nk == 0) {
    for (int64_t i = 0; i <= nq; ++i) pair_start[i] = 0;
    return EPHW_OK;
  }
  if (nk > 0x7fffffff || nq > 0x7fffffff) {
    set_error("ephw_window_pairs: more than 2^31 points");
    return EPHW_EUNSUPPORTED;
  }
  // workspace: start [nq + 1] and count [nq] (int64), k flags [nk] (int32)
  EPHW_TRY(ws_need(s, WS_WINDOW, (size_t)(2 * nq + 1) * 8 + (size_t)nk * 4 + 256));
  char* base = static_cast<char*>(wsp(s, WS_WINDOW));
  int64_t* start = reinterpret_cast<int64_t*>(base);
  int64_t* count = start + nq + 1;
  int32_t* kflag = reinterpret_cast<int32_t*>(count + nq);
  hipLaunchKernelGGL(band_window_flags_kernel, dim3((unsigned)grid_of(nk, 256)), dim3(256), 0, st, ks->eps, nk,
                     s->nw, e_lo, e_hi, kflag);
  EPHW_CHECK_LAUNCH();
  hipLaunchKernelGGL(pair_count_kernel, dim3((unsigned)nq), dim3(kPairThreads), 0, st, kq_index, nk, kflag, count,
                     s->ctx->status);
  EPHW_CHECK_LAUNCH();
  hipLaunchKernelGGL(exclusive_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, count, nq, start);
  EPHW_CHECK_LAUNCH();
  EPHW_HIP(hipMemcpyAsync(pair_start, start, (size_t)(nq + 1) * 8, hipMemcpyDeviceToHost, st));
  EPHW_HIP(hipStreamSynchronize(st));
  const int64_t total = pair_start[nq];
  if (total > capacity) {
    set_error("ephw_window_pairs: " + std::to_string(total) + " pairs kept, more than the capacity of " +
              std::to_string(capacity) + " (pair_start holds the counts)");
    return EPHW_EINVAL;
  }
  if (total > 0) {
    if (!pair_k || !pair_kq) {
      set_error("ephw_window_pairs: pair_k and pair_kq are required when pairs are kept");
      return EPHW_EINVAL;
    }
    hipLaunchKernelGGL(pair_fill_kernel, dim3((unsigned)nq), dim3(kPairThreads), 0, st, kq_index, nk, kflag, start,
                       pair_k, pair_kq, s->ctx->status);
    EPHW_CHECK_LAUNCH();
  }
  return EPHW_OK;
}

}  // extern "C"
