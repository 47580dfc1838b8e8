// Energy-window prescreening of k and q points (the pre-screening the paper
// applies before interpolating: matrix elements whose states lie outside an
// energy window are not computed).  A k point is active when one of its bands
// lies in [e_lo, e_hi]; a pair (k, q) when both k and k+q are; a q point when
// it has an active pair.  The screen compacts the active k and q points (in
// ascending order), maps each selected pair's k+q grid index into the
// compacted k list and marks the pairs whose k+q is active, so that Eq. (7)
// then runs on the compacted sets only.  ephw_window_pairs goes one step
// further and lists the kept pairs themselves (CSR by q or by k), the input
// of ephw_interpolate_pairs, which computes nothing for the pairs it drops.
#include <vector>

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

// bflag[b] = 1 when band b has an energy in the window at some k of the set
__global__ void band_any_kernel(const double* __restrict__ eps, int64_t nk, int nw, double lo, double hi,
                                int32_t* __restrict__ bflag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nk * nw) return;
  const double e = eps[i];
  if (e >= lo && e <= hi) atomicOr(&bflag[i % nw], 1);
}

// Pair lists of the pairs whose k and k+q both have a band in the window,
// grouped by q (CSR over the q list, each q's k ascending) or by k (CSR over
// the k-set, each k's q ascending).  One workgroup per q or per k; a thread
// takes a contiguous run of the other index.
constexpr int kPairThreads = 256;

// whether pair (q row `kq_row`, k = ik) is kept; j = index of k+q
__device__ __forceinline__ bool pair_kept(int32_t j, const int32_t* __restrict__ kflag, int64_t nk, int64_t ik,
                                          uint32_t* status) {
  if (j < 0 || j >= nk) {
    atomicOr(status, kStatusIndex);
    return false;
  }
  return kflag[ik] && kflag[j];
}

// by q: count[iq] = kept k of q iq.  by k: count[ik] = kept q of k ik.
__global__ void __launch_bounds__(kPairThreads)
    pair_count_kernel(const int32_t* __restrict__ kq, int64_t nq, int64_t nk, const int32_t* __restrict__ kflag,
                      int by_k, int64_t* __restrict__ count, uint32_t* status) {
  __shared__ int64_t part[kPairThreads];
  const int64_t major = blockIdx.x;
  const int64_t n_other = by_k ? nq : nk;
  int64_t c = 0;
  if (!by_k || kflag[major]) {
    for (int64_t o = threadIdx.x; o < n_other; o += kPairThreads) {
      const int64_t iq = by_k ? o : major, ik = by_k ? major : o;
      c += pair_kept(kq[iq * nk + ik], kflag, nk, ik, status) ? 1 : 0;
    }
  }
  part[threadIdx.x] = c;
  __syncthreads();
  for (int w = kPairThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) count[major] = part[0];
}

// the kept pairs of one q (by k: of one k) in ascending order of the other
// index: other = k (by q) or q (by k), pair_kq = index of k+q
__global__ void __launch_bounds__(kPairThreads)
    pair_fill_kernel(const int32_t* __restrict__ kq, int64_t nq, int64_t nk, const int32_t* __restrict__ kflag,
                     int by_k, const int64_t* __restrict__ start, int32_t* __restrict__ other,
                     int32_t* __restrict__ pair_kq, uint32_t* status) {
  __shared__ int64_t part[kPairThreads];
  const int64_t major = blockIdx.x;
  if (start[major + 1] == start[major]) return;   // uniform across the workgroup
  const int64_t n_other = by_k ? nq : nk;
  const int t = threadIdx.x;
  const int64_t chunk = (n_other + kPairThreads - 1) / kPairThreads;
  const int64_t b = t * chunk, e = (b + chunk) < n_other ? (b + chunk) : n_other;
  int64_t c = 0;
  for (int64_t o = b; o < e; ++o) {
    const int64_t iq = by_k ? o : major, ik = by_k ? major : o;
    c += pair_kept(kq[iq * nk + ik], kflag, nk, ik, status) ? 1 : 0;
  }
  part[t] = c;
  __syncthreads();
  for (int off = 1; off < kPairThreads; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t pos = start[major] + part[t] - c;
  for (int64_t o = b; o < e; ++o) {
    const int64_t iq = by_k ? o : major, ik = by_k ? major : o;
    const int32_t j = kq[iq * nk + ik];
    if (pair_kept(j, kflag, nk, ik, status)) {
      other[pos] = (int32_t)o;
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
                             int32_t order, int32_t* order_out, int64_t* pair_start, int32_t* pair_other,
                             int32_t* pair_kq, int64_t capacity, int32_t* band_range, void* stream) {
  if (!ks || nq < 0 || (nq > 0 && !kq_index) || !pair_start || capacity < 0 || !(e_lo <= e_hi) ||
      (order != EPHW_PAIRS_BY_Q && order != EPHW_PAIRS_BY_K && order != EPHW_PAIRS_AUTO)) {
    set_error("ephw_window_pairs: invalid argument");
    return EPHW_EINVAL;
  }
  ephw_system* s = ks->sys;
  hipStream_t st = as_stream(stream);
  const int64_t nk = ks->nk;
  if (nq == 0 || nk == 0) {
    const int32_t ord = order == EPHW_PAIRS_BY_K ? EPHW_PAIRS_BY_K : EPHW_PAIRS_BY_Q;
    const int64_t n = ord == EPHW_PAIRS_BY_K ? nk : nq;
    for (int64_t i = 0; i <= n; ++i) pair_start[i] = 0;
    if (order_out) *order_out = ord;
    if (band_range) band_range[0] = band_range[1] = 0;
    return EPHW_OK;
  }
  if (nk > 0x7fffffff || nq > 0x7fffffff) {
    set_error("ephw_window_pairs: more than 2^31 points");
    return EPHW_EUNSUPPORTED;
  }
  const bool want_q = order != EPHW_PAIRS_BY_K, want_k = order != EPHW_PAIRS_BY_Q;
  // workspace: start [max(nq, nk) + 1], counts by q [nq] and by k [nk] (int64),
  // k flags [nk] and band flags [nw] (int32)
  const int64_t nmax = nq > nk ? nq : nk;
  EPHW_TRY(ws_need(s, WS_WINDOW, (size_t)(nmax + 1 + nq + nk) * 8 + (size_t)(nk + s->nw) * 4 + 256));
  char* base = static_cast<char*>(wsp(s, WS_WINDOW));
  int64_t* start = reinterpret_cast<int64_t*>(base);
  int64_t* cnt_q = start + nmax + 1;
  int64_t* cnt_k = cnt_q + nq;
  int32_t* kflag = reinterpret_cast<int32_t*>(cnt_k + nk);
  int32_t* bflag = kflag + nk;
  hipLaunchKernelGGL(band_window_flags_kernel, dim3((unsigned)grid_of(nk, 256)), dim3(256), 0, st, ks->eps, nk,
                     s->nw, e_lo, e_hi, kflag);
  EPHW_CHECK_LAUNCH();
  if (band_range) {
    EPHW_HIP(hipMemsetAsync(bflag, 0, (size_t)s->nw * 4, st));
    hipLaunchKernelGGL(band_any_kernel, dim3((unsigned)grid_of(nk * s->nw, 256)), dim3(256), 0, st, ks->eps, nk,
                       s->nw, e_lo, e_hi, bflag);
    EPHW_CHECK_LAUNCH();
  }
  if (want_q) {
    hipLaunchKernelGGL(pair_count_kernel, dim3((unsigned)nq), dim3(kPairThreads), 0, st, kq_index, nq, nk, kflag, 0,
                       cnt_q, s->ctx->status);
    EPHW_CHECK_LAUNCH();
  }
  if (want_k) {
    hipLaunchKernelGGL(pair_count_kernel, dim3((unsigned)nk), dim3(kPairThreads), 0, st, kq_index, nq, nk, kflag, 1,
                       cnt_k, s->ctx->status);
    EPHW_CHECK_LAUNCH();
  }
  std::vector<int64_t> hq(want_q ? nq : 0), hk(want_k ? nk : 0);
  std::vector<int32_t> hb(band_range ? s->nw : 0);
  if (want_q) EPHW_HIP(hipMemcpyAsync(hq.data(), cnt_q, (size_t)nq * 8, hipMemcpyDeviceToHost, st));
  if (want_k) EPHW_HIP(hipMemcpyAsync(hk.data(), cnt_k, (size_t)nk * 8, hipMemcpyDeviceToHost, st));
  if (band_range) EPHW_HIP(hipMemcpyAsync(hb.data(), bflag, (size_t)s->nw * 4, hipMemcpyDeviceToHost, st));
  EPHW_HIP(hipStreamSynchronize(st));
  if (band_range) {
    // the smallest band range holding every band with an energy in the window
    int lo = -1, hi = -1;
    for (int b = 0; b < s->nw; ++b)
      if (hb[b]) {
        if (lo < 0) lo = b;
        hi = b;
      }
    band_range[0] = lo < 0 ? 0 : lo;
    band_range[1] = lo < 0 ? 0 : hi - lo + 1;
  }
  // the cheaper nesting order (see ephw_interpolate_pairs): group by the
  // index with fewer points that own a pair
  int32_t ord = order;
  if (order == EPHW_PAIRS_AUTO) {
    int64_t aq = 0, ak = 0;
    for (int64_t c : hq) aq += c > 0;
    for (int64_t c : hk) ak += c > 0;
    ord = ak < aq ? EPHW_PAIRS_BY_K : EPHW_PAIRS_BY_Q;
  }
  if (order_out) *order_out = ord;
  const std::vector<int64_t>& cnt = ord == EPHW_PAIRS_BY_K ? hk : hq;
  const int64_t n = (int64_t)cnt.size();
  pair_start[0] = 0;
  for (int64_t i = 0; i < n; ++i) pair_start[i + 1] = pair_start[i] + cnt[i];
  const int64_t total = pair_start[n];
  if (total > capacity) {
    set_error("ephw_window_pairs: " + std::to_string(total) + " pairs kept, more than the capacity of " +
              std::to_string(capacity) + " (pair_start holds the counts)");
    return EPHW_EINVAL;
  }
  if (total == 0) return EPHW_OK;
  if (!pair_other || !pair_kq) {
    set_error("ephw_window_pairs: pair_other and pair_kq are required when pairs are kept");
    return EPHW_EINVAL;
  }
  EPHW_HIP(hipMemcpyAsync(start, pair_start, (size_t)(n + 1) * 8, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(pair_fill_kernel, dim3((unsigned)n), dim3(kPairThreads), 0, st, kq_index, nq, nk, kflag,
                     ord == EPHW_PAIRS_BY_K ? 1 : 0, start, pair_other, pair_kq, s->ctx->status);
  EPHW_CHECK_LAUNCH();
  // the offsets were copied from the caller's host array: finish before returning
  EPHW_HIP(hipStreamSynchronize(st));
  return EPHW_OK;
}

}  // extern "C"
