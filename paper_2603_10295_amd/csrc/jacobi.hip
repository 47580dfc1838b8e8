// Batched Hermitian eigensolver in FP64: cyclic two-sided Jacobi with the
// round-robin (tournament) ordering, so every step rotates n/2 disjoint
// (p, q) planes at once.
//
// Rotation of plane (p, q) with a = A_pp, d = A_qq, b = A_pq = |b| e^{i phi}:
//   tau = (d - a) / (2|b|), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1/sqrt(1 + t^2), s = t c,
//   J = [[c, s e^{i phi}], [-s e^{-i phi}, c]]  (unitary; J^H A J zeroes A_pq).
// A <- A J (columns), V <- V J, then A <- J^H A (rows).  A sweep visits every
// plane once; sweeps repeat until the off-diagonal Frobenius norm is below
// 1e-14 of the total norm.
//
// Small matrices (n <= 32) live in LDS, one 64-lane wavefront per matrix, with
// the LDS sized to the order (about 4.4 KB at n = 11) so that the CU holds as
// many solves as its registers allow: the solve is latency-bound.
// Large matrices (n > 32) live in a global workspace, one 256-thread
// workgroup per matrix (the rotation parameters stay in LDS).
#include "kernels.h"

namespace ephw {
namespace {

constexpr int kMaxSweeps = 40;
constexpr double kOffTol2 = 1e-28;  // (off-diagonal norm / total norm)^2 at convergence

__device__ __forceinline__ int player_at(int pos, int round, int n2) {
  return pos == 0 ? 0 : 1 + ((pos - 1 + round) % (n2 - 1));
}

template <int NT>
__device__ double block_sum(double v, double* red) {
  // wave reduction then across waves through LDS
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double tot = 0;
  for (int w = 0; w < NT / 64; ++w) tot += red[w];
  return tot;
}

// Core solver.  Ar/Ai/Vr/Vi: n*n row-major planes (LDS or global).
// On exit the diagonal of A holds the eigenvalues and V the eigenvectors.
template <int NT>
__device__ bool jacobi_core(double* Ar, double* Ai, double* Vr, double* Vi, int n, double* rc,
                            double* rs, double* rer, double* rei, int* rp, int* rq, double* red) {
  const int tid = threadIdx.x;
  const int n2 = n + (n & 1);
  const int npairs = n2 / 2;
  for (int e = tid; e < n * n; e += NT) {
    Vr[e] = (e / n == e % n) ? 1.0 : 0.0;
    Vi[e] = 0.0;
  }
  __syncthreads();
  bool converged = (n <= 1);
  for (int sweep = 0; sweep < kMaxSweeps && !converged; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += NT) {
      const double v = Ar[e] * Ar[e] + Ai[e] * Ai[e];
      tot += v;
      if (e / n != e % n) off += v;
    }
    off = block_sum<NT>(off, red);
    tot = block_sum<NT>(tot, red);
    if (off <= kOffTol2 * tot) {
      converged = true;
      break;
    }
    for (int round = 0; round < n2 - 1; ++round) {
      if (tid < npairs) {
        const int a = player_at(tid, round, n2), b = player_at(n2 - 1 - tid, round, n2);
        const int p = a < b ? a : b, q = a < b ? b : a;
        int pp = -1;
        double c = 1.0, s = 0.0, er = 1.0, ei = 0.0;
        if (q < n) {
          const double br = Ar[p * n + q], bi = Ai[p * n + q];
          const double bm = hypot(br, bi);
          if (bm > 0.0) {
            const double tau = (Ar[q * n + q] - Ar[p * n + p]) / (2.0 * bm);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            er = br / bm;
            ei = bi / bm;
            pp = p;
          }
        }
        rc[tid] = c;
        rs[tid] = s;
        rer[tid] = er;
        rei[tid] = ei;
        rp[tid] = pp;
        rq[tid] = q;
      }
      __syncthreads();
      // columns: A <- A J and V <- V J
      for (int w = tid; w < n * npairs; w += NT) {
        const int row = w / npairs, k = w % npairs;
        const int p = rp[k];
        if (p < 0) continue;
        const int q = rq[k];
        const double c = rc[k], s = rs[k], er = rer[k], ei = rei[k];
        // x' = c x - s conj(e) y ; y' = s e x + c y
        {
          const double xr = Ar[row * n + p], xi = Ai[row * n + p];
          const double yr = Ar[row * n + q], yi = Ai[row * n + q];
          Ar[row * n + p] = c * xr - s * (er * yr + ei * yi);
          Ai[row * n + p] = c * xi - s * (er * yi - ei * yr);
          Ar[row * n + q] = s * (er * xr - ei * xi) + c * yr;
          Ai[row * n + q] = s * (er * xi + ei * xr) + c * yi;
        }
        {
          const double xr = Vr[row * n + p], xi = Vi[row * n + p];
          const double yr = Vr[row * n + q], yi = Vi[row * n + q];
          Vr[row * n + p] = c * xr - s * (er * yr + ei * yi);
          Vi[row * n + p] = c * xi - s * (er * yi - ei * yr);
          Vr[row * n + q] = s * (er * xr - ei * xi) + c * yr;
          Vi[row * n + q] = s * (er * xi + ei * xr) + c * yi;
        }
      }
      __syncthreads();
      // rows: A <- J^H A ; x' = c x - s e y ; y' = s conj(e) x + c y
      for (int w = tid; w < npairs * n; w += NT) {
        const int k = w / n, col = w % n;
        const int p = rp[k];
        if (p < 0) continue;
        const int q = rq[k];
        const double c = rc[k], s = rs[k], er = rer[k], ei = rei[k];
        const double xr = Ar[p * n + col], xi = Ai[p * n + col];
        const double yr = Ar[q * n + col], yi = Ai[q * n + col];
        Ar[p * n + col] = c * xr - s * (er * yr - ei * yi);
        Ai[p * n + col] = c * xi - s * (er * yi + ei * yr);
        Ar[q * n + col] = s * (er * xr + ei * xi) + c * yr;
        Ai[q * n + col] = s * (er * xi - ei * xr) + c * yi;
      }
      __syncthreads();
    }
  }
  return converged;
}

// Sort ascending, fix each column's phase, write eps and V (c128).
template <int NT>
__device__ void jacobi_finish(const double* Ar, const double* Vr, const double* Vi, int n, int* perm,
                              double* phr, double* phi, double* eps_out, double* V_out) {
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += NT) {
    const double li = Ar[i * n + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = Ar[j * n + j];
      rank += (lj < li) || (lj == li && j < i);
    }
    perm[rank] = i;
  }
  __syncthreads();
  for (int c = tid; c < n; c += NT) {
    const int src = perm[c];
    eps_out[c] = Ar[src * n + src];
    double best = -1.0, br = 1.0, bi = 0.0;
    for (int r = 0; r < n; ++r) {
      const double vr = Vr[r * n + src], vi = Vi[r * n + src];
      const double m = vr * vr + vi * vi;
      if (m > best) {
        best = m;
        br = vr;
        bi = vi;
      }
    }
    const double mag = sqrt(best);
    phr[c] = mag > 0 ? br / mag : 1.0;   // multiply by conj(v_max)/|v_max|
    phi[c] = mag > 0 ? -bi / mag : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += NT) {
    const int r = e / n, c = e % n, src = perm[c];
    const double vr = Vr[r * n + src], vi = Vi[r * n + src];
    V_out[2 * e] = vr * phr[c] - vi * phi[c];
    V_out[2 * e + 1] = vr * phi[c] + vi * phr[c];
  }
}

constexpr int kSmallN = 32;

// LDS of one small solve, sized to its order so that many solves share a CU:
// A and V (re/im planes), the rotation parameters of one round, the sort
// permutation and the phase fix of each column, one reduction slot.
__host__ __device__ constexpr size_t small_lds_doubles(int n) {
  return 4 * (size_t)n * n + 4 * (size_t)((n + 1) / 2) + 2 * (size_t)n + 1;
}
__host__ __device__ constexpr size_t small_lds_bytes(int n) {
  return small_lds_doubles(n) * 8 + (2 * (size_t)((n + 1) / 2) + (size_t)n) * 4;
}

__device__ __forceinline__ void jacobi_small_body(const double* __restrict__ H, int n, double* __restrict__ eps,
                                                  double* __restrict__ V, uint32_t* status, int64_t b) {
  extern __shared__ double lds[];
  const int nn = n * n, np = (n + 1) / 2;
  double* Ar = lds;
  double* Ai = Ar + nn;
  double* Vr = Ai + nn;
  double* Vi = Vr + nn;
  double* rc = Vi + nn;
  double* rs = rc + np;
  double* rer = rs + np;
  double* rei = rer + np;
  double* phr = rei + np;
  double* phi = phr + n;
  double* red = phi + n;
  int* rp = reinterpret_cast<int*>(lds + small_lds_doubles(n));
  int* rq = rp + np;
  int* perm = rq + np;
  const double* h = H + 2 * b * nn;
  for (int e = threadIdx.x; e < nn; e += 64) {
    Ar[e] = h[2 * e];
    Ai[e] = h[2 * e + 1];
  }
  __syncthreads();
  const bool ok = jacobi_core<64>(Ar, Ai, Vr, Vi, n, rc, rs, rer, rei, rp, rq, red);
  if (!ok && threadIdx.x == 0) atomicOr(status, kStatusNoConv);
  jacobi_finish<64>(Ar, Vr, Vi, n, perm, phr, phi, eps + b * n, V + 2 * b * nn);
}

__global__ void __launch_bounds__(64)
    jacobi_small_kernel(const double* __restrict__ H, int n, double* __restrict__ eps,
                        double* __restrict__ V, uint32_t* status) {
  jacobi_small_body(H, n, eps, V, status, blockIdx.x);
}

// dynamic LDS sized for the largest order among the jobs
__global__ void __launch_bounds__(64) jacobi_grouped_kernel(const EighJob* __restrict__ jobs, int njobs,
                                                             uint32_t* status) {
  const int64_t b = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block_base <= b) lo = mid; else hi = mid - 1;
  }
  const EighJob& j = jobs[lo];
  jacobi_small_body(j.H, j.n, j.eps, j.V, status, b - j.block_base);
}

__global__ void __launch_bounds__(256)
    jacobi_large_kernel(const double* __restrict__ H, int n, double* __restrict__ eps,
                        double* __restrict__ V, double* __restrict__ work, uint32_t* status) {
  __shared__ double rc[128], rs[128], rer[128], rei[128], phr[256], phi[256], red[4];
  __shared__ int rp[128], rq[128], perm[256];
  const int64_t b = blockIdx.x;
  const int64_t nn = (int64_t)n * n;
  double* Ar = work + 4 * nn * blockIdx.x;
  double* Ai = Ar + nn;
  double* Vr = Ai + nn;
  double* Vi = Vr + nn;
  const double* h = H + 2 * b * nn;
  for (int64_t e = threadIdx.x; e < nn; e += 256) {
    Ar[e] = h[2 * e];
    Ai[e] = h[2 * e + 1];
  }
  __syncthreads();
  const bool ok = jacobi_core<256>(Ar, Ai, Vr, Vi, n, rc, rs, rer, rei, rp, rq, red);
  if (!ok && threadIdx.x == 0) atomicOr(status, kStatusNoConv);
  jacobi_finish<256>(Ar, Vr, Vi, n, perm, phr, phi, eps + b * n, V + 2 * b * nn);
}

constexpr int64_t kLargeChunk = 1024;  // matrices per large-n launch (bounds the workspace)

}  // namespace

int64_t jacobi_work_doubles(int n, int64_t batch) {
  if (n <= kSmallN) return 0;
  const int64_t chunk = batch < kLargeChunk ? batch : kLargeChunk;
  return 4 * (int64_t)n * n * chunk;
}

ephw_status jacobi_eigh_grouped(const EighJob* d_jobs, int njobs, int64_t blocks, int max_n, uint32_t* status,
                                hipStream_t s) {
  if (njobs <= 0 || blocks <= 0) return EPHW_OK;
  if (max_n < 1 || max_n > kSmallN) {
    set_error("jacobi_eigh_grouped: matrix orders must be in [1, 32]");
    return EPHW_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(jacobi_grouped_kernel, dim3((unsigned)blocks), dim3(64), small_lds_bytes(max_n), s, d_jobs,
                     njobs, status);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status jacobi_eigh(const double* H, int64_t batch, int n, double* eps, double* V, double* work,
                        uint32_t* status, hipStream_t s) {
  if (batch <= 0) return EPHW_OK;
  if (n < 1 || n > 256) {
    set_error("jacobi_eigh: matrix order must be in [1, 256]");
    return EPHW_EUNSUPPORTED;
  }
  if (n <= kSmallN) {
    for (int64_t b0 = 0; b0 < batch; b0 += 0x7fffffff) {
      const int64_t nb = (batch - b0) < 0x7fffffff ? (batch - b0) : 0x7fffffff;
      hipLaunchKernelGGL(jacobi_small_kernel, dim3((unsigned)nb), dim3(64), small_lds_bytes(n), s,
                         H + 2 * b0 * n * n, n, eps + b0 * n, V + 2 * b0 * n * n, status);
      EPHW_CHECK_LAUNCH();
    }
    return EPHW_OK;
  }
  if (!work) {
    set_error("jacobi_eigh: large matrices need a workspace");
    return EPHW_EINVAL;
  }
  for (int64_t b0 = 0; b0 < batch; b0 += kLargeChunk) {
    const int64_t nb = (batch - b0) < kLargeChunk ? (batch - b0) : kLargeChunk;
    hipLaunchKernelGGL(jacobi_large_kernel, dim3((unsigned)nb), dim3(256), 0, s,
                       H + 2 * b0 * (int64_t)n * n, n, eps + b0 * n, V + 2 * b0 * (int64_t)n * n,
                       work, status);
    EPHW_CHECK_LAUNCH();
  }
  return EPHW_OK;
}

}  // namespace ephw
