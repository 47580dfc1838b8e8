// Large-band rotations and the adjoint of the weighted loss
//   L = sum_{q,k,nu,m,n} w_{mn nu}(k,q) |g_{mn nu}(k,q)|^2,
// with g_nu = V(k+q)^dagger W_nu V(k), W_nu = sum_Re e^{ik.Re} G_nu(Re,q),
// G_nu = sum_ka G_ka u_{ka,nu}(q), G = sum_Rp e^{iq.Rp} g(Re,Rp)  (Eqs. (7), (9), (10)).
//
// Per (q batch, k tile) unit the forward is recomputed (phase tiles are
// regenerated from the k and q lists, never stored across units) and the
// chain rule runs backwards through it:
//   Ybar = 2 w g                           (fused into the GEMM producing g)
//   Wbar_nu = V(k+q) Ybar_nu V(k)^dagger
//   Vbar(k) = sum W_nu^dagger V(k+q) Ybar_nu,  Vbar(k+q) = sum W_nu V(k) Ybar_nu^dagger
//   G_nu bar(Re,q) = sum_k e^{-ik.Re} Wbar(k,q);  G bar = conj(u) G_nu bar;  ubar = conj(G) G_nu bar^T
//   dL/dg(Re,Rp) = sum_q e^{-iq.Rp} G bar(Re,q)
// and k, q enter through (i) the phase factors, whose derivative is the phase
// times 2 pi i R_d (so dL/dk_d = Re <Wbar, W'_d> with W'_d the Re sum taken
// with those scaled phases), (ii) the eigenvectors: dL/dk_d = Re <Vbar, dV/dk_d>
// with dV = V (F o (V^dagger dH V)), F_ij = 1/(eps_j - eps_i), the
// first-order change of the eigenvectors (their phases held fixed; the loss
// does not depend on them).  For k+q on the k grid, dV at the grid point
// serves both dL/dk_i and dL/dq_j of the pair.
//
// The coarse Bloch -> Wannier transform of Eq. (6) runs through the same
// back-rotations and conjugate-phase sums (it is the inverse of Eq. (7) on a
// commensurate grid): W_nu = V(k+q) g_nu V(k)^dagger, sum_k e^{-ik.Re},
// then u^-1 in place of conj(u), sum_q e^{-iq.Rp}, and 1/(Ne Np).
#include <algorithm>

#include "internal.h"

namespace ephw {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// out[d][i][r] = ph[i][r] * (2 pi i R[r][d])
template <typename T>
__global__ void scale_phase_kernel(const T* __restrict__ ph, int64_t n, const int32_t* __restrict__ R, int64_t nr,
                                   T* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 3 * n * nr) return;
  const int64_t d = idx / (n * nr), ir = idx % (n * nr), r = ir % nr;
  const T f = (T)(kTwoPi * (double)R[3 * r + d]);
  const T re = ph[2 * ir], im = ph[2 * ir + 1];
  out[2 * idx] = -f * im;
  out[2 * idx + 1] = f * re;
}

// M[b][i][j] /= (eps[j] - eps[i]) off the diagonal, 0 on it; eps row = b % nrow
__global__ void eig_mid_kernel(double* __restrict__ M, const double* __restrict__ eps, int64_t batch, int n,
                               int64_t nrow) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= batch * n * n) return;
  const int64_t b = idx / ((int64_t)n * n);
  const int i = (int)((idx / n) % n), j = (int)(idx % n);
  const double* e = eps + (b % nrow) * n;
  if (i == j) {
    M[2 * idx] = 0.0;
    M[2 * idx + 1] = 0.0;
  } else {
    const double f = 1.0 / (e[j] - e[i]);
    M[2 * idx] *= f;
    M[2 * idx + 1] *= f;
  }
}

// uinvT[q][a][v] = conj(e[q][a][v]) / ism[a]: the transpose of u^-1 for
// u = diag(ism) e with e unitary (u^-1 = e^dagger diag(1/ism))
template <typename T>
__global__ void mode_inverse_kernel(const double* __restrict__ e, int64_t nq, int nm, const double* __restrict__ ism,
                                    T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)nm * nm;
  if (i >= nq * per) return;
  const int a = (int)((i % per) / nm);
  out[2 * i] = (T)(e[2 * i] / ism[a]);
  out[2 * i + 1] = (T)(-e[2 * i + 1] / ism[a]);
}

template <typename T>
__global__ void scale_complex_kernel(T* __restrict__ x, int64_t n, double f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[2 * i] = (T)((double)x[2 * i] * f);
  x[2 * i + 1] = (T)((double)x[2 * i + 1] * f);
}

// Complex offset of V(k+q) for each (k, q) pair of a unit:
//   offp[il qb + iq] = kq_index[(q0+iq) nk + k0+il] * nw2
// (an out-of-range index sets the status bit and reads V(k_0)).
__global__ void kq_offsets_kernel(const int32_t* __restrict__ kq, int64_t nk, int64_t q0, int64_t k0, int kl, int qb,
                                  int64_t nw2, int64_t* __restrict__ offp, uint32_t* status) {
  const int64_t pair = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (pair >= (int64_t)kl * qb) return;
  const int64_t il = pair / qb, iq = pair % qb;
  int64_t j = kq[(q0 + iq) * nk + k0 + il];
  if (j < 0 || j >= nk) {
    atomicOr(status, kStatusIndex);
    j = 0;
  }
  offp[pair] = j * nw2;
}

// out[(r / inner) so + (r % inner) si] (+)= Re sum_c conj(a[r][c]) b[row(r)][c].
// Block (s, r) sums columns [s cc, (s+1) cc) of row r in a fixed-order tree;
// with one chunk per row it writes the result, otherwise part[r * S + s].
template <typename T>
__global__ void row_dot_kernel(const T* __restrict__ a, int64_t lda, const T* __restrict__ b, int64_t ldb,
                               const int64_t* __restrict__ boff, int64_t cols, int64_t cc, double* __restrict__ out,
                               int64_t inner, int64_t so, int64_t si, int accumulate, double* __restrict__ part) {
  __shared__ double red[256];
  const int64_t r = blockIdx.y, sidx = blockIdx.x, S = gridDim.x;
  const T* ar = a + 2 * r * lda;
  const T* br = b + 2 * (boff ? boff[r] : r * ldb);
  const int64_t c0 = sidx * cc, c1 = (c0 + cc) < cols ? (c0 + cc) : cols;
  double s = 0.0;
  for (int64_t c = c0 + threadIdx.x; c < c1; c += 256)
    s += (double)ar[2 * c] * (double)br[2 * c] + (double)ar[2 * c + 1] * (double)br[2 * c + 1];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (S > 1) {
      part[r * S + sidx] = red[0];
    } else {
      double* o = out + (r / inner) * so + (r % inner) * si;
      if (accumulate) *o += red[0];
      else *o = red[0];
    }
  }
}

// second stage: out (+)= sum over the S chunk partials of each row, in order
__global__ void row_dot_finish_kernel(const double* __restrict__ part, int64_t rows, int64_t S,
                                      double* __restrict__ out, int64_t inner, int64_t so, int64_t si,
                                      int accumulate) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double s = 0.0;
  for (int64_t i = 0; i < S; ++i) s += part[r * S + i];
  double* o = out + (r / inner) * so + (r % inner) * si;
  if (accumulate) *o += s;
  else *o = s;
}

// dk[k][d] += sum_q ps[q][k][d]  and  dq[q][d] += sum_k ps[q][k][d]
__global__ void pair_sums_kernel(const double* __restrict__ ps, int64_t nq, int64_t nk, double* __restrict__ dk,
                                 double* __restrict__ dq) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < nk * 3) {
    const int64_t k = idx / 3, d = idx % 3;
    double s = 0.0;
    for (int64_t q = 0; q < nq; ++q) s += ps[(q * nk + k) * 3 + d];
    dk[idx] += s;
  } else if (idx < nk * 3 + nq * 3) {
    const int64_t j = idx - nk * 3, q = j / 3, d = j % 3;
    double s = 0.0;
    for (int64_t k = 0; k < nk; ++k) s += ps[(q * nk + k) * 3 + d];
    dq[j] += s;
  }
}

// C (+)= sum over chunks of partial[b][chunk] (M*N values each)
template <typename T>
__global__ void splitk_reduce_kernel(const T* __restrict__ part, int64_t batch, int chunks, int64_t mn, T* __restrict__ C,
                                     int64_t ldc, int64_t n, int64_t strideC, int accumulate) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= batch * mn) return;
  const int64_t b = idx / mn, e = idx % mn, row = e / n, col = e % n;
  T re = 0, im = 0;
  for (int c = 0; c < chunks; ++c) {
    const T* p = part + 2 * ((b * chunks + c) * mn + e);
    re += p[0];
    im += p[1];
  }
  T* c = C + 2 * (b * strideC + row * ldc + col);
  if (accumulate) {
    re += c[0];
    im += c[1];
  }
  c[0] = re;
  c[1] = im;
}

template <typename T>
__global__ void fill_zero_kernel(T* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (T)0;
}

// per (pair, nu): ||W_nu||_F^2 (band sums need no rotation: V is unitary)
template <typename T>
__global__ void frob_kernel(const T* __restrict__ W, int64_t nw2, double* __restrict__ out, int64_t qb, int64_t nm,
                            int64_t nk, int64_t k0, int64_t kl) {
  __shared__ double red[256];
  const int64_t b = blockIdx.x;  // (il, iq, nu)
  const T* w = W + 2 * b * nw2;
  double s = 0.0;
  for (int64_t c = threadIdx.x; c < nw2; c += 256) s += (double)w[2 * c] * w[2 * c] + (double)w[2 * c + 1] * w[2 * c + 1];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int t = 128; t > 0; t >>= 1) {
    if (threadIdx.x < t) red[threadIdx.x] += red[threadIdx.x + t];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t nu = b % nm, iq = (b / nm) % qb, il = b / (nm * qb);
    out[((iq * nk) + k0 + il) * nm + nu] = red[0];
  }
}

inline unsigned grid1(int64_t n, int bs) { return (unsigned)ceil_div(n, bs); }

// chunks per row: enough blocks to fill the chip (about 2048) when rows are
// few, each chunk at least 4096 columns; the partials need rows * S doubles
// (at most kRowDotPart in all, see row_dot_chunks)
constexpr int64_t kRowDotPart = 4096;
int64_t row_dot_chunks(int64_t rows, int64_t cols) {
  if (rows <= 0 || rows >= 2048) return 1;
  int64_t S = std::min<int64_t>(ceil_div(cols, 4096), ceil_div(2048, rows));
  S = std::max<int64_t>(1, std::min<int64_t>(S, kRowDotPart / rows));
  return S;
}

template <typename T>
ephw_status launch_row_dot(const void* a, int64_t lda, const void* b, int64_t ldb, const int64_t* boff, int64_t rows,
                           int64_t cols, double* out, int64_t inner, int64_t so, int64_t si, bool acc, double* part,
                           hipStream_t s) {
  if (rows <= 0) return EPHW_OK;
  if (rows > 65535 * 1024ll) {
    set_error("row_dot: too many rows");
    return EPHW_EUNSUPPORTED;
  }
  const int64_t S = part ? row_dot_chunks(rows, cols) : 1;
  const int64_t cc = ceil_div(cols, S);
  // grid.y holds rows: split very tall launches at multiples of `inner`
  const int64_t rstep = std::max<int64_t>(inner, (65535 / inner) * inner);
  if (rstep > 65535) {
    set_error("row_dot: output block too tall");
    return EPHW_EUNSUPPORTED;
  }
  for (int64_t r0 = 0; r0 < rows; r0 += rstep) {
    const int64_t nr = std::min<int64_t>(rstep, rows - r0);
    const T* ab = static_cast<const T*>(a) + 2 * r0 * lda;
    const T* bb = static_cast<const T*>(b) + (boff ? 0 : 2 * r0 * ldb);
    const int64_t* bo = boff ? boff + r0 : nullptr;
    double* ob = out + (r0 / inner) * so + (r0 % inner) * si;
    hipLaunchKernelGGL(row_dot_kernel<T>, dim3((unsigned)S, (unsigned)nr), dim3(256), 0, s, ab, lda, bb, ldb, bo,
                       cols, cc, ob, inner, so, si, acc ? 1 : 0, part);
    EPHW_CHECK_LAUNCH();
    if (S > 1) {
      hipLaunchKernelGGL(row_dot_finish_kernel, dim3(grid1(nr, 256)), dim3(256), 0, s, part, nr, S, ob, inner, so,
                         si, acc ? 1 : 0);
      EPHW_CHECK_LAUNCH();
    }
  }
  return EPHW_OK;
}

// plain form: out[r * ostride]
ephw_status row_dot(int kind, const void* a, int64_t lda, const void* b, int64_t ldb, const int64_t* boff,
                    int64_t rows, int64_t cols, double* out, int64_t ostride, bool acc, double* part, hipStream_t s) {
  return kind == 0 ? launch_row_dot<double>(a, lda, b, ldb, boff, rows, cols, out, 1, ostride, 0, acc, part, s)
                   : launch_row_dot<float>(a, lda, b, ldb, boff, rows, cols, out, 1, ostride, 0, acc, part, s);
}

ephw_status row_dot2(int kind, const void* a, int64_t lda, const void* b, int64_t ldb, const int64_t* boff,
                     int64_t rows, int64_t cols, double* out, int64_t inner, int64_t so, int64_t si, bool acc,
                     double* part, hipStream_t s) {
  return kind == 0 ? launch_row_dot<double>(a, lda, b, ldb, boff, rows, cols, out, inner, so, si, acc, part, s)
                   : launch_row_dot<float>(a, lda, b, ldb, boff, rows, cols, out, inner, so, si, acc, part, s);
}

ephw_status fill_zero(int kind_or_f64, void* p, int64_t complex_count, hipStream_t s) {
  // kind 0/1: complex double/float elements; 2: plain doubles
  if (complex_count <= 0) return EPHW_OK;
  if (kind_or_f64 == 1) {
    const int64_t n = 2 * complex_count;
    hipLaunchKernelGGL(fill_zero_kernel<float>, dim3(grid1(n, 256)), dim3(256), 0, s, static_cast<float*>(p), n);
  } else {
    const int64_t n = kind_or_f64 == 0 ? 2 * complex_count : complex_count;
    hipLaunchKernelGGL(fill_zero_kernel<double>, dim3(grid1(n, 256)), dim3(256), 0, s, static_cast<double*>(p), n);
  }
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

ephw_status scale_phase(int kind, const void* ph, int64_t n, const int32_t* R, int64_t nr, void* out, hipStream_t s) {
  const int64_t total = 3 * n * nr;
  if (total <= 0) return EPHW_OK;
  if (kind == 0)
    hipLaunchKernelGGL(scale_phase_kernel<double>, dim3(grid1(total, 256)), dim3(256), 0, s,
                       static_cast<const double*>(ph), n, R, nr, static_cast<double*>(out));
  else
    hipLaunchKernelGGL(scale_phase_kernel<float>, dim3(grid1(total, 256)), dim3(256), 0, s,
                       static_cast<const float*>(ph), n, R, nr, static_cast<float*>(out));
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

// Split-K GEMM for small M x N with a long K: the K range is cut into `chunks`
// equal pieces (chunks divides K), each a batch entry writing a partial
// product; the partials are then summed in a fixed order into C.
ephw_status cgemm_splitk(int kind, const GemmParams& p, int chunks, void* scratch, hipStream_t s) {
  if (chunks <= 1 || p.K % chunks != 0 || p.offA || p.offB || p.offC || p.n1 != 1 || p.n2 != 1) return cgemm(kind, p, s);
  const int64_t kc = p.K / chunks;
  GemmParams q = p;
  q.K = kc;
  q.batch = p.batch * chunks;
  q.n2 = chunks;
  q.strideA = p.strideA;
  q.strideA2 = p.transA ? kc * p.lda : kc;
  q.strideB = p.strideB;
  q.strideB2 = p.transB ? kc : kc * p.ldb;
  q.C = scratch;
  q.ldc = p.N;
  q.strideC = p.M * p.N * chunks;
  q.strideC2 = p.M * p.N;
  q.accumulate = false;
  q.loss = LossEpilogue();
  EPHW_TRY(cgemm(kind, q, s));
  const int64_t mn = p.M * p.N, total = p.batch * mn;
  if (kind == 0)
    hipLaunchKernelGGL(splitk_reduce_kernel<double>, dim3(grid1(total, 256)), dim3(256), 0, s,
                       static_cast<const double*>(scratch), p.batch, chunks, mn, static_cast<double*>(p.C), p.ldc, p.N,
                       p.strideC, p.accumulate ? 1 : 0);
  else
    hipLaunchKernelGGL(splitk_reduce_kernel<float>, dim3(grid1(total, 256)), dim3(256), 0, s,
                       static_cast<const float*>(scratch), p.batch, chunks, mn, static_cast<float*>(p.C), p.ldc, p.N,
                       p.strideC, p.accumulate ? 1 : 0);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

// the number of K chunks: a divisor of K, at most `target`, chunks of >= min_len
int splitk_chunks(int64_t K, int target, int64_t min_len) {
  for (int c = target; c > 1; --c)
    if (K % c == 0 && K / c >= min_len) return c;
  return 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// eigenvector derivatives dV/dp_d = V (F o (V^H dM_d V)), d = 0..2, for n
// points: phase [n][nr] (c128), R [nr][3], mats [nr][dim][dim] (c128), eps,
// V (c128).  Output dV [3][n][dim][dim] in c128 (`out64`) and, if prec 1,
// cast to c64 in `out`.
// ---------------------------------------------------------------------------
ephw_status eigvec_derivatives(ephw_system* s, const double* phase, const int32_t* R, int64_t n, int64_t nr,
                               const double* mats, int dim, const double* eps, const double* V, double* out64,
                               void* out, int kind, hipStream_t st) {
  const int64_t d2 = (int64_t)dim * dim;
  // scratch: scaled phases [3][n][nr], dM [3][n][d2], tmp [3][n][d2]
  EPHW_TRY(ws_need(s, WS_ADJ_A, (size_t)3 * n * nr * 16));
  EPHW_TRY(ws_need(s, WS_ADJ_B, (size_t)3 * n * d2 * 16));
  EPHW_TRY(ws_need(s, WS_ADJ_C, (size_t)3 * n * d2 * 16));
  double* sph = static_cast<double*>(wsp(s, WS_ADJ_A));
  double* dm = static_cast<double*>(wsp(s, WS_ADJ_B));
  double* tmp = static_cast<double*>(wsp(s, WS_ADJ_C));
  EPHW_TRY(scale_phase(0, phase, n, R, nr, sph, st));
  GemmParams g;
  g.M = 3 * n;  // all three directions stacked as rows
  g.N = d2;
  g.K = nr;
  g.A = sph;
  g.lda = nr;
  g.B = mats;
  g.ldb = d2;
  g.C = dm;
  g.ldc = d2;
  EPHW_TRY(cgemm(0, g, st));
  // tmp = dM V   (batch (d, i): V index i)
  GemmParams a;
  a.M = dim;
  a.N = dim;
  a.K = dim;
  a.batch = 3 * n;
  a.n2 = n;
  a.A = dm;
  a.lda = dim;
  a.strideA = n * d2;
  a.strideA2 = d2;
  a.B = V;
  a.ldb = dim;
  a.strideB = 0;
  a.strideB2 = d2;
  a.C = tmp;
  a.ldc = dim;
  a.strideC = n * d2;
  a.strideC2 = d2;
  EPHW_TRY(cgemm(0, a, st));
  // dm = V^H tmp
  GemmParams b = a;
  b.A = V;
  b.transA = true;
  b.conjA = true;
  b.strideA = 0;
  b.strideA2 = d2;
  b.B = tmp;
  b.strideB = n * d2;
  b.strideB2 = d2;
  b.C = dm;
  EPHW_TRY(cgemm(0, b, st));
  hipLaunchKernelGGL(eig_mid_kernel, dim3(grid1(3 * n * d2, 256)), dim3(256), 0, st, dm, eps, 3 * n, dim, n);
  EPHW_CHECK_LAUNCH();
  // out64 = V dm
  GemmParams c = a;
  c.A = V;
  c.strideA = 0;
  c.strideA2 = d2;
  c.B = dm;
  c.strideB = n * d2;
  c.strideB2 = d2;
  c.C = out64;
  EPHW_TRY(cgemm(0, c, st));
  if (kind == 1 && out) EPHW_TRY(cast_complex(1, out64, out, 3 * n * d2, st));
  return EPHW_OK;
}

}  // namespace ephw

using namespace ephw;

namespace {

// (q batch, k tile) of the unit loops.  The four g(Re,q)-sized buffers get up
// to 8 GB and the `nbuf` pair-sized buffers up to 48 GB of the 288 GB of HBM.
// The k tile is the M of the Re GEMM (for small Ne a short-K, store-bound
// GEMM whose 128-row tiles want many k) and every k tile re-reads g(Re,q);
// a larger q batch at the same pair budget would shorten the k tile, which
// measured slower on the ribbon than the Eq. (9) GEMM it speeds up.
void unit_shape(const ephw_system* s, int64_t nq, int64_t nk, int64_t E, size_t cs, int nbuf, int64_t* qb_out,
                int64_t* kt_out) {
  int64_t qb = s->q_batch;
  if (qb <= 0) {
    qb = (int64_t)(8.0e9 / (4.0 * (double)s->ne * E * cs));
    qb = std::max<int64_t>(1, std::min<int64_t>(qb, 8));
  }
  qb = std::min(qb, nq);
  int64_t kt = (int64_t)(48.0e9 / ((double)nbuf * cs * qb * E));
  if (kt < 1) kt = 1;
  if (kt >= 64) kt -= kt % 16;
  if (s->k_tile > 0) kt = s->k_tile;
  *qb_out = qb;
  *kt_out = std::min(kt, nk);
}

// Pair-stacked rotation GEMM: batch b = il nb + iq runs over the (k, q) pairs
// of a unit; A is the pair's nm nw x nw stack of per-mode blocks (rows
// (nu, row)), so every launch has nm nw rows and nw columns instead of nm
// separate nw x nw products.  Pair buffers are [il][iq][E].
GemmParams pair_params(int64_t nw, int64_t nm, int64_t nb, int64_t kl, int64_t E) {
  GemmParams p;
  p.M = nm * nw;
  p.N = nw;
  p.K = nw;
  p.batch = kl * nb;
  p.n1 = nb;
  p.lda = nw;
  p.ldb = nw;
  p.ldc = nw;
  p.strideA = nb * E;
  p.strideA1 = E;
  p.strideC = nb * E;
  p.strideC1 = E;
  return p;
}

}  // namespace

namespace ephw {

// Eq. (7) for systems with more than 32 bands: the band rotations run as
// batched GEMMs per (q batch, k tile) unit; outputs as in ephw_interpolate.
ephw_status interpolate_large(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index, int64_t q_offset,
                              uint32_t flags, void* g_out, double* band_sum, double* loss, uint64_t loss_seed,
                              double* eps_kq, double* omega, hipStream_t st) {
  ephw_system* s = ks->sys;
  if (!kq_index) {
    set_error("ephw_interpolate: systems with more than 32 bands need a k+q grid index table");
    return EPHW_EUNSUPPORTED;
  }
  if (flags & EPHW_OUT_WANNIER) {
    set_error("ephw_interpolate: the Wannier-gauge output is limited to nw <= 32");
    return EPHW_EUNSUPPORTED;
  }
  const int kind = prec_kind(ks->prec);
  const size_t cs = csize(kind);
  const int64_t nw = s->nw, nm = s->nm, nw2 = nw * nw, E = nm * nw2, nk = ks->nk, ne = s->ne, np = s->np;
  int64_t qb, kt;
  unit_shape(s, nq, nk, E, cs, 2, &qb, &kt);
  // q side
  EPHW_TRY(ws_need(s, WS_PQ, (size_t)nq * np * cs));
  EPHW_TRY(phase_matrix(kind, q, nq, s->r_p, s->w_p, np, wsp(s, WS_PQ), st));
  EPHW_TRY(ws_need(s, WS_PQC, (size_t)nq * s->nc * 16));
  EPHW_TRY(phase_matrix(0, q, nq, s->r_c, s->w_c, s->nc, wsp(s, WS_PQC), st));
  EPHW_TRY(ws_need(s, WS_LAM, (size_t)nq * nm * 8));
  EPHW_TRY(ws_need(s, WS_E, (size_t)nq * nm * nm * 16));
  EPHW_TRY(ws_need(s, WS_HK, (size_t)nq * nm * nm * 16));
  {
    GemmParams g;
    g.M = nq;
    g.N = nm * nm;
    g.K = s->nc;
    g.A = wsp(s, WS_PQC);
    g.lda = s->nc;
    g.B = s->c_scaled;
    g.ldb = nm * nm;
    g.C = wsp(s, WS_HK);
    g.ldc = nm * nm;
    EPHW_TRY(cgemm(0, g, st));
    const int64_t jw = jacobi_work_doubles((int)nm, nq);
    if (jw > 0) EPHW_TRY(ws_need(s, WS_JWORK, (size_t)jw * 8));
    EPHW_TRY(jacobi_eigh(static_cast<const double*>(wsp(s, WS_HK)), nq, (int)nm, static_cast<double*>(wsp(s, WS_LAM)),
                         static_cast<double*>(wsp(s, WS_E)), jw > 0 ? static_cast<double*>(wsp(s, WS_JWORK)) : nullptr,
                         s->ctx->status, st));
  }
  if (omega) EPHW_TRY(abs_sqrt(static_cast<const double*>(wsp(s, WS_LAM)), omega, nq * nm, st));
  EPHW_TRY(ws_need(s, WS_U, (size_t)nq * nm * nm * cs));
  EPHW_TRY(mode_vectors(kind, static_cast<const double*>(wsp(s, WS_E)), nq, (int)nm, s->ism, wsp(s, WS_U), st));
  const bool rot = (flags & (EPHW_OUT_G | EPHW_OUT_LOSS)) != 0;
  const bool need_g = (flags & (EPHW_OUT_G | EPHW_OUT_BAND_SUM | EPHW_OUT_LOSS)) != 0;
  const size_t gsz = (size_t)qb * ne * E * cs, wsz = (size_t)kt * qb * E * cs;
  const int64_t rot_tiles = cgemm_tiles(kind, nm * nw, nw);  // per pair
  if (need_g) {
    EPHW_TRY(ws_need(s, WS_G, gsz));
    EPHW_TRY(ws_need(s, WS_GNU, gsz));
    EPHW_TRY(ws_need(s, WS_W, wsz));
    EPHW_TRY(ws_need(s, WS_T, wsz));
    EPHW_TRY(ws_need(s, WS_OFF, (size_t)kt * qb * 8));
    EPHW_TRY(ws_need(s, WS_LOSS, (size_t)kt * qb * rot_tiles * 8));
  }
  char* pq = static_cast<char*>(wsp(s, WS_PQ));
  char* u = static_cast<char*>(wsp(s, WS_U));
  char* vt = static_cast<char*>(ks->vt);
  for (int64_t q0 = 0; q0 < nq; q0 += qb) {
    const int64_t nb = std::min(qb, nq - q0);
    if (eps_kq)
      EPHW_TRY(gather_rows(ks->eps, nk, kq_index + q0 * nk, nb * nk, (int)nw, eps_kq + q0 * nk * nw, s->ctx->status,
                           st));
    if (!need_g) continue;
    char* G = static_cast<char*>(wsp(s, WS_G));
    char* Gnu = static_cast<char*>(wsp(s, WS_GNU));
    char* W = static_cast<char*>(wsp(s, WS_W));
    char* Tm = static_cast<char*>(wsp(s, WS_T));
    int64_t* offp = static_cast<int64_t*>(wsp(s, WS_OFF));
    double* lossp = static_cast<double*>(wsp(s, WS_LOSS));
    GemmParams rp;
    rp.M = nb;
    rp.N = ne * E;
    rp.K = np;
    rp.A = pq + (size_t)q0 * np * cs;
    rp.lda = np;
    rp.B = s->g;
    rp.ldb = rp.N;
    rp.C = G;
    rp.ldc = rp.N;
    {
      Stage sg_(s, EPHW_STAGE_RP_GEMM, st);
      EPHW_TRY(cgemm(kind, rp, st));
    }
    {
    Stage sgm_(s, EPHW_STAGE_MODE_ROT, st);
    if (nm <= 24) {
      EPHW_TRY(mode_rotate(kind, G, u + (size_t)q0 * nm * nm * cs, Gnu, ne, (int)nb, (int)nm, nw2, st));
    } else {
      GemmParams mr;
      mr.M = nm;
      mr.N = nw2;
      mr.K = nm;
      mr.batch = nb * ne;
      mr.n2 = ne;
      mr.A = u + (size_t)q0 * nm * nm * cs;
      mr.transA = true;
      mr.lda = nm;
      mr.strideA = nm * nm;
      mr.B = G;
      mr.ldb = nw2;
      mr.strideB = ne * E;
      mr.strideB2 = E;
      mr.C = Gnu;
      mr.ldc = nw2;
      mr.strideC = E;
      mr.strideC2 = nb * E;
      EPHW_TRY(cgemm(kind, mr, st));
    }
    }
    for (int64_t k0 = 0; k0 < nk; k0 += kt) {
      const int64_t kl = std::min(kt, nk - k0);
      const int64_t nbat = kl * nb * nm;
      GemmParams re;
      re.M = kl;
      re.N = nb * E;
      re.K = ne;
      re.A = static_cast<const char*>(ks->pk) + (size_t)k0 * ne * cs;
      re.lda = ne;
      re.B = Gnu;
      re.ldb = re.N;
      re.C = W;
      re.ldc = re.N;
      {
        Stage sg_(s, EPHW_STAGE_RE_GEMM, st);
        EPHW_TRY(cgemm(kind, re, st));
      }
      if (flags & EPHW_OUT_BAND_SUM) {
        // T_nu = ||W_nu||_F^2: the band rotations are unitary
        if (kind == 0)
          hipLaunchKernelGGL(frob_kernel<double>, dim3((unsigned)nbat), dim3(256), 0, st,
                             reinterpret_cast<const double*>(W), nw2, band_sum + q0 * nk * nm, nb, nm, nk, k0, kl);
        else
          hipLaunchKernelGGL(frob_kernel<float>, dim3((unsigned)nbat), dim3(256), 0, st,
                             reinterpret_cast<const float*>(W), nw2, band_sum + q0 * nk * nm, nb, nm, nk, k0, kl);
        EPHW_CHECK_LAUNCH();
      }
      if (!rot) continue;
      hipLaunchKernelGGL(kq_offsets_kernel, dim3(grid1(kl * nb, 256)), dim3(256), 0, st, kq_index, nk, q0, k0, (int)kl,
                         (int)nb, nw2, offp, s->ctx->status);
      EPHW_CHECK_LAUNCH();
      Stage sgr_(s, EPHW_STAGE_BAND_ROT, st);
      // T'_nu = (W_nu V(k))^T: rows (nu, m) of W, each nw-row block stored transposed
      GemmParams f4 = pair_params(nw, nm, nb, kl, E);
      f4.A = W;
      f4.B = vt + (size_t)k0 * nw2 * cs;
      f4.strideB = nw2;
      f4.C = Tm;
      f4.tblock = nw;
      f4.ldc = nw2;
      EPHW_TRY(cgemm(kind, f4, st));
      // g_nu[m'][n] = sum_m T'_nu[n][m] conj(V(k+q))[m][m']: rows (nu, n), columns m',
      // stored block-transposed, i.e. in the [nu][m'][n] order of g
      GemmParams f5 = pair_params(nw, nm, nb, kl, E);
      f5.A = Tm;
      f5.B = vt;
      f5.offB = offp;
      f5.conjB = true;
      f5.tblock = nw;
      f5.ldc = nw2;
      if (flags & EPHW_OUT_G) {
        // g_out[(q0+iq) nk + k0+il][nu][m][n]
        f5.C = static_cast<char*>(g_out) + ((size_t)q0 * nk + k0) * E * cs;
        f5.strideC = E;
        f5.strideC1 = nk * E;
      } else {
        f5.C = Tm;  // not written (loss only)
      }
      if (flags & EPHW_OUT_LOSS) {
        f5.loss.on = true;
        f5.loss.layout = 1;
        f5.loss.store = (flags & EPHW_OUT_G) != 0;
        f5.loss.seed = loss_seed;
        f5.loss.nk = nk;
        f5.loss.nm = (int)nm;
        f5.loss.nw = (int)nw;
        f5.loss.qb = (int)nb;
        f5.loss.q0 = q_offset + q0;
        f5.loss.k0 = k0;
        f5.loss.partial = lossp;
      }
      EPHW_TRY(cgemm(kind, f5, st));
      if (flags & EPHW_OUT_LOSS) EPHW_TRY(sum_into(lossp, kl * nb * rot_tiles, loss, st));
    }
  }
  return EPHW_OK;
}

}  // namespace ephw

extern "C" {

ephw_status ephw_loss_backward(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index, int64_t q_offset,
                               uint64_t loss_seed, double* loss, void* dL_dg, double* dL_dk, double* dL_dq,
                               void* stream) {
  if (!ks || (!q && nq > 0) || nq < 0 || q_offset < 0 || !kq_index) {
    set_error("ephw_loss_backward: need a k-set, a q list and a k+q index table");
    return EPHW_EINVAL;
  }
  if (!loss && !dL_dg && !dL_dk && !dL_dq) {
    set_error("ephw_loss_backward: nothing requested");
    return EPHW_EINVAL;
  }
  if (ks->prec == EPHW_FP32_COMP) {
    set_error("ephw_loss_backward: FP64 or FP32 k-sets only");
    return EPHW_EUNSUPPORTED;
  }
  if (nq == 0) return EPHW_OK;
  ephw_system* s = ks->sys;
  hipStream_t st = as_stream(stream);
  const int kind = prec_kind(ks->prec);
  const size_t cs = csize(kind);
  const int64_t nw = s->nw, nm = s->nm, nw2 = nw * nw, E = nm * nw2, nk = ks->nk, ne = s->ne, np = s->np;
  // unit shape: q batch and k tile within a workspace budget
  int64_t qb, kt;
  unit_shape(s, nq, nk, E, cs, 7, &qb, &kt);

  // ---- k side: eigenvector derivatives and scaled phases (cached in the k-set) ----
  if (!ks->dv) {
    void* p = nullptr;
    EPHW_TRY(dev_alloc(&p, (size_t)3 * nk * nw2 * 16, ks->mem.get()));
    ks->dv64 = static_cast<double*>(p);
    ks->bytes += (int64_t)3 * nk * nw2 * 16;
    if (kind == 1) {
      EPHW_TRY(dev_alloc(&p, (size_t)3 * nk * nw2 * 8, ks->mem.get()));
      ks->dv = p;
      ks->bytes += (int64_t)3 * nk * nw2 * 8;
    } else {
      ks->dv = ks->dv64;
    }
    EPHW_TRY(dev_alloc(&p, (size_t)3 * nk * ne * cs, ks->mem.get()));
    ks->dpk = p;
    ks->bytes += (int64_t)3 * nk * ne * cs;
    EPHW_TRY(eigvec_derivatives(s, ks->pkh, s->r_h, nk, s->nh, s->h_r, (int)nw, ks->eps, ks->v64, ks->dv64,
                                kind == 1 ? ks->dv : nullptr, kind, st));
    EPHW_TRY(scale_phase(kind, ks->pk, nk, s->r_e, ne, ks->dpk, st));
  }
  // directions with a nonzero lattice component (the others have zero phase derivatives)
  bool dir_e[3] = {false, false, false}, dir_p[3] = {false, false, false};
  {
    std::vector<int32_t> re(3 * ne), rp(3 * np);
    EPHW_HIP(hipMemcpy(re.data(), s->r_e, re.size() * 4, hipMemcpyDeviceToHost));
    EPHW_HIP(hipMemcpy(rp.data(), s->r_p, rp.size() * 4, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < ne; ++i)
      for (int d = 0; d < 3; ++d) dir_e[d] = dir_e[d] || re[3 * i + d] != 0;
    for (int64_t i = 0; i < np; ++i)
      for (int d = 0; d < 3; ++d) dir_p[d] = dir_p[d] || rp[3 * i + d] != 0;
  }

  // ---- q side: phases, D(q) eigensolve, u, du/dq ----
  EPHW_TRY(ws_need(s, WS_PQ, (size_t)nq * np * cs));
  EPHW_TRY(phase_matrix(kind, q, nq, s->r_p, s->w_p, np, wsp(s, WS_PQ), st));
  EPHW_TRY(ws_need(s, WS_DPQ, (size_t)3 * nq * np * cs));
  EPHW_TRY(scale_phase(kind, wsp(s, WS_PQ), nq, s->r_p, np, wsp(s, WS_DPQ), st));
  EPHW_TRY(ws_need(s, WS_PQC, (size_t)nq * s->nc * 16));
  EPHW_TRY(phase_matrix(0, q, nq, s->r_c, s->w_c, s->nc, wsp(s, WS_PQC), st));
  EPHW_TRY(ws_need(s, WS_LAM, (size_t)nq * nm * 8));
  EPHW_TRY(ws_need(s, WS_E, (size_t)nq * nm * nm * 16));
  {
    // D(q) = PqC C_scaled, then Jacobi
    EPHW_TRY(ws_need(s, WS_HK, (size_t)nq * nm * nm * 16));
    GemmParams g;
    g.M = nq;
    g.N = nm * nm;
    g.K = s->nc;
    g.A = wsp(s, WS_PQC);
    g.lda = s->nc;
    g.B = s->c_scaled;
    g.ldb = nm * nm;
    g.C = wsp(s, WS_HK);
    g.ldc = nm * nm;
    EPHW_TRY(cgemm(0, g, st));
    const int64_t jw = jacobi_work_doubles((int)nm, nq);
    if (jw > 0) EPHW_TRY(ws_need(s, WS_JWORK, (size_t)jw * 8));
    EPHW_TRY(jacobi_eigh(static_cast<const double*>(wsp(s, WS_HK)), nq, (int)nm, static_cast<double*>(wsp(s, WS_LAM)),
                         static_cast<double*>(wsp(s, WS_E)), jw > 0 ? static_cast<double*>(wsp(s, WS_JWORK)) : nullptr,
                         s->ctx->status, st));
  }
  EPHW_TRY(ws_need(s, WS_U, (size_t)nq * nm * nm * cs));
  EPHW_TRY(mode_vectors(kind, static_cast<const double*>(wsp(s, WS_E)), nq, (int)nm, s->ism, wsp(s, WS_U), st));
  EPHW_TRY(ws_need(s, WS_DE64, (size_t)3 * nq * nm * nm * 16));
  EPHW_TRY(ws_need(s, WS_DU, (size_t)3 * nq * nm * nm * cs));
  EPHW_TRY(eigvec_derivatives(s, static_cast<const double*>(wsp(s, WS_PQC)), s->r_c, nq, s->nc, s->c_scaled, (int)nm,
                              static_cast<const double*>(wsp(s, WS_LAM)), static_cast<const double*>(wsp(s, WS_E)),
                              static_cast<double*>(wsp(s, WS_DE64)), nullptr, 0, st));
  // du = de / sqrt(M) (per row), for the three directions
  EPHW_TRY(mode_vectors(kind, static_cast<const double*>(wsp(s, WS_DE64)), 3 * nq, (int)nm, s->ism,
                        wsp(s, WS_DU), st));

  // ---- accumulators ----
  EPHW_TRY(ws_need(s, WS_VKBAR, (size_t)nk * nw2 * cs));
  EPHW_TRY(fill_zero(kind, wsp(s, WS_VKBAR), nk * nw2, st));
  EPHW_TRY(ws_need(s, WS_PAIRS, (size_t)nq * nk * 3 * 8));
  EPHW_TRY(fill_zero(2, wsp(s, WS_PAIRS), nq * nk * 3, st));
  // dL/dk and dL/dq accumulate in the caller's buffers (scratch when not requested)
  EPHW_TRY(ws_need(s, WS_DKACC, (size_t)(nk + nq) * 3 * 8));
  double* dk_acc = dL_dk ? dL_dk : static_cast<double*>(wsp(s, WS_DKACC));
  double* dq_acc = dL_dq ? dL_dq : static_cast<double*>(wsp(s, WS_DKACC)) + nk * 3;

  // ---- per-unit buffers ----
  const size_t gsz = (size_t)qb * ne * E * cs, wsz = (size_t)kt * qb * E * cs;
  EPHW_TRY(ws_need(s, WS_G, gsz));
  EPHW_TRY(ws_need(s, WS_GNU, gsz));
  EPHW_TRY(ws_need(s, WS_GBAR, gsz));
  EPHW_TRY(ws_need(s, WS_GNUBAR, gsz));
  EPHW_TRY(ws_need(s, WS_W, wsz));
  EPHW_TRY(ws_need(s, WS_T, wsz));
  EPHW_TRY(ws_need(s, WS_YBAR, wsz));
  EPHW_TRY(ws_need(s, WS_Z, wsz));
  EPHW_TRY(ws_need(s, WS_WBAR, wsz));
  EPHW_TRY(ws_need(s, WS_PAIRBAR, (size_t)kt * qb * nw2 * cs * 2));
  EPHW_TRY(ws_need(s, WS_OFF, (size_t)kt * qb * 8));
  const int64_t rot_tiles = cgemm_tiles(kind, nm * nw, nw);  // per pair
  EPHW_TRY(ws_need(s, WS_LOSS, (size_t)kt * qb * rot_tiles * 8));
  EPHW_TRY(ws_need(s, WS_UBAR, (size_t)qb * nm * nm * cs));
  const int chunks_u = splitk_chunks(nw2, 16, 256);
  EPHW_TRY(ws_need(s, WS_SPLIT, (size_t)std::max<int64_t>(qb * chunks_u * nm * nm, 1) * cs));
  // the per-pair Vbar GEMMs (Nw x Nw outputs, K = Nm Nw) split K until a unit
  // has about 1024 tiles
  const int64_t pair_out_tiles = cgemm_tiles(kind, nw, nw);
  const int chunks_b = splitk_chunks(
      nm * nw, (int)std::min<int64_t>(16, std::max<int64_t>(1, ceil_div(1024, kt * qb * pair_out_tiles))), 256);
  if (chunks_b > 1) EPHW_TRY(ws_need(s, WS_SPLITB, (size_t)kt * qb * chunks_b * nw2 * cs));
  EPHW_TRY(ws_need(s, WS_DOTPART, (size_t)kRowDotPart * 8));
  double* dotpart = static_cast<double*>(wsp(s, WS_DOTPART));
  char* G = static_cast<char*>(wsp(s, WS_G));
  char* Gnu = static_cast<char*>(wsp(s, WS_GNU));
  char* Gbar = static_cast<char*>(wsp(s, WS_GBAR));
  char* Gnubar = static_cast<char*>(wsp(s, WS_GNUBAR));
  char* W = static_cast<char*>(wsp(s, WS_W));
  char* Tm = static_cast<char*>(wsp(s, WS_T));
  char* Yb = static_cast<char*>(wsp(s, WS_YBAR));
  char* Z = static_cast<char*>(wsp(s, WS_Z));
  char* Wb = static_cast<char*>(wsp(s, WS_WBAR));
  char* Vkb_pair = static_cast<char*>(wsp(s, WS_PAIRBAR));
  char* Vkqb_pair = Vkb_pair + (size_t)kt * qb * nw2 * cs;
  int64_t* offp = static_cast<int64_t*>(wsp(s, WS_OFF));
  double* lossp = static_cast<double*>(wsp(s, WS_LOSS));
  char* ubar = static_cast<char*>(wsp(s, WS_UBAR));
  char* pq = static_cast<char*>(wsp(s, WS_PQ));
  char* dpq = static_cast<char*>(wsp(s, WS_DPQ));
  char* u = static_cast<char*>(wsp(s, WS_U));
  char* du = static_cast<char*>(wsp(s, WS_DU));
  char* vt = static_cast<char*>(ks->vt);
  char* vkbar = static_cast<char*>(wsp(s, WS_VKBAR));
  double* pairs = static_cast<double*>(wsp(s, WS_PAIRS));

  for (int64_t q0 = 0; q0 < nq; q0 += qb) {
    const int64_t nb = std::min(qb, nq - q0);
    // Eq. (9): G [nb][ne E]
    GemmParams rp;
    rp.M = nb;
    rp.N = ne * E;
    rp.K = np;
    rp.A = pq + (size_t)q0 * np * cs;
    rp.lda = np;
    rp.B = s->g;
    rp.ldb = rp.N;
    rp.C = G;
    rp.ldc = rp.N;
    EPHW_TRY(cgemm(kind, rp, st));
    // mode vectors: Gnu[e][q] = u[q]^T G[q][e]  (batch (q, e))
    GemmParams mr;
    mr.M = nm;
    mr.N = nw2;
    mr.K = nm;
    mr.batch = nb * ne;
    mr.n2 = ne;
    mr.A = u + (size_t)q0 * nm * nm * cs;
    mr.transA = true;
    mr.lda = nm;
    mr.strideA = nm * nm;
    mr.B = G;
    mr.ldb = nw2;
    mr.strideB = ne * E;
    mr.strideB2 = E;
    mr.C = Gnu;
    mr.ldc = nw2;
    mr.strideC = E;
    mr.strideC2 = nb * E;
    EPHW_TRY(cgemm(kind, mr, st));
    for (int64_t k0 = 0; k0 < nk; k0 += kt) {
      const int64_t kl = std::min(kt, nk - k0);
      const int64_t nbat = kl * nb * nm;
      // Eq. (10) Re sum: W [kl][nb E]
      GemmParams re;
      re.M = kl;
      re.N = nb * E;
      re.K = ne;
      re.A = static_cast<const char*>(ks->pk) + (size_t)k0 * ne * cs;
      re.lda = ne;
      re.B = Gnu;
      re.ldb = re.N;
      re.C = W;
      re.ldc = re.N;
      EPHW_TRY(cgemm(kind, re, st));
      hipLaunchKernelGGL(kq_offsets_kernel, dim3(grid1(kl * nb, 256)), dim3(256), 0, st, kq_index, nk, q0, k0, (int)kl,
                         (int)nb, nw2, offp, s->ctx->status);
      EPHW_CHECK_LAUNCH();
      // T'_nu = (W_nu V(k))^T, block-transposed store: [pair][nu][n][m']
      GemmParams f4 = pair_params(nw, nm, nb, kl, E);
      f4.A = W;
      f4.B = vt + (size_t)k0 * nw2 * cs;
      f4.strideB = nw2;
      f4.C = Tm;
      f4.tblock = nw;
      f4.ldc = nw2;
      EPHW_TRY(cgemm(kind, f4, st));
      // Ybar'_nu = 2 w (V(k+q)^H T_nu)^T: rows (nu, n), columns m, [pair][nu][n][m]; loss partials
      GemmParams f5 = pair_params(nw, nm, nb, kl, E);
      f5.A = Tm;
      f5.B = vt;
      f5.offB = offp;
      f5.conjB = true;
      f5.C = Yb;
      f5.loss.on = true;
      f5.loss.layout = 1;
      f5.loss.store = true;
      f5.loss.grad_scale = true;
      f5.loss.seed = loss_seed;
      f5.loss.nk = nk;
      f5.loss.nm = (int)nm;
      f5.loss.nw = (int)nw;
      f5.loss.qb = (int)nb;
      f5.loss.q0 = q_offset + q0;
      f5.loss.k0 = k0;
      f5.loss.partial = lossp;
      EPHW_TRY(cgemm(kind, f5, st));
      if (loss) EPHW_TRY(sum_into(lossp, kl * nb * rot_tiles, loss, st));
      // Z_nu = V(k+q) Ybar_nu: rows (nu, n) of Ybar', B = V(k+q)^T; block-transposed
      // store gives the standard [pair][nu][m][n]
      GemmParams b1 = pair_params(nw, nm, nb, kl, E);
      b1.A = Yb;
      b1.B = vt;
      b1.offB = offp;
      b1.transB = true;
      b1.C = Z;
      b1.tblock = nw;
      b1.ldc = nw2;
      EPHW_TRY(cgemm(kind, b1, st));
      // Wbar_nu = Z_nu V(k)^H: rows (nu, m) of Z
      GemmParams b2 = pair_params(nw, nm, nb, kl, E);
      b2.A = Z;
      b2.B = vt + (size_t)k0 * nw2 * cs;
      b2.transB = true;
      b2.conjB = true;
      b2.strideB = nw2;
      b2.C = Wb;
      EPHW_TRY(cgemm(kind, b2, st));
      // per pair: Vbar(k) part = sum_nu W_nu^H Z_nu; Vbar(k+q) part = sum_nu T_nu Ybar_nu^H
      GemmParams b3;
      b3.M = nw;
      b3.N = nw;
      b3.K = nm * nw;
      b3.batch = kl * nb;
      b3.A = W;
      b3.transA = true;
      b3.conjA = true;
      b3.lda = nw;
      b3.strideA = E;
      b3.B = Z;
      b3.ldb = nw;
      b3.strideB = E;
      b3.C = Vkb_pair;
      b3.ldc = nw;
      b3.strideC = nw2;
      EPHW_TRY(cgemm_splitk(kind, b3, chunks_b, wsp(s, WS_SPLITB), st));
      GemmParams b4 = b3;
      b4.A = Tm;  // T' rows (nu, n) = K, columns m
      b4.transA = true;
      b4.conjA = false;
      b4.B = Yb;  // Ybar' rows (nu, n) = K, columns m''
      b4.conjB = true;
      b4.C = Vkqb_pair;
      EPHW_TRY(cgemm_splitk(kind, b4, chunks_b, wsp(s, WS_SPLITB), st));
      // Vbar(k) += sum over the unit's q of the pair parts (fixed order: iq ascending)
      {
        const int64_t total = kl * nw2;
        if (kind == 0)
          hipLaunchKernelGGL(splitk_reduce_kernel<double>, dim3(grid1(total, 256)), dim3(256), 0, st,
                             reinterpret_cast<const double*>(Vkb_pair), kl, (int)nb, nw2,
                             reinterpret_cast<double*>(vkbar + (size_t)k0 * nw2 * cs), nw2, nw2, nw2, 1);
        else
          hipLaunchKernelGGL(splitk_reduce_kernel<float>, dim3(grid1(total, 256)), dim3(256), 0, st,
                             reinterpret_cast<const float*>(Vkb_pair), kl, (int)nb, nw2,
                             reinterpret_cast<float*>(vkbar + (size_t)k0 * nw2 * cs), nw2, nw2, nw2, 1);
        EPHW_CHECK_LAUNCH();
      }
      // pair scalars Re <Vbar(k+q), dV_d at the k+q grid point> -> pairs[(q0+iq) nk + k0+il][d];
      // row r = il nb + iq of the pair buffers, offp[r] = grid index * nw2
      for (int d = 0; d < 3; ++d)
        EPHW_TRY(row_dot2(kind, Vkqb_pair, nw2, static_cast<const char*>(ks->dv) + (size_t)d * nk * nw2 * cs, 0, offp,
                          kl * nb, nw2, pairs + (q0 * nk + k0) * 3 + d, nb, 3, nk * 3, false, dotpart, st));
      // Eq. (10) adjoint: Gnubar (+)= Pk^H Wbar
      GemmParams b6;
      b6.M = ne;
      b6.N = nb * E;
      b6.K = kl;
      b6.A = static_cast<const char*>(ks->pk) + (size_t)k0 * ne * cs;
      b6.transA = true;
      b6.conjA = true;
      b6.lda = ne;
      b6.B = Wb;
      b6.ldb = nb * E;
      b6.C = Gnubar;
      b6.ldc = nb * E;
      b6.accumulate = k0 > 0;
      EPHW_TRY(cgemm(kind, b6, st));
      // k through the Re phases: dk_d += Re <Wbar, W'_d>, W'_d = (2 pi i Re_d Pk) Gnu
      for (int d = 0; d < 3; ++d) {
        if (!dir_e[d]) continue;
        GemmParams wd = re;
        wd.A = static_cast<const char*>(ks->dpk) + ((size_t)d * nk + k0) * ne * cs;
        wd.C = Z;  // Z is free now: reuse as W'_d
        EPHW_TRY(cgemm(kind, wd, st));
        EPHW_TRY(row_dot(kind, Wb, nb * E, Z, nb * E, nullptr, kl, nb * E, dk_acc + k0 * 3 + d, 3, true, dotpart, st));
      }
    }
    // mode-vector adjoint: Gbar[q][e] = conj(u[q]) Gnubar[e][q]
    GemmParams ma;
    ma.M = nm;
    ma.N = nw2;
    ma.K = nm;
    ma.batch = nb * ne;
    ma.n2 = ne;
    ma.A = u + (size_t)q0 * nm * nm * cs;
    ma.conjA = true;
    ma.lda = nm;
    ma.strideA = nm * nm;
    ma.B = Gnubar;
    ma.ldb = nw2;
    ma.strideB = E;
    ma.strideB2 = nb * E;
    ma.C = Gbar;
    ma.ldc = nw2;
    ma.strideC = ne * E;
    ma.strideC2 = E;
    EPHW_TRY(cgemm(kind, ma, st));
    // ubar[q] = sum_e conj(G[q][e]) Gnubar[e][q]^T   (split-K over the band pairs)
    for (int64_t e = 0; e < ne; ++e) {
      GemmParams ub;
      ub.M = nm;
      ub.N = nm;
      ub.K = nw2;
      ub.batch = nb;
      ub.A = G + (size_t)e * E * cs;
      ub.conjA = true;
      ub.lda = nw2;
      ub.strideA = ne * E;
      ub.B = Gnubar + (size_t)e * nb * E * cs;
      ub.transB = true;
      ub.ldb = nw2;
      ub.strideB = E;
      ub.C = ubar;
      ub.ldc = nm;
      ub.strideC = nm * nm;
      ub.accumulate = e > 0;
      EPHW_TRY(cgemm_splitk(kind, ub, chunks_u, wsp(s, WS_SPLIT), st));
    }
    // q through u: dq_d += Re <ubar[q], du_d[q]>
    for (int d = 0; d < 3; ++d)
      EPHW_TRY(row_dot(kind, ubar, nm * nm, du + ((size_t)d * nq + q0) * nm * nm * cs, nm * nm, nullptr, nb, nm * nm,
                       dq_acc + q0 * 3 + d, 3, true, dotpart, st));
    // dL/dg += Pq^H Gbar
    if (dL_dg) {
      GemmParams dg;
      dg.M = np;
      dg.N = ne * E;
      dg.K = nb;
      dg.A = pq + (size_t)q0 * np * cs;
      dg.transA = true;
      dg.conjA = true;
      dg.lda = np;
      dg.B = Gbar;
      dg.ldb = ne * E;
      dg.C = dL_dg;
      dg.ldc = ne * E;
      dg.accumulate = true;
      EPHW_TRY(cgemm(kind, dg, st));
    }
    // q through the Rp phases: dq_d += Re <Gbar, G'_d>, G'_d = (2 pi i Rp_d Pq) g
    for (int d = 0; d < 3; ++d) {
      if (!dir_p[d]) continue;
      GemmParams gd = rp;
      gd.A = dpq + ((size_t)d * nq + q0) * np * cs;
      gd.C = Gnu;  // free after the k loop
      EPHW_TRY(cgemm(kind, gd, st));
      EPHW_TRY(row_dot(kind, Gbar, ne * E, Gnu, ne * E, nullptr, nb, ne * E, dq_acc + q0 * 3 + d, 3, true, dotpart, st));
    }
  }
  // k through V(k): dk_d += Re <Vbar(k), dV_d(k)>
  for (int d = 0; d < 3; ++d)
    EPHW_TRY(row_dot(kind, vkbar, nw2, static_cast<const char*>(ks->dv) + (size_t)d * nk * nw2 * cs, nw2, nullptr, nk,
                     nw2, dk_acc + d, 3, true, dotpart, st));
  // k and q through V(k+q): sum the pair scalars over q (for k) and over k (for q)
  hipLaunchKernelGGL(pair_sums_kernel, dim3(grid1((nk + nq) * 3, 256)), dim3(256), 0, st, pairs, nq, nk, dk_acc,
                     dq_acc);
  EPHW_CHECK_LAUNCH();
  return EPHW_OK;
}

// Eq. (6) on the k-set (coarse k' grid) and a q' list whose k'+q' fall on it.
ephw_status ephw_wannier_transform(ephw_kset* ks, const double* q, int64_t nq, const int32_t* kq_index,
                                   const void* g_bloch, void* g_out, void* stream) {
  if (!ks || !q || nq <= 0 || !kq_index || !g_bloch || !g_out) {
    set_error("ephw_wannier_transform: need a k-set, a q list, a k+q index table and both buffers");
    return EPHW_EINVAL;
  }
  if (ks->prec == EPHW_FP32_COMP) {
    set_error("ephw_wannier_transform: FP64 or FP32 k-sets only");
    return EPHW_EUNSUPPORTED;
  }
  ephw_system* s = ks->sys;
  hipStream_t st = as_stream(stream);
  const int kind = prec_kind(ks->prec);
  const size_t cs = csize(kind);
  const int64_t nw = s->nw, nm = s->nm, nw2 = nw * nw, E = nm * nw2, nk = ks->nk, ne = s->ne, np = s->np;
  // q batch: up to 128 q (the Re sum's N = qb E) within 8 GB for the two
  // g(Re,q) buffers; k tile within 16 GB for the two pair buffers
  int64_t qb = s->q_batch > 0 ? s->q_batch : (int64_t)(8.0e9 / (2.0 * (double)ne * E * cs));
  qb = std::max<int64_t>(1, std::min<int64_t>({qb, 128, nq}));
  int64_t kt = s->k_tile > 0 ? s->k_tile : (int64_t)(16.0e9 / (2.0 * (double)cs * qb * E));
  kt = std::max<int64_t>(1, std::min(kt, nk));

  // phases as Eq. (6) writes them (no lattice-vector weights); the q ones
  // carry 1/(Ne Np)
  EPHW_TRY(ws_need(s, WS_CPK, (size_t)nk * ne * cs));
  EPHW_TRY(phase_matrix(kind, ks->k, nk, s->r_e, nullptr, ne, wsp(s, WS_CPK), st));
  EPHW_TRY(ws_need(s, WS_PQ, (size_t)nq * np * cs));
  EPHW_TRY(phase_matrix(kind, q, nq, s->r_p, nullptr, np, wsp(s, WS_PQ), st));
  {
    const int64_t n = nq * np;
    const double f = 1.0 / ((double)ne * (double)np);
    if (kind == 0)
      hipLaunchKernelGGL(scale_complex_kernel<double>, dim3(grid1(n, 256)), dim3(256), 0, st,
                         static_cast<double*>(wsp(s, WS_PQ)), n, f);
    else
      hipLaunchKernelGGL(scale_complex_kernel<float>, dim3(grid1(n, 256)), dim3(256), 0, st,
                         static_cast<float*>(wsp(s, WS_PQ)), n, f);
    EPHW_CHECK_LAUNCH();
  }
  // modes at q': D(q') eigensolve, then (u^-1)^T
  EPHW_TRY(ws_need(s, WS_PQC, (size_t)nq * s->nc * 16));
  EPHW_TRY(phase_matrix(0, q, nq, s->r_c, s->w_c, s->nc, wsp(s, WS_PQC), st));
  EPHW_TRY(ws_need(s, WS_LAM, (size_t)nq * nm * 8));
  EPHW_TRY(ws_need(s, WS_E, (size_t)nq * nm * nm * 16));
  {
    EPHW_TRY(ws_need(s, WS_HK, (size_t)nq * nm * nm * 16));
    GemmParams g;
    g.M = nq;
    g.N = nm * nm;
    g.K = s->nc;
    g.A = wsp(s, WS_PQC);
    g.lda = s->nc;
    g.B = s->c_scaled;
    g.ldb = nm * nm;
    g.C = wsp(s, WS_HK);
    g.ldc = nm * nm;
    EPHW_TRY(cgemm(0, g, st));
    const int64_t jw = jacobi_work_doubles((int)nm, nq);
    if (jw > 0) EPHW_TRY(ws_need(s, WS_JWORK, (size_t)jw * 8));
    EPHW_TRY(jacobi_eigh(static_cast<const double*>(wsp(s, WS_HK)), nq, (int)nm, static_cast<double*>(wsp(s, WS_LAM)),
                         static_cast<double*>(wsp(s, WS_E)), jw > 0 ? static_cast<double*>(wsp(s, WS_JWORK)) : nullptr,
                         s->ctx->status, st));
  }
  EPHW_TRY(ws_need(s, WS_UINV, (size_t)nq * nm * nm * cs));
  {
    const int64_t n = nq * nm * nm;
    const double* e = static_cast<const double*>(wsp(s, WS_E));
    if (kind == 0)
      hipLaunchKernelGGL(mode_inverse_kernel<double>, dim3(grid1(n, 256)), dim3(256), 0, st, e, nq, (int)nm, s->ism,
                         static_cast<double*>(wsp(s, WS_UINV)));
    else
      hipLaunchKernelGGL(mode_inverse_kernel<float>, dim3(grid1(n, 256)), dim3(256), 0, st, e, nq, (int)nm, s->ism,
                         static_cast<float*>(wsp(s, WS_UINV)));
    EPHW_CHECK_LAUNCH();
  }

  const size_t gsz = (size_t)qb * ne * E * cs, wsz = (size_t)kt * qb * E * cs;
  EPHW_TRY(ws_need(s, WS_GBAR, gsz));
  EPHW_TRY(ws_need(s, WS_GNUBAR, gsz));
  EPHW_TRY(ws_need(s, WS_T, wsz));
  EPHW_TRY(ws_need(s, WS_WBAR, wsz));
  EPHW_TRY(ws_need(s, WS_OFF, (size_t)kt * qb * 8));
  char* Gbar = static_cast<char*>(wsp(s, WS_GBAR));
  char* Gnubar = static_cast<char*>(wsp(s, WS_GNUBAR));
  char* Tm = static_cast<char*>(wsp(s, WS_T));
  char* Wb = static_cast<char*>(wsp(s, WS_WBAR));
  int64_t* offp = static_cast<int64_t*>(wsp(s, WS_OFF));
  const char* cpk = static_cast<const char*>(wsp(s, WS_CPK));
  const char* cpq = static_cast<const char*>(wsp(s, WS_PQ));
  const char* uinv = static_cast<const char*>(wsp(s, WS_UINV));
  const char* gb = static_cast<const char*>(g_bloch);
  char* vt = static_cast<char*>(ks->vt);

  for (int64_t q0 = 0; q0 < nq; q0 += qb) {
    const int64_t nb = std::min(qb, nq - q0);
    for (int64_t k0 = 0; k0 < nk; k0 += kt) {
      const int64_t kl = std::min(kt, nk - k0);
      hipLaunchKernelGGL(kq_offsets_kernel, dim3(grid1(kl * nb, 256)), dim3(256), 0, st, kq_index, nk, q0, k0, (int)kl,
                         (int)nb, nw2, offp, s->ctx->status);
      EPHW_CHECK_LAUNCH();
      // T'_nu = (g_nu V(k)^dagger)^T, rows (nu, n') and columns m; the input
      // pairs are q-major ([q][k][E]), the unit's pair buffers [il][iq][E]
      GemmParams r1 = pair_params(nw, nm, nb, kl, E);
      r1.A = gb + ((size_t)q0 * nk + k0) * E * cs;
      r1.strideA = E;
      r1.strideA1 = nk * E;
      r1.B = vt + (size_t)k0 * nw2 * cs;
      r1.strideB = nw2;
      r1.transB = true;
      r1.conjB = true;
      r1.C = Tm;
      r1.tblock = nw;
      r1.ldc = nw2;
      EPHW_TRY(cgemm(kind, r1, st));
      // W_nu = V(k+q) g_nu V(k)^dagger: rows (nu, n') of T' times V(k+q)^T, stored
      // block-transposed into [pair][nu][m'][n']
      GemmParams r2 = pair_params(nw, nm, nb, kl, E);
      r2.A = Tm;
      r2.B = vt;
      r2.offB = offp;
      r2.transB = true;
      r2.C = Wb;
      r2.tblock = nw;
      r2.ldc = nw2;
      EPHW_TRY(cgemm(kind, r2, st));
      // G_nu(Re, q) (+)= sum_k e^{-ik.Re} W_nu(k, q)
      GemmParams rk;
      rk.M = ne;
      rk.N = nb * E;
      rk.K = kl;
      rk.A = cpk + (size_t)k0 * ne * cs;
      rk.transA = true;
      rk.conjA = true;
      rk.lda = ne;
      rk.B = Wb;
      rk.ldb = nb * E;
      rk.C = Gnubar;
      rk.ldc = nb * E;
      rk.accumulate = k0 > 0;
      EPHW_TRY(cgemm(kind, rk, st));
    }
    // G[q][e][ka] = sum_nu u^-1_{nu,ka}(q) G_nu[e][q]
    GemmParams mi;
    mi.M = nm;
    mi.N = nw2;
    mi.K = nm;
    mi.batch = nb * ne;
    mi.n2 = ne;
    mi.A = uinv + (size_t)q0 * nm * nm * cs;
    mi.lda = nm;
    mi.strideA = nm * nm;
    mi.B = Gnubar;
    mi.ldb = nw2;
    mi.strideB = E;
    mi.strideB2 = nb * E;
    mi.C = Gbar;
    mi.ldc = nw2;
    mi.strideC = ne * E;
    mi.strideC2 = E;
    EPHW_TRY(cgemm(kind, mi, st));
    // g(Re, Rp) (+)= 1/(Ne Np) sum_q e^{-iq.Rp} G(Re, q)
    GemmParams rq;
    rq.M = np;
    rq.N = ne * E;
    rq.K = nb;
    rq.A = cpq + (size_t)q0 * np * cs;
    rq.transA = true;
    rq.conjA = true;
    rq.lda = np;
    rq.B = Gbar;
    rq.ldb = ne * E;
    rq.C = g_out;
    rq.ldc = ne * E;
    rq.accumulate = q0 > 0;
    EPHW_TRY(cgemm(kind, rq, st));
  }
  return EPHW_OK;
}

}  // extern "C"
