// Launchers of the non-GEMM kernels of libephw.
#pragma once

#include "common.h"

namespace ephw {

// out[i][r] = w_r exp(2 pi i p_i.R_r) (w = NULL -> 1), argument reduced in FP64.
// prec 0: out is c128.  prec 1: out is c64, the FP64 phase rounded.
ephw_status phase_matrix(int prec, const double* pts, int64_t n, const int32_t* R, const double* w,
                         int64_t nr, void* out, hipStream_t s);

// Hermitian eigensolve of a batch of n x n c128 matrices (cyclic Jacobi, FP64).
// eps [batch][n] ascending; V [batch][n][n] c128, column j the eigenvector of eps j,
// scaled so its largest-magnitude entry is real positive.  `work` must hold
// jacobi_work_doubles(n, batch) doubles (0 for n <= 32).
int64_t jacobi_work_doubles(int n, int64_t batch);
// off_tol2: convergence when (off-diagonal norm / total norm)^2 <= off_tol2
// (not below 1e-28, the FP64 default; n <= 32 only, larger orders keep 1e-28)
ephw_status jacobi_eigh(const double* H, int64_t batch, int n, double* eps, double* V, double* work,
                        uint32_t* status, hipStream_t s, double off_tol2 = 1e-28);

// many small (n <= 32) eigensolves of different orders in one launch;
// matrix m of the launch belongs to the job with the largest block_base <= m
// (count matrices each); total = all jobs' matrices, max_n their largest order
struct EighJob {
  const double* H;
  double* eps;
  double* V;
  int n;
  int64_t count, block_base;
};
ephw_status jacobi_eigh_grouped(const EighJob* d_jobs, int njobs, int64_t total, int max_n, uint32_t* status,
                                hipStream_t s);

// out[q][k][nu][m][n] = sum of |g|^2 over the degenerate blocks of nu (lam[q]),
// m (eps_kq[q][k]) and n (eps_k[k]); g c128 (prec 0) or c64
ephw_status degenerate_sums(int prec, const void* g, int64_t nq, int64_t nk, int nm, int nw,
                            const double* eps_kq, const double* eps_k, const double* lam, double rel_tol,
                            double* out, hipStream_t s);

// gamma[k][n] += phonon-limited linewidth contributions of the q list (see epilogue.hip)
// out[i] += scale * sum_c x[c][i] for i < n, c < ncol: partial sums over
// fixed chunks of c into `scratch` (column_sum_scratch(n) bytes), then the
// chunks in order (deterministic)
size_t column_sum_scratch(int64_t n);
ephw_status add_column_sums(const double* x, int64_t ncol, int64_t n, double scale, double* out, double* scratch,
                            hipStream_t s);
ephw_status linewidth(int prec, const void* g, int64_t nq, int64_t nk, int nm, int nw, const double* eps_k,
                      const double* eps_kq, const double* omega, double temperature, double mu, double sigma,
                      double omega_min, int64_t nq_total, double* gamma, hipStream_t s);

// dst[i] = (T) src[i] for n complex values; T = float (prec 1) or a plain copy (prec 0)
ephw_status cast_complex(int prec, const double* src, void* dst, int64_t n, hipStream_t s);

// u[q][a][v] = e[q][a][v] * inv_sqrt_mass[a], stored as c128 (prec 0) or c64 (prec 1)
ephw_status mode_vectors(int prec, const double* e, int64_t nq, int nm, const double* inv_sqrt_mass,
                         void* u, hipStream_t s);
// omega = sqrt(|lambda|)
ephw_status abs_sqrt(const double* lam, double* omega, int64_t n, hipStream_t s);

// B[q][r][ab] = phase[q][r] * H[r][ab]  (c128), the q factor of H(k+q)
ephw_status scale_rows_by_phase(const double* phase, int64_t nq, const double* H, int64_t nr,
                                int64_t nab, double* B, hipStream_t s);

// Gnu[e][q][nu][mn] = sum_a u[q][a][nu] G[q][e][a][mn]  (u = NULL: Gnu = G transposed)
ephw_status mode_rotate(int prec, const void* G, const void* u, void* Gnu, int64_t ne, int qb,
                        int nm, int64_t nw2, hipStream_t s);

struct BandRotateArgs {
  const void* W;          // [nk_tile][qb][nm][nw][nw]  (Re-GEMM output, row stride qb*nm*nw*nw)
  const void* Vk;         // [nk][nw][nw] or NULL (identity: Wannier-gauge output)
  const void* Vkq;        // [qb][nk][nw][nw] or NULL
  const int32_t* kq_index;  // [qb][nk] (already offset to the batch) or NULL
  int64_t nk;             // size of the k set (row stride of kq_index, g_out, band_sum)
  int64_t k0 = 0;         // global index of the tile's first k
  int64_t nk_tile = 0;    // k points in this tile (grid x)
  int qb, nm, nw;
  uint32_t flags;
  void* g_out;            // [qb][nk][nm][nw][nw], offset to the batch
  double* band_sum;       // [qb][nk][nm], offset to the batch
  double* loss_partial;   // [qb][nk_tile] per-pair partial sums, or NULL
  uint64_t loss_seed;
  int64_t q_global0;      // global index of the batch's first q
  uint32_t* status;
  // Pair mode (pair_k set): the "k points" are a list of (k, q) pairs with
  // qb = 1; W, g_out, band_sum and loss_partial are indexed by pair, V(k) is
  // Vk[pair_k[p]], V(k+q) is Vk[kq_index[p]], and the loss element index uses
  // the pair's own (q_global0 + pair_q[p], pair_k[p]) in a set of nk_set points.
  const int32_t* pair_k = nullptr;
  const int32_t* pair_q = nullptr;
  int64_t nk_set = 0;
  // Band window (band_n > 0, rotations only): g, band sums and the loss keep
  // the bands band_lo .. band_lo+band_n-1 at k+q (m) and at k (n); g_out is
  // then [..][nm][band_n][band_n] and the loss element index stays that of
  // the full [nm][nw][nw] layout.
  int band_lo = 0, band_n = 0;
};
ephw_status band_rotate(int prec, const BandRotateArgs& a, hipStream_t s);
// Work split of a band-rotation launch (Nw <= 32, rotations without a band
// window): P consecutive k per workgroup, nuc modes per LDS chunk, dynamic
// LDS bytes.  The matrix-core kernel takes P = 4 (one wavefront per pair,
// all modes, static LDS).
struct BandPlan {
  int P = 1, nuc = 1;
  size_t lds = 0;
};
BandPlan band_rotate_plan(int prec, int nw, int nm);
// kernel instance of a band count: -16 or -32 (the padded size) for the
// matrix-core kernel, else Nw rounded up to a multiple of 4 (row kernel)
int band_rotate_class(int nw);
// whether the rotations of this band count run on the matrix cores
// (8 < Nw <= 32; band_rotate keeps the row kernel for a band window and for
// the Wannier-gauge output).  Loss partials stay one per pair either way.
bool band_rotate_on_mfma(int nw);

// grouped launches over many systems: block b belongs to the job with the
// largest block_base <= b (jobs sorted by block_base)
struct ModeRotateJob {
  const void* G;
  const void* u;
  void* Gnu;
  int64_t ne, nw2;
  int qb, nm;
  int64_t block_base;     // blocks: qb * ceil(ne*nw2/256)
};
ephw_status mode_rotate_grouped(int prec, const ModeRotateJob* d_jobs, int n, int64_t blocks, size_t lds,
                                hipStream_t s);
struct BandRotateJob {
  BandRotateArgs args;
  int P, nuc;             // from band_rotate_plan
  int64_t block_base;     // blocks: qb * ceil(nk_tile / P)
};
// All jobs of one grouped launch share the kernel instance `nwb`
// (band_rotate_class).  Launches never change kernel attributes (they may be
// captured in a graph): call band_rotate_grouped_prepare for each instance
// with its largest LDS size first.
ephw_status band_rotate_grouped_prepare(int prec, int nwb, size_t lds);
ephw_status band_rotate_grouped(int prec, int nwb, const BandRotateJob* d_jobs, int n, int64_t blocks, size_t lds,
                                hipStream_t s);
struct SumJob {
  const double* x;
  int64_t n;
  double* out;
};
ephw_status sum_into_grouped(const SumJob* d_jobs, int n, hipStream_t s);

// dst[r][c] = src[idx[r]][c] (rows of width w); an index outside [0, nsrc) sets kStatusIndex
ephw_status gather_rows(const double* src, int64_t nsrc, const int32_t* idx, int64_t cnt, int w,
                        double* dst, uint32_t* status, hipStream_t s);

// out[0] += sum of x[0..n) in a fixed order (deterministic)
ephw_status sum_into(const double* x, int64_t n, double* out, hipStream_t s);

}  // namespace ephw
